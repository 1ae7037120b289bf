#!/usr/bin/env python3
"""Throughput of batched biased-Langevin trial paths on one MI355X.

Workload: 64 trial trajectories of the 12,560-atom solvated system (560-atom
synthetic solute + 4,000 flexible three-site waters, 5.0 nm box, 1.0 nm
cutoff, dt = 1 fs, contact-map bias ramped toward a seeded target map), all
replicas in one batch, every step replayed from captured hipGraphs.  Seeded
synthetic inputs stand in for the paper's protein systems.

One benchmark step = one pass of the whole hot path over the batch: a block
of MD steps (pair-list maintenance, nonbonded + bonded forces, collective
variable and bias, BAOAB integration with Philox noise, FP64 functional
accumulation) followed by reading the functional and the variational
selection.  The reported value is whole-job atom-steps per second.

Beside it: the plain one-trajectory form (one replica, every kernel launched
per step, no graph), the nonbonded kernel against the FP32 vector roofline
(average duration from HIP events around every force launch of a second
timed pass that continues the same trajectories by direct launches on the
same stream), and the FP64 CPU oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_PAIR = 35          # algorithmic flops per unique in-cutoff pair (force only)
PEAK_FP32_TFLOPS = 157.3    # MI355X FP32 vector peak
# HBM bytes per launch of the force kernel on this workload, from rocprofv3
# FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 (factors from a 256 MiB device copy);
# see profiles/counters_64x12560.md.  Set to None when the kernel changes.
FORCE_TRAFFIC_BYTES = (306680 * 2.000 + 19200 * 1.000) * 1024


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(job):
    """Run the oracle on one replica for about `seconds`: (atom-steps, seconds, steps)."""
    desc, seconds = job
    import numpy as np
    from oracle import oracle as O  # CPU baseline leg only
    o = O.Oracle(desc)
    x = np.array(desc["x0"], dtype=np.float64)
    v = o.maxwell()
    st = o.init(x)
    n = 0
    t = time.perf_counter()
    while time.perf_counter() - t < seconds:
        o.run(x, v, st, 1)
        n += 1
    return int(desc["n_atoms"]) * n, time.perf_counter() - t, n


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30, help="timed benchmark steps")
    ap.add_argument("--warmup", type=int, default=5, help="untimed benchmark steps")
    ap.add_argument("--md-per-step", type=int, default=120,
                    help="MD steps per benchmark step (captured as graphs of 20 steps)")
    ap.add_argument("--replicas", type=int, default=64)
    ap.add_argument("--plain-steps", type=int, default=200)
    ap.add_argument("--timing-steps", type=int, default=5, help="blocks timed with HIP events")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="seconds of oracle work per process for the CPU baseline")
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="oracle processes for the CPU baseline (0: one per core, at most 16)")
    ap.add_argument("--workload", choices=("batch", "uneven", "derivative", "toy"), default="batch",
                    help="batch: 64 replicas of the 12,560-atom system; uneven: 32 replicas of "
                         "5,000-40,000 atoms with cutoffs 0.9 / 1.2 nm; derivative: 16 replicas of the "
                         "12,560-atom system carrying dPhi/d(bias_k, ramp_rate); toy: the 2-D toy "
                         "funnel, 20,000 plain trials of 90,000 steps and 2,000 ratchet trials of "
                         "30,000 steps at each of 8 bias constants")
    ap.add_argument("--equilibrate", type=int, default=6000, metavar="MD_STEPS",
                    help="untimed MD steps without bias of each distinct system before the trials "
                         "start: the synthetic start relaxes from ~800 K to 300 K, and the trials "
                         "then begin at t = 0 from the relaxed structure with Maxwell velocities "
                         "(0: start from the generated structures)")
    ap.add_argument("--nstlist", type=int, default=0,
                    help="pair-list rebuild interval (vp_options.nstlist; 0: the library default)")
    ap.add_argument("--skin", type=float, default=0.0,
                    help="pair-list buffer in nm (vp_options.skin; 0: the library default)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="run every block with --force-shape instead of timing the tile shapes "
                         "per size bucket at creation")
    ap.add_argument("--force-shape", type=int, default=0,
                    help="tile shape of the force kernel with --no-autotune (vp_options.force_shape)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one device-to-device copy of MIB MiB (a known amount of HBM "
                         "traffic that calibrates rocprofv3's FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the trial paths are "
              "independent, so several GPUs would each run this benchmark on their own share.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1405_6104_amd import synth, vp

    if args.workload == "toy":
        return toy_bench(args)
    B = args.md_per_step
    G = 20  # MD steps per captured graph
    t0 = time.time()
    if args.workload == "batch":
        base = synth.solvated_chain_12560()
        reps = synth.trial_batch(args.replicas, base=base,
                              n_steps=B * (args.steps + args.warmup + args.timing_steps))
        workload = ("64 trial paths x 12,560 atoms (560-atom solute + 4,000 flexible waters), "
                    "5.0 nm box, rc 1.0 nm, dt 1 fs, contact-map bias, graph-captured batch")
    elif args.workload == "derivative":
        base = synth.solvated_chain_12560()
        reps = synth.derivative_batch(16, base=base)
        workload = ("16 trial paths x 12,560 atoms with forward tangents of dPhi/d(bias_k, ramp_rate), "
                    "2,000-step bias ramp, rc 1.0 nm, dt 1 fs, contact-map bias, graph-captured batch")
    else:
        # replicas are independent: built by forked workers before the GPU is touched
        workers = max(1, min(16, os.cpu_count() or 1))
        reps = synth.uneven_batch(workers=workers, progress=lambda r, n: print(
            f"# replica {r}: {n} atoms ({time.time() - t0:.0f} s)", file=sys.stderr, flush=True))
        base = reps[0]
        workload = ("32 trial paths of 5,000-40,000 atoms (log-uniform; 280-560-atom solute, "
                    "water at 33.4 /nm^3), rc 0.9 or 1.2 nm, dt 1 fs, contact-map bias, "
                    "graph-captured batch")
    n_atoms = sum(int(d["n_atoms"]) for d in reps)
    print(f"# generated {len(reps)} replicas, {n_atoms} atoms in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on the host's cores: one single-threaded oracle process per
        # core, each on its own replica of the batch, forked before the GPU is used
        import multiprocessing as mp
        procs = args.cpu_procs if args.cpu_procs > 0 else max(1, min(16, os.cpu_count() or 1))
        tc = time.time()
        with mp.get_context("fork").Pool(procs) as pool:
            res = pool.map(_oracle_rate, [(reps[k % len(reps)], args.cpu_seconds) for k in range(procs)])
        steps_cpu = sum(n for _, _, n in res)
        sizes = sorted({int(reps[k % len(reps)]["n_atoms"]) for k in range(procs)})
        # one process alone on the workload's system (and on the 1,512-atom system),
        # a few seconds each, for the single-core figures
        alone = _oracle_rate((reps[0], min(5.0, args.cpu_seconds)))
        small = _oracle_rate((synth.small_chain_system(), min(5.0, args.cpu_seconds)))
        cpu = {"value": sum(a / t for a, t, _ in res), "unit": "atom-steps/s", "cores": procs,
               "kind": "oracle", "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
               "single_core": {"value": alone[0] / alone[1], "atoms": int(reps[0]["n_atoms"]),
                               "small_1512_atoms": small[0] / small[1]},
               "sample": f"{procs} processes in parallel, each the single-threaded FP64 oracle (cell-list "
                         f"pairs) on its own replica of the batch ({', '.join(f'{n:,}' for n in sizes)} "
                         f"atoms) for ~{args.cpu_seconds:.0f} s; {steps_cpu} BAOAB steps in all; "
                         f"single_core: one process alone for ~5 s on the same system and on the "
                         f"1,512-atom system"}
        print(f"# cpu oracle: {cpu['value']:.4e} atom-steps/s on {procs} cores ({time.time() - tc:.1f} s)",
              file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    if args.equilibrate > 0:
        # Thermalise each distinct system without bias (the batch and derivative
        # workloads run one system 64 / 16 times; the uneven batch has 32), then
        # start every trial at t = 0 from its system's equilibrated structure
        # with fresh Maxwell velocities at kT from the trial's own seed: all
        # trials of a system share the initial configuration and differ in noise.
        te = time.time()
        distinct = list(range(len(reps))) if args.workload == "uneven" else [0]
        src = (lambda r: r) if args.workload == "uneven" else (lambda r: 0)
        eq = vp.System([dict(reps[i], bias=vp.BIAS_NONE) for i in distinct], steps_per_graph=G,
                       nstlist=args.nstlist, skin=args.skin)
        for k in range(0, args.equilibrate, 1000):
            eq.step_batch(min(1000, args.equilibrate - k))
            torch.cuda.synchronize()
            print(f"# equilibration: {k + min(1000, args.equilibrate - k)} steps "
                  f"({time.time() - te:.1f} s)", file=sys.stderr, flush=True)
        obs = eq.observables()
        ke = obs[:, list(vp.OBS).index("ke")]
        temp = [2.0 * ke[k] / (3.0 * int(reps[i]["n_atoms"]) * 0.0083144626) for k, i in enumerate(distinct)]
        xe = eq.get_state()[0].cpu().numpy().astype(np.float64)
        reps = [dict(d, x0=xe[eq.offsets[src(r)]:eq.offsets[src(r) + 1]].copy(), v0=None)
                for r, d in enumerate(reps)]
        del eq
        print(f"# equilibrated {len(distinct)} system(s): T = {np.mean(temp):.1f} K "
              f"(min {np.min(temp):.1f}, max {np.max(temp):.1f})", file=sys.stderr, flush=True)
    tangent = args.workload == "derivative"
    system = vp.System(reps, steps_per_graph=G, force_shape=args.force_shape,
                       autotune=not args.no_autotune, nstlist=args.nstlist, skin=args.skin,
                       tangent=tangent)
    buckets, split = system.tile_buckets()
    for b in buckets:
        print(f"# bucket rc {b['r_cut']} 2^{b['log2_atoms']}: {b['replicas']} replicas, tile {b['tile']}, "
              f"ms per shape {['%.4f' % t for t in b['ms']]}", file=sys.stderr, flush=True)
    print(f"# system created (split launches: {split})", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        system.step_batch(B)
        system.functional(gradient=tangent)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        system.step_batch(B)
        system.functional(gradient=tangent)
        system.select_path()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    # force-kernel duration: the same blocks of steps continue on the same
    # stream by direct launches, with HIP events around every force launch
    system.set_timing(True)
    system.kernel_timing(reset=True)
    for _ in range(args.timing_steps):
        system.step_batch(B)
    torch.cuda.synchronize()
    force_ms, n_launch = system.kernel_timing()
    system.set_timing(False)
    obs = system.observables()
    unstable = int(np.sum((obs[:, 5].astype(int) & 1) != 0))
    overflow = int(np.sum((obs[:, 5].astype(int) & 2) != 0))
    col = {k: i for i, k in enumerate(vp.OBS)}
    list_stats = {"stage_max": int(obs[:, col["stage_max"]].max()),
                  "stage_cap": int(obs[:, col["stage_cap"]].max()),
                  "list_max": int(obs[:, col["list_max"]].max()),
                  "list_cap": int(obs[:, col["list_cap"]].max()),
                  "exact_builds": int(obs[:, col["exact_builds"]].sum())}
    pairs = [system.pair_count(r) for r in range(len(reps))]
    pairs_total = int(sum(pairs))
    md_steps = args.steps * B
    value = n_atoms * md_steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    achieved = FLOP_PER_PAIR * pairs_total / (force_ms * 1e-3) / 1e12
    dt_fs = float(base["dt"]) * 1000.0
    ns_day = (md_steps / elapsed) * dt_fs * 1e-6 * 86400.0
    print(f"# batched: {value:.4e} atom-steps/s, force kernel {force_ms:.4f} ms x {n_launch}, "
          f"{pairs_total} pairs, rebuilds/replica {obs[:, 6].mean():.1f}, unstable {unstable}, "
          f"lists {list_stats}",
          file=sys.stderr, flush=True)
    del system
    torch.cuda.empty_cache()

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy calibration: {args.copy_calibration} MiB read + written", file=sys.stderr, flush=True)
        del src, dst

    plain = None
    if not args.no_plain:
        ps = vp.System([dict(reps[0])], use_graph=False, steps_per_graph=1, tangent=tangent)
        for _ in range(20):
            ps.step_batch(1)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for _ in range(args.plain_steps):
            ps.step_batch(1)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp
        plain = int(reps[0]["n_atoms"]) * args.plain_steps / tp
        print(f"# plain: {plain:.4e} atom-steps/s ({1e3 * tp / args.plain_steps:.3f} ms/step)",
              file=sys.stderr, flush=True)
        del ps

    out = {
        "metric": "atom-steps/sec (ns/day) for batched biased Langevin MD vs plain form; % VALU peak",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair arithmetic, i64 fixed-point forces, f64 functional",
        "data": "synthetic",
        "config": {
            "workload": workload + (f"; trials start at t = 0 from the structure of a {args.equilibrate}-step "
                                    "unbiased equilibration of their system, with Maxwell velocities "
                                    "from their own seeds" if args.equilibrate > 0 else ""),
            "replicas": len(reps),
            "atoms_per_replica": (int(base["n_atoms"]) if args.workload != "uneven"
                                  else [int(d["n_atoms"]) for d in reps]),
            "md_steps_per_bench_step": B, "global_batch": n_atoms, "parallelism": "replicas",
        },
        "ns_per_day_per_replica": ns_day,
        "plain_atom_steps_per_s": plain,
        "batched_over_plain": (value / plain) if plain else None,
        "pair_interactions_per_s": pairs_total / (force_ms * 1e-3),
        "unstable_replicas": unstable,
        "list_overflow_replicas": overflow,
        "list_stats": list_stats,
        "tiles": {"autotuned": not args.no_autotune, "split_launches": split,
                  "buckets": [{k: b[k] for k in ("r_cut", "log2_atoms", "replicas", "blocks", "tile", "ms")}
                              for b in buckets]},
        "roofline": {
            "bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": (FORCE_TRAFFIC_BYTES if args.workload == "batch" and args.replicas == 64
                        else None),
            "kernel": "k_forces (nonbonded LJ + reaction field)",
            "flop_per_unit": FLOP_PER_PAIR, "units_per_launch": pairs_total,
            "avg_launch_ms": force_ms, "launches_timed": n_launch,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))



def toy_bench(args):
    """The 2-D toy funnel of the supplement: 20,000 plain trials of 90,000 steps
    and 2,000 ratchet trials of 30,000 steps at each of 8 bias constants, one
    GPU thread per trial (FP64).  value = particle-steps/s over both launches;
    the outcome per bias constant (fraction reached, the selected trial's Phi
    and gate angle) is reported beside it (parity unpinned: the supplement's
    figures are not in the text, and its printed constants give no ring
    barrier)."""
    import numpy as np
    import torch

    from paper_1405_6104_amd import vp

    params = dict(A1=30.0, A2=20.0, A3=6.0, s1=1.0, s2=2.0, s3=2.0, w=0.03, xm=1.5, ym=0.0,
                  gamma=1.0, mass=1.0, kT=0.2, dt=0.02, x0=0.0, y0=5.0, r_product=0.5, r_gate=2.0)
    kvals = [0.25, 0.5, 1.0, 2.0, 4.0, 8.0, 16.0, 32.0]
    n_plain, n_rmd = 20000, 2000
    torch.cuda.set_device(0)
    plain = dict(params, n_steps=90000)
    rmd = dict(params, n_steps=30000)
    # warm-up (short runs of the same kernels)
    vp.toy_trials(dict(plain, n_steps=100), [vp.TOY_PLAIN] * 64, [0.0] * 64, list(range(64)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res_p = vp.toy_trials(plain, [vp.TOY_PLAIN] * n_plain, [0.0] * n_plain, list(range(1, n_plain + 1)))
    kinds = [vp.TOY_RMD] * (n_rmd * len(kvals))
    ks = [k for k in kvals for _ in range(n_rmd)]
    res_r = vp.toy_trials(rmd, kinds, ks, list(range(100001, 100001 + len(kinds))))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    steps = n_plain * plain["n_steps"] + len(kinds) * rmd["n_steps"]
    col = {c: i for i, c in enumerate(vp.TOY_COLUMNS)}
    outcome = {"plain_reached": float(res_p[:, col["reached"]].mean()),
               "plain_median_first_passage_steps": float(np.median(res_p[res_p[:, col["reached"]] > 0, col["t_reach"]]))
               if res_p[:, col["reached"]].any() else None, "rmd": []}
    for j, k in enumerate(kvals):
        part = res_r[j * n_rmd:(j + 1) * n_rmd]
        best, bphi = vp.toy_select(part)
        outcome["rmd"].append({"k_R": k, "reached": float(part[:, col["reached"]].mean()),
                               "best_phi": bphi if best >= 0 else None,
                               "best_theta_gate": float(part[best, col["theta_gate"]]) if best >= 0 else None})
    out = {
        "metric": "particle-steps/s of toy-funnel trial paths (supplement toy model)",
        "value": steps / elapsed, "unit": "particle-steps/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1e3 * elapsed, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "toy funnel: 20,000 plain trials x 90,000 steps + 8 x 2,000 ratchet trials x "
                               "30,000 steps (K_R 0.25-32), dt 0.02, gamma 1, kT 0.2, start (0, 5)"},
        "outcome": outcome,
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
