"""GPU parity of the selection-side rows and the library's bookkeeping against
the FP64 oracle, through the C ABI: pair-list overflow, exact-mode list
builds, the ratchet bias in action, selection with finite tolerances, the
RMSD criterion, energies and the virial (vp_forces and trajectory records),
the device-memory hook and stream ordering.

Tolerances as in test_gpu_parity.py; energies and the virial: FP64 sums of
terms computed from FP32 intermediates, 2e-5 of the largest term of their
kind; RMSD: 1e-7 nm on identical positions (near zero the square root of the
cancellation in sum |x|^2 + |y|^2 - 2 sum s_k).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import oracle as O  # noqa: E402
from paper_1405_6104_amd import synth, vp  # noqa: E402

pytestmark = pytest.mark.gpu

F_REL, F_MAX, X_TOL, PHI_REL = 1e-5, 1e-4, 1e-4, 1e-4
GRID = 2.0 ** 22
COL = {k: i for i, k in enumerate(vp.OBS)}
E = {k: i for i, k in enumerate(vp.RECORD_COLUMNS)}
WCOLS = [E[k] for k in ("w_xx", "w_xy", "w_xz", "w_yx", "w_yy", "w_yz", "w_zx", "w_zy", "w_zz")]
WKEYS = ("w_xx", "w_xy", "w_xz", "w_yx", "w_yy", "w_yz", "w_zx", "w_zy", "w_zz")


def say(*a):
    print(*a, flush=True)


def grid(x):
    return np.rint(np.asarray(x, np.float64) * GRID) / GRID


def f32(x):
    return grid(np.asarray(x, np.float32).astype(np.float64))


def force_errors(fg, fo):
    rel = np.linalg.norm(fg - fo) / np.linalg.norm(fo)
    mx = np.abs(fg - fo).max() / np.sqrt(np.mean(np.sum(fo ** 2, 1)))
    return rel, mx


def gpu_forces(system, x_list, t=0.0):
    x = torch.from_numpy(np.concatenate([np.asarray(a, np.float32) for a in x_list])).cuda()
    f, e = system.forces(x, t, energies=True)
    torch.cuda.synchronize()
    return f.cpu().numpy().astype(np.float64), e.cpu().numpy()


def assert_same_pairs(got, want):
    got = np.sort(np.asarray(got, np.int64).reshape(-1, 2), axis=1)
    want = np.asarray(want, np.int64).reshape(-1, 2)
    key = lambda a: a[:, 0] * (1 << 32) + a[:, 1]
    kg, kw = np.unique(key(got)), np.unique(key(want))
    assert len(got) == len(kg) and np.array_equal(kg, kw), (len(kg), len(kw))


def check_energy_row(row, terms, tag=""):
    """One row of VP_E_* columns against the oracle's terms at the same positions."""
    scale_u = max(1.0, abs(terms["e_lj"]), abs(terms["e_rf"]), abs(terms["e_bond"]), abs(terms["e_angle"]))
    for k, col in (("e_lj", "lj"), ("e_rf", "rf"), ("e_bond", "bond"), ("e_angle", "angle"),
                   ("u_total", "total")):
        assert abs(row[E[col]] - terms[k]) <= 2e-5 * scale_u + 1e-9, (tag, k, row[E[col]], terms[k])
    for k, col in (("e_bias", "bias"), ("z", "z"), ("S", "S")):
        assert abs(row[E[col]] - terms[k]) <= 2e-5 * max(1.0, abs(terms[k])) + 1e-9, (tag, k, row[E[col]], terms[k])
    wo = np.array([terms[k] for k in WKEYS])
    wg = row[WCOLS]
    assert np.abs(wg - wo).max() <= 2e-5 * np.abs(wo).max() + 1e-6, (tag, wg, wo)


# ------------------------------------------------------------------ energies and virial
@pytest.mark.parametrize("name", ["tiny", "small", "tiny_rg", "no_solute", "tiny_const"])
def test_forces_energy_table_with_total_and_virial(name):
    say("energy table:", name)
    if name == "tiny_const":
        d = synth.tiny(seed=3, bias=synth.BIAS_CONST)
        d["const_force"] = np.random.default_rng(4).normal(size=(d["n_solute"], 3))
    else:
        d = {"tiny": lambda: dict(synth.tiny(seed=4), bias_k=0.05),
             "small": synth.small_chain_system,
             "tiny_rg": lambda: synth.tiny(seed=5, bias=synth.BIAS_RG),
             "no_solute": lambda: synth.lj_box(seed=3, n=500, box=2.6, r_cut=1.0)}[name]()
    # off the bonded rest state, so the bonded virial is not zero
    d = dict(d, x0=synth.perturbed(d, 0.004, 9)["x0"])
    system = vp.System([d])
    x = f32(d["x0"])
    t = 0.05
    fg, e = gpu_forces(system, [x], t)
    o = O.Oracle(d)
    st = o.init(grid(d["x0"]))
    fo, _, terms = o.forces(x, t, st)
    rel, mx = force_errors(fg, fo)
    say(f"  forces rel {rel:.2e}; W_gpu {e[0, WCOLS[0]]:.6e} vs {terms['w_xx']:.6e}")
    assert rel <= F_REL and mx <= F_MAX
    check_energy_row(e[0], terms, name)
    assert e[0, E["status"]] == 0.0


def test_constant_bias_energy_gradient_is_minus_force():
    """VpEnergy: the constant test force is the gradient of -sum F0.x, so the
    autograd gradient is -F for it too."""
    d = synth.tiny(seed=3, bias=synth.BIAS_CONST)
    d["const_force"] = np.random.default_rng(4).normal(size=(d["n_solute"], 3))
    system = vp.System([d])
    x = torch.from_numpy(f32(d["x0"]).astype(np.float32)).cuda().requires_grad_(True)
    e = vp.energy(x, system, 0.0)
    e.sum().backward()
    assert torch.equal(x.grad, -system.forces(x.detach()))


def test_energy_records_along_a_trajectory():
    """nst_out = 4: records at steps 0, 4, ..., 20, each against the oracle's
    energies and virial at the GPU's own (exact) positions of that step, the
    kinetic energy of its velocities and the functional vp_functional reports."""
    d = dict(synth.tiny(seed=6), bias_k=0.08, ramp_rate=30.0)
    system = vp.System([d], nst_out=4, steps_per_graph=3)
    o = O.Oracle(d)
    st = o.init(grid(d["x0"]))
    snaps = []
    for n in range(0, 21, 4):
        if n > 0:
            system.step_batch(4)
        x, v = system.trajectory_state()
        snaps.append((n, x, v, system.functional()[0]))
    rec = system.energy_records()
    say("records:", rec.shape)
    assert rec.shape == (1, len(snaps), len(vp.RECORD_COLUMNS))
    for k, (n, x, v, phi) in enumerate(snaps):
        row = rec[0, k]
        assert row[E["step"]] == n
        _, _, terms = o.forces(x, n * d["dt"], st)
        check_energy_row(row, terms, f"step {n}")
        ke = 0.5 * float(np.sum(d["mass"][:, None] * v * v))
        assert row[E["ke"]] == pytest.approx(ke, rel=1e-12)
        assert row[E["phi"]] == pytest.approx(phi, rel=1e-13, abs=1e-300)
        assert row[E["status"]] == 0.0


def test_energy_records_keep_the_latest_ones():
    d = synth.lj_box(seed=5, n=120, box=2.4, r_cut=1.0)
    system = vp.System([d, synth.with_seed(d, 77)], nst_out=2, out_capacity=3, steps_per_graph=5)
    system.step_batch(11)
    rec = system.energy_records()
    assert rec.shape[:2] == (2, 3)
    assert list(rec[0, :, E["step"]]) == [6.0, 8.0, 10.0] and list(rec[1, :, E["step"]]) == [6.0, 8.0, 10.0]
    with pytest.raises(vp.VpError):
        vp.System([d]).energy_records()


# ------------------------------------------------------------------ list overflow
def test_list_overflow_freezes_the_replica_and_is_never_selected():
    """A per-atom capacity too small for the dense replica: its pair lists are
    truncated, so it is flagged, frozen, has Phi = +inf and is skipped by the
    selection; the sparse replica runs on bitwise as it does alone, and
    vp_forces writes NaN forces and the flag for the dense one."""
    dense = dict(synth.tiny(seed=14), bias_k=0.2, ramp_rate=40.0)
    sparse = synth.lj_box(seed=21, n=24, box=4.0, r_cut=1.0)
    system = vp.System([dense, sparse], max_neighbors=24, steps_per_graph=4)
    obs = system.observables()
    say("overflow: status", obs[:, COL["status"]], "list max/cap", obs[:, COL["list_max"]], obs[:, COL["list_cap"]])
    assert int(obs[0, COL["status"]]) & vp.REPLICA_LIST_OVERFLOW
    assert int(obs[1, COL["status"]]) == 0
    x_before = system.get_state()[0].cpu().numpy()
    system.step_batch(9)
    phi = system.functional()
    assert math.isinf(phi[0]) and np.isfinite(phi[1])
    x_after = system.get_state()[0].cpu().numpy()
    a = system.offsets[1]
    assert np.array_equal(x_before[:a], x_after[:a])  # frozen
    best, bp = system.select_path()
    assert best == 1 and bp == phi[1]
    solo = vp.System([sparse], max_neighbors=24, steps_per_graph=4)
    solo.step_batch(9)
    assert np.array_equal(solo.get_state()[0].cpu().numpy(), x_after[a:])
    assert solo.functional()[0] == phi[1]
    f, e = gpu_forces(system, [f32(dense["x0"]), f32(sparse["x0"])])
    assert np.all(np.isnan(f[:a])) and np.all(np.isfinite(f[a:]))
    assert e[0, E["status"]] == vp.REPLICA_LIST_OVERFLOW and e[1, E["status"]] == 0
    obs = system.observables()
    assert obs[0, COL["eval_status"]] == vp.REPLICA_LIST_OVERFLOW and obs[1, COL["eval_status"]] == 0


def test_exact_mode_list_build_gives_exact_pairs_and_forces():
    """A staging capacity below what the quarter-box prefilter stages for the
    fullest blocks sends those into the exact-mode rebuild (only atoms within
    the list radius of one of the block's atoms are staged): pair set exact
    and forces within 1e-5 of the oracle.  (At 80% of the prefilter's largest
    count some blocks no longer fit even in exact mode: the replica is then
    flagged, as the overflow test checks.)"""
    d = synth.solvated_chain_12560()
    fast = vp.System([d]).observables()[0]
    cap = int(0.95 * fast[COL["stage_max"]])
    say(f"exact mode: fast staging max {fast[COL['stage_max']]:.0f}, cap {cap}")
    system = vp.System([d], stage_cap=cap)
    obs = system.observables()[0]
    say("  exact builds", obs[COL["exact_builds"]], "stage max", obs[COL["stage_max"]], "status", obs[COL["status"]])
    assert obs[COL["exact_builds"]] > 0 and obs[COL["status"]] == 0
    assert obs[COL["stage_max"]] <= cap
    o = O.Oracle(d)
    assert_same_pairs(system.debug_pairs(0), o.pairs(grid(d["x0"]), cells=True))
    x = f32(d["x0"])
    fg, _ = gpu_forces(system, [x])
    fo, _, _ = o.forces(x, 0.0, o.init(grid(d["x0"])))
    rel, mx = force_errors(fg, fo)
    say(f"  forces rel {rel:.2e} max {mx:.2e}")
    assert rel <= F_REL and mx <= F_MAX


# ------------------------------------------------------------------ ratchet in action
def _native_start(seed=7, n_water=60):
    """A tiny ratchet replica that starts at its product structure X_f, with
    waters placed around it by the generator: z(X_0) = 0 is the running
    minimum, so every later step has z > z_m and the ratchet acts."""
    d = dict(synth.tiny(seed=seed, bias=synth.BIAS_RMD_CONTACT), bias_k=2.0)
    ns = d["n_solute"]
    rng = np.random.default_rng(seed + 100)
    Ow, H = synth._place_waters(np.asarray(d["box"], float), n_water, d["x_final"], rng)
    x0 = np.array(d["x0"], float)
    x0[:ns] = d["x_final"]
    x0[ns::3], x0[ns + 1::3], x0[ns + 2::3] = Ow, H[:, 0], H[:, 1]
    d["x0"] = x0
    return d


def test_ratchet_acts_from_the_product_and_matches_the_oracle():
    d = _native_start()
    system = vp.System([d], steps_per_graph=5)
    system.step_batch(10)
    xg = system.get_state()[0].cpu().numpy()
    o = O.Oracle(d)
    x = grid(d["x0"])
    v = o.maxwell()
    st = o.init(x)
    zs = []
    for _ in range(10):
        o.run(x, v, st, 1)
        zs.append((st.z_last, st.z_m))
    phi_o = o.phi(st)
    say(f"ratchet: z_m {st.z_m:.3e}, z {st.z_last:.3e}, phi {phi_o:.4e}")
    assert phi_o > 0 and all(z > zm for z, zm in zs)
    dx = np.abs(xg - x).max()
    assert dx <= X_TOL, dx
    phi_g = system.functional()[0]
    assert abs(phi_g - phi_o) <= PHI_REL * phi_o, (phi_g, phi_o)
    obs = system.observables()[0]
    assert obs[COL["z_min"]] == pytest.approx(st.z_m, rel=1e-3, abs=1e-9)
    # the force of the current state (ratchet minimum of the trajectory)
    xs = f32(system.trajectory_state()[0])
    fg, e = gpu_forces(system, [xs], 10 * d["dt"])
    fo, fb, terms = o.forces(xs, 10 * d["dt"], st)
    assert np.abs(fb).max() > 0
    rel, mx = force_errors(fg, fo)
    assert rel <= F_REL and mx <= F_MAX
    assert e[0, E["bias"]] == pytest.approx(terms["e_bias"], rel=1e-4)


def test_contact_sum_range_on_the_gpu():
    """The construction of the oracle pin: one pair (0, 4) at r0 with
    min_sep = 3 gives z = 0.36; the pair (6, 9) at separation 3 adds nothing."""
    n = 12
    d = synth.lj_box(n=n, box=30.0, r_cut=1.0, charged=False)
    x = np.zeros((n, 3)) + 1.0
    x[:, 0] += 1.5 * np.arange(n)
    xf = x.copy()
    x[4] = x[0] + np.array([0.0, 0.75, 0.0])
    x[9] = x[6] + np.array([0.0, 0.0, 0.5])
    d.update(n_solute=n, x0=x, x_final=xf, bias=synth.BIAS_CONTACT, contact_min_sep=3, bias_k=0.1,
             ramp_rate=0.0)
    fg, e = gpu_forces(vp.System([d]), [x])
    assert e[0, E["z"]] == pytest.approx(0.36, rel=1e-6)


# ------------------------------------------------------------------ selection and RMSD
def _gap_threshold(values):
    """A threshold in the middle of the widest gap near the median of the
    values, so that no value lies within rounding of it."""
    v = np.sort(np.asarray(values))
    gaps = np.diff(v)
    lo, hi = len(v) // 4, max(len(v) // 4 + 1, 3 * len(v) // 4)
    k = lo + int(np.argmax(gaps[lo:hi]))
    assert gaps[k] > 1e-4 * max(1.0, abs(v[k])), v
    return 0.5 * (v[k] + v[k + 1])


def test_selection_with_finite_tolerances_matches_the_oracle():
    """Trials of a radius-of-gyration bias with finite reach_tol and reach_rmsd
    (to a given X_f): the reached flags, the selected trial and its functional
    are those of the oracle's brute-force selection over its own trajectories."""
    base = dict(synth.tiny(seed=32, bias=synth.BIAS_RG), bias_k=500.0, ramp_rate=20.0)
    base["x_final"] = synth.tiny(seed=32)["x_final"]   # same solute size: the RMSD reference
    reps = [synth.with_seed(base, 900 + r) for r in range(8)]
    nsteps = 30
    runs = []
    for d in reps:
        o = O.Oracle(d)
        x = grid(d["x0"])
        v = o.maxwell()
        st = o.init(x)
        o.run(x, v, st, nsteps)
        runs.append((o, x, st))
    dz = [abs(st.z_last - base["z_target"]) for _, _, st in runs]
    rm = [o.rmsd(x) for o, x, _ in runs]
    tol, rtol = _gap_threshold(dz), _gap_threshold(rm) * 1.0
    say(f"selection: |z - z_t| {np.round(dz, 4)} tol {tol:.4f}; rmsd {np.round(rm, 4)} tol {rtol:.4f}")
    reps = [dict(d, reach_tol=tol, reach_rmsd=rtol) for d in reps]
    reached_o, phi_o = [], []
    for d, (_, x, st) in zip(reps, runs):
        o = O.Oracle(d)
        reached_o.append(o.reached(st, x))
        phi_o.append(o.phi(st))
    rc, best_o, bp_o = O.select(phi_o, np.array(reached_o, np.uint8))
    system = vp.System(reps, steps_per_graph=10)
    system.step_batch(nsteps)
    obs = system.observables()
    reached_g = obs[:, COL["reached"]].astype(bool)
    say("  reached gpu", reached_g.astype(int), "oracle", np.array(reached_o, int))
    assert list(reached_g) == reached_o
    assert 0 < sum(reached_o) < len(reps)
    for r, (o, x, st) in enumerate(runs):
        assert obs[r, COL["rmsd"]] == pytest.approx(rm[r], abs=1e-5)
    best, bp = system.select_path()
    assert rc == 0 and best == best_o
    assert abs(bp - bp_o) <= PHI_REL * bp_o


def test_rmsd_kernel_matches_the_oracle_on_given_structures():
    """The GPU RMSD (singular values of the correlation matrix) against the
    oracle's (explicit quaternion rotation) on the same grid positions:
    a rotated and translated copy of X_f (zero) and perturbed copies."""
    d = synth.tiny(seed=12)
    ns = d["n_solute"]
    from scipy.stats import special_ortho_group
    R = special_ortho_group.rvs(3, random_state=3)
    reps = []
    for k, scale in enumerate((0.0, 0.05, 0.3)):
        x0 = np.array(d["x0"], float)
        rng = np.random.default_rng(k)
        x0[:ns] = (d["x_final"] - d["x_final"].mean(0)) @ R.T + x0[:ns].mean(0) + rng.normal(scale=scale, size=(ns, 3))
        reps.append(dict(d, x0=x0, bias_k=0.0))
    system = vp.System(reps)
    obs = system.observables()
    for r, dr in enumerate(reps):
        want = O.Oracle(dr).rmsd(grid(dr["x0"]))
        say(f"  rmsd gpu {obs[r, COL['rmsd']]:.9f} oracle {want:.9f}")
        assert obs[r, COL["rmsd"]] == pytest.approx(want, abs=1e-7)
    assert obs[0, COL["rmsd"]] < 1e-6
    assert np.isnan(vp.System([synth.lj_box(seed=2, n=50)]).observables()[0, COL["rmsd"]])


# ------------------------------------------------------------------ memory and streams
def test_device_memory_from_torch_caching_allocator():
    """vp_options.dev_alloc: every device buffer of the system comes from
    torch's caching allocator (the footprint shows up in memory_allocated and
    goes away with the system), and the trajectories are bitwise the same."""
    d = dict(synth.tiny(seed=11), bias_k=0.1, ramp_rate=20.0)
    torch.cuda.synchronize()
    base_mem = torch.cuda.memory_allocated()
    s_t = vp.System([d, synth.with_seed(d, 5)], torch_memory=True, steps_per_graph=5)
    grown = torch.cuda.memory_allocated() - base_mem
    held = s_t.device_bytes()
    say(f"torch allocator: library holds {held} B, torch memory_allocated grew {grown} B")
    assert held > 0 and grown >= held
    s_h = vp.System([d, synth.with_seed(d, 5)], steps_per_graph=5)
    assert s_h.device_bytes() == held
    for s in (s_t, s_h):
        s.step_batch(12)
    assert np.array_equal(s_t.get_state()[0].cpu().numpy(), s_h.get_state()[0].cpu().numpy())
    assert np.array_equal(s_t.functional(), s_h.functional())
    f_t, e_t = gpu_forces(s_t, [f32(d["x0"])] * 2)
    f_h, e_h = gpu_forces(s_h, [f32(d["x0"])] * 2)
    assert np.array_equal(f_t, f_h) and np.array_equal(e_t, e_h)
    torch.cuda.synchronize()
    before_close = torch.cuda.memory_allocated()
    s_t.close()
    assert before_close - torch.cuda.memory_allocated() >= held


def test_calls_on_different_streams_are_ordered():
    """Steps on one stream, then forces and state reads on another, without
    any synchronisation by the caller: the same bits as everything on one."""
    d = dict(synth.tiny(seed=12), bias_k=0.1, ramp_rate=20.0)
    x = torch.from_numpy(f32(d["x0"]).astype(np.float32)).cuda()
    a = vp.System([d], steps_per_graph=5)
    a.step_batch(15)
    fa = a.forces(x)
    xa, va = a.get_state()
    torch.cuda.synchronize()
    b = vp.System([d], steps_per_graph=5)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s1):
        b.step_batch(15)
    with torch.cuda.stream(s2):
        fb = b.forces(x)
        xb, vb = b.get_state()
    s2.synchronize()
    assert torch.equal(fa, fb) and torch.equal(xa, xb) and torch.equal(va, vb)
    assert b.functional()[0] == a.functional()[0]
