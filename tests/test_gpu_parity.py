"""GPU parity of the HIP path against the FP64 CPU oracle, through the C ABI.

Tolerances (stated per quantity):
  pair sets             exact (same FP32 membership predicate on both sides)
  Philox words          exact (first uniform), normals <= 5e-6 absolute
  forces                ||F_gpu - F_ora|| / ||F_ora|| <= 1e-5 and
                        max_i |dF_i| <= 1e-4 * rms|F|   (FP32 pair arithmetic)
  10-step trajectories  max |dx| <= 1e-4 nm
  functional            relative 1e-4 (plus 1e-12 absolute)
  dPhi/d(k, rho), force directional derivatives   relative 1e-4
Both sides start from the generator's inputs; the oracle is evaluated at the
positions the library holds (FP32 values on its 2^-22 nm grid) for
single-frame comparisons.
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


def say(*a):
    print(*a, flush=True)


GRID = 2.0 ** 22  # the library holds positions in units of 2^-22 nm


def f32(x):
    """FP32 positions on the library's grid, as float64.  The library rounds
    every position it receives to the nearest multiple of 2^-22 nm; below
    1 nm that moves an FP32 value by up to 3e-8 nm, which alone changes the
    net forces of stiff water by ~1e-5 relative, so the oracle is given the
    configuration the library evaluates.  The values are exact in FP32, so
    the library's rounding leaves them unchanged."""
    x = np.asarray(x, np.float32).astype(np.float64)
    return np.rint(x * GRID) / GRID


def x0_of(d):
    """Initial positions of a description as the library holds them (the FP64
    x0 rounded once to the 2^-22 nm grid)."""
    return np.rint(np.asarray(d["x0"], np.float64) * GRID) / GRID


def assert_same_pairs(got, want):
    """Exact equality of two pair sets, reported by counts and a few examples
    (a plain set comparison of millions of pairs makes pytest render a diff
    whose cost grows far faster than the sets)."""
    got = np.sort(np.asarray(got, np.int64).reshape(-1, 2), axis=1)
    want = np.asarray(want, np.int64).reshape(-1, 2)
    key = lambda a: a[:, 0] * (1 << 32) + a[:, 1]
    kg, kw = np.unique(key(got)), np.unique(key(want))
    dup = len(got) - len(kg)
    missing, extra = np.setdiff1d(kw, kg), np.setdiff1d(kg, kw)
    ok = dup == 0 and len(missing) == 0 and len(extra) == 0
    pairs = lambda k: [(int(v >> 32), int(v & 0xFFFFFFFF)) for v in k[:5]]
    assert ok, (f"{len(want)} oracle pairs: {len(missing)} missing {pairs(missing)}, "
                f"{len(extra)} extra {pairs(extra)}, {dup} duplicates")


def force_errors(fg, fo):
    rel = np.linalg.norm(fg - fo) / np.linalg.norm(fo)
    mx = np.abs(fg - fo).max() / np.sqrt(np.mean(np.sum(fo ** 2, 1)))
    return rel, mx


def gpu_forces(system, x_list, t=0.0):
    x = torch.from_numpy(np.concatenate([np.asarray(a, np.float32) for a in x_list])).cuda()
    f, e = system.forces(x, t, energies=True)
    torch.cuda.synchronize()
    return f.cpu().numpy().astype(np.float64), e.cpu().numpy()


@pytest.fixture(scope="module")
def solvated():
    return synth.solvated_chain_12560()


# ------------------------------------------------------------------ noise
def test_philox_normals_match_oracle():
    say("noise: seed 0x1234, 5000 atoms")
    seed = 0x1234_5678_9ABC
    out = vp.debug_noise(seed, 0, 17, 0, 5000).cpu().numpy().astype(np.float64)
    for a in range(0, 5000, 7):
        u = O.uniforms(seed, a, 17, 0)
        g = O.normals(seed, a, 17, 0)
        assert out[a, 3] == u[0]
        assert np.abs(out[a, :3] - g).max() <= 5e-6


# ------------------------------------------------------------------ pair sets
@pytest.mark.parametrize("name", ["tiny", "small", "lj_small_box"])
def test_pair_set_exact(name):
    say("pairs:", name)
    d = {"tiny": lambda: synth.tiny(seed=2), "small": synth.small_chain_system,
         "lj_small_box": lambda: synth.lj_box(seed=9, n=300, box=2.05, r_cut=1.0)}[name]()
    system = vp.System([d], skin=0.02 if name == "lj_small_box" else 0.0)
    assert system.observables()[0][5] == 0  # no list overflow
    assert_same_pairs(system.debug_pairs(0), O.Oracle(d).pairs(x0_of(d), cells=True))


def test_pair_set_exact_solvated(solvated):
    say("pairs: solvated")
    system = vp.System([solvated])
    assert system.observables()[0][5] == 0  # no list overflow
    want = O.Oracle(solvated).pairs(x0_of(solvated), cells=True)
    assert len(want) > 2_000_000
    assert_same_pairs(system.debug_pairs(0), want)


def _waters_not_consecutive(d):
    """The same system with its waters' atoms reordered (all oxygens, then
    all first hydrogens, then all second hydrogens), so that no three
    consecutive atoms form a water and the library lists every atom alone.
    Returns the description and new_of_old (old atom index -> new index)."""
    ns, n = int(d["n_solute"]), int(d["n_atoms"])
    w = np.arange(ns, n).reshape(-1, 3)
    old_of_new = np.concatenate([np.arange(ns), w[:, 0], w[:, 1], w[:, 2]])
    new_of_old = np.empty(n, np.int64)
    new_of_old[old_of_new] = np.arange(n)
    e = dict(d)
    for k in ("mass", "gamma", "charge", "sigma", "epsilon", "x0"):
        e[k] = np.ascontiguousarray(np.asarray(d[k])[old_of_new])
    for k in ("bonds", "angles", "excl"):
        e[k] = np.ascontiguousarray(new_of_old[np.asarray(d[k])].astype(np.int32))
    return e, new_of_old


def test_water_sites_and_single_atom_lists_agree():
    """Lists that name a water molecule by one entry and lists of single
    atoms (the same system with its water atoms reordered, so no site is
    found) hold the same pairs, give the same forces up to the FP32
    summation order, and the site lists are the shorter ones."""
    say("pairs/forces: water sites vs single atoms")
    d = synth.small_chain_system()
    e, new_of_old = _waters_not_consecutive(d)
    sa, sb = vp.System([d]), vp.System([e])
    col = list(vp.OBS).index("list_max")
    la, lb = sa.observables()[0][col], sb.observables()[0][col]
    say(f"  longest list: {la:.0f} entries with sites, {lb:.0f} without")
    assert la < 0.6 * lb
    pa = new_of_old[np.asarray(sa.debug_pairs(0), np.int64)]
    assert_same_pairs(pa, np.sort(np.asarray(sb.debug_pairs(0), np.int64), axis=1))
    x = f32(d["x0"])
    fa, _ = gpu_forces(sa, [x])
    fb, _ = gpu_forces(sb, [x[np.argsort(new_of_old)]])
    rel, mx = force_errors(fa[np.argsort(new_of_old)], fb)
    say(f"  forces rel {rel:.2e}, max {mx:.2e}")
    assert rel <= 2e-6 and mx <= 2e-5


# ------------------------------------------------------------------ forces
@pytest.mark.parametrize("name", ["tiny", "small", "tiny_rg", "no_solute"])
def test_forces_small(name):
    say("forces:", name)
    d = {"tiny": lambda: dict(synth.tiny(seed=4), bias_k=0.05),
         "small": synth.small_chain_system,
         "tiny_rg": lambda: synth.tiny(seed=5, bias=synth.BIAS_RG),
         "no_solute": lambda: synth.lj_box(seed=3, n=500, box=2.6, r_cut=1.0)}[name]()
    system = vp.System([d])
    x = f32(d["x0"])
    t = 0.05
    fg, e = gpu_forces(system, [x], t)
    o = O.Oracle(d)
    st = o.init(x)
    fo, fb, terms = o.forces(x, t, st)
    rel, mx = force_errors(fg, fo)
    say(f"  rel {rel:.2e} max {mx:.2e}")
    assert rel <= F_REL and mx <= F_MAX
    for k, col in (("e_lj", 0), ("e_rf", 1), ("e_bond", 2), ("e_angle", 3), ("e_bias", 4), ("z", 5),
                   ("z_ref", 6), ("S", 7)):
        scale = max(1.0, abs(terms["e_lj"]) if col < 4 else abs(terms[k]))
        assert abs(e[0, col] - terms[k]) <= 2e-5 * scale + 1e-9, (k, e[0, col], terms[k])


def test_bonded_groups_of_every_form():
    """Water molecules whose bonded terms take every form a three-atom group
    can hold, against the oracle: as generated (two bonds and the angle), bonds
    and angle written from the other end, no angle, the angle alone, and an
    extra H-H bond (four terms: evaluated per atom instead)."""
    say("forces: bonded groups of every form")
    d = dict(synth.small_chain_system())
    ns, n = int(d["n_solute"]), int(d["n_atoms"])
    bonds = [tuple(b) for b in np.asarray(d["bonds"]) if b[0] < ns]
    bk = [k for b, k in zip(np.asarray(d["bonds"]), d["bond_k"]) if b[0] < ns]
    br = [r for b, r in zip(np.asarray(d["bonds"]), d["bond_r0"]) if b[0] < ns]
    angles = [tuple(a) for a in np.asarray(d["angles"]) if a[0] < ns]
    ak = [k for a, k in zip(np.asarray(d["angles"]), d["angle_k"]) if a[0] < ns]
    at = [t for a, t in zip(np.asarray(d["angles"]), d["angle_theta0"]) if a[0] < ns]
    wb = {(int(b[0]), int(b[1])): (k, r) for b, k, r in zip(np.asarray(d["bonds"]), d["bond_k"], d["bond_r0"])
          if b[0] >= ns}
    wa = {int(a[1]): (k, t) for a, k, t in zip(np.asarray(d["angles"]), d["angle_k"], d["angle_theta0"])
          if a[1] >= ns}
    for w, o in enumerate(range(ns, n, 3)):
        h1, h2 = o + 1, o + 2
        (k1, r1), (k2, r2) = wb[(o, h1)], wb[(o, h2)]
        ka, ta = wa[o]
        form = w % 5
        if form in (0, 2, 3):
            bonds += [(o, h1), (o, h2)]; bk += [k1, k2]; br += [r1, r2]
        elif form == 1:
            bonds += [(h2, o), (h1, o)]; bk += [k2, k1]; br += [r2, r1]
        if form == 3:
            bonds.append((h1, h2)); bk.append(0.5 * k1); br.append(0.15)
        if form in (0, 3, 4):
            angles.append((h1, o, h2)); ak.append(ka); at.append(ta)
        elif form == 1:
            angles.append((h2, o, h1)); ak.append(ka); at.append(ta)
    d.update(bonds=np.asarray(bonds, np.int32), bond_k=np.asarray(bk), bond_r0=np.asarray(br),
             angles=np.asarray(angles, np.int32), angle_k=np.asarray(ak), angle_theta0=np.asarray(at))
    system = vp.System([d])
    # off the generated equilibrium geometry, so every bonded term carries force
    x = f32(np.asarray(d["x0"]) + np.random.default_rng(11).normal(0.0, 0.005, (n, 3)))
    fg, e = gpu_forces(system, [x], 0.0)
    o = O.Oracle(d)
    fo, _, terms = o.forces(x, 0.0, o.init(x))
    rel, mx = force_errors(fg, fo)
    say(f"  rel {rel:.2e} max {mx:.2e}; bond {terms['e_bond']:.3f} angle {terms['e_angle']:.3f}")
    assert rel <= F_REL and mx <= F_MAX
    for k, col in (("e_bond", 2), ("e_angle", 3)):
        assert abs(e[0, col] - terms[k]) <= 2e-5 * max(1.0, abs(terms["e_lj"])), (k, e[0, col], terms[k])


def test_forces_solvated_frame(solvated):
    say("forces: solvated frame")
    system = vp.System([solvated])
    x = f32(solvated["x0"])
    fg, e = gpu_forces(system, [x], 0.0)
    o = O.Oracle(solvated)
    st = o.init(x)
    fo, _, terms = o.forces(x, 0.0, st)
    rel, mx = force_errors(fg, fo)
    say(f"  rel {rel:.2e} max {mx:.2e}; z {e[0, 5]:.6f} vs {terms['z']:.6f}")
    assert rel <= F_REL and mx <= F_MAX
    assert abs(e[0, 5] - terms["z"]) <= 1e-5 * terms["z"]


def test_forces_bias_midramp(solvated):
    """Contact-map bias at t with z_ref between z(X_0) and the target."""
    say("forces: solvated bias mid-ramp")
    d = dict(solvated, bias_k=0.05, ramp_rate=20.0)
    system = vp.System([d])
    x0 = x0_of(d)
    x = f32(synth.perturbed(d, 0.01, 5)["x0"])
    fg, e = gpu_forces(system, [x], 0.02)
    o = O.Oracle(d)
    st = o.init(x0)
    fo, fb, terms = o.forces(x, 0.02, st)
    assert np.abs(fb).max() > 1.0
    rel, mx = force_errors(fg, fo)
    assert rel <= F_REL and mx <= F_MAX
    assert abs(e[0, 7] - terms["S"]) <= 1e-4 * terms["S"]


# ------------------------------------------------------------------ trajectories
def oracle_traj(d, nsteps):
    o = O.Oracle(d)
    x = x0_of(d)
    v = o.maxwell() if d.get("v0") is None else np.array(d["v0"], dtype=np.float64)
    st = o.init(x)
    o.run(x, v, st, nsteps)
    return o, x, v, st


@pytest.mark.parametrize("name,graph", [("tiny", True), ("tiny", False), ("small", True), ("rmd", True)])
def test_ten_step_trajectory(name, graph):
    say("trajectory:", name, "graph" if graph else "direct")
    d = {"tiny": lambda: dict(synth.tiny(seed=6), bias_k=0.08, ramp_rate=30.0),
         "small": synth.small_chain_system,
         "rmd": lambda: dict(synth.tiny(seed=7, bias=synth.BIAS_RMD_CONTACT), bias_k=0.5)}[name]()
    system = vp.System([d], use_graph=graph, steps_per_graph=4)
    system.step_batch(3)
    system.step_batch(7)
    xg, vg = system.get_state()
    xg = xg.cpu().numpy()
    o, x, v, st = oracle_traj(d, 10)
    dx = np.abs(xg - x).max()
    say(f"  max dx {dx:.2e}")
    assert dx <= X_TOL
    phi_g, phi_o = system.functional()[0], o.phi(st)
    assert abs(phi_g - phi_o) <= PHI_REL * abs(phi_o) + 1e-12, (phi_g, phi_o)
    obs = system.observables()[0]
    assert obs[0] == 10 and obs[5] == 0


def test_ten_step_trajectory_solvated(solvated):
    say("trajectory: solvated 10 steps")
    d = dict(solvated, bias_k=0.05, ramp_rate=50.0)
    system = vp.System([d])
    system.step_batch(10)
    xg, _ = system.get_state()
    o, x, v, st = oracle_traj(d, 10)
    dx = np.abs(xg.cpu().numpy() - x).max()
    say(f"  max dx {dx:.2e}")
    assert dx <= X_TOL
    phi_g, phi_o = system.functional()[0], o.phi(st)
    assert phi_o > 0
    assert abs(phi_g - phi_o) <= PHI_REL * abs(phi_o), (phi_g, phi_o)


def test_functional_constant_force_closed_form():
    """Phi = T |F0|^2 / (4 kT gamma m) for a constant bias on one atom."""
    say("functional: constant force")
    d = synth.tiny(seed=3, bias=synth.BIAS_CONST)
    cf = np.zeros((d["n_solute"], 3))
    F0 = np.array([3.0, -4.0, 12.0])
    cf[5] = F0
    d["const_force"] = cf
    system = vp.System([d])
    system.step_batch(17)
    T = 17 * d["dt"]
    expect = T * float(F0 @ F0) / (4 * d["kT"] * d["gamma"][5] * d["mass"][5])
    assert system.functional()[0] == pytest.approx(expect, rel=1e-6)


# ------------------------------------------------------------------ batching
def test_batch_matches_solo_runs_bitwise():
    say("batch vs solo")
    base = dict(synth.tiny(seed=11), bias_k=0.1, ramp_rate=20.0)
    reps = [synth.with_seed(base, 100 + r) for r in range(3)] + [dict(synth.small_chain_system())]
    batch = vp.System(reps, steps_per_graph=5)
    batch.step_batch(12)
    xb, vb = batch.get_state()
    phib = batch.functional()
    xb, vb = xb.cpu().numpy(), vb.cpu().numpy()
    for r, d in enumerate(reps):
        solo = vp.System([d], steps_per_graph=5)
        solo.step_batch(12)
        xs, vs = solo.get_state()
        a, b = batch.offsets[r], batch.offsets[r + 1]
        assert np.array_equal(xs.cpu().numpy(), xb[a:b])
        assert np.array_equal(vs.cpu().numpy(), vb[a:b])
        assert solo.functional()[0] == phib[r]


def test_run_twice_and_graph_equal_direct_bitwise():
    say("determinism")
    d = dict(synth.tiny(seed=12), bias_k=0.1, ramp_rate=20.0)
    outs = []
    for graph in (True, True, False):
        s = vp.System([d], use_graph=graph, steps_per_graph=6)
        s.step_batch(15)
        x, v = s.get_state()
        outs.append((x.cpu().numpy(), v.cpu().numpy(), s.functional()[0]))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1]) and o[2] == outs[0][2]


def test_heterogeneous_batch_forces():
    say("heterogeneous batch forces")
    reps = [dict(synth.tiny(seed=21), bias_k=0.05), synth.small_chain_system(),
            synth.lj_box(seed=4, n=777, box=3.0, r_cut=1.2),
            synth.tiny(seed=22, n_solute=30, n_water=101, box=2.3, r_cut=0.95, bias=synth.BIAS_RG)]
    system = vp.System(reps)
    xs = [f32(d["x0"]) for d in reps]
    fg, e = gpu_forces(system, xs, 0.0)
    for r, d in enumerate(reps):
        o = O.Oracle(d)
        st = o.init(xs[r])
        fo, _, _ = o.forces(xs[r], 0.0, st)
        a, b = system.offsets[r], system.offsets[r + 1]
        rel, mx = force_errors(fg[a:b], fo)
        assert rel <= F_REL and mx <= F_MAX, (r, rel, mx)


def test_selection_picks_least_functional():
    say("selection")
    base = dict(synth.tiny(seed=13), bias_k=0.2, ramp_rate=40.0)
    reps = [synth.with_seed(base, 500 + r) for r in range(6)]
    system = vp.System(reps)
    system.step_batch(20)
    phi = system.functional()
    best, bp = system.select_path()
    assert best == int(np.argmin(phi)) and bp == phi[best]
    elig = np.ones(6, np.uint8)
    elig[best] = 0
    b2, _ = system.select_path(elig)
    assert b2 != best and phi[b2] == np.min(np.where(elig > 0, phi, np.inf))
    assert system.select_path(np.zeros(6, np.uint8))[0] == -1
    # the oracle reproduces each trajectory's functional
    for r in (0, best):
        o, _, _, st = oracle_traj(reps[r], 20)
        assert abs(phi[r] - o.phi(st)) <= PHI_REL * o.phi(st)


def test_unstable_replica_is_flagged_and_never_selected():
    say("instability")
    base = dict(synth.tiny(seed=14), bias_k=0.2, ramp_rate=40.0)
    bad = dict(base)
    x0 = base["x0"].copy()
    x0[20] = x0[1] + 0.01  # two non-bonded solute atoms 0.1 A apart
    bad["x0"] = x0
    system = vp.System([base, bad, synth.with_seed(base, 77)])
    system.step_batch(5)
    phi = system.functional()
    obs = system.observables()
    assert math.isinf(phi[1]) and int(obs[1, 5]) & vp.REPLICA_UNSTABLE
    assert np.isfinite(phi[0]) and np.isfinite(phi[2])
    assert system.select_path()[0] in (0, 2)
    solo = vp.System([base])
    solo.step_batch(5)
    xs, _ = solo.get_state()
    xb, _ = system.get_state()
    assert np.array_equal(xs.cpu().numpy(), xb.cpu().numpy()[: base["n_atoms"]])


def test_autograd_energy_backward_is_minus_force():
    say("autograd")
    d = dict(synth.tiny(seed=15), bias_k=0.05)
    system = vp.System([d])
    x = torch.from_numpy(d["x0"].astype(np.float32)).cuda().requires_grad_(True)
    e = vp.energy(x, system, 0.0)
    e.sum().backward()
    f = system.forces(x.detach())
    assert torch.equal(x.grad, -f)


# ------------------------------------------- derivative w.r.t. (bias_k, ramp_rate)
G_REL = 1e-4  # functional gradients and their ingredients, relative to the FP64 oracle


def _tangent_case(name):
    return {"tiny": lambda: dict(synth.tiny(seed=31), bias_k=0.08, ramp_rate=30.0),
            "tiny_rg": lambda: dict(synth.tiny(seed=32, bias=synth.BIAS_RG), ramp_rate=20.0),
            "small": synth.small_chain_system,
            "solvated": lambda: dict(synth.solvated_chain_12560(), bias_k=0.05, ramp_rate=50.0)}[name]()


@pytest.mark.parametrize("name", ["tiny", "tiny_rg", "small", "solvated"])
def test_force_directional_derivative(name):
    """-H_U dx + bias terms along two random displacements against the oracle's
    dual-number derivative at the same (grid) positions."""
    say("force derivative:", name)
    d = _tangent_case(name)
    system = vp.System([d], tangent=True)
    x = f32(d["x0"])
    rng = np.random.default_rng(7)
    dx = rng.normal(scale=1e-2, size=(2, d["n_atoms"], 3)).astype(np.float32)
    t = 0.003
    out = system.force_dir(torch.from_numpy(x.astype(np.float32)).cuda(), torch.from_numpy(dx).cuda(), t)
    torch.cuda.synchronize()
    out = out.cpu().numpy().astype(np.float64)
    o = O.Oracle(d)
    st = o.init(x0_of(d))
    _, fdot, _, _, _ = o.forces_dir(x, dx.astype(np.float64), False, t, st)
    for k in range(2):
        rel = np.linalg.norm(out[k] - fdot[k]) / np.linalg.norm(fdot[k])
        say(f"  direction {k}: rel {rel:.2e}")
        assert rel <= G_REL


@pytest.mark.parametrize("name,nsteps", [("tiny", 20), ("tiny_rg", 20), ("small", 20), ("solvated", 10)])
def test_functional_gradient(name, nsteps):
    """dPhi/d(bias_k, ramp_rate) carried by the tangents along a trajectory,
    against the oracle's dual-number run of the same trajectory."""
    say("functional gradient:", name, nsteps)
    d = _tangent_case(name)
    system = vp.System([d], tangent=True, steps_per_graph=5)
    system.step_batch(nsteps)
    phi, grad = system.functional(gradient=True)
    o = O.Oracle(d)
    x = x0_of(d)
    v = o.maxwell()
    st = o.init(x)
    pd = o.init_tangent(x, st)
    xt = np.zeros((2, o.n, 3))
    vt = np.zeros((2, o.n, 3))
    assert o.run_tangent(x, v, st, xt, vt, pd, nsteps) == 0
    go = o.phi_grad(st, pd)
    say(f"  phi {phi[0]:.6e} vs {o.phi(st):.6e}; grad {grad[0]} vs {go}")
    for k in range(2):
        assert abs(grad[0, k] - go[k]) <= G_REL * abs(go[k]), (k, grad[0, k], go[k])


def test_tangents_leave_the_trajectory_unchanged():
    say("tangents: primal unchanged")
    d = _tangent_case("tiny")
    outs = []
    for tan in (False, True):
        s = vp.System([d], tangent=tan, steps_per_graph=6)
        s.step_batch(14)
        x, v = s.get_state()
        outs.append((x.cpu().numpy(), v.cpu().numpy(), s.functional()[0]))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


def test_tangent_batch_matches_solo_runs_bitwise():
    say("tangents: batch vs solo")
    base = _tangent_case("tiny")
    reps = [synth.with_seed(base, 200 + r) for r in range(3)] + [_tangent_case("tiny_rg")]
    batch = vp.System(reps, tangent=True, steps_per_graph=5)
    batch.step_batch(12)
    phib, gb = batch.functional(gradient=True)
    for r, d in enumerate(reps):
        solo = vp.System([d], tangent=True, steps_per_graph=5)
        solo.step_batch(12)
        phis, gs = solo.functional(gradient=True)
        assert phis[0] == phib[r] and np.array_equal(gs[0], gb[r])


def test_tangent_errors():
    say("tangents: errors")
    d = _tangent_case("tiny")
    s = vp.System([d])
    with pytest.raises(vp.VpError):
        s.functional(gradient=True)
    with pytest.raises(vp.VpError):
        vp.System([dict(synth.tiny(seed=7, bias=synth.BIAS_RMD_CONTACT), bias_k=0.5)], tangent=True)


# ------------------------------------------- uneven batch (5,000-40,000 atoms, rc 0.9 / 1.2)
@pytest.fixture(scope="module")
def uneven_subset():
    # three replicas of the uneven batch: 5,028 atoms rc 1.2; 5,135 rc 0.9; 10,312 rc 1.2
    return synth.uneven_batch(only=(9, 15, 26))


def test_uneven_batch_forces_and_pairs(uneven_subset):
    say("uneven batch: forces and pairs", [int(d["n_atoms"]) for d in uneven_subset])
    system = vp.System(uneven_subset)
    xs = [f32(d["x0"]) for d in uneven_subset]
    fg, e = gpu_forces(system, xs, 0.0)
    for r, d in enumerate(uneven_subset):
        o = O.Oracle(d)
        st = o.init(x0_of(d))
        fo, _, _ = o.forces(xs[r], 0.0, st)
        a, b = system.offsets[r], system.offsets[r + 1]
        rel, mx = force_errors(fg[a:b], fo)
        say(f"  replica {r}: {d['n_atoms']} atoms rc {d['r_cut']}: rel {rel:.2e} max {mx:.2e}")
        assert rel <= F_REL and mx <= F_MAX
    # the exact pair set of the first rc 1.2 replica (trajectory lists at creation)
    r = next(i for i, d in enumerate(uneven_subset) if d["r_cut"] > 1.0)
    assert_same_pairs(system.debug_pairs(r), O.Oracle(uneven_subset[r]).pairs(x0_of(uneven_subset[r]), cells=True))
    obs = system.observables()
    assert np.all(obs[:, 5] == 0)


def test_uneven_batch_runs_and_matches_solo(uneven_subset):
    say("uneven batch: 200 steps, batch vs solo")
    batch = vp.System(uneven_subset, steps_per_graph=20)
    batch.step_batch(200)
    obs = batch.observables()
    col = {k: i for i, k in enumerate(vp.OBS)}
    say("  stage max/cap", obs[:, col["stage_max"]], obs[:, col["stage_cap"]],
        "list max/cap", obs[:, col["list_max"]], obs[:, col["list_cap"]],
        "exact builds", obs[:, col["exact_builds"]])
    assert np.all(obs[:, col["status"]] == 0)
    assert np.all(np.isfinite(batch.functional()))
    xb, _ = batch.get_state()
    xb = xb.cpu().numpy()
    r = 1
    solo = vp.System([uneven_subset[r]], steps_per_graph=20)
    solo.step_batch(200)
    xs, _ = solo.get_state()
    a, b = batch.offsets[r], batch.offsets[r + 1]
    assert np.array_equal(xs.cpu().numpy(), xb[a:b])


def s_dot_term_scale(o, d, x, xt, state):
    """Size of the terms of dS/dtheta_k = sum_i 2 F_b,i . dF_b,i/dtheta_k / (gamma_i m_i)
    at (x, xt): sum_i 2 |F_b,i| |dF_b,i/dtheta_k| / (gamma_i m_i), with the bias
    force F_b from the oracle and its derivative as the total force's minus
    that of the same system without bias.  Late in a segment the tangents
    have grown by many orders of magnitude and the terms cancel, so the
    rounding error of the sum is bounded relative to this size, not to the
    sum itself."""
    t = state.step * d["dt"]
    _, fb, _ = o.forces(x, t=t, state=state)
    _, fdot, _, _, _ = o.forces_dir(x, xt, theta=True, t=t, state=state)
    free = O.Oracle(dict(d, bias_k=0.0))
    _, fdot_u, _, _, _ = free.forces_dir(x, xt, theta=False, t=t, state=state)
    w = 2.0 / (np.asarray(d["gamma"], np.float64) * np.asarray(d["mass"], np.float64))
    nb = np.linalg.norm(fb, axis=1)
    return np.array([np.sum(w * nb * np.linalg.norm(fdot[k] - fdot_u[k], axis=1)) for k in range(2)])


def test_functional_gradient_late_in_a_2000_step_segment():
    """Trials of the 12,560-atom system with the 2,000-step ramp: after 1,990
    GPU steps the oracle continues the GPU's exact state and tangents for 10
    steps; the tangents and the increments of the derivative accumulators
    must agree (the trajectories themselves diverge chaotically over 2,000
    steps, so only a continuation from the same state is comparable).  The
    increments are sums of terms that cancel: their tolerance is G_REL of the
    summed term sizes over the ten steps (bounded by ten times the larger of
    the sizes at the two ends)."""
    say("functional gradient: steps 1990-2000 of a 2000-step segment")
    reps = synth.derivative_batch(n_rep=2)
    system = vp.System(reps, tangent=True, steps_per_graph=10)
    system.step_batch(1990)
    x, v, xt, vt, pd0 = system.trajectory_state(tangents=True)
    system.step_batch(10)
    x1, _, xt1, _, pd1 = system.trajectory_state(tangents=True)
    for r, d in enumerate(reps):
        a, b = system.offsets[r], system.offsets[r + 1]
        o = O.Oracle(d)
        st = o.init(x0_of(d))        # z(X_0) of the ramp
        st.step = 1990
        xr, vr = x[a:b].copy(), v[a:b].copy()
        xtr, vtr = np.ascontiguousarray(xt[:, a:b]), np.ascontiguousarray(vt[:, a:b])
        pd = np.zeros(4)
        scale0 = s_dot_term_scale(o, d, xr, xtr, st)
        assert o.run_tangent(xr, vr, st, xtr, vtr, pd, 10) == 0
        scale = 10.0 * np.maximum(scale0, s_dot_term_scale(o, d, xr, xtr, st))
        dx = np.abs(xr - x1[a:b]).max()
        rel_t = [np.linalg.norm(xtr[k] - xt1[k, a:b]) / np.linalg.norm(xtr[k]) for k in range(2)]
        inc = pd1[r, :2] - pd0[r, :2]
        say(f"  replica {r}: 10-step dx {dx:.2e}, tangent rel {rel_t[0]:.2e} {rel_t[1]:.2e}, "
            f"dS/dtheta sums {inc} vs {pd[:2]}, term sizes {scale}, "
            f"error / term size {np.abs(inc - pd[:2]) / scale}")
        assert dx <= X_TOL
        for k in range(2):
            assert rel_t[k] <= G_REL
            assert abs(inc[k] - pd[k]) <= G_REL * scale[k]


# ------------------------------------------------------------------ tile shapes
def test_every_force_tile_shape_gives_the_same_bits(uneven_subset):
    """The force kernel sums list chunk c of an atom into partial sum c mod 16
    whatever its tile shape, so forces and energies agree bit for bit."""
    reps = list(uneven_subset) + [synth.tiny(seed=3), synth.lj_box()]
    say("tile shapes: bitwise agreement", [int(d["n_atoms"]) for d in reps])
    xs = [f32(d["x0"]) for d in reps]
    ref = None
    for k in range(vp.FORCE_SHAPES):
        f, e = gpu_forces(vp.System(reps, force_shape=k), xs, 0.0)
        if ref is None:
            ref = (f, e)
            continue
        assert np.array_equal(f, ref[0]), k
        assert np.array_equal(e, ref[1]), k


def test_autotuned_uneven_batch(uneven_subset):
    say("autotune: uneven batch buckets")
    tuned = vp.System(uneven_subset, autotune=True, steps_per_graph=10)
    buckets, split = tuned.tile_buckets()
    for b in buckets:
        say(f"  rc {b['r_cut']} 2^{b['log2_atoms']}: {b['replicas']} replicas, {b['blocks']} blocks, "
            f"tile {b['tile']}, ms {['%.4f' % t for t in b['ms']]}")
    say("  split launches:", split)
    keys = sorted((d["r_cut"], int(np.floor(np.log2(d["n_atoms"])))) for d in uneven_subset)
    assert sorted((b["r_cut"], b["log2_atoms"]) for b in buckets) == sorted(set(keys))
    assert sum(b["replicas"] for b in buckets) == len(uneven_subset)
    for b in buckets:
        assert 0 <= b["shape"] < vp.FORCE_SHAPES and all(t > 0 for t in b["ms"])
        if not split:
            assert b["shape"] == buckets[0]["shape"]
    plain = vp.System(uneven_subset, steps_per_graph=10)
    for s in (tuned, plain):
        s.step_batch(40)
    assert np.array_equal(tuned.get_state()[0].cpu().numpy(), plain.get_state()[0].cpu().numpy())
    b0, _ = plain.tile_buckets()
    assert all(b["shape"] == 0 and b["ms"] == [0.0] * vp.FORCE_SHAPES for b in b0)


def test_default_list_parameters_per_replica(uneven_subset):
    """Default interval: the largest power of two in which a 5-sigma-fast
    lightest atom moves less than half the largest admissible skin (at most
    0.14 nm, less where the staged neighbourhood or half the box limits it);
    default skin: just enough for that interval.  Given values are taken as
    they are."""
    say("list parameters per replica")
    reps = [synth.solvated_chain_12560(), synth.small_chain_system(), synth.tiny(seed=3)] + list(uneven_subset)
    obs = vp.System(reps).observables()
    col = {k: i for i, k in enumerate(vp.OBS)}
    for r, d in enumerate(reps):
        skin, nst = obs[r, col["skin"]], int(obs[r, col["nstlist"]])
        step = 5.0 * np.sqrt(d["kT"] / float(np.min(d["mass"]))) * d["dt"]
        say(f"  replica {r}: {d['n_atoms']} atoms rc {d['r_cut']} dt {d['dt']}: skin {skin:.2f} nstlist {nst}")
        assert nst in (1, 2, 4, 8, 16, 32)
        assert 0.02 <= skin <= 0.14 + 1e-12 and d["r_cut"] + skin < 0.5 * min(d["box"])
        assert nst * step <= 0.49 * skin + 1e-12            # the interval fits the skin
        assert obs[r, col["stage_max"]] <= obs[r, col["stage_cap"]]
    assert abs(obs[0, col["skin"]] - 0.13) < 1e-12 and int(obs[0, col["nstlist"]]) == 8
    assert int(obs[1, col["nstlist"]]) == 16            # the 1,512-atom system at 0.5 fs
    given = vp.System(reps[:1], nstlist=4, skin=0.1).observables()
    assert abs(given[0, col["skin"]] - 0.1) < 1e-12 and int(given[0, col["nstlist"]]) == 4


def test_split_launch_plan_matches_single_launch(uneven_subset):
    """Every size bucket on its own tile shape (one launch per shape over
    per-bucket block lists) gives bitwise the trajectories of the plain
    single-shape launch: each block is covered exactly once."""
    reps = list(uneven_subset) + [synth.tiny(seed=3)]
    say("split launch plan", [int(d["n_atoms"]) for d in reps])
    plain = vp.System(reps, steps_per_graph=10)
    split = vp.System(reps, steps_per_graph=10)
    buckets, _ = split.tile_buckets()
    shapes = [(i + 1) % vp.FORCE_SHAPES for i in range(len(buckets))]
    split.set_tiles(shapes)
    got, was_split = split.tile_buckets()
    assert was_split and [b["shape"] for b in got] == shapes
    for s in (plain, split):
        s.step_batch(30)
    assert np.array_equal(plain.get_state()[0].cpu().numpy(), split.get_state()[0].cpu().numpy())
    assert np.array_equal(plain.functional(), split.functional())
    xs = [f32(d["x0"]) for d in reps]
    fa, ea = gpu_forces(plain, xs, 0.0)
    fb, eb = gpu_forces(split, xs, 0.0)
    assert np.array_equal(fa, fb) and np.array_equal(ea, eb)
    with pytest.raises(vp.VpError):
        split.set_tiles(shapes[:-1])


def test_forces_match_central_differences():
    """Force kernel against central differences (h = 1e-5 nm) on a 300-atom
    subset of the 1,512-atom system: of the oracle's FP64 energy (the
    definition of U; the difference quotient is exact to ~1e-8 here), and of
    the GPU's own energies.  Every displaced configuration is one replica of
    a single batched evaluation.  Atoms with a pair within 2h of the cutoff
    are left out: the potential-shifted LJ and the reaction field are
    continuous at r_c but their forces jump there (~2 kJ/mol/nm for an O-O
    pair), so a difference quotient across r_c is not a derivative.

    The GPU energies are FP64 sums of pair terms computed from FP32
    intermediates (relative rounding ~2e-7 per term); moving one atom changes
    the rounding of its ~300 pair terms (Coulomb pairs up to ~300 kJ/mol), so
    E(x+h) - E(x-h) carries ~1e-4 to 1e-3 kJ/mol of noise against a
    difference of ~F 2h = 2e-2 kJ/mol: that check can only hold to a few
    times 1e-2."""
    d = synth.small_chain_system()
    n, ns = int(d["n_atoms"]), int(d["n_solute"])
    rng = np.random.default_rng(7)
    x0 = f32(d["x0"])
    h = 1e-5
    box = np.asarray(d["box"], float)

    def straddles_cutoff(a):
        dd = x0.astype(np.float64) - x0[a].astype(np.float64)
        dd -= box * np.rint(dd / box)
        r = np.sqrt((dd ** 2).sum(1))
        r[a] = np.inf
        return bool(np.any(np.abs(r - d["r_cut"]) < 2 * h))

    solute = [a for a in range(ns) if not straddles_cutoff(a)]
    pool = [a for a in rng.permutation(np.arange(ns, n)) if not straddles_cutoff(a)]
    atoms = np.array(solute + sorted(pool[:300 - len(solute)]), dtype=np.int64)
    assert len(atoms) == 300
    axis = rng.integers(0, 3, len(atoms))  # one Cartesian direction per atom
    xs = [x0]
    for a, k in zip(atoms, axis):
        for sgn in (1.0, -1.0):
            x = x0.copy()
            x[a, k] = np.float32(float(x0[a, k]) + sgn * h)
            xs.append(x)
    say("forces vs central differences:", len(xs), "configurations")
    f, e = gpu_forces(vp.System([d] * len(xs)), xs)
    o = O.Oracle(d)
    st = o.init(x0_of(d))
    terms = ("e_lj", "e_rf", "e_bond", "e_angle", "e_bias")
    e_ora = np.array([sum(o.forces(x.astype(np.float64), 0.0, st)[2][k] for k in terms) for x in xs])
    e_gpu = e[:, :5].sum(1)
    fd_ora = np.zeros(len(atoms))
    fd_gpu = np.zeros(len(atoms))
    for i, (a, k) in enumerate(zip(atoms, axis)):
        rp = 1 + 2 * i
        step = float(xs[rp][a, k]) - float(xs[rp + 1][a, k])  # the displacement actually taken
        fd_ora[i] = -(e_ora[rp] - e_ora[rp + 1]) / step
        fd_gpu[i] = -(e_gpu[rp] - e_gpu[rp + 1]) / step
    fa = f[:n][atoms, axis]
    rms = np.sqrt(np.mean(fa ** 2))
    rel_o, mx_o = np.linalg.norm(fa - fd_ora) / np.linalg.norm(fa), np.abs(fa - fd_ora).max() / rms
    rel_g, mx_g = np.linalg.norm(fa - fd_gpu) / np.linalg.norm(fa), np.abs(fa - fd_gpu).max() / rms
    say(f"  vs oracle energies: rel {rel_o:.2e} max {mx_o:.2e}; vs GPU energies: rel {rel_g:.2e} max {mx_g:.2e}")
    assert rel_o <= F_REL and mx_o <= F_MAX
    assert rel_g <= 3e-2 and mx_g <= 1e-1


def test_degenerate_replicas_in_a_batch():
    """A one-atom replica (empty lists), a lone pair inside the cutoff and a
    256-atom replica that fills its tile exactly, batched with a ragged one:
    forces and 10-step trajectories against the oracle, pair sets exact."""
    one = synth.lj_box(seed=11, n=1)
    two = synth.lj_box(seed=12, n=2)
    two["x0"] = np.array([[1.0, 1.0, 1.0], [1.37, 1.1, 0.95]])
    full_tile = synth.lj_box(seed=13, n=256)
    ragged = synth.lj_box(seed=14, n=199)
    reps = [one, two, full_tile, ragged]
    say("degenerate replicas:", [d["n_atoms"] for d in reps])
    system = vp.System(reps, steps_per_graph=5)
    xs = [f32(d["x0"]) for d in reps]
    fg, _ = gpu_forces(system, xs, 0.0)
    for r, d in enumerate(reps):
        a, b = system.offsets[r], system.offsets[r + 1]
        o = O.Oracle(d)
        fo, _, _ = o.forces(xs[r], 0.0, o.init(x0_of(d)))
        if r == 0:
            assert np.all(fg[a:b] == 0.0) and np.all(fo == 0.0)
        else:
            rel, mx = force_errors(fg[a:b], fo)
            say(f"  replica {r}: rel {rel:.2e} max {mx:.2e}")
            assert rel <= F_REL and mx <= F_MAX
        assert_same_pairs(system.debug_pairs(r), o.pairs(x0_of(d), cells=True))
    assert np.array_equal(fg[system.offsets[1]], -fg[system.offsets[1] + 1])  # the lone pair: action = reaction
    system.step_batch(10)
    xg = system.get_state()[0].cpu().numpy()
    for r, d in enumerate(reps):
        a, b = system.offsets[r], system.offsets[r + 1]
        _, x, _, _ = oracle_traj(d, 10)
        dx = np.abs(xg[a:b] - x).max()
        say(f"  replica {r}: 10-step max dx {dx:.2e}")
        assert dx <= X_TOL
    assert np.all(system.observables()[:, 5] == 0)
