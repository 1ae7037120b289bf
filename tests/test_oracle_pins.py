"""Pins of the FP64 oracle against facts other than itself: published
known-answer vectors, closed forms, invariances, special cases that reduce to
textbook results, finite differences and brute force on tiny inputs.

Each test names the passage of the paper (or the published definition) it
follows.  These run on the CPU only.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

from paper_1405_6104_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def two_body(r, sig=(0.315, 0.315), eps=(0.636, 0.636), q=(0.0, 0.0), rc=1.0, eps_rf=78.0, L=6.0):
    d = synth.lj_box(n=2, box=L, r_cut=rc, charged=False)
    d.update(sigma=np.array(sig, float), epsilon=np.array(eps, float), charge=np.array(q, float),
             eps_rf=eps_rf)
    d["x0"] = np.array([[1.0, 1.0, 1.0], [1.0 + r, 1.0, 1.0]])
    return d


def energy(o, x, t=0.0, st=None):
    _, _, tt = o.forces(x, t, st)
    return tt["e_lj"] + tt["e_rf"] + tt["e_bond"] + tt["e_angle"] + tt["e_bias"]


# --------------------------------------------------------------- noise
def test_philox_known_answers(oracle_mod):
    """Philox4x32-10 reproduces the published known-answer vectors."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        assert oracle_mod.philox(v[0:4], v[4:6]) == v[6:10]


def test_uniforms_exact_fp32_and_open_interval(oracle_mod):
    for a in range(200):
        u = oracle_mod.uniforms(0x1234_5678_9ABC_DEF0, a, 7, 0)
        assert np.all(u > 0) and np.all(u < 1)
        assert np.all(u.astype(np.float32).astype(np.float64) == u)


def test_normals_are_standard_normal(oracle_mod):
    """White noise of Eq. Lang: Box-Muller normals pass a KS test against
    N(0,1) and are uncorrelated across components, atoms and steps."""
    g = np.array([oracle_mod.normals(99, a, s, 0) for a in range(300) for s in range(20)])
    for k in range(3):
        assert scipy.stats.kstest(g[:, k], "norm").pvalue > 1e-3
    c = np.corrcoef(g.T)
    assert np.all(np.abs(c - np.eye(3)) < 0.05)
    g1 = np.array([oracle_mod.normals(99, a, 0, 1) for a in range(2000)])
    g0 = np.array([oracle_mod.normals(99, a, 0, 0) for a in range(2000)])
    assert abs(np.corrcoef(g0[:, 0], g1[:, 0])[0, 1]) < 0.08  # tags are independent streams


# --------------------------------------------------------------- pair law
def test_lj_minimum_and_well_depth(oracle_mod):
    """Lennard-Jones: zero force at 2^(1/6) sigma_ij, well depth eps_ij,
    Lorentz-Berthelot mixing (sigma arithmetic, eps geometric)."""
    s1, s2, e1, e2 = 0.30, 0.38, 0.4, 0.9
    sij, eij = 0.5 * (s1 + s2), math.sqrt(e1 * e2)
    rmin = 2 ** (1 / 6) * sij
    o = oracle_mod.Oracle(two_body(rmin, (s1, s2), (e1, e2)))
    f, _, _ = o.forces(o.desc["x0"])
    assert np.abs(f).max() < 1e-10
    oz = oracle_mod.Oracle(two_body(sij, (s1, s2), (e1, e2)))
    assert energy(oz, oz.desc["x0"]) - energy(o, o.desc["x0"]) == pytest.approx(eij, rel=1e-12)


def test_lj_shift_continuity_and_cutoff(oracle_mod):
    """Potential-shifted LJ vanishes continuously at the cutoff and is zero beyond."""
    for r, expect_small in ((1.0 - 1e-9, True), (1.0 + 1e-6, True)):
        o = oracle_mod.Oracle(two_body(r))
        assert abs(energy(o, o.desc["x0"])) < 1e-8
    o = oracle_mod.Oracle(two_body(1.05))
    f, _, t = o.forces(o.desc["x0"])
    assert t["e_lj"] == 0.0 and np.all(f == 0.0)


def test_rf_special_cases(oracle_mod):
    """Reaction field: eps_rf = 1 reduces to plain Coulomb shifted to zero at
    rc; a conducting boundary (eps_rf -> inf) makes the force vanish at rc."""
    fq = 138.935458
    q = (0.5, -0.7)
    r, rc = 0.43, 1.0
    o = oracle_mod.Oracle(two_body(r, eps=(0, 0), q=q, rc=rc, eps_rf=1.0))
    e = energy(o, o.desc["x0"])
    assert e == pytest.approx(fq * q[0] * q[1] * (1 / r - 1 / rc), rel=1e-12)
    f, _, _ = o.forces(o.desc["x0"])
    assert f[1, 0] == pytest.approx(fq * q[0] * q[1] / r ** 2, rel=1e-12)
    oc = oracle_mod.Oracle(two_body(rc - 1e-7, eps=(0, 0), q=q, rc=rc, eps_rf=1e15))
    fc, _, tc = oc.forces(oc.desc["x0"])
    assert abs(fc[1, 0]) < 1e-4 and abs(tc["e_rf"]) < 1e-4


def test_pair_forces_match_finite_differences(oracle_mod):
    d = synth.lj_box(seed=5, n=60, box=2.2, r_cut=0.95)
    o = oracle_mod.Oracle(d)
    x = d["x0"]
    f, _, _ = o.forces(x)
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(12):
        i, a = int(rng.integers(len(x))), int(rng.integers(3))
        xp, xm = x.copy(), x.copy()
        xp[i, a] += h
        xm[i, a] -= h
        fd = -(energy(o, xp) - energy(o, xm)) / (2 * h)
        assert fd == pytest.approx(f[i, a], abs=1e-5 * max(1.0, abs(f[i, a])))
    assert np.abs(f.sum(0)).max() < 1e-9 * np.abs(f).sum()


# --------------------------------------------------------------- pair sets
def _numpy_pairs(x, L, rc, excl):
    """Independent vectorised statement of the fixed-point membership
    predicate: X = round(x 2^22), nearest image in integers, one rounding to
    FP32, r2 = fma(dz, dz, fma(dy, dy, dx*dx)) < fl32((rc 2^22)^2)."""
    q = 2.0 ** 22
    X = np.rint(x * q).astype(np.int64)
    Lq = int(np.rint(L * q))
    n = len(x)
    i, j = np.triu_indices(n, 1)
    D = X[j] - X[i]
    nimg = np.floor_divide(2 * D + Lq, 2 * Lq)
    dp = (D - nimg * Lq).astype(np.float32)
    # every FP32 value here is an integer below 2^31, so a*a + b is exact in
    # int64 and one int64 -> FP32 conversion is the single rounding of fma
    a = dp.astype(np.int64)
    sq = (a[:, 0] * a[:, 0]).astype(np.float32)
    r2 = (a[:, 1] * a[:, 1] + sq.astype(np.int64)).astype(np.float32)
    r2 = (a[:, 2] * a[:, 2] + r2.astype(np.int64)).astype(np.float32)
    keep = r2 < np.float32((rc * q) ** 2)
    s = set(zip(i[keep].tolist(), j[keep].tolist()))
    s -= set((min(a, b), max(a, b)) for a, b in excl.tolist())
    return s


@pytest.mark.parametrize("L,rc,n", [(2.5, 0.9, 150), (1.9, 0.9, 60), (3.1, 1.0, 220), (1.85, 0.92, 40)])
def test_pair_sets_brute_cells_and_independent_predicate(oracle_mod, L, rc, n):
    """Cell list with 1-3 cells per side (wrapped stencils) finds exactly the
    brute-force set, which equals an independent statement of the predicate."""
    d = synth.lj_box(seed=int(L * 100), n=n, box=L, r_cut=rc)
    rng = np.random.default_rng(3)
    d["x0"] = d["x0"] + rng.normal(scale=0.05, size=d["x0"].shape) + rng.integers(-2, 3, size=(n, 3)) * L
    d["excl"] = np.array([[0, 1], [2, 5], [7, 9]], np.int32)
    o = oracle_mod.Oracle(d)
    x = d["x0"]
    pb = set(map(tuple, o.pairs(x, cells=False).tolist()))
    pc = set(map(tuple, o.pairs(x, cells=True).tolist()))
    assert pb == pc
    assert pb == _numpy_pairs(x, L, rc, d["excl"])
    assert (0, 1) not in pb


def test_small_system_box_has_two_cells_per_side_and_matches(oracle_mod):
    d = synth.small_chain_system()
    o = oracle_mod.Oracle(d)
    x = d["x0"].astype(np.float32).astype(np.float64)
    assert int(2.5 // 0.9) == 2
    pb = o.pairs(x, cells=False)
    pc = o.pairs(x, cells=True)
    assert set(map(tuple, pb.tolist())) == set(map(tuple, pc.tolist()))


# --------------------------------------------------------------- bonded
def test_bonded_rest_state_and_invariances(oracle_mod):
    """Harmonic bond and angle: zero force at (r0, theta0); internal forces sum
    to zero with zero net torque; forces are the energy's gradient."""
    d = synth.lj_box(n=3, box=6.0, charged=False)
    d.update(sigma=np.zeros(3), epsilon=np.zeros(3),
             bonds=np.array([[0, 1], [1, 2]], np.int32), bond_k=np.array([1000.0, 345000.0]),
             bond_r0=np.array([0.38, 0.0957]), angles=np.array([[0, 1, 2]], np.int32),
             angle_k=np.array([100.0]), angle_theta0=np.array([math.radians(110.0)]),
             excl=np.array([[0, 1], [1, 2], [0, 2]], np.int32))
    th = math.radians(110.0)
    x = np.array([[2.0 + 0.38, 2.0, 2.0], [2.0, 2.0, 2.0],
                  [2.0 + 0.0957 * math.cos(th), 2.0 + 0.0957 * math.sin(th), 2.0]])
    d["x0"] = x
    o = oracle_mod.Oracle(d)
    f, _, t = o.forces(x)
    assert np.abs(f).max() < 1e-9 and t["e_bond"] < 1e-20 and t["e_angle"] < 1e-20
    rng = np.random.default_rng(0)
    xr = x + rng.normal(scale=0.03, size=x.shape)
    f, _, _ = o.forces(xr)
    assert np.abs(f.sum(0)).max() < 1e-9
    assert np.abs(np.cross(xr, f).sum(0)).max() < 1e-9
    h = 1e-7
    for i in range(3):
        for a in range(3):
            xp, xm = xr.copy(), xr.copy()
            xp[i, a] += h
            xm[i, a] -= h
            fd = -(energy(o, xp) - energy(o, xm)) / (2 * h)
            assert fd == pytest.approx(f[i, a], rel=1e-5, abs=1e-3)


# --------------------------------------------------------------- collective variables
def test_contact_function_closed_forms(oracle_mod):
    """Supplement, contact map: C = (1-(r/r0)^6)/(1-(r/r0)^10) with r0 = 7.5 A;
    C(0) = 1, C(r0) = 3/5 (removable 0/0), C ~ (r0/r)^4 far out; the smooth
    switch makes C~ vanish at rc = 12 A with continuous value and slope."""
    cv = oracle_mod.contact_value
    assert cv(0.0, rs=10, rc=11)[0] == 1.0
    assert cv(0.75, rs=10, rc=11)[0] == pytest.approx(0.6, rel=1e-15)
    for r in (0.2, 0.5, 0.7, 0.8, 0.95):
        u = (r / 0.75) ** 2
        assert cv(r, rs=10, rc=11)[0] == pytest.approx((1 - u ** 3) / (1 - u ** 5), rel=1e-13)
    r = 40.0
    assert cv(r, rs=100, rc=101)[0] * (r / 0.75) ** 4 == pytest.approx(1.0, rel=2e-3)
    assert cv(1.2)[0] == 0.0 and cv(1.3)[0] == 0.0
    e = 1e-7
    for r0 in (1.0, 1.2):
        lo, hi = cv(r0 - e), cv(r0 + e)
        assert abs(lo[0] - hi[0]) < 1e-6 and abs(lo[1] - hi[1]) < 1e-5
    for r in (0.3, 0.75, 1.05, 1.15):
        h = 1e-6
        fd = (cv(r + h)[0] - cv(r - h)[0]) / (2 * h)
        assert cv(r)[1] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_rg_two_masses_and_gradient(oracle_mod):
    d = synth.tiny(n_solute=2, n_water=4, bias=synth.BIAS_RG)
    x = d["x0"].copy()
    x[0] = [0.5, 0.5, 0.5]
    x[1] = [0.5, 0.5, 0.5 + 0.42]
    o = oracle_mod.Oracle(d)
    z, g = o.cv(x)
    assert z == pytest.approx(0.21, rel=1e-14)
    assert g[1, 2] == pytest.approx(0.5, rel=1e-12) and g[0, 2] == pytest.approx(-0.5, rel=1e-12)


@pytest.mark.parametrize("bias", [synth.BIAS_CONTACT, synth.BIAS_RG])
def test_cv_invariance_and_finite_differences(oracle_mod, bias):
    d = synth.tiny(seed=4, bias=bias)
    o = oracle_mod.Oracle(d)
    x = d["x0"]
    z, g = o.cv(x)
    ns = d["n_solute"]
    R = scipy.stats.special_ortho_group.rvs(3, random_state=1)
    xr = x @ R.T + np.array([0.3, -1.1, 2.0])
    z2, g2 = o.cv(xr)
    assert z2 == pytest.approx(z, rel=1e-12)
    assert np.abs(g.sum(0)).max() < 1e-10 * max(1.0, np.abs(g).sum())
    assert np.abs(np.cross(x[:ns], g).sum(0)).max() < 1e-9 * max(1.0, np.abs(g).sum())
    rng = np.random.default_rng(2)
    h = 1e-6
    for _ in range(10):
        i, a = int(rng.integers(ns)), int(rng.integers(3))
        xp, xm = x.copy(), x.copy()
        xp[i, a] += h
        xm[i, a] -= h
        fd = (o.cv(xp)[0] - o.cv(xm)[0]) / (2 * h)
        assert fd == pytest.approx(g[i, a], rel=1e-6, abs=1e-8)


def test_contact_cv_vanishes_at_native_structure(oracle_mod):
    """z measures the distance to the native contact map: z(X_f) = 0."""
    d = synth.tiny(seed=6)
    o = oracle_mod.Oracle(d)
    x = d["x0"].copy()
    x[: d["n_solute"]] = d["x_final"]
    z, g = o.cv(x)
    assert z == 0.0 and np.all(g == 0.0)
    assert o.cv(d["x0"])[0] > 1.0


def test_bias_force_is_solute_only_gradient_and_ramp(oracle_mod):
    """External bias acts on solute atoms only (text after Eq. Lang); harmonic
    in z toward a reference ramped from z(X_0) to z_target."""
    d = synth.tiny(seed=7)
    d["bias_k"] = 0.7
    d["ramp_rate"] = 2.0
    o = oracle_mod.Oracle(d)
    x = d["x0"]
    st = o.init(x)
    ns = d["n_solute"]
    z0 = o.cv(x)[0]
    _, fb, t0 = o.forces(x, 0.0, st)
    assert t0["z_ref"] == pytest.approx(z0) and np.abs(fb).max() == 0.0
    _, fb, t1 = o.forces(x, 0.25, st)
    assert t1["z_ref"] == pytest.approx(0.5 * z0)
    assert np.all(fb[ns:] == 0.0) and np.abs(fb[:ns]).max() > 0
    assert np.abs(fb.sum(0)).max() < 1e-10 * np.abs(fb).sum()
    _, _, t2 = o.forces(x, 3.0, st)
    assert t2["z_ref"] == d["z_target"]
    # F_bias = -dU_bias/dx (finite differences at fixed t)
    h = 1e-6
    for i, a in ((0, 0), (ns // 2, 1), (ns - 1, 2)):
        xp, xm = x.copy(), x.copy()
        xp[i, a] += h
        xm[i, a] -= h
        fd = -(o.forces(xp, 0.25, st)[2]["e_bias"] - o.forces(xm, 0.25, st)[2]["e_bias"]) / (2 * h)
        assert fd == pytest.approx(fb[i, a], rel=1e-6, abs=1e-9)
    # S = sum |F_bias|^2 / (gamma m) is the integrand of Eq. VMDcondition
    S = float(np.sum(np.sum(fb[:ns] ** 2, 1) / (d["gamma"][:ns] * d["mass"][:ns])))
    assert t1["S"] == pytest.approx(S, rel=1e-13)


# --------------------------------------------------------------- integrator
def free_particles(n=400, gamma=3.0, dt=0.004, kT=2.494, m=2.0):
    d = synth.lj_box(n=n, box=20.0, r_cut=0.3, charged=False)
    d.update(sigma=np.zeros(n), epsilon=np.zeros(n), mass=np.full(n, m), gamma=np.full(n, gamma),
             dt=dt, kT=kT)
    return d


def test_free_particle_ou_velocity_statistics(oracle_mod):
    """Without forces the velocity is an Ornstein-Uhlenbeck process: the O-step
    is exact, so <v_n v_0> = c1^n kT/m and <v^2> = kT/m at every step."""
    d = free_particles()
    o = oracle_mod.Oracle(d)
    x = d["x0"].copy()
    v = o.maxwell()
    v0 = v.copy()
    st = o.init(x)
    nsteps = 60
    o.run(x, v, st, nsteps)
    c1 = math.exp(-d["gamma"][0] * d["dt"])
    kTm = d["kT"] / d["mass"][0]
    n = v0.size
    assert np.mean(v0 ** 2) == pytest.approx(kTm, rel=4 * math.sqrt(2 / n))
    assert np.mean(v ** 2) == pytest.approx(kTm, rel=4 * math.sqrt(2 / n))
    corr = np.mean(v * v0) / kTm
    assert corr == pytest.approx(c1 ** nsteps, abs=4 / math.sqrt(n))


def test_harmonic_baoab_matches_discrete_lyapunov(oracle_mod):
    """Dumbbells joined by a zero-length harmonic bond: the relative coordinate
    is a 3-D harmonic oscillator and BAOAB is a linear map on (r, v_r); its
    stationary covariance solves a discrete Lyapunov equation (scipy).  BAOAB
    samples <r^2> = kT/k_eff exactly while <v^2> carries an O(dt^2) shift, so
    the test also identifies the splitting order."""
    npair, m, k, gamma, dt, kT = 200, 1.0, 200.0, 8.0, 0.04, 2.494
    n = 2 * npair
    d = synth.lj_box(n=n, box=20.0, r_cut=0.3, charged=False)
    rng = np.random.default_rng(0)
    x = np.repeat(rng.uniform(1, 19, (npair, 3)), 2, axis=0) + rng.normal(scale=0.05, size=(n, 3))
    d.update(sigma=np.zeros(n), epsilon=np.zeros(n), mass=np.full(n, m), gamma=np.full(n, gamma),
             dt=dt, kT=kT, x0=x, bonds=np.arange(n, dtype=np.int32).reshape(-1, 2),
             bond_k=np.full(npair, k), bond_r0=np.zeros(npair),
             excl=np.arange(n, dtype=np.int32).reshape(-1, 2))
    o = oracle_mod.Oracle(d)
    v = o.maxwell()
    st = o.init(x)
    o.run(x, v, st, 100)  # burn-in
    rs, vs = [], []
    for _ in range(150):
        o.run(x, v, st, 4)
        rs.append(x[1::2] - x[0::2])
        vs.append(v[1::2] - v[0::2])
    rs, vs = np.array(rs).ravel(), np.array(vs).ravel()
    # relative coordinate: mu = m/2, omega^2 = k/mu; noise on v_r has twice the
    # single-atom variance (difference of two independent O-steps)
    w2 = k / (m / 2)
    c1 = math.exp(-gamma * dt)
    B = np.array([[1, 0], [-0.5 * dt * w2, 1]])
    A = np.array([[1, 0.5 * dt], [0, 1]])
    O = np.diag([1.0, c1])
    M = B @ A @ O @ A @ B
    sv2 = 2 * (1 - c1 ** 2) * kT / m
    Q = B @ A @ np.diag([0.0, sv2]) @ A.T @ B.T
    S = scipy.linalg.solve_discrete_lyapunov(M, Q)
    assert S[0, 0] == pytest.approx(kT / k, rel=1e-9)  # <r^2> = kT/(mu w^2) exactly
    nsamp = 150 * npair  # samples 4 steps apart, treated conservatively
    tol = 4 * math.sqrt(2 / nsamp)
    assert np.mean(rs ** 2) == pytest.approx(S[0, 0], rel=tol)
    assert np.mean(vs ** 2) == pytest.approx(S[1, 1], rel=tol)
    assert abs(S[1, 1] / (2 * kT / m) - 1) > 3 * tol  # the dt^2 shift is resolved


def nve_fluctuation(oracle_mod, dt, nsteps, d0):
    d = dict(d0)
    d["dt"] = dt
    d["gamma"] = np.zeros(d["n_atoms"])
    o = oracle_mod.Oracle(d)
    x = d["x0"].copy()
    v = o.maxwell() * 0.5
    st = o.init(x)
    es = []
    for _ in range(nsteps):
        o.run(x, v, st, 1)
        _, _, t = o.forces(x, st.step * dt, st)
        pe = t["e_lj"] + t["e_rf"] + t["e_bond"] + t["e_angle"]
        ke = 0.5 * np.sum(d["mass"][:, None] * v ** 2)
        es.append(pe + ke)
    es = np.array(es)
    return np.std(es), es


def test_nve_energy_error_is_second_order(oracle_mod):
    """gamma = 0 turns BAOAB into velocity Verlet: the energy fluctuation of a
    fixed time window scales as dt^2 (halving dt divides it by ~4)."""
    d0 = synth.lj_box(seed=11, n=64, box=1.9, r_cut=0.9)
    d0["x0"] = d0["x0"]
    s1, _ = nve_fluctuation(oracle_mod, 0.004, 100, d0)
    s2, _ = nve_fluctuation(oracle_mod, 0.002, 200, d0)
    assert 3.0 < s1 / s2 < 5.3


# --------------------------------------------------------------- functional and selection
def test_functional_constant_force_closed_form(oracle_mod):
    """Eq. VMDcondition with the 1/(4kT) prefactor of Eq. StrVMD: a constant
    bias F0 on one solute atom for time T gives Phi = T |F0|^2/(4 kT gamma m)
    (the trapezoid rule is exact for a constant integrand)."""
    d = synth.tiny(seed=3, bias=synth.BIAS_CONST)
    ns = d["n_solute"]
    cf = np.zeros((ns, 3))
    F0 = np.array([3.0, -4.0, 12.0])
    cf[5] = F0
    d["const_force"] = cf
    o = oracle_mod.Oracle(d)
    x = d["x0"].copy()
    v = o.maxwell()
    st = o.init(x)
    assert o.phi(st) == 0.0
    nsteps = 17
    o.run(x, v, st, nsteps)
    T = nsteps * d["dt"]
    expect = T * float(F0 @ F0) / (4 * d["kT"] * d["gamma"][5] * d["mass"][5])
    assert o.phi(st) == pytest.approx(expect, rel=1e-13)


def test_functional_zero_without_bias_and_nonnegative(oracle_mod):
    """The functional is non-negative and vanishes for unbiased dynamics
    (main text, convergence criterion)."""
    d = synth.tiny(seed=8)
    d0 = dict(d, bias_k=0.0)
    o = oracle_mod.Oracle(d0)
    x, v = d0["x0"].copy(), None
    v = o.maxwell()
    st = o.init(x)
    o.run(x, v, st, 5)
    assert o.phi(st) == 0.0
    d1 = dict(d, bias_k=0.5, ramp_rate=5.0)
    o = oracle_mod.Oracle(d1)
    x = d1["x0"].copy()
    v = o.maxwell()
    st = o.init(x)
    o.run(x, v, st, 5)
    assert o.phi(st) > 0.0


def test_segments_resume_bit_identically(oracle_mod):
    """Counter-based noise: 12 steps == 7 steps + 5 steps, bit for bit."""
    d = synth.tiny(seed=9)
    d["bias_k"] = 0.3
    o = oracle_mod.Oracle(d)
    xa = d["x0"].copy()
    va = o.maxwell()
    xb, vb = xa.copy(), va.copy()
    sa = o.init(xa)
    sb = o.init(xb)
    o.run(xa, va, sa, 12)
    o.run(xb, vb, sb, 7)
    o.run(xb, vb, sb, 5)
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    assert o.phi(sa) == o.phi(sb)


def test_ratchet_bias_only_resists_backtracking(oracle_mod):
    """Eq. VR: no force while z is at its running minimum; z_m never rises."""
    d = synth.tiny(seed=10, bias=synth.BIAS_RMD_CONTACT)
    d["bias_k"] = 0.05
    o = oracle_mod.Oracle(d)
    x = d["x0"].copy()
    v = o.maxwell()
    st = o.init(x)
    zm_prev = st.z_m
    _, fb, t = o.forces(x, 0.0, st)
    assert np.all(fb == 0.0)  # z(X_0) is the initial minimum
    for _ in range(25):
        o.run(x, v, st, 1)
        assert st.z_m <= zm_prev
        _, fb, t = o.forces(x, st.step * d["dt"], st)
        if t["z"] <= st.z_m:
            assert np.all(fb == 0.0)
        else:
            assert np.abs(fb).max() > 0.0
        zm_prev = st.z_m


def test_selection_brute_force(oracle_mod):
    rng = np.random.default_rng(0)
    for _ in range(50):
        n = int(rng.integers(1, 12))
        phi = rng.choice([0.5, 1.0, 2.0, np.inf, np.nan, 0.25], size=n)
        reached = rng.integers(0, 2, n).astype(np.uint8)
        elig = rng.integers(0, 2, n).astype(np.uint8)
        rc, best, bp = oracle_mod.select(phi, reached, elig)
        ok = [r for r in range(n) if reached[r] and elig[r] and np.isfinite(phi[r])]
        if not ok:
            assert rc == -1 and best == -1
        else:
            m = min(phi[r] for r in ok)
            assert best == min(r for r in ok if phi[r] == m) and bp == m


# ------------------------------------------- derivative w.r.t. (bias_k, ramp_rate)
def _tangent_systems():
    return {"contact": dict(synth.tiny(seed=31), bias_k=0.08, ramp_rate=30.0),
            "rg": dict(synth.tiny(seed=32, bias=synth.BIAS_RG), ramp_rate=20.0)}


@pytest.mark.parametrize("kind", ["contact", "rg"])
def test_force_directional_derivative_matches_central_differences(oracle_mod, kind):
    """d/dh F(x + h dx) at h = 0 (dual numbers) against (F(x+h dx) - F(x-h dx))/2h,
    for the whole force including the bias and for the functional integrand S."""
    d = _tangent_systems()[kind]
    o = oracle_mod.Oracle(d)
    x = np.asarray(d["x0"], np.float64)
    st = o.init(x)
    rng = np.random.default_rng(5)
    dx = rng.normal(size=(2, o.n, 3))
    t = 0.013
    f, fdot, S, Sdot, bad = o.forces_dir(x, dx, False, t, st, cells=False)
    assert not bad
    h = 1e-6
    for k in range(2):
        fp, _, tp = o.forces(x + h * dx[k], t, st, cells=False)
        fm, _, tm = o.forces(x - h * dx[k], t, st, cells=False)
        fd = (fp - fm) / (2 * h)
        assert np.linalg.norm(fdot[k] - fd) <= 1e-6 * np.linalg.norm(fd)
        sd = (tp["S"] - tm["S"]) / (2 * h)
        assert abs(Sdot[k] - sd) <= 1e-6 * abs(sd) + 1e-12


@pytest.mark.parametrize("kind", ["contact", "rg"])
def test_force_parameter_derivative_matches_central_differences(oracle_mod, kind):
    d = _tangent_systems()[kind]
    o = oracle_mod.Oracle(d)
    x = np.asarray(d["x0"], np.float64)
    st = o.init(x)
    t = 0.011
    _, fdot, _, Sdot, _ = o.forces_dir(x, None, True, t, st, cells=False)
    for k, key in enumerate(("bias_k", "ramp_rate")):
        h = 1e-6 * d[key]
        out = []
        for sgn in (1, -1):
            dd = dict(d)
            dd[key] = d[key] + sgn * h
            f, _, terms = oracle_mod.Oracle(dd).forces(x, t, st, cells=False)
            out.append((f, terms["S"]))
        fd = (out[0][0] - out[1][0]) / (2 * h)
        assert np.linalg.norm(fdot[k] - fd) <= 1e-6 * np.linalg.norm(fd)
        assert abs(Sdot[k] - (out[0][1] - out[1][1]) / (2 * h)) <= 1e-6 * abs(Sdot[k])


def _phi_and_grad(oracle_mod, d, nsteps):
    o = oracle_mod.Oracle(d)
    x = np.array(d["x0"], np.float64)
    v = o.maxwell()
    st = o.init(x)
    pd = o.init_tangent(x, st)
    xt = np.zeros((2, o.n, 3))
    vt = np.zeros((2, o.n, 3))
    assert o.run_tangent(x, v, st, xt, vt, pd, nsteps) == 0
    return o.phi(st), o.phi_grad(st, pd), x, v


def _phi_plain(oracle_mod, d, nsteps):
    o = oracle_mod.Oracle(d)
    x = np.array(d["x0"], np.float64)
    v = o.maxwell()
    st = o.init(x)
    assert o.run(x, v, st, nsteps) == 0
    return o.phi(st), x, v


@pytest.mark.parametrize("kind", ["contact", "rg"])
def test_functional_gradient_matches_central_differences(oracle_mod, kind):
    """dPhi/d(bias_k, ramp_rate) along a 30-step trajectory with the noise held
    fixed, against central differences of separate plain runs."""
    d = _tangent_systems()[kind]
    n = 30
    phi, grad, x, v = _phi_and_grad(oracle_mod, d, n)
    phi0, x0, v0 = _phi_plain(oracle_mod, d, n)
    # the dual run's values are the plain run
    assert abs(phi - phi0) <= 1e-12 * phi0
    assert np.abs(x - x0).max() <= 1e-12 and np.abs(v - v0).max() <= 1e-9
    for k, key in enumerate(("bias_k", "ramp_rate")):
        h = 1e-5 * d[key]
        pp = _phi_plain(oracle_mod, dict(d, **{key: d[key] + h}), n)[0]
        pm = _phi_plain(oracle_mod, dict(d, **{key: d[key] - h}), n)[0]
        fd = (pp - pm) / (2 * h)
        assert abs(grad[k] - fd) <= 1e-6 * abs(fd), (key, grad[k], fd)
        assert abs(grad[k]) > 0


def test_functional_gradient_vanishes_at_zero_stiffness(oracle_mod):
    """Phi is quadratic in the bias force, so at bias_k = 0 both derivatives are 0."""
    d = dict(_tangent_systems()["contact"], bias_k=0.0)
    _, grad, _, _ = _phi_and_grad(oracle_mod, d, 10)
    assert np.all(grad == 0.0)


def test_ramp_rate_derivative_vanishes_when_the_ramp_ends_in_the_first_step(oracle_mod):
    """With rho dt > 1 the reference sits at z_target from step 1 on and
    z_ref(0) = z(X_0) for every rho, so Phi does not depend on rho."""
    d = _tangent_systems()["contact"]
    d = dict(d, ramp_rate=2.0 / d["dt"])
    _, grad, _, _ = _phi_and_grad(oracle_mod, d, 10)
    assert grad[1] == 0.0 and grad[0] != 0.0


# --------------------------------------------------------------- contact-sum range
def _line_solute(n, spacing=1.5, box=30.0, min_sep=3, bias=synth.BIAS_CONTACT):
    """n solute beads and no solvent in a large box: every bead starts on a line
    with `spacing` between neighbours (all pairs beyond the 1.2 nm switch)."""
    d = synth.lj_box(n=n, box=box, r_cut=1.0, charged=False)
    x = np.zeros((n, 3)) + 1.0
    x[:, 0] += spacing * np.arange(n)
    d.update(n_solute=n, x0=x, x_final=x.copy(), bias=bias, contact_min_sep=min_sep,
             contact_r0=0.75, contact_rs=1.0, contact_rc=1.2, bias_k=0.1, gamma=np.full(n, 1.0))
    return d


def test_contact_sum_runs_over_unordered_pairs_beyond_the_separation(oracle_mod):
    """Supplement, collective coordinate: z sums over pairs with |i - j| > 35
    (here min_sep = 3) once per unordered pair.  With the target map empty
    (every X_f pair beyond the switch), one pair (i, i + min_sep + 1) at
    r = r0 gives z = C(r0)^2 = (3/5)^2, and a pair at separation exactly
    min_sep adds nothing; counting |i - j| >= min_sep or ordered pairs would
    give a different z."""
    d = _line_solute(12, min_sep=3)
    x = d["x0"].copy()
    x[4] = x[0] + np.array([0.0, 0.75, 0.0])   # pair (0, 4): separation 4 > 3, at r0
    x[9] = x[6] + np.array([0.0, 0.0, 0.5])    # pair (6, 9): separation 3, not counted
    o = oracle_mod.Oracle(d)
    assert o.cv(d["x_final"])[0] == 0.0
    z, g = o.cv(x)
    assert z == pytest.approx(0.36, rel=1e-14)
    # only the counted pair carries a gradient: equal and opposite on atoms 0 and 4
    moved = np.flatnonzero(np.abs(g).sum(1) > 0)
    assert list(moved) == [0, 4] and np.array_equal(g[0], -g[4])


# --------------------------------------------------------------- reached
def _two_bead_rg(tol, z_target, reach_rmsd=float("inf")):
    d = _line_solute(2, spacing=0.5, bias=synth.BIAS_RG)
    d.update(bias_k=0.0, ramp_rate=0.0, z_target=z_target, reach_tol=tol, reach_rmsd=reach_rmsd,
             sigma=np.full(2, 0.3), epsilon=np.full(2, 0.5))
    return d


def test_reached_compares_the_final_z_with_the_tolerance_inclusively(oracle_mod):
    """Folding-event criterion read as |z(X_T) - z_target| <= reach_tol on the
    z of the last step, never for an unstable trajectory.  Two equal masses
    0.5 nm apart: Rg = 0.25 exactly."""
    O = oracle_mod
    d = _two_bead_rg(0.125, 0.375)
    o = O.Oracle(d)
    st = o.init(d["x0"])
    assert st.z_last == 0.25
    assert o.reached(st)
    assert not O.Oracle(dict(d, reach_tol=np.nextafter(0.125, 0.0))).reached(st)
    # after some steps z_last differs from z(X_0): the decision follows z_last
    x, v = d["x0"].copy(), o.maxwell()
    o.run(x, v, st, 40)
    delta = st.z_last - 0.25
    assert abs(delta) > 1e-6
    zt = st.z_last + delta            # |z_last - zt| = |delta|, |z(X_0) - zt| = 2 |delta|
    tol = abs(st.z_last - zt)
    assert O.Oracle(dict(d, z_target=zt, reach_tol=tol)).reached(st)
    assert not O.Oracle(dict(d, z_target=zt, reach_tol=np.nextafter(tol, 0.0))).reached(st)
    st.status = 1
    assert not O.Oracle(dict(d, reach_tol=np.inf)).reached(st)


# --------------------------------------------------------------- ratchet prefactor
def test_ratchet_force_is_half_the_harmonic_force_toward_the_running_minimum(oracle_mod):
    """Eq. VR: F = -(k_R/2)(z - z_m) grad z while z > z_m.  At a configuration
    with z > z_m this is exactly half of the harmonic bias -k (z - z_ref) grad z
    with z_ref = z_m, and it is the gradient of (k_R/4)(z - z_m)^2 at fixed z_m."""
    O = oracle_mod
    base = dict(synth.tiny(seed=10, bias=synth.BIAS_RMD_CONTACT), bias_k=0.05)
    x = np.asarray(base["x0"], np.float64)
    ornd = O.Oracle(base)
    st = ornd.init(x)
    z = st.z0
    st.z_m = 0.8 * z                                  # z > z_m: the ratchet acts
    _, f_rmd, t_rmd = ornd.forces(x, 0.0, st)
    harm = dict(base, bias=synth.BIAS_CONTACT, ramp_rate=0.0)
    oh = O.Oracle(harm)
    sh = oh.init(x)
    sh.z0 = st.z_m                                    # z_ref(t) = z0 when the ramp is off
    _, f_h, t_h = oh.forces(x, 0.0, sh)
    assert t_h["z_ref"] == st.z_m and np.abs(f_h).max() > 0
    assert np.array_equal(f_rmd, 0.5 * f_h)
    assert t_rmd["e_bias"] == pytest.approx(0.5 * t_h["e_bias"], rel=1e-15)
    assert t_rmd["e_bias"] == pytest.approx(0.25 * 0.05 * (z - st.z_m) ** 2, rel=1e-14)
    h = 1e-6
    ns = base["n_solute"]
    for i, a in ((0, 0), (ns // 2, 1), (ns - 1, 2)):
        xp, xm = x.copy(), x.copy()
        xp[i, a] += h
        xm[i, a] -= h
        fd = -(ornd.forces(xp, 0.0, st)[2]["e_bias"] - ornd.forces(xm, 0.0, st)[2]["e_bias"]) / (2 * h)
        assert fd == pytest.approx(f_rmd[i, a], rel=1e-6, abs=1e-10)
    st.z_m = z                                        # at the minimum: no force
    assert np.all(ornd.forces(x, 0.0, st)[1] == 0.0)


def test_constant_bias_is_the_gradient_of_minus_its_projection(oracle_mod):
    """The constant test force F0 derives from U_b = -sum_i F0_i . x_i."""
    d = synth.tiny(seed=3, bias=synth.BIAS_CONST)
    rng = np.random.default_rng(4)
    d["const_force"] = rng.normal(size=(d["n_solute"], 3))
    o = oracle_mod.Oracle(d)
    x = np.asarray(d["x0"], np.float64)
    st = o.init(x)
    _, fb, t = o.forces(x, 0.0, st)
    assert t["e_bias"] == pytest.approx(-float(np.sum(d["const_force"] * x[: d["n_solute"]])), rel=1e-13)
    h = 1e-6
    for i, a in ((0, 0), (7, 2)):
        xp, xm = x.copy(), x.copy()
        xp[i, a] += h
        xm[i, a] -= h
        fd = -(o.forces(xp, 0.0, st)[2]["e_bias"] - o.forces(xm, 0.0, st)[2]["e_bias"]) / (2 * h)
        assert fd == pytest.approx(fb[i, a], rel=1e-8)


# --------------------------------------------------------------- virial
VIR = ("w_xx", "w_xy", "w_xz", "w_yx", "w_yy", "w_yz", "w_zx", "w_zy", "w_zz")


def _virial(terms):
    return np.array([terms[k] for k in VIR]).reshape(3, 3)


def _u_of(oracle_mod, d, x):
    o = oracle_mod.Oracle(dict(d, bias=synth.BIAS_NONE))
    t = o.forces(x, 0.0, None)[2]
    return t["e_lj"] + t["e_rf"] + t["e_bond"] + t["e_angle"]


def test_virial_is_minus_the_box_scaling_derivative_of_the_energy(oracle_mod):
    """W_aa = -dU/d(ln L_a) when the box edge a and every coordinate along a
    are scaled together (periodic solvated system, pair and bonded terms);
    the shifted potentials are continuous at r_c, so the difference quotient
    is a derivative even if a pair crosses the cutoff."""
    d = dict(synth.tiny(seed=8), bias=synth.BIAS_NONE)
    x = np.asarray(synth.perturbed(d, 0.005, 1)["x0"], np.float64)  # bonds and angles off rest
    W = _virial(oracle_mod.Oracle(d).forces(x, 0.0, None)[2])
    h = 1e-6
    for a in range(3):
        ups = []
        for lam in (1 + h, 1 - h):
            xs, box = x.copy(), np.array(d["box"], float)
            xs[:, a] *= lam
            box[a] *= lam
            ups.append(_u_of(oracle_mod, dict(d, box=box), xs))
        fd = -(ups[0] - ups[1]) / (2 * h)
        assert fd == pytest.approx(W[a, a], rel=1e-6, abs=1e-6)
    assert np.allclose(W, W.T, rtol=1e-12, atol=1e-9)


def test_virial_of_an_isolated_molecule_equals_sum_of_position_times_force(oracle_mod):
    """Without periodic images every term is internal to the cluster, so the
    pair/term form of the virial equals sum_i x_i (x) F_i, and a homogeneous
    deformation x -> (1 + h E_ab) x changes U by -h W_ba."""
    t = synth.tiny(seed=9)
    ns = t["n_solute"]
    keep = {k: t[k] for k in ("bonds", "angles", "excl")}
    d = dict(t, n_atoms=ns, mass=t["mass"][:ns], gamma=t["gamma"][:ns], charge=t["charge"][:ns],
             sigma=t["sigma"][:ns], epsilon=t["epsilon"][:ns], x0=t["x0"][:ns] + 5.0,
             box=np.full(3, 20.0), r_cut=2.5, bias=synth.BIAS_NONE,
             bonds=keep["bonds"][np.all(keep["bonds"] < ns, 1)],
             excl=keep["excl"][np.all(keep["excl"] < ns, 1)])
    sel = np.all(keep["angles"] < ns, 1)
    d["angles"] = keep["angles"][sel]
    d["angle_k"], d["angle_theta0"] = t["angle_k"][sel], t["angle_theta0"][sel]
    bsel = np.all(keep["bonds"] < ns, 1)
    d["bond_k"], d["bond_r0"] = t["bond_k"][bsel], t["bond_r0"][bsel]
    x = np.asarray(synth.perturbed(d, 0.01, 2)["x0"], np.float64)  # bonds and angles off rest
    o = oracle_mod.Oracle(d)
    f, _, terms = o.forces(x, 0.0, None)
    W = _virial(terms)
    assert terms["e_bond"] > 1.0 and terms["e_angle"] > 0 and terms["e_lj"] != 0
    assert np.allclose(W, x.T @ f, rtol=1e-10, atol=1e-8)
    h = 1e-6
    for a in range(3):
        for b in range(3):
            E = np.zeros((3, 3))
            E[a, b] = 1.0
            up = _u_of(oracle_mod, d, x @ (np.eye(3) + h * E).T)
            um = _u_of(oracle_mod, d, x @ (np.eye(3) - h * E).T)
            assert -(up - um) / (2 * h) == pytest.approx(W[b, a], rel=1e-6, abs=1e-6)


# --------------------------------------------------------------- RMSD to the product
def _rmsd_oracle(oracle_mod, xf):
    n = len(xf)
    d = _line_solute(n)
    d["x_final"] = np.asarray(xf, np.float64)
    return oracle_mod.Oracle(d)


def test_rmsd_of_a_rigidly_moved_copy_is_zero(oracle_mod):
    rng = np.random.default_rng(1)
    xf = rng.normal(size=(30, 3))
    o = _rmsd_oracle(oracle_mod, xf)
    R = scipy.stats.special_ortho_group.rvs(3, random_state=2)
    assert o.rmsd(xf @ R.T + np.array([3.0, -2.0, 0.5])) < 1e-12
    assert o.rmsd(xf + 0.7) < 1e-12


def test_rmsd_two_points_closed_form(oracle_mod):
    """Two atoms d1 and d2 apart: after centring and aligning the axes each
    atom is off by |d1 - d2| / 2."""
    xf = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    o = _rmsd_oracle(oracle_mod, xf)
    x = np.array([[2.0, 1.0, 0.0], [2.0, 1.0 + 0.6, 0.8]])  # distance 1.0 as well
    assert o.rmsd(x) < 1e-12
    x[1] = [2.0, 1.0, 1.4]                                 # distance 1.4
    assert o.rmsd(x) == pytest.approx(0.2, rel=1e-12)


def test_rmsd_matches_the_kabsch_alignment_of_scipy(oracle_mod):
    """scipy's Rotation.align_vectors solves the same least-squares rotation
    (Kabsch); its root-sum-square residual over centred sets, divided by
    sqrt(n), is the RMSD."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(5)
    for n in (3, 7, 40):
        xf = rng.normal(size=(n, 3))
        x = xf @ scipy.stats.special_ortho_group.rvs(3, random_state=n).T + rng.normal(scale=0.3, size=(n, 3))
        o = _rmsd_oracle(oracle_mod, xf)
        a, b = xf - xf.mean(0), x - x.mean(0)
        _, rssd = Rotation.align_vectors(a, b)
        assert o.rmsd(x) == pytest.approx(rssd / np.sqrt(n), rel=1e-9)


def test_rmsd_admits_no_reflection(oracle_mod):
    """Superposition by proper rotations only: the mirror image of a chiral
    set keeps a positive RMSD, that of a planar set (a rotation away) none."""
    chiral = np.array([[0, 0, 0], [1, 0, 0], [0, 2, 0], [0, 0, 3]], float)
    o = _rmsd_oracle(oracle_mod, chiral)
    mirror = chiral * np.array([-1.0, 1.0, 1.0])
    assert o.rmsd(mirror) > 0.1
    planar = np.array([[0, 0, 0], [1, 0, 0], [0, 2, 0], [3, 1, 0]], float)
    assert _rmsd_oracle(oracle_mod, planar).rmsd(planar * np.array([1.0, 1.0, -1.0]) + 0.0) < 1e-12
    assert _rmsd_oracle(oracle_mod, planar).rmsd(planar * np.array([-1.0, 1.0, 1.0])) < 1e-12


def test_reached_with_an_rmsd_criterion(oracle_mod):
    """With reach_rmsd finite, the product is reached only within that RMSD of X_f."""
    O = oracle_mod
    d = _line_solute(6, min_sep=1)
    rng = np.random.default_rng(3)
    d["x_final"] = d["x0"] + rng.normal(scale=0.4, size=(6, 3))
    d.update(reach_tol=np.inf)
    x = d["x0"].copy()
    r = O.Oracle(d).rmsd(x)
    st = O.Oracle(d).init(x)
    assert O.Oracle(dict(d, reach_rmsd=r)).reached(st, x)
    assert not O.Oracle(dict(d, reach_rmsd=np.nextafter(r, 0.0))).reached(st, x)
    assert not O.Oracle(dict(d, reach_rmsd=r)).reached(st, None)
