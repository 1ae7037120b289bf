"""Pins of the oracle's toy model (supplement, "Illustrative Application in a
Toy Model") and of the contact-formation order and path similarity (main
text, mechanism analysis): special cases with closed forms, finite
differences, equilibrium statistics, brute force and an independent library
routine (Kendall's tau).  CPU only."""
import math

import numpy as np
import pytest
import scipy.stats

from paper_1405_6104_amd import synth

PAPER_TOY = dict(A1=30.0, A2=20.0, A3=6.0, s1=1.0, s2=2.0, s3=2.0, w=0.03, xm=1.5, ym=0.0,
                 gamma=1.0, mass=1.0, kT=0.2, dt=0.02, x0=0.0, y0=5.0, r_product=0.5, r_gate=2.0,
                 n_steps=2000)


def only(**kw):
    """The toy potential with every term off except the given constants."""
    p = dict(PAPER_TOY, A1=0.0, A2=0.0, A3=0.0, w=0.0)
    p.update(kw)
    return p


# --------------------------------------------------------------- potential
def test_toy_potential_terms_reduce_to_closed_forms(oracle_mod):
    """Each term of U alone: w^2 r^4; -A1 s1^2/(r^2+s1^2)^2 (value -A1/s1^2 at
    the origin and -A1/(4 s1^2) at r = s1); the A2 bump likewise with the
    opposite sign; the A3 well centred at (xm, ym) with depth -A3/s3^2."""
    tp = oracle_mod.toy_potential
    assert tp(only(w=0.3), 1.0, 1.0)[0] == pytest.approx(4 * 0.09, rel=1e-14)
    assert tp(only(A1=30.0, s1=1.3), 0.0, 0.0)[0] == pytest.approx(-30.0 / 1.69, rel=1e-14)
    assert tp(only(A1=30.0, s1=1.3), 0.0, 1.3)[0] == pytest.approx(-30.0 / (4 * 1.69), rel=1e-14)
    assert tp(only(A2=20.0, s2=2.0), 2.0, 0.0)[0] == pytest.approx(20.0 / 16.0, rel=1e-14)
    p3 = only(A3=6.0, s3=2.0, xm=1.5, ym=-0.7)
    assert tp(p3, 1.5, -0.7)[0] == pytest.approx(-6.0 / 4.0, rel=1e-14)
    assert tp(p3, 1.5, -0.7)[1:] == (0.0, 0.0)
    assert tp(p3, 1.5 + 2.0, -0.7)[0] == pytest.approx(-6.0 / 16.0, rel=1e-14)
    # the radial terms do not depend on the direction
    pr = dict(PAPER_TOY, A3=0.0)
    vals = [tp(pr, 2.2 * math.cos(a), 2.2 * math.sin(a))[0] for a in np.linspace(0, 2 * np.pi, 7)]
    assert np.ptp(vals) < 1e-13


def test_toy_gradient_matches_central_differences(oracle_mod):
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(20):
        x, y = rng.uniform(-4, 4, 2)
        u, gx, gy = oracle_mod.toy_potential(PAPER_TOY, x, y)
        fx = (oracle_mod.toy_potential(PAPER_TOY, x + h, y)[0] - oracle_mod.toy_potential(PAPER_TOY, x - h, y)[0]) / (2 * h)
        fy = (oracle_mod.toy_potential(PAPER_TOY, x, y + h)[0] - oracle_mod.toy_potential(PAPER_TOY, x, y - h)[0]) / (2 * h)
        assert gx == pytest.approx(fx, rel=1e-7, abs=1e-9) and gy == pytest.approx(fy, rel=1e-7, abs=1e-9)


# --------------------------------------------------------------- dynamics
def test_toy_free_particle_velocity_statistics(oracle_mod):
    """With U = 0 the velocity is an Ornstein-Uhlenbeck process started at
    equilibrium, so the mean square displacement per component after time t
    is 2 D (t - (1 - exp(-gamma t))/gamma) with D = kT/(m gamma) (BAOAB's O-step
    is exact; its splitting error here is O((gamma dt)^2) ~ 4e-4)."""
    p = only(n_steps=4000, gamma=1.0, kT=0.2, dt=0.02, x0=0.0, y0=0.0, r_product=-1.0, r_gate=-1.0)
    finals = np.array([[r["x"], r["y"]] for r in (oracle_mod.toy_run(p, 0, 0.0, 1000 + k) for k in range(600))])
    t = p["n_steps"] * p["dt"]
    D = p["kT"] / (p["mass"] * p["gamma"])
    msd = np.mean(finals ** 2, 0)
    # exact underdamped result: 2 D (t - (1 - exp(-gamma t))/gamma) for a start at equilibrium velocity
    want = 2 * D * (t - (1 - math.exp(-p["gamma"] * t)) / p["gamma"])
    se = want * math.sqrt(2.0 / len(finals))
    assert np.all(np.abs(msd - want) < 4 * se), (msd, want)


def test_toy_quartic_well_equilibrium(oracle_mod):
    """U = w^2 r^4 in two dimensions: Boltzmann weight exp(-w^2 r^4 / kT) gives
    <r^4> = kT / (2 w^2) exactly (substitute s = r^2)."""
    w, kT = 0.5, 0.2
    p = only(w=w, kT=kT, dt=0.02, gamma=1.0, n_steps=3000, x0=0.3, y0=0.0, r_product=-1.0, r_gate=-1.0)
    r4 = []
    for k in range(400):
        _, path = oracle_mod.toy_run(p, 0, 0.0, 7000 + k, path=True)
        q = path[1000::200]
        r4.extend(((q ** 2).sum(1) ** 2).tolist())
    r4 = np.array(r4)
    want = kT / (2 * w * w)
    assert abs(r4.mean() - want) < 4 * r4.std() / math.sqrt(len(r4) / 2), (r4.mean(), want)


def test_toy_functional_reached_and_gate(oracle_mod):
    """Plain trials have Phi = 0; steered-MD trials Phi = dt/(4 kT) sum_n w_n K^2 z_n^2/(gamma m)
    (trapezoid) over their own path; the ratchet acts only while z > z_m, and
    z_m is the running minimum of z; the first passage and the gate angle are
    read off the path."""
    p = dict(PAPER_TOY, n_steps=1500)
    r0, path0 = oracle_mod.toy_run(p, oracle_mod.TOY_PLAIN, 3.0, 11, path=True)
    assert r0["phi"] == 0.0
    z0 = np.sqrt((path0 ** 2).sum(1))
    first = np.flatnonzero(z0 <= p["r_product"])
    assert r0["t_reach"] == (first[0] if len(first) else -1)
    g = np.flatnonzero(z0 <= p["r_gate"])
    assert r0["theta_gate"] == pytest.approx(math.atan2(path0[g[0], 1], path0[g[0], 0]), abs=0, rel=0)
    K = 0.4
    rs, paths = oracle_mod.toy_run(p, oracle_mod.TOY_SMD, K, 12, path=True)
    zs = np.sqrt((paths ** 2).sum(1))
    w = np.ones(len(zs))
    w[0] = w[-1] = 0.5
    want = p["dt"] / (4 * p["kT"]) * np.sum(w * K * K * zs ** 2) / (p["gamma"] * p["mass"])
    assert rs["phi"] == pytest.approx(want, rel=1e-12)
    rr, pathr = oracle_mod.toy_run(p, oracle_mod.TOY_RMD, K, 13, path=True)
    zr = np.sqrt((pathr ** 2).sum(1))
    assert rr["z_min"] == pytest.approx(np.min(zr), rel=1e-15)
    zm = np.minimum.accumulate(zr)
    w = np.ones(len(zr))
    w[0] = w[-1] = 0.5
    want = p["dt"] / (4 * p["kT"]) * np.sum(w * (0.5 * K * (zr - zm)) ** 2) / (p["gamma"] * p["mass"])
    assert rr["phi"] == pytest.approx(want, rel=1e-10)
    assert rr["phi"] > 0
    assert oracle_mod.toy_run(p, oracle_mod.TOY_RMD, 0.0, 13)["phi"] == 0.0
    reached = 0
    for res, z in ((r0, z0), (rs, zs), (rr, zr)):
        first = np.flatnonzero(z <= p["r_product"])
        assert res["t_reach"] == (first[0] if len(first) else -1)
        assert res["reached"] == (1.0 if len(first) else 0.0)
        reached += len(first) > 0
    assert reached >= 1


# --------------------------------------------------------------- path similarity
def test_path_similarity_closed_forms(oracle_mod):
    """s = 1/(Nc (Nc-1)) sum_{i != j} delta(M_ij(k) - M_ij(k')), M_ij = 1, 0, 1/2
    for t_i <, >, = t_j."""
    s = oracle_mod.path_similarity
    assert s([0, 1, 2], [0, 2, 1]) == pytest.approx(4 / 6, rel=1e-15)
    assert s([0, 0, 1], [0, 1, 1]) == pytest.approx(2 / 6, rel=1e-15)
    t = np.arange(20)
    assert s(t, t) == 1.0
    assert s(t, t[::-1].copy()) == 0.0
    assert s(np.zeros(20, np.int64), t) == 0.0   # all tied against a strict order
    assert s(np.zeros(20, np.int64), np.full(20, 7)) == 1.0


def test_path_similarity_without_ties_is_kendall_concordance(oracle_mod):
    """For orders without ties s = (1 + tau)/2 with Kendall's tau."""
    rng = np.random.default_rng(3)
    for n in (5, 17, 60):
        a, b = rng.permutation(n), rng.permutation(n)
        tau = scipy.stats.kendalltau(a, b).statistic
        assert oracle_mod.path_similarity(a, b) == pytest.approx((1 + tau) / 2, rel=1e-12)


def test_native_contacts_and_formation_brute_force(oracle_mod):
    """Native contacts: j - i > min_sep and |X_f,i - X_f,j| <= r0 (squared
    integer distances on the 2^-22 nm grid); formation at a configuration by
    the same rule."""
    d = synth.tiny(seed=6)
    o = oracle_mod.Oracle(d)
    pairs = o.native_contacts()
    q = 2.0 ** 24
    xf = np.rint(d["x_final"] * q).astype(np.int64)
    r0 = int(np.rint(0.75 * q))
    ns, sep = d["n_solute"], d["contact_min_sep"]
    want = [(i, j) for i in range(ns) for j in range(i + sep + 1, ns)
            if int(((xf[j] - xf[i]) ** 2).sum()) <= r0 * r0]
    assert [tuple(p) for p in pairs] == want and len(want) > 10
    x = np.asarray(d["x0"], np.float64)
    xg = np.rint(x * q).astype(np.int64)
    formed = o.contacts_formed(x, pairs)
    assert list(formed) == [int(((xg[j] - xg[i]) ** 2).sum()) <= r0 * r0 for i, j in want]
    xs = x.copy()
    xs[: ns] = d["x_final"]
    assert np.all(o.contacts_formed(xs, pairs))
