"""Seeded synthetic inputs for the batched biased-Langevin trial-path workloads.

This module only *builds inputs*: topology, parameters, starting coordinates,
the target (native) structure and the Philox seeds.  It contains none of the
method's arithmetic (no forces, no collective variables, no integrator), so it
can feed both the FP64 CPU oracle and the HIP path without coupling them.

The paper's own workloads (Fip35 WW domain and villin headpiece in TIP3P water
with the AMBER99SB-ILDN force field, main text "application to folding") are
not available here; the systems below stand in for them with the same shapes:
a ~35-residue-sized solute chain in explicit three-site water in a periodic
cubic box, with a native target structure that defines the contact map of the
collective variable (supplement, "Collective coordinate for rMD").

Units: nm, ps, amu, kJ/mol, elementary charge.

A replica description is a plain ``dict`` of numpy arrays and scalars with the
keys listed in ``REPLICA_KEYS``; both the oracle wrapper and the library
binding consume it.
"""
from __future__ import annotations

import math

import numpy as np

KB = 0.0083144626  # kJ/(mol K)

# bias kinds (same integer codes as the C ABI)
BIAS_NONE, BIAS_CONST, BIAS_RG, BIAS_CONTACT, BIAS_RMD_CONTACT = 0, 1, 2, 3, 4

# Synthetic force-field constants (solute beads and flexible three-site water).
SOLUTE_MASS = 12.011
SOLUTE_BOND_K, SOLUTE_BOND_R0 = 1000.0, 0.38
SOLUTE_ANGLE_K, SOLUTE_ANGLE_T0 = 100.0, math.radians(110.0)
SOLUTE_CHARGE = 0.3
O_MASS, H_MASS = 15.9994, 1.008
O_SIGMA, O_EPS = 0.315, 0.636
O_CHARGE, H_CHARGE = -0.834, 0.417
OH_R0, OH_K = 0.0957, 345000.0
HOH_T0, HOH_K = math.radians(104.52), 383.0

REPLICA_KEYS = (
    "n_atoms", "n_solute", "mass", "gamma", "charge", "sigma", "epsilon",
    "bonds", "bond_k", "bond_r0", "angles", "angle_k", "angle_theta0", "excl",
    "box", "r_cut", "eps_rf", "kT", "dt", "x0", "v0", "x_final",
    "bias", "bias_k", "ramp_rate", "z_target", "contact_r0", "contact_rs",
    "contact_rc", "contact_min_sep", "reach_tol", "seed", "const_force",
)

WORKLOAD_SEED = 14056104


# --------------------------------------------------------------------------
# solute growth
# --------------------------------------------------------------------------
def _tree_parents(n, rng, branching):
    """Parent of each atom i>0: i-1, or (prob. 0.25) i-2 / i-3 if degree allows."""
    parent = np.full(n, -1, np.int64)
    deg = np.zeros(n, np.int64)
    for i in range(1, n):
        p = i - 1
        if branching and i >= 3 and rng.random() < 0.25:
            cand = i - 2 if rng.random() < 0.5 else i - 3
            if deg[cand] < 4:
                p = cand
        if deg[p] >= 4:
            p = i - 1
        parent[i] = p
        deg[p] += 1
        deg[i] += 1
    return parent


def _grow(parent, center, radius, dmin, rng, n_cand=48, pull=0.0, box=None, escape=False):
    """Self-avoiding confined growth: each atom sits 0.38 nm from its parent at
    110 deg to a placed neighbour of the parent (random dihedral), inside the
    confining sphere, at least ``dmin`` from every atom that is not a 1-2 or
    1-3 partner and at least 0.5 nm from its 1-3 partners.  Among valid candidates one is drawn with weight
    exp(-pull |x-c|^2/R^2) (pull > 0 packs the chain toward the centre).  Dead
    ends backtrack by a growing number of atoms.  With ``box`` (periodic edge
    length) the distances are minimum-image ones, for spheres wider than the
    box.  With ``escape`` the backtracking depth keeps growing until the chain
    passes the furthest atom it had reached (a dead end that needs siblings
    placed long before is then undone instead of retried forever), and after
    40 n attempts the growth starts over (continuing the same random stream,
    so the result stays a function of the seed)."""
    n = len(parent)
    nbrs = [[] for _ in range(n)]
    for i in range(1, n):
        nbrs[parent[i]].append(i)
        nbrs[i].append(int(parent[i]))
    x = np.zeros((n, 3))
    d = rng.normal(size=3)
    x[0] = center + d * (0.25 * radius * rng.random() / np.linalg.norm(d))
    dmin2 = dmin * dmin
    i = 1
    streak = 0
    best = 1
    attempts = 0
    while i < n:
        attempts += 1
        if escape and attempts > 40 * n:
            d = rng.normal(size=3)
            x[0] = center + d * (0.25 * radius * rng.random() / np.linalg.norm(d))
            i, streak, best, attempts = 1, 0, 1, 0
            continue
        p = int(parent[i])
        placed_nb = [q for q in nbrs[p] if q < i]
        if placed_nb:
            q = placed_nb[int(rng.integers(len(placed_nb)))]
            e = x[q] - x[p]
            e /= np.linalg.norm(e)
            a = np.array([1.0, 0.0, 0.0]) if abs(e[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
            u = np.cross(e, a)
            u /= np.linalg.norm(u)
            w = np.cross(e, u)
            phi = rng.random(n_cand)[:, None] * (2.0 * math.pi)
            dirs = math.cos(SOLUTE_ANGLE_T0) * e + math.sin(SOLUTE_ANGLE_T0) * (np.cos(phi) * u + np.sin(phi) * w)
        else:
            dirs = rng.normal(size=(n_cand, 3))
            dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        cand = x[p] + SOLUTE_BOND_R0 * dirs
        r2c = np.sum((cand - center) ** 2, 1)
        ok = r2c <= radius * radius
        # every placed atom but the parent must keep its distance; 1-3
        # partners (other neighbours of the parent) at least 0.5 nm, which
        # keeps every bond angle at the parent above ~82 deg
        lim = np.full(i, dmin2)
        lim[placed_nb] = 0.25
        lim[p] = 0.0
        diff = cand[:, None, :] - x[None, :i]
        if box is not None:
            diff -= box * np.round(diff / box)
        dd = np.sum(diff ** 2, -1)
        ok &= np.all(dd >= lim[None, :], 1)
        if ok.any():
            w = np.exp(-pull * r2c[ok] / (radius * radius))
            pick = np.flatnonzero(ok)[rng.choice(int(ok.sum()), p=w / w.sum())]
            x[i] = cand[pick]
            i += 1
            if not escape:
                streak = max(0, streak - 1)
            elif i > best:
                best = i
                streak = 0
        else:
            streak += 1
            back = min(i - 1, int(rng.integers(1, 2 + min(streak, 40 if not escape else 400))))
            i = max(1, i - back)
    return x


def _solute_topology(parent):
    n = len(parent)
    bonds = np.array([[parent[i], i] for i in range(1, n)], np.int32).reshape(-1, 2)
    nbrs = [[] for _ in range(n)]
    for a, b in bonds:
        nbrs[a].append(int(b))
        nbrs[b].append(int(a))
    angles = []
    for c in range(n):
        nb = sorted(nbrs[c])
        for u in range(len(nb)):
            for w in range(u + 1, len(nb)):
                angles.append([nb[u], c, nb[w]])
    angles = np.array(angles, np.int32).reshape(-1, 3)
    ex = set()
    for a, b in bonds:
        ex.add((min(a, b), max(a, b)))
    for a, _, b in angles:
        ex.add((min(a, b), max(a, b)))
    return bonds, angles, ex


# --------------------------------------------------------------------------
# water
# --------------------------------------------------------------------------
def _random_rotations(rng, k):
    q = rng.normal(size=(k, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
    ], 1)


def _place_waters(box, n_water, solute_x, rng, clearance=0.26, tries=24):
    """Cubic lattice filling the periodic box; sites whose O would sit within
    ``clearance`` of a solute atom are dropped; ``n_water`` of the rest are
    chosen; each water gets the random orientation (of ``tries``) that keeps
    its hydrogens farthest from already placed atoms."""
    L = float(box[0])
    n = max(2, int(math.ceil(n_water ** (1.0 / 3.0))))
    while True:
        a = L / n
        g = (np.arange(n) + 0.5) * a
        sites = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
        keep = np.ones(len(sites), bool)
        if len(solute_x):
            sw = solute_x - L * np.floor(solute_x / L)
            for s in range(0, len(sites), 4096):
                d = sites[s:s + 4096, None, :] - sw[None, :, :]
                d -= L * np.round(d / L)
                keep[s:s + 4096] = np.min(np.sum(d * d, -1), 1) >= clearance ** 2
        if keep.sum() >= n_water:
            break
        n += 1
    idx = np.flatnonzero(keep)
    idx = np.sort(rng.choice(idx, size=n_water, replace=False))
    O = sites[idx]
    # lattice coordinates for a neighbour hash
    ijk = np.floor(O / a).astype(np.int64) % n
    occupant = -np.ones((n, n, n), np.int64)
    occupant[ijk[:, 0], ijk[:, 1], ijk[:, 2]] = np.arange(n_water)
    h1 = np.array([OH_R0 * math.sin(HOH_T0 / 2), OH_R0 * math.cos(HOH_T0 / 2), 0.0])
    h2 = np.array([-OH_R0 * math.sin(HOH_T0 / 2), OH_R0 * math.cos(HOH_T0 / 2), 0.0])
    H = np.zeros((n_water, 2, 3))
    placed = np.zeros(n_water, bool)
    offs = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)
                     if (i, j, k) != (0, 0, 0)])
    sol_w = solute_x - L * np.floor(solute_x / L) if len(solute_x) else np.zeros((0, 3))
    for w in rng.permutation(n_water):
        R = _random_rotations(rng, tries)
        cand = O[w][None, None, :] + np.stack([R @ h1, R @ h2], 1)  # (tries,2,3)
        nb = (ijk[w][None, :] + offs) % n
        occ = occupant[nb[:, 0], nb[:, 1], nb[:, 2]]
        occ = occ[occ >= 0]
        pts = [O[occ]]
        done = occ[placed[occ]]
        if len(done):
            pts.append(H[done].reshape(-1, 3))
        if len(sol_w):
            ds = sol_w - O[w]
            ds -= L * np.round(ds / L)
            near = np.sum(ds * ds, 1) < 0.6 ** 2
            pts.append(sol_w[near])
        P = np.concatenate(pts, 0)
        if len(P):
            d = cand[:, :, None, :] - P[None, None, :, :]
            d -= L * np.round(d / L)
            score = np.min(np.sum(d * d, -1).reshape(tries, -1), 1)
            best = int(np.argmax(score))
        else:
            best = 0
        H[w] = cand[best]
        placed[w] = True
    return O, H


# --------------------------------------------------------------------------
# systems
# --------------------------------------------------------------------------
def make_system(*, n_solute, n_water, box, r_cut, dt, seed, bias, branching=True,
                init_radius=None, final_radius=None, periodic_growth=False, gamma=1.0, T=300.0,
                eps_rf=78.0, bias_k=None, ramp_rate=None, z_target=None,
                n_steps_for_ramp=None, reach_tol=None, contact_min_sep=35):
    """One replica description (see module docstring)."""
    rng = np.random.default_rng(seed)
    L = float(box)
    center = np.full(3, L / 2)
    parent = _tree_parents(n_solute, rng, branching)
    if init_radius is None:
        init_radius = 1.0 if n_solute <= 32 else 2.0
    xs = (_grow(parent, center, init_radius, 0.30, rng, pull=0.3 if periodic_growth else 0.5,
                box=L if periodic_growth else None, escape=periodic_growth)
          if n_solute else np.zeros((0, 3)))
    xf = None
    if bias in (BIAS_CONTACT, BIAS_RMD_CONTACT):
        if final_radius is None:
            final_radius = 1.7
        xf = _grow(parent, center, final_radius, 0.25, rng, pull=1.0, escape=periodic_growth)
    bonds, angles, ex = _solute_topology(parent) if n_solute else (
        np.zeros((0, 2), np.int32), np.zeros((0, 3), np.int32), set())
    sig = rng.uniform(0.30, 0.40, n_solute)
    eps = rng.uniform(0.2, 1.0, n_solute)
    q = np.where(np.arange(n_solute) % 2 == 0, SOLUTE_CHARGE, -SOLUTE_CHARGE)
    O, H = _place_waters(np.full(3, L), n_water, xs, rng)
    N = n_solute + 3 * n_water
    x0 = np.zeros((N, 3))
    x0[:n_solute] = xs
    x0[n_solute::3] = O
    x0[n_solute + 1::3] = H[:, 0]
    x0[n_solute + 2::3] = H[:, 1]
    mass = np.concatenate([np.full(n_solute, SOLUTE_MASS), np.tile([O_MASS, H_MASS, H_MASS], n_water)])
    charge = np.concatenate([q, np.tile([O_CHARGE, H_CHARGE, H_CHARGE], n_water)])
    sigma = np.concatenate([sig, np.tile([O_SIGMA, 0.0, 0.0], n_water)])
    epsilon = np.concatenate([eps, np.tile([O_EPS, 0.0, 0.0], n_water)])
    wO = n_solute + 3 * np.arange(n_water)
    wb = np.stack([np.stack([wO, wO + 1], 1), np.stack([wO, wO + 2], 1)], 1).reshape(-1, 2)
    wa = np.stack([wO + 1, wO, wO + 2], 1)
    all_bonds = np.concatenate([bonds, wb]).astype(np.int32)
    bond_k = np.concatenate([np.full(len(bonds), SOLUTE_BOND_K), np.full(len(wb), OH_K)])
    bond_r0 = np.concatenate([np.full(len(bonds), SOLUTE_BOND_R0), np.full(len(wb), OH_R0)])
    all_angles = np.concatenate([angles, wa]).astype(np.int32)
    angle_k = np.concatenate([np.full(len(angles), SOLUTE_ANGLE_K), np.full(len(wa), HOH_K)])
    angle_t0 = np.concatenate([np.full(len(angles), SOLUTE_ANGLE_T0), np.full(len(wa), HOH_T0)])
    wex = np.concatenate([np.stack([wO, wO + 1], 1), np.stack([wO, wO + 2], 1), np.stack([wO + 1, wO + 2], 1)])
    sex = np.array(sorted(ex), np.int64).reshape(-1, 2)
    excl = np.concatenate([sex, wex]).astype(np.int32)
    kT = KB * T
    if n_steps_for_ramp is None:
        n_steps_for_ramp = 1000
    desc = dict(
        n_atoms=N, n_solute=n_solute, mass=mass, gamma=np.full(N, float(gamma)),
        charge=charge, sigma=sigma, epsilon=epsilon,
        bonds=all_bonds, bond_k=bond_k, bond_r0=bond_r0,
        angles=all_angles, angle_k=angle_k, angle_theta0=angle_t0, excl=excl,
        box=np.full(3, L), r_cut=float(r_cut), eps_rf=float(eps_rf), kT=kT, dt=float(dt),
        x0=x0, v0=None, x_final=xf, bias=int(bias),
        bias_k=0.0, ramp_rate=0.0, z_target=0.0,
        contact_r0=0.75, contact_rs=1.0, contact_rc=1.2, contact_min_sep=int(contact_min_sep),
        reach_tol=float("inf"), seed=int(seed) + 1, const_force=None,
    )
    if bias == BIAS_RG:
        desc["bias_k"] = 2000.0 if bias_k is None else bias_k
        desc["z_target"] = 0.30 if z_target is None else z_target
        desc["reach_tol"] = 0.05 if reach_tol is None else reach_tol
    elif bias in (BIAS_CONTACT, BIAS_RMD_CONTACT):
        desc["bias_k"] = 5e-3 if bias_k is None else bias_k
        desc["z_target"] = 0.0 if z_target is None else z_target
        desc["reach_tol"] = float("inf") if reach_tol is None else reach_tol
    desc["ramp_rate"] = (1.0 / (n_steps_for_ramp * dt)) if ramp_rate is None else ramp_rate
    return desc


def with_seed(desc, seed):
    """Same system, another Philox key (an independent trial path)."""
    d = dict(desc)
    d["seed"] = int(seed)
    return d


# Workload recipes -----------------------------------------------------------
def small_chain_system(seed=WORKLOAD_SEED):
    """12-bead chain + 500 waters, 2.5 nm box, rc 0.9, dt 0.5 fs, Rg bias."""
    return make_system(n_solute=12, n_water=500, box=2.5, r_cut=0.9, dt=0.0005,
                       seed=seed, bias=BIAS_RG, branching=False, init_radius=1.0,
                       n_steps_for_ramp=2000)


def solvated_chain_12560(seed=WORKLOAD_SEED, bias=BIAS_CONTACT):
    """560-atom solute + 4000 waters (12,560 atoms), 5.0 nm box, rc 1.0,
    dt 1 fs, contact-map bias toward a seeded target map."""
    return make_system(n_solute=560, n_water=4000, box=5.0, r_cut=1.0, dt=0.001,
                       seed=seed, bias=bias, init_radius=2.2, final_radius=1.8,
                       n_steps_for_ramp=20000)


def trial_batch(n_rep=64, seed=WORKLOAD_SEED, base=None, n_steps=10000):
    """n_rep trial paths of the 12,560-atom system: same start, independent Philox keys
    (seed + r + 1), so independent Maxwell velocities and noise."""
    if base is None:
        base = solvated_chain_12560(seed)
    base = dict(base)
    base["ramp_rate"] = 1.0 / (n_steps * base["dt"])
    return [with_seed(base, seed + r + 1) for r in range(n_rep)]


def _make_system_kw(kw):
    return make_system(**kw)


def uneven_batch(n_rep=32, seed=WORKLOAD_SEED, only=None, workers=1, progress=None):
    """Replicas with atom counts log-uniform in [5000, 40000], solute 280-560
    atoms, water at 33.4 /nm^3, cutoffs 0.9 or 1.2 nm.  The initial solute is
    grown at 9 atoms/nm^3 (in the smaller boxes its sphere is wider than the
    box and the growth uses minimum-image distances), the target structure at
    15 atoms/nm^3.  Each replica depends on its own seed only, so ``workers``
    processes (forked; call this before the GPU is initialised) may build them
    in parallel with the same result; ``progress(r, n_atoms)`` is called as
    each one is done."""
    rng = np.random.default_rng(seed + 4)
    jobs = []
    for r in range(n_rep):
        N = int(math.exp(rng.uniform(math.log(5000), math.log(40000))))
        ns = int(rng.integers(280, 561))
        nw = (N - ns) // 3
        L = (nw / 33.4) ** (1.0 / 3.0)
        rc = 0.9 if rng.random() < 0.5 else 1.2
        if only is not None and r not in only:
            continue  # the parameters are still drawn, so replica r is the same either way
        r_init = (3.0 * ns / (4.0 * math.pi * 9.0)) ** (1.0 / 3.0)
        r_final = (3.0 * ns / (4.0 * math.pi * 15.0)) ** (1.0 / 3.0)
        jobs.append((r, dict(n_solute=ns, n_water=nw, box=L, r_cut=rc, dt=0.001,
                             seed=seed + 100 * (r + 1), bias=BIAS_CONTACT,
                             init_radius=r_init, final_radius=r_final, periodic_growth=True,
                             n_steps_for_ramp=2000)))
    if workers <= 1 or len(jobs) <= 1:
        reps = []
        for r, kw in jobs:
            reps.append(make_system(**kw))
            if progress:
                progress(r, reps[-1]["n_atoms"])
        return reps
    import multiprocessing as mp
    with mp.get_context("fork").Pool(min(workers, len(jobs))) as pool:
        pending = [pool.apply_async(_make_system_kw, (kw,)) for _, kw in jobs]
        reps = []
        for (r, _), p in zip(jobs, pending):
            reps.append(p.get())
            if progress:
                progress(r, reps[-1]["n_atoms"])
    return reps


def derivative_batch(n_rep=16, seed=WORKLOAD_SEED, base=None):
    """16 trial paths of the 12,560-atom system for the functional gradient."""
    if base is None:
        base = solvated_chain_12560(seed)
    base = dict(base)
    base["ramp_rate"] = 1.0 / (2000 * base["dt"])
    return [with_seed(base, seed + r + 1) for r in range(n_rep)]


def tiny(seed=1, n_solute=40, n_water=60, box=2.1, r_cut=0.9, bias=BIAS_CONTACT,
         contact_min_sep=5, dt=0.001):
    """Small system for parity tests that the FP64 oracle finishes in
    milliseconds; the contact-map separation is reduced so that the CV has
    pairs at this chain length."""
    return make_system(n_solute=n_solute, n_water=n_water, box=box, r_cut=r_cut, dt=dt,
                       seed=seed, bias=bias, init_radius=0.8, final_radius=0.7,
                       contact_min_sep=contact_min_sep, n_steps_for_ramp=200)


def lj_box(seed=2, n=200, box=2.6, r_cut=1.0, charged=True, dt=0.001):
    """Solvent-free box of free LJ(+charged) particles with no bonds: used by
    pair-set and energy-conservation pins."""
    rng = np.random.default_rng(seed)
    L = float(box)
    m = int(math.ceil(n ** (1 / 3)))
    a = L / m
    g = (np.arange(m) + 0.5) * a
    sites = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    x0 = sites[np.sort(rng.choice(len(sites), n, replace=False))]
    x0 += rng.uniform(-0.05, 0.05, x0.shape) * a
    q = np.where(np.arange(n) % 2 == 0, 0.3, -0.3) if charged else np.zeros(n)
    return dict(
        n_atoms=n, n_solute=0, mass=np.full(n, 39.948), gamma=np.full(n, 1.0),
        charge=q, sigma=rng.uniform(0.30, 0.36, n), epsilon=rng.uniform(0.5, 1.0, n),
        bonds=np.zeros((0, 2), np.int32), bond_k=np.zeros(0), bond_r0=np.zeros(0),
        angles=np.zeros((0, 3), np.int32), angle_k=np.zeros(0), angle_theta0=np.zeros(0),
        excl=np.zeros((0, 2), np.int32), box=np.full(3, L), r_cut=float(r_cut), eps_rf=78.0,
        kT=KB * 300.0, dt=float(dt), x0=x0, v0=None, x_final=None, bias=BIAS_NONE,
        bias_k=0.0, ramp_rate=0.0, z_target=0.0, contact_r0=0.75, contact_rs=1.0,
        contact_rc=1.2, contact_min_sep=35, reach_tol=float("inf"), seed=int(seed) + 1,
        const_force=None,
    )


def perturbed(desc, scale, seed):
    """Copy with starting coordinates displaced by N(0, scale^2) per component."""
    d = dict(desc)
    rng = np.random.default_rng(seed)
    d["x0"] = desc["x0"] + rng.normal(scale=scale, size=desc["x0"].shape)
    return d
