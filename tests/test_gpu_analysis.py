"""GPU parity of the toy-model trials (supplement, "Illustrative Application
in a Toy Model") and of the contact-formation order and path similarity
(main text, mechanism analysis) against the FP64 oracle, through the C ABI.

Tolerances: toy trials run in FP64 on both sides with products and sums
rounded separately; they differ only in the last bits of the transcendental
functions (log, sin, cos of the noise, exp, atan2), so positions and Phi
agree to 1e-9 relative over thousands of steps and the integer outcomes
(first passage) exactly.  Contact formation and path similarity are integer
decisions on the same grid positions: exact.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import oracle as O  # noqa: E402
from paper_1405_6104_amd import synth, vp  # noqa: E402

pytestmark = pytest.mark.gpu

PAPER_TOY = dict(A1=30.0, A2=20.0, A3=6.0, s1=1.0, s2=2.0, s3=2.0, w=0.03, xm=1.5, ym=0.0,
                 gamma=1.0, mass=1.0, kT=0.2, dt=0.02, x0=0.0, y0=5.0, r_product=0.5, r_gate=2.0)


def say(*a):
    print(*a, flush=True)


def toy_batch(n_each=48, seed0=5000):
    kinds, ks, seeds = [], [], []
    for kind, kvals in ((vp.TOY_PLAIN, [0.0]), (vp.TOY_RMD, [0.5, 2.0, 8.0]), (vp.TOY_SMD, [0.05, 0.5])):
        for k in kvals:
            for r in range(n_each):
                kinds.append(kind)
                ks.append(k)
                seeds.append(seed0 + len(seeds))
    return kinds, ks, seeds


@pytest.mark.parametrize("n_steps", [3000, 30000])
def test_toy_trials_match_the_oracle(n_steps):
    params = dict(PAPER_TOY, n_steps=n_steps)
    kinds, ks, seeds = toy_batch(n_each=48 if n_steps <= 3000 else 8)
    stride = 100
    res, paths = vp.toy_trials(params, kinds, ks, seeds, path_stride=stride)
    col = {c: i for i, c in enumerate(vp.TOY_COLUMNS)}
    worst = 0.0
    for t, (kind, k, seed) in enumerate(zip(kinds, ks, seeds)):
        o, path = O.toy_run(params, kind, k, seed, path=True)
        g = res[t]
        assert g[col["reached"]] == o["reached"] and g[col["t_reach"]] == o["t_reach"], (t, g, o)
        for c in ("x", "y"):
            worst = max(worst, abs(g[col[c]] - o[c]))
            assert abs(g[col[c]] - o[c]) <= 1e-9 * max(1.0, abs(o[c])), (t, c, g[col[c]], o[c])
        assert abs(g[col["phi"]] - o["phi"]) <= 1e-9 * abs(o["phi"]) + 1e-300, (t, g[col["phi"]], o["phi"])
        for c in ("z_min", "theta_gate"):
            if np.isnan(o[c]):
                assert np.isnan(g[col[c]])
            else:
                assert abs(g[col[c]] - o[c]) <= 1e-9 * max(1.0, abs(o[c])), (t, c)
        assert np.abs(paths[t] - path[::stride].astype(np.float32)).max() <= 1e-5
    say(f"toy {n_steps} steps: {len(kinds)} trials, largest |dx| {worst:.2e}, "
        f"reached {int(res[:, col['reached']].sum())}")


def test_toy_selection_matches_the_oracle():
    params = dict(PAPER_TOY, n_steps=2000)
    kinds = [vp.TOY_RMD] * 64
    ks = [2.0] * 64
    seeds = list(range(900, 964))
    res = vp.toy_trials(params, kinds, ks, seeds)
    ora = [O.toy_run(params, k, kk, s) for k, kk, s in zip(kinds, ks, seeds)]
    phi = np.array([o["phi"] for o in ora])
    reached = np.array([o["reached"] for o in ora], np.uint8)
    assert 0 < reached.sum()
    rc, best_o, bp_o = O.select(phi, reached)
    best, bp = vp.toy_select(res)
    assert best == best_o and abs(bp - bp_o) <= 1e-9 * bp_o
    elig = np.ones(64, np.uint8)
    elig[best] = 0
    assert vp.toy_select(res, elig)[0] == O.select(phi, reached, elig)[1]
    assert vp.toy_select(res, np.zeros(64, np.uint8))[0] == -1


def test_contact_formation_order_and_similarity_match_the_oracle():
    """Replicas biased toward their product: the first-formation step of each
    native contact, tracked on the GPU every step, equals the oracle's rule
    applied to the GPU's exact positions at every step; the path similarity
    of the replicas equals the oracle's on those formation steps."""
    base = dict(synth.tiny(seed=6), bias_k=2.0, ramp_rate=60.0)
    reps = [synth.with_seed(base, 300 + r) for r in range(4)]
    system = vp.System(reps, contact_order=True, steps_per_graph=5)
    o = O.Oracle(reps[0])
    pairs = o.native_contacts()
    nsteps = 40
    first = np.full((len(reps), len(pairs)), -1, np.int64)

    def mark(step):
        x, _ = system.trajectory_state()
        for r in range(len(reps)):
            a, b = system.offsets[r], system.offsets[r + 1]
            formed = o.contacts_formed(x[a:b], pairs)
            first[r, (first[r] < 0) & formed] = step

    mark(0)
    for n in range(1, nsteps + 1):
        system.step_batch(1)
        mark(n)
    for r in range(len(reps)):
        gp, gt = system.contact_order(r)
        assert np.array_equal(gp, pairs)
        assert np.array_equal(gt, first[r]), (r, np.flatnonzero(gt != first[r])[:5])
    formed_during = int(np.sum(first > 0))
    say(f"contacts {len(pairs)}, formed at step 0: {int(np.sum(first == 0))}, during the run: {formed_during}")
    assert formed_during > 0
    sim = system.path_similarity()
    key = np.where(first < 0, np.iinfo(np.int64).max, first)
    for a in range(len(reps)):
        assert sim[a, a] == 1.0
        for b in range(len(reps)):
            if a != b:
                assert sim[a, b] == O.path_similarity(key[a], key[b]), (a, b, sim[a, b])
    say("similarity", np.round(sim, 4).tolist())


def test_path_similarity_of_a_64_replica_batch_is_symmetric_and_bounded():
    """All pairs of a 64-trial batch of the 12,560-atom system after a short
    run (the analysis call the trial ensembles need), against the oracle on
    a few pairs."""
    reps = synth.trial_batch(64, n_steps=200)
    system = vp.System(reps, contact_order=True)
    system.step_batch(40)
    sim = system.path_similarity()
    assert np.allclose(sim, sim.T, equal_nan=False) and np.all((sim >= 0) & (sim <= 1))
    times = [system.contact_order(r)[1] for r in (0, 1, 63)]
    key = [np.where(t < 0, np.iinfo(np.int64).max, t) for t in times]
    assert sim[0, 1] == O.path_similarity(key[0], key[1])
    assert sim[1, 63] == O.path_similarity(key[1], key[2])
