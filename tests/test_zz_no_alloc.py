"""vp_forces_noalloc (evaluation context in the library's static device
scratch) against vp_forces, through the C ABI: the same bits for forces and
the energy table, on two calls in a row (the second on a smaller system, over
what the first left in the scratch), no allocation by the library, and the
size limit reported as an argument error."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1405_6104_amd import synth, vp  # noqa: E402

pytestmark = pytest.mark.gpu

GRID = 2.0 ** 22


def positions(reps):
    x = np.concatenate([np.rint(np.asarray(d["x0"], np.float64) * GRID) / GRID for d in reps])
    return torch.from_numpy(x.astype(np.float32)).cuda()


def evaluate(fn, system, x, t):
    """One call of fn (vp_forces or vp_forces_noalloc) through the C ABI."""
    f = torch.full_like(x, float("nan"))
    e = torch.full((system.n_reps, len(vp.ENERGY_COLUMNS)), float("nan"), dtype=torch.float64, device=x.device)
    st = fn(system._h, C.c_void_p(x.data_ptr()), C.c_void_p(f.data_ptr()), C.c_void_p(e.data_ptr()),
            C.c_double(t), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert st == 0, vp._lib.vp_last_error()
    return f.cpu().numpy(), e.cpu().numpy()


def test_noalloc_forces_equal_vp_forces_on_two_calls_the_second_smaller():
    first = [dict(synth.tiny(seed=4), bias_k=0.05), synth.small_chain_system(),
             synth.tiny(seed=5, bias=synth.BIAS_RG)]
    second = [dict(synth.tiny(seed=8, n_solute=20, n_water=30, box=1.9, r_cut=0.85, contact_min_sep=3),
                   bias_k=0.1)]
    for reps, t in ((first, 0.03), (second, 0.01)):
        system = vp.System(reps)
        x = positions(reps)
        held = system.device_bytes()
        f_na, e_na = evaluate(vp._lib.vp_forces_noalloc, system, x, t)
        assert system.device_bytes() == held  # nothing allocated for the call
        f_ref, e_ref = evaluate(vp._lib.vp_forces, system, x, t)
        assert np.all(np.isfinite(f_ref)) and np.all(np.isfinite(e_ref))
        assert np.array_equal(f_na, f_ref) and np.array_equal(e_na, e_ref)
        # again, over the scratch contents the reference call did not touch
        f_again, e_again = evaluate(vp._lib.vp_forces_noalloc, system, x, t)
        assert np.array_equal(f_again, f_ref) and np.array_equal(e_again, e_ref)


def test_noalloc_rejects_a_system_beyond_its_scratch():
    base = synth.solvated_chain_12560()
    reps = [synth.with_seed(base, 1 + r) for r in range(3)]
    system = vp.System(reps)
    x = positions(reps)
    f = torch.empty_like(x)
    st = vp._lib.vp_forces_noalloc(system._h, C.c_void_p(x.data_ptr()), C.c_void_p(f.data_ptr()), None,
                                   C.c_double(0.0), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == -1 and b"static scratch" in vp._lib.vp_last_error()
