"""CPU checks of the C ABI: the built library loads, exports every function
that include/vp.h declares, and rejects invalid arguments before touching
the GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1405_6104_amd", "libvp.so")
HEADER = os.path.join(ROOT, "include", "vp.h")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:vp_status|const char \*)\s*(vp_[a-z_]+)\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("vp_system_create", "vp_forces", "vp_step_batch", "vp_functional", "vp_select_path"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvp.so not built")
def test_library_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n
    from paper_1405_6104_amd import vp
    assert set(vp.EXPORTED) == set(declared())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvp.so not built")
def test_invalid_arguments_are_rejected_without_a_gpu():
    from paper_1405_6104_amd import synth, vp
    d = synth.tiny(seed=1)
    bad = dict(d, r_cut=1.2)  # >= box/2 for the 2.1 nm box
    with pytest.raises(vp.VpError) as e:
        vp.System([bad])
    assert e.value.status == -1 and "half the box" in str(e.value)
    bad = dict(d, bonds=np.array([[0, 10_000]], np.int32), bond_k=np.ones(1), bond_r0=np.ones(1))
    with pytest.raises(vp.VpError) as e:
        vp.System([bad])
    assert e.value.status == -1 and "bond index" in str(e.value)
    bad = dict(d, bonds=np.array([[3, 3]], np.int32), bond_k=np.ones(1), bond_r0=np.ones(1))
    with pytest.raises(vp.VpError) as e:
        vp.System([bad])
    assert e.value.status == -1 and "itself" in str(e.value)
    bad = dict(d, angles=np.array([[2, 3, 2]], np.int32), angle_k=np.ones(1), angle_theta0=np.ones(1))
    with pytest.raises(vp.VpError) as e:
        vp.System([bad])
    assert e.value.status == -1 and "twice" in str(e.value)
    bad = dict(d, x_final=None)
    with pytest.raises(vp.VpError) as e:
        vp.System([bad])
    assert "x_final" in str(e.value)
    with pytest.raises(vp.VpError):
        vp.System([])


def test_binding_fails_loudly_without_the_library(tmp_path):
    """A copy of the package without libvp.so cannot be imported: there is no
    fallback path."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_1405_6104_amd"
    shutil.copytree(os.path.join(ROOT, "paper_1405_6104_amd"), pkg,
                    ignore=shutil.ignore_patterns("*.so", "__pycache__", "csrc"))
    r = subprocess.run([sys.executable, "-c", "import paper_1405_6104_amd.vp"], cwd=tmp_path,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "libvp.so" in (r.stderr + r.stdout)


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
