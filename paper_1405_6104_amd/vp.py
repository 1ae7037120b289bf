"""Python binding of the vp C ABI (include/vp.h): argument marshalling only.

Every computation runs in the HIP kernels of libvp.so; this module converts
replica descriptions (dicts of numpy arrays, see ``synth``) into the C
structures, hands device pointers of torch tensors and the current HIP stream
to the library, and raises ``VpError`` on any non-zero status.  Importing it
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libvp.so is missing at {LIB_PATH}: build it with __graft_entry__.build()")

_lib = C.CDLL(LIB_PATH)

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)

BIAS_NONE, BIAS_CONST, BIAS_RG, BIAS_CONTACT, BIAS_RMD_CONTACT = 0, 1, 2, 3, 4
OBS = ("step", "z", "z_ref", "z_min", "phi", "status", "rebuilds", "ke", "stage_max", "stage_cap",
       "list_max", "list_cap", "exact_builds", "skin", "nstlist", "rmsd", "reached", "eval_status")
# columns of the vp_forces energy table (VP_E_*) and of an energy record (VP_REC_*)
ENERGY_COLUMNS = ("lj", "rf", "bond", "angle", "bias", "z", "z_ref", "S", "total",
                  "w_xx", "w_xy", "w_xz", "w_yx", "w_yy", "w_yz", "w_zx", "w_zy", "w_zz", "status")
RECORD_COLUMNS = ENERGY_COLUMNS + ("step", "ke", "phi")
REPLICA_UNSTABLE, REPLICA_LIST_OVERFLOW = 1, 2

STATUS = {0: "VP_OK", -1: "VP_ERR_ARG", -2: "VP_ERR_HIP", -3: "VP_ERR_NOMEM", -4: "VP_ERR_STATE",
          -5: "VP_ERR_NOPATH"}


class VpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class ReplicaDesc(C.Structure):
    _fields_ = [
        ("n_atoms", C.c_int32), ("n_solute", C.c_int32),
        ("mass", _dp), ("gamma", _dp), ("charge", _dp), ("sigma", _dp), ("epsilon", _dp),
        ("n_bonds", C.c_int32), ("bonds", _ip), ("bond_k", _dp), ("bond_r0", _dp),
        ("n_angles", C.c_int32), ("angles", _ip), ("angle_k", _dp), ("angle_theta0", _dp),
        ("n_excl", C.c_int32), ("excl", _ip),
        ("box", C.c_double * 3), ("r_cut", C.c_double), ("eps_rf", C.c_double),
        ("kT", C.c_double), ("dt", C.c_double),
        ("x0", _dp), ("v0", _dp), ("x_final", _dp),
        ("bias", C.c_int32), ("bias_k", C.c_double), ("ramp_rate", C.c_double),
        ("z_target", C.c_double),
        ("contact_r0", C.c_double), ("contact_rs", C.c_double), ("contact_rc", C.c_double),
        ("contact_min_sep", C.c_int32), ("reach_tol", C.c_double), ("seed", C.c_uint64),
        ("const_force", _dp), ("reach_rmsd", C.c_double),
    ]


DEV_ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEV_FREE = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Options(C.Structure):
    _fields_ = [("nstlist", C.c_int32), ("skin", C.c_double), ("steps_per_graph", C.c_int32),
                ("use_graph", C.c_int32), ("max_neighbors", C.c_int32),
                ("tangent", C.c_int32), ("force_shape", C.c_int32), ("autotune", C.c_int32),
                ("nst_out", C.c_int32), ("out_capacity", C.c_int32), ("stage_cap", C.c_int32),
                ("contact_order", C.c_int32),
                ("dev_alloc", DEV_ALLOC), ("dev_free", DEV_FREE), ("alloc_ctx", C.c_void_p)]

FORCE_SHAPES = 4


class TileBucket(C.Structure):
    _fields_ = [("r_cut", C.c_double), ("log2_atoms", C.c_int32), ("n_replicas", C.c_int32),
                ("n_blocks", C.c_int32), ("shape", C.c_int32), ("waves", C.c_int32),
                ("entries", C.c_int32), ("ms", C.c_double * FORCE_SHAPES)]


_vp = C.c_void_p
_lib.vp_system_create.restype = C.c_int
_lib.vp_system_create.argtypes = [C.POINTER(ReplicaDesc), C.c_int32, C.POINTER(Options), C.POINTER(_vp)]
_lib.vp_system_destroy.restype = C.c_int
_lib.vp_system_destroy.argtypes = [_vp]
_lib.vp_forces.restype = C.c_int
_lib.vp_forces.argtypes = [_vp, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]
_lib.vp_forces_noalloc.restype = C.c_int
_lib.vp_forces_noalloc.argtypes = [_vp, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]
_lib.vp_step_batch.restype = C.c_int
_lib.vp_step_batch.argtypes = [_vp, C.c_int32, C.c_void_p]
_lib.vp_functional.restype = C.c_int
_lib.vp_functional.argtypes = [_vp, _dp, _dp]
_lib.vp_select_path.restype = C.c_int
_lib.vp_select_path.argtypes = [_vp, C.POINTER(C.c_uint8), _ip, _dp]
_lib.vp_get_state.restype = C.c_int
_lib.vp_get_state.argtypes = [_vp, C.c_void_p, C.c_void_p, C.c_void_p]
_lib.vp_observables.restype = C.c_int
_lib.vp_observables.argtypes = [_vp, _dp]
_lib.vp_sizes.restype = C.c_int
_lib.vp_sizes.argtypes = [_vp, C.POINTER(C.c_int64), _ip]
_lib.vp_debug_pairs.restype = C.c_int
_lib.vp_debug_pairs.argtypes = [_vp, C.c_int32, _ip, C.c_int64, C.POINTER(C.c_int64)]
_lib.vp_debug_noise.restype = C.c_int
_lib.vp_debug_noise.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int32,
                                C.c_void_p, C.c_void_p]
_lib.vp_set_timing.restype = C.c_int
_lib.vp_set_timing.argtypes = [_vp, C.c_int32]
_lib.vp_kernel_timing.restype = C.c_int
_lib.vp_kernel_timing.argtypes = [_vp, _dp, C.POINTER(C.c_int64), C.c_int32]
_lib.vp_debug_force_dir.restype = C.c_int
_lib.vp_debug_force_dir.argtypes = [_vp, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]
_lib.vp_debug_trajectory_state.restype = C.c_int
_lib.vp_debug_trajectory_state.argtypes = [_vp, _dp, _dp, _dp, _dp, _dp]
_lib.vp_tile_buckets.restype = C.c_int
_lib.vp_tile_buckets.argtypes = [_vp, C.POINTER(TileBucket), C.c_int32, C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32)]
_lib.vp_debug_set_tiles.restype = C.c_int
_lib.vp_debug_set_tiles.argtypes = [_vp, C.POINTER(C.c_int32), C.c_int32]
_lib.vp_pair_count.restype = C.c_int
_lib.vp_pair_count.argtypes = [_vp, C.c_int32, C.POINTER(C.c_int64)]
_lib.vp_energy_records.restype = C.c_int
_lib.vp_energy_records.argtypes = [_vp, _dp, C.c_int32, C.POINTER(C.c_int32)]
_lib.vp_device_bytes.restype = C.c_int
_lib.vp_device_bytes.argtypes = [_vp, C.POINTER(C.c_int64)]
_lib.vp_contact_order.restype = C.c_int
_lib.vp_contact_order.argtypes = [_vp, C.c_int32, _ip, C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_int32)]
_lib.vp_path_similarity.restype = C.c_int
_lib.vp_path_similarity.argtypes = [_vp, _dp]


class ToyParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("A1", "A2", "A3", "s1", "s2", "s3", "w", "xm", "ym",
                                          "gamma", "mass", "kT", "dt", "x0", "y0", "r_product",
                                          "r_gate")] + [("n_steps", C.c_int32), ("path_stride", C.c_int32)]


TOY_PLAIN, TOY_RMD, TOY_SMD = 0, 1, 2
TOY_COLUMNS = ("phi", "reached", "t_reach", "x", "y", "z_min", "theta_gate")
_lib.vp_toy_trials.restype = C.c_int
_lib.vp_toy_trials.argtypes = [C.POINTER(ToyParams), C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p]
_lib.vp_toy_select.restype = C.c_int
_lib.vp_toy_select.argtypes = [_dp, C.c_int32, C.POINTER(C.c_uint8), _ip, _dp]
_lib.vp_last_error.restype = C.c_char_p
_lib.vp_last_error.argtypes = []

EXPORTED = ("vp_system_create", "vp_system_destroy", "vp_forces", "vp_step_batch",
            "vp_functional", "vp_select_path", "vp_get_state", "vp_observables", "vp_sizes",
            "vp_debug_pairs", "vp_debug_noise", "vp_set_timing", "vp_kernel_timing", "vp_pair_count",
            "vp_debug_force_dir", "vp_debug_trajectory_state", "vp_tile_buckets", "vp_debug_set_tiles",
            "vp_energy_records", "vp_device_bytes", "vp_forces_noalloc", "vp_contact_order",
            "vp_path_similarity", "vp_toy_trials", "vp_toy_select", "vp_last_error")


def _check(st):
    if st != 0:
        raise VpError(st, (_lib.vp_last_error() or b"").decode(errors="replace"))


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


def _desc(d, keep):
    n, ns = int(d["n_atoms"]), int(d["n_solute"])
    arrs = {}
    for k in ("mass", "gamma", "charge", "sigma", "epsilon", "bond_k", "bond_r0", "angle_k",
              "angle_theta0"):
        arrs[k] = _f64(d[k])
    for k in ("bonds", "angles", "excl"):
        arrs[k] = np.ascontiguousarray(d[k], dtype=np.int32)
    arrs["x0"] = _f64(d["x0"], (n, 3))
    for k, shape in (("v0", (n, 3)), ("x_final", (ns, 3)), ("const_force", (ns, 3))):
        v = d.get(k)
        arrs[k] = None if v is None else _f64(v, shape)
    keep.append(arrs)
    s = ReplicaDesc()
    s.n_atoms, s.n_solute = n, ns
    for k in ("mass", "gamma", "charge", "sigma", "epsilon", "bond_k", "bond_r0", "angle_k",
              "angle_theta0", "x0"):
        setattr(s, k, arrs[k].ctypes.data_as(_dp))
    for k in ("v0", "x_final", "const_force"):
        setattr(s, k, arrs[k].ctypes.data_as(_dp) if arrs[k] is not None else _dp())
    s.n_bonds, s.bonds = len(arrs["bonds"]), arrs["bonds"].ctypes.data_as(_ip)
    s.n_angles, s.angles = len(arrs["angles"]), arrs["angles"].ctypes.data_as(_ip)
    s.n_excl, s.excl = len(arrs["excl"]), arrs["excl"].ctypes.data_as(_ip)
    for a in range(3):
        s.box[a] = float(d["box"][a])
    s.r_cut, s.eps_rf, s.kT, s.dt = (float(d[k]) for k in ("r_cut", "eps_rf", "kT", "dt"))
    s.bias = int(d["bias"])
    s.bias_k, s.ramp_rate, s.z_target = (float(d[k]) for k in ("bias_k", "ramp_rate", "z_target"))
    s.contact_r0, s.contact_rs, s.contact_rc = (float(d[k]) for k in ("contact_r0", "contact_rs", "contact_rc"))
    s.contact_min_sep = int(d["contact_min_sep"])
    s.reach_tol = float(d["reach_tol"])
    s.reach_rmsd = float(d.get("reach_rmsd", float("inf")))
    s.seed = int(d["seed"]) & 0xFFFFFFFFFFFFFFFF
    return s


def _torch_allocator():
    """dev_alloc / dev_free callbacks that take the library's device memory from
    torch's caching allocator on the current device and stream."""
    import torch

    def alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except RuntimeError:
            return None

    def free(ptr, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    return DEV_ALLOC(alloc), DEV_FREE(free)


class System:
    """A batch of trial trajectories (vp_system)."""

    def __init__(self, reps, nstlist=0, skin=0.0, steps_per_graph=0, use_graph=True,
                 max_neighbors=0, tangent=False, force_shape=0, autotune=False, nst_out=0,
                 out_capacity=0, stage_cap=0, contact_order=False, torch_memory=False):
        """torch_memory: the library takes all its device memory from torch's
        caching allocator (vp_options.dev_alloc) instead of hipMalloc."""
        keep = []
        descs = (ReplicaDesc * len(reps))(*[_desc(d, keep) for d in reps])
        opt = Options()
        opt.nstlist, opt.skin, opt.steps_per_graph = nstlist, skin, steps_per_graph
        opt.use_graph, opt.max_neighbors = int(bool(use_graph)), max_neighbors
        opt.tangent = int(bool(tangent))
        opt.force_shape = int(force_shape)
        opt.autotune = int(bool(autotune))
        opt.nst_out, opt.out_capacity, opt.stage_cap = int(nst_out), int(out_capacity), int(stage_cap)
        opt.contact_order = int(bool(contact_order))
        self._alloc = _torch_allocator() if torch_memory else None  # kept alive with the system
        if self._alloc is not None:
            opt.dev_alloc, opt.dev_free = self._alloc
        h = _vp()
        _check(_lib.vp_system_create(descs, len(reps), C.byref(opt), C.byref(h)))
        self._h = h
        self.n_reps = len(reps)
        self.counts = [int(d["n_atoms"]) for d in reps]
        self.offsets = np.concatenate([[0], np.cumsum(self.counts)]).astype(np.int64)
        self.n_total = int(self.offsets[-1])

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.vp_system_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------------- calls
    def forces(self, x, t=0.0, energies=False):
        """Total forces (and the [R, len(ENERGY_COLUMNS)] FP64 energy table) at
        positions x (float32 CUDA tensor [N_total, 3], user order)."""
        import torch
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.shape == (self.n_total, 3)
        f = torch.empty_like(x)
        e = (torch.zeros((self.n_reps, len(ENERGY_COLUMNS)), dtype=torch.float64, device=x.device)
             if energies else None)
        _check(_lib.vp_forces(self._h, _ptr(x), _ptr(f), _ptr(e) if e is not None else None,
                              float(t), _stream()))
        return (f, e) if energies else f

    def forces_noalloc(self, x, f, e=None, t=0.0):
        """vp_forces_noalloc into caller-provided tensors f ([N_total, 3] float32)
        and e ([R, len(ENERGY_COLUMNS)] float64 or None)."""
        _check(_lib.vp_forces_noalloc(self._h, _ptr(x), _ptr(f), _ptr(e) if e is not None else None,
                                      float(t), _stream()))

    def step_batch(self, n):
        _check(_lib.vp_step_batch(self._h, int(n), _stream()))

    def functional(self, gradient=False):
        """Phi per replica; with gradient=True also dPhi/d(bias_k, ramp_rate)
        as an [R, 2] array (needs tangent=True at creation)."""
        phi = np.zeros(self.n_reps)
        g = np.zeros((self.n_reps, 2)) if gradient else None
        _check(_lib.vp_functional(self._h, phi.ctypes.data_as(_dp), g.ctypes.data_as(_dp) if gradient else None))
        return (phi, g) if gradient else phi

    def tile_buckets(self):
        """Size buckets (cutoff, floor(log2 n)) with the force tile shape each
        runs with and, when autotuned, the timed ms per shape; plus whether the
        buckets run as separate launches."""
        n = C.c_int32(0)
        split = C.c_int32(0)
        _check(_lib.vp_tile_buckets(self._h, None, 0, C.byref(n), C.byref(split)))
        arr = (TileBucket * max(n.value, 1))()
        _check(_lib.vp_tile_buckets(self._h, arr, n.value, C.byref(n), C.byref(split)))
        out = []
        for b in arr[:n.value]:
            out.append({"r_cut": b.r_cut, "log2_atoms": b.log2_atoms, "replicas": b.n_replicas,
                        "blocks": b.n_blocks, "shape": b.shape, "tile": f"{b.waves}x{b.entries}",
                        "ms": [float(t) for t in b.ms]})
        return out, bool(split.value)

    def set_tiles(self, shapes):
        """Diagnostic: force tile shape per size bucket (tile_buckets order),
        one launch per shape."""
        arr = (C.c_int32 * len(shapes))(*[int(k) for k in shapes])
        _check(_lib.vp_debug_set_tiles(self._h, arr, len(shapes)))

    def trajectory_state(self, tangents=False):
        """Exact state in user order (FP64): x, v [N, 3]; with tangents also
        xt, vt [2, N, 3] and the derivative accumulators pd [R, 4]."""
        x = np.zeros((self.n_total, 3))
        v = np.zeros((self.n_total, 3))
        if not tangents:
            _check(_lib.vp_debug_trajectory_state(self._h, x.ctypes.data_as(_dp), v.ctypes.data_as(_dp),
                                                  None, None, None))
            return x, v
        xt = np.zeros((2, self.n_total, 3))
        vt = np.zeros((2, self.n_total, 3))
        pd = np.zeros((self.n_reps, 4))
        _check(_lib.vp_debug_trajectory_state(self._h, x.ctypes.data_as(_dp), v.ctypes.data_as(_dp),
                                              xt.ctypes.data_as(_dp), vt.ctypes.data_as(_dp),
                                              pd.ctypes.data_as(_dp)))
        return x, v, xt, vt, pd

    def force_dir(self, x, dx, t=0.0):
        """Directional derivatives of the total force along dx ([2, N_total, 3]
        float32 CUDA tensor), parameters fixed (needs tangent=True)."""
        import torch
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.shape == (self.n_total, 3)
        assert dx.is_cuda and dx.dtype == torch.float32 and dx.is_contiguous() and dx.shape == (2, self.n_total, 3)
        out = torch.empty_like(dx)
        _check(_lib.vp_debug_force_dir(self._h, _ptr(x), _ptr(dx), _ptr(out), float(t), _stream()))
        return out

    def select_path(self, eligible=None):
        """(best replica or -1, its functional)."""
        best = C.c_int32()
        bp = C.c_double()
        el = None
        if eligible is not None:
            el = np.ascontiguousarray(eligible, dtype=np.uint8)
        st = _lib.vp_select_path(self._h, el.ctypes.data_as(C.POINTER(C.c_uint8)) if el is not None else None,
                                 C.byref(best), C.byref(bp))
        if st == -5:
            return -1, float("inf")
        _check(st)
        return best.value, bp.value

    def get_state(self):
        import torch
        x = torch.empty((self.n_total, 3), dtype=torch.float32, device="cuda")
        v = torch.empty_like(x)
        _check(_lib.vp_get_state(self._h, _ptr(x), _ptr(v), _stream()))
        return x, v

    def observables(self):
        o = np.zeros((self.n_reps, len(OBS)))
        _check(_lib.vp_observables(self._h, o.ctypes.data_as(_dp)))
        return o

    def energy_records(self):
        """Energy records [R, n, len(RECORD_COLUMNS)] held so far, oldest first
        (needs nst_out > 0 at creation)."""
        n = C.c_int32()
        _check(_lib.vp_energy_records(self._h, None, 0, C.byref(n)))
        out = np.zeros((self.n_reps, n.value, len(RECORD_COLUMNS)))
        if n.value:
            _check(_lib.vp_energy_records(self._h, out.ctypes.data_as(_dp), n.value, C.byref(n)))
        return out

    def contact_order(self, rep):
        """Native contacts of replica rep ([n, 2] int32) and the step at which each
        first formed ([n] int64, -1 = not yet)."""
        n = C.c_int32()
        _check(_lib.vp_contact_order(self._h, int(rep), None, None, 0, C.byref(n)))
        pairs = np.zeros((max(n.value, 1), 2), np.int32)
        steps = np.zeros(max(n.value, 1), np.int64)
        if n.value:
            _check(_lib.vp_contact_order(self._h, int(rep), pairs.ctypes.data_as(_ip),
                                         steps.ctypes.data_as(C.POINTER(C.c_int64)), n.value, C.byref(n)))
        return pairs[: n.value], steps[: n.value]

    def path_similarity(self):
        """[R, R] path similarity of every pair of replicas with the same native contacts."""
        out = np.zeros((self.n_reps, self.n_reps))
        _check(_lib.vp_path_similarity(self._h, out.ctypes.data_as(_dp)))
        return out

    def device_bytes(self):
        b = C.c_int64()
        _check(_lib.vp_device_bytes(self._h, C.byref(b)))
        return b.value

    def set_timing(self, on):
        _check(_lib.vp_set_timing(self._h, int(bool(on))))

    def kernel_timing(self, reset=False):
        """(mean force-kernel duration in ms, number of launches timed)."""
        ms = C.c_double()
        n = C.c_int64()
        _check(_lib.vp_kernel_timing(self._h, C.byref(ms), C.byref(n), int(bool(reset))))
        return ms.value, n.value

    def pair_count(self, rep):
        n = C.c_int64()
        _check(_lib.vp_pair_count(self._h, int(rep), C.byref(n)))
        return n.value

    def debug_pairs(self, rep):
        cnt = C.c_int64()
        _check(_lib.vp_debug_pairs(self._h, int(rep), None, 0, C.byref(cnt)))
        out = np.zeros((max(cnt.value, 1), 2), np.int32)
        _check(_lib.vp_debug_pairs(self._h, int(rep), out.ctypes.data_as(_ip), cnt.value, C.byref(cnt)))
        return out[: cnt.value]


def debug_noise(seed, atom0, step, tag, n):
    import torch
    out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    _check(_lib.vp_debug_noise(int(seed) & 0xFFFFFFFFFFFFFFFF, atom0, step, tag, n, _ptr(out), _stream()))
    return out


def _energy_autograd():
    import torch

    class VpEnergy(torch.autograd.Function):
        """U(X,Y) + U_bias per replica as a differentiable function of the
        positions: forward runs the energy kernels, backward the force kernels
        (grad_x = -F scaled by the incoming gradient of each replica)."""

        @staticmethod
        def forward(ctx, x, system, t):
            f, e = system.forces(x.detach().contiguous(), t, energies=True)
            ctx.save_for_backward(f)
            ctx.offsets = system.offsets
            return e[:, ENERGY_COLUMNS.index("total")].clone()

        @staticmethod
        def backward(ctx, gout):
            (f,) = ctx.saved_tensors
            reps = torch.repeat_interleave(
                gout.to(f.dtype), torch.as_tensor(np.diff(ctx.offsets), device=f.device))
            return -f * reps[:, None], None, None

    return VpEnergy


def energy(x, system, t=0.0):
    """Differentiable total energy per replica (torch autograd)."""
    return _energy_autograd().apply(x, system, t)


def toy_trials(params, kinds, ks, seeds, path_stride=0):
    """Toy-model trials on the GPU: params dict (keys of ToyParams), kinds /
    ks / seeds per trial.  Returns results [n, len(TOY_COLUMNS)] (numpy) and,
    with path_stride > 0, the paths [n, n_steps // path_stride + 1, 2]."""
    import torch
    p = ToyParams()
    for k, _ in ToyParams._fields_:
        if k in params:
            setattr(p, k, params[k])
    p.path_stride = int(path_stride)
    n = len(kinds)
    dev = torch.device("cuda")
    kd = torch.as_tensor(np.asarray(kinds, np.int32), device=dev)
    kk = torch.as_tensor(np.asarray(ks, np.float64), device=dev)
    sd = torch.as_tensor(np.asarray(seeds, np.uint64).view(np.int64), device=dev)
    out = torch.empty((n, len(TOY_COLUMNS)), dtype=torch.float64, device=dev)
    path = (torch.empty((n, p.n_steps // path_stride + 1, 2), dtype=torch.float32, device=dev)
            if path_stride > 0 else None)
    _check(_lib.vp_toy_trials(C.byref(p), n, _ptr(kd), _ptr(kk), _ptr(sd), _ptr(out),
                              _ptr(path) if path is not None else None, _stream()))
    res = out.cpu().numpy()
    return (res, path.cpu().numpy()) if path is not None else res


def toy_select(results, eligible=None):
    """(best trial or -1, its functional) over toy results."""
    r = np.ascontiguousarray(results, dtype=np.float64)
    best = C.c_int32()
    bp = C.c_double()
    el = None if eligible is None else np.ascontiguousarray(eligible, dtype=np.uint8)
    st = _lib.vp_toy_select(r.ctypes.data_as(_dp), len(r),
                            el.ctypes.data_as(C.POINTER(C.c_uint8)) if el is not None else None,
                            C.byref(best), C.byref(bp))
    if st == -5:
        return -1, float("inf")
    _check(st)
    return best.value, bp.value
