"""ctypes wrapper of the FP64 CPU oracle (liboracle.so, built from oracle.c).

TEST INFRASTRUCTURE ONLY.  Imported by the test-suite, by the smoke check and
by the benchmark's CPU-baseline leg; the product library never imports it.
It takes replica descriptions from the synthetic input generator (plain dicts
of numpy arrays) and nothing from the HIP path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_up = C.POINTER(C.c_uint32)
_u8p = C.POINTER(C.c_uint8)


class _Sys(C.Structure):
    _fields_ = [
        ("n_atoms", C.c_int32), ("n_solute", C.c_int32),
        ("mass", _dp), ("gamma", _dp), ("charge", _dp), ("sigma", _dp), ("epsilon", _dp),
        ("n_bonds", C.c_int32), ("bonds", _ip), ("bond_k", _dp), ("bond_r0", _dp),
        ("n_angles", C.c_int32), ("angles", _ip), ("angle_k", _dp), ("angle_theta0", _dp),
        ("n_excl", C.c_int32), ("excl", _ip),
        ("box", C.c_double * 3), ("r_cut", C.c_double), ("eps_rf", C.c_double),
        ("kT", C.c_double), ("dt", C.c_double),
        ("x_final", _dp),
        ("bias", C.c_int32), ("bias_k", C.c_double), ("ramp_rate", C.c_double),
        ("z_target", C.c_double),
        ("contact_r0", C.c_double), ("contact_rs", C.c_double), ("contact_rc", C.c_double),
        ("contact_min_sep", C.c_int32),
        ("reach_tol", C.c_double), ("seed", C.c_uint64), ("const_force", _dp),
        ("reach_rmsd", C.c_double),
    ]


class State(C.Structure):
    _fields_ = [("step", C.c_int64), ("phi_acc", C.c_double), ("s_last", C.c_double),
                ("z0", C.c_double), ("z_m", C.c_double), ("z_last", C.c_double),
                ("status", C.c_int32), ("pad", C.c_int32)]


class ToyParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("A1", "A2", "A3", "s1", "s2", "s3", "w", "xm", "ym",
                                          "gamma", "mass", "kT", "dt", "x0", "y0", "r_product",
                                          "r_gate")] + [("n_steps", C.c_int32), ("pad", C.c_int32)]


TOY_COLUMNS = ("phi", "reached", "t_reach", "x", "y", "z_min", "theta_gate")
TOY_PLAIN, TOY_RMD, TOY_SMD = 0, 1, 2

TERMS = ("e_lj", "e_rf", "e_bond", "e_angle", "e_bias", "z", "z_ref", "S", "u_total",
         "w_xx", "w_xy", "w_xz", "w_yx", "w_yy", "w_yz", "w_zx", "w_zy", "w_zz")

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library missing: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        L.ora_create.restype = C.c_void_p
        L.ora_create.argtypes = [C.POINTER(_Sys)]
        L.ora_destroy.argtypes = [C.c_void_p]
        L.ora_philox4x32_10.argtypes = [_up, _up, _up]
        L.ora_uniforms.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _dp]
        L.ora_normals.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _dp]
        L.ora_pairs.restype = C.c_int64
        L.ora_pairs.argtypes = [C.c_void_p, _dp, C.c_int32, _ip, C.c_int64]
        L.ora_forces.restype = C.c_int
        L.ora_forces.argtypes = [C.c_void_p, _dp, C.c_double, C.POINTER(State), C.c_int32, _dp, _dp, _dp]
        L.ora_cv.restype = C.c_double
        L.ora_cv.argtypes = [C.c_void_p, _dp, _dp]
        L.ora_contact_value.restype = C.c_double
        L.ora_contact_value.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, _dp]
        L.ora_init.restype = C.c_int
        L.ora_init.argtypes = [C.c_void_p, _dp, C.POINTER(State)]
        L.ora_maxwell.argtypes = [C.c_void_p, _dp]
        L.ora_run.restype = C.c_int
        L.ora_run.argtypes = [C.c_void_p, _dp, _dp, C.POINTER(State), C.c_int32, C.c_int32, _dp]
        L.ora_phi.restype = C.c_double
        L.ora_phi.argtypes = [C.c_void_p, C.POINTER(State)]
        L.ora_reached.restype = C.c_int
        L.ora_reached.argtypes = [C.c_void_p, C.POINTER(State), _dp]
        L.ora_rmsd.restype = C.c_double
        L.ora_rmsd.argtypes = [C.c_void_p, _dp]
        L.ora_select.restype = C.c_int
        L.ora_select.argtypes = [C.c_int32, _dp, _u8p, _u8p, _ip, _dp]
        L.ora_forces_dir.restype = C.c_int
        L.ora_forces_dir.argtypes = [C.c_void_p, _dp, _dp, C.c_int32, C.c_double, C.POINTER(State),
                                     C.c_int32, _dp, _dp, _dp, _dp]
        L.ora_init_tangent.restype = C.c_int
        L.ora_init_tangent.argtypes = [C.c_void_p, _dp, C.POINTER(State), _dp]
        L.ora_run_tangent.restype = C.c_int
        L.ora_run_tangent.argtypes = [C.c_void_p, _dp, _dp, C.POINTER(State), _dp, _dp, _dp,
                                      C.c_int32, C.c_int32]
        L.ora_phi_grad.argtypes = [C.c_void_p, C.POINTER(State), _dp, _dp]
        L.ora_toy_potential.restype = C.c_double
        L.ora_toy_potential.argtypes = [C.POINTER(ToyParams), C.c_double, C.c_double, _dp, _dp]
        L.ora_toy_run.argtypes = [C.POINTER(ToyParams), C.c_int32, C.c_double, C.c_uint64, _dp, _dp]
        L.ora_native_contacts.restype = C.c_int64
        L.ora_native_contacts.argtypes = [C.c_void_p, _ip, C.c_int64]
        L.ora_contacts_formed.argtypes = [C.c_void_p, _dp, _ip, C.c_int64, _u8p]
        L.ora_path_similarity.restype = C.c_double
        L.ora_path_similarity.argtypes = [C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


class Oracle:
    """One replica of the FP64 oracle."""

    def __init__(self, desc):
        self.desc = desc
        self.n = int(desc["n_atoms"])
        self.ns = int(desc["n_solute"])
        keep = {}
        for k in ("mass", "gamma", "charge", "sigma", "epsilon", "bond_k", "bond_r0",
                  "angle_k", "angle_theta0"):
            keep[k] = _f64(desc[k])
        for k in ("bonds", "angles", "excl"):
            keep[k] = np.ascontiguousarray(desc[k], dtype=np.int32)
        xf = desc.get("x_final")
        keep["x_final"] = None if xf is None else _f64(xf)
        cf = desc.get("const_force")
        keep["const_force"] = None if cf is None else _f64(cf)
        self._keep = keep
        s = _Sys()
        s.n_atoms, s.n_solute = self.n, self.ns
        for k in ("mass", "gamma", "charge", "sigma", "epsilon", "bond_k", "bond_r0",
                  "angle_k", "angle_theta0"):
            setattr(s, k, _d(keep[k]))
        s.n_bonds = len(keep["bonds"])
        s.bonds = keep["bonds"].ctypes.data_as(_ip)
        s.n_angles = len(keep["angles"])
        s.angles = keep["angles"].ctypes.data_as(_ip)
        s.n_excl = len(keep["excl"])
        s.excl = keep["excl"].ctypes.data_as(_ip)
        for a in range(3):
            s.box[a] = float(desc["box"][a])
        s.r_cut, s.eps_rf, s.kT, s.dt = (float(desc[k]) for k in ("r_cut", "eps_rf", "kT", "dt"))
        s.x_final = _d(keep["x_final"]) if keep["x_final"] is not None else _dp()
        s.bias = int(desc["bias"])
        s.bias_k, s.ramp_rate, s.z_target = (float(desc[k]) for k in ("bias_k", "ramp_rate", "z_target"))
        s.contact_r0, s.contact_rs, s.contact_rc = (float(desc[k]) for k in ("contact_r0", "contact_rs", "contact_rc"))
        s.contact_min_sep = int(desc["contact_min_sep"])
        s.reach_tol = float(desc["reach_tol"])
        s.seed = int(desc["seed"]) & 0xFFFFFFFFFFFFFFFF
        s.const_force = _d(keep["const_force"]) if keep["const_force"] is not None else _dp()
        s.reach_rmsd = float(desc.get("reach_rmsd", float("inf")))
        self._sys = s
        self.ctx = lib().ora_create(C.byref(s))
        if not self.ctx:
            raise MemoryError("ora_create failed")

    def __del__(self):
        if getattr(self, "ctx", None) and _lib is not None:
            _lib.ora_destroy(self.ctx)
            self.ctx = None

    # ---------------------------------------------------------------- pairs
    def pairs(self, x, cells=False):
        x = _f64(x, (self.n, 3))
        cnt = lib().ora_pairs(self.ctx, _d(x), int(cells), None, 0)
        out = np.zeros((max(cnt, 1), 2), np.int32)
        lib().ora_pairs(self.ctx, _d(x), int(cells), out.ctypes.data_as(_ip), cnt)
        return out[:cnt]

    # --------------------------------------------------------------- forces
    def forces(self, x, t=0.0, state=None, cells=True):
        x = _f64(x, (self.n, 3))
        f = np.zeros((self.n, 3))
        fb = np.zeros((self.n, 3))
        terms = np.zeros(len(TERMS))
        st = C.byref(state) if state is not None else None
        bad = lib().ora_forces(self.ctx, _d(x), float(t), st, int(cells), _d(f), _d(fb), _d(terms))
        return f, fb, dict(zip(TERMS, terms.tolist()), unstable=bool(bad))

    def cv(self, x):
        x = _f64(x, (self.n, 3))
        g = np.zeros((max(self.ns, 1), 3))
        z = lib().ora_cv(self.ctx, _d(x), _d(g))
        return z, g[: self.ns]

    # ----------------------------------------------------------- trajectory
    def init(self, x0):
        st = State()
        lib().ora_init(self.ctx, _d(_f64(x0, (self.n, 3))), C.byref(st))
        return st

    def maxwell(self):
        v = np.zeros((self.n, 3))
        lib().ora_maxwell(self.ctx, _d(v))
        return v

    def run(self, x, v, state, nsteps, cells=True, traj=False):
        """Advance (x, v, state) in place by nsteps BAOAB steps."""
        assert x.dtype == np.float64 and x.flags.c_contiguous and x.shape == (self.n, 3)
        assert v.dtype == np.float64 and v.flags.c_contiguous and v.shape == (self.n, 3)
        tr = np.zeros((nsteps, self.n, 3)) if traj else None
        bad = lib().ora_run(self.ctx, _d(x), _d(v), C.byref(state), int(nsteps), int(cells),
                            _d(tr) if traj else None)
        return (bad, tr) if traj else bad

    def phi(self, state):
        return lib().ora_phi(self.ctx, C.byref(state))

    # ------------------------------------------- derivative w.r.t. (k, rho)
    def forces_dir(self, x, dx=None, theta=False, t=0.0, state=None, cells=True):
        """Forces and S with their derivatives along dx ([2][n][3]) and, if
        theta, the bias parameters (direction 0: bias_k, 1: ramp_rate)."""
        x = _f64(x, (self.n, 3))
        dxa = None if dx is None else _f64(dx, (2, self.n, 3))
        f = np.zeros((self.n, 3))
        fdot = np.zeros((2, self.n, 3))
        S = C.c_double()
        Sdot = np.zeros(2)
        st = C.byref(state) if state is not None else None
        bad = lib().ora_forces_dir(self.ctx, _d(x), _d(dxa) if dxa is not None else None, int(theta),
                                   float(t), st, int(cells), _d(f), _d(fdot), C.byref(S), _d(Sdot))
        return f, fdot, S.value, Sdot, bool(bad)

    def init_tangent(self, x0, state):
        """Trapezoid accumulators of dS/dtheta at step 0."""
        pd = np.zeros(4)
        lib().ora_init_tangent(self.ctx, _d(_f64(x0, (self.n, 3))), C.byref(state), _d(pd))
        return pd

    def run_tangent(self, x, v, state, xt, vt, pd, nsteps, cells=True):
        """Advance (x, v, state) and the tangents xt, vt ([2][n][3]) and pd in place."""
        for a, shape in ((x, (self.n, 3)), (v, (self.n, 3)), (xt, (2, self.n, 3)),
                         (vt, (2, self.n, 3)), (pd, (4,))):
            assert a.dtype == np.float64 and a.flags.c_contiguous and a.shape == shape
        return lib().ora_run_tangent(self.ctx, _d(x), _d(v), C.byref(state), _d(xt), _d(vt), _d(pd),
                                     int(nsteps), int(cells))

    def phi_grad(self, state, pd):
        out = np.zeros(2)
        lib().ora_phi_grad(self.ctx, C.byref(state), _d(pd), _d(out))
        return out

    def reached(self, state, x=None):
        xa = None if x is None else _f64(x, (self.n, 3))
        return bool(lib().ora_reached(self.ctx, C.byref(state), _d(xa) if xa is not None else None))

    def native_contacts(self):
        """Native contact pairs [nc, 2] (i < j) of X_f."""
        n = lib().ora_native_contacts(self.ctx, None, 0)
        out = np.zeros((max(n, 1), 2), np.int32)
        lib().ora_native_contacts(self.ctx, out.ctypes.data_as(_ip), n)
        return out[:n]

    def contacts_formed(self, x, pairs):
        pairs = np.ascontiguousarray(pairs, dtype=np.int32)
        out = np.zeros(len(pairs), np.uint8)
        lib().ora_contacts_formed(self.ctx, _d(_f64(x, (self.n, 3))), pairs.ctypes.data_as(_ip),
                                  len(pairs), out.ctypes.data_as(_u8p))
        return out.astype(bool)

    def rmsd(self, x):
        """RMSD of the solute of x ([n][3]) from X_f after optimal superposition."""
        return lib().ora_rmsd(self.ctx, _d(_f64(x, (self.n, 3))))


# ------------------------------------------------------------------ helpers
def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().ora_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def uniforms(seed, atom, step, tag):
    u = (C.c_double * 4)()
    lib().ora_uniforms(seed & 0xFFFFFFFFFFFFFFFF, atom, step, tag, u)
    return np.array(list(u))


def normals(seed, atom, step, tag):
    g = (C.c_double * 3)()
    lib().ora_normals(seed & 0xFFFFFFFFFFFFFFFF, atom, step, tag, g)
    return np.array(list(g))


def contact_value(r, r0=0.75, rs=1.0, rc=1.2):
    d = C.c_double()
    v = lib().ora_contact_value(float(r), float(r0), float(rs), float(rc), C.byref(d))
    return v, d.value


def select(phi, reached=None, eligible=None):
    phi = _f64(phi)
    n = len(phi)
    r = None if reached is None else np.ascontiguousarray(reached, dtype=np.uint8)
    e = None if eligible is None else np.ascontiguousarray(eligible, dtype=np.uint8)
    best = C.c_int32()
    bp = C.c_double()
    rc = lib().ora_select(n, _d(phi), r.ctypes.data_as(_u8p) if r is not None else None,
                          e.ctypes.data_as(_u8p) if e is not None else None, C.byref(best), C.byref(bp))
    return rc, best.value, bp.value


def build_command(out=LIB_PATH):
    """The compiler command that builds liboracle.so (plain C99, FP64, no
    contraction so that the FP32 pair predicate is evaluated as written)."""
    return ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
            os.path.join(_HERE, "oracle.c"), "-o", out, "-lm"]


# ------------------------------------------------------------------ toy model
def toy_params(p):
    """ToyParams from a dict (keys of ToyParams._fields_)."""
    t = ToyParams()
    for k, _ in ToyParams._fields_:
        if k in p:
            setattr(t, k, p[k])
    return t


def toy_potential(p, x, y):
    gx, gy = C.c_double(), C.c_double()
    u = lib().ora_toy_potential(C.byref(toy_params(p)), float(x), float(y), C.byref(gx), C.byref(gy))
    return u, gx.value, gy.value


def toy_run(p, kind, k_bias, seed, path=False):
    """One toy trial: dict of TOY_COLUMNS (and the path [n_steps + 1, 2])."""
    t = toy_params(p)
    out = np.zeros(len(TOY_COLUMNS))
    pa = np.zeros((t.n_steps + 1, 2)) if path else None
    lib().ora_toy_run(C.byref(t), int(kind), float(k_bias), int(seed) & 0xFFFFFFFFFFFFFFFF, _d(out),
                      _d(pa) if path else None)
    res = dict(zip(TOY_COLUMNS, out.tolist()))
    return (res, pa) if path else res


def path_similarity(ta, tb):
    a = np.ascontiguousarray(ta, dtype=np.int64)
    b = np.ascontiguousarray(tb, dtype=np.int64)
    assert a.shape == b.shape
    p64 = C.POINTER(C.c_int64)
    return lib().ora_path_similarity(len(a), a.ctypes.data_as(p64), b.ctypes.data_as(p64))
