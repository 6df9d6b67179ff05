"""FP64 CPU oracle of the two-component pseudopotential MRT LBM step with the
corrected open boundaries (arXiv:2512.12934).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports,
links or runs anything from here, and this package imports nothing from the
product package: a case is any object with the attributes listed in
``_params`` below (the seeded case generators provide them).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None

MAX_INLETS = 8


class _Inlet(C.Structure):
    _fields_ = [("axis", C.c_int), ("side", C.c_int),
                ("lo", C.c_int * 3), ("hi", C.c_int * 3),
                ("rho", C.c_double * 2), ("u_n", C.c_double),
                ("alpha_on", C.c_int)]


class _Outlet(C.Structure):
    _fields_ = [("axis", C.c_int), ("side", C.c_int),
                ("lo", C.c_int * 3), ("hi", C.c_int * 3),
                ("chi_on", C.c_int)]


class _Params(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("periodic", C.c_int * 3),
                ("nu", C.c_double * 2), ("s_q", C.c_double),
                ("s_eps_policy", C.c_int), ("G12", C.c_double),
                ("Gw", C.c_double * 2), ("Fb", C.c_double * 3),
                ("n_inlets", C.c_int), ("inlets", _Inlet * MAX_INLETS),
                ("has_outlet", C.c_int), ("outlet", _Outlet)]


class Diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("q_in", C.c_double), ("q_out", C.c_double),
                ("chi", C.c_double), ("u_conv", C.c_double),
                ("mass", C.c_double * 2), ("mass0", C.c_double * 2),
                ("uc_clamps", C.c_int64)]

    def as_dict(self):
        return {"step": self.step, "q_in": self.q_in, "q_out": self.q_out,
                "chi": self.chi, "u_conv": self.u_conv,
                "mass": [self.mass[0], self.mass[1]],
                "mass0": [self.mass0[0], self.mass0[1]],
                "uc_clamps": self.uc_clamps}


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def lib():
    global _LIB
    if _LIB is None:
        path = _build.ensure_built()
        L = C.CDLL(path)
        L.orc_Q.argtypes = [C.c_int]
        L.orc_Q.restype = C.c_int
        L.orc_tables.argtypes = [C.c_int, _ip, _dp, _dp, _dp]
        L.orc_relaxation.argtypes = [C.POINTER(_Params), C.c_int, _dp]
        L.orc_feq.argtypes = [C.c_int, C.c_double, _dp, _dp]
        L.orc_forcing.argtypes = [C.c_int, _dp, _dp, _dp]
        L.orc_collide_node.argtypes = [C.c_int, _dp, _dp, C.c_double, _dp, _dp, _dp]
        L.orc_stencil.argtypes = [C.c_int, _ip, _dp]
        L.orc_stencil.restype = C.c_int
        L.orc_create.argtypes = [C.POINTER(_Params), C.c_void_p, _dp, _dp]
        L.orc_create.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_get_f.argtypes = [C.c_void_p, _dp]
        L.orc_set_f.argtypes = [C.c_void_p, _dp]
        L.orc_moments.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_diagnostics.argtypes = [C.c_void_p, C.POINTER(Diag)]
        L.orc_nodes.argtypes = [C.c_void_p]
        L.orc_nodes.restype = C.c_int64
        L.orc_set_wall_velocity.argtypes = [C.c_void_p, _dp]
        L.orc_set_next.argtypes = [C.c_void_p, _dp]
        L.orc_get_next.argtypes = [C.c_void_p, _dp]
        L.orc_set_force.argtypes = [C.c_void_p, _dp]
        L.orc_stage.argtypes = [C.c_void_p, C.c_int]
        L.orc_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        _LIB = L
    return _LIB


def threads():
    """OpenMP threads the oracle's node loops run on."""
    return int(lib().orc_threads())


def set_threads(n):
    lib().orc_set_threads(int(n))


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# Building blocks (used by the pins)
# ---------------------------------------------------------------------------

def Q(dim):
    return lib().orc_Q(dim)


def tables(dim):
    """Return (e [Q,3] int, w [Q], T [Q,Q], Tinv [Q,Q])."""
    q = Q(dim)
    e = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q)
    T = np.zeros((q, q))
    Ti = np.zeros((q, q))
    lib().orc_tables(dim, e.ctypes.data_as(_ip), _ptr(w), _ptr(T), _ptr(Ti))
    return e.astype(np.int64), w, T, Ti


def relaxation(case, k):
    p = _params(case)
    s = np.zeros(Q(case.dim))
    lib().orc_relaxation(C.byref(p), k, _ptr(s))
    return s


def feq(dim, rho, u):
    out = np.zeros(Q(dim))
    lib().orc_feq(dim, float(rho), _ptr(_f64(u)), _ptr(out))
    return out


def forcing(dim, u, F):
    out = np.zeros(Q(dim))
    lib().orc_forcing(dim, _ptr(_f64(u)), _ptr(_f64(F)), _ptr(out))
    return out


def collide_node(dim, s, f, rho, u, F):
    out = np.zeros(Q(dim))
    lib().orc_collide_node(dim, _ptr(_f64(s)), _ptr(_f64(f)), float(rho),
                           _ptr(_f64(u)), _ptr(_f64(F)), _ptr(out))
    return out


def stencil(dim):
    """Return (offsets [K,3] int, weights [K])."""
    off = np.zeros((128, 3), dtype=np.int32)
    w = np.zeros(128)
    K = lib().orc_stencil(dim, off.ctypes.data_as(_ip), _ptr(w))
    return off[:K].astype(np.int64), w[:K].copy()


# ---------------------------------------------------------------------------
# Whole-domain simulation
# ---------------------------------------------------------------------------

def _params(case):
    p = _Params()
    p.dim = case.dim
    n = list(case.n) + [1] * (3 - len(case.n))
    for a in range(3):
        p.n[a] = int(n[a])
        p.periodic[a] = int(bool(case.periodic[a]))
    p.nu[0], p.nu[1] = case.nu
    p.s_q = case.s_q
    p.s_eps_policy = int(case.s_eps_policy)
    p.G12 = case.G12
    p.Gw[0], p.Gw[1] = case.Gw
    for a in range(3):
        p.Fb[a] = case.Fb[a]
    if len(case.inlets) > MAX_INLETS:
        raise ValueError("too many inlet patches")
    p.n_inlets = len(case.inlets)
    for j, inl in enumerate(case.inlets):
        q = p.inlets[j]
        q.axis, q.side = inl["axis"], inl["side"]
        for a in range(3):
            q.lo[a], q.hi[a] = inl["lo"][a], inl["hi"][a]
        q.rho[0], q.rho[1] = inl["rho"]
        q.u_n = inl["u_n"]
        q.alpha_on = int(inl.get("alpha_on", 1))
    if case.outlet is not None:
        o = case.outlet
        p.has_outlet = 1
        p.outlet.axis, p.outlet.side = o["axis"], o["side"]
        for a in range(3):
            p.outlet.lo[a], p.outlet.hi[a] = o["lo"][a], o["hi"][a]
        p.outlet.chi_on = int(o.get("chi_on", 1))
    return p


class Sim:
    """FP64 oracle run of one case."""

    def __init__(self, case):
        self.case = case
        self.dim = case.dim
        self.q = Q(case.dim)
        self._p = _params(case)
        self.N = int(np.prod(case.n))
        solid = np.ascontiguousarray(case.solid, dtype=np.uint8).reshape(-1)
        rho0 = _f64(case.rho0).reshape(-1)
        u0 = None if case.u0 is None else _f64(case.u0).reshape(-1)
        assert solid.size == self.N and rho0.size == 2 * self.N
        self._keep = (solid, rho0, u0)
        self._h = lib().orc_create(C.byref(self._p), solid.ctypes.data_as(C.c_void_p),
                                   _ptr(rho0), None if u0 is None else _ptr(u0))
        uw = getattr(case, "wall_u", None)
        if uw is not None:
            uw = _f64(uw).reshape(-1)
            assert uw.size == 3 * self.N
            lib().orc_set_wall_velocity(self._h, _ptr(uw))

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        lib().orc_step(self._h, int(n))

    def get_f(self):
        f = np.zeros((2, self.q, self.N))
        lib().orc_get_f(self._h, _ptr(f))
        return f

    def set_f(self, f):
        lib().orc_set_f(self._h, _ptr(_f64(f)))

    def moments(self):
        """Return (rho [2,N], u [3,N], F [2,3,N])."""
        rho = np.zeros((2, self.N))
        u = np.zeros((3, self.N))
        F = np.zeros((2, 3, self.N))
        lib().orc_moments(self._h, _ptr(rho), _ptr(u), _ptr(F))
        return rho, u, F

    def diag(self):
        d = Diag()
        lib().orc_diagnostics(self._h, C.byref(d))
        return d.as_dict()

    # -- test hooks: single stages on a planted state (see lbm_oracle.h) --
    def set_next(self, fn):
        lib().orc_set_next(self._h, _ptr(_f64(fn)))

    def get_next(self):
        fn = np.zeros((2, self.q, self.N))
        lib().orc_get_next(self._h, _ptr(fn))
        return fn

    def set_force(self, F):
        lib().orc_set_force(self._h, _ptr(_f64(F)))

    def stage(self, k):
        lib().orc_stage(self._h, int(k))
