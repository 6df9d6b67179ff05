"""Thin ctypes binding of the C ABI in ``include/lbm.h``.

Argument marshalling only: every step of the method runs in the HIP kernels
of ``liblbm.so``.  PyTorch provides the device workspace and the stream.  If
the library is missing the constructor raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE = range(6)
STATUS = {0: "LBM_OK", 1: "LBM_EINVAL", 2: "LBM_ENOMEM", 3: "LBM_EDEVICE", 4: "LBM_EUNSTABLE", 5: "LBM_ESTATE"}
STORE = {"f32": 0, "f16": 1, "f16fixed": 2}
MAX_INLETS = 8


class LBMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Inlet(C.Structure):
    _fields_ = [("axis", C.c_int), ("side", C.c_int), ("lo", C.c_int * 3), ("hi", C.c_int * 3),
                ("rho", C.c_double * 2), ("u_n", C.c_double), ("alpha_on", C.c_int)]


class Outlet(C.Structure):
    _fields_ = [("axis", C.c_int), ("side", C.c_int), ("lo", C.c_int * 3), ("hi", C.c_int * 3),
                ("chi_on", C.c_int)]


class Config(C.Structure):
    _fields_ = [("dim", C.c_int), ("storage", C.c_int), ("n", C.c_int * 3), ("periodic", C.c_int * 3),
                ("nu", C.c_double * 2), ("s_q", C.c_double), ("s_eps_policy", C.c_int),
                ("G12", C.c_double), ("Gw", C.c_double * 2), ("Fb", C.c_double * 3),
                ("n_inlets", C.c_int), ("inlets", Inlet * MAX_INLETS), ("has_outlet", C.c_int),
                ("outlet", Outlet), ("tile_config", C.c_int), ("layout", C.c_int),
                ("solid", C.c_void_p), ("rho0", C.c_void_p), ("u0", C.c_void_p),
                ("wall_u", C.c_void_p)]


class Box(C.Structure):
    _fields_ = [("lo", C.c_int * 3), ("hi", C.c_int * 3)]


class Component(C.Structure):
    _fields_ = [("first", C.c_int64), ("size", C.c_int64), ("lo", C.c_int * 3), ("hi", C.c_int * 3)]


def make_box(lo, hi):
    b = Box()
    for a in range(3):
        b.lo[a] = int(lo[a]) if a < len(lo) else 0
        b.hi[a] = int(hi[a]) if a < len(hi) else 1
    return b


class Flux(C.Structure):
    _fields_ = [("step", C.c_int64), ("q_in", C.c_double), ("q_out", C.c_double), ("chi", C.c_double),
                ("u_conv", C.c_double), ("mass", C.c_double * 2), ("mass0", C.c_double * 2),
                ("uc_clamps", C.c_int64)]

    def as_dict(self):
        return {"step": self.step, "q_in": self.q_in, "q_out": self.q_out, "chi": self.chi,
                "u_conv": self.u_conv, "mass": [self.mass[0], self.mass[1]],
                "mass0": [self.mass0[0], self.mass0[1]], "uc_clamps": self.uc_clamps}


_lib = None


def lib():
    """Load liblbm.so (torch is imported first so that both share one HIP runtime)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads the HIP runtime the workspace comes from)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        cp, vp, dp = C.POINTER(Config), C.c_void_p, C.POINTER(C.c_double)
        L.lbm_workspace_bytes.argtypes = [cp]
        L.lbm_workspace_bytes.restype = C.c_size_t
        L.lbm_create.argtypes = [cp, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.lbm_step.argtypes = [vp, C.c_int64]
        L.lbm_moments.argtypes = [vp, vp, vp, C.c_int]
        L.lbm_mass_flux.argtypes = [vp, C.POINTER(Flux)]
        L.lbm_get_state.argtypes = [vp, vp, C.c_size_t]
        L.lbm_set_state.argtypes = [vp, vp, C.c_size_t]
        L.lbm_time_kernels.argtypes = [vp, C.c_int64, C.POINTER(C.c_double)]
        L.lbm_time_kernels.restype = C.c_int
        L.lbm_tile_configs.argtypes = [C.c_int]
        L.lbm_tile_configs.restype = C.c_int
        L.lbm_tile_config_desc.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int)]
        L.lbm_tile_config_desc.restype = C.c_int
        L.lbm_set_graph_steps.argtypes = [vp, C.c_int]
        L.lbm_steps_done.argtypes = [vp]
        L.lbm_steps_done.restype = C.c_int64
        L.lbm_destroy.argtypes = [vp]
        L.lbm_destroy.restype = None
        L.lbm_last_error.argtypes = [vp]
        L.lbm_last_error.restype = C.c_char_p
        L.lbm_probe.argtypes = [vp, C.c_int, C.POINTER(Box), C.c_double, vp]
        L.lbm_probe.restype = C.c_int
        L.lbm_components.argtypes = [vp, C.c_int, C.POINTER(Box), C.c_double, C.POINTER(Component), C.c_int,
                                     C.POINTER(C.c_int)]
        L.lbm_components.restype = C.c_int
        L.lbm_components_static.argtypes = L.lbm_components.argtypes
        L.lbm_components_static.restype = C.c_int
        L.lbm_batch_workspace_bytes.argtypes = [cp, C.c_int]
        L.lbm_batch_workspace_bytes.restype = C.c_size_t
        L.lbm_batch_create.argtypes = [cp, C.c_int, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.lbm_batch_step.argtypes = [vp, C.c_int64]
        L.lbm_batch_set_graph_steps.argtypes = [vp, C.c_int]
        L.lbm_batch_size.argtypes = [vp]
        L.lbm_batch_size.restype = C.c_int
        L.lbm_batch_member.argtypes = [vp, C.c_int]
        L.lbm_batch_member.restype = vp
        L.lbm_batch_destroy.argtypes = [vp]
        L.lbm_batch_destroy.restype = None
        L.lbm_batch_last_error.argtypes = [vp]
        L.lbm_batch_last_error.restype = C.c_char_p
        for name in ("lbm_create", "lbm_step", "lbm_moments", "lbm_mass_flux", "lbm_get_state", "lbm_set_state",
                     "lbm_batch_create", "lbm_batch_step", "lbm_batch_set_graph_steps", "lbm_set_graph_steps"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


_probe_lib = None
PROBE_LIB_PATH = os.path.join(HERE, "libprobe.so")


def probe_lib():
    """The measurement library (streaming probes), separate from the solver."""
    global _probe_lib
    if _probe_lib is None:
        import torch  # noqa: F401
        if not os.path.exists(PROBE_LIB_PATH):
            raise RuntimeError(f"{PROBE_LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(PROBE_LIB_PATH)
        vp = C.c_void_p
        L.lbm_stream_probe.argtypes = [vp, vp, C.c_size_t, C.c_int, C.c_int, vp, C.POINTER(C.c_double)]
        L.lbm_stream_probe.restype = C.c_int
        _probe_lib = L
    return _probe_lib


LAYOUT = {"caller": 0, "face_last": 1}


def make_config(case, storage="f32", tile_config=-1, layout="caller"):
    """Fill an ``lbm_config`` from a case; returns (config, arrays kept alive)."""
    cfg = Config()
    cfg.tile_config = int(tile_config)
    cfg.layout = LAYOUT[layout]
    cfg.dim = case.dim
    cfg.storage = STORE[storage]
    for a in range(3):
        cfg.n[a] = int(case.n[a])
        cfg.periodic[a] = int(bool(case.periodic[a]))
    cfg.nu[0], cfg.nu[1] = case.nu
    cfg.s_q = case.s_q
    cfg.s_eps_policy = int(case.s_eps_policy)
    cfg.G12 = case.G12
    cfg.Gw[0], cfg.Gw[1] = case.Gw
    for a in range(3):
        cfg.Fb[a] = case.Fb[a]
    if len(case.inlets) > MAX_INLETS:
        raise ValueError("too many inlet patches")
    cfg.n_inlets = len(case.inlets)
    for j, inl in enumerate(case.inlets):
        q = cfg.inlets[j]
        q.axis, q.side = inl["axis"], inl["side"]
        for a in range(3):
            q.lo[a], q.hi[a] = inl["lo"][a], inl["hi"][a]
        q.rho[0], q.rho[1] = inl["rho"]
        q.u_n = inl["u_n"]
        q.alpha_on = int(inl.get("alpha_on", 1))
    if case.outlet is not None:
        o = case.outlet
        cfg.has_outlet = 1
        cfg.outlet.axis, cfg.outlet.side = o["axis"], o["side"]
        for a in range(3):
            cfg.outlet.lo[a], cfg.outlet.hi[a] = o["lo"][a], o["hi"][a]
        cfg.outlet.chi_on = int(o.get("chi_on", 1))
    solid = np.ascontiguousarray(case.solid, dtype=np.uint8).reshape(-1)
    rho0 = np.ascontiguousarray(case.rho0, dtype=np.float64).reshape(-1)
    u0 = None if case.u0 is None else np.ascontiguousarray(case.u0, dtype=np.float64).reshape(-1)
    uw = getattr(case, "wall_u", None)
    uw = None if uw is None else np.ascontiguousarray(uw, dtype=np.float64).reshape(-1)
    cfg.solid = solid.ctypes.data
    cfg.rho0 = rho0.ctypes.data
    cfg.u0 = None if u0 is None else u0.ctypes.data
    cfg.wall_u = None if uw is None else uw.ctypes.data
    return cfg, (solid, rho0, u0, uw)


def tile_configs(dim):
    """Number of node-update configurations of the tuning space."""
    return int(lib().lbm_tile_configs(int(dim)))


def stream_probe(nbytes=1 << 30, reps=20, device="cuda:0"):
    """Rates (GB/s) of plain streaming kernels on this device: copy at 4 and
    16 bytes per thread, read at 16 bytes per thread, copy of eight 4-byte
    elements per thread, and the D3Q19 pull pattern of the node update (38
    shifted loads and 38 stores per node, no arithmetic) with each node's
    loads after / before the previous node's stores, and the same bytes with
    both components of a population in one 8-byte slot."""
    import torch
    a = torch.zeros(nbytes, dtype=torch.uint8, device=device)
    b = torch.zeros(nbytes, dtype=torch.uint8, device=device)
    s = torch.cuda.current_stream(device)
    out = {}
    for kind, name in enumerate(("copy_b32", "copy_b128", "read_b128", "copy_b32x8", "pull_d3q19",
                                 "pull_d3q19_ahead", "pull_d3q19_pairs")):
        r = C.c_double(0.0)
        st = probe_lib().lbm_stream_probe(a.data_ptr(), b.data_ptr(), nbytes, kind, reps, s.cuda_stream, C.byref(r))
        if st != LBM_OK:
            raise LBMError(st, "stream probe failed")
        out[name] = round(r.value, 1)
    del a, b
    return out


def tile_config_desc(dim, i):
    """Configuration i as a dict: psi source, lateral tile, sweep planes per
    iteration and per work item, register policy."""
    out = (C.c_int * 6)()
    st = lib().lbm_tile_config_desc(int(dim), int(i), out)
    if st != LBM_OK:
        raise LBMError(st, f"no tile configuration {i} for dim {dim}")
    return dict(zip(("psrc", "tx", "ty", "w", "zc", "keepb"), list(out)))


def resolve_tile_config(case, storage, tile_config):
    """'auto' looks the lattice / storage / size class up in the autotuner table."""
    if tile_config == "auto":
        from .autotune import lookup
        return lookup(case.dim, storage, case.N)
    return int(tile_config)


def workspace_bytes(case, storage="f32", tile_config=-1, layout="caller"):
    cfg, keep = make_config(case, storage, tile_config, layout)
    return int(lib().lbm_workspace_bytes(C.byref(cfg)))


class LBM:
    """One simulation context on a GPU (device memory from torch)."""

    def __init__(self, case, storage="f32", device="cuda:0", stream=None, tile_config=-1, layout="caller"):
        import torch
        L = lib()
        self.case = case
        self.dim = case.dim
        self.Q = 9 if case.dim == 2 else 19
        self.N = int(np.prod(case.n))
        self.device = torch.device(device)
        self.tile_config = resolve_tile_config(case, storage, tile_config)
        cfg, keep = make_config(case, storage, self.tile_config, layout)
        nbytes = int(L.lbm_workspace_bytes(C.byref(cfg)))
        if nbytes == 0:
            h = C.c_void_p()
            st = L.lbm_create(C.byref(cfg), None, 0, None, C.byref(h))
            raise LBMError(st, L.lbm_last_error(None).decode())
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        st = L.lbm_create(C.byref(cfg), C.c_void_p(self.ws.data_ptr()), nbytes,
                          C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != LBM_OK:
            raise LBMError(st, L.lbm_last_error(None).decode())
        self._h = h
        self.workspace_bytes = nbytes

    def _check(self, st):
        if st != LBM_OK:
            raise LBMError(st, lib().lbm_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        self._check(lib().lbm_step(self._h, int(n)))

    def set_graph_steps(self, k):
        """Steps per replayed HIP graph in step() (0: plain launches)."""
        self._check(lib().lbm_set_graph_steps(self._h, int(k)))

    def moments(self, check=True):
        """Return (rho [2,N], u [3,N]) as float64 numpy arrays."""
        rho = np.zeros((2, self.N))
        u = np.zeros((3, self.N))
        st = lib().lbm_moments(self._h, rho.ctypes.data, u.ctypes.data, 0)
        if check:
            self._check(st)
        return rho, u

    def moments_device(self, rho, u):
        """Write moments into caller-owned float64 CUDA tensors [2,N] and [3,N]."""
        return lib().lbm_moments(self._h, rho.data_ptr(), u.data_ptr(), 1)

    def mass_flux(self, check=True):
        out = Flux()
        st = lib().lbm_mass_flux(self._h, C.byref(out))
        if check:
            self._check(st)
        return out.as_dict()

    def get_state(self):
        f = np.zeros((2, self.Q, self.N))
        self._check(lib().lbm_get_state(self._h, f.ctypes.data, f.nbytes))
        return f

    def set_state(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (2, self.Q, self.N)
        self._check(lib().lbm_set_state(self._h, f.ctypes.data, f.nbytes))

    def time_kernels(self, n):
        """Run n steps with HIP events around every launch; mean ms of
        (node update, outlet collision, inlet reconstruction, outlet fill,
        density pass)."""
        ms = (C.c_double * 5)()
        self._check(lib().lbm_time_kernels(self._h, int(n), ms))
        return list(ms)

    @property
    def steps(self):
        return int(lib().lbm_steps_done(self._h))

    def probe(self, k, lo, hi, threshold, out):
        """Enqueue the count of component-k nodes above threshold in the box
        [lo, hi) into ``out`` (an int64 CUDA tensor element, e.g. series[i:i+1])."""
        box = make_box(lo, hi)
        self._check(lib().lbm_probe(self._h, int(k), C.byref(box), float(threshold), C.c_void_p(out.data_ptr())))

    def components(self, k, lo, hi, threshold, max_out=4096, static=False):
        """Face-connected components of {rho_k > threshold} in the box:
        list of dicts (first node, size, bbox lo/hi), by first node.
        ``static`` calls the allocation-free entry point."""
        box = make_box(lo, hi)
        out = (Component * max_out)()
        n = C.c_int(0)
        fn = lib().lbm_components_static if static else lib().lbm_components
        self._check(fn(self._h, int(k), C.byref(box), float(threshold), out, int(max_out), C.byref(n)))
        return [{"first": out[i].first, "size": out[i].size, "lo": tuple(out[i].lo), "hi": tuple(out[i].hi)}
                for i in range(min(n.value, max_out))], n.value


class _Member(LBM):
    """A batch member seen as a context (owned by its batch)."""

    def __init__(self, batch, i, case):
        self.case = case
        self.dim = case.dim
        self.Q = 9 if case.dim == 2 else 19
        self.N = int(np.prod(case.n))
        self.device = batch.device
        self.stream = batch.stream
        self.tile_config = batch.tile_config
        self._batch = batch              # keeps the workspace alive
        self._h = C.c_void_p(lib().lbm_batch_member(batch._h, int(i)))

    def close(self):
        self._h = None                   # the batch owns the member


class Batch:
    """Many contexts stepped together (one launch per stage for all members)."""

    def __init__(self, case_list, storage="f32", device="cuda:0", stream=None, tile_config="auto"):
        import torch
        L = lib()
        self.cases = list(case_list)
        n = len(self.cases)
        self.device = torch.device(device)
        if tile_config == "auto" and n:
            # the tuned configuration of the lattice and storage for the
            # batch's total size
            from .autotune import lookup
            self.tile_config = lookup(self.cases[0].dim, storage, sum(c.N for c in self.cases))
        else:
            self.tile_config = resolve_tile_config(self.cases[0], storage, tile_config) if n else -1
        cfgs = (Config * n)()
        self._keep = []
        for i, c in enumerate(self.cases):
            cfg, keep = make_config(c, storage, self.tile_config)
            cfgs[i] = cfg
            self._keep.append(keep)
        nbytes = int(L.lbm_batch_workspace_bytes(cfgs, n))
        if nbytes == 0:
            h = C.c_void_p()
            st = L.lbm_batch_create(cfgs, n, None, 0, None, C.byref(h))
            raise LBMError(st, L.lbm_batch_last_error(None).decode())
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        st = L.lbm_batch_create(cfgs, n, C.c_void_p(self.ws.data_ptr()), nbytes,
                                C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != LBM_OK:
            raise LBMError(st, L.lbm_batch_last_error(None).decode())
        self._h = h
        self.workspace_bytes = nbytes
        self.members = [_Member(self, i, c) for i, c in enumerate(self.cases)]

    def _check(self, st):
        if st != LBM_OK:
            raise LBMError(st, lib().lbm_batch_last_error(self._h).decode())

    def step(self, n=1):
        self._check(lib().lbm_batch_step(self._h, int(n)))

    def set_graph_steps(self, k):
        self._check(lib().lbm_batch_set_graph_steps(self._h, int(k)))

    def __len__(self):
        return len(self.members)

    def __getitem__(self, i):
        return self.members[i]

    def close(self):
        if getattr(self, "_h", None):
            for m in self.members:
                m._h = None
            lib().lbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
