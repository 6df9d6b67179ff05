"""ctypes binding of the surrogate ensemble (argument marshalling only; the
training and inference run in the HIP kernels of liblbm.so)."""
from __future__ import annotations

import ctypes as C

import numpy as np

from .lbm import LBM_OK, LBMError, lib


def _setup(L):
    if getattr(L, "_surr_ready", False):
        return L
    vp = C.c_void_p
    L.surr_workspace_bytes.argtypes = [C.c_int, C.c_int, C.c_int]
    L.surr_workspace_bytes.restype = C.c_size_t
    L.surr_param_count.argtypes = [C.c_int]
    L.surr_param_count.restype = C.c_int
    L.surr_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_uint64, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.surr_train.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_float, vp]
    L.surr_forward_backward.argtypes = [vp, vp, vp, C.c_int, vp, vp]
    L.surr_predict.argtypes = [vp, vp, C.c_int, vp, vp, vp, C.c_float, C.POINTER(C.c_float), C.POINTER(C.c_float)]
    L.surr_get_params.argtypes = [vp, vp, C.c_size_t]
    L.surr_set_params.argtypes = [vp, vp, C.c_size_t]
    L.surr_destroy.argtypes = [vp]
    L.surr_destroy.restype = None
    L.surr_last_error.argtypes = [vp]
    L.surr_last_error.restype = C.c_char_p
    for name in ("surr_create", "surr_train", "surr_forward_backward", "surr_predict", "surr_get_params",
                 "surr_set_params"):
        getattr(L, name).restype = C.c_int
    L._surr_ready = True
    return L


def param_count(hidden=128):
    return int(_setup(lib()).surr_param_count(hidden))


class Surrogate:
    """Ensemble of ``members`` MLPs 4 -> hidden -> hidden -> 2 on one GPU."""

    def __init__(self, members=5, hidden=128, max_n=4096, seed=0, device="cuda:0", stream=None):
        import torch
        L = _setup(lib())
        self.members, self.hidden, self.max_n = members, hidden, max_n
        self.P = int(L.surr_param_count(hidden))
        self.device = torch.device(device)
        nbytes = int(L.surr_workspace_bytes(members, hidden, max_n))
        if nbytes == 0:
            raise LBMError(1, "invalid surrogate size")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        st = L.surr_create(members, hidden, max_n, seed, C.c_void_p(self.ws.data_ptr()), nbytes,
                           C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != LBM_OK:
            raise LBMError(st, L.surr_last_error(None).decode())
        self._h = h

    def _check(self, st):
        if st != LBM_OK:
            raise LBMError(st, lib().surr_last_error(self._h).decode())

    @staticmethod
    def _dev(a, torch, device, cols):
        t = torch.as_tensor(np.asarray(a, np.float32) if not torch.is_tensor(a) else a, device=device)
        t = t.to(torch.float32).contiguous()
        assert t.dim() == 2 and t.shape[1] == cols
        return t

    def train(self, X, Y, epochs, lr=1e-3):
        import torch
        Xd, Yd = self._dev(X, torch, self.device, 4), self._dev(Y, torch, self.device, 2)
        loss = np.zeros(self.members, np.float32)
        self._check(lib().surr_train(self._h, C.c_void_p(Xd.data_ptr()), C.c_void_p(Yd.data_ptr()), len(Xd),
                                     int(epochs), float(lr), C.c_void_p(loss.ctypes.data)))
        return loss

    def forward_backward(self, X, Y):
        """(grads [members][P], loss [members]) without an update."""
        import torch
        Xd, Yd = self._dev(X, torch, self.device, 4), self._dev(Y, torch, self.device, 2)
        g = torch.empty((self.members, self.P), dtype=torch.float32, device=self.device)
        l = torch.empty(self.members, dtype=torch.float32, device=self.device)
        self._check(lib().surr_forward_backward(self._h, C.c_void_p(Xd.data_ptr()), C.c_void_p(Yd.data_ptr()),
                                                len(Xd), C.c_void_p(g.data_ptr()), C.c_void_p(l.data_ptr())))
        return g.cpu().numpy(), l.cpu().numpy()

    def predict(self, X, threshold=0.05, out_scale=None, out_shift=None):
        """(mean [n][2], std [n][2], fallback [n]) as device tensors, in the
        units y * out_scale + out_shift of each output (identity by default);
        the fallback test std > threshold * |mean| is taken in those units."""
        import torch
        Xd = self._dev(X, torch, self.device, 4)
        n = len(Xd)
        mean = torch.empty((n, 2), dtype=torch.float32, device=self.device)
        sd = torch.empty((n, 2), dtype=torch.float32, device=self.device)
        fb = torch.empty(n, dtype=torch.uint8, device=self.device)
        sc = None if out_scale is None else (C.c_float * 2)(*[float(v) for v in out_scale])
        sh = None if out_shift is None else (C.c_float * 2)(*[float(v) for v in out_shift])
        self._check(lib().surr_predict(self._h, C.c_void_p(Xd.data_ptr()), n, C.c_void_p(mean.data_ptr()),
                                       C.c_void_p(sd.data_ptr()), C.c_void_p(fb.data_ptr()), float(threshold),
                                       sc, sh))
        return mean, sd, fb

    def get_params(self):
        p = np.zeros((self.members, self.P), np.float32)
        self._check(lib().surr_get_params(self._h, C.c_void_p(p.ctypes.data), p.nbytes))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.shape == (self.members, self.P)
        self._check(lib().surr_set_params(self._h, C.c_void_p(p.ctypes.data), p.nbytes))

    def close(self):
        if getattr(self, "_h", None):
            lib().surr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
