"""ctypes binding of the surrogate part of libbbfd (include/bbsur.h).

Argument marshalling only: forward, backward, Adam training steps and input
featurisation all run in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from .bbfd import _check, _stream, lib

_SIG_DONE = False


class Config(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("n", "cin", "width", "layers", "mx", "my", "mz")] + [
        ("loss_focus", C.c_float)]


def _sigs():
    global _SIG_DONE
    if _SIG_DONE:
        return lib()
    L = lib()
    vp = C.c_void_p
    L.bbsur_create.argtypes = [C.POINTER(Config), C.POINTER(vp)]
    L.bbsur_destroy.argtypes = [vp]
    L.bbsur_destroy.restype = None
    L.bbsur_sizes.argtypes = [vp, C.c_int32, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
    L.bbsur_init_params.argtypes = [vp, vp, C.c_uint64, vp]
    L.bbsur_forward.argtypes = [vp, vp, vp, vp, C.c_int32, vp, C.c_uint64, vp]
    L.bbsur_backward.argtypes = [vp, vp, vp, vp, vp, C.c_int32, vp, C.c_uint64, vp]
    L.bbsur_train_step.argtypes = [vp, vp, vp, vp, vp, C.c_int32, C.c_float, vp, vp, C.c_int32,
                                   vp, vp, C.c_uint64, vp]
    L.bbsur_features.argtypes = [vp, vp, C.c_int32, vp, vp, C.c_int64, vp]
    L.bbsur_gemm.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_int32,
                             C.c_int32, C.c_float, C.c_float, vp]
    _SIG_DONE = True
    return L


def _p(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def gemm(A, a_strides, B, b_strides, Cm, c_strides, M, N, K, batch, alpha=1.0, beta=0.0,
         bias=None, stream=None):
    """C = alpha A B + beta C (+ bias[m]) on the BF16 matrix cores (strided)."""
    L = _sigs()
    arr = lambda s: (C.c_int64 * 3)(*[int(v) for v in s])
    _check(L.bbsur_gemm(_p(A), arr(a_strides), _p(B), arr(b_strides), _p(Cm), arr(c_strides),
                        _p(bias), M, N, K, batch, alpha, beta, C.c_void_p(_stream(stream))))


def features(mat, table, field, x, stream=None):
    """x [4][cells] from a uint8 map, a float2 table and a complex64 field."""
    L = _sigs()
    _check(L.bbsur_features(_p(mat), _p(table), table.numel() // 2, _p(field), _p(x),
                            mat.numel(), C.c_void_p(_stream(stream))))


class TrainState:
    def __init__(self, params, grad, m, v):
        self.params, self.grad, self.m, self.v = params, grad, m, v
        self.step = 0


class Surrogate:
    """3D Fourier neural operator (see include/bbsur.h)."""

    def __init__(self, n=64, cin=4, width=32, layers=4, mx=8, my=8, mz=8, loss_focus=0.0):
        L = _sigs()
        self.cfg = Config(n, cin, width, layers, mx, my, mz, loss_focus)
        self.h = C.c_void_p()
        _check(L.bbsur_create(C.byref(self.cfg), C.byref(self.h)))
        np_ = C.c_uint64(0)
        _check(L.bbsur_sizes(self.h, 1, C.byref(np_), None))
        self.n_params = int(np_.value)
        self.n = n
        self._ws = {}

    def close(self):
        if self.h:
            lib().bbsur_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, batch, device="cuda"):
        import torch
        if batch not in self._ws:
            b = C.c_uint64(0)
            _check(lib().bbsur_sizes(self.h, batch, None, C.byref(b)))
            self._ws = {batch: torch.empty(int(b.value), dtype=torch.uint8, device=device)}
        return self._ws[batch]

    def init_params(self, seed=0, device="cuda"):
        import torch
        p = torch.empty(self.n_params, dtype=torch.float32, device=device)
        _check(lib().bbsur_init_params(self.h, _p(p), seed, C.c_void_p(_stream(None))))
        return p

    def forward(self, params, x, y=None):
        import torch
        B = x.shape[0]
        if y is None:
            y = torch.empty((B, 1) + (self.n,) * 3, dtype=torch.float32, device=x.device)
        ws = self.workspace(B)
        _check(lib().bbsur_forward(self.h, _p(params), _p(x), _p(y), B, _p(ws), ws.numel(),
                                   C.c_void_p(_stream(None))))
        return y

    def backward(self, params, x, dy):
        import torch
        B = x.shape[0]
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        ws = self.workspace(B)
        _check(lib().bbsur_backward(self.h, _p(params), _p(x), _p(dy), _p(g), B, _p(ws),
                                    ws.numel(), C.c_void_p(_stream(None))))
        return g

    def train_state(self, params):
        import torch
        z = lambda: torch.zeros_like(params)
        return TrainState(params, z(), z(), z())

    def train_step(self, st: TrainState, x, target, lr=1e-3, sync=True):
        import torch
        B = x.shape[0]
        st.step += 1
        if not hasattr(st, "loss"):
            st.loss = torch.zeros(1, dtype=torch.float32, device=x.device)
        ws = self.workspace(B)
        _check(lib().bbsur_train_step(self.h, _p(st.params), _p(st.grad), _p(st.m), _p(st.v),
                                      st.step, lr, _p(x), _p(target), B, _p(st.loss), _p(ws),
                                      ws.numel(), C.c_void_p(_stream(None))))
        return float(st.loss.item()) if sync else None


def as_numpy(t) -> np.ndarray:
    return t.detach().cpu().numpy()
