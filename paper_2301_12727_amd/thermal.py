"""ctypes binding of the thermal step (BHTE) of libbbfd (include/bbfd.h,
bbfd_bhte_*): argument marshalling only; the heat source, the time loop, the
maximal temperature and the thermal dose run in the library's HIP kernels."""
from __future__ import annotations

import ctypes as C

import numpy as np

from .bbfd import Material, _check, _stream, lib


class ThermalRow(C.Structure):
    _fields_ = [("k", C.c_double), ("c", C.c_double), ("perfusion", C.c_double),
                ("heat_frac", C.c_double)]


class BHTEProblem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dt", C.c_double), ("n_on", C.c_int32), ("n_off", C.c_int32),
                ("duty", C.c_double), ("t_body", C.c_double), ("intensity_scale", C.c_double),
                ("n_materials", C.c_int32), ("acoustic", C.POINTER(Material)),
                ("thermal", C.POINTER(ThermalRow))]


_SIG = False


def _sigs():
    global _SIG
    L = lib()
    if not _SIG:
        vp = C.c_void_p
        L.bbfd_bhte_create.argtypes = [C.POINTER(BHTEProblem), C.POINTER(vp)]
        L.bbfd_bhte_destroy.argtypes = [vp]
        L.bbfd_bhte_destroy.restype = None
        L.bbfd_bhte_info.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_double)]
        L.bbfd_bhte_run.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.c_uint64, vp]
        _SIG = True
    return L


class Thermal:
    """A validated BHTE problem (bbfd_bhte plan).  acoustic: [n, 5] rows (rho,
    c_l, c_s, alpha_l, alpha_s) as the FDTD table; thermal: [n, 4] rows (k, C,
    perfusion, heat share h)."""

    def __init__(self, shape, dx, dt, acoustic, thermal, n_on, n_off, duty=1.0, t_body=37.0,
                 intensity_scale=1.0):
        nz, ny, nx = shape
        ac = np.ascontiguousarray(acoustic, dtype=np.float64).reshape(-1, 5)
        th = np.ascontiguousarray(thermal, dtype=np.float64).reshape(-1, 4)
        self._ac = (Material * len(ac))(*[Material(*map(float, r)) for r in ac])
        self._th = (ThermalRow * len(th))(*[ThermalRow(*map(float, r)) for r in th])
        self.problem = BHTEProblem(nx, ny, nz, dx, dt, n_on, n_off, duty, t_body, intensity_scale,
                                   len(ac), self._ac, self._th)
        self.shape = (nz, ny, nx)
        self.h = C.c_void_p()
        L = _sigs()
        _check(L.bbfd_bhte_create(C.byref(self.problem), C.byref(self.h)))
        ws, dtm = C.c_uint64(0), C.c_double(0.0)
        _check(L.bbfd_bhte_info(self.h, C.byref(ws), C.byref(dtm)))
        self.workspace_bytes, self.dt_max = int(ws.value), float(dtm.value)

    def close(self):
        if self.h:
            lib().bbfd_bhte_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, device="cuda"):
        import torch
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)

    def run(self, mat, peak, t_final, t_max, dose, ws, stream=None):
        """Enqueue the whole sonication (asynchronous); outputs float32 [nz, ny, nx]."""
        p = lambda t: C.c_void_p(t.data_ptr())
        _check(_sigs().bbfd_bhte_run(self.h, p(mat), p(peak), p(t_final), p(t_max), p(dose), p(ws),
                                     ws.numel(), C.c_void_p(_stream(stream))))
