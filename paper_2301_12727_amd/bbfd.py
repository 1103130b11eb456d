"""ctypes binding of libbbfd (include/bbfd.h): argument marshalling only.

Every step of the solve runs in the HIP library; this module passes device
pointers (torch tensors' ``data_ptr()``) and HIP stream handles through.  It
raises if the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbbfd.so")

OK, EINVAL, EMATERIAL, EINDEX, EGEOMETRY, EDIVERGED, EHIP, ENOMEM = 0, -1, -2, -3, -4, -5, -6, -7
ERROR_NAMES = {EINVAL: "EINVAL", EMATERIAL: "EMATERIAL", EINDEX: "EINDEX",
               EGEOMETRY: "EGEOMETRY", EDIVERGED: "EDIVERGED", EHIP: "EHIP", ENOMEM: "ENOMEM"}


class BBFDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class Material(C.Structure):
    _fields_ = [("rho", C.c_double), ("c_l", C.c_double), ("c_s", C.c_double),
                ("alpha_l", C.c_double), ("alpha_s", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("pml", C.c_int32),
                ("freq_hz", C.c_double), ("ppw", C.c_double), ("qc", C.c_double),
                ("cfl_safety", C.c_double),
                ("n_steps", C.c_int32), ("capture_start", C.c_int32), ("source_k", C.c_int32),
                ("n_materials", C.c_int32), ("materials", C.POINTER(Material)),
                ("index_bits", C.c_int32)]


class Transducer(C.Structure):
    _fields_ = [("kind", C.c_int32), ("radius_m", C.c_double), ("focal_m", C.c_double),
                ("apex_m", C.c_double * 3), ("axis", C.c_double * 3), ("u0", C.c_double)]


class Element(C.Structure):
    _fields_ = [("radius_m", C.c_double), ("centre_m", C.c_double * 3), ("axis", C.c_double * 3),
                ("w_re", C.c_double), ("w_im", C.c_double)]


def element_array(elements):
    """ctypes array of bbfd_element from rows (radius, cx, cy, cz, ax, ay, az,
    w_re, w_im)."""
    rows = np.asarray(elements, dtype=np.float64).reshape(-1, 9)
    return (Element * len(rows))(*[Element(r[0], (C.c_double * 3)(*r[1:4]),
                                           (C.c_double * 3)(*r[4:7]), r[7], r[8]) for r in rows])


class PlanInfo(C.Structure):
    _fields_ = [("dx", C.c_double), ("dt", C.c_double), ("c_max", C.c_double),
                ("steps_per_period", C.c_int32), ("capture_start", C.c_int32),
                ("source_k", C.c_int32), ("pitch", C.c_int32),
                ("workspace_bytes", C.c_uint64), ("cells", C.c_uint64),
                ("tile_rows", C.c_int32), ("tile_planes", C.c_int32),
                ("graph_captures", C.c_uint64)]


EXPORTS = ["bbfd_plan_create", "bbfd_plan_get_info", "bbfd_plan_destroy",
           "bbfd_material_constants", "bbfd_transducer_elements", "bbfd_source_rayleigh",
           "bbfd_solve", "bbfd_solve_direct", "bbfd_solve_profiled", "bbfd_status",
           "bbfd_segment_classes", "bbfd_tile_counts",
           "bbfd_last_error", "bbfd_rayleigh_volume", "bbfd_batch_create", "bbfd_batch_destroy", "bbfd_batch_info",
           "bbfd_batch_plan", "bbfd_batch_offset", "bbfd_batch_set_shape", "bbfd_batch_solve",
           "bbfd_batch_status", "bbfd_batch_autotune", "bbfd_solve_static", "bbfd_energy_loss",
           "bbfd_bhte_create", "bbfd_bhte_destroy", "bbfd_bhte_info", "bbfd_bhte_run",
           "bbfd_array_elements", "bbfd_array_rayleigh", "bbfd_array_steer", "bbfd_array_refocus"]

_lib = None


def lib():
    """Load libbbfd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.bbfd_plan_create.argtypes = [C.POINTER(Problem), C.POINTER(vp)]
        L.bbfd_plan_get_info.argtypes = [vp, C.POINTER(PlanInfo)]
        L.bbfd_plan_destroy.argtypes = [vp]
        L.bbfd_plan_destroy.restype = None
        L.bbfd_material_constants.argtypes = [vp, vp, C.c_int32]
        L.bbfd_transducer_elements.argtypes = [vp, C.POINTER(Transducer), vp, C.c_int64,
                                               C.POINTER(C.c_int64)]
        L.bbfd_source_rayleigh.argtypes = [vp, C.POINTER(Transducer), vp, vp, C.c_uint64, vp]
        L.bbfd_rayleigh_volume.argtypes = [vp, C.POINTER(Transducer), vp, vp, C.c_uint64, vp]
        L.bbfd_solve.argtypes = [vp, vp, vp, vp, vp, C.c_uint64, vp]
        L.bbfd_solve_direct.argtypes = [vp, vp, vp, vp, vp, C.c_uint64, vp]
        L.bbfd_solve_profiled.argtypes = [vp, vp, vp, vp, vp, C.c_uint64, vp, vp]
        L.bbfd_status.argtypes = [vp, vp, C.POINTER(C.c_int64), C.POINTER(C.c_float), vp]
        L.bbfd_array_elements.argtypes = [vp, vp, C.c_int32, vp, C.c_int64, C.POINTER(C.c_int64)]
        L.bbfd_array_rayleigh.argtypes = [vp, vp, C.c_int32, vp, vp, C.c_uint64, vp]
        L.bbfd_array_steer.argtypes = [vp, vp, C.c_int32, vp, vp]
        L.bbfd_array_refocus.argtypes = [vp, vp, vp, C.c_int32, vp, vp, vp, vp, vp, C.c_uint64, vp]
        L.bbfd_energy_loss.argtypes = [vp, vp, vp, vp, vp, C.c_int32, vp, C.c_uint64, vp, vp]
        L.bbfd_solve_static.argtypes = [vp, vp, vp, vp, vp, C.POINTER(C.c_int64),
                                        C.POINTER(C.c_float)]
        L.bbfd_segment_classes.argtypes = [vp, vp, vp, C.c_uint64, vp]
        L.bbfd_tile_counts.argtypes = [vp, vp, vp, vp]
        L.bbfd_last_error.restype = C.c_char_p
        L.bbfd_batch_create.argtypes = [C.POINTER(Problem), C.c_int32, C.POINTER(vp)]
        L.bbfd_batch_destroy.argtypes = [vp]
        L.bbfd_batch_destroy.restype = None
        L.bbfd_batch_info.argtypes = [vp, C.POINTER(C.c_uint64), vp]
        L.bbfd_batch_plan.argtypes = [vp, C.c_int32]
        L.bbfd_batch_plan.restype = vp
        L.bbfd_batch_offset.argtypes = [vp, C.c_int32]
        L.bbfd_batch_offset.restype = C.c_uint64
        L.bbfd_batch_set_shape.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32]
        L.bbfd_batch_solve.argtypes = [vp, vp, vp, vp, vp, C.c_uint64, vp]
        L.bbfd_batch_status.argtypes = [vp, vp, C.c_int32, C.POINTER(C.c_int64),
                                        C.POINTER(C.c_float), vp]
        L.bbfd_batch_autotune.argtypes = [vp, vp, vp, vp, vp, C.c_uint64, vp, C.c_char_p,
                                          C.c_int32, C.POINTER(C.c_double)]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != OK:
        raise BBFDError(rc, lib().bbfd_last_error().decode())


def _stream(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def transducer_struct(t) -> Transducer:
    return Transducer(int(t.kind), float(t.radius), float(t.focal), (C.c_double * 3)(*t.apex),
                      (C.c_double * 3)(*t.axis), float(t.u0))


class Plan:
    """A validated problem with its derived device tables (libbbfd plan)."""

    def __init__(self, nx, ny, nz, freq_hz, ppw, n_steps, materials, pml=8, qc=1.0,
                 cfl_safety=0.95, capture_start=-1, source_k=-1, index_bits=8):
        mats = np.ascontiguousarray(materials, dtype=np.float64).reshape(-1, 5)
        self._mats = (Material * len(mats))(*[Material(*map(float, r)) for r in mats])
        self.problem = Problem(nx, ny, nz, pml, freq_hz, ppw, qc, cfl_safety, n_steps,
                               capture_start, source_k, len(mats), self._mats, index_bits)
        self.index_bits = index_bits
        self.h = C.c_void_p()
        _check(lib().bbfd_plan_create(C.byref(self.problem), C.byref(self.h)))
        info = PlanInfo()
        _check(lib().bbfd_plan_get_info(self.h, C.byref(info)))
        self.info = {n: getattr(info, n) for n, _ in PlanInfo._fields_}
        self.shape = (nz, ny, nx)
        self.n_materials = len(mats)

    @classmethod
    def from_case(cls, case, n_steps=None, **over):
        kw = dict(nx=case.nx, ny=case.ny, nz=case.nz, freq_hz=case.freq_hz, ppw=case.ppw,
                  n_steps=case.n_steps if n_steps is None else n_steps,
                  materials=case.materials, pml=case.pml, qc=case.qc,
                  cfl_safety=case.cfl_safety, capture_start=case.capture_start,
                  source_k=case.source_k,
                  index_bits=16 if case.mat is not None and case.mat.dtype == np.uint16 else 8)
        kw.update(over)
        return cls(**kw)

    def close(self):
        if self.h:
            lib().bbfd_plan_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def workspace_bytes(self) -> int:
        return int(self.info["workspace_bytes"])

    @property
    def graph_captures(self) -> int:
        """Time loops bbfd_solve has captured on this plan so far."""
        info = PlanInfo()
        _check(lib().bbfd_plan_get_info(self.h, C.byref(info)))
        return int(info.graph_captures)

    def material_constants(self) -> np.ndarray:
        out = np.empty((self.n_materials, 9), dtype=np.float64)
        _check(lib().bbfd_material_constants(self.h, out.ctypes.data_as(C.c_void_p),
                                             self.n_materials))
        return out

    def elements(self, t) -> np.ndarray:
        ts = transducer_struct(t)
        n = C.c_int64(0)
        _check(lib().bbfd_transducer_elements(self.h, C.byref(ts), None, 0, C.byref(n)))
        out = np.empty((n.value, 4), dtype=np.float64)
        _check(lib().bbfd_transducer_elements(self.h, C.byref(ts), out.ctypes.data_as(C.c_void_p),
                                              n.value, C.byref(n)))
        return out

    # --------------------------------------------------------- device calls
    def workspace(self, device="cuda"):
        import torch
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)

    def source_rayleigh(self, t, src, ws, stream=None):
        """Fill ``src`` (torch complex64 or float32 [ny, nx, 2], device) with the
        Rayleigh field on the source plane."""
        ts = transducer_struct(t)
        _check(lib().bbfd_source_rayleigh(self.h, C.byref(ts), C.c_void_p(src.data_ptr()),
                                          C.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                          C.c_void_p(_stream(stream))))

    def rayleigh_volume(self, t, field, ws, stream=None):
        """Fill ``field`` (torch complex64 [nz, ny, nx], device) with the free field."""
        ts = transducer_struct(t)
        _check(lib().bbfd_rayleigh_volume(self.h, C.byref(ts), C.c_void_p(field.data_ptr()),
                                          C.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                          C.c_void_p(_stream(stream))))

    def solve(self, mat, src, peak, ws, stream=None, graph=True):
        """Enqueue a full solve (asynchronous)."""
        fn = lib().bbfd_solve if graph else lib().bbfd_solve_direct
        _check(fn(self.h, C.c_void_p(mat.data_ptr()), C.c_void_p(src.data_ptr()),
                  C.c_void_p(peak.data_ptr()), C.c_void_p(ws.data_ptr()),
                  ws.numel() * ws.element_size(), C.c_void_p(_stream(stream))))

    # ----------------------------------------------------------- phased arrays
    def array_elements(self, elements) -> np.ndarray:
        """Sub-elements [m, 6] = (x, y, z, area, w_re, w_im) of an array given as
        rows (radius, cx, cy, cz, ax, ay, az, w_re, w_im)."""
        el = element_array(elements)
        n = C.c_int64(0)
        _check(lib().bbfd_array_elements(self.h, el, len(el), None, 0, C.byref(n)))
        out = np.empty((n.value, 6), dtype=np.float64)
        _check(lib().bbfd_array_elements(self.h, el, len(el), out.ctypes.data_as(C.c_void_p),
                                         n.value, C.byref(n)))
        return out

    def array_rayleigh(self, elements, src, ws, stream=None):
        el = element_array(elements)
        _check(lib().bbfd_array_rayleigh(self.h, el, len(el), C.c_void_p(src.data_ptr()),
                                         C.c_void_p(ws.data_ptr()), ws.numel(),
                                         C.c_void_p(_stream(stream))))

    def array_steer(self, elements, target) -> np.ndarray:
        """Unit complex drives focusing the array on target (m) in water."""
        el = element_array(elements)
        w = np.empty(2 * len(el), dtype=np.float64)
        t = np.ascontiguousarray(target, dtype=np.float64)
        _check(lib().bbfd_array_steer(self.h, el, len(el), t.ctypes.data_as(C.c_void_p),
                                      w.ctypes.data_as(C.c_void_p)))
        return w[0::2] + 1j * w[1::2]

    def array_refocus(self, mat, elements, cell, peak, ws, stream=None):
        """Time-reversal drives through mat for the target cell (i, j, k);
        returns (drives, back-propagated field at the elements), both complex [n]."""
        el = element_array(elements)
        w = np.empty(2 * len(el), dtype=np.float64)
        f = np.empty(2 * len(el), dtype=np.float64)
        c = np.ascontiguousarray(cell, dtype=np.int32)
        _check(lib().bbfd_array_refocus(self.h, C.c_void_p(mat.data_ptr()), el, len(el),
                                        c.ctypes.data_as(C.c_void_p), C.c_void_p(peak.data_ptr()),
                                        w.ctypes.data_as(C.c_void_p), f.ctypes.data_as(C.c_void_p),
                                        C.c_void_p(ws.data_ptr()), ws.numel(),
                                        C.c_void_p(_stream(stream))))
        return w[0::2] + 1j * w[1::2], f[0::2] + 1j * f[1::2]

    def energy_loss(self, mat_skull, peak_skull, mat_water, peak_water, ws, z_m=-1, stream=None):
        """bbfd_energy_loss: (E_L, T_S, z_m, skull plane sum, water plane sum) of
        a transcranial solve against its water-only companion (waits)."""
        out = np.zeros(5, dtype=np.float64)
        _check(lib().bbfd_energy_loss(self.h, C.c_void_p(mat_skull.data_ptr()),
                                      C.c_void_p(peak_skull.data_ptr()),
                                      C.c_void_p(mat_water.data_ptr()),
                                      C.c_void_p(peak_water.data_ptr()), int(z_m),
                                      C.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                      C.c_void_p(_stream(stream)),
                                      out.ctypes.data_as(C.c_void_p)))
        return float(out[0]), float(out[1]), int(out[2]), float(out[3]), float(out[4])

    def solve_static(self, mat, src, peak, stream=None, status=True):
        """bbfd_solve_static: the solve with the library's fixed per-GPU device
        array as its workspace (nothing allocated).  With status=True it waits
        and returns (peak_index, peak_value), else returns None once enqueued."""
        idx = C.c_int64(-1)
        val = C.c_float(0.0)
        _check(lib().bbfd_solve_static(self.h, C.c_void_p(mat.data_ptr()),
                                       C.c_void_p(src.data_ptr()), C.c_void_p(peak.data_ptr()),
                                       C.c_void_p(_stream(stream)),
                                       C.byref(idx) if status else None,
                                       C.byref(val) if status else None))
        return (int(idx.value), float(val.value)) if status else None

    def solve_profiled(self, mat, src, peak, ws, stream=None):
        """Direct-launch solve with per-kernel HIP events on the launch stream;
        returns the summed milliseconds of the five step kernels over the time
        loop: (acoustic velocity, general velocity, acoustic stress, general
        stress, fused step of the deep tiles)."""
        out = np.zeros(5, dtype=np.float64)
        _check(lib().bbfd_solve_profiled(self.h, C.c_void_p(mat.data_ptr()),
                                         C.c_void_p(src.data_ptr()), C.c_void_p(peak.data_ptr()),
                                         C.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                         C.c_void_p(_stream(stream)),
                                         out.ctypes.data_as(C.c_void_p)))
        return tuple(float(v) for v in out)

    def status(self, ws, stream=None):
        """Synchronise and return (peak_index, peak_value); raises on device errors."""
        idx = C.c_int64(-1)
        val = C.c_float(0.0)
        _check(lib().bbfd_status(self.h, C.c_void_p(ws.data_ptr()), C.byref(idx), C.byref(val),
                                 C.c_void_p(_stream(stream))))
        return int(idx.value), float(val.value)

    def tile_counts(self, ws, stream=None):
        """Tiles of each kind in the last solve in ws: (acoustic, general, deep)."""
        out = (C.c_int32 * 3)()
        _check(lib().bbfd_tile_counts(self.h, C.c_void_p(ws.data_ptr()), out,
                                      C.c_void_p(_stream(stream))))
        return tuple(out)

    def segment_classes(self, ws, stream=None):
        """Row-segment classes of the last solve in ws, uint8 [nz][ny][ceil(nx/64)]
        (0: elastic branch, m + 1: acoustic branch for lossless fluid m)."""
        nz, ny, nx = self.shape
        out = np.zeros((nz, ny, (nx + 63) // 64), dtype=np.uint8)
        _check(lib().bbfd_segment_classes(self.h, C.c_void_p(ws.data_ptr()),
                                          out.ctypes.data_as(C.c_void_p), out.size,
                                          C.c_void_p(_stream(stream))))
        return out


def _ptr_array(tensors):
    return (C.c_void_p * len(tensors))(*[C.c_void_p(t.data_ptr()) for t in tensors])


class Batch:
    """Uneven sweep of independent solves run by one captured graph: tiled
    kernels walking per-kind (solve, tile) tables, or every solve's own step
    kernels one after the other (the per-solve shape); autotuned."""

    def __init__(self, cases, n_steps=None):
        self._plans_py = [Plan.from_case(c, n_steps=n_steps) for c in cases]  # validation, info
        probs = (Problem * len(cases))(*[p.problem for p in self._plans_py])
        self._probs = probs
        self.h = C.c_void_p()
        _check(lib().bbfd_batch_create(probs, len(cases), C.byref(self.h)))
        self.n = len(cases)
        self.shapes = [p.shape for p in self._plans_py]

    def close(self):
        if self.h:
            lib().bbfd_batch_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        ws = C.c_uint64(0)
        shape = (C.c_int32 * 4)()
        _check(lib().bbfd_batch_info(self.h, C.byref(ws), shape))
        return int(ws.value), tuple(shape)

    @property
    def workspace_bytes(self) -> int:
        return self.info()[0]

    def workspace(self, device="cuda"):
        import torch
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)

    def source_rayleigh(self, i, t, src, ws, stream=None):
        """Rayleigh plane of solve i, staged in solve i's part of the workspace."""
        plan = lib().bbfd_batch_plan(self.h, i)
        if not plan:
            _check(EINVAL)
        off = int(lib().bbfd_batch_offset(self.h, i))
        sub = ws[off:]
        ts = transducer_struct(t)
        _check(lib().bbfd_source_rayleigh(C.c_void_p(plan), C.byref(ts),
                                          C.c_void_p(src.data_ptr()), C.c_void_p(sub.data_ptr()),
                                          sub.numel(), C.c_void_p(_stream(stream))))

    def rayleigh_volume(self, i, t, field, ws, stream=None):
        """Free field of solve i's transducer on its whole grid (complex64 [nz, ny, nx])."""
        plan = lib().bbfd_batch_plan(self.h, i)
        if not plan:
            _check(EINVAL)
        off = int(lib().bbfd_batch_offset(self.h, i))
        sub = ws[off:]
        ts = transducer_struct(t)
        _check(lib().bbfd_rayleigh_volume(C.c_void_p(plan), C.byref(ts),
                                          C.c_void_p(field.data_ptr()), C.c_void_p(sub.data_ptr()),
                                          sub.numel(), C.c_void_p(_stream(stream))))

    def set_shape(self, by, blocks, kchunk):
        """Tiled launch shape (rows per block 1/2/4/8, persistent blocks or 0,
        z cells per tile), or by = 0 for the per-solve shape."""
        _check(lib().bbfd_batch_set_shape(self.h, by, blocks, kchunk))

    def solve(self, mats, srcs, peaks, ws, stream=None):
        self._keep = (_ptr_array(mats), _ptr_array(srcs), _ptr_array(peaks))
        _check(lib().bbfd_batch_solve(self.h, *self._keep, C.c_void_p(ws.data_ptr()),
                                      ws.numel(), C.c_void_p(_stream(stream))))

    def status(self, ws, i, stream=None):
        idx = C.c_int64(-1)
        val = C.c_float(0.0)
        _check(lib().bbfd_batch_status(self.h, C.c_void_p(ws.data_ptr()), i, C.byref(idx),
                                       C.byref(val), C.c_void_p(_stream(stream))))
        return int(idx.value), float(val.value)

    def autotune(self, mats, srcs, peaks, ws, cache_path=None, probe_steps=10, stream=None):
        arrs = (_ptr_array(mats), _ptr_array(srcs), _ptr_array(peaks))
        best = C.c_double(0.0)
        _check(lib().bbfd_batch_autotune(self.h, *arrs, C.c_void_p(ws.data_ptr()), ws.numel(),
                                         C.c_void_p(_stream(stream)),
                                         None if cache_path is None else cache_path.encode(),
                                         probe_steps, C.byref(best)))
        return float(best.value), self.info()[1]


def run_case(case, n_steps=None, device="cuda", graph=True, **over):
    """Rayleigh source + full solve of a synthetic case on the GPU.
    Returns (peak torch.float32 [nz, ny, nx], peak_index, peak_value, plan)."""
    import torch
    plan = Plan.from_case(case, n_steps=n_steps, **over)
    ws = plan.workspace(device)
    src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device=device)
    plan.source_rayleigh(case.transducer, src, ws)
    mat = torch.from_numpy(np.ascontiguousarray(case.mat)).to(device)
    peak = torch.empty(plan.shape, dtype=torch.float32, device=device)
    plan.solve(mat, src, peak, ws, graph=graph)
    idx, val = plan.status(ws)
    return peak, idx, val, plan
