"""Python access to the FP64 CPU oracle (``libbbref.so``).

TEST INFRASTRUCTURE ONLY: the checker of the HIP library.  Only the test
suite, the smoke entry and the benchmark's CPU-baseline leg may import this
package; the product path never does.  It imports nothing from the product
package and shares no code with it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbbref.so")

EINVAL, EMATERIAL, EINDEX, EGEOMETRY, EDIVERGED = -1, -2, -3, -4, -5
LATERAL_PERIODIC = 1
SOURCE_SHEAR_XZ = 2

FIELDS = ["vx", "vy", "vz", "sxx", "syy", "szz", "sxy", "sxz", "syz",
          "rxx", "ryy", "rzz", "rxy", "rxz", "ryz", "peak"]


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed with code {code}")
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
                ("mode", C.c_int32), ("index_bits", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("dx", C.c_double), ("dt", C.c_double), ("omega", C.c_double),
                ("c_max", C.c_double), ("d0", C.c_double),
                ("steps_per_period", C.c_int32), ("capture_start", C.c_int32),
                ("source_k", C.c_int32)]


class MatConst(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("q_p", "q_s", "tau_p", "tau_s", "pi_r", "mu_r", "pi_u", "mu_u", "nu")]


class Transducer(C.Structure):
    _fields_ = [("kind", C.c_int32), ("radius", C.c_double), ("focal", C.c_double),
                ("apex", C.c_double * 3), ("axis", C.c_double * 3), ("u0", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library missing: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        L.bbref_setup.argtypes = [C.POINTER(Problem), C.POINTER(Info), C.POINTER(MatConst)]
        L.bbref_sim_create.argtypes = [C.POINTER(Problem), C.c_void_p, C.POINTER(C.c_void_p)]
        L.bbref_sim_destroy.argtypes = [C.c_void_p]
        L.bbref_sim_field.argtypes = [C.c_void_p, C.c_int32]
        L.bbref_sim_field.restype = C.POINTER(C.c_double)
        L.bbref_sim_step.argtypes = [C.c_void_p, C.c_int32, C.c_void_p]
        L.bbref_solve.argtypes = [C.POINTER(Problem), C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.bbref_elements.argtypes = [C.POINTER(Transducer), C.c_double, C.c_double, C.c_void_p,
                                     C.c_int64, C.POINTER(C.c_int64)]
        L.bbref_rayleigh.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.c_double, C.c_void_p,
                                     C.c_int64, C.c_void_p]
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Thread count of the oracle's OpenMP loops from now on (libgomp's
    omp_set_num_threads, reached through the oracle library's own handle);
    returns the previous maximum."""
    L = lib()
    prev = int(L.omp_get_max_threads())
    L.omp_set_num_threads(C.c_int(int(n)))
    return prev


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class _Prob:
    """Keeps the ctypes problem and its material array alive together."""

    def __init__(self, nx, ny, nz, pml, freq_hz, ppw, n_steps, materials, qc=1.0,
                 cfl_safety=0.95, capture_start=-1, source_k=-1, mode=0, index_bits=8):
        mats = np.ascontiguousarray(materials, dtype=np.float64).reshape(-1, 5)
        self.mats = (Material * len(mats))(*[Material(*map(float, r)) for r in mats])
        self.p = Problem(nx, ny, nz, pml, freq_hz, ppw, qc, cfl_safety, n_steps,
                         capture_start, source_k, len(mats), self.mats, mode, index_bits)

    @property
    def map_dtype(self):
        return np.uint16 if self.p.index_bits == 16 else np.uint8


def problem_from_case(case, n_steps=None, mode=0, **over):
    kw = dict(nx=case.nx, ny=case.ny, nz=case.nz, pml=case.pml, freq_hz=case.freq_hz,
              ppw=case.ppw, n_steps=case.n_steps if n_steps is None else n_steps,
              materials=case.materials, qc=case.qc, cfl_safety=case.cfl_safety,
              capture_start=case.capture_start, source_k=case.source_k, mode=mode,
              index_bits=16 if case.mat is not None and case.mat.dtype == np.uint16 else 8)
    kw.update(over)
    return _Prob(**kw)


def setup(prob: _Prob):
    info = Info()
    mc = (MatConst * prob.p.n_materials)()
    rc = lib().bbref_setup(C.byref(prob.p), C.byref(info), mc)
    if rc:
        raise OracleError(rc, "bbref_setup")
    consts = [{n: getattr(m, n) for n, _ in MatConst._fields_} for m in mc]
    return {n: getattr(info, n) for n, _ in Info._fields_}, consts


class Sim:
    """Stateful oracle run (fields start at rest)."""

    def __init__(self, prob: _Prob, mat: np.ndarray):
        self.prob = prob
        self.mat = np.ascontiguousarray(mat, dtype=prob.map_dtype)
        self.h = C.c_void_p()
        rc = lib().bbref_sim_create(C.byref(prob.p), _ptr(self.mat), C.byref(self.h))
        if rc:
            raise OracleError(rc, "bbref_sim_create")
        self.shape = (prob.p.nz, prob.p.ny, prob.p.nx)

    def field(self, name: str) -> np.ndarray:
        """Writable view of a field (no copy)."""
        p = lib().bbref_sim_field(self.h, FIELDS.index(name))
        return np.ctypeslib.as_array(p, shape=self.shape)

    def step(self, n: int, src: np.ndarray | None):
        s = None if src is None else np.ascontiguousarray(src, dtype=np.complex128)
        lib().bbref_sim_step(self.h, n, None if s is None else _ptr(s))
        self._keep = s

    def close(self):
        if self.h:
            lib().bbref_sim_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(prob: _Prob, mat: np.ndarray, src: np.ndarray):
    """Full solve; returns (peak [nz,ny,nx] float64, peak_index, loop seconds)."""
    mat = np.ascontiguousarray(mat, dtype=prob.map_dtype)
    s = np.ascontiguousarray(src, dtype=np.complex128)
    peak = np.empty((prob.p.nz, prob.p.ny, prob.p.nx), dtype=np.float64)
    idx = C.c_int64(-1)
    secs = C.c_double(0.0)
    rc = lib().bbref_solve(C.byref(prob.p), _ptr(mat), _ptr(s), _ptr(peak), C.byref(idx),
                           C.byref(secs))
    if rc:
        raise OracleError(rc, "bbref_solve")
    return peak, int(idx.value), float(secs.value)


def transducer(t) -> Transducer:
    return Transducer(int(t.kind), float(t.radius), float(t.focal),
                      (C.c_double * 3)(*t.apex), (C.c_double * 3)(*t.axis), float(t.u0))


def elements(t, freq_hz: float, area_div: float = 16.0) -> np.ndarray:
    """Surface elements [n, 4] = (x, y, z, area)."""
    tr = transducer(t)
    n = C.c_int64(0)
    rc = lib().bbref_elements(C.byref(tr), freq_hz, area_div, None, 0, C.byref(n))
    if rc:
        raise OracleError(rc, "bbref_elements")
    out = np.empty((n.value, 4), dtype=np.float64)
    rc = lib().bbref_elements(C.byref(tr), freq_hz, area_div, _ptr(out), n.value, C.byref(n))
    if rc:
        raise OracleError(rc, "bbref_elements")
    return out


def rayleigh(el: np.ndarray, freq_hz: float, u0: float, pts: np.ndarray) -> np.ndarray:
    el = np.ascontiguousarray(el, dtype=np.float64)
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    out = np.empty(len(pts), dtype=np.complex128)
    lib().bbref_rayleigh(_ptr(el), len(el), freq_hz, u0, _ptr(pts), len(pts), _ptr(out))
    return out


def source_plane(case, area_div: float = 16.0) -> np.ndarray:
    """Rayleigh field on the source plane z = (k_s + 1/2) dx at the (x, y) cell
    centres, complex [ny, nx]."""
    t = case.transducer
    el = elements(t, case.freq_hz, area_div)
    dx = case.dx
    ks = case.pml if case.source_k < 0 else case.source_k
    if np.any(el[:, 2] >= ks * dx):
        raise OracleError(EGEOMETRY, "transducer crosses the source plane")
    jj, ii = np.meshgrid(np.arange(case.ny), np.arange(case.nx), indexing="ij")
    pts = np.stack([ii * dx, jj * dx, np.full(ii.shape, (ks + 0.5) * dx)], axis=-1)
    return rayleigh(el, case.freq_hz, t.u0, pts).reshape(case.ny, case.nx)


def solve_case(case, n_steps=None, **over):
    """Rayleigh source plane + full solve for a synthetic case."""
    prob = problem_from_case(case, n_steps=n_steps, **over)
    src = source_plane(case)
    return solve(prob, case.mat, src)
