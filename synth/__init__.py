"""Seeded synthetic inputs for the transcranial FDTD solve.

This module builds the *inputs* of the solve and nothing else: uint8 material
maps, material property rows (density, longitudinal/shear speed, longitudinal/
shear attenuation at the drive frequency) and transducer poses.  It holds none
of the solver's arithmetic (no moduli, relaxation constants, time step, absorbing
layer, surface discretisation or Rayleigh sum); the FP64 oracle and the HIP
library each derive those from these inputs on their own.

Recipes (all distances in metres, frequencies in Hz):

* Property rows follow the homogenised-material table of the paper (Section
  2.2.1, Table 1).  Speeds take the frequency term with f in Hz, attenuations
  are Np/m/MHz times f in MHz.  Water has no attenuation and no shear speed.
* ``plate_case``: 64^3 water box with a 3-voxel bone plate (the 64^3 plate
  workload) and a flat piston 3 mm outside the source plane.
* ``skull_case``: spherical skull shell of outer radius 70 mm whose centre sits
  80 mm beyond the source plane on the acoustic axis; thickness 6.5 +- 1.5 mm
  from seeded value noise; cortical/trabecular/cortical split 10/80/10 (Section
  2.2.1); trabecular porosity 0.2-0.6 from a second noise field, quantised to 8
  bins mixed linearly between cortical bone and water; skin and brain are water
  (Section 3.2.4).  Source: spherical bowl, aperture 64 mm, F#1 by default,
  rim 3 mm before the source plane.
* ``batch_cases``: 32 uneven solves (96..160 cells per axis) at 250/500/700 kHz
  with seeded bowl tilts of +-15 degrees about the focus.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

C_WATER = 1500.0
RHO_WATER = 1000.0

# Property-row layout shared by every consumer: rho, c_l, c_s, alpha_l, alpha_s.
N_PROP = 5


def table1(freq_hz: float) -> dict:
    """Homogenised properties at ``freq_hz`` (paper Section 2.2.1, Table 1).

    Returns name -> (rho, c_l, c_s, alpha_l [Np/m], alpha_s [Np/m]).
    The speed terms use f in Hz; the attenuation coefficients are Np/m/MHz.
    """
    f_mhz = freq_hz * 1e-6
    return {
        "water": (1000.0, 1500.0, 0.0, 0.0, 0.0),
        "skin": (1116.0, 1537.0, 0.0, 4.6 * f_mhz, 0.0),
        "brain": (1041.0, 1562.0, 0.0, 6.9 * f_mhz, 0.0),
        "cortical": (1896.5, 2415.0 + 1.2e-4 * freq_hz, 1369.0 + 3.4e-4 * freq_hz,
                     163.0 * f_mhz, 329.0 * f_mhz),
        "trabecular": (1738.0, 2063.0 + 2.8e-4 * freq_hz, 1206.0 + 2.1e-4 * freq_hz,
                       162.0 * f_mhz, 329.0 * f_mhz),
    }


@dataclasses.dataclass
class Transducer:
    """Single-element source.  kind 0: flat piston (``radius`` = face radius,
    ``apex`` = face centre); kind 1: spherical bowl (``radius`` = aperture
    radius, ``focal`` = radius of curvature, ``apex`` = bowl apex on the axis).
    ``axis`` is the unit propagation direction; ``u0`` the normal surface
    velocity amplitude in m/s."""
    kind: int
    radius: float
    focal: float
    apex: tuple
    axis: tuple
    u0: float = 1.0


@dataclasses.dataclass
class Case:
    name: str
    nx: int
    ny: int
    nz: int
    pml: int
    freq_hz: float
    ppw: float
    n_steps: int
    materials: np.ndarray          # float64 [n_materials, 5]
    mat: np.ndarray | None         # uint8 [nz, ny, nx] (None until built)
    transducer: Transducer
    qc: float = 1.0
    cfl_safety: float = 0.95
    capture_start: int = -1        # < 0: last two periods
    source_k: int = -1             # < 0: first interior plane (= pml)

    @property
    def dx(self) -> float:
        # Grid spacing fixed by frequency and points per wavelength in water
        # (Section 2.2); an input-side quantity both solvers receive as ppw.
        return C_WATER / (self.freq_hz * self.ppw)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    def source_plane_z(self) -> float:
        k = self.pml if self.source_k < 0 else self.source_k
        return k * self.dx


def _rows(*rows) -> np.ndarray:
    return np.ascontiguousarray(np.array(rows, dtype=np.float64).reshape(-1, N_PROP))


# ---------------------------------------------------------------- plate (64^3)

PLATE = (1900.0, 2800.0, 1500.0, 85.0, 280.0)


def plate_case(n: int = 64, n_steps: int = 600, plate_k=(20, 21, 22),
               plate=PLATE, freq_hz: float = 250e3, ppw: float = 6.0,
               pml: int = 8, piston_radius: float = 15e-3) -> Case:
    """Water box with a flat bone plate across x-y at ``plate_k`` and a flat
    piston 3 mm outside the source plane, centred on cell (n/2, n/2)."""
    mat = np.zeros((n, n, n), dtype=np.uint8)
    for k in plate_k:
        mat[k] = 1
    c = Case("plate64", n, n, n, pml, freq_hz, ppw, n_steps,
             _rows(table1(freq_hz)["water"], plate), mat, None)
    dx = c.dx
    zs = c.source_plane_z()
    c.transducer = Transducer(0, piston_radius, 0.0,
                              ((n // 2) * dx, (n // 2) * dx, zs - 3e-3), (0.0, 0.0, 1.0))
    return c


# ---------------------------------------------------------------- skull shell

class _ValueNoise:
    """Seeded 3D value noise in [-1, 1]: uniform lattice values (PCG64) with
    trilinear interpolation, lattice spacing ``cell`` metres, covering
    ``lo``..``hi`` (metres, per axis)."""

    def __init__(self, rng: np.random.Generator, cell: float, lo, hi):
        self.cell = float(cell)
        self.lo = np.asarray(lo, dtype=np.float64) - 2 * cell
        n = np.ceil((np.asarray(hi, dtype=np.float64) + 2 * cell - self.lo) / cell).astype(int) + 2
        self.vals = rng.uniform(-1.0, 1.0, size=tuple(n[::-1]))  # [z, y, x]

    def __call__(self, x, y, z):
        u = [(c - lo) / self.cell for c, lo in zip((x, y, z), self.lo)]
        i0 = [np.floor(v).astype(np.int64) for v in u]
        f = [v - i for v, i in zip(u, i0)]
        out = np.zeros(np.shape(x), dtype=np.float64)
        for dz in (0, 1):
            wz = f[2] if dz else 1.0 - f[2]
            for dy in (0, 1):
                wy = f[1] if dy else 1.0 - f[1]
                for dxi in (0, 1):
                    wx = f[0] if dxi else 1.0 - f[0]
                    out += wx * wy * wz * self.vals[i0[2] + dz, i0[1] + dy, i0[0] + dxi]
        return out


N_PORO_BINS = 8
PORO_LO, PORO_HI = 0.2, 0.6


def skull_materials(freq_hz: float) -> np.ndarray:
    """10 rows: 0 water, 1 cortical, 2..9 trabecular porosity bins.  A bin of
    porosity phi mixes cortical bone and water linearly in density and
    longitudinal speed, scales the shear speed by (1 - phi) and keeps the
    trabecular attenuation row of Table 1."""
    t = table1(freq_hz)
    rho_c, cl_c, cs_c, _, _ = t["cortical"]
    _, _, _, al_t, as_t = t["trabecular"]
    rows = [t["water"], t["cortical"]]
    for b in range(N_PORO_BINS):
        phi = PORO_LO + b * (PORO_HI - PORO_LO) / (N_PORO_BINS - 1)
        rows.append(((1 - phi) * rho_c + phi * RHO_WATER,
                     (1 - phi) * cl_c + phi * C_WATER,
                     (1 - phi) * cs_c, al_t, as_t))
    return _rows(*rows)


# Thermal rows for the thermal step (k W/(m K), C J/(kg K), perfusion 1/s,
# heating share h of alpha_l).  The paper gives no thermal properties; these
# are typical literature values for brain and skull bone, and the bone share
# h = 0.16 is the paper's (Section 2.4).
THERMAL_BRAIN = (0.51, 3630.0, 0.0095, 1.0)
THERMAL_CORTICAL = (0.32, 1313.0, 0.0003, 0.16)
THERMAL_TRABECULAR = (0.31, 2274.0, 0.0029, 0.16)


def thermal_materials(freq_hz: float):
    """Acoustic and thermal tables for the thermal step on a skull map of
    ``skull_materials`` indices: index 0 is brain tissue (Table 1 density,
    speed and attenuation at ``freq_hz``), 1 cortical bone, 2..9 trabecular
    bins (thermal rows mixing trabecular bone and brain by porosity).
    Returns (acoustic [10, 5], thermal [10, 4])."""
    ac = skull_materials(freq_hz).copy()
    ac[0] = table1(freq_hz)["brain"]
    rows = [THERMAL_BRAIN, THERMAL_CORTICAL]
    for b in range(N_PORO_BINS):
        phi = PORO_LO + b * (PORO_HI - PORO_LO) / (N_PORO_BINS - 1)
        rows.append(tuple((1 - phi) * t + phi * w for t, w in zip(THERMAL_TRABECULAR[:3],
                                                                   THERMAL_BRAIN[:3])) + (0.16,))
    return ac, np.array(rows, dtype=np.float64)


def focus_map(shape, centre, width: float, amplitude: float, seed: int = 0,
              floor: float = 0.05) -> np.ndarray:
    """Synthetic peak-pressure map [nz, ny, nx] (Pa): a Gaussian focal spot of
    the given width (cells) and amplitude at ``centre`` (k, j, i), over a
    seeded smooth background of ``floor`` times the amplitude."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r2 = (k - centre[0]) ** 2 + (j - centre[1]) ** 2 + (i - centre[2]) ** 2
    bg = rng.uniform(0.5, 1.0, size=shape)
    return (amplitude * (np.exp(-r2 / (2.0 * width ** 2)) + floor * bg)).astype(np.float32)


def bowl_pose(focus, tilt_x: float, tilt_y: float, focal: float):
    """Apex and axis of a bowl rotated by ``tilt_x`` about x then ``tilt_y``
    about y (radians) around its geometric focus."""
    cx, sx = math.cos(tilt_x), math.sin(tilt_x)
    cy, sy = math.cos(tilt_y), math.sin(tilt_y)
    # R_y(ty) @ R_x(tx) @ e_z
    ax = np.array([sy * cx, -sx, cy * cx])
    ax /= np.linalg.norm(ax)
    apex = np.asarray(focus, dtype=np.float64) - focal * ax
    return tuple(apex), tuple(ax)


def bowl_focus_for_standoff(zs: float, radius: float, focal: float, axis, standoff: float):
    """z of the focus such that the highest rim point of the (tilted) bowl
    sits ``standoff`` before the source plane ``zs``."""
    nz = axis[2]
    sin_t = radius / focal
    cos_t = math.sqrt(1.0 - sin_t * sin_t)
    rim_top = -focal * cos_t * nz + focal * sin_t * math.sqrt(max(0.0, 1.0 - nz * nz))
    return zs - standoff - rim_top


# ------------------------------------------------------------ phased arrays

def cap_array(focus, focal: float, aperture_radius: float, n: int, piston_radius: float,
              rings: int = 0) -> np.ndarray:
    """n flat circular pistons on a spherical cap of curvature radius ``focal``
    and aperture radius ``aperture_radius`` around the axis +z through
    ``focus``, each facing the focus; rows (radius, cx, cy, cz, ax, ay, az,
    w_re, w_im) with unit drive.  rings = 0: centres on a golden-angle spiral
    over the cap (a hemispherical-array layout, like the paper's multi-element
    H317); rings > 0: ``rings`` annuli of equal area, each with n // rings
    pistons equally spaced in azimuth (an annular-array layout, like its
    CTX-500).  Stands in for the paper's transducers, whose geometry it does
    not print."""
    f = np.asarray(focus, dtype=np.float64)
    th_max = math.asin(aperture_radius / focal)
    # polar angles of element centres, measured from -z at the focus
    if rings > 0:
        per = max(1, n // rings)
        c_edges = np.linspace(1.0, math.cos(th_max), rings + 1)      # equal-area annuli
        th = []
        ph = []
        for r in range(rings):
            t = math.acos(0.5 * (c_edges[r] + c_edges[r + 1]))
            for q in range(per):
                th.append(t)
                ph.append(2 * math.pi * (q + 0.5 * (r % 2)) / per)
        th, ph = np.array(th), np.array(ph)
    else:
        q = np.arange(n) + 0.5
        th = np.arccos(1.0 - (1.0 - math.cos(th_max)) * q / n)
        ph = q * math.pi * (3.0 - math.sqrt(5.0))
    pos = f[None, :] + focal * np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph),
                                         -np.cos(th)], axis=1)
    ax = (f[None, :] - pos) / focal
    rows = np.zeros((len(th), 9))
    rows[:, 0] = piston_radius
    rows[:, 1:4] = pos
    rows[:, 4:7] = ax
    rows[:, 7] = 1.0
    return rows


def flat_array(centre, aperture_radius: float, n: int, piston_radius: float,
               rings: int) -> np.ndarray:
    """n flat circular pistons on the plane z = centre[2], facing +z, on
    ``rings`` annuli of equal area around ``centre`` (n // rings pistons each,
    equally spaced in azimuth); rows as ``cap_array``, unit drive."""
    c = np.asarray(centre, dtype=np.float64)
    per = max(1, n // rings)
    rows = []
    for r in range(rings):
        rho = aperture_radius * math.sqrt((r + 0.5) / rings)   # mid-area radius of the annulus
        for q in range(per):
            ph = 2 * math.pi * (q + 0.5 * (r % 2)) / per
            rows.append((piston_radius, c[0] + rho * math.cos(ph), c[1] + rho * math.sin(ph), c[2],
                         0.0, 0.0, 1.0, 1.0, 0.0))
    return np.array(rows, dtype=np.float64)


# The paper's multi-element transducers (Section 2), by what it states of
# them: the number of elements or rings, the focal length F and F-number
# (aperture diameter F / F#) of the curved ones, the diameter of the flat one,
# and the frequencies it drives them at.  What it does not state -- element
# size and layout -- is this module's choice: pistons covering half of the
# radiating surface, a golden-angle spiral for the 128-element cap, and each
# ring of an annular device as pistons sharing its radius (which steering on
# the axis drives alike).
DEVICES = {
    # name: (pistons, rings (0: independent elements), F in m (None: flat),
    #        aperture diameter in m, frequencies in Hz)
    "H317": (128, 0, 135e-3, 135e-3 / 0.9, (250e3, 700e3)),
    "CTX-500": (64, 4, 63.2e-3, 63.2e-3 / 0.98, (500e3,)),
    "H246": (24, 2, None, 33.6e-3, (500e3,)),
}


def device_array(name: str, apex) -> np.ndarray:
    """Element rows of one of the paper's devices with the centre of its
    radiating face (the bowl's apex) at ``apex``, axis +z: the geometric focus
    of a curved device is apex + (0, 0, F)."""
    n, rings, F, D, _ = DEVICES[name]
    a = np.asarray(apex, dtype=np.float64)
    R = 0.5 * D
    # piston centres within R - rp, so that every piston lies inside the aperture
    if F is None:
        area = math.pi * R * R
        rp = math.sqrt(0.5 * area / (n * math.pi))
        return flat_array(a, R - rp, n, rp, rings)
    area = 2 * math.pi * F * F * (1.0 - math.sqrt(1.0 - (R / F) ** 2))
    rp = math.sqrt(0.5 * area / (n * math.pi))
    return cap_array(a + np.array([0.0, 0.0, F]), F, R - rp, n, rp, rings)


def device_case(name: str, freq_hz: float, ppw: float = 6.0, seed: int = 1, skull: bool = True,
                lateral: float | None = None, depth: float | None = None,
                n_steps: int | None = None):
    """A head-scale domain for one of the paper's devices: lateral extent
    ``lateral`` (default: the aperture plus 10 mm), depth ``depth`` (default:
    F + 30 mm for a curved device, 80 mm for the flat one), the device on the
    middle column with its highest piston edge 3 mm before the source plane,
    and (skull) the skull
    shell of ``skull_case`` (outer radius 70 mm, outer surface 10 mm after the
    source plane on the axis).  The step count (default) covers 1.5 passes
    over the depth plus 4 periods.  Returns (case, element rows, geometric
    focus cell (i, j, k); the cell 60 mm deep on the axis for the flat
    device)."""
    n_el, rings, F, D, _ = DEVICES[name]
    dx = C_WATER / (freq_hz * ppw)
    lat = lateral if lateral is not None else D + 10e-3
    dep = depth if depth is not None else ((F + 30e-3) if F is not None else 80e-3)
    pml = 8
    nx = ny = int(math.ceil(lat / dx)) + 2 * pml
    nz = int(math.ceil(dep / dx)) + 2 * pml
    mats = skull_materials(freq_hz)
    zs = (pml + 0.5) * dx
    mat = (skull_map(nx, ny, nz, dx, zs, seed, r_out=70e-3, centre_depth=80e-3) if skull
           else np.zeros((nz, ny, nx), dtype=np.uint8))
    periods = math.ceil(1.5 * nz / ppw) + 4
    steps = n_steps if n_steps is not None else periods * math.ceil(3.9 * ppw)
    c = Case(f"{name}_{int(freq_hz / 1e3)}kHz", nx, ny, nz, pml, freq_hz, ppw, steps, mats, mat,
             None)
    rows = device_array(name, ((nx // 2) * dx, (ny // 2) * dx, 0.0))
    apex_z = zs - 3e-3 - float(np.max(rows[:, 3] + rows[:, 0]))
    rows[:, 3] += apex_z
    fz = apex_z + (F if F is not None else 60e-3)
    return c, rows, (nx // 2, ny // 2, int(round(fz / dx)))


def array_for_case(case: "Case", elements: int = 32, rings: int = 0):
    """A phased array for a case in place of its bowl: a cap of aperture 0.6 x
    the smaller lateral extent, F#1, rim 3 mm (plus 0.2 wavelengths) before the
    source plane, centred on the grid's middle column, with ``elements``
    pistons of radius 0.2 wavelengths.  Returns (element rows, target cell
    (i, j, k) of the geometric focus)."""
    dx, zs = case.dx, case.source_plane_z()
    aperture_r = 0.3 * min(case.nx, case.ny) * dx
    focal = 2.0 * aperture_r
    lam = C_WATER / case.freq_hz
    fz = bowl_focus_for_standoff(zs, aperture_r, focal, (0.0, 0.0, 1.0), 3e-3 + 0.2 * lam)
    focus = ((case.nx // 2) * dx, (case.ny // 2) * dx, fz)
    rows = cap_array(focus, focal, aperture_r, elements, 0.2 * lam, rings)
    return rows, (case.nx // 2, case.ny // 2, int(round(fz / dx)))


def array_case(seed: int, n: int = 64, rings: int = 0, elements: int = 32,
               freq_hz: float = 500e3, n_steps: int | None = None):
    """A 64^3-style skull patch (``surrogate_case`` map at ``freq_hz``) with a
    phased array in place of the bowl (``array_for_case``).  Returns (case,
    element rows, target cell (i, j, k))."""
    c = surrogate_case(seed, n, freq_hz=freq_hz)
    if n_steps is not None:
        c.n_steps = n_steps
    rows, cell = array_for_case(c, elements, rings)
    return c, rows, cell


def skull_map(nx: int, ny: int, nz: int, dx: float, zs: float, seed: int,
              r_out: float = 70e-3, centre_depth: float = 80e-3,
              axis_ij=None, chunk: int = 16, thick_scale: float = 1.0) -> np.ndarray:
    """uint8 [nz, ny, nx] skull-shell map (indices as ``skull_materials``);
    thickness 6.5 +- 1.5 mm times ``thick_scale``."""
    rng = np.random.default_rng(seed)
    ci, cj = (nx // 2, ny // 2) if axis_ij is None else axis_ij
    centre = np.array([ci * dx, cj * dx, zs + centre_depth])
    lo = (-dx, -dx, -dx)
    hi = (nx * dx, ny * dx, nz * dx)
    n_thick = _ValueNoise(rng, 10e-3, lo, hi)
    n_poro = _ValueNoise(rng, 4e-3, lo, hi)
    t_max = 8.0e-3 * thick_scale
    out = np.zeros((nz, ny, nx), dtype=np.uint8)
    xs = np.arange(nx) * dx
    ys = np.arange(ny) * dx
    for k0 in range(0, nz, chunk):
        k1 = min(nz, k0 + chunk)
        zz, yy, xx = np.meshgrid(np.arange(k0, k1) * dx, ys, xs, indexing="ij")
        rx, ry, rz = xx - centre[0], yy - centre[1], zz - centre[2]
        r = np.sqrt(rx * rx + ry * ry + rz * rz)
        cand = (r <= r_out) & (r >= r_out - t_max)
        if not cand.any():
            continue
        rc = r[cand]
        s = r_out / rc
        sx = centre[0] + rx[cand] * s
        sy = centre[1] + ry[cand] * s
        sz = centre[2] + rz[cand] * s
        thick = (6.5e-3 + 1.5e-3 * n_thick(sx, sy, sz)) * thick_scale
        depth = r_out - rc
        bone = depth <= thick
        cort = bone & ((depth < 0.1 * thick) | (depth > 0.9 * thick))
        trab = bone & ~cort
        phi = np.clip(0.4 + 0.2 * n_poro(xx[cand], yy[cand], zz[cand]), PORO_LO, PORO_HI)
        b = np.rint((phi - PORO_LO) / ((PORO_HI - PORO_LO) / (N_PORO_BINS - 1))).astype(np.int64)
        b = np.clip(b, 0, N_PORO_BINS - 1)
        idx = np.zeros(rc.shape, dtype=np.uint8)
        idx[cort] = 1
        idx[trab] = (2 + b[trab]).astype(np.uint8)
        sub = out[k0:k1]
        sub[cand] = idx
    return out


def skull_case(nx: int = 200, ny: int = 200, nz: int = 280, freq_hz: float = 500e3,
               ppw: float = 6.0, n_steps: int = 3000, seed: int = 1, pml: int = 8,
               aperture: float = 64e-3, fnum: float = 1.0, tilt=(0.0, 0.0),
               standoff: float = 3e-3, name: str = "skull", build_map: bool = True,
               surface_depth: float = 10e-3, thick_scale: float = 1.0) -> Case:
    """Skull-shell workload with a focused bowl (aperture = diameter); the
    shell's outer surface crosses the axis ``surface_depth`` after the source
    plane."""
    c = Case(name, nx, ny, nz, pml, freq_hz, ppw, n_steps, skull_materials(freq_hz), None, None)
    dx, zs = c.dx, c.source_plane_z()
    radius = 0.5 * aperture
    focal = fnum * aperture
    ci, cj = nx // 2, ny // 2
    _, ax = bowl_pose((0.0, 0.0, 0.0), tilt[0], tilt[1], focal)
    fz = bowl_focus_for_standoff(zs, radius, focal, ax, standoff)
    apex, ax = bowl_pose((ci * dx, cj * dx, fz), tilt[0], tilt[1], focal)
    c.transducer = Transducer(1, radius, focal, apex, ax)
    if build_map:
        c.mat = skull_map(nx, ny, nz, dx, zs, seed, centre_depth=surface_depth + 70e-3,
                          thick_scale=thick_scale)
    return c


def skull200(n_steps: int = 3000, build_map: bool = True) -> Case:
    """200x200x280 skull at 500 kHz, PPW 6 (seed 1)."""
    return skull_case(200, 200, 280, 500e3, 6.0, n_steps, seed=1,
                      name="skull200x200x280_500kHz", build_map=build_map)


def skull400(n_steps: int = 5000, build_map: bool = True) -> Case:
    """400x400x520 skull at 700 kHz, PPW 9 (seed 4)."""
    return skull_case(400, 400, 520, 700e3, 9.0, n_steps, seed=4,
                      name="skull400x400x520_700kHz", build_map=build_map)


# ---------------------------------------------------------- 12-bit CT maps

CT_LEVELS = 4096            # 12-bit CT values (Section 2.2.2)
CT_HU_MAX = 3000.0          # Hounsfield range quantised onto levels 1..4095
CT_HU_CORTICAL = 2400.0     # HU of non-porous bone in the synthetic mapping


def ct_materials(freq_hz: float) -> np.ndarray:
    """4096-row table for 12-bit CT maps: row 0 water (brain and skin as
    water), row l >= 1 the bone of HU = (l - 1) / 4094 * CT_HU_MAX, porosity
    phi = 1 - HU / CT_HU_CORTICAL clipped to [0, 1], mixing cortical bone and
    water linearly in density and longitudinal speed, shear speed scaled by
    (1 - phi), trabecular attenuation (the mapping functions of the paper's
    CT study are cited there, not printed; this linear porosity mapping stands
    in for them)."""
    t = table1(freq_hz)
    rho_c, cl_c, cs_c, _, _ = t["cortical"]
    _, _, _, al_t, as_t = t["trabecular"]
    rows = [t["water"]]
    for lvl in range(1, CT_LEVELS):
        hu = (lvl - 1) / (CT_LEVELS - 2) * CT_HU_MAX
        phi = min(1.0, max(0.0, 1.0 - hu / CT_HU_CORTICAL))
        cs = (1 - phi) * cs_c
        rows.append(((1 - phi) * rho_c + phi * RHO_WATER, (1 - phi) * cl_c + phi * C_WATER,
                     cs, al_t, as_t if cs > 0 else 0.0))
    return _rows(*rows)


def ct_levels(skull: np.ndarray, dx: float, seed: int) -> np.ndarray:
    """uint16 12-bit CT map of a skull-shell map (``skull_map`` indices): water
    stays 0; bone cells get the level of HU = CT_HU_CORTICAL (1 - phi), with
    porosity phi = 0.05 + 0.05 n in cortical cells and 0.4 + 0.2 n (clipped to
    [0.15, 0.65]) in trabecular ones, n seeded value noise on a 2 mm lattice."""
    rng = np.random.default_rng(seed + 7919)
    nz, ny, nx = skull.shape
    noise = _ValueNoise(rng, 2e-3, (-dx, -dx, -dx), (nx * dx, ny * dx, nz * dx))
    out = np.zeros(skull.shape, dtype=np.uint16)
    kk, jj, ii = np.nonzero(skull)
    n = noise(ii * dx, jj * dx, kk * dx)
    cort = skull[kk, jj, ii] == 1
    phi = np.where(cort, 0.05 + 0.05 * n, np.clip(0.4 + 0.2 * n, 0.15, 0.65))
    hu = CT_HU_CORTICAL * (1.0 - phi)
    lvl = 1 + np.rint(hu / CT_HU_MAX * (CT_LEVELS - 2)).astype(np.int64)
    out[kk, jj, ii] = np.clip(lvl, 1, CT_LEVELS - 1).astype(np.uint16)
    return out


def ct_case(base: "Case", seed: int = 0) -> "Case":
    """The 12-bit CT version of a skull-shell case: same grid, source and step
    count, the uint16 map of ``ct_levels`` and the 4096-row ``ct_materials``."""
    c = dataclasses.replace(base)
    c.name = base.name + "_ct12"
    c.materials = ct_materials(base.freq_hz)
    c.mat = ct_levels(base.mat, base.dx, seed)
    return c


BATCH_FREQS = (250e3, 500e3, 700e3)


def batch_cases(n: int = 32, lo: int = 96, hi: int = 160, build_map: bool = True,
                base_seed: int = 1000, steps_per_period: int = 23) -> list:
    """Uneven sweep: solve s draws its sizes and tilts from PCG64(base_seed+s),
    runs at BATCH_FREQS[s % 3], PPW 6, bowl aperture 0.6 x lateral extent,
    F#1, and lasts enough periods to cross 1.5x the depth plus two periods.
    ``steps_per_period`` only sizes the step count (the solver fixes its own)."""
    cases = []
    for s in range(n):
        rng = np.random.default_rng(base_seed + s)
        nx, ny, nz = (int(v) for v in rng.integers(lo, hi + 1, size=3))
        tx, ty = (float(v) for v in rng.uniform(-15.0, 15.0, size=2))
        f = BATCH_FREQS[s % 3]
        ppw = 6.0
        dx = C_WATER / (f * ppw)
        aperture = 0.6 * min(nx, ny) * dx
        periods = math.ceil(1.5 * nz / ppw) + 2
        c = skull_case(nx, ny, nz, f, ppw, periods * steps_per_period, seed=s, pml=8,
                       aperture=aperture, fnum=1.0,
                       tilt=(math.radians(tx), math.radians(ty)),
                       name=f"batch{s}", build_map=build_map)
        cases.append(c)
    return cases


def surrogate_case(seed: int, n: int = 64, build_map: bool = True, freq_hz: float | None = None) -> Case:
    """n^3 sample for the learned surrogate, batch-sweep style: frequency
    BATCH_FREQS[seed % 3], PPW 6, bowl tilts from PCG64(seed) in +-15 degrees,
    bowl aperture 0.6 x lateral extent, F#1, rim 3 mm before the source plane.
    The shell's outer surface crosses the axis 15 % of the interior depth after
    the source plane and its thickness is scaled to at most a quarter of that
    depth, so the focus lies beyond the skull at every frequency.  ``freq_hz``
    overrides the frequency (e.g. an out-of-distribution case)."""
    rng = np.random.default_rng(seed)
    tx, ty = (float(v) for v in rng.uniform(-15.0, 15.0, size=2))
    f = BATCH_FREQS[seed % 3] if freq_hz is None else float(freq_hz)
    ppw = 6.0
    dx = C_WATER / (f * ppw)
    pml = 8
    depth = (n - 2 * pml) * dx
    periods = math.ceil(1.5 * n / ppw) + 2
    return skull_case(n, n, n, f, ppw, periods * 23, seed=seed, pml=pml,
                      aperture=0.6 * n * dx, fnum=1.0,
                      tilt=(math.radians(tx), math.radians(ty)), name=f"sur{seed}",
                      build_map=build_map, surface_depth=0.15 * depth,
                      thick_scale=min(1.0, 0.25 * depth / 6.5e-3))


def random_small_case(seed: int, n=(24, 40), n_mat: int = 4, pml: int = 4,
                      n_steps: int = 80, freq_hz: float = 500e3) -> Case:
    """Random heterogeneous grid (sizes, blobs of random materials) for parity
    sweeps.  Materials: water plus ``n_mat - 1`` random solids/fluids."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = (int(v) for v in rng.integers(n[0], n[1] + 1, size=3))
    rows = [table1(freq_hz)["water"]]
    for m in range(1, n_mat):
        rho = rng.uniform(1000.0, 2000.0)
        cl = rng.uniform(1500.0, 3000.0)
        fluid = rng.uniform() < 0.25
        cs = 0.0 if fluid else rng.uniform(0.3, 0.6) * cl
        al = rng.uniform(0.0, 120.0)
        a_s = 0.0 if fluid else rng.uniform(0.0, 250.0)
        rows.append((rho, cl, cs, al, a_s))
    mats = _rows(*rows)
    mat = np.zeros((nz, ny, nx), dtype=np.uint8)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for _ in range(6):
        c = rng.uniform(0, 1, 3) * np.array([nx, ny, nz])
        r = rng.uniform(3, 10)
        m = int(rng.integers(0, n_mat))
        blob = (xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2 <= r * r
        mat[blob] = m
    c = Case(f"random{seed}", nx, ny, nz, pml, freq_hz, 6.0, n_steps, mats, mat, None)
    dx, zs = c.dx, c.source_plane_z()
    radius = 0.3 * min(nx, ny) * dx
    c.transducer = Transducer(1, radius, 2.0 * radius * 1.2,
                              ((nx // 2) * dx, (ny // 2) * dx, 0.0), (0.0, 0.0, 1.0))
    # place the bowl rim 2 mm before the source plane
    focal = c.transducer.focal
    fz = bowl_focus_for_standoff(zs, radius, focal, (0.0, 0.0, 1.0), 2e-3)
    c.transducer.apex = ((nx // 2) * dx, (ny // 2) * dx, fz - focal)
    return c
