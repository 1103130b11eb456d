"""Energy-loss factor and pressure transmission of a transcranial solve, FP64.

TEST INFRASTRUCTURE ONLY (part of the oracle): only the test suite, the smoke
entry and the benchmark's CPU-baseline leg may import it.  Plain numpy; it
imports nothing from the product package.

Paper, Section 2.4 (thermal modelling step), Eq. 2: the energy loss E_L is the
ratio of the pulse-average intensity summed over one x-y plane in the
transcranial (skull) solve to the same sum in the water-only solve, taken on
the plane z_m where the water-only field has its maximal intensity.  Section
3.2 defines the pressure transmission coefficient T_S = sqrt(E_L).

Readings (the paper is silent on them):
  * I_PA of a cell is p^2 / (2 rho c) with p the peak-pressure amplitude of
    the solve there and rho, c the density and longitudinal speed of the
    cell's material (of that solve's own map);
  * the sums run over the plane's cells outside the absorbing layer;
  * z_m is the z index of the water-only map's peak voxel over the interior
    outside the layer (the solver's own peak voxel, ties to the lowest linear
    index), unless the caller names the plane.
"""
from __future__ import annotations

import numpy as np


def water_peak_plane(p_water: np.ndarray, pml: int) -> int:
    """z index of the largest value of the water-only peak map over the
    interior outside the layer; ties go to the lowest linear index."""
    p = np.asarray(p_water, dtype=np.float64)
    nz, ny, nx = p.shape
    L = pml
    best, best_idx = -1.0, -1
    for k in range(L, nz - L):
        sub = p[k, L:ny - L, L:nx - L]
        j, i = np.unravel_index(int(np.argmax(sub)), sub.shape)   # first maximum in x-fastest order
        v = float(sub[j, i])
        if v > best:                                              # strictly larger: earlier planes win ties
            best, best_idx = v, k
    return best_idx


def plane_intensity_sum(p: np.ndarray, mat: np.ndarray, materials: np.ndarray, k: int,
                        pml: int) -> float:
    """Sum over the plane k (cells outside the layer) of p^2 / (2 rho c)."""
    p = np.asarray(p, dtype=np.float64)
    nz, ny, nx = p.shape
    L = pml
    tab = np.asarray(materials, dtype=np.float64).reshape(-1, 5)
    m = np.asarray(mat)[k, L:ny - L, L:nx - L].astype(np.int64)
    rho, c = tab[m, 0], tab[m, 1]
    a = p[k, L:ny - L, L:nx - L]
    return float(np.sum(a * a / (2.0 * rho * c)))


def energy_loss(p_skull, mat_skull, p_water, mat_water, materials, pml: int,
                z_m: int | None = None):
    """(E_L, T_S, z_m) of a skull solve against its water-only companion."""
    if z_m is None or z_m < 0:
        z_m = water_peak_plane(p_water, pml)
    num = plane_intensity_sum(p_skull, mat_skull, materials, z_m, pml)
    den = plane_intensity_sum(p_water, mat_water, materials, z_m, pml)
    e_l = num / den
    return e_l, float(np.sqrt(e_l)), int(z_m)
