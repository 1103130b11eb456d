"""Pins of the oracle's BHTE thermal step (Section 2.4) against closed forms
(no GPU): the discrete Laplacian on a separable eigenfunction with the border
held fixed, perfusion decay, flux continuity across a conductivity jump (the
harmonic-mean faces), the CEM43 dose of a constant temperature, and the heat
source formula with the 0.16 heating share in bone."""
import math

import numpy as np
import pytest

from oracle import bhte

WATERLIKE = (1000.0, 1500.0, 0.0, 0.0, 0.0)


def uniform(n, k=0.5, c=3600.0, w=0.0, rho=1040.0, alpha=10.0):
    acoustic = np.array([(rho, 1560.0, 0.0, alpha, 0.0)])
    thermal = np.array([(k, c, w)])
    return np.zeros(n, dtype=np.uint8), acoustic, thermal


@pytest.mark.parametrize("shape", [(9, 12, 15), (20, 7, 11)])
def test_one_step_on_discrete_eigenfunction(shape):
    """T - T_a = A sin(pi i/(nx-1)) sin(pi j/(ny-1)) sin(pi k/(nz-1)) vanishes on
    the border and is an eigenfunction of the 7-point Laplacian with
    eigenvalue -sum_a (2 - 2 cos(pi/(n_a - 1))) / dx^2: one explicit step
    multiplies it by 1 - dt k lambda / (rho C), to rounding."""
    nz, ny, nx = shape
    mat, ac, th = uniform(shape)
    dx = 5e-4
    dt = 0.5 * bhte.stable_dt(mat, ac, th, dx)
    s = bhte.BHTE(mat, ac, th, dx, dt)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phi = (np.sin(np.pi * i / (nx - 1)) * np.sin(np.pi * j / (ny - 1))
           * np.sin(np.pi * k / (nz - 1)))
    s.T = 37.0 + 4.0 * phi
    s.T[0], s.T[-1], s.T[:, 0], s.T[:, -1], s.T[:, :, 0], s.T[:, :, -1] = (37.0,) * 6
    lam = sum((2 - 2 * math.cos(math.pi / (m - 1))) / dx ** 2 for m in shape)
    factor = 1.0 - dt * th[0, 0] * lam / (ac[0, 0] * th[0, 1])
    s.step(np.zeros(shape))
    np.testing.assert_allclose(s.T - 37.0, factor * 4.0 * phi, atol=1e-12, rtol=0)
    assert np.all(s.T[0] == 37.0) and np.all(s.T[:, :, -1] == 37.0)


def test_perfusion_decay_without_conduction():
    """k = 0: every interior cell relaxes on its own, T - T_a shrinking by
    1 - dt w rho_b C_b / (rho C) per step, which tends to exp(-w rho_b C_b t/(rho C))."""
    shape = (6, 6, 6)
    mat, ac, th = uniform(shape, k=0.0, w=0.01)
    dt = 0.05
    s = bhte.BHTE(mat, ac, th, 1e-3, dt)
    s.T[1:-1, 1:-1, 1:-1] = 42.0
    n = 400
    for _ in range(n):
        s.step(np.zeros(shape))
    g = th[0, 2] * bhte.RHO_C_BLOOD / (ac[0, 0] * th[0, 1])
    exact_discrete = 5.0 * (1 - dt * g) ** n
    assert s.T[3, 3, 3] - 37.0 == pytest.approx(exact_discrete, rel=1e-12)
    assert s.T[3, 3, 3] - 37.0 == pytest.approx(5.0 * math.exp(-g * n * dt), rel=2e-3)
    assert s.t_max[3, 3, 3] == 42.0 - 5.0 * dt * g   # the first step's end


def test_flux_continuity_across_a_conductivity_jump():
    """Two materials stacked in z (k1 = 0.5, k2 = 2.0): a z profile whose steps
    carry the same flux F through every face (F/k1 inside material 1, F/k_f
    across the interface with k_f = 2 k1 k2/(k1 + k2), F/k2 inside material 2)
    is steady: one step leaves every cell unchanged that no border touches."""
    nz, ny, nx = 16, 7, 7
    mat = np.zeros((nz, ny, nx), dtype=np.uint8)
    mat[8:] = 1
    ac = np.array([(1040.0, 1560.0, 0.0, 0.0, 0.0), (1900.0, 2800.0, 0.0, 0.0, 0.0)])
    th = np.array([(0.5, 3600.0, 0.0), (2.0, 1300.0, 0.0)])
    k1, k2 = 0.5, 2.0
    kf = 2 * k1 * k2 / (k1 + k2)
    F = 0.3
    prof = [37.0]
    for k in range(1, nz):
        kk = k1 if k < 8 else (kf if k == 8 else k2)
        prof.append(prof[-1] + F / kk)
    s = bhte.BHTE(mat, ac, th, 1e-3, 0.01)
    s.T = np.broadcast_to(np.array(prof)[:, None, None], (nz, ny, nx)).copy()
    before = s.T.copy()
    s.step(np.zeros(mat.shape))
    inner = (slice(1, nz - 2), slice(2, ny - 2), slice(2, nx - 2))
    np.testing.assert_allclose(s.T[inner], before[inner], rtol=0, atol=1e-12)
    # with the arithmetic mean on the interface face instead, the cells beside it move
    assert abs(kf - 0.5 * (k1 + k2)) > 0.4


@pytest.mark.parametrize("temp,expect", [(45.0, 4.0), (41.0, 0.0625), (43.0, 1.0)])
def test_cem43_dose_of_a_constant_temperature(temp, expect):
    """Sixty seconds at constant T: CEM43 = 1 min x R^(43 - T) with R = 0.5 at or
    above 43 degC and 0.25 below (4 min at 45 degC, 1/16 min at 41)."""
    shape = (5, 5, 5)
    mat, ac, th = uniform(shape, k=0.0)
    s = bhte.BHTE(mat, ac, th, 1e-3, 0.25, t_body=temp)
    for _ in range(240):
        s.step(np.zeros(shape))
    np.testing.assert_allclose(s.dose, expect, rtol=1e-12)


def test_heat_source_formula_with_bone_heating_share():
    """Q = scale * 2 h alpha_l p^2 / (2 rho c_l): h = 1 in soft tissue, 0.16 in
    bone (the paper's share of bone attenuation turned into heat), none in
    lossless water."""
    acoustic = np.array([WATERLIKE, (1041.0, 1562.0, 0.0, 6.9 * 0.5, 0.0),
                         (1896.5, 2475.0, 1539.0, 81.5, 164.5)])
    h = np.array([1.0, 1.0, 0.16])
    mat = np.array([[[0, 1, 2]]], dtype=np.uint8)
    p = np.array([[[2e5, 3e5, 4e5]]])
    q = bhte.heat_source(mat, p, acoustic, h, scale=2.0)
    assert q[0, 0, 0] == 0.0
    assert q[0, 0, 1] == pytest.approx(2.0 * 2 * 3.45 * (3e5) ** 2 / (2 * 1041.0 * 1562.0), rel=1e-14)
    assert q[0, 0, 2] == pytest.approx(2.0 * 2 * 0.16 * 81.5 * (4e5) ** 2 / (2 * 1896.5 * 2475.0),
                                       rel=1e-14)


def test_sonication_regime_heats_then_cools():
    """A uniform source switched on for n_on steps at duty cycle D, then off:
    the centre warms while on (at first by D Q dt / (rho C) per step) and cools
    once off; the maximum is reached at the end of the on period."""
    shape = (11, 11, 11)
    mat, ac, th = uniform(shape, k=0.5, w=0.005)
    dx, dt = 1e-3, 0.1
    q = np.full(shape, 2e5)
    s = bhte.BHTE(mat, ac, th, dx, dt)
    s.step(0.5 * q)
    assert s.T[5, 5, 5] - 37.0 == pytest.approx(0.5 * 2e5 * dt / (ac[0, 0] * th[0, 1]), rel=1e-12)
    s = bhte.BHTE(mat, ac, th, dx, dt)
    T, t_max, dose = s.run(q, 100, 100, 0.5)
    centre_peak = t_max[5, 5, 5]
    assert T[5, 5, 5] < centre_peak
    s2 = bhte.BHTE(mat, ac, th, dx, dt)
    s2.run(q, 100, 0, 0.5)
    assert s2.T[5, 5, 5] == centre_peak
    assert np.all(dose > 0)
