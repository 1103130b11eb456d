"""Pins of the oracle's energy-loss factor E_L (Eq. 2) and pressure transmission
T_S = sqrt(E_L) (Section 3.2) against closed forms (no GPU).

E_L of a skull solve against its water-only companion is, behind a plate at
normal incidence, the plate's intensity transmission |T|^2 from the layer
formula; the plane sums weight p^2 by 1 / (2 rho c) of each cell's own
material, skip the absorbing layer, and take the plane of the water map's
peak voxel."""
import numpy as np
import pytest

import oracle
from oracle import energy
import synth
from tests import closed_forms as cf

WATER = synth.table1(250e3)["water"]
PLATE = synth.PLATE
PLATE_LOSSLESS = (1900.0, 2800.0, 1500.0, 0.0, 0.0)


def column_peaks(mats, col, n_steps, ppw=6.0, pml=8):
    """Peak maps of a laterally periodic column (plane wave along z) solved by
    the oracle, for the map col and for water only."""
    col = np.asarray(col, dtype=np.uint8)
    nz = len(col)
    out = []
    for m in (col, np.zeros(nz, dtype=np.uint8)):
        prob = oracle._Prob(1, 1, nz, pml, 250e3, ppw, n_steps, np.array(mats),
                            mode=oracle.LATERAL_PERIODIC)
        P, _, _ = oracle.solve(prob, m.reshape(nz, 1, 1), np.ones((1, 1), dtype=complex))
        out.append((P, m.reshape(nz, 1, 1)))
    info, consts = oracle.setup(prob)
    return out, info, consts


@pytest.mark.parametrize("ppw,tol", [(6, 0.08), (12, 0.015), (24, 0.004)])
def test_energy_loss_behind_lossless_plate_is_intensity_transmission(ppw, tol):
    """3 mm lossless bone plate between water: E_L on planes behind the plate
    equals |T|^2 = 4 / (4 cos^2(kd) + (Z2/Z1 + Z1/Z2)^2 sin^2(kd)); the error
    (staggered-interface error plus the peak's time sampling) falls about
    fourfold per doubling of PPW: measured 5-7 % at 6 PPW, 0.7-1.4 % at 12,
    0.2 % at 24."""
    s = ppw // 6
    nz = 400 * s
    col = np.zeros(nz)
    col[150 * s:153 * s] = 1
    mats = [WATER, PLATE_LOSSLESS]
    ((ps, ms), (pw, mw)), info, _ = column_peaks(mats, col, 1800 * s, ppw=ppw, pml=8 * s)
    rho, c = PLATE_LOSSLESS[0], PLATE_LOSSLESS[1]
    k2 = info["omega"] / c
    t = cf.layer_transmission(1.5e6, rho * c, k2, 3e-3)
    t2 = abs(t) ** 2
    assert abs(t2 - 0.2754) < 1e-4     # by hand: kd = 1.683 rad, Z2/Z1 = 3.547
    els = []
    for z in range(200 * s, 380 * s, 20 * s):
        e_l, t_s, zm = energy.energy_loss(ps, ms, pw, mw, np.array(mats), 0, z_m=z)
        assert zm == z and t_s == pytest.approx(np.sqrt(e_l))
        els.append(e_l)
    els = np.array(els)
    assert np.all(np.abs(els / t2 - 1) < tol), (els / t2 - 1)


def test_energy_loss_behind_lossy_plate_uses_zener_wavenumber():
    """The 64^3 plate workload's lossy bone (3 voxels): E_L = |T|^2 with the
    layer's complex Zener wavenumber and impedance at the drive frequency."""
    nz = 400
    col = np.zeros(nz)
    col[150:153] = 1
    mats = [WATER, PLATE]
    ((ps, ms), (pw, mw)), info, consts = column_peaks(mats, col, 1800)
    w0 = info["omega"]
    m = cf.sls_modulus(consts[1]["pi_r"], consts[1]["tau_p"], w0, w0)
    k2 = cf.continuum_k(PLATE[0], m, w0)
    t2 = abs(cf.layer_transmission(1.5e6, PLATE[0] * w0 / k2, k2, 3 * info["dx"])) ** 2
    assert abs(t2 - 0.4535 ** 2) < 1e-3
    e_l, t_s, _ = energy.energy_loss(ps, ms, pw, mw, np.array(mats), 0, z_m=300)
    assert abs(e_l / t2 - 1) < 0.1
    assert abs(t_s / np.sqrt(t2) - 1) < 0.05


def test_plane_sums_weight_by_each_cells_impedance_and_skip_the_layer():
    """Constructed maps: in plane z_m the skull solve has amplitude a in a
    second fluid (rho2, c2) on half of the cells and in water on the other
    half; the water solve has amplitude b.  Layer cells carry huge values that
    must not count.  E_L = (a^2/(rho2 c2) + a^2/(rho_w c_w)) / (2 b^2/(rho_w c_w))."""
    L, n, zm = 3, 14, 6
    mats = np.array([WATER, (1200.0, 1800.0, 0.0, 0.0, 0.0)])
    a, b = 2.5, 4.0
    ps = np.full((n, n, n), 1e9)
    pw = np.full((n, n, n), 1e9)
    ps[zm, L:n - L, L:n - L] = a
    pw[zm, L:n - L, L:n - L] = b
    ms = np.zeros((n, n, n), dtype=np.uint8)
    ms[zm, :, : n // 2] = 1
    mw = np.zeros_like(ms)
    inner = n - 2 * L
    n2 = inner * (n // 2 - L)          # interior cells of the second fluid
    n0 = inner * inner - n2
    zw = WATER[0] * WATER[1]
    z2 = mats[1, 0] * mats[1, 1]
    exact = (n2 * a * a / z2 + n0 * a * a / zw) / (inner * inner * b * b / zw)
    e_l, t_s, got_zm = energy.energy_loss(ps, ms, pw, mw, mats, L, z_m=zm)
    assert got_zm == zm
    assert e_l == pytest.approx(exact, rel=1e-14)
    assert t_s == pytest.approx(np.sqrt(exact), rel=1e-14)


def test_water_peak_plane_is_the_peak_voxels_plane_with_lowest_index_ties():
    """z_m is the plane of the water map's largest interior value; between
    equal maxima the lowest linear index (lowest plane) wins; layer cells never
    count."""
    L, n = 2, 10
    pw = np.zeros((n, n, n))
    pw[1, 5, 5] = 9.0                     # inside the layer: ignored
    pw[6, 4, 4] = 3.0
    pw[4, 7, 7] = 3.0                     # equal maximum, lower plane
    assert energy.water_peak_plane(pw, L) == 4
    pw[7, 3, 3] = 3.5
    assert energy.water_peak_plane(pw, L) == 7


def test_water_against_itself_gives_unit_transmission():
    """A solve compared with itself (the transcranial map is all water): E_L =
    T_S = 1 on the plane the oracle picks, here the focal plane of a bowl."""
    case = synth.random_small_case(7, n_steps=60)
    case.mat[:] = 0
    P, ridx, _ = oracle.solve_case(case)
    zm = energy.water_peak_plane(P, case.pml)
    assert zm == ridx // (case.nx * case.ny)
    e_l, t_s, z = energy.energy_loss(P, case.mat, P, case.mat, case.materials, case.pml)
    assert z == zm and e_l == 1.0 and t_s == 1.0
