"""Pins of the FP64 oracle against closed forms (no GPU).

Every check compares the oracle with something other than itself: textbook
dispersion, transmission and attenuation relations, exact polynomial
differentiation, discrete energy conservation, and O'Neil's on-axis field.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from tests import closed_forms as cf

WATER = synth.table1(250e3)["water"]
PLATE = synth.PLATE                                  # 64^3 plate workload bone
PLATE_LOSSLESS = (1900.0, 2800.0, 1500.0, 0.0, 0.0)


def run_1d(mats, col, n_steps, fields=("szz",), src=1.0 + 0j, mode=oracle.LATERAL_PERIODIC,
           freq=250e3, ppw=6.0, pml=8, source_k=-1, probe=None):
    """March a 1D column (nx = ny = 1, lateral derivatives vanish) and return the
    complex phasors (e^{+i w t}) of ``fields`` over the last period, plus info.
    ``probe`` (k index) additionally returns the pressure time series there."""
    col = np.asarray(col, dtype=np.uint8)
    nz = len(col)
    prob = oracle._Prob(1, 1, nz, pml, freq, ppw, n_steps, np.array(mats), mode=mode,
                        source_k=source_k)
    info, consts = oracle.setup(prob)
    sim = oracle.Sim(prob, col.reshape(nz, 1, 1))
    nt, w, dt = info["steps_per_period"], info["omega"], info["dt"]
    s = np.full((1, 1), src, dtype=complex)
    acc = {f: np.zeros(nz, dtype=complex) for f in fields}
    series = []
    for n in range(n_steps):
        sim.step(n, s)
        if probe is not None:
            series.append(-(sim.field("sxx")[probe, 0, 0] + sim.field("syy")[probe, 0, 0]
                            + sim.field("szz")[probe, 0, 0]) / 3.0)
        if n >= n_steps - nt:
            t = (n + 1) * dt
            for f in fields:
                acc[f] += sim.field(f)[:, 0, 0] * np.exp(-1j * w * t)
    out = {f: 2.0 * acc[f] / nt for f in fields}
    sim.close()
    return out, info, consts, np.array(series)


# ------------------------------------------------------------- operators

@pytest.mark.parametrize("deg", [1, 2, 3, 4])
def test_dplus_exact_on_polynomials(deg):
    """One velocity half-step from a polynomial sigma_xx gives v_x = dt/rho * D+ sigma_xx;
    D+ is exact for degree <= 4 away from the walls."""
    n = 24
    prob = oracle._Prob(n, 8, 8, 0, 250e3, 6.0, 1, np.array([WATER]))
    info, _ = oracle.setup(prob)
    sim = oracle.Sim(prob, np.zeros((8, 8, n), np.uint8))
    i = np.arange(n, dtype=float)
    coef = np.arange(1, deg + 2, dtype=float) * 0.37
    P = np.polynomial.Polynomial(coef)
    sim.field("sxx")[:] = P(i)[None, None, :]
    sim.step(0, None)
    d = sim.field("vx")[4, 4, :] * WATER[0] / info["dt"] * info["dx"]
    want = P.deriv()(i + 0.5)
    sl = slice(2, n - 3)
    assert np.max(np.abs(d[sl] - want[sl])) <= 1e-10 * np.max(np.abs(want[sl]))


def test_dplus_fifth_degree_error_term():
    """For f = i^5 the staggered operator's error is exactly -(3/640) f^(5) = -0.5625."""
    n = 24
    prob = oracle._Prob(n, 8, 8, 0, 250e3, 6.0, 1, np.array([WATER]))
    info, _ = oracle.setup(prob)
    sim = oracle.Sim(prob, np.zeros((8, 8, n), np.uint8))
    i = np.arange(n, dtype=float)
    sim.field("sxx")[:] = (i ** 5)[None, None, :]
    sim.step(0, None)
    d = sim.field("vx")[4, 4, :] * WATER[0] / info["dt"] * info["dx"]
    want = 5 * (i + 0.5) ** 4 - 0.5625
    sl = slice(2, n - 3)
    np.testing.assert_allclose(d[sl], want[sl], rtol=1e-11)


@pytest.mark.parametrize("deg", [2, 4])
def test_dminus_exact_on_polynomials(deg):
    """With sigma = 0 the velocity step leaves v_z alone and the stress step gives
    sigma_zz = dt * rho c^2 * D- v_z (water: no shear, no memory)."""
    n = 24
    prob = oracle._Prob(8, 8, n, 0, 250e3, 6.0, 1, np.array([WATER]))
    info, _ = oracle.setup(prob)
    sim = oracle.Sim(prob, np.zeros((n, 8, 8), np.uint8))
    k = np.arange(n, dtype=float)
    P = np.polynomial.Polynomial(np.linspace(0.3, 1.1, deg + 1))
    sim.field("vz")[:] = P(k)[:, None, None]     # stored at k + 1/2
    sim.step(0, None)
    d = sim.field("szz")[:, 4, 4] / (info["dt"] * WATER[0] * WATER[1] ** 2) * info["dx"]
    # D- evaluates at integer k from samples at k' + 1/2 = P(k'): derivative of P(s - 1/2)
    want = P.deriv()(k - 0.5)
    sl = slice(3, n - 2)
    assert np.max(np.abs(d[sl] - want[sl])) <= 1e-10 * np.max(np.abs(want[sl]))


# ------------------------------------------------------------- plane waves

def test_water_phase_speed_matches_discrete_dispersion():
    """Steady plane wave in water at the 64^3 plate workload's grid (dx 1 mm,
    27 steps/period): measured wavenumber equals the closed-form discrete root."""
    nz = 260
    ph, info, _, _ = run_1d([WATER, PLATE], np.zeros(nz), 1500)
    assert info["steps_per_period"] == 27
    A = ph["szz"]
    ks = np.arange(40, 220)
    phase = np.unwrap(np.angle(A[ks]))
    slope = np.polyfit(ks * info["dx"], phase, 1)[0]
    k_num = -slope
    k_cf = cf.discrete_k_lossless(info["omega"], 1500.0, info["dt"], info["dx"])
    assert abs(k_num / k_cf - 1) < 1e-4
    c_num = info["omega"] / k_cf
    assert abs(c_num - 1495.35) < 0.01        # -0.31 % numerical dispersion at 6 PPW
    # soft source: each outgoing wave carries |S| in the continuum limit; on the
    # lattice the residue at the propagating pole fixes it exactly (the 8-cell
    # layer behind the source adds an echo below 1e-3)
    amp = np.abs(A[ks])
    assert abs(amp.mean() - 1.0) < 0.03
    assert abs(amp.mean() / cf.soft_source_amplitude(k_cf, info["dx"]) - 1) < 1.5e-3


@pytest.mark.parametrize("ppw,tol", [(6, 0.03), (24, 1e-3)])
def test_water_to_solid_transmission(ppw, tol):
    """Normal incidence water -> lossless solid half-space: T = 2 Z2/(Z1 + Z2);
    the staggered interface error (-2.2 % at 6 PPW) vanishes with refinement."""
    s = ppw // 6
    nz, k_if = 400 * s, 150 * s
    col = np.zeros(nz)
    col[k_if:] = 1
    mats = [WATER, PLATE_LOSSLESS]
    ph, info, _, _ = run_1d(mats, col, 1800 * s, ppw=ppw, pml=8 * s)
    ref, _, _, _ = run_1d(mats, np.zeros(nz), 1800 * s, ppw=ppw, pml=8 * s)
    at = np.abs(ph["szz"][200 * s:380 * s]).mean()
    ai = np.abs(ref["szz"][200 * s:380 * s]).mean()
    z1, z2 = 1000.0 * 1500.0, PLATE_LOSSLESS[0] * PLATE_LOSSLESS[1]
    t_exact = 2 * z2 / (z1 + z2)
    assert abs(t_exact - 1.5601) < 1e-4
    assert abs(at / ai / t_exact - 1) < tol


def test_lossy_plate_layer_transmission():
    """3-voxel lossy bone plate (the 64^3 plate workload) between water: |T| from the
    layer formula with the Zener modulus at the drive frequency."""
    nz = 400
    col = np.zeros(nz)
    col[150:153] = 1
    mats = [WATER, PLATE]
    ph, info, consts, _ = run_1d(mats, col, 1800)
    ref, _, _, _ = run_1d(mats, np.zeros(nz), 1800)
    t_meas = np.abs(ph["szz"][200:380]).mean() / np.abs(ref["szz"][200:380]).mean()
    w0 = info["omega"]
    c = consts[1]
    m = cf.sls_modulus(c["pi_r"], c["tau_p"], w0, w0)
    k2 = cf.continuum_k(PLATE[0], m, w0)
    z2 = PLATE[0] * w0 / k2
    t_exact = abs(cf.layer_transmission(1.5e6, z2, k2, 3 * info["dx"]))
    assert abs(t_exact - 0.4535) < 5e-4
    assert abs(t_meas / t_exact - 1) < 0.05


def test_zener_constants_reproduce_q_and_phase_speed():
    """The relaxation strengths give Re M / Im M = q_c w/(2 c alpha) (Eq. 3) and a
    phase speed equal to the table speed at the drive frequency; the unrelaxed
    modulus is the w -> inf limit."""
    for qc in (1.0, 3.0):
        mats = synth.skull_materials(500e3)
        prob = oracle._Prob(32, 32, 32, 8, 500e3, 6.0, 10, mats, qc=qc)
        info, consts = oracle.setup(prob)
        w0 = info["omega"]
        for row, c in zip(mats, consts):
            rho, cl, cs, al, a_s = row
            for mod_r, tau, speed, alpha, mod_u, q in (
                    (c["pi_r"], c["tau_p"], cl, al, c["pi_u"], c["q_p"]),
                    (c["mu_r"], c["tau_s"], cs, a_s, c["mu_u"], c["q_s"])):
                if speed == 0:
                    assert mod_r == 0
                    continue
                m = cf.sls_modulus(mod_r, tau, w0, w0)
                if alpha > 0:
                    assert abs(m.real / m.imag / (qc * w0 / (2 * speed * alpha)) - 1) < 1e-12
                    assert abs(q / (qc * w0 / (2 * speed * alpha)) - 1) < 1e-12
                k = cf.continuum_k(rho, m, w0)
                assert abs(w0 / k.real / speed - 1) < 1e-12
                minf = cf.sls_modulus(mod_r, tau, 1e9 * w0, w0)
                assert abs(minf.real / mod_u - 1) < 1e-6


@pytest.mark.parametrize("wave", ["P", "S"])
def test_attenuation_decay_matches_zener_wavenumber(wave):
    """Steady 1D wave in the plate bone (Q_P 3.30, Q_S 1.87 at 250 kHz): the
    amplitude ratio between two depths is exp(-|Im k| dz), k from the Zener
    modulus: within 1 % (P) / 2.5 % (S, 6 points per shear wavelength) of the
    continuum value and within 1e-4 of the exact root of the discrete scheme
    (leapfrog, Crank-Nicolson memory variable, 4th-order staggered space)."""
    nz = 260
    if wave == "P":
        col = np.zeros(nz)
        col[60:] = 1
        ph, info, consts, _ = run_1d([WATER, PLATE], col, 1500, fields=("szz",))
        A = np.abs(ph["szz"])
        k1, k2 = 100, 130
        mod_r, tau = consts[1]["pi_r"], consts[1]["tau_p"]
        cont_target, cont_tol = 83.13, 0.01
    else:
        col = np.ones(nz)
        ph, info, consts, _ = run_1d([WATER, PLATE], col, 1500, fields=("sxz",),
                                     mode=oracle.LATERAL_PERIODIC | oracle.SOURCE_SHEAR_XZ)
        A = np.abs(ph["sxz"])
        k1, k2 = 20, 30        # deeper samples sit at 1e-6 of the incident amplitude
        mod_r, tau = consts[1]["mu_r"], consts[1]["tau_s"]
        cont_target, cont_tol = None, 0.025
    dx = info["dx"]
    meas = math.log(A[k1] / A[k2]) / ((k2 - k1) * dx)
    w0 = info["omega"]
    kc = cf.continuum_k(PLATE[0], cf.sls_modulus(mod_r, tau, w0, w0), w0)
    kd = cf.discrete_k_lossy(PLATE[0], mod_r, tau, w0, info["dt"], dx)
    if cont_target is not None:
        assert abs(-kc.imag - cont_target) < 0.01
    assert abs(meas / -kc.imag - 1) < cont_tol
    assert abs(meas / -kd.imag - 1) < 1e-4


def test_cpml_reflection_below_one_percent():
    """8-cell CPML: pressure at a probe in a short column minus the same probe in a
    4x longer column (whose far-wall echo has not arrived) stays below 1% of the
    incident amplitude."""
    short, long_ = 120, 480
    n = 1100
    _, _, _, ps = run_1d([WATER, PLATE], np.zeros(short), n, probe=60)
    _, _, _, pl = run_1d([WATER, PLATE], np.zeros(long_), n, probe=60)
    inc = np.abs(pl).max()
    assert abs(inc - 1.0) < 0.1          # ramp overshoot on top of ~1.03
    assert np.abs(ps - pl).max() < 1e-2 * inc


# ------------------------------------------------------------- energy

def _energy(sim, mats_const, rho_cells, mat, s_old):
    """E^{n+1/2} = 1/2 sum rho_v v^2 + 1/2 <sigma^n, C^-1 sigma^{n+1}> on the staggered grid."""
    nz, ny, nx = mat.shape
    rho = rho_cells[mat]
    def pad_rep(a, ax):
        idx = [slice(None)] * 3
        idx[ax] = slice(1, None)
        last = [slice(None)] * 3
        last[ax] = slice(-1, None)
        return np.concatenate([a[tuple(idx)], a[tuple(last)]], axis=ax)
    rv = [(rho + pad_rep(rho, ax)) / 2 for ax in (2, 1, 0)]
    ekin = 0.5 * sum((r * sim.field(v) ** 2).sum() for r, v in zip(rv, ("vx", "vy", "vz")))
    pi_ = np.array([c["pi_u"] for c in mats_const])[mat]
    mu_ = np.array([c["mu_u"] for c in mats_const])[mat]
    lam = pi_ - 2 * mu_
    s_new = {f: sim.field(f).copy() for f in ("sxx", "syy", "szz", "sxy", "sxz", "syz")}
    # normal block [[pi, l, l], [l, pi, l], [l, l, pi]] inverted per cell
    Cn = np.empty(mat.shape + (3, 3))
    for a in range(3):
        for b in range(3):
            Cn[..., a, b] = pi_ if a == b else lam
    Ci = np.linalg.inv(Cn)
    so = np.stack([s_old["sxx"], s_old["syy"], s_old["szz"]], -1)
    sn = np.stack([s_new["sxx"], s_new["syy"], s_new["szz"]], -1)
    epot = 0.5 * float((so * np.einsum("...ab,...b->...a", Ci, sn)).sum())
    inv_mu = 1.0 / mu_
    for f, (a1, a2) in (("sxy", (2, 1)), ("sxz", (2, 0)), ("syz", (1, 0))):
        q = inv_mu + pad_rep(inv_mu, a1) + pad_rep(inv_mu, a2) + pad_rep(pad_rep(inv_mu, a1), a2)
        mue = 4.0 / q
        epot += 0.5 * (s_old[f] * s_new[f] / mue).sum()
    return ekin + epot


def test_discrete_energy_conserved_without_loss_or_layer():
    """Heterogeneous all-solid medium, no attenuation, no absorbing layer, no source,
    rigid walls: the staggered leapfrog conserves E^{n+1/2} to round-off."""
    rng = np.random.default_rng(7)
    mats = np.array([(1900.0, 2800.0, 1500.0, 0.0, 0.0), (1500.0, 2200.0, 1000.0, 0.0, 0.0),
                     (1200.0, 1800.0, 600.0, 0.0, 0.0)])
    n = 14
    mat = rng.integers(0, 3, size=(n, n, n)).astype(np.uint8)
    prob = oracle._Prob(n, n, n, 0, 500e3, 6.0, 10, mats)
    info, consts = oracle.setup(prob)
    sim = oracle.Sim(prob, mat)
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    g = 1e5 * np.exp(-((x - 6.3) ** 2 + (y - 7.1) ** 2 + (z - 6.7) ** 2) / 4.0)
    for f in ("sxx", "syy", "szz"):
        sim.field(f)[:] = g
    sim.field("sxy")[:] = 0.3 * g
    E = []
    for step in range(2000):
        s_old = {f: sim.field(f).copy() for f in ("sxx", "syy", "szz", "sxy", "sxz", "syz")}
        sim.step(step, None)
        if step % 100 == 0 or step == 1999:
            E.append(_energy(sim, consts, mats[:, 0], mat, s_old))
    E = np.array(E)
    assert E[0] > 0
    assert np.max(np.abs(E / E[0] - 1)) < 1e-10


# ------------------------------------------------------------- Rayleigh

def test_element_areas_and_sizes():
    for t, area in ((synth.Transducer(1, 32e-3, 64e-3, (0, 0, 0), (0, 0, 1)), None),
                    (synth.Transducer(0, 15e-3, 0.0, (0, 0, 0), (0, 0, 1)), math.pi * 15e-3 ** 2)):
        for f in (250e3, 500e3, 700e3):
            el = oracle.elements(t, f)
            lam = 1500.0 / f
            if area is None:
                h = 64e-3 - math.sqrt(64e-3 ** 2 - 32e-3 ** 2)
                area = 2 * math.pi * 64e-3 * h
            assert abs(el[:, 3].sum() / area - 1) < 1e-12
            assert el[:, 3].max() <= lam * lam / 16 * (1 + 1e-12)
            if t.kind == 1:   # every element on the sphere of radius F about the focus
                r = np.linalg.norm(el[:, :3] - np.array([0, 0, 64e-3]), axis=1)
                np.testing.assert_allclose(r, 64e-3, rtol=1e-12)


def test_bowl_on_axis_matches_oneil():
    """Rayleigh sum on the axis of the 64 mm F#1 bowl at 500 kHz converges to
    O'Neil's closed form; focal gain k h = 17.96."""
    a, F, f = 32e-3, 64e-3, 500e3
    k = 2 * math.pi * f / 1500.0
    h = F - math.sqrt(F * F - a * a)
    assert abs(k * h - 17.96) < 0.005
    t = synth.Transducer(1, a, F, (0, 0, 0), (0, 0, 1))
    zs = np.array([20e-3, 45e-3, 55e-3, F, 70e-3, 90e-3])
    pts = np.stack([np.zeros_like(zs), np.zeros_like(zs), zs], -1)
    exact = np.array([cf.oneil_on_axis(z, a, F, k) for z in zs])
    errs = []
    for div in (16.0, 256.0, 1024.0):
        p = np.abs(oracle.rayleigh(oracle.elements(t, f, div), f, 1.0, pts))
        # every element is F from the focus: the focal value is exact at any size
        assert abs(p[3] / exact[3] - 1) < 1e-12
        errs.append(np.max(np.abs(p / exact - 1)))
    assert errs[0] < 3e-2                    # paper's lambda^2/16 elements (2.2 % at 20 mm)
    assert errs[2] < 5e-4
    assert errs[0] > errs[1] > errs[2]       # second order in the element width
    assert errs[1] / errs[2] > 3.0


def test_flat_piston_on_axis_and_far_field():
    from scipy.special import j1
    a, f = 15e-3, 250e3
    k = 2 * math.pi * f / 1500.0
    t = synth.Transducer(0, a, 0.0, (0, 0, 0), (0, 0, 1))
    el = oracle.elements(t, f, 1024.0)
    zs = np.array([10e-3, 30e-3, 60e-3, 120e-3])
    pts = np.stack([np.zeros_like(zs), np.zeros_like(zs), zs], -1)
    p = np.abs(oracle.rayleigh(el, f, 1.0, pts))
    exact = np.array([cf.oneil_on_axis(z, a, math.inf, k) for z in zs])
    np.testing.assert_allclose(p, exact, rtol=1e-3)
    # far field directivity 2 J1(ka sin th)/(ka sin th)
    r = 5.0
    th = np.radians([0.0, 3.0, 6.0, 9.0])
    pts = np.stack([r * np.sin(th), np.zeros_like(th), r * np.cos(th)], -1)
    p = np.abs(oracle.rayleigh(el, f, 1.0, pts))
    u = k * a * np.sin(th[1:])
    d = np.abs(2 * j1(u) / u)
    np.testing.assert_allclose(p[1:] / p[0], d, atol=2e-3)


def test_fdtd_on_axis_field_of_bowl_matches_oneil():
    """End to end in 3D water: Rayleigh plane + traction source + FDTD give the
    bowl's on-axis amplitude of O'Neil's closed form (within 5 % from 3 cells past
    the source plane; 2.5 % from 12 cells on, the rest is numerical dispersion)."""
    n, nz = 48, 96
    case = synth.skull_case(n, n, nz, 500e3, 6.0, 700, seed=0, aperture=16e-3, build_map=False)
    case.mat = np.zeros((nz, n, n), np.uint8)
    case.materials = case.materials[:1]
    P, _, _ = oracle.solve_case(case)
    t = case.transducer
    k = 2 * math.pi * case.freq_hz / 1500.0
    ks = case.pml
    errs = []
    for kk in range(ks + 3, nz - case.pml - 4):
        z = kk * case.dx - t.apex[2]
        errs.append((kk, P[kk, n // 2, n // 2] / cf.oneil_on_axis(z, t.radius, t.focal, k) - 1))
    errs = np.array(errs)
    assert np.max(np.abs(errs[:, 1])) < 0.05
    assert np.max(np.abs(errs[errs[:, 0] >= ks + 12, 1])) < 0.025


# ------------------------------------------------------------- setup / errors

def test_time_step_within_stability_and_integer_per_period():
    mats = synth.skull_materials(500e3)
    prob = oracle._Prob(40, 40, 40, 8, 500e3, 6.0, 10, mats)
    info, consts = oracle.setup(prob)
    T = 1 / 500e3
    assert abs(T / info["dt"] - info["steps_per_period"]) < 1e-9
    # von Neumann: the 3D symbol max of the staggered operator must keep w real
    th = np.linspace(0, math.pi, 2001)
    sym = np.abs(2 * (cf.C1 * np.sin(th / 2) + cf.C2 * np.sin(3 * th / 2)))
    cmax = max(math.sqrt(c["pi_u"] / r[0]) for c, r in zip(consts, mats))
    assert abs(cmax - info["c_max"]) < 1e-9
    courant = cmax * info["dt"] / info["dx"]
    assert courant * math.sqrt(3) * sym.max() / 2 <= 0.95 + 1e-9
    assert info["steps_per_period"] == 23


def _tiny(mats, **kw):
    return oracle._Prob(24, 24, 24, 4, 500e3, 6.0, 20, np.array(mats), **kw)


def test_rejects_bad_materials_and_sizes():
    with pytest.raises(oracle.OracleError) as e:
        oracle.setup(_tiny([WATER, (1900.0, 2000.0, 1800.0, 0.0, 0.0)]))   # nu = -1.63
    assert e.value.code == oracle.EMATERIAL
    with pytest.raises(oracle.OracleError) as e:
        oracle.setup(_tiny([WATER, (1900.0, 2800.0, 1500.0, 2000.0, 0.0)]))  # Q_P <= 1
    assert e.value.code == oracle.EMATERIAL
    with pytest.raises(oracle.OracleError) as e:
        oracle.setup(_tiny([WATER, (-1.0, 2800.0, 0.0, 0.0, 0.0)]))
    assert e.value.code == oracle.EMATERIAL
    with pytest.raises(oracle.OracleError) as e:
        oracle.setup(oracle._Prob(8, 24, 24, 4, 500e3, 6.0, 20, np.array([WATER])))
    assert e.value.code == oracle.EINVAL
    with pytest.raises(oracle.OracleError) as e:
        oracle.setup(_tiny([WATER], source_k=2))
    assert e.value.code == oracle.EGEOMETRY
    # nu exactly 0.5 is a fluid and accepted only with c_s = 0
    oracle.setup(_tiny([WATER, (1041.0, 1562.0, 0.0, 3.45, 0.0)]))


def test_index_out_of_range_and_divergence():
    mat = np.zeros((24, 24, 24), np.uint8)
    mat[5, 5, 5] = 2
    with pytest.raises(oracle.OracleError) as e:
        oracle.Sim(_tiny([WATER, PLATE]), mat)
    assert e.value.code == oracle.EINDEX
    mat[5, 5, 5] = 1
    src = np.ones((24, 24), complex)
    oracle.solve(_tiny([WATER, PLATE]), mat, src)
    mat[10:] = 1   # a bone slab, whose Courant number is 1.5x the 3D limit here
    with pytest.raises(oracle.OracleError) as e:
        oracle.solve(oracle._Prob(24, 24, 24, 4, 500e3, 6.0, 400, np.array([WATER, PLATE]),
                                  cfl_safety=1.6), mat, src)
    assert e.value.code == oracle.EDIVERGED


def test_solve_is_linear_in_the_source():
    case = synth.random_small_case(3, n_steps=60)
    prob = oracle.problem_from_case(case)
    src = oracle.source_plane(case)
    p1, i1, _ = oracle.solve(prob, case.mat, src)
    p2, i2, _ = oracle.solve(prob, case.mat, 2.0 * src)
    np.testing.assert_allclose(p2, 2.0 * p1, rtol=1e-13, atol=0)
    assert i1 == i2


def _mirror_case():
    """A lossy, heterogeneous grid whose materials and source plane are both
    symmetric under the x reflection about cell 0 of a laterally periodic grid,
    i -> (nx - i) mod nx (which maps cells to cells and v_x faces to faces):
    a solid block, a lossy fluid and a bone sliver, random source values."""
    nx, ny, nz, L = 30, 22, 28, 4
    mats = synth._rows(synth.table1(500e3)["water"], (1850.0, 2700.0, 1300.0, 80.0, 200.0),
                       (1050.0, 1560.0, 0.0, 30.0, 0.0))
    mat = np.zeros((nz, ny, nx), dtype=np.uint8)
    mat[12:17, 5:13, 0:7] = 1
    mat[18:22, 8:18, 9:13] = 2
    case = synth.Case("mirror", nx, ny, nz, L, 500e3, 6.0, 70, mats, mat, None)
    rng = np.random.default_rng(11)
    src = rng.normal(size=(ny, nx)) + 1j * rng.normal(size=(ny, nx))
    m = (-np.arange(nx)) % nx
    upper = np.arange(nx) > nx // 2
    mat[:, :, upper] = mat[:, :, m[upper]]
    src[:, upper] = src[:, m[upper]]
    return case, src, m


def test_solve_is_mirror_symmetric_in_x():
    """The staggered x operators are antisymmetric under the reflection (v_x
    faces map to faces, with a sign), so with laterally periodic boundaries
    symmetric materials and source give a symmetric peak map: exactly, up to
    the order of additions.  A transposed or shifted x stencil breaks it."""
    case, src, m = _mirror_case()
    assert np.array_equal(case.mat, case.mat[:, :, m]) and np.array_equal(src, src[:, m])
    prob = oracle.problem_from_case(case, mode=oracle.LATERAL_PERIODIC)
    p, _, _ = oracle.solve(prob, case.mat, src)
    assert p.max() > 0
    np.testing.assert_allclose(p, p[:, :, m], rtol=1e-12, atol=1e-12 * p.max())
    # the same check fails for a source that is not symmetric
    p2, _, _ = oracle.solve(prob, case.mat, src * np.linspace(1.0, 1.5, case.nx)[None, :])
    assert np.abs(p2 - p2[:, :, m]).max() > 1e-3 * p2.max()


# ------------------------------------------------------------- x/y absorbing layers

# Component relabelling under a swap of two axes: (velocities, normal stresses,
# shear stresses and their memory variables follow the axes they carry).
_SWAP = {
    "xz": ((2, 1, 0), {"vx": "vz", "vz": "vx", "sxx": "szz", "szz": "sxx", "sxy": "syz",
                       "syz": "sxy", "rxx": "rzz", "rzz": "rxx", "rxy": "ryz", "ryz": "rxy"}),
    "yz": ((1, 0, 2), {"vy": "vz", "vz": "vy", "syy": "szz", "szz": "syy", "sxy": "sxz",
                       "sxz": "sxy", "ryy": "rzz", "rzz": "ryy", "rxy": "rxz", "rxz": "rxy"}),
}
_BONE_T = (1850.0, 2700.0, 1300.0, 80.0, 200.0)
_LOSSY_FLUID = (1050.0, 1560.0, 0.0, 30.0, 0.0)


def _pulse_run(mat, pml, steps, centre, shear, materials, fields=None, probes=None):
    """Free evolution (no source) of a Gaussian stress pulse: isotropic normal
    stresses plus a shear component ``shear``; returns the final fields, and
    the pressure time series at ``probes`` ((i, j, k) cells) if given."""
    nz, ny, nx = mat.shape
    prob = oracle._Prob(nx, ny, nz, pml, 500e3, 6.0, steps, np.array(materials))
    sim = oracle.Sim(prob, mat)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    g = 1e5 * np.exp(-((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2) / 3.0)
    for f in ("sxx", "syy", "szz"):
        sim.field(f)[:] = g
    sim.field(shear)[:] += 0.3 * g
    series = []
    for n in range(steps):
        sim.step(n, None)
        if probes:
            p = -(sim.field("sxx") + sim.field("syy") + sim.field("szz")) / 3.0
            series.append([p[k, j, i] for (i, j, k) in probes])
    out = {f: sim.field(f).copy() for f in (fields or ())}
    sim.close()
    return out, np.array(series)


@pytest.mark.parametrize("swap", ["xz", "yz"])
def test_xy_layers_are_the_z_layer_with_axes_swapped(swap):
    """The scheme treats the three axes alike, so swapping x (or y) with z in
    the material map and the initial state must swap every field exactly (up
    to the order of additions): a lossy heterogeneous cube whose pulse runs
    into the z layer near a bone slab crossing it, against the same cube with
    the axes swapped, whose pulse then runs into the x (or y) layer.  Every
    x/y absorbing-layer term (which staggered coordinate sets its depth, its
    memory, its side) is thereby tied to the z layer's, which the 1D
    reflection pin measures.  A half-cell slip of one x or y derivative's
    layer coordinate makes fields differ by ~1e-2 of their scale."""
    n, pml, steps = 32, 6, 240
    mats = [WATER, _BONE_T, _LOSSY_FLUID]
    mat = np.zeros((n, n, n), np.uint8)
    mat[:, :, 12:20] = 1               # slab crossing the z layer at both ends
    mat[20:31, 4:14, 22:30] = 2
    mat[25:32, 18:26, 3:9] = 1
    names = oracle.FIELDS
    c = np.array([15.3, 14.2, n - pml - 5.6])          # pulse near the high z layer
    a, _ = _pulse_run(mat, pml, steps, c, "sxy", mats, fields=names)
    axes, rel = _SWAP[swap]
    cb = c[[2, 1, 0]] if swap == "xz" else c[[0, 2, 1]]
    b, _ = _pulse_run(np.ascontiguousarray(mat.transpose(axes)), pml, steps, cb, rel["sxy"],
                      mats, fields=names)
    assert np.abs(a["peak"]).max() > 0
    for f in names:
        want = a[rel.get(f, f)].transpose(axes)
        scale = np.abs(want).max()
        assert scale > 0, f
        assert np.abs(b[f] - want).max() <= 1e-12 * scale, (swap, f)


@pytest.mark.parametrize("axis", ["x", "y"])
@pytest.mark.parametrize("medium", ["water", "bone_slab"])
def test_cpml_oblique_reflection_from_x_and_y_faces(axis, medium):
    """A pressure pulse 8 cells from the high x (or y) layer: pressure at three
    probes 3 cells from the layer (on the pulse's line and 6 cells to either
    side, so the echo reaching them left the face obliquely) against the same
    probes in a grid 4x wider along that axis, whose far layer is too far to
    echo back within the run.  The difference, the layer's reflection, stays
    below 1 % of the incident amplitude, in water and inside a lossy bone slab
    that runs through the layer (P and S waves at grazing incidence)."""
    n, pml, steps = 40, 8, 300
    mats = [WATER, _BONE_T]
    ax = 0 if axis == "x" else 1
    centre = [n // 2, n // 2, n // 2]
    centre[ax] = n - pml - 8
    probes = []
    for d in (-6, 0, 6):
        p = [n // 2, n // 2, n // 2]
        p[ax] = n - pml - 3
        p[1 - ax] += d
        probes.append(tuple(p))

    def grid(width):
        shape = [n, n, n]
        shape[2 - ax] = width
        mat = np.zeros(shape, np.uint8)
        if medium == "bone_slab":
            mat[14:26] = 1
        return mat

    _, short = _pulse_run(grid(n), pml, steps, centre, "sxy", mats, probes=probes)
    _, wide = _pulse_run(grid(4 * n), pml, steps, centre, "sxy", mats, probes=probes)
    inc = np.abs(wide).max(axis=0)
    assert (inc > 0).all()
    refl = np.abs(short - wide).max(axis=0) / inc
    assert (refl < 1e-2).all(), refl
    assert (refl > 1e-6).all()            # the short grid's layer is within reach


# ------------------------------------------------------------- peak voxel ties

def test_peak_voxel_ties_go_to_the_lowest_linear_index():
    """Two exact ties.  (1) With a zero source the peak map is zero everywhere,
    and the peak voxel is the first interior cell (L, L, L).  (2) Laterally
    periodic, uniform source over a water/plate column: every cell of a plane
    evolves by the same operations on the same values, so each plane of the map
    is one value repeated bit for bit; the peak voxel is the first cell (0, 0)
    of the peak plane, not any other of its nx*ny equal cells."""
    case = synth.random_small_case(7, n_steps=20)
    prob = oracle.problem_from_case(case)
    zero = np.zeros((case.ny, case.nx), complex)
    p, idx, _ = oracle.solve(prob, case.mat, zero)
    L = case.pml
    assert p.max() == 0.0
    assert idx == (L * case.ny + L) * case.nx + L
    nx, ny, nz = 5, 4, 90
    col = np.zeros(nz, np.uint8)
    col[40:43] = 1
    mat = np.ascontiguousarray(np.broadcast_to(col[:, None, None], (nz, ny, nx)))
    prob = oracle._Prob(nx, ny, nz, 8, 250e3, 6.0, 500, np.array([WATER, PLATE]),
                        mode=oracle.LATERAL_PERIODIC)
    p, idx, _ = oracle.solve(prob, mat, np.full((ny, nx), 1.0 + 0.5j))
    k = int(np.argmax(p[8:nz - 8, 0, 0])) + 8
    assert p.max() > 0 and (p == p[:, :1, :1]).all()
    assert idx == k * ny * nx
