"""Pins of the oracle's phased-array pieces (Section 2, 2.3) against closed
forms and the oracle's own pinned single transducers (no GPU): a one-piston
array is the flat piston, drives act linearly, steering puts every element's
wave in phase at the target, and refocusing by time reversal through water
reproduces the geometric steering phases."""
import numpy as np
import pytest

import oracle
from oracle import array
import synth


def test_one_element_array_is_the_flat_piston_and_drives_are_linear():
    case = synth.plate_case()
    t = case.transducer
    row = np.array([[t.radius, *t.apex, *t.axis, 1.0, 0.0]])
    a = array.source_plane(case, row)
    b = oracle.source_plane(case)
    assert np.allclose(a, b, rtol=0, atol=1e-12 * np.abs(b).max())
    w = 0.3 - 1.7j
    assert np.allclose(array.source_plane(case, row, [w]), w * b, rtol=0,
                       atol=1e-12 * np.abs(b).max())


@pytest.mark.parametrize("rings", [0, 4])
def test_steered_waves_arrive_in_phase_at_the_target(rings):
    """With w_e = exp(+i k |c_e - T|) every element's contribution at the
    target has the phase of i (the Rayleigh kernel's i e^{-ikR} at the centre
    distance): |p(T)| is within 1 % of the sum of the element amplitudes, and
    steering 4 mm off axis moves the field's maximum there."""
    case, rows, cell = synth.array_case(20001, rings=rings)
    f = case.freq_hz
    T = np.array(cell) * case.dx
    w = array.steer(rows, T, f)
    each = np.array([array.field(rows[e:e + 1], f, T[None, :])[0] for e in range(len(rows))])
    p = np.sum(w * each)
    assert abs(p) >= 0.99 * np.sum(np.abs(each))
    T2 = T + np.array([4e-3, 0.0, 0.0])
    w2 = array.steer(rows, T2, f)
    xs = T2[0] + np.linspace(-6e-3, 6e-3, 49)
    line = np.stack([xs, np.full_like(xs, T2[1]), np.full_like(xs, T2[2])], axis=1)
    amp = np.abs(array.field(rows, f, line, w2))
    assert abs(xs[np.argmax(amp)] - T2[0]) <= 0.5e-3


def test_time_reversal_through_water_reproduces_geometric_steering():
    """Refocusing drives from a point source at the target, recorded on the
    source plane by the FDTD oracle in water and carried back to the elements
    by the Rayleigh integral, equal the steering drives up to one global phase
    (residual below 0.1 rad RMS: discretisation, the radiation pattern of the
    point source and the finite plane)."""
    case, rows, cell = synth.array_case(20001, n_steps=330)
    case.mat[:] = 0
    w_tr, p = array.refocus(case, rows, cell)
    w_geo = array.steer(rows, np.array(cell) * case.dx, case.freq_hz)
    d = np.angle(w_tr * np.conj(w_geo))
    g = np.angle(np.mean(np.exp(1j * d)))
    res = np.angle(np.exp(1j * (d - g)))
    assert np.sqrt(np.mean(res ** 2)) < 0.1, res
    assert np.all(np.abs(p) > 0)


def _axis_pressure_phasors(case, i, j, faces, cells):
    """Phasors of sigma_xx at cells (i, j, kc), kc in cells, over the last
    period of the oracle's solve in water driven by z forces on the v_z faces
    above cells kf (faces: kf -> force) -- the point-source mechanism of
    refocusing."""
    from oracle import Sim, problem_from_case, setup
    out = np.zeros(len(cells), dtype=np.complex128)
    for kf, force in faces.items():
        prob = problem_from_case(case, source_k=kf)
        info, _ = setup(prob)
        nt, w, dt = info["steps_per_period"], info["omega"], info["dt"]
        src = np.zeros((case.ny, case.nx), dtype=np.complex128)
        src[j, i] = force
        sim = Sim(prob, case.mat)
        for n in range(case.n_steps):
            sim.step(n, src)
            if n >= case.n_steps - nt:
                s = sim.field("sxx")
                e = np.exp(-1j * w * (n + 1) * dt)
                out += 2.0 / nt * e * np.array([s[kc, j, i] for kc in cells])
        sim.close()
    return out


def test_point_source_pair_radiates_like_a_monopole_along_the_axis():
    """The refocusing point source (outward z forces on both v_z faces of the
    target cell k) radiates the same pressure phasor to the cells d planes
    above and below it (equal amplitude within 5 %, phase within 0.1 rad), as a
    monopole does, while one z force alone (on the face above cell k) radiates
    to the cells symmetric about that face in opposite phase, as a dipole does:
    the reading that makes the record the transfer to pressure."""
    case = synth.random_small_case(7, n=(40, 40), n_steps=260)
    case.nx = case.ny = case.nz = 40
    case.mat = np.zeros((40, 40, 40), dtype=np.uint8)
    i = j = 20
    k, d = 20, 6
    pair = _axis_pressure_phasors(case, i, j, {k: 1.0, k - 1: -1.0}, (k + d, k - d))
    single = _axis_pressure_phasors(case, i, j, {k: 1.0}, (k + d, k + 1 - d))
    r = pair[0] / pair[1]
    assert abs(abs(r) - 1.0) < 0.05 and abs(np.angle(r)) < 0.1, r
    r1 = single[0] / single[1]
    assert abs(abs(r1) - 1.0) < 0.05 and abs(abs(np.angle(r1)) - np.pi) < 0.1, r1
