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
    (residual below 0.1 rad RMS: discretisation, the dipole pattern of the
    point force and the finite plane)."""
    case, rows, cell = synth.array_case(20001, n_steps=330)
    case.mat[:] = 0
    w_tr, p = array.refocus(case, rows, cell)
    w_geo = array.steer(rows, np.array(cell) * case.dx, case.freq_hz)
    d = np.angle(w_tr * np.conj(w_geo))
    g = np.angle(np.mean(np.exp(1j * d)))
    res = np.angle(np.exp(1j * (d - g)))
    assert np.sqrt(np.mean(res ** 2)) < 0.1, res
    assert np.all(np.abs(p) > 0)
