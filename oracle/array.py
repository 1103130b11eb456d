"""Phased arrays in FP64: the driven array's Rayleigh field, electronic
steering, and refocusing by time reversal through the FDTD model.

TEST INFRASTRUCTURE ONLY (part of the oracle): only the test suite, the smoke
entry and the benchmark's CPU-baseline leg may import it.  Built from the
oracle's own pinned pieces (surface elements, Rayleigh integral, stepping
simulator) plus plain numpy; it imports nothing from the product package.

Paper, Section 2 and 2.3: the multi-element transducers are steered
electronically; for refocusing, a point source is placed at the target, its
field is back-propagated to the domain interface and then carried by the
Rayleigh-Sommerfeld integral to the transducer elements, giving the corrected
phases of the elements; the forward field is then computed with them.

Readings:
  * an element is a flat circular piston with a complex drive w (normal
    velocity u e^{i phi}); its field is w times the unit-drive piston field,
    and the array's field is the sum over elements (linearity);
  * steering in water: w_e = exp(+i k |c_e - T|) for element centre c_e and
    target T (the waves arrive in phase);
  * the point source is a pair of unit z forces pushing outward on the two
    v_z faces of the target cell (+1 on the face above, -1 on the face below),
    the solver's source mechanism applied to one cell: for the near-axial
    waves a focus collects it acts as a monopole, so by reciprocity the record
    is the transfer to the pressure at the target (one z force would give the
    transfer to v_z, whose sign flips for waves reflected back from beyond the
    target); the interface record is the phasor of v_z on the faces of the
    source plane over the last period, (2 / N_T) sum_n v_z exp(-i omega t_n),
    t_n = (n + 1/2) dt, of the pair's field (one solve per face, summed);
  * back-propagation: the first Rayleigh integral of that plane (normal
    velocity, cells of area dx^2) at the element centres;
  * refocused drives: w_e = conj(p_e) / |p_e| (phase conjugation, unit
    amplitude).
"""
from __future__ import annotations

import types

import numpy as np

from . import elements, problem_from_case, rayleigh, setup, Sim

RHO_W, C_W = 1000.0, 1500.0


def _piston(row):
    return types.SimpleNamespace(kind=0, radius=float(row[0]), focal=0.0, apex=tuple(row[1:4]),
                                 axis=tuple(row[4:7]), u0=1.0)


def drives(rows):
    rows = np.asarray(rows, dtype=np.float64).reshape(-1, 9)
    return rows[:, 7] + 1j * rows[:, 8]


def field(rows, freq_hz, pts, w=None):
    """Complex pressure of the driven array at pts [m, 3] (Rayleigh integral of
    every element's sub-elements, times its drive)."""
    rows = np.asarray(rows, dtype=np.float64).reshape(-1, 9)
    w = drives(rows) if w is None else np.asarray(w, dtype=np.complex128)
    out = np.zeros(len(np.asarray(pts).reshape(-1, 3)), dtype=np.complex128)
    for e, r in enumerate(rows):
        el = elements(_piston(r), freq_hz)
        out += w[e] * rayleigh(el, freq_hz, 1.0, pts)
    return out


def source_plane(case, rows, w=None):
    """The array's field on the source plane z = (k_s + 1/2) dx, [ny, nx]."""
    dx = case.dx
    ks = case.pml if case.source_k < 0 else case.source_k
    jj, ii = np.meshgrid(np.arange(case.ny), np.arange(case.nx), indexing="ij")
    pts = np.stack([ii * dx, jj * dx, np.full(ii.shape, (ks + 0.5) * dx)], axis=-1)
    return field(rows, case.freq_hz, pts.reshape(-1, 3), w).reshape(case.ny, case.nx)


def steer(rows, target, freq_hz):
    rows = np.asarray(rows, dtype=np.float64).reshape(-1, 9)
    k = 2 * np.pi * freq_hz / C_W
    r = np.linalg.norm(rows[:, 1:4] - np.asarray(target, dtype=np.float64)[None, :], axis=1)
    return np.exp(1j * k * r)


def record_face(case, i, j, kf, force):
    """Phasor of v_z on the faces of the source plane over the last period of a
    solve of case.mat driven by a z force of the given value on the v_z face
    above cell (i, j, kf)."""
    ks = case.pml if case.source_k < 0 else case.source_k
    prob = problem_from_case(case, source_k=kf)
    info, _ = setup(prob)
    nt, w, dt = info["steps_per_period"], info["omega"], info["dt"]
    src = np.zeros((case.ny, case.nx), dtype=np.complex128)
    src[j, i] = force
    sim = Sim(prob, case.mat)
    acc = np.zeros((case.ny, case.nx), dtype=np.complex128)
    for n in range(case.n_steps):
        sim.step(n, src)
        if n >= case.n_steps - nt:
            acc += sim.field("vz")[ks] * np.exp(-1j * w * (n + 0.5) * dt)
    sim.close()
    return 2.0 * acc / nt


def record(case, cell):
    """The interface record of the point source at the target cell (i, j, k):
    +1 on the v_z face above the cell, -1 on the face below it."""
    i, j, k = cell
    return record_face(case, i, j, k, 1.0) + record_face(case, i, j, k - 1, -1.0)


def backprop(case, plane, centres):
    """First Rayleigh integral of the recorded plane (normal velocity, cell area
    dx^2 at z = (k_s + 1/2) dx) at the points centres [n, 3]."""
    dx = case.dx
    ks = case.pml if case.source_k < 0 else case.source_k
    w = 2 * np.pi * case.freq_hz
    k = w / C_W
    jj, ii = np.meshgrid(np.arange(case.ny), np.arange(case.nx), indexing="ij")
    xs, ys, zp = ii.ravel() * dx, jj.ravel() * dx, (ks + 0.5) * dx
    v = np.asarray(plane, dtype=np.complex128).ravel()
    out = np.empty(len(centres), dtype=np.complex128)
    for e, c in enumerate(np.asarray(centres, dtype=np.float64)):
        R = np.sqrt((xs - c[0]) ** 2 + (ys - c[1]) ** 2 + (zp - c[2]) ** 2)
        out[e] = 1j * w * RHO_W / (2 * np.pi) * dx * dx * np.sum(v * np.exp(-1j * k * R) / R)
    return out


def refocus(case, rows, cell):
    """(drives, back-propagated field at the element centres) for the target cell."""
    rows = np.asarray(rows, dtype=np.float64).reshape(-1, 9)
    p = backprop(case, record(case, cell), rows[:, 1:4])
    a = np.abs(p)
    return np.where(a > 0, np.conj(p) / np.where(a > 0, a, 1.0), 0.0), p
