"""Thermal step of the pipeline in FP64: the Pennes bio-heat transfer equation
(BHTE) solved by explicit finite differences, with the acoustic heat source,
the sonication regime, the maximal temperature and the thermal dose.

TEST INFRASTRUCTURE ONLY (part of the oracle): only the test suite, the smoke
entry and the benchmark's CPU-baseline leg may import it.  Plain numpy; it
imports nothing from the product package and shares no code with it.

Paper, Section 2.4: the BHTE is solved with a finite-difference time-domain
scheme in Cartesian coordinates, with the domain's border held at 37 degC; the
user gives the sonication's on time, off time and duty cycle and the spatial-
peak pulse-average intensity in the brain; in skull bone a fraction 0.16 of the
attenuation turns into heat; safety metrics include the maximal temperature and
the thermal dose (Damianou et al., the Sapareto-Dewey CEM43 form).

Readings (the paper defers the rest to its references):
  * Pennes: rho C dT/dt = div(k grad T) - w rho_b C_b (T - T_a) + Q, with
    blood rho_b C_b = 1050 * 3617 J/(m^3 K) and T_a = the border temperature;
  * explicit Euler in time, second-order central differences in space, the
    conductivity of a face the harmonic mean of its two cells'; the outermost
    cells of the grid are the border and stay at T_a;
  * heat source Q = 2 alpha_h I with I = p^2 / (2 rho c_l) from the peak-
    pressure map p, alpha_h = h alpha_l the heating share of the longitudinal
    attenuation (h = 1 in soft tissue and water, 0.16 in bone), all scaled by
    the caller's intensity factor;
  * the duty cycle scales Q while the ultrasound is on (time-averaged power);
    steps [0, n_on) are on, [n_on, n_on + n_off) off;
  * CEM43 dose: sum over steps of dt/60 * R^(43 - T), R = 0.5 at T >= 43 degC,
    0.25 below, in minutes; the temperature of a step is the one at its end.
"""
from __future__ import annotations

import numpy as np

RHO_C_BLOOD = 1050.0 * 3617.0


def heat_source(mat, peak, acoustic, heat_frac, scale=1.0):
    """Q [W/m^3] per cell: scale * 2 * h alpha_l * p^2 / (2 rho c_l).
    acoustic: [n_mat, 5] rows (rho, c_l, c_s, alpha_l, alpha_s) as the FDTD
    table; heat_frac: [n_mat] the share h of alpha_l that heats."""
    tab = np.asarray(acoustic, dtype=np.float64).reshape(-1, 5)
    h = np.asarray(heat_frac, dtype=np.float64)
    m = np.asarray(mat).astype(np.int64)
    p = np.asarray(peak, dtype=np.float64)
    intensity = p * p / (2.0 * tab[m, 0] * tab[m, 1])
    return scale * 2.0 * h[m] * tab[m, 3] * intensity


def stable_dt(mat, acoustic, thermal, dx):
    """Largest explicit step of the scheme: dt < rho C / (6 k / dx^2 + w rho_b C_b)
    over the materials present."""
    tab = np.asarray(acoustic, dtype=np.float64).reshape(-1, 5)
    th = np.asarray(thermal, dtype=np.float64).reshape(-1, 3)
    used = np.unique(np.asarray(mat))
    rc = tab[used, 0] * th[used, 1]
    return float(np.min(rc / (6.0 * th[used, 0] / dx ** 2 + th[used, 2] * RHO_C_BLOOD)))


class BHTE:
    """Explicit Pennes solver on a [nz, ny, nx] grid.
    thermal: [n_mat, 3] rows (k W/(m K), C J/(kg K), perfusion w 1/s)."""

    def __init__(self, mat, acoustic, thermal, dx, dt, t_body=37.0):
        self.mat = np.asarray(mat).astype(np.int64)
        tab = np.asarray(acoustic, dtype=np.float64).reshape(-1, 5)
        th = np.asarray(thermal, dtype=np.float64).reshape(-1, 3)
        self.dx, self.dt, self.t_body = float(dx), float(dt), float(t_body)
        self.k = th[self.mat, 0]
        self.rho_c = tab[self.mat, 0] * th[self.mat, 1]
        self.perf = th[self.mat, 2] * RHO_C_BLOOD
        self.T = np.full(self.mat.shape, self.t_body)
        self.t_max = self.T.copy()
        self.dose = np.zeros(self.mat.shape)

    @staticmethod
    def _face(ka, kb):
        """Harmonic mean of two conductivities (0 if either is 0)."""
        s = ka + kb
        return np.where(s > 0, 2.0 * ka * kb / np.where(s > 0, s, 1.0), 0.0)

    def step(self, q):
        """One step with heat source q (W/m^3, already duty-scaled or zero)."""
        T, k = self.T, self.k
        inner = (slice(1, -1),) * 3
        tc = T[inner]
        div = np.zeros_like(tc)
        for axis in range(3):
            for d in (-1, 1):
                sl = [slice(1, -1)] * 3
                sl[axis] = slice(1 + d, T.shape[axis] - 1 + d)
                nb = tuple(sl)
                div += self._face(k[inner], k[nb]) * (T[nb] - tc)
        rhs = div / self.dx ** 2 - self.perf[inner] * (tc - self.t_body) + q[inner]
        new = T.copy()
        new[inner] = tc + self.dt * rhs / self.rho_c[inner]
        self.T = new
        np.maximum(self.t_max, new, out=self.t_max)
        r = np.where(new >= 43.0, 0.5, 0.25)
        self.dose += self.dt / 60.0 * np.power(r, 43.0 - new)

    def run(self, q, n_on, n_off, duty):
        zero = np.zeros_like(q)
        for n in range(n_on + n_off):
            self.step(duty * q if n < n_on else zero)
        return self.T, self.t_max, self.dose
