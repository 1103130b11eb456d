"""Closed forms the oracle is pinned against (test-side only).

Each function restates a textbook result, not the oracle's update rules:
plane-wave dispersion of the 4th-order staggered leapfrog (Levander 1988),
the standard-linear-solid modulus (Zener), normal-incidence transmission
through an interface and a layer, and the on-axis field of a baffled spherical
cap (O'Neil 1949).
"""
import math

import numpy as np
from scipy import optimize

C1, C2 = 9.0 / 8.0, -1.0 / 24.0
RHO_W, C_W = 1000.0, 1500.0


def spatial_symbol(k, dx):
    """Magnitude of the staggered 4th-order first derivative applied to exp(ikz)."""
    return (2.0 / dx) * (C1 * np.sin(k * dx / 2) + C2 * np.sin(3 * k * dx / 2))


def soft_source_amplitude(k, dx):
    """Far-field amplitude per unit |S| radiated by a soft source of strength
    2 c |S| / dx on one cell of the discrete 1D lattice: the propagating-pole
    residue gives 1 / (dK/dk) = 1 / (c1 cos(k dx/2) + 3 c2 cos(3 k dx/2))."""
    return 1.0 / (C1 * math.cos(k * dx / 2) + 3 * C2 * math.cos(3 * k * dx / 2))


def discrete_k_lossless(omega, c, dt, dx):
    """Real wavenumber solving sin(w dt/2) = (c dt/dx)(c1 sin(k dx/2) + c2 sin(3k dx/2))."""
    lhs = math.sin(omega * dt / 2)
    f = lambda k: (c * dt / dx) * (C1 * math.sin(k * dx / 2) + C2 * math.sin(3 * k * dx / 2)) - lhs
    return optimize.brentq(f, 1e-9, math.pi / dx)


def sls_modulus(m_relaxed, tau, omega, omega0):
    """Zener element: M(w) = M_R (1 + i w tau_eps)/(1 + i w tau_sig), tau_sig = 1/w0,
    tau_eps = tau_sig (1 + tau)."""
    ts = 1.0 / omega0
    te = ts * (1.0 + tau)
    return m_relaxed * (1 + 1j * omega * te) / (1 + 1j * omega * ts)


def continuum_k(rho, modulus, omega):
    """Complex wavenumber (e^{i(wt - kz)}, Im k < 0 for decay) of a plane wave."""
    k = omega * np.sqrt(rho / complex(modulus))
    return k if k.imag <= 0 else np.conj(k)


def discrete_k_lossy(rho, m_relaxed, tau, omega0, dt, dx):
    """Complex wavenumber of the discrete scheme: leapfrog in time, Crank-Nicolson
    memory variable (modulus seen at the prewarped frequency (2/dt) tan(w dt/2)),
    4th-order staggered space.  Solves rho wt^2 = M_d K(k)^2 by Newton."""
    wt = (2.0 / dt) * math.sin(omega0 * dt / 2)
    wh = (2.0 / dt) * math.tan(omega0 * dt / 2)
    md = sls_modulus(m_relaxed, tau, wh, omega0)
    target = wt * np.sqrt(rho / md)
    target = target if target.imag <= 0 else np.conj(target)
    k = continuum_k(rho, sls_modulus(m_relaxed, tau, omega0, omega0), omega0)
    for _ in range(60):
        f = spatial_symbol(k, dx) - target
        fp = C1 * np.cos(k * dx / 2) + 3 * C2 * np.cos(3 * k * dx / 2)
        k = k - f / fp
    return k


def layer_transmission(z1, z_layer, k_layer, d):
    """Pressure transmission through a layer between two identical fluids."""
    return 2.0 / (2 * np.cos(k_layer * d) + 1j * (z_layer / z1 + z1 / z_layer) * np.sin(k_layer * d))


def oneil_on_axis(z, a, F, k, rho=RHO_W, c=C_W, u0=1.0):
    """|p| on the axis of a spherical cap (aperture radius a, curvature radius F),
    z measured from the apex; F = inf gives the flat piston."""
    if math.isinf(F):
        return 2 * rho * c * u0 * abs(math.sin(k * (math.sqrt(z * z + a * a) - z) / 2))
    h = F - math.sqrt(F * F - a * a)
    if abs(z - F) < 1e-12:
        return rho * c * u0 * k * h
    re = math.sqrt((z - h) ** 2 + a * a)
    return 2 * rho * c * u0 / abs(1 - z / F) * abs(math.sin(k * (re - z) / 2))
