"""Pins of the FP64 surrogate reference (no GPU): central-difference gradients
on a tiny network, and the spectral layer acting as an exact band-pass
(identity on kept Fourier modes, zero outside) when its weights are the
identity."""
import math

import numpy as np
import pytest

from oracle import nn_ref

TINY = nn_ref.Config(n=8, cin=3, width=4, layers=2, mx=2, my=2, mz=2)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    p = nn_ref.init_params(TINY, 1) + rng.normal(0, 0.05, nn_ref.init_params(TINY, 1).shape)
    x = rng.normal(0, 1, (2, TINY.cin) + (TINY.n,) * 3)
    dy = rng.normal(0, 1, (2, 1) + (TINY.n,) * 3)
    g, dx, _ = nn_ref.backward(p, x, dy, TINY)
    f = lambda q, xx: float((nn_ref.forward(q, xx, TINY) * dy).sum())
    idx = rng.choice(p.size, 40, replace=False)
    eps = 1e-4          # central-difference truncation ~eps^2, round-off ~1e-16/eps
    for i in idx:
        e = np.zeros_like(p)
        e[i] = eps
        num = (f(p + e, x) - f(p - e, x)) / (2 * eps)
        assert num == pytest.approx(g[i], rel=1e-6, abs=1e-8)
    for _ in range(10):
        a = tuple(rng.integers(0, s) for s in x.shape)
        e = np.zeros_like(x)
        e[a] = eps
        num = (f(p, x + e) - f(p, x - e)) / (2 * eps)
        assert num == pytest.approx(dx[a], rel=1e-6, abs=1e-8)


def test_spectral_layer_is_band_pass_with_identity_weights():
    cfg = nn_ref.Config(n=16, cin=1, width=2, layers=1, mx=3, my=3, mz=3)
    R = np.zeros((2, cfg.q, 2, 2))
    R[0, :, 0, 0] = R[0, :, 1, 1] = 1.0
    z, y, x = np.meshgrid(*(np.arange(cfg.n),) * 3, indexing="ij")
    two_pi = 2 * math.pi / cfg.n
    kept = np.cos(two_pi * (2 * x - 1 * y + 2 * z) + 0.3)     # |kx| 2 < 3, |ky| 1, |kz| 2
    dropped = np.sin(two_pi * (5 * x + y))                      # kx = 5 outside
    h = np.stack([kept + dropped, 2 * kept])[None]
    s, _ = nn_ref._spectral(R, h, cfg)
    np.testing.assert_allclose(s[0, 0], kept, atol=1e-12)
    np.testing.assert_allclose(s[0, 1], 2 * kept, atol=1e-12)


def test_param_layout_roundtrip():
    p = nn_ref.init_params(TINY, 3)
    assert np.array_equal(nn_ref.pack(nn_ref.unpack(p, TINY), TINY), p)


def test_features_phase_and_table_lookup():
    """The phase channels give back the field's phase (atan2 of the pair) and
    do not depend on its magnitude; a zero field reads as phase 0; material
    indices past the table read as zero contrast."""
    rng = np.random.default_rng(5)
    n = 500
    theta = rng.uniform(-np.pi, np.pi, n)
    r = 10.0 ** rng.uniform(-20, 3, n)
    field = r * np.exp(1j * theta)
    field[:7] = 0.0
    table = rng.normal(size=(5, 2))
    mat = rng.integers(0, 8, n).astype(np.uint8)
    x = nn_ref.features(mat, table, field)
    assert x.shape == (4, n)
    np.testing.assert_allclose(np.arctan2(x[3, 7:], x[2, 7:]), theta[7:], rtol=0, atol=1e-12)
    np.testing.assert_allclose(x[2] ** 2 + x[3] ** 2, 1.0, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(x[2:, :7], [[1.0] * 7, [0.0] * 7])
    np.testing.assert_allclose(nn_ref.features(mat, table, 3.5 * field)[2:], x[2:], rtol=0, atol=1e-15)
    for c in range(n):
        want = table[mat[c]] if mat[c] < 5 else (0.0, 0.0)
        assert tuple(x[:2, c]) == tuple(want)
