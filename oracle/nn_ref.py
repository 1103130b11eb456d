"""FP64 numpy reference of the Fourier-neural-operator surrogate.

TEST INFRASTRUCTURE ONLY: checks the HIP surrogate kernels (forward values and
gradients).  Uses numpy's real FFTs for the spectral layers, so it shares no
formulation with the GPU path (which writes the truncated transforms as
matrix products on the matrix cores).

Network (all layers act on [B, C, N, N, N] volumes, x fastest):
  h0 = W_lift x + b_lift                                   (pointwise, Cin -> W)
  for l = 1..L:  z_l = S_l(h_{l-1}) + W_l h_{l-1} + b_l,  h_l = GELU(z_l)
  y  = W_proj h_L + b_proj                                 (pointwise, W -> 1)
S_l keeps the Fourier modes kx in [0, Mx), ky in {0..My-1, -My..-1},
kz in {0..Mz-1, -Mz..-1} of rfftn(h), mixes channels per mode with complex
weights R_l[q][c][o], and returns irfftn of the zero-padded result.
GELU(z) = z/2 (1 + erf(z/sqrt 2)).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import erf


@dataclasses.dataclass(frozen=True)
class Config:
    n: int = 64
    cin: int = 4
    width: int = 32
    layers: int = 4
    mx: int = 8
    my: int = 8
    mz: int = 8

    @property
    def q(self) -> int:
        return self.mx * 2 * self.my * 2 * self.mz


def param_layout(cfg: Config):
    """Ordered (name, shape) of the flat FP32 parameter vector."""
    W = cfg.width
    out = [("lift_w", (W, cfg.cin)), ("lift_b", (W,))]
    for l in range(cfg.layers):
        out += [(f"r{l}", (2, cfg.q, W, W)), (f"w{l}", (W, W)), (f"b{l}", (W,))]
    out += [("proj_w", (1, W)), ("proj_b", (1,))]
    return out


def unpack(flat: np.ndarray, cfg: Config) -> dict:
    p, o = {}, 0
    for name, shape in param_layout(cfg):
        n = int(np.prod(shape))
        p[name] = flat[o:o + n].reshape(shape).astype(np.float64)
        o += n
    assert o == flat.size
    return p


def pack(p: dict, cfg: Config) -> np.ndarray:
    return np.concatenate([p[name].reshape(-1) for name, _ in param_layout(cfg)])


def _kidx(m: int, n: int):
    return np.concatenate([np.arange(m), np.arange(n - m, n)])


def _modes(U: np.ndarray, cfg: Config) -> np.ndarray:
    """Kept modes of an rfftn spectrum [B, C, Z, Y, X//2+1] -> [B, C, Q]
    ordered (kz', ky', kx) with kx fastest."""
    kz = _kidx(cfg.mz, cfg.n)
    ky = _kidx(cfg.my, cfg.n)
    sub = U[:, :, kz][:, :, :, ky][..., :cfg.mx]
    return sub.reshape(U.shape[0], U.shape[1], -1)


def _unmodes(V: np.ndarray, cfg: Config) -> np.ndarray:
    B, O, _ = V.shape
    full = np.zeros((B, O, cfg.n, cfg.n, cfg.n // 2 + 1), dtype=np.complex128)
    kz = _kidx(cfg.mz, cfg.n)
    ky = _kidx(cfg.my, cfg.n)
    v = V.reshape(B, O, 2 * cfg.mz, 2 * cfg.my, cfg.mx)
    for a, zz in enumerate(kz):
        for b_, yy in enumerate(ky):
            full[:, :, zz, yy, :cfg.mx] = v[:, :, a, b_]
    return full


def _hermitian_weight(cfg: Config) -> np.ndarray:
    c = np.full(cfg.mx, 2.0)
    c[0] = 1.0
    return np.tile(c, 2 * cfg.mz * 2 * cfg.my)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def _pointwise(w, b, h):
    B = h.shape[0]
    out = np.einsum("oc,bcp->bop", w, h.reshape(B, h.shape[1], -1))
    if b is not None:
        out = out + b[None, :, None]
    return out.reshape((B, w.shape[0]) + h.shape[2:])


def _spectral(R, h, cfg):
    U = _modes(np.fft.rfftn(h, axes=(2, 3, 4)), cfg)         # [B, C, Q]
    Rc = R[0] + 1j * R[1]                                      # [Q, C, O]
    V = np.einsum("qco,bcq->boq", Rc, U)
    s = np.fft.irfftn(_unmodes(V, cfg), s=(cfg.n,) * 3, axes=(2, 3, 4))
    return s, U


def forward(flat: np.ndarray, x: np.ndarray, cfg: Config, keep: bool = False):
    p = unpack(flat, cfg)
    h = _pointwise(p["lift_w"], p["lift_b"], x.astype(np.float64))
    tape = []
    for l in range(cfg.layers):
        s, U = _spectral(p[f"r{l}"], h, cfg)
        z = s + _pointwise(p[f"w{l}"], p[f"b{l}"], h)
        tape.append((h, U, z))
        h = gelu(z)
    y = _pointwise(p["proj_w"], p["proj_b"], h)
    return (y, tape, h) if keep else y


def backward(flat: np.ndarray, x: np.ndarray, dy: np.ndarray, cfg: Config):
    """Gradient of <dy, forward(x)> with respect to the flat parameters and x."""
    p = unpack(flat, cfg)
    y, tape, hL = forward(flat, x, cfg, keep=True)
    g = {}
    B = x.shape[0]
    N3 = cfg.n ** 3
    dyf = dy.reshape(B, 1, -1)
    g["proj_w"] = np.einsum("bop,bcp->oc", dyf, hL.reshape(B, cfg.width, -1))
    g["proj_b"] = dyf.sum(axis=(0, 2))
    dh = _pointwise(p["proj_w"].T, None, dy)
    cw = _hermitian_weight(cfg)
    for l in reversed(range(cfg.layers)):
        h, U, z = tape[l]
        dz = dh * gelu_grad(z)
        dzf = dz.reshape(B, cfg.width, -1)
        g[f"w{l}"] = np.einsum("bop,bcp->oc", dzf, h.reshape(B, cfg.width, -1))
        g[f"b{l}"] = dzf.sum(axis=(0, 2))
        dh = _pointwise(p[f"w{l}"].T, None, dz)
        # s = Re sum_k c_k V(k) e^{ikx} / N^3  ->  dV = c_k rfftn(dz)(k) / N^3
        dV = _modes(np.fft.rfftn(dz, axes=(2, 3, 4)), cfg) * cw[None, None, :] / N3
        Rr, Ri = p[f"r{l}"][0], p[f"r{l}"][1]
        Ur, Ui = U.real, U.imag
        dVr, dVi = dV.real, dV.imag
        g[f"r{l}"] = np.stack([np.einsum("bcq,boq->qco", Ur, dVr) + np.einsum("bcq,boq->qco", Ui, dVi),
                               np.einsum("bcq,boq->qco", Ur, dVi) - np.einsum("bcq,boq->qco", Ui, dVr)])
        dUr = np.einsum("qco,boq->bcq", Rr, dVr) + np.einsum("qco,boq->bcq", Ri, dVi)
        dUi = np.einsum("qco,boq->bcq", Rr, dVi) - np.einsum("qco,boq->bcq", Ri, dVr)
        # U(k) = sum_x h e^{-ikx}  ->  dh = Re sum_k dU(k) e^{ikx} = N^3 irfftn(dU / c_k)
        dUc = (dUr + 1j * dUi) / cw[None, None, :]
        dh = dh + N3 * np.fft.irfftn(_unmodes(dUc, cfg), s=(cfg.n,) * 3, axes=(2, 3, 4))
    g["lift_w"] = np.einsum("bop,bcp->oc", dh.reshape(B, cfg.width, -1), x.reshape(B, cfg.cin, -1))
    g["lift_b"] = dh.reshape(B, cfg.width, -1).sum(axis=(0, 2))
    dx = _pointwise(p["lift_w"].T, None, dh)
    return pack(g, cfg), dx, y


def init_params(cfg: Config, seed: int) -> np.ndarray:
    """Reference initialisation (tests only; the GPU path has its own)."""
    rng = np.random.default_rng(seed)
    p = {}
    W = cfg.width
    p["lift_w"] = rng.normal(0, 1 / math.sqrt(cfg.cin), (W, cfg.cin))
    p["lift_b"] = np.zeros(W)
    for l in range(cfg.layers):
        p[f"r{l}"] = rng.uniform(0, 1, (2, cfg.q, W, W)) / (W * W)
        p[f"w{l}"] = rng.normal(0, 1 / math.sqrt(W), (W, W))
        p[f"b{l}"] = np.zeros(W)
    p["proj_w"] = rng.normal(0, 1 / math.sqrt(W), (1, W))
    p["proj_b"] = np.zeros(1)
    return pack(p, cfg)


def features(mat: np.ndarray, table: np.ndarray, field: np.ndarray) -> np.ndarray:
    """Input channels of one sample, [4][cells]: the relative sound speed and
    density c/c_w - 1 and rho/rho_w - 1 of each cell's material (rows of
    ``table``, [n_table][2]; indices past the table read as 0) and the cosine
    and sine of the phase of the free field there (phase 0 where the field is
    exactly zero)."""
    m = np.asarray(mat).ravel().astype(np.int64)
    t = np.asarray(table, dtype=np.float64).reshape(-1, 2)
    inside = m < len(t)
    row = t[np.where(inside, m, 0)]
    row[~inside] = 0.0
    phase = np.angle(np.asarray(field).ravel().astype(np.complex128))
    return np.stack([row[:, 0], row[:, 1], np.cos(phase), np.sin(phase)])
