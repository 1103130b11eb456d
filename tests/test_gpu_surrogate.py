"""Surrogate kernels on the GPU: the BF16 matrix-core GEMM (exact against
numpy on BF16-rounded operands) and the network's forward pass and gradients
against the FP64 numpy reference (FFT-based)."""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

from oracle import nn_ref
import paper_2301_12727_amd as bb
from paper_2301_12727_amd import surrogate as sg
import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def bf16(a):
    """Round FP32 to BF16 (nearest even), returned as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


# "n" stores an operand as written, "t" transposed; a third letter "c" stores C
# column-major.  Sizes that are multiples of 4 take the float4 staging paths
# (and the transposed epilogue for "c"), the others the element-wise ones.
@pytest.mark.parametrize("M,N,K,batch,trans", [(64, 64, 32, 1, "nn"), (50, 70, 45, 3, "nn"),
                                                (33, 17, 130, 2, "tn"), (1, 300, 7, 2, "nt"),
                                                (128, 96, 64, 1, "tt"), (256, 16, 64, 3, "nnc"),
                                                (200, 132, 96, 2, "ttc"), (96, 40, 36, 2, "tnc"),
                                                (52, 200, 100, 1, "ntc"), (68, 20, 8, 2, "nt"),
                                                (50, 36, 44, 2, "nnc")])
def test_gemm_matches_bf16_reference(M, N, K, batch, trans):
    rng = np.random.default_rng(M * 1000 + N)
    A = rng.normal(size=(batch, M, K)).astype(np.float32)
    B = rng.normal(size=(batch, K, N)).astype(np.float32)
    C0 = rng.normal(size=(batch, M, N)).astype(np.float32)
    bias = rng.normal(size=M).astype(np.float32)
    # storage layouts: "t" stores the operand transposed in memory
    Ad = np.ascontiguousarray(A.transpose(0, 2, 1) if trans[0] == "t" else A)
    Bd = np.ascontiguousarray(B.transpose(0, 2, 1) if trans[1] == "t" else B)
    a_str = (M * K, 1, M) if trans[0] == "t" else (M * K, K, 1)
    b_str = (K * N, 1, K) if trans[1] == "t" else (K * N, N, 1)
    tA, tB = torch.from_numpy(Ad).cuda(), torch.from_numpy(Bd).cuda()
    colmajor = trans[2:] == "c"
    tC = torch.from_numpy(np.ascontiguousarray(C0.transpose(0, 2, 1) if colmajor else C0)).cuda()
    c_str = (M * N, 1, M) if colmajor else (M * N, N, 1)
    tb = torch.from_numpy(bias).cuda()
    sg.gemm(tA, a_str, tB, b_str, tC, c_str, M, N, K, batch, alpha=1.5, beta=0.5, bias=tb)
    torch.cuda.synchronize()
    want = 1.5 * np.einsum("bmk,bkn->bmn", bf16(A), bf16(B)) + 0.5 * C0 + bias[None, :, None]
    got = tC.cpu().numpy()
    if colmajor:
        got = got.transpose(0, 2, 1)
    err = np.abs(got - want).max() / np.abs(want).max()
    say(f"[gemm] {M}x{N}x{K} b{batch} {trans}: max rel {err:.2e}")
    assert err < 1e-5


CFG = nn_ref.Config(n=16, cin=4, width=8, layers=2, mx=3, my=3, mz=3)


def _setup(batch, seed):
    rng = np.random.default_rng(seed)
    p = nn_ref.init_params(CFG, seed).astype(np.float32)
    p += rng.normal(0, 0.02, p.shape).astype(np.float32)
    x = rng.normal(0, 1, (batch, CFG.cin) + (CFG.n,) * 3).astype(np.float32)
    return p, x


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def test_forward_matches_fp64_reference():
    p, x = _setup(2, 1)
    model = sg.Surrogate(**CFG.__dict__)
    assert model.n_params == p.size
    y = model.forward(torch.from_numpy(p).cuda(), torch.from_numpy(x).cuda())
    ref = nn_ref.forward(p.astype(np.float64), x.astype(np.float64), CFG)
    err = rel(y.cpu().numpy(), ref)
    say(f"[surrogate] forward rel-L2 {err:.3e}")
    assert err < 2e-2


# The wide configuration's per-mode weights (80 x 80) are too large for the
# LDS mixing-gradient kernels and take the global-memory ones; its weight
# gradients have 6400 columns, so their row sums use several row groups.
WIDE = nn_ref.Config(n=8, cin=4, width=80, layers=1, mx=2, my=2, mz=2)


@pytest.mark.parametrize("cfg", [CFG, WIDE], ids=["narrow", "wide"])
def test_gradients_match_fp64_reference(cfg):
    rng = np.random.default_rng(2)
    p = nn_ref.init_params(cfg, 2).astype(np.float32)
    p += rng.normal(0, 0.02, p.shape).astype(np.float32)
    x = rng.normal(0, 1, (2, cfg.cin) + (cfg.n,) * 3).astype(np.float32)
    rng = np.random.default_rng(3)
    dy = rng.normal(0, 1, (2, 1) + (cfg.n,) * 3).astype(np.float32)
    model = sg.Surrogate(**cfg.__dict__)
    g = model.backward(torch.from_numpy(p).cuda(), torch.from_numpy(x).cuda(),
                       torch.from_numpy(dy).cuda()).cpu().numpy()
    gref, _, _ = nn_ref.backward(p.astype(np.float64), x.astype(np.float64),
                                 dy.astype(np.float64), cfg)
    errs = {}
    off = 0
    for name, shape in nn_ref.param_layout(cfg):
        n = int(np.prod(shape))
        errs[name] = rel(g[off:off + n], gref[off:off + n])
        off += n
    say("[surrogate] grad rel-L2 " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    assert rel(g, gref) < 2e-2
    assert max(errs.values()) < 5e-2


def test_training_reduces_loss_on_a_fixed_batch():
    p, x = _setup(2, 4)
    rng = np.random.default_rng(5)
    target = np.tanh(nn_ref.forward(nn_ref.init_params(CFG, 9), x.astype(np.float64), CFG))
    model = sg.Surrogate(**CFG.__dict__)
    st = model.train_state(torch.from_numpy(p).cuda())
    xs, ts = torch.from_numpy(x).cuda(), torch.from_numpy(target.astype(np.float32)).cuda()
    losses = [model.train_step(st, xs, ts, lr=3e-3) for _ in range(60)]
    say(f"[surrogate] loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert losses[-1] < 0.5 * losses[0]
    del rng


def test_weighted_loss_value_and_step():
    """Loss of a training step equals mean(w (y - t)^2) with w = 1 + f exp(t),
    y the forward output at the step's starting parameters; training with the
    weight still reduces the loss."""
    p, x = _setup(2, 4)
    target = np.tanh(nn_ref.forward(nn_ref.init_params(CFG, 9), x.astype(np.float64), CFG))
    focus = 3.0
    model = sg.Surrogate(**CFG.__dict__, loss_focus=focus)
    xs = torch.from_numpy(x).cuda()
    ts = torch.from_numpy(target.astype(np.float32)).cuda()
    pt = torch.from_numpy(p).cuda()
    y = model.forward(pt, xs).cpu().numpy().astype(np.float64)
    t64 = target.astype(np.float32).astype(np.float64)
    w = 1.0 + focus * np.exp(t64)
    expect = float(np.mean(w * (y.reshape(t64.shape) - t64) ** 2))
    st = model.train_state(pt.clone())
    got = model.train_step(st, xs, ts, lr=3e-3)
    say(f"[surrogate] weighted loss {got:.6e} vs {expect:.6e}")
    assert abs(got - expect) <= 1e-4 * expect
    losses = [model.train_step(st, xs, ts, lr=3e-3) for _ in range(60)]
    assert losses[-1] < 0.5 * got


def test_features_match_reference():
    """Input channels from a material map, a contrast table and a complex free
    field (ragged cell count; indices past the table; zero and tiny fields)."""
    rng = np.random.default_rng(8)
    cells, n_table = 5 * 7 * 11 * 13 + 3, 6
    mat = rng.integers(0, n_table + 4, cells).astype(np.uint8)
    table = rng.normal(size=(n_table, 2)).astype(np.float32)
    field = (rng.normal(size=cells) + 1j * rng.normal(size=cells)).astype(np.complex64)
    field *= (10.0 ** rng.uniform(-12, 4, cells)).astype(np.float32)
    field[::97] = 0.0
    ref = nn_ref.features(mat, table, field)
    x = torch.empty((4, cells), dtype=torch.float32, device="cuda")
    sg.features(torch.from_numpy(mat).cuda(), torch.from_numpy(table).cuda(),
                torch.from_numpy(field).cuda(), x)
    got = x.cpu().numpy().astype(np.float64)
    say(f"[features] {cells} cells: phase max err {np.abs(got[2:] - ref[2:]).max():.2e}")
    np.testing.assert_array_equal(got[:2], ref[:2])
    np.testing.assert_allclose(got[2:], ref[2:], rtol=0, atol=2e-6)


def test_init_params_layout_and_scales():
    """Seeded initialisation: reproducible per seed, zero biases, lift and
    pointwise weights normal with standard deviation 1/sqrt(fan-in), spectral
    weights uniform in [-1/W, 1/W], all in the documented parameter order."""
    model = sg.Surrogate(**WIDE.__dict__)
    a = model.init_params(3).cpu().numpy()
    assert a.size == model.n_params == sum(int(np.prod(s)) for _, s in nn_ref.param_layout(WIDE))
    assert np.array_equal(a, model.init_params(3).cpu().numpy())
    assert not np.array_equal(a, model.init_params(4).cpu().numpy())
    p = nn_ref.unpack(a, WIDE)
    W = WIDE.width
    for name, v in p.items():
        if name.startswith(("lift_b", "proj_b")) or (name[0] == "b" and name[1:].isdigit()):
            assert np.all(v == 0.0), name
    for name, fan, tol in (("lift_w", WIDE.cin, 0.2), ("w0", W, 0.05), ("proj_w", W, 0.35)):
        v = p[name]
        assert abs(v.mean()) < 4 * tol / np.sqrt(fan) and abs(v.std() * np.sqrt(fan) - 1) < tol, name
    r = p["r0"]
    assert np.abs(r).max() <= float(np.float32(1.0 / W)) and abs(r.mean()) < 5e-3 / W
    assert abs(r.std() * W * np.sqrt(3.0) - 1) < 0.01


def test_forward_at_largest_size_equivariance_and_pointwise_samples():
    """The largest accepted volume, n = 256 (width 32, 4 layers, 8 modes per
    axis).  (1) Every layer commutes with circular shifts (the truncated
    Fourier transforms are periodic and the rest acts per cell), so the output
    of a shifted input is the shifted output, up to BF16 rounding; a wrong
    stride or axis in any transform stage breaks this.  (2) With the spectral
    weights set to zero the network acts per cell, and its output at 512
    sampled cells equals the FP64 reference run on those cells alone."""
    cfg = nn_ref.Config(n=256, cin=4, width=32, layers=4, mx=8, my=8, mz=8)
    model = sg.Surrogate(**cfg.__dict__)
    params = model.init_params(5)
    gen = torch.Generator(device="cuda").manual_seed(5)
    x = torch.randn((1, 4) + (cfg.n,) * 3, device="cuda", generator=gen)
    shifts, dims = (37, 101, 3), (2, 3, 4)
    y = model.forward(params, x)
    ys = model.forward(params, torch.roll(x, shifts, dims))
    eq = float(torch.linalg.norm(torch.roll(y, shifts, dims) - ys) / torch.linalg.norm(ys))
    p = nn_ref.unpack(params.cpu().numpy(), cfg)
    small = nn_ref.Config(n=8, cin=4, width=32, layers=4, mx=1, my=1, mz=1)
    for l in range(cfg.layers):
        p[f"r{l}"] = np.zeros((2, cfg.q, cfg.width, cfg.width))
    y0 = model.forward(torch.from_numpy(nn_ref.pack(p, cfg).astype(np.float32)).cuda(), x)
    for l in range(cfg.layers):
        p[f"r{l}"] = np.zeros((2, small.q, cfg.width, cfg.width))
    cells = torch.from_numpy(np.random.default_rng(5).choice(cfg.n ** 3, 512, replace=False)).cuda()
    xs = x.reshape(4, -1)[:, cells].cpu().numpy().astype(np.float64).reshape(1, 4, 8, 8, 8)
    ref = nn_ref.forward(nn_ref.pack(p, small), xs, small).ravel()
    got = y0.reshape(-1)[cells].cpu().numpy()
    pw = rel(got, ref)
    say(f"[surrogate] n=256: shift equivariance rel-L2 {eq:.3e}, pointwise samples rel-L2 {pw:.3e}")
    assert eq < 2e-2
    assert pw < 2e-2


@pytest.mark.timeout(900)
def test_trained_network_beats_no_learning_baseline_and_falls_back_to_fdtd():
    """Gain of the learned part: a network trained on the GPU by the library's
    own kernels (320 FDTD solves of 64^3 skull patches, 75 s of training)
    predicts the held-out post-skull focal pressure of 40 unseen seeds with a
    mean error well below the no-learning baseline (the free field scaled by
    the training-mean transmission).  The predictor answers an in-distribution
    case with the network and sends a 1 MHz case (a frequency never trained
    on) to the FDTD solve, whose map equals a direct bbfd_solve bit for bit."""
    from paper_2301_12727_amd import surrogate_run as sr
    tr = sr.generate(list(range(10000, 10320)), 64)
    ev = sr.generate(list(range(20000, 20040)), 64, keep_masks=True)
    ratio = float(np.mean(tr.peak_post / tr.free_post))
    model = sg.Surrogate(n=64, cin=4, width=32, layers=4, mx=8, my=8, mz=8, loss_focus=10.0)
    params, hist = sr.train(model, tr, 75.0, batch=4, lr=1e-3, n_val=32, focus=10.0, flips=True)
    res = sr.evaluate(model, params, ev, ratio)
    say(f"[surrogate] 320 solves / 75 s: focal error mean {res['focal_err_mean']:.4f} "
        f"(median {res['focal_err_median']:.4f}); baseline {res['baseline_focal_err_mean']:.4f}")
    assert res["focal_err_mean"] < 0.75 * res["baseline_focal_err_mean"]
    gate = sr.Gate(tr.stats)
    pred = sr.Predictor(model, params, gate)
    inside = next(c for c in (synth.surrogate_case(s) for s in range(20000, 20040))
                  if pred.route(c) == "surrogate")
    P, path = pred(inside)
    assert path == "surrogate" and bool(torch.isfinite(P).all()) and float(P.max()) > 0
    odd = synth.surrogate_case(30000, freq_hz=1e6)
    P2, path2 = pred(odd)
    assert path2 == "fdtd" and pred.counts == {"surrogate": 1, "fdtd": 1}
    ref, _, _, _ = bb.run_case(odd)
    assert torch.equal(P2, ref)
