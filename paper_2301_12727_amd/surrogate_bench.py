"""Throughput of the surrogate's kernels on one GPU.

Times the forward pass and the training step of the 3D FNO at its working size
on synthetic inputs, and sets the forward pass against the HBM and matrix-core
rooflines: the algorithmic bytes and FLOPs of every launch the forward pass
issues are counted from the layer shapes (the contractions, the truncated
transforms as three strided stages each way, the per-mode mixing; GELU is
applied in the last inverse stage), and divided by the measured time.
Prints one JSON line.

    python -m paper_2301_12727_amd.surrogate_bench [--batch 4] [--reps 20]
"""
from __future__ import annotations

import argparse
import json
import sys

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 matrix cores


def forward_counts(n, cin, W, L, mx, my, mz, B):
    """Algorithmic bytes (activations read and written once per launch: the
    GELU outputs h_l in BF16, everything else FP32; weights and transform
    matrices counted once) and FLOPs of one forward pass of B samples, launch by
    launch."""
    P, n2 = n ** 3, n * n
    Q = mx * 2 * my * 2 * mz
    f = 4
    vol = B * W * P * f                     # one FP32 activation tensor
    hb = B * W * P * 2                      # one BF16 tensor h_l
    T1 = B * W * 2 * mx * n2 * f            # after the x stage
    T2 = B * W * 4 * my * mx * n * f        # after the y stage
    U = B * W * 2 * Q * f                   # kept modes (real, imaginary planes)
    I1 = B * W * 2 * n * 4 * mz * my * f    # inverse x stage
    I2 = B * W * 2 * n * n * 2 * mz * f     # inverse y stage
    nb = B * W
    rows = [("lift", B * cin * P * f + hb, 2 * W * cin * P * B)]
    for _ in range(L):
        rows += [
            ("pointwise", hb + vol + W * W * f, 2 * W * W * P * B),
            ("dft_x", hb + T1, 2 * n2 * 2 * mx * n * nb),
            ("dft_y", T1 + T2, 2 * (mx * n) * (4 * my) * (2 * n) * nb),
            ("dft_z", T2 + U, 2 * (2 * my * mx) * (4 * mz) * (2 * n) * nb),
            ("mix", 2 * U + 2 * Q * W * W * f, 8 * Q * W * W * B),
            ("idft_x", U + I1, 2 * (4 * mz * my) * (2 * n) * (2 * mx) * nb),
            ("idft_y", I1 + I2, 2 * (n * 2 * mz) * (2 * n) * (4 * my) * nb),
            # last stage: reads I2 and z, writes z and h = GELU(z)
            ("idft_z_gelu", I2 + 2 * vol + hb, 2 * n2 * n * (4 * mz) * nb),
        ]
    rows.append(("project", hb + B * P * f, 2 * W * P * B))
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--width", type=int, default=32)
    ap.add_argument("--layers", type=int, default=4)
    ap.add_argument("--modes", type=int, default=8)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args(argv)
    import torch
    from . import surrogate as sg
    if not torch.cuda.is_available():
        sys.exit("surrogate_bench needs a GPU")
    dev = torch.device("cuda:0")
    n, W, L, m, B = args.n, args.width, args.layers, args.modes, args.batch
    model = sg.Surrogate(n=n, cin=4, width=W, layers=L, mx=m, my=m, mz=m, loss_focus=10.0)
    gen = torch.Generator(device=dev).manual_seed(0)
    params = model.init_params(0)
    x = torch.randn((B, 4, n, n, n), device=dev, generator=gen)
    target = 0.1 * torch.randn((B, 1, n, n, n), device=dev, generator=gen)
    y = torch.empty((B, 1, n, n, n), device=dev)
    st = model.train_state(params.clone())
    model.forward(params, x, y)
    model.train_step(st, x, target, lr=1e-4)
    torch.cuda.synchronize()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.reps

    fwd_ms = timed(lambda: model.forward(params, x, y))
    train_ms = timed(lambda: model.train_step(st, x, target, lr=1e-4, sync=False))
    rows = forward_counts(n, 4, W, L, m, m, m, B)
    fbytes = sum(r[1] for r in rows)
    fflops = sum(r[2] for r in rows)
    gbs = fbytes / (fwd_ms * 1e-3) / 1e9
    tfl = fflops / (fwd_ms * 1e-3) / 1e12
    out = {"metric": "surrogate samples/s", "n": n, "width": W, "layers": L, "modes": m,
           "batch": B, "params": model.n_params, "reps": args.reps,
           "forward_ms": round(fwd_ms, 4), "forward_samples_per_s": round(B / fwd_ms * 1e3, 1),
           "train_step_ms": round(train_ms, 4),
           "train_samples_per_s": round(B / train_ms * 1e3, 1),
           "forward_roofline": {"algorithmic_bytes": int(fbytes), "flops": int(fflops),
                                "achieved_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                                "achieved_tflops": round(tfl, 2),
                                "bf16_frac": round(tfl / BF16_PEAK_TFLOPS, 5),
                                "flop_per_byte": round(fflops / fbytes, 2)},
           "forward_launches": {k: {"bytes": int(b), "flops": int(fl)} for k, b, fl in rows[:9]}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
