"""Benchmark: whole-solve throughput of the viscoelastic FDTD hot path on one GPU.

A step is one pass of the hot path over the workload: Rayleigh source plane,
full time loop (velocity, stress + memory variables, absorbing layer, soft
source, peak capture) and the peak-voxel reduction, with the plan (material
tables, time step, layer profile) built once beforehand and the inputs already
resident in HBM.  Default workload: 400x400x520 skull at 700 kHz, PPW 9, 5000
time steps.

Prints one JSON line: Gcell-updates/s, the dominant kernel's roofline (its
algorithmic bytes over its HIP-event-timed average launch), and the FP64 oracle
timed on the host cores over a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2301_12727_amd", "csrc", f)
                  for f in ("fdtd.hip", "bbfd_dev.h")]

WORKLOADS = {
    "skull400": lambda: __import__("synth").skull400(),
    "skull200": lambda: __import__("synth").skull200(),
    "plate64": lambda: __import__("synth").plate_case(),
    "skull200_ct12": lambda: __import__("synth").ct_case(__import__("synth").skull200(), 1),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the step kernels' sources with comments and blank lines removed,
    so that the stored traffic counters stay valid across comment edits and go
    stale on any change of the code itself."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, encoding="utf-8") as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            line = line.split("//", 1)[0].strip()
            if line:
                h.update(line.encode() + b"\n")
    return h.hexdigest()[:16]


KERNELS = ("velocity_ac", "velocity", "stress_ac", "stress", "step_deep")
REACH = 3   # cells around a deep tile that its fused step reads
LARGE_TILES = 2048   # plans with fewer tiles run no fused step


def keep_flags(classes):
    """Segment keep flags [nz][ny][nseg]: an acoustic segment within rows j-2..j+1
    or planes k-2..k+1 of an elastic (class 0) segment of the same x segment
    stores sigma_yy and sigma_zz too (the elastic one reads them)."""
    import numpy as np
    el = classes == 0
    near = np.zeros_like(el)
    for d in (-2, -1, 0, 1):
        if d < 0:
            near[:, -d:] |= el[:, :d]
            near[-d:] |= el[:d]
        elif d > 0:
            near[:, :-d] |= el[:, d:]
            near[:-d] |= el[d:]
        else:
            near |= el
    return near


def tile_kinds(case, info, classes):
    """Kind of every tile as the library assigns it: 0 general, 1 acoustic,
    2 deep: an acoustic tile whose rows and planes, with REACH around them, lie
    inside the grid and outside the layer, whose recomputed x faces beyond its
    segment (i0-2, i0-1, i0+64) are outside the grid or outside the x layer,
    whose reach inside the grid holds
    its fluid only (segment classes one row and one plane around it, the
    material map for the third cell in x) and whose sigma_yy / sigma_zz no
    elastic segment reads (keep flags 0); plans of fewer than LARGE_TILES
    tiles have no deep tiles.  Returns kinds [nz-chunks][row blocks][segments]."""
    import numpy as np
    nx, ny, nz, L = case.nx, case.ny, case.nz, case.pml
    R, K = int(info["tile_rows"]), int(info["tile_planes"])
    seg = classes != 0
    keep = keep_flags(classes)
    nseg = seg.shape[2]
    nby, nzc = -(-ny // R), -(-nz // K)
    pad = np.ones((nzc * K, nby * R, nseg), dtype=bool)
    pad[:nz, :ny] = seg
    kind = pad.reshape(nzc, K, nby, R, nseg).all(axis=(1, 3)).astype(np.int8)
    if kind.size < LARGE_TILES:     # small plans do not launch the fused step
        return kind
    for kc, by, bx in zip(*np.nonzero(kind)):
        i0, j0, k0 = 64 * bx, R * by, K * kc
        k1 = min(k0 + K, nz)
        face_ok = lambda p: p < 0 or p >= nx or L <= p < nx - L
        x_ok = face_ok(i0 - 2) and face_ok(i0 - 1) and face_ok(i0 + 64)
        if not (x_ok and j0 - REACH >= L and j0 + R - 1 + REACH < ny - L
                and k0 - REACH >= L and k1 - 1 + REACH < nz - L):
            continue
        c = classes[k0, j0, bx]
        if not (classes[k0 - 1:k1 + 1, j0 - 1:j0 + R + 1, bx] == c).all():
            continue
        if keep[k0:k1, j0:j0 + R, bx].any():
            continue
        xs = [x for x in (i0 - REACH, i0 + 63 + REACH) if 0 <= x < nx]
        shell = case.mat[k0 - REACH:k1 + REACH, j0 - REACH:j0 + R + REACH, xs]
        if (shell == c - 1).all():
            kind[kc, by, bx] = 2
    return kind


def algorithmic_bytes(case, info, classes, capture_share=None) -> dict:
    """Bytes each step kernel must move per launch at perfect on-chip reuse
    (FP32 state, 1-byte index), averaged over the time loop.  ``classes`` is
    the library's row-segment class map: cells of class > 0 are acoustic (one
    lossless fluid throughout the stencil's reach).  Tiles (64 x tile_rows x
    tile_planes cells) run by kind (see tile_kinds): deep tiles the fused step,
    other acoustic tiles the *_ac kernels, the rest the general ones.
      velocity, elastic cell: read 6 stresses + 3 velocities + index, write 3
                velocities = 49 B; acoustic cell: read 1 normal stress + 3
                velocities, write 3 velocities = 28 B.  Per absorbing-layer axis
                the cell lies in: 3 (elastic) or 1 (acoustic) layer memories read
                and written (8 B each).  Source plane: 8 B per column.
      stress,   elastic cell: read 3 velocities + 6 stresses + 6 memories +
                index, write 6 + 6 = 109 B; acoustic cell: read 3 velocities +
                1 normal stress, write 3 normal stresses = 28 B, or only sigma_xx
                (20 B) in an acoustic tile where no elastic segment within 2 rows
                or planes reads sigma_yy / sigma_zz (keep flag).  Layer memories
                as above.  Capture steps add 8 B/cell (peak read + write).
      step_deep, fused velocity + stress of a deep tile: read sigma_xx and 3
                velocities, write them = 32 B per cell; cells in the x layer
                also read and write the two x memories (16 B); + capture as
                above."""
    import numpy as np
    nx, ny, nz, L = case.nx, case.ny, case.nz, case.pml
    R, K = int(info["tile_rows"]), int(info["tile_planes"])
    seg = (classes != 0)
    kind = tile_kinds(case, info, classes)
    cell_kind = np.repeat(np.repeat(np.repeat(kind, K, 0)[:nz], R, 1)[:, :ny], 64, 2)[:, :, :nx]
    fluid = np.repeat(seg, 64, axis=2)[:, :, :nx]
    near = keep_flags(classes)
    keep = np.repeat(near, 64, axis=2)[:, :, :nx]
    axes_in_layer = np.zeros((nz, ny, nx), dtype=np.int8)
    for a, n in ((2, nx), (1, ny), (0, nz)):
        sl = [slice(None)] * 3
        sl[a] = np.r_[0:L, n - L:n]
        axes_in_layer[tuple(sl)] += 1
    cap = ((case.n_steps - info["capture_start"]) / case.n_steps if capture_share is None
           else capture_share)
    out = {}
    for name, mask in (("ac", cell_kind == 1), ("gen", cell_kind == 0)):
        fl = fluid & mask
        el_c = ~fluid & mask
        nf, ne = int(fl.sum()), int(el_c.sum())
        lf = int(axes_in_layer[fl].sum())
        le = int(axes_in_layer[el_c].sum())
        src_cols = int(mask[info["source_k"]].sum())
        cls_bytes = int(mask.sum()) / 64
        suffix = "_ac" if name == "ac" else ""
        out["velocity" + suffix] = 28 * nf + 49 * ne + 8 * lf + 24 * le + 8 * src_cols + cls_bytes
        # acoustic tiles store sigma_yy, sigma_zz only where kept (20 B otherwise)
        nk = int((fl & keep).sum()) if name == "ac" else nf
        out["stress" + suffix] = (20 * nf + 8 * nk + 109 * ne + 8 * lf + 24 * le
                                  + 8 * (nf + ne) * cap + cls_bytes * (2 if name == "ac" else 1))
    nd = int((cell_kind == 2).sum())
    # deep cells in the x layer also read and write two layer memories
    xlay = np.zeros(nx, dtype=bool)
    xlay[:L] = True
    xlay[nx - L:] = True
    ndl = int(((cell_kind == 2) & xlay[None, None, :]).sum())
    out["step_deep"] = 32 * nd + 16 * ndl + 8 * nd * cap + nd / 64
    out["per_cell_update"] = sum(out[k] for k in KERNELS) / case.cells
    out["acoustic_fraction"] = float(fluid.mean())
    out["acoustic_tile_fraction"] = float((cell_kind >= 1).mean())
    out["deep_tile_fraction"] = nd / case.cells
    return out


def load_traffic(kernel: str, workload: str):
    """Measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE scaled by
    a copy kernel's counters), valid only for the kernel sources it was taken on."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash() or t.get("workload") != workload:
        return None
    return t.get("kernels", {}).get(kernel)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case, sample_steps: int = 8, single_steps: int = 1) -> dict:
    """FP64 oracle on the host cores: full workload grid, one untimed step
    (first touch), then ``sample_steps`` timed steps with all threads and
    ``single_steps`` more with one thread."""
    import oracle
    prob = oracle.problem_from_case(case)
    src = oracle.source_plane(case)
    sim = oracle.Sim(prob, case.mat)
    threads = int(oracle.lib().omp_get_max_threads())
    sim.step(0, src)
    t0 = time.perf_counter()
    for n in range(1, 1 + sample_steps):
        sim.step(n, src)
    dt = time.perf_counter() - t0
    prev = oracle.set_threads(1)
    t1 = time.perf_counter()
    for n in range(1 + sample_steps, 1 + sample_steps + single_steps):
        sim.step(n, src)
    dt1 = time.perf_counter() - t1
    oracle.set_threads(prev)
    sim.close()
    return {"value": case.cells * sample_steps / dt / 1e9, "unit": "Gcell-updates/s",
            "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "single_thread_value": case.cells * single_steps / dt1 / 1e9,
            "sample": f"{case.name}: full grid, {sample_steps} time steps on {threads} threads "
                      f"after one untimed step ({dt:.1f} s), then {single_steps} on one thread "
                      f"({dt1:.1f} s); FP64, OpenMP"}


TUNE_CACHE = os.path.join(ROOT, "paper_2301_12727_amd", "tune_cache.txt")


def batched_section(bb, torch, n_solves: int = 32, repeats: int = 5) -> dict:
    """Uneven sweep (sizes 96..160 per axis, 250/500/700 kHz, tilted bowls): one
    captured persistent launch for all solves vs the same solves run one after
    another as plain captured solves (medians of ``repeats`` timings each).
    Both sides include no Rayleigh time."""
    import numpy as np
    import synth
    cases = synth.batch_cases(n_solves)
    dev = torch.device("cuda:0")
    b = bb.Batch(cases)
    ws = b.workspace(dev)
    mats = [torch.from_numpy(c.mat).to(dev) for c in cases]
    srcs = [torch.empty((c.ny, c.nx), dtype=torch.complex64, device=dev) for c in cases]
    peaks = [torch.empty((c.nz, c.ny, c.nx), dtype=torch.float32, device=dev) for c in cases]
    for i, c in enumerate(cases):
        b.source_rayleigh(i, c.transducer, srcs[i], ws)
    t0 = time.perf_counter()
    best, shape = b.autotune(mats, srcs, peaks, ws, cache_path=TUNE_CACHE, probe_steps=10)
    tune_s = time.perf_counter() - t0
    log(f"[bench] batched shape {shape} (autotune {tune_s:.1f} s)")
    b.solve(mats, srcs, peaks, ws)                     # capture + warm
    torch.cuda.synchronize()
    tb = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        b.solve(mats, srcs, peaks, ws)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
    t_batch = float(np.median(tb))
    for i in range(n_solves):
        b.status(ws, i)
    log(f"[bench] batched sweep {t_batch:.3f} s (median of {repeats}: "
        + ", ".join(f"{t:.3f}" for t in tb) + ")")
    plans = [bb.Plan.from_case(c) for c in cases]
    wss = [p.workspace(dev) for p in plans]
    seq = [torch.empty_like(p) for p in peaks]
    for p, w, m, sr, o in zip(plans, wss, mats, srcs, seq):   # capture + warm
        p.solve(m, sr, o, w)
    torch.cuda.synchronize()
    ts = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        for p, w, m, sr, o in zip(plans, wss, mats, srcs, seq):
            p.solve(m, sr, o, w)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    t_seq = float(np.median(ts))
    log("[bench] sequential repeats " + ", ".join(f"{t:.3f}" for t in ts))
    # the same captured single solves spread over 4 streams (independent solves overlap)
    streams = [torch.cuda.Stream() for _ in range(4)]
    for q, (p, w, m, sr, o) in enumerate(zip(plans, wss, mats, srcs, seq)):
        p.solve(m, sr, o, w, stream=streams[q % 4])
    torch.cuda.synchronize()
    tc = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        for q, (p, w, m, sr, o) in enumerate(zip(plans, wss, mats, srcs, seq)):
            p.solve(m, sr, o, w, stream=streams[q % 4])
        torch.cuda.synchronize()
        tc.append(time.perf_counter() - t0)
    t_con = float(np.median(tc))
    log("[bench] 4-stream repeats " + ", ".join(f"{t:.3f}" for t in tc))
    equal = all(bool(torch.equal(a, c)) for a, c in zip(peaks, seq))
    updates = sum(c.cells * c.n_steps for c in cases)
    log(f"[bench] sequential {t_seq:.3f} s; maps equal {equal}")
    return {"solves": n_solves, "batched_solves_per_s": round(n_solves / t_batch, 3),
            "sequential_solves_per_s": round(n_solves / t_seq, 3),
            "four_stream_solves_per_s": round(n_solves / t_con, 3),
            "speedup": round(t_seq / t_batch, 3),
            "batched_gcell_updates_per_s": round(updates / t_batch / 1e9, 3),
            "shape": {"rows_per_block": shape[0], "blocks": shape[1], "kchunk": shape[2],
                      "tiles": shape[3]},
            "autotune_s": round(tune_s, 2), "maps_equal_to_plain_solves": equal,
            "repeats": repeats,
            "cells": int(sum(c.cells for c in cases))}


def energy_loss_section(bb, torch, repeats: int = 3) -> dict:
    """The paper's pair of runs per target on the 200x200x280 skull at 500 kHz
    (3000 steps): the transcranial solve, its water-only companion on the same
    plan (each pointer set keeps its captured graph) and the energy loss E_L
    with T_S = sqrt(E_L) on the plane of the water field's peak.  Reports pairs
    per second (median of ``repeats``) and the reduction's own time."""
    import numpy as np
    import synth
    case = synth.skull200()
    dev = torch.device("cuda:0")
    plan = bb.Plan.from_case(case)
    ws = plan.workspace(dev)
    src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device=dev)
    plan.source_rayleigh(case.transducer, src, ws)
    ms = torch.from_numpy(case.mat).to(dev)
    mw = torch.zeros_like(ms)
    ps = torch.empty(plan.shape, dtype=torch.float32, device=dev)
    pw = torch.empty_like(ps)

    def pair():
        plan.solve(ms, src, ps, ws)
        plan.solve(mw, src, pw, ws)
        return plan.energy_loss(ms, ps, mw, pw, ws)

    res = pair()                                      # captures both graphs
    caps = plan.graph_captures
    times = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = pair()
        times.append(time.perf_counter() - t0)
    assert plan.graph_captures == caps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        plan.energy_loss(ms, ps, mw, pw, ws)
    t_red = (time.perf_counter() - t0) / 20
    t = float(np.median(times))
    log(f"[bench] E_L pair {t:.3f} s: E_L {res[0]:.4f}, T_S {res[1]:.4f}, z_m {res[2]}")
    return {"workload": case.name, "pairs_per_s": round(1.0 / t, 3), "pair_s": round(t, 4),
            "e_l": round(res[0], 6), "t_s": round(res[1], 6), "z_m": res[2],
            "reduction_ms_with_sync": round(t_red * 1e3, 4), "graph_captures": caps}


def copy_gbs(torch, n: int = 1 << 28, repeats: int = 5) -> float:
    """Bytes read + written per second of torch's device copy of n floats."""
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(repeats):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / repeats
    del a, b
    torch.cuda.empty_cache()
    return 8.0 * n / (ms * 1e-3) / 1e9


def paper_domain_section(bb, torch, repeats: int = 3) -> dict:
    """The domain the paper times its transcranial step on: 54 x 54 x 76 mm at
    600 kHz and 6 points per wavelength (130 x 130 x 182 cells plus the 8-cell
    layer), a focused bowl of 50 mm focal length at F#1 and the skull-shell
    map; one transcranial step as the paper counts it = the Rayleigh plane, the
    skull solve, its water-only companion and E_L (1200 time steps each, 52
    periods).  Reports seconds per step (median of ``repeats``); the paper's
    51-58 s on its hardware include more than these solves and are context,
    not a like-for-like target."""
    import numpy as np
    import synth
    L = 8
    case = synth.skull_case(130 + 2 * L, 130 + 2 * L, 182 + 2 * L, 600e3, 6.0, 1200, seed=3,
                            pml=L, aperture=50e-3, fnum=1.0, name="paper_domain_54x54x76mm_600kHz")
    dev = torch.device("cuda:0")
    plan = bb.Plan.from_case(case)
    ws = plan.workspace(dev)
    src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device=dev)
    ms = torch.from_numpy(case.mat).to(dev)
    mw = torch.zeros_like(ms)
    ps = torch.empty(plan.shape, dtype=torch.float32, device=dev)
    pw = torch.empty_like(ps)

    def step():
        plan.source_rayleigh(case.transducer, src, ws)
        plan.solve(ms, src, ps, ws)
        plan.solve(mw, src, pw, ws)
        return plan.energy_loss(ms, ps, mw, pw, ws)

    step()
    times = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = step()
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    log(f"[bench] paper domain {case.nx}x{case.ny}x{case.nz}: transcranial step {t:.3f} s "
        f"(T_S {res[1]:.3f})")
    return {"workload": f"{case.name} {case.nx}x{case.ny}x{case.nz}, {case.n_steps} steps",
            "transcranial_step_s": round(t, 4), "t_s": round(res[1], 5),
            "paper_gpu_only_s_context": {"M1 Max": 51, "RTX A6000": 58}}


def ct12_section(bb, torch, repeats: int = 3) -> dict:
    """The 200x200x280 skull at 500 kHz as a 12-bit CT map (uint16 indices into
    4096 rows; the general kernels stage the table's buoyancy and edge-input
    columns in LDS) against the same grid with the 10-row 8-bit table:
    Gcell-updates/s of each (median of ``repeats`` captured solves), the
    per-kernel time per step and the tile counts, and a q_c sweep (0.4, 1, 2,
    3, 4) of the 8-bit map as one batch against the same five solves one by
    one."""
    import numpy as np
    import synth
    dev = torch.device("cuda:0")
    base = synth.skull200()
    out = {}
    for name, case in (("u8", base), ("u16_ct12", synth.ct_case(base, 1))):
        plan = bb.Plan.from_case(case)
        ws = plan.workspace(dev)
        src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device=dev)
        plan.source_rayleigh(case.transducer, src, ws)
        mat = torch.from_numpy(case.mat).to(dev)
        peak = torch.empty(plan.shape, dtype=torch.float32, device=dev)
        plan.solve(mat, src, peak, ws)
        plan.status(ws)
        ts = []
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.solve(mat, src, peak, ws)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        t = float(np.median(ts))
        kms = plan.solve_profiled(mat, src, peak, ws)
        out[name] = {"gcell_updates_per_s": round(case.cells * case.n_steps / t / 1e9, 2),
                     "levels_in_map": int(len(np.unique(case.mat))),
                     "table_rows": int(case.materials.shape[0]),
                     "kernel_ms_per_step": {f"k_{k}": round(m / case.n_steps, 4)
                                            for k, m in zip(KERNELS, kms)},
                     "tiles_acoustic_general_deep": list(plan.tile_counts(ws))}
        del ws, peak
        torch.cuda.empty_cache()
    qcs = (0.4, 1.0, 2.0, 3.0, 4.0)
    cases = [synth.Case(**{**base.__dict__, "qc": q, "name": f"qc{q}"}) for q in qcs]
    b = bb.Batch(cases)
    ws = b.workspace(dev)
    mat = torch.from_numpy(base.mat).to(dev)
    srcs = [torch.empty((base.ny, base.nx), dtype=torch.complex64, device=dev) for _ in cases]
    peaks = [torch.empty((base.nz, base.ny, base.nx), dtype=torch.float32, device=dev)
             for _ in cases]
    for i, c in enumerate(cases):
        b.source_rayleigh(i, c.transducer, srcs[i], ws)
    t0 = time.perf_counter()
    _, qshape = b.autotune([mat] * len(cases), srcs, peaks, ws, probe_steps=10)
    t_tune = time.perf_counter() - t0
    b.solve([mat] * len(cases), srcs, peaks, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.solve([mat] * len(cases), srcs, peaks, ws)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    del ws
    torch.cuda.empty_cache()
    plans = [bb.Plan.from_case(c) for c in cases]
    wss = [p.workspace(dev) for p in plans[:1]]
    seq = torch.empty_like(peaks[0])
    for p in plans:
        p.solve(mat, srcs[0], seq, wss[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p in plans:
        p.solve(mat, srcs[0], seq, wss[0])
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    out["qc_sweep"] = {"qc": list(qcs), "batched_s": round(t_b, 4), "sequential_s": round(t_s, 4),
                       "speedup": round(t_s / t_b, 3),
                       "shape": dict(zip(("rows_per_block", "blocks", "kchunk", "tiles"), qshape)),
                       "autotune_s": round(t_tune, 2)}
    log(f"[bench] ct12 {out['u16_ct12']['gcell_updates_per_s']} vs u8 {out['u8']['gcell_updates_per_s']} "
        f"Gcell/s; qc sweep batched {t_b:.3f} s vs {t_s:.3f} s")
    return out


def array_section(bb, torch) -> dict:
    """Refocusing the paper's 128-element device (F 135 mm, F#0.9, 250 kHz;
    synth.DEVICES["H317"]) through a head-scale skull (176x176x181 cells of 1
    mm) on its geometric focus (time reversal: two point-source solves recording
    the source plane, back-propagation to the elements), then the forward field
    of the refocused and of the geometrically steered drives; reports the
    times and the pressure each puts on the target."""
    import numpy as np
    import synth
    dev = torch.device("cuda:0")
    case, rows, cell = synth.device_case("H317", 250e3)
    plan = bb.Plan.from_case(case)
    ws = plan.workspace(dev)
    mat = torch.from_numpy(case.mat).to(dev)
    peak = torch.empty(plan.shape, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w_tr, _ = plan.array_refocus(mat, rows, cell, peak, ws)
    t_ref = time.perf_counter() - t0
    i, j, k = cell
    res = {"workload": f"{case.name} {case.nx}x{case.ny}x{case.nz}, {case.n_steps} steps",
           "elements": len(rows), "target_cell": list(cell), "refocus_s": round(t_ref, 4)}
    for name, w in (("steered", plan.array_steer(rows, np.array(cell) * case.dx)),
                    ("refocused", w_tr)):
        drv = np.array(rows)
        drv[:, 7], drv[:, 8] = w.real, w.imag
        src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.array_rayleigh(drv, src, ws)
        plan.solve(mat, src, peak, ws, graph=False)
        plan.status(ws)
        res[f"{name}_forward_s"] = round(time.perf_counter() - t0, 4)
        res[f"{name}_target_pa"] = float(peak[k, j, i])
    res["gain"] = round(res["refocused_target_pa"] / res["steered_target_pa"], 4)
    log(f"[bench] array refocus {t_ref:.3f} s; target gain {res['gain']}")
    return res


BHTE_BYTES_PER_CELL_UPDATE = 29   # theta in/out, Q, material byte, max and dose in/out


def thermal_section(bb, torch, repeats: int = 3) -> dict:
    """Thermal step (BHTE) on the 200x200x280 skull at 500 kHz: the acoustic
    peak map of the transcranial solve, scaled so that the brain's spatial-peak
    intensity is the paper's default 5 W/cm^2, heats for 40 s at 30 % duty
    cycle and cools for 20 s (dt = 0.1 s, 600 steps).  Reports Gcell-updates/s
    of the thermal loop (median of ``repeats``) and its HBM rate at 29 B per
    cell update."""
    import numpy as np
    import synth
    from paper_2301_12727_amd.thermal import Thermal
    case = synth.skull200()
    dev = torch.device("cuda:0")
    plan = bb.Plan.from_case(case)
    ws = plan.workspace(dev)
    src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device=dev)
    plan.source_rayleigh(case.transducer, src, ws)
    mat = torch.from_numpy(case.mat).to(dev)
    peak = torch.empty(plan.shape, dtype=torch.float32, device=dev)
    plan.solve(mat, src, peak, ws, graph=False)  # direct launches: the BHTE loop is timed
    plan.status(ws)
    del ws
    ac, th = synth.thermal_materials(case.freq_hz)
    brain = torch.from_numpy(np.ascontiguousarray(case.mat == 0)).to(dev)
    L = case.pml
    brain[:L + 30] = False          # beyond the near skull wall
    inten = peak.double() ** 2 / (2.0 * ac[0, 0] * ac[0, 1])
    scale = 5e4 / float(torch.where(brain, inten, torch.zeros_like(inten)).max())
    n_on, n_off, dt = 400, 200, 0.1
    tp = Thermal(plan.shape, case.dx, dt, ac, th, n_on, n_off, duty=0.3, intensity_scale=scale)
    tws = tp.workspace(dev)
    outs = [torch.empty(plan.shape, dtype=torch.float32, device=dev) for _ in range(3)]
    tp.run(mat, peak, *outs, tws)
    torch.cuda.synchronize()
    times = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        tp.run(mat, peak, *outs, tws)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    updates = case.cells * (n_on + n_off)
    g = updates / t / 1e9
    t_max, dose = float(outs[1].max()), float(outs[2].max())
    log(f"[bench] BHTE {t:.3f} s: {g:.1f} Gcell-updates/s, T_max {t_max:.2f} C, dose {dose:.3g} min")
    return {"workload": f"{case.name} thermal, {n_on}+{n_off} steps of {dt} s, duty 0.3, "
                        f"I_SPPA-brain 5 W/cm^2",
            "gcell_updates_per_s": round(g, 2), "seconds": round(t, 4),
            "hbm_gbs_at_29B": round(g * BHTE_BYTES_PER_CELL_UPDATE, 1),
            "frac_of_8TBs": round(g * BHTE_BYTES_PER_CELL_UPDATE / HBM_PEAK_GBS, 4),
            "t_max_c": round(t_max, 3), "dose_max_min": dose, "intensity_scale": scale}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="skull400", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-sweep section")
    ap.add_argument("--only", default=None,
                    help="comma-separated sections to run alone (batched, energy_loss, thermal, "
                         "ct12, paper_domain, phased_array), printing their JSON (for profiling)")
    ap.add_argument("--time-steps", type=int, default=None,
                    help="override the workload's time-step count (short profiling runs)")
    ap.add_argument("--capture-start", type=int, default=None,
                    help="override the first captured step (counter runs: n_steps leaves one "
                         "capture launch, so the per-dispatch medians are capture-free)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (PMC byte-counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(see the sharding design); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2301_12727_amd as bb

    if args.only:
        sections = {"batched": batched_section, "energy_loss": energy_loss_section,
                    "thermal": thermal_section, "ct12": ct12_section,
                    "paper_domain": paper_domain_section, "phased_array": array_section}
        res = {}
        for name in args.only.split(","):
            res[name] = sections[name](bb, torch)
            torch.cuda.empty_cache()
        print(json.dumps(res))
        return

    if args.calibrate_copy:
        n = 1 << 28                       # 2^28 floats = 1 GiB read + 1 GiB written
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        # a second, independent calibration: a read-only reduction of the same 1 GiB
        tot = a.sum()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(5):
            tot = a.sum()
        e1.record()
        torch.cuda.synchronize()
        ms_r = e0.elapsed_time(e1) / 5
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "repeats": 6,
                          "copy_ms": round(ms, 4), "copy_gbs": round(8 * n / ms / 1e6, 1),
                          "sum_bytes_read": 4 * n, "sum_ms": round(ms_r, 4),
                          "sum_gbs": round(4 * n / ms_r / 1e6, 1), "sum": float(tot)}))
        return

    case = WORKLOADS[args.workload]()
    if args.time_steps:
        case.n_steps = args.time_steps
    if args.capture_start is not None:
        case.capture_start = args.capture_start
    log(f"[bench] workload {case.name}: {case.nx}x{case.ny}x{case.nz}, {case.n_steps} steps")
    plan = bb.Plan.from_case(case)
    info = plan.info
    dev = torch.device("cuda:0")
    ws = plan.workspace(dev)
    mat = torch.from_numpy(case.mat).to(dev)
    src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device=dev)
    peak = torch.empty(plan.shape, dtype=torch.float32, device=dev)

    def step():
        plan.source_rayleigh(case.transducer, src, ws)
        plan.solve(mat, src, peak, ws)

    first_s = None
    for w in range(args.warmup):
        t0 = time.perf_counter()
        step()
        plan.status(ws)
        if w == 0:
            first_s = time.perf_counter() - t0   # includes capturing and instantiating the graph
        log(f"[bench] warmup {w} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pidx, pval = plan.status(ws)
    log(f"[bench] timed {args.steps} steps in {elapsed:.3f} s; peak voxel {pidx} ({pval:.4e} Pa)")
    updates = case.cells * case.n_steps
    value = args.steps * updates / elapsed / 1e9

    # dominant kernel: per-launch HIP events on the launch stream
    ms = plan.solve_profiled(mat, src, peak, ws)
    pidx2, _ = plan.status(ws)
    assert pidx2 == pidx
    classes = plan.segment_classes(ws)
    ab = algorithmic_bytes(case, info, classes)
    # the byte model's tile kinds must be the library's own
    kinds = tile_kinds(case, info, classes)
    counts = plan.tile_counts(ws)
    if counts != tuple(int((kinds == k).sum()) for k in (1, 0, 2)):
        raise RuntimeError(f"byte model tile kinds disagree with the library: {counts}")
    avg = {k: m / case.n_steps for k, m in zip(KERNELS, ms)}
    dom = max(KERNELS, key=lambda k: avg[k])
    achieved = ab[dom] / (avg[dom] * 1e-3) / 1e9
    log("[bench] kernel avg ms: " + ", ".join(f"{k} {avg[k]:.4f}" for k in KERNELS))
    traffic = load_traffic(dom, case.name)
    # measured traffic comes from capture-free launches: compare it with the
    # algorithmic bytes of a capture-free launch
    ab0 = algorithmic_bytes(case, info, classes, capture_share=0.0)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "algorithmic_bytes_capture_free_launch": int(ab0[dom]),
            "traffic_over_algorithmic": (round(traffic / ab0[dom], 3) if traffic else None),
            "kernel": f"k_{dom}", "avg_launch_ms": round(avg[dom], 5),
            "algorithmic_bytes_per_launch": int(ab[dom]),
            "kernels": {f"k_{k}": {"avg_launch_ms": round(avg[k], 5),
                                   "algorithmic_bytes": int(ab[k]),
                                   "achieved_gbs": round(ab[k] / (avg[k] * 1e-3) / 1e9, 1)
                                   if avg[k] > 0 else None} for k in KERNELS},
            "step_achieved_gbs": round(sum(ab[k] for k in KERNELS)
                                       / (sum(avg.values()) * 1e-3) / 1e9, 1),
            "bytes_per_cell_update": round(ab["per_cell_update"], 2),
            "acoustic_cell_fraction": round(ab["acoustic_fraction"], 4),
            "acoustic_tile_cell_fraction": round(ab["acoustic_tile_fraction"], 4),
            "deep_tile_cell_fraction": round(ab["deep_tile_fraction"], 4),
            "tiles_acoustic_general_deep": list(counts)}
    # the runtime's own device copy of 1 GiB on the same box, for scale
    cp = copy_gbs(torch)
    measured_rate = (traffic / (avg[dom] * 1e-3) / 1e9) if traffic else None
    roof["stream_copy_gbs"] = round(cp, 1)
    roof["frac_of_stream_copy"] = round(achieved / cp, 3)
    roof["measured_traffic_gbs"] = round(measured_rate, 1) if measured_rate else None

    out = {
        "metric": "Gcell-updates/s",
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": case.name, "grid": [case.nx, case.ny, case.nz],
                   "time_steps": case.n_steps, "freq_hz": case.freq_hz, "ppw": case.ppw,
                   "pml": case.pml, "materials": int(case.materials.shape[0])},
        "effective_hbm_gbs": round(value * ab["per_cell_update"], 1),
        "first_solve_s": None if first_s is None else round(first_s, 3),
        "roofline": roof,
    }
    del ws, mat, src, peak
    torch.cuda.empty_cache()
    out["batched"] = None if args.no_batch else batched_section(bb, torch)
    torch.cuda.empty_cache()
    out["energy_loss"] = None if args.no_batch else energy_loss_section(bb, torch)
    torch.cuda.empty_cache()
    out["thermal"] = None if args.no_batch else thermal_section(bb, torch)
    torch.cuda.empty_cache()
    out["ct12"] = None if args.no_batch else ct12_section(bb, torch)
    out["paper_domain"] = None if args.no_batch else paper_domain_section(bb, torch)
    torch.cuda.empty_cache()
    out["phased_array"] = None if args.no_batch else array_section(bb, torch)
    torch.cuda.empty_cache()
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_steps)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
