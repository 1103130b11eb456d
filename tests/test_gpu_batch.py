"""Batched sweeps (uneven sizes, frequencies and step counts in one captured
persistent launch) against the same problems solved one by one."""
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2301_12727_amd as bb
import synth

from ._parity import assert_map_matches

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def uneven_cases():
    freqs = (250e3, 500e3, 700e3, 500e3, 250e3)
    cases = []
    for s, f in enumerate(freqs):
        c = synth.random_small_case(40 + s, n=(24, 44), n_steps=30 + 17 * s, freq_hz=f)
        cases.append(c)
    return cases


def batch_inputs(b, cases, ws):
    mats = [torch.from_numpy(c.mat).cuda() for c in cases]
    srcs = [torch.empty((c.ny, c.nx), dtype=torch.complex64, device="cuda") for c in cases]
    for i, c in enumerate(cases):
        b.source_rayleigh(i, c.transducer, srcs[i], ws)
    peaks = [torch.empty((c.nz, c.ny, c.nx), dtype=torch.float32, device="cuda") for c in cases]
    return mats, srcs, peaks


def assert_same_map(got, ref, idx, val, ref_idx, ref_val, what):
    """Batched and single solves tile the grid differently, so a lossless-fluid
    cell may be updated by the acoustic-tile kernels in one and by the general
    kernels' acoustic branch in the other.  Both spell out the same operations
    (no compiler contraction in the step kernels), so the maps are identical
    bit for bit."""
    assert np.array_equal(got, ref), (what, float(np.abs(got.astype(np.float64) - ref).max()))
    assert idx == ref_idx and val == ref_val, what


def test_batched_equals_single_solves(tmp_path):
    cases = uneven_cases()
    say("[batch] sizes " + ", ".join(f"{c.nx}x{c.ny}x{c.nz}/{c.n_steps}" for c in cases))
    single = []
    for c in cases:
        P, idx, val, _ = bb.run_case(c)
        single.append((P.cpu().numpy(), idx, val))
    b = bb.Batch(cases)
    ws = b.workspace()
    mats, srcs, peaks = batch_inputs(b, cases, ws)
    for shape in ((4, 1024, 16), (1, 64, 4), (8, 3, 7), (2, 5000, 64), (4, 0, 8), (0, 0, 0)):
        say(f"[batch] shape {shape}")
        b.set_shape(*shape)
        b.solve(mats, srcs, peaks, ws)
        for _ in range(2):                   # replay of the captured graph
            b.solve(mats, srcs, peaks, ws)
        for i, c in enumerate(cases):
            idx, val = b.status(ws, i)
            got = peaks[i].cpu().numpy()
            assert_same_map(got, single[i][0], idx, val, single[i][1], single[i][2], (shape, i))
    cache = str(tmp_path / "tune.txt")
    best, shape = b.autotune(mats, srcs, peaks, ws, cache_path=cache, probe_steps=3)
    say(f"[batch] autotuned shape {shape}, {best:.3f} ms per 3 steps")
    assert best > 0 and os.path.exists(cache)
    b.solve(mats, srcs, peaks, ws)
    for i in range(len(cases)):
        idx, val = b.status(ws, i)
        assert_same_map(peaks[i].cpu().numpy(), single[i][0], idx, val, single[i][1],
                        single[i][2], ("tuned", i))
    # a second batch of the same size class reads the cached shape
    b2 = bb.Batch(cases)
    ws2 = b2.workspace()
    m2, s2, p2 = batch_inputs(b2, cases, ws2)
    best2, shape2 = b2.autotune(m2, s2, p2, ws2, cache_path=cache, probe_steps=3)
    assert shape2[:3] == shape[:3] and best2 == pytest.approx(best)


def test_batch_reports_per_solve_errors():
    cases = uneven_cases()[:3]
    cases[1].mat = cases[1].mat.copy()
    cases[1].mat[2, 3, 4] = cases[1].materials.shape[0]     # out-of-range index in solve 1 only
    b = bb.Batch(cases)
    ws = b.workspace()
    mats, srcs, peaks = batch_inputs(b, cases, ws)
    b.solve(mats, srcs, peaks, ws)
    b.status(ws, 0)
    b.status(ws, 2)
    with pytest.raises(bb.BBFDError) as e:
        b.status(ws, 1)
    assert e.value.code == bb.EINDEX


def test_batched_maps_match_oracle():
    """Every solve of the uneven five-solve batch (sizes 24-44, 250/500/700
    kHz, 30-98 steps) against the FP64 oracle, to the single-solve bar."""
    cases = uneven_cases()
    b = bb.Batch(cases)
    ws = b.workspace()
    mats, srcs, peaks = batch_inputs(b, cases, ws)
    b.solve(mats, srcs, peaks, ws)
    for i, c in enumerate(cases):
        idx, _ = b.status(ws, i)
        ref, ridx, _ = oracle.solve_case(c)
        assert_map_matches(peaks[i].cpu().numpy(), ref, idx, ridx, c.pml, f"batch solve {i}")


def test_sweep_generator_cases_against_oracle():
    """Three solves of the sweep generator (96-160 cells per axis, tilted
    bowls, 250/500/700 kHz, skull shells at each solve's own dx) in one batch,
    each against the FP64 oracle.  Step counts are cut to 150/190/230 (still
    uneven) so the oracle finishes in seconds; by then the wave has crossed
    the near skull wall in every solve."""
    cases = synth.batch_cases(n=3)
    for s, c in enumerate(cases):
        c.n_steps = 150 + 40 * s
    say_sizes = ", ".join(f"{c.nx}x{c.ny}x{c.nz}@{c.freq_hz / 1e3:.0f}kHz/{c.n_steps}" for c in cases)
    say(f"[batch] sweep cases {say_sizes}")
    b = bb.Batch(cases)
    ws = b.workspace()
    mats, srcs, peaks = batch_inputs(b, cases, ws)
    b.solve(mats, srcs, peaks, ws)
    for i, c in enumerate(cases):
        idx, _ = b.status(ws, i)
        ref, ridx, secs = oracle.solve_case(c)
        say(f"[batch] oracle solve {i}: {secs:.1f} s")
        assert_map_matches(peaks[i].cpu().numpy(), ref, idx, ridx, c.pml, f"sweep solve {i}")


def test_back_to_back_batches_keep_their_own_pointers():
    """Two batched solves of the same batch with different output buffers,
    enqueued back to back without a synchronisation in between (the second
    one captures a new graph while the first may still be queued): each map
    equals the single-solve result.  Guards the host staging that the
    captured table uploads read."""
    cases = uneven_cases()[:3]
    single = []
    for c in cases:
        P, idx, val, _ = bb.run_case(c)
        single.append((P.cpu().numpy(), idx, val))
    b = bb.Batch(cases)
    ws_a = b.workspace()
    ws_b = b.workspace()
    mats, srcs, peaks_a = batch_inputs(b, cases, ws_a)
    peaks_b = [torch.empty_like(p) for p in peaks_a]
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    # a long queue ahead of both so the first graph is still pending when the
    # second pointer set is staged
    big = torch.empty(1 << 26, device="cuda")
    for _ in range(20):
        big.mul_(1.0)
    b.solve(mats, srcs, peaks_a, ws_a, stream=stream)
    b.solve(mats, srcs, peaks_b, ws_b, stream=stream)
    for i in range(len(cases)):
        for ws, peaks, tag in ((ws_a, peaks_a, "a"), (ws_b, peaks_b, "b")):
            idx, val = b.status(ws, i)
            assert_same_map(peaks[i].cpu().numpy(), single[i][0], idx, val, single[i][1],
                            single[i][2], (tag, i))


def _deep_case(blob_x, src_k=-1):
    """A 128 x 64 x 70 water grid with a solid blob: over 2048 tiles, so its
    single solve runs the fused step of deep tiles in two captured branches."""
    nx, ny, nz, pml, f = 128, 64, 70, 4, 500e3
    mats = synth._rows(synth.table1(f)["water"], (1850.0, 2700.0, 1300.0, 80.0, 200.0))
    mat = np.zeros((nz, ny, nx), dtype=np.uint8)
    mat[20:26, 8:18, blob_x[0]:blob_x[1]] = 1
    case = synth.Case("deep", nx, ny, nz, pml, f, 6.0, 70, mats, mat, None)
    case.source_k = src_k
    dx, zs = case.dx, case.source_plane_z()
    radius = 0.3 * min(nx, ny) * dx
    focal = 2.4 * radius
    fz = synth.bowl_focus_for_standoff(zs, radius, focal, (0.0, 0.0, 1.0), 2e-3)
    case.transducer = synth.Transducer(1, radius, focal, (nx // 2 * dx, ny // 2 * dx, fz - focal),
                                       (0.0, 0.0, 1.0))
    return case


def test_per_solve_shape_equals_single_solves_with_fused_steps():
    """The per-solve batch shape on solves large enough for the fused step of
    deep tiles and the two-branch capture (and one with the source plane moved
    inside): each solve's own step kernels in the batch graph give the single
    solves' maps bit for bit, over graph replays; the tiled shape (no fused
    step) gives them too."""
    cases = [_deep_case((70, 90)), _deep_case((20, 40), src_k=16), _deep_case((40, 60))]
    single = []
    for c in cases:
        P, idx, val, plan = bb.run_case(c)
        single.append((P.cpu().numpy(), idx, val))
    b = bb.Batch(cases)
    ws = b.workspace()
    mats, srcs, peaks = batch_inputs(b, cases, ws)
    for shape in ((0, 0, 0), (4, 0, 8)):
        b.set_shape(*shape)
        assert b.info()[1][0] == shape[0]
        for _ in range(3):                    # capture, then replays
            b.solve(mats, srcs, peaks, ws)
        for i in range(len(cases)):
            idx, val = b.status(ws, i)
            assert_same_map(peaks[i].cpu().numpy(), single[i][0], idx, val, single[i][1],
                            single[i][2], (shape, i))
