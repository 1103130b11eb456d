"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bar: relative L2 error of the peak-pressure map over the interior outside the
absorbing layer <= 2e-4 and the same peak voxel (ties: the oracle's runner-up
within 1e-5 relative); Rayleigh source plane rel-L2 <= 1e-5.
"""
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2301_12727_amd as bb
import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "skull200_oracle.npz")
GOLDEN400 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                         "skull400_short_oracle.npz")
TOL_MAP = 2e-4
TOL_SRC = 1e-5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_err_complex(a, ref):
    a = np.asarray(a, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


def interior(P, L):
    return P[L:P.shape[0] - L, L:P.shape[1] - L, L:P.shape[2] - L]


def assert_same_peak(gpu_idx, ref_idx, ref_map, L):
    if gpu_idx == ref_idx:
        return
    # accept only a tie inside the oracle's own 1e-5 relative margin
    v_ref = ref_map.flat[ref_idx]
    v_alt = ref_map.flat[gpu_idx]
    assert abs(v_ref - v_alt) <= 1e-5 * v_ref, (gpu_idx, ref_idx, v_ref, v_alt)


def compare_case(case, n_steps=None):
    say(f"[parity] {case.name} {case.nx}x{case.ny}x{case.nz} steps {n_steps or case.n_steps}")
    P, idx, val, plan = bb.run_case(case, n_steps=n_steps)
    P = P.cpu().numpy()
    ref, ridx, _ = oracle.solve_case(case, n_steps=n_steps)
    L = case.pml
    err = rel_l2(interior(P, L), interior(ref, L))
    say(f"[parity] {case.name}: rel-L2 {err:.3e}, peak {idx} vs {ridx}")
    assert err <= TOL_MAP
    assert_same_peak(idx, ridx, ref, L)
    assert val == pytest.approx(P.flat[idx])
    return P, ref


@pytest.mark.parametrize("which", ["plate", "skull200", "tilted"])
def test_rayleigh_plane_matches_oracle(which):
    case = {"plate": lambda: synth.plate_case(),
            "skull200": lambda: synth.skull200(build_map=False),
            "tilted": lambda: synth.batch_cases(2, build_map=False)[1]}[which]()
    say(f"[rayleigh] {which}")
    plan = bb.Plan.from_case(case, n_steps=10)
    ws = plan.workspace()
    src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device="cuda")
    plan.source_rayleigh(case.transducer, src, ws)
    torch.cuda.synchronize()
    ref = oracle.source_plane(case)
    err = rel_err_complex(src.cpu().numpy(), ref)
    say(f"[rayleigh] {which}: rel-L2 {err:.3e}")
    assert err <= TOL_SRC


def test_rayleigh_volume_matches_oracle():
    """Free field of a focused bowl at every cell centre (i, j, k) dx of a
    ragged 50 x 37 x 45 grid against the oracle's Rayleigh sum over the same
    elements, on every plane (the bowl sits just below plane 0, so the first
    planes hold its near field)."""
    nx, ny, nz, pml, f = 50, 37, 45, 4, 500e3
    mats = synth._rows(synth.table1(f)["water"])
    case = synth.Case("volume", nx, ny, nz, pml, f, 6.0, 10, mats, None, None)
    dx, zs = case.dx, case.source_plane_z()
    radius = 0.3 * min(nx, ny) * dx
    focal = 2.4 * radius
    fz = synth.bowl_focus_for_standoff(zs, radius, focal, (0.0, 0.0, 1.0), 2e-3)
    case.transducer = synth.Transducer(1, radius, focal, (nx // 2 * dx, ny // 2 * dx, fz - focal),
                                       (0.0, 0.0, 1.0))
    plan = bb.Plan.from_case(case)
    ws = plan.workspace()
    field = torch.empty((nz, ny, nx), dtype=torch.complex64, device="cuda")
    plan.rayleigh_volume(case.transducer, field, ws)
    torch.cuda.synchronize()
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pts = np.stack([ii * dx, jj * dx, kk * dx], axis=-1)
    el = oracle.elements(case.transducer, f)
    ref = oracle.rayleigh(el, f, case.transducer.u0, pts).reshape(kk.shape)
    got = field.cpu().numpy()
    err = rel_err_complex(got, ref)
    far = rel_err_complex(got[nz // 2:], ref[nz // 2:])
    say(f"[rayleigh] volume {nx}x{ny}x{nz}: rel-L2 {err:.3e}, upper half {far:.3e}")
    assert err <= TOL_SRC and far <= TOL_SRC


@pytest.mark.parametrize("seed", range(6))
def test_random_heterogeneous_grids(seed):
    case = synth.random_small_case(seed, n_steps=90)
    compare_case(case)


def test_plate64_full():
    compare_case(synth.plate_case())


def test_ragged_sizes_and_thin_layer():
    # x not a multiple of the 64-wide tile, y not a multiple of 4, odd z
    case = synth.random_small_case(11, n=(17, 17), pml=2, n_steps=60)
    case.nx, case.ny, case.nz = case.mat.shape[2], case.mat.shape[1], case.mat.shape[0]
    compare_case(case)
    case = synth.random_small_case(12, n=(65, 71), pml=8, n_steps=40)
    compare_case(case)


def test_no_layer_and_few_steps():
    case = synth.random_small_case(5, pml=0, n_steps=3)   # the ramp is 0 at step 0
    case.capture_start = 0
    compare_case(case)
    case = synth.random_small_case(6, pml=3, n_steps=30)
    case.capture_start = 0
    case.source_k = 10
    compare_case(case)


def test_graph_replay_is_bitwise_equal_to_direct_and_deterministic():
    case = synth.random_small_case(2, n_steps=70)
    plan = bb.Plan.from_case(case)
    ws = plan.workspace()
    src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device="cuda")
    plan.source_rayleigh(case.transducer, src, ws)
    mat = torch.from_numpy(case.mat).cuda()
    outs = []
    for graph in (True, True, False):
        peak = torch.empty(plan.shape, dtype=torch.float32, device="cuda")
        for _ in range(2):     # second call replays the captured graph
            plan.solve(mat, src, peak, ws, graph=graph)
            torch.cuda.synchronize()
        plan.status(ws)
        outs.append(peak.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[2])



def test_two_branch_graph_replays_match_direct_solve():
    """A plan with over 2048 tiles captures each step as two branches on a
    second stream.  Replays of that graph, with eager work on the same tensors
    in between (the peak map overwritten, and a direct solve with another
    source plane leaving its own state in the workspace), give the
    direct-launch map bit for bit every time."""
    nx, ny, nz, pml, f = 128, 64, 70, 4, 500e3
    mats = synth._rows(synth.table1(f)["water"], (1850.0, 2700.0, 1300.0, 80.0, 200.0))
    mat = np.zeros((nz, ny, nx), dtype=np.uint8)
    mat[20:26, 8:18, 70:90] = 1
    case = synth.Case("branches", nx, ny, nz, pml, f, 6.0, 60, mats, mat, None)
    case.capture_start = 0
    plan = bb.Plan.from_case(case)
    ws = plan.workspace()
    rng = np.random.default_rng(4)
    plane = np.zeros((ny, nx), dtype=np.complex64)
    plane[20:44, 40:88] = rng.normal(size=(24, 48)) + 1j * rng.normal(size=(24, 48))
    src = torch.from_numpy(plane).cuda()
    mat_d = torch.from_numpy(mat).cuda()
    peak = torch.empty(plan.shape, dtype=torch.float32, device="cuda")
    plan.solve(mat_d, src, peak, ws, graph=False)
    plan.status(ws)
    direct = peak.cpu().numpy()
    counts = plan.tile_counts(ws)
    assert sum(counts) >= 2048 and counts[2] > 0
    other = torch.roll(src, (5, -9), (0, 1)) * 3.0
    scratch = torch.empty_like(peak)
    for r in range(3):
        plan.solve(mat_d, other, scratch, ws, graph=False)
        plan.status(ws)
        peak.fill_(float(r + 7))
        torch.cuda.synchronize()
        plan.solve(mat_d, src, peak, ws)
        plan.status(ws)
        got = peak.cpu().numpy()
        say(f"[parity] two-branch graph replay {r}: max |diff| {np.abs(got - direct).max()}")
        assert np.array_equal(got, direct)


def test_linear_in_source():
    case = synth.random_small_case(4, n_steps=80)
    plan = bb.Plan.from_case(case)
    ws = plan.workspace()
    src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device="cuda")
    plan.source_rayleigh(case.transducer, src, ws)
    mat = torch.from_numpy(case.mat).cuda()
    p1 = torch.empty(plan.shape, device="cuda")
    p2 = torch.empty(plan.shape, device="cuda")
    plan.solve(mat, src, p1, ws)
    plan.status(ws)
    src2 = src * 2
    plan.solve(mat, src2, p2, ws)
    plan.status(ws)
    np.testing.assert_allclose(p2.cpu().numpy(), 2 * p1.cpu().numpy(), rtol=1e-6, atol=1e-30)


def test_index_out_of_range_reported():
    case = synth.random_small_case(1, n_steps=5)
    mat = case.mat.copy()
    mat[3, 4, 5] = case.materials.shape[0]
    plan = bb.Plan.from_case(case)
    ws = plan.workspace()
    src = torch.zeros((case.ny, case.nx), dtype=torch.complex64, device="cuda")
    peak = torch.empty(plan.shape, device="cuda")
    plan.solve(torch.from_numpy(mat).cuda(), src, peak, ws)
    with pytest.raises(bb.BBFDError) as e:
        plan.status(ws)
    assert e.value.code == bb.EINDEX


def test_divergence_reported():
    case = synth.random_small_case(0, n_steps=400)
    case.mat[10:] = 1
    case.cfl_safety = 1.6
    with pytest.raises(bb.BBFDError) as e:
        bb.run_case(case)
    assert e.value.code == bb.EDIVERGED


def test_transducer_crossing_source_plane_rejected():
    case = synth.plate_case()
    t = case.transducer
    t.apex = (t.apex[0], t.apex[1], case.source_plane_z() + 1e-3)
    plan = bb.Plan.from_case(case, n_steps=10)
    ws = plan.workspace()
    src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device="cuda")
    with pytest.raises(bb.BBFDError) as e:
        plan.source_rayleigh(t, src, ws)
    assert e.value.code == bb.EGEOMETRY


def test_workspace_too_small_rejected():
    case = synth.random_small_case(0, n_steps=5)
    plan = bb.Plan.from_case(case)
    ws = torch.empty(plan.workspace_bytes - 256, dtype=torch.uint8, device="cuda")
    src = torch.zeros((case.ny, case.nx), dtype=torch.complex64, device="cuda")
    peak = torch.empty(plan.shape, device="cuda")
    with pytest.raises(bb.BBFDError) as e:
        plan.solve(torch.from_numpy(case.mat).cuda(), src, peak, ws)
    assert e.value.code == bb.ENOMEM


def test_long_run_stays_bounded_where_skull_crosses_the_layer():
    """200x200x280 skull for 6000 steps (twice the workload's length): the shell
    runs into the absorbing layer's edges; the peak map must stay bounded
    everywhere, layer included (the unshifted CPML grew without bound here)."""
    case = synth.skull200(n_steps=6000)
    P, idx, val, _ = bb.run_case(case)
    P = P.cpu().numpy()
    say(f"[stability] interior peak {val:.4e}, global max {P.max():.4e}")
    assert np.isfinite(P).all()
    assert P.max() <= 1.5 * val
    assert 5e6 < val < 1e8


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="full-size oracle golden not generated")
def test_skull200_full_size_against_oracle_samples():
    """200x200x280, 3000 steps, in the launch configuration the benchmark times
    (captured graph): compare the oracle's stored samples."""
    g = np.load(GOLDEN)
    case = synth.skull200()
    say("[parity] skull200 full size")
    P, idx, val, plan = bb.run_case(case)
    P = P.cpu().numpy()
    L = case.pml
    sub = g["sub4"].astype(np.float64)
    mine = P[::4, ::4, ::4]
    lo = (L + 3) // 4
    sl = (slice(lo, (case.nz - L) // 4), slice(lo, (case.ny - L) // 4), slice(lo, (case.nx - L) // 4))
    errs = {
        "sub4": rel_l2(mine[sl], sub[sl]),
        "xz": rel_l2(P[L:-L, case.ny // 2, L:-L], g["xz"][L:-L, L:-L]),
        "yz": rel_l2(P[L:-L, L:-L, case.nx // 2], g["yz"][L:-L, L:-L]),
    }
    k = int(np.unravel_index(int(g["peak_index"]), P.shape)[0])
    errs["xy_peak"] = rel_l2(P[k, L:-L, L:-L], g["xy_peak"][L:-L, L:-L])
    say(f"[parity] skull200: {errs}, peak {idx} vs {int(g['peak_index'])}")
    for v in errs.values():
        assert v <= TOL_MAP
    if idx != int(g["peak_index"]):
        margin = (float(g["peak_value"]) - float(g["second_value"])) / float(g["peak_value"])
        assert margin <= 1e-5
        assert abs(P.flat[idx] - float(g["peak_value"])) <= 1e-4 * float(g["peak_value"])
    ref_src = g["src"].astype(np.complex128)
    ws = plan.workspace()
    src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device="cuda")
    plan.source_rayleigh(case.transducer, src, ws)
    torch.cuda.synchronize()
    assert rel_err_complex(src.cpu().numpy(), ref_src) <= TOL_SRC


def test_skull400_full_grid_short_run_against_oracle_samples():
    """The benchmark's 400x400x520 grid at 700 kHz in the launch configuration
    it times (captured graph, two branches per step, the fused step of deep
    tiles including those at the x edges), run for 300 steps so the wave
    crosses the near skull wall: compare the oracle's stored samples."""
    g = np.load(GOLDEN400)
    case = synth.skull400()
    case.n_steps = int(g["n_steps"])
    say("[parity] skull400 full grid, short run")
    plan = bb.Plan.from_case(case)
    ws = plan.workspace()
    src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device="cuda")
    plan.source_rayleigh(case.transducer, src, ws)
    mat = torch.from_numpy(np.ascontiguousarray(case.mat)).cuda()
    peak = torch.empty(plan.shape, dtype=torch.float32, device="cuda")
    plan.solve(mat, src, peak, ws)
    idx, val = plan.status(ws)
    counts = plan.tile_counts(ws)
    P = peak.cpu().numpy()
    del peak, ws
    torch.cuda.empty_cache()
    L = case.pml
    lo = (L + 7) // 8
    sl = (slice(lo, (case.nz - L) // 8), slice(lo, (case.ny - L) // 8), slice(lo, (case.nx - L) // 8))
    errs = {
        "sub8": rel_l2(P[::8, ::8, ::8][sl], g["sub8"].astype(np.float64)[sl]),
        "xz": rel_l2(P[L:-L, case.ny // 2, L:-L], g["xz"][L:-L, L:-L]),
        "yz": rel_l2(P[L:-L, L:-L, case.nx // 2], g["yz"][L:-L, L:-L]),
    }
    k = int(np.unravel_index(int(g["peak_index"]), P.shape)[0])
    errs["xy_peak"] = rel_l2(P[k, L:-L, L:-L], g["xy_peak"][L:-L, L:-L])
    say(f"[parity] skull400 short: {errs}, peak {idx} vs {int(g['peak_index'])}, tiles {counts}")
    assert counts[2] > 0
    for v in errs.values():
        assert v <= TOL_MAP
    if idx != int(g["peak_index"]):
        margin = (float(g["peak_value"]) - float(g["second_value"])) / float(g["peak_value"])
        assert margin <= 1e-5
        assert abs(P.flat[idx] - float(g["peak_value"])) <= 1e-4 * float(g["peak_value"])


def mixed_tile_case(n_steps=90):
    """90x36x60 water grid with a lossy solid block, a second lossless fluid
    and a lossy fluid: acoustic tiles (two fluid classes), general tiles, and
    acoustic segments next to elastic ones (which keep all normal stresses)."""
    nx, ny, nz, pml, f = 90, 36, 60, 6, 500e3
    mats = synth._rows(synth.table1(f)["water"],
                       (1850.0, 2700.0, 1300.0, 80.0, 200.0),     # lossy solid
                       (1100.0, 1700.0, 0.0, 0.0, 0.0),           # lossless fluid
                       (1050.0, 1560.0, 0.0, 30.0, 0.0))          # lossy fluid
    mat = np.zeros((nz, ny, nx), dtype=np.uint8)
    mat[25:35, 10:26, 40:70] = 1
    mat[40:52, :, 0:67] = 2                                     # spans x segment 0 and its reach
    mat[12:20, 20:30, 70:85] = 3
    case = synth.Case("mixedtiles", nx, ny, nz, pml, f, 6.0, n_steps, mats, mat, None)
    dx, zs = case.dx, case.source_plane_z()
    radius = 0.3 * min(nx, ny) * dx
    focal = 2.4 * radius
    fz = synth.bowl_focus_for_standoff(zs, radius, focal, (0.0, 0.0, 1.0), 2e-3)
    case.transducer = synth.Transducer(1, radius, focal, (nx // 2 * dx, ny // 2 * dx, fz - focal),
                                       (0.0, 0.0, 1.0))
    return case


def test_acoustic_and_general_tiles_side_by_side():
    case = mixed_tile_case()
    P, ref = compare_case(case)
    # the case does exercise both tile kinds and both fluid classes
    plan = bb.Plan.from_case(case)
    ws = plan.workspace()
    src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device="cuda")
    plan.source_rayleigh(case.transducer, src, ws)
    mat = torch.from_numpy(case.mat).cuda()
    peak = torch.empty(plan.shape, dtype=torch.float32, device="cuda")
    plan.solve(mat, src, peak, ws)
    plan.status(ws)
    cls = plan.segment_classes(ws)
    R, K = plan.info["tile_rows"], plan.info["tile_planes"]
    nseg = cls.shape[2]
    nby, nzc = -(-case.ny // R), -(-case.nz // K)
    pad = np.ones((nzc * K, nby * R, nseg), dtype=bool)
    pad[:case.nz, :case.ny] = cls != 0
    kinds = pad.reshape(nzc, K, nby, R, nseg).all(axis=(1, 3))
    say(f"[parity] classes {sorted(set(cls.ravel().tolist()))}, acoustic tiles "
        f"{int(kinds.sum())} of {kinds.size}")
    assert {0, 1, 3} <= set(cls.ravel().tolist())
    assert 0 < kinds.sum() < kinds.size
    assert np.array_equal(peak.cpu().numpy(), P)


@pytest.mark.parametrize("nx,nz,blob_x,src_k", [(150, 44, (20, 40), -1), (128, 70, (70, 90), -1),
                                                 (40, 128, (15, 25), -1), (128, 70, (70, 90), 16)])
def test_deep_tiles_fused_step(nx, nz, blob_x, src_k):
    """Wide water grid with a solid blob: x segments hold deep tiles,
    including segments at the grid's x edges whose fused step also carries
    the x absorbing layer (left edge and a partial last segment, 22 cells
    wide, for nx = 150; both edges for nx = 128; both edges within one
    40-cell segment for nx = 40).  With the source plane moved 12 planes into
    the interior (src_k = 16) deep tiles also carry the source force on their
    v_z faces.
    The one-pass step must agree with the oracle and with the two-pass
    kernels (the profiled solve times the fused kernel separately).  The grids
    have enough tiles (over 2048) for the plan to launch the fused step."""
    ny, pml, f = 64, 4, 500e3
    mats = synth._rows(synth.table1(f)["water"], (1850.0, 2700.0, 1300.0, 80.0, 200.0))
    mat = np.zeros((nz, ny, nx), dtype=np.uint8)
    mat[20:26, 8:18, blob_x[0]:blob_x[1]] = 1
    case = synth.Case("deeptiles", nx, ny, nz, pml, f, 6.0, 70, mats, mat, None)
    case.source_k = src_k
    dx, zs = case.dx, case.source_plane_z()
    radius = 0.3 * min(nx, ny) * dx
    focal = 2.4 * radius
    fz = synth.bowl_focus_for_standoff(zs, radius, focal, (0.0, 0.0, 1.0), 2e-3)
    case.transducer = synth.Transducer(1, radius, focal, (nx // 2 * dx, ny // 2 * dx, fz - focal),
                                       (0.0, 0.0, 1.0))
    P, ref = compare_case(case)
    plan = bb.Plan.from_case(case)
    ws = plan.workspace()
    src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device="cuda")
    plan.source_rayleigh(case.transducer, src, ws)
    mat_d = torch.from_numpy(case.mat).cuda()
    peak = torch.empty(plan.shape, dtype=torch.float32, device="cuda")
    ms = plan.solve_profiled(mat_d, src, peak, ws)
    plan.status(ws)
    counts = plan.tile_counts(ws)
    say(f"[parity] deep tiles: kernel ms {[round(m, 3) for m in ms]}, tiles {counts}")
    # the benchmark's byte model classifies tiles the same way as the library
    import bench
    kinds = bench.tile_kinds(case, plan.info, plan.segment_classes(ws))
    assert counts[2] > 0 and sum(counts) == kinds.size
    assert counts == tuple(int((kinds == k).sum()) for k in (1, 0, 2))
    assert np.array_equal(peak.cpu().numpy(), P)
    # batched sweeps run the two-pass kernels in place: same map bit for bit
    b = bb.Batch([case])
    bws = b.workspace()
    bsrc = torch.empty((case.ny, case.nx), dtype=torch.complex64, device="cuda")
    b.source_rayleigh(0, case.transducer, bsrc, bws)
    bpeak = torch.empty(plan.shape, dtype=torch.float32, device="cuda")
    b.solve([mat_d], [bsrc], [bpeak], bws)
    b.status(bws, 0)
    assert np.array_equal(bpeak.cpu().numpy(), P)


def test_largest_accepted_grid_against_oracle_window():
    """The largest grid the plan accepts for a 1000 x 1000 cross-section
    (1000 x 1000 x 1040 cells: every padded field array just under the 4 GiB
    the step kernels' 32-bit byte offsets address; ragged last x segment of 40
    cells; deep, general and acoustic tiles).  The source is a random 8 x 8
    patch on plane 970, near the top of the arrays, beside a solid block.  In 12
    steps no disturbance travels more than 48 cells (each stencil reaches two
    cells, two stencils per step), so the peak map inside a 128^3 window around
    the patch equals the oracle's solve of that window as a grid of its own
    with the same patch (whose absorbing layers the field never reaches either),
    and the map outside the window stays exactly zero: a wrapped address
    would carry the field somewhere else."""
    NX, NY, NZ, pml, f, steps = 1000, 1000, 1040, 8, 500e3, 12
    w, ox, oy, oz, ks = 128, 860, 864, 906, 64
    mats = synth._rows(synth.table1(f)["water"], (1850.0, 2700.0, 1300.0, 80.0, 200.0))
    small = np.zeros((w, w, w), dtype=np.uint8)
    small[66:74, 56:72, 58:90] = 1
    rng = np.random.default_rng(2026)
    patch = (rng.normal(size=(8, 8)) + 1j * rng.normal(size=(8, 8))).astype(np.complex64)
    src_s = np.zeros((w, w), dtype=np.complex64)
    src_s[60:68, 60:68] = patch
    case = synth.Case("window", w, w, w, pml, f, 6.0, steps, mats, small, None)
    case.capture_start, case.source_k = 0, ks
    ref, ridx, _ = oracle.solve(oracle.problem_from_case(case), small, src_s.astype(np.complex128))
    assert ref.max() > 0
    # the field stays clear of the window's own absorbing layers
    reach = np.argwhere(ref > 0)
    assert reach.min() >= pml and reach.max() < w - pml
    rk, rj, ri = np.unravel_index(ridx, ref.shape)

    torch.cuda.empty_cache()
    plan = bb.Plan(NX, NY, NZ, f, 6.0, steps, mats, pml=pml, capture_start=0, source_k=oz + ks)
    say(f"[parity] largest grid {NX}x{NY}x{NZ}: workspace {plan.workspace_bytes / 2**30:.1f} GiB, "
        f"free {torch.cuda.mem_get_info()[0] / 2**30:.1f} GiB")
    ws = plan.workspace()
    mat = np.zeros((NZ, NY, NX), dtype=np.uint8)
    mat[oz:oz + w, oy:oy + w, ox:ox + w] = small
    mat_d = torch.from_numpy(mat).cuda()
    del mat
    src = torch.zeros((NY, NX), dtype=torch.complex64, device="cuda")
    src[oy:oy + w, ox:ox + w] = torch.from_numpy(src_s).cuda()
    peak = torch.empty((NZ, NY, NX), dtype=torch.float32, device="cuda")
    plan.solve(mat_d, src, peak, ws)
    idx, val = plan.status(ws)
    counts = plan.tile_counts(ws)
    win = peak[oz:oz + w, oy:oy + w, ox:ox + w].cpu().numpy()
    outside = max(float(peak[:oz].abs().max()), float(peak[oz + w:].abs().max()),
                  float(peak[oz:oz + w, :oy].abs().max()), float(peak[oz:oz + w, oy + w:].abs().max()),
                  float(peak[oz:oz + w, oy:oy + w, :ox].abs().max()),
                  float(peak[oz:oz + w, oy:oy + w, ox + w:].abs().max()))
    del ws, peak, mat_d, src
    torch.cuda.empty_cache()
    err = rel_l2(win, ref)
    say(f"[parity] largest grid: tiles {counts}, window rel-L2 {err:.3e}, outside max {outside}, "
        f"peak {np.unravel_index(idx, (NZ, NY, NX))} vs {(oz + rk, oy + rj, ox + ri)}")
    assert counts[1] > 0 and counts[2] > 0
    assert err <= TOL_MAP
    assert outside == 0.0
    k, j, i = np.unravel_index(idx, (NZ, NY, NX))
    assert_same_peak(int(np.ravel_multi_index((k - oz, j - oy, i - ox), ref.shape)), ridx, ref, pml)
    assert val == pytest.approx(float(win[k - oz, j - oy, i - ox]))


def test_zero_source_peak_voxel_is_first_interior_cell():
    """With a zero source every peak value is 0: the tie goes to the lowest
    linear index of the interior outside the layer, cell (L, L, L), as in the
    oracle's tie pin."""
    case = synth.random_small_case(3, n_steps=20)
    plan = bb.Plan.from_case(case)
    ws = plan.workspace()
    src = torch.zeros((case.ny, case.nx), dtype=torch.complex64, device="cuda")
    peak = torch.empty(plan.shape, dtype=torch.float32, device="cuda")
    plan.solve(torch.from_numpy(case.mat).cuda(), src, peak, ws)
    idx, val = plan.status(ws)
    L = case.pml
    assert float(peak.abs().max()) == 0.0
    assert idx == (L * case.ny + L) * case.nx + L and val == 0.0
    ref, ridx, _ = oracle.solve(oracle.problem_from_case(case), case.mat,
                                np.zeros((case.ny, case.nx), dtype=np.complex128))
    assert ridx == idx


def test_plan_alternates_pointer_sets_without_recapture():
    """A skull-like map and its water-only companion (the paper's pair of runs
    per target), each in its own workspace, alternate on one plan: each pointer
    set is captured once and replayed afterwards, and every replay equals the
    direct-launch map bit for bit."""
    case = synth.random_small_case(5, n_steps=60)
    plan = bb.Plan.from_case(case)
    src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device="cuda")
    ws = [plan.workspace(), plan.workspace()]
    plan.source_rayleigh(case.transducer, src, ws[0])
    mats = [torch.from_numpy(case.mat).cuda(), torch.zeros_like(torch.from_numpy(case.mat)).cuda()]
    peaks = [torch.empty(plan.shape, dtype=torch.float32, device="cuda") for _ in range(2)]
    direct = []
    for q in range(2):
        plan.solve(mats[q], src, peaks[q], ws[q], graph=False)
        plan.status(ws[q])
        direct.append(peaks[q].cpu().numpy())
    assert not np.array_equal(direct[0], direct[1])
    before = plan.graph_captures
    for r in range(3):
        for q in range(2):
            peaks[q].fill_(-1.0)
            plan.solve(mats[q], src, peaks[q], ws[q])
        for q in range(2):
            plan.status(ws[q])
            assert np.array_equal(peaks[q].cpu().numpy(), direct[q]), (r, q)
    assert plan.graph_captures - before == 2


@pytest.mark.timeout(900)
def test_full_map_every_tile_kind_against_oracle():
    """Element-by-element parity of a whole 160 x 128 x 176 skull map at 500
    kHz (3.6 M cells, 8448 tiles: acoustic, general and deep tiles, fused
    step, two-branch captured graph), run 1000 steps (about 43 periods, past
    the transit of the whole depth, so the field behind the near skull wall is
    steady), against the FP64 oracle run live: rel-L2 over the whole interior
    and the largest single-cell deviation."""
    case = synth.skull_case(160, 128, 176, 500e3, 6.0, 1000, seed=7, name="skull160x128x176_500kHz")
    P, idx, val, plan = bb.run_case(case)
    ws = plan.workspace()
    src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device="cuda")
    plan.source_rayleigh(case.transducer, src, ws)
    peak = torch.empty(plan.shape, dtype=torch.float32, device="cuda")
    plan.solve(torch.from_numpy(case.mat).cuda(), src, peak, ws)
    plan.status(ws)
    counts = plan.tile_counts(ws)
    say(f"[parity] full map: tiles (acoustic, general, deep) {counts}")
    assert sum(counts) >= 2048 and min(counts) > 0
    P = P.cpu().numpy()
    assert np.array_equal(peak.cpu().numpy(), P)
    ref, ridx, secs = oracle.solve_case(case)
    L = case.pml
    a, b = interior(P, L), interior(ref, L)
    err = rel_l2(a, b)
    dev = float(np.abs(a - b).max() / np.abs(b).max())
    say(f"[parity] full map: oracle {secs:.1f} s, rel-L2 {err:.3e}, max |diff| / max {dev:.3e}, "
        f"peak {idx} vs {ridx}")
    assert err <= TOL_MAP
    assert dev <= 1e-3
    assert_same_peak(idx, ridx, ref, L)
