"""12-bit CT maps (uint16 indices into tables of up to 4096 rows, Section
2.2.2) and the q_c sweep (Section 3.2) as a batched workload, on the GPU
against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from oracle import energy
import paper_2301_12727_amd as bb
import synth

from ._parity import assert_map_matches, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed", [20001, 20002])
def test_ct12_skull_patch_against_oracle(seed):
    """A 64^3 skull patch whose bone carries 12-bit CT levels (about 1600
    distinct rows of a 4096-row table in use), 300 steps: the 16-bit path
    (general kernels reading the table through the caches) against the
    oracle."""
    case = synth.ct_case(synth.surrogate_case(seed), seed)
    case.n_steps = 300
    used = len(np.unique(case.mat))
    P, idx, _, plan = bb.run_case(case)
    assert plan.index_bits == 16
    ref, ridx, _ = oracle.solve_case(case)
    assert_map_matches(P.cpu().numpy(), ref, idx, ridx, case.pml, f"ct12 {seed} ({used} levels)")
    assert used > 1000


@pytest.mark.parametrize("nx,nz", [(128, 70), (150, 44)])
def test_uint16_map_equals_uint8_map_bit_for_bit(nx, nz):
    """The same two-material map solved as uint8 (table in LDS) and as uint16
    with the solid moved to row 3000 of a 4096-row table (table through the
    caches): acoustic, general and deep tiles give the same map bit for bit."""
    ny, pml, f = 64, 4, 500e3
    solid = (1850.0, 2700.0, 1300.0, 80.0, 200.0)
    mats = synth._rows(synth.table1(f)["water"], solid)
    mat = np.zeros((nz, ny, nx), dtype=np.uint8)
    mat[20:26, 8:18, 70:90] = 1
    case = synth.Case("u16", nx, ny, nz, pml, f, 6.0, 70, mats, mat, None)
    dx, zs = case.dx, case.source_plane_z()
    radius = 0.3 * min(nx, ny) * dx
    focal = 2.4 * radius
    fz = synth.bowl_focus_for_standoff(zs, radius, focal, (0.0, 0.0, 1.0), 2e-3)
    case.transducer = synth.Transducer(1, radius, focal, (nx // 2 * dx, ny // 2 * dx, fz - focal),
                                       (0.0, 0.0, 1.0))
    P8, i8, v8, plan8 = bb.run_case(case)
    table = np.tile(mats[0], (4096, 1))
    table[3000] = solid
    c16 = synth.Case(**{**case.__dict__, "materials": table,
                        "mat": np.where(mat == 1, 3000, 0).astype(np.uint16)})
    P16, i16, v16, plan16 = bb.run_case(c16)
    ws = plan16.workspace()
    src = torch.empty((ny, nx), dtype=torch.complex64, device="cuda")
    plan16.source_rayleigh(case.transducer, src, ws)
    peak = torch.empty(plan16.shape, dtype=torch.float32, device="cuda")
    plan16.solve(torch.from_numpy(c16.mat).cuda(), src, peak, ws)
    plan16.status(ws)
    counts = plan16.tile_counts(ws)
    say(f"[ct] {nx}x{ny}x{nz} uint16 tiles {counts}")
    assert min(counts) > 0
    assert torch.equal(P8, P16) and (i8, v8) == (i16, v16)


def test_energy_loss_on_16_bit_maps_matches_oracle():
    rng = np.random.default_rng(5)
    shape = (30, 41, 52)
    table = synth.ct_materials(500e3)
    ps = rng.gamma(2.0, 5e4, size=shape).astype(np.float32)
    pw = rng.gamma(2.0, 6e4, size=shape).astype(np.float32)
    ms = rng.integers(0, 4096, size=shape).astype(np.uint16)
    mw = np.zeros_like(ms)
    plan = bb.Plan(shape[2], shape[1], shape[0], 500e3, 6.0, 4, table, pml=4, index_bits=16)
    ws = plan.workspace()
    d = [torch.from_numpy(a).cuda() for a in (ms, ps, mw, pw)]
    for z in (-1, 12):
        got = plan.energy_loss(d[0], d[1], d[2], d[3], ws, z_m=z)
        ref = energy.energy_loss(ps, ms, pw, mw, table, 4, z_m=None if z < 0 else z)
        assert got[2] == ref[2] and got[0] == pytest.approx(ref[0], rel=1e-12)


def test_qc_sweep_as_a_batch_against_oracle():
    """The attenuation correction q_c of the paper's mapping study (Q = Q0 q_c)
    swept over 0.4, 1, 2, 3, 4 on one 64^3 skull patch: five problems that
    differ only in qc run as one batched sweep; each map matches the oracle,
    and T_S = sqrt(E_L) against the water-only solve rises with q_c (less
    attenuation) and matches the oracle's T_S."""
    base = synth.surrogate_case(20004)
    base.n_steps = 300
    qcs = (0.4, 1.0, 2.0, 3.0, 4.0)
    cases = [synth.Case(**{**base.__dict__, "qc": q, "name": f"qc{q}"}) for q in qcs]
    b = bb.Batch(cases)
    ws = b.workspace()
    mat = torch.from_numpy(base.mat).cuda()
    srcs = [torch.empty((base.ny, base.nx), dtype=torch.complex64, device="cuda") for _ in cases]
    for i, c in enumerate(cases):
        b.source_rayleigh(i, c.transducer, srcs[i], ws)
    peaks = [torch.empty((base.nz, base.ny, base.nx), dtype=torch.float32, device="cuda")
             for _ in cases]
    b.solve([mat] * len(cases), srcs, peaks, ws)
    water = synth.Case(**{**base.__dict__, "mat": np.zeros_like(base.mat)})
    Pw, widx, _, wplan = bb.run_case(water)
    ref_w, _, _ = oracle.solve_case(water)
    wws = wplan.workspace()
    mw = torch.zeros_like(mat)
    ts, ref_ts = [], []
    for i, c in enumerate(cases):
        idx, _ = b.status(ws, i)
        ref, ridx, _ = oracle.solve_case(c)
        assert_map_matches(peaks[i].cpu().numpy(), ref, idx, ridx, c.pml, f"qc {c.qc}")
        t = wplan.energy_loss(mat, peaks[i], mw, Pw, wws)[1]
        r = energy.energy_loss(ref, base.mat, ref_w, water.mat, base.materials, base.pml)[1]
        say(f"[ct] q_c {c.qc}: T_S {t:.5f} (oracle {r:.5f})")
        ts.append(t)
        ref_ts.append(r)
        assert t == pytest.approx(r, rel=1e-3)
    assert all(a < b for a, b in zip(ts, ts[1:]))
