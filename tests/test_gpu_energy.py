"""Energy-loss factor E_L (Eq. 2) and T_S = sqrt(E_L) on the GPU
(bbfd_energy_loss) against the oracle: the plane reduction on seeded maps,
and the whole skull / water-only pair solved by each side."""
import numpy as np
import pytest
import torch

import oracle
from oracle import energy
import paper_2301_12727_amd as bb
import synth

from ._parity import say

pytestmark = pytest.mark.gpu


def seeded_maps(seed, nx, ny, nz, n_mat):
    rng = np.random.default_rng(seed)
    ps = rng.gamma(2.0, 5e4, size=(nz, ny, nx)).astype(np.float32)
    pw = rng.gamma(2.0, 6e4, size=(nz, ny, nx)).astype(np.float32)
    ms = rng.integers(0, n_mat, size=(nz, ny, nx)).astype(np.uint8)
    mw = np.zeros_like(ms)
    return ps, ms, pw, mw


@pytest.mark.parametrize("seed,shape", [(1, (70, 45, 33)), (2, (129, 64, 40)), (3, (17, 90, 21))])
def test_plane_reduction_matches_oracle_on_seeded_maps(seed, shape):
    """Seeded random peak and material maps (ragged sizes, 4 materials): the
    GPU's FP64 plane sums equal the oracle's to rounding, on a named plane and
    on the plane of the water map's peak voxel (also when that maximum is tied
    between two planes: the lower plane wins)."""
    nx, ny, nz = shape
    case = synth.random_small_case(seed, n_steps=4)
    mats = case.materials
    plan = bb.Plan(nx, ny, nz, case.freq_hz, 6.0, 4, mats, pml=4)
    ws = plan.workspace()
    ps, ms, pw, mw = seeded_maps(seed, nx, ny, nz, len(mats))
    for tie in (False, True):
        if tie:   # equal maximum on an earlier plane, inside the interior
            k, j, i = np.unravel_index(int(np.argmax(pw[4:-4, 4:-4, 4:-4])), (nz - 8, ny - 8, nx - 8))
            top = pw[4 + k, 4 + j, 4 + i]
            pw[4, 6, 7] = top
        d = [torch.from_numpy(a).cuda() for a in (ms, ps, mw, pw)]
        for z in (-1, 4, nz // 2):
            got = plan.energy_loss(d[0], d[1], d[2], d[3], ws, z_m=z)
            ref = energy.energy_loss(ps, ms, pw, mw, mats, 4, z_m=None if z < 0 else z)
            say(f"[energy] {shape} tie={tie} z={z}: E_L {got[0]:.12g} vs {ref[0]:.12g}, z_m {got[2]} vs {ref[2]}")
            assert got[2] == ref[2]
            assert got[0] == pytest.approx(ref[0], rel=1e-12)
            assert got[1] == pytest.approx(ref[1], rel=1e-12)
            if tie and z < 0:
                assert got[2] == 4


def test_plane_outside_interior_rejected():
    case = synth.random_small_case(4, n_steps=4)
    plan = bb.Plan.from_case(case)
    ws = plan.workspace()
    m = torch.zeros(plan.shape, dtype=torch.uint8, device="cuda")
    p = torch.ones(plan.shape, dtype=torch.float32, device="cuda")
    with pytest.raises(bb.BBFDError) as e:
        plan.energy_loss(m, p, m, p, ws, z_m=case.pml - 1)
    assert e.value.code == bb.EINVAL
    with pytest.raises(bb.BBFDError) as e:
        plan.energy_loss(m, p, m, torch.zeros_like(p), ws, z_m=case.pml)
    assert e.value.code == bb.EDIVERGED


@pytest.mark.parametrize("seed", [20001, 20005])
def test_skull_and_water_pair_against_oracle(seed):
    """A 64^3 skull patch with a tilted focused bowl (the surrogate's data
    recipe, 414 steps): the GPU solves the skull map and its water-only
    companion on one plan (two captured graphs, then E_L on the plane of the
    water field's peak); the oracle solves both itself.  The maps agree to
    2e-4 rel-L2, so the plane sums of squares agree to about 1e-3."""
    case = synth.surrogate_case(seed)
    plan = bb.Plan.from_case(case)
    ws = plan.workspace()
    src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device="cuda")
    plan.source_rayleigh(case.transducer, src, ws)
    ms = torch.from_numpy(case.mat).cuda()
    mw = torch.zeros_like(ms)
    ps = torch.empty(plan.shape, dtype=torch.float32, device="cuda")
    pw = torch.empty_like(ps)
    plan.solve(ms, src, ps, ws)
    plan.status(ws)
    plan.solve(mw, src, pw, ws)
    widx, _ = plan.status(ws)
    got = plan.energy_loss(ms, ps, mw, pw, ws)
    ref_s, _, _ = oracle.solve_case(case)
    water = synth.Case(**{**case.__dict__, "mat": np.zeros_like(case.mat)})
    ref_w, ref_widx, _ = oracle.solve_case(water)
    ref = energy.energy_loss(ref_s, case.mat, ref_w, water.mat, case.materials, case.pml)
    say(f"[energy] pair {seed}: E_L {got[0]:.6f} vs {ref[0]:.6f}, T_S {got[1]:.6f} vs {ref[1]:.6f}, "
        f"z_m {got[2]} vs {ref[2]}")
    assert got[2] == ref[2] == widx // (case.nx * case.ny)
    assert widx == ref_widx
    assert 0.0 < ref[0] < 1.0
    assert got[0] == pytest.approx(ref[0], rel=1e-3)
    assert got[1] == pytest.approx(ref[1], rel=5e-4)
