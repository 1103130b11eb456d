"""Thermal step (BHTE, Section 2.4) on the GPU against the FP64 oracle: seeded
skull maps and synthetic focal peak-pressure maps, an on/off sonication at a
duty cycle; final temperature, maximal temperature and CEM43 dose compared
cell by cell.  Inputs come from the seeded generators only."""
import numpy as np
import pytest
import torch

from oracle import bhte as ref_bhte
import paper_2301_12727_amd as bb
from paper_2301_12727_amd.thermal import Thermal
import synth

from ._parity import rel_l2, say

pytestmark = pytest.mark.gpu

# Each step rounds the FP32 temperature rise once (relative 2^-24); the errors
# add at most linearly over the steps: tolerance 2 x steps x 2^-24 on the rise
# (rel-L2).  The dose is exponential in T, so its relative error is ln 4 times
# the rise's absolute error in K, well inside 1e-4.
TOL_DOSE = 1e-4


def thermal_case(shape, seed, freq=500e3):
    nz, ny, nx = shape
    dx = synth.C_WATER / (freq * 6.0)
    mat = synth.skull_map(nx, ny, nz, dx, 0.0, seed, centre_depth=70e-3 + 10 * dx,
                          thick_scale=0.5)
    ac, th = synth.thermal_materials(freq)
    peak = synth.focus_map(shape, (0.7 * nz, 0.5 * ny, 0.5 * nx), 4.0, 2.5e6, seed=seed)
    return mat, peak, ac, th, dx


@pytest.mark.parametrize("shape,seed,n_on,n_off,duty",
                         [((50, 60, 70), 1, 300, 150, 0.3), ((37, 41, 29), 2, 120, 0, 1.0),
                          ((20, 70, 130), 3, 40, 200, 0.5)])
def test_bhte_matches_oracle(shape, seed, n_on, n_off, duty):
    mat, peak, ac, th, dx = thermal_case(shape, seed)
    assert (mat > 0).any() and (mat == 0).any()
    dt = 0.1
    plan = Thermal(shape, dx, dt, ac, th, n_on, n_off, duty=duty, intensity_scale=1.0)
    assert dt < plan.dt_max
    ws = plan.workspace()
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    t_final, t_max, dose = (torch.empty(shape, dtype=torch.float32, device="cuda") for _ in range(3))
    plan.run(d(mat), d(peak), t_final, t_max, dose, ws)
    torch.cuda.synchronize()
    q = ref_bhte.heat_source(mat, peak, ac, th[:, 3])
    sim = ref_bhte.BHTE(mat, ac, th[:, :3], dx, dt)
    T, Tm, D = sim.run(q, n_on, n_off, duty)
    got_T, got_Tm, got_D = (x.cpu().numpy().astype(np.float64) for x in (t_final, t_max, dose))
    e_t = rel_l2(got_T - 37.0, T - 37.0)
    e_m = rel_l2(got_Tm - 37.0, Tm - 37.0)
    e_d = rel_l2(got_D, D)
    say(f"[bhte] {shape}: max rise {Tm.max() - 37:.2f} K, peak dose {D.max():.3g} min; "
        f"rel-L2 final {e_t:.2e}, max {e_m:.2e}, dose {e_d:.2e}")
    assert Tm.max() > 43.0                    # both branches of the dose rate are exercised
    tol_rise = 2.0 * (n_on + n_off) * 2.0 ** -24
    assert e_t <= tol_rise and e_m <= tol_rise and e_d <= TOL_DOSE
    assert np.all(got_T[0] == 37.0) and np.all(got_T[:, :, -1] == 37.0)
    k, j, i = np.unravel_index(int(np.argmax(Tm)), shape)
    assert got_Tm[k, j, i] == pytest.approx(Tm[k, j, i], abs=1e-4)


def test_bhte_rejects_unstable_step_and_bad_inputs():
    mat, peak, ac, th, dx = thermal_case((20, 20, 20), 4)
    with pytest.raises(bb.BBFDError) as e:
        Thermal((20, 20, 20), dx, 10.0, ac, th, 10, 0)
    assert e.value.code == bb.EINVAL
    bad = th.copy()
    bad[1, 3] = 1.5
    with pytest.raises(bb.BBFDError) as e:
        Thermal((20, 20, 20), dx, 0.1, ac, bad, 10, 0)
    assert e.value.code == bb.EMATERIAL
    plan = Thermal((20, 20, 20), dx, 0.1, ac, th, 10, 0)
    small = torch.empty(plan.workspace_bytes - 256, dtype=torch.uint8, device="cuda")
    out = torch.empty((20, 20, 20), device="cuda")
    m = torch.from_numpy(mat).cuda()
    with pytest.raises(bb.BBFDError) as e:
        plan.run(m, out, out, out, out, small)
    assert e.value.code == bb.ENOMEM
