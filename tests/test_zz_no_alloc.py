"""bbfd_solve_static (the solve whose workspace is the library's fixed
per-GPU device array) against bbfd_solve with a caller workspace: the same
maps bit for bit, the same peak voxel and value, on two calls in a row, the
second on a smaller grid (the array keeps the first call's contents)."""
import sys

import numpy as np
import pytest
import torch

import paper_2301_12727_amd as bb
import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_static_solve_equals_workspace_solve_on_two_calls():
    cases = [synth.random_small_case(21, n=(44, 52), n_steps=70),
             synth.random_small_case(22, n=(24, 30), n_steps=45)]
    assert cases[1].cells < cases[0].cells
    for case in cases:
        say(f"[static] {case.nx}x{case.ny}x{case.nz}, {case.n_steps} steps")
        P, idx, val, plan = bb.run_case(case)
        ws = plan.workspace()
        src = torch.empty((case.ny, case.nx), dtype=torch.complex64, device="cuda")
        plan.source_rayleigh(case.transducer, src, ws)
        del ws
        mat = torch.from_numpy(case.mat).cuda()
        peak = torch.full(plan.shape, -1.0, dtype=torch.float32, device="cuda")
        sidx, sval = plan.solve_static(mat, src, peak)
        got = peak.cpu().numpy()
        ref = P.cpu().numpy()
        say(f"[static] max |diff| {float(np.abs(got - ref).max())}, peak {sidx} vs {idx}")
        assert np.array_equal(got, ref)
        assert (sidx, sval) == (idx, val)


def test_static_solve_reports_device_errors():
    case = synth.random_small_case(23, n_steps=5)
    mat = case.mat.copy()
    mat[2, 3, 4] = case.materials.shape[0]
    plan = bb.Plan.from_case(case)
    src = torch.zeros((case.ny, case.nx), dtype=torch.complex64, device="cuda")
    peak = torch.empty(plan.shape, device="cuda")
    with pytest.raises(bb.BBFDError) as e:
        plan.solve_static(torch.from_numpy(mat).cuda(), src, peak)
    assert e.value.code == bb.EINDEX
