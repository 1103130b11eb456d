"""Comparison helpers shared by the GPU parity tests (HIP path against the FP64
oracle): relative L2 error over the interior outside the absorbing layer and
the peak-voxel check."""
import sys

import numpy as np

TOL_MAP = 2e-4


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def interior(P, L):
    return P[L:P.shape[0] - L, L:P.shape[1] - L, L:P.shape[2] - L]


def assert_same_peak(gpu_idx, ref_idx, ref_map):
    """Same peak voxel; a different voxel is accepted only as a tie inside the
    oracle's own 1e-5 relative margin."""
    if gpu_idx == ref_idx:
        return
    v_ref = ref_map.flat[ref_idx]
    v_alt = ref_map.flat[gpu_idx]
    assert abs(v_ref - v_alt) <= 1e-5 * v_ref, (gpu_idx, ref_idx, v_ref, v_alt)


def assert_map_matches(P, ref, gpu_idx, ref_idx, L, what, tol=TOL_MAP):
    err = rel_l2(interior(P, L), interior(ref, L))
    say(f"[parity] {what}: rel-L2 {err:.3e}, peak {gpu_idx} vs {ref_idx}")
    assert err <= tol, (what, err)
    assert_same_peak(gpu_idx, ref_idx, ref)
    return err
