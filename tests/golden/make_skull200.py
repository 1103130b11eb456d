"""Write skull200_oracle.npz: FP64-oracle samples of the full 200x200x280 skull
solve at 500 kHz (PPW 6, 3000 steps, seed 1) for full-size parity checks.

Calls only the oracle and the seeded input generators.  Stored (float32 where
a map): the peak map on every 4th cell per axis, the three planes through the
acoustic axis / the peak voxel, the oracle's peak voxel and value, the runner-up
interior value (tie margin), and the FP64 Rayleigh source plane.

Run from the repository root:  python tests/golden/make_skull200.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "skull200_oracle.npz")


def main():
    case = synth.skull200()
    t0 = time.time()
    src = oracle.source_plane(case)
    print(f"source plane {time.time() - t0:.1f}s", flush=True)
    prob = oracle.problem_from_case(case)
    peak, idx, secs = oracle.solve(prob, case.mat, src)
    print(f"solve loop {secs:.1f}s ({case.cells * case.n_steps / secs / 1e6:.2f} Mcell/s)", flush=True)
    k, j, i = np.unravel_index(idx, peak.shape)
    L = case.pml
    inner = peak[L:-L, L:-L, L:-L].copy()
    flat = np.sort(inner.ravel())
    np.savez_compressed(
        OUT,
        sub4=peak[::4, ::4, ::4].astype(np.float32),
        xz=peak[:, case.ny // 2, :].astype(np.float32),
        yz=peak[:, :, case.nx // 2].astype(np.float32),
        xy_peak=peak[k].astype(np.float32),
        peak_index=np.int64(idx),
        peak_value=np.float64(peak.flat[idx]),
        second_value=np.float64(flat[-2]),
        src=src.astype(np.complex64),
        loop_seconds=np.float64(secs),
        threads=np.int64(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))),
    )
    print(f"peak voxel (k, j, i) = {(k, j, i)} value {peak.flat[idx]:.6e}; wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
