"""Write skull400_short_oracle.npz: FP64-oracle samples of the full 400x400x520
skull grid at 700 kHz (PPW 9, the benchmark's workload) run for 300 steps (the
wave crosses the near skull wall; peaks captured over the last two periods),
for a full-grid parity check of the launch configuration the benchmark times.

Calls only the oracle and the seeded input generators.  Stored (float32 where
a map): the peak map on every 8th cell per axis, the x-z and y-z planes
through the acoustic axis, the x-y plane through the peak voxel, the oracle's
peak voxel and value and the runner-up interior value (tie margin).

Run from the repository root:  python tests/golden/make_skull400_short.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "skull400_short_oracle.npz")
N_STEPS = 300


def main():
    case = synth.skull400()
    case.n_steps = N_STEPS
    t0 = time.time()
    src = oracle.source_plane(case)
    print(f"source plane {time.time() - t0:.1f}s", flush=True)
    prob = oracle.problem_from_case(case)
    peak, idx, secs = oracle.solve(prob, case.mat, src)
    print(f"solve loop {secs:.1f}s ({case.cells * case.n_steps / secs / 1e6:.2f} Mcell/s)", flush=True)
    k, j, i = np.unravel_index(idx, peak.shape)
    L = case.pml
    flat = np.sort(peak[L:-L, L:-L, L:-L].ravel())
    np.savez_compressed(
        OUT,
        n_steps=np.int64(N_STEPS),
        sub8=peak[::8, ::8, ::8].astype(np.float32),
        xz=peak[:, case.ny // 2, :].astype(np.float32),
        yz=peak[:, :, case.nx // 2].astype(np.float32),
        xy_peak=peak[k].astype(np.float32),
        peak_index=np.int64(idx),
        peak_value=np.float64(peak.flat[idx]),
        second_value=np.float64(flat[-2]),
        loop_seconds=np.float64(secs),
        threads=np.int64(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))),
    )
    print(f"peak voxel (k, j, i) = {(k, j, i)} value {peak.flat[idx]:.6e}; wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
