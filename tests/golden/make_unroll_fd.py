"""Writes unroll_fd.npz: FP64 central differences of the differentiation
workload's loss (T = 10 unrolled steps from 128 seeds on the 64x64 crop of the
512x512, D = 32 frame; L = sum_j y_T,j . target_j) at 200 sampled (pixel,
dimension) coordinates, so that the GPU gradient can be checked against
finite differences without the ~1 minute of oracle runs.  Calls only oracle/
(through the crop case and difference helpers of tests/test_oracle_unroll.py)
and synth/.  Run from the repository root:

    python tests/golden/make_unroll_fd.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from tests.test_oracle_unroll import crop_case, fd_at  # noqa: E402


def main():
    e, seeds, h, steps, targets, coords = crop_case()
    fd = fd_at(e, seeds, h, steps, targets, coords)
    np.savez_compressed(os.path.join(HERE, "unroll_fd.npz"), seeds=seeds.astype(np.int64), targets=targets,
                        coords=coords.astype(np.int64), fd=fd, bandwidth=np.float64(h), steps=np.int64(steps))
    print(len(fd), "differences;", int(np.count_nonzero(np.abs(fd) > 1e-3)), "above 1e-3")


if __name__ == "__main__":
    main()
