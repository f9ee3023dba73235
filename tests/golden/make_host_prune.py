"""Writes host_prune_oracle.npz: the FP64 oracle's result on the 256x256,
30-cell, D = 32 frame (seed 7) clustered with N carried in at 20,000 seeds,
whose first round holds more candidates than the device ranking takes, so
that the GPU test of that path can compare with the oracle.  Calls only
oracle/ (and synth/ for the input).  Run from the repository root:

    python tests/golden/make_host_prune.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import cluster as C  # noqa: E402
from tests.golden.make_batch_oracle import provenance  # noqa: E402

BAND = 1e-4  # the exempt band of the label comparison
SPEC = synth.FrameSpec(256, 256, 30, 8, 30, 32, 0.08, 0.05, 7)
N_STATE_IN = 20000


def main():
    f = synth.make_frame(SPEC)
    t0 = time.time()
    r = C.cluster(f.emb, f.mask, C.Params(bandwidth=f.bandwidth, n_state_in=N_STATE_IN))
    thr = 1.0 - f.bandwidth
    stats = {k: (float(v) if isinstance(v, float) else int(v)) for k, v in r.stats.items()}
    np.savez_compressed(os.path.join(HERE, "host_prune_oracle.npz"),
                        modes=r.modes.astype(np.float64), mode_counts=np.asarray(r.mode_counts, np.int32),
                        fg_labels=np.asarray(r.labels).reshape(-1)[r.fg].astype(np.int16),
                        band=np.packbits(np.abs(r.best - thr) < BAND),
                        tie=np.packbits(np.abs(r.best - r.second) < BAND), n_fg=np.int64(len(r.fg)),
                        bandwidth=np.float64(f.bandwidth), n_state_in=np.int64(N_STATE_IN), **provenance(r),
                        stats=np.frombuffer(json.dumps(stats).encode(), np.uint8))
    print(len(r.modes), "modes;", stats, f"{time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
