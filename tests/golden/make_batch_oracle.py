"""Writes batch_oracle.npz: the FP64 oracle's results on five frames of the
64-frame uneven batching workload (synth.batch_specs(64), frames 1, 2, 3, 10
and 15: sides 512, 1024, 512, 768, 1024; noise 0.054-0.1, so bandwidths from
0.1 to 0.3), so that GPU tests and the benchmark can check the batched call
at full frame size without re-running the oracle.  Calls only oracle/ (and
synth/ for the inputs).  Run from the repository root:

    python tests/golden/make_batch_oracle.py
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

BAND = 1e-4  # the exempt band of the label comparison
GAP_KEEP = 0.02
FRAMES = (1, 2, 3, 10, 15)



def provenance(r):
    """Where each mode came from: every round's seed list (foreground
    ordinals, concatenated, with offsets) with each seed's converged flag and
    step count, and, per mode, its round, its index in that round's list and
    its step count, so that a test can iterate the same rounds again on
    another arithmetic and compare seed by seed."""
    seeds = [lg.seeds.astype(np.int32) for lg in r.rounds]
    off = np.cumsum([0] + [len(s) for s in seeds]).astype(np.int64)
    conv = np.concatenate([lg.converged for lg in r.rounds]) if seeds else np.zeros(0, bool)
    iters = np.concatenate([lg.iters for lg in r.rounds]) if seeds else np.zeros(0, np.int64)
    rnd, loc, its = [], [], []
    for ri, lg in enumerate(r.rounds):
        for a in lg.accepted:
            rnd.append(ri)
            loc.append(a)
            its.append(int(lg.iters[a]))
    return {"round_seeds": np.concatenate(seeds) if seeds else np.zeros(0, np.int32), "round_off": off,
            "round_conv": np.packbits(conv), "round_iters": np.minimum(iters, 255).astype(np.uint8),
            "mode_round": np.array(rnd, np.int32), "mode_local": np.array(loc, np.int32),
            "mode_iters": np.array(its, np.int32)}


def main():
    specs = synth.batch_specs(64)
    out = {"frames": np.array(FRAMES, np.int64)}
    for i in FRAMES:
        f = synth.make_frame(specs[i])
        t0 = time.time()
        r = C.cluster(f.emb, f.mask, C.Params(bandwidth=f.bandwidth))
        thr = 1.0 - f.bandwidth
        stats = {k: (float(v) if isinstance(v, float) else int(v)) for k, v in r.stats.items()}
        out[f"f{i}_modes"] = r.modes.astype(np.float64)
        out[f"f{i}_mode_counts"] = np.asarray(r.mode_counts, np.int32)
        out[f"f{i}_fg_labels"] = np.asarray(r.labels).reshape(-1)[r.fg].astype(np.int16)
        out[f"f{i}_band"] = np.packbits(np.abs(r.best - thr) < BAND)
        out[f"f{i}_tie"] = np.packbits(np.abs(r.best - r.second) < BAND)
        # Best minus second-best similarity, kept where it is below GAP_KEEP
        # (argmax near-ties of a wider band than BAND can be exempted).
        gap = r.best - r.second
        near = np.flatnonzero(gap < GAP_KEEP)
        out[f"f{i}_near_idx"] = near.astype(np.int32)
        out[f"f{i}_near_gap"] = gap[near].astype(np.float32)
        out.update({f"f{i}_{k}": v for k, v in provenance(r).items()})
        out[f"f{i}_bandwidth"] = np.float64(f.bandwidth)
        out[f"f{i}_stats"] = np.frombuffer(json.dumps(stats).encode(), np.uint8)
        print(f"frame {i}: {specs[i].height}^2, h {f.bandwidth}, {len(r.modes)} modes, "
              f"{time.time() - t0:.1f} s; {stats}", flush=True)
    np.savez_compressed(os.path.join(HERE, "batch_oracle.npz"), **out)


if __name__ == "__main__":
    main()
