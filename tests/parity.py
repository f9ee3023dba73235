"""Comparison of GPU results with the FP64 oracle (test infrastructure).

Modes are matched by mutual best cosine; the mode error is 1 - cos in FP64.
Labels are compared after remapping GPU mode indices through the matching and
must agree exactly except on two counted exempt sets: pixels whose best
similarity lies within BAND of the bandwidth threshold, and pixels whose best
and second-best similarities lie within BAND of each other (argmax near-ties).
"""
from __future__ import annotations

import dataclasses

import numpy as np

BAND = 1e-4


@dataclasses.dataclass
class ModeMatch:
    pairs: np.ndarray        # (k, 2): (gpu index, oracle index)
    errors: np.ndarray       # 1 - cos for each pair
    unmatched_gpu: int
    unmatched_oracle: int

    @property
    def max_error(self) -> float:
        return float(self.errors.max()) if len(self.errors) else 0.0


def match_modes(gpu_modes, oracle_modes) -> ModeMatch:
    g = np.asarray(gpu_modes, np.float64)
    o = np.asarray(oracle_modes, np.float64)
    if len(g) == 0 or len(o) == 0:
        return ModeMatch(np.zeros((0, 2), np.int64), np.zeros(0), len(g), len(o))
    gn = g / np.linalg.norm(g, axis=1, keepdims=True)
    on = o / np.linalg.norm(o, axis=1, keepdims=True)
    s = gn @ on.T
    bg = np.argmax(s, axis=1)
    bo = np.argmax(s, axis=0)
    pairs = np.array([(i, bg[i]) for i in range(len(g)) if bo[bg[i]] == i], np.int64).reshape(-1, 2)
    err = 1.0 - s[pairs[:, 0], pairs[:, 1]] if len(pairs) else np.zeros(0)
    return ModeMatch(pairs, err, len(g) - len(pairs), len(o) - len(pairs))


@dataclasses.dataclass
class LabelCompare:
    n_fg: int
    mismatched: int           # mismatches outside the exempt sets
    exempt_band: int          # pixels within BAND of the bandwidth threshold
    exempt_tie: int           # argmax near-ties
    mismatched_exempt: int    # mismatches inside the exempt sets
    unmatched_mode_pixels: int


def compare_labels(gpu_labels, res, match: ModeMatch, thr: float) -> LabelCompare:
    """Compare GPU labels (H*W, -1 background) with the oracle result."""
    ol = np.asarray(res.labels).reshape(-1)
    band = np.abs(res.best - thr) < BAND
    tie = np.abs(res.best - res.second) < BAND
    return compare_labels_fg(gpu_labels, res.fg, ol[res.fg], band, tie, match)


def compare_labels_fg(gpu_labels, fg, o_fg, band, tie, match: ModeMatch) -> LabelCompare:
    """The same from the oracle's foreground labels and exempt masks (per
    foreground pixel, raster order)."""
    gl = np.asarray(gpu_labels).reshape(-1).astype(np.int64)
    bg_ok = np.all(gl[np.setdiff1d(np.arange(len(gl)), fg)] == -1)
    assert bg_ok, "background pixels must be labelled -1"
    remap = np.full(max(1, gl.max() + 1), -2, np.int64)
    for gi, oi in match.pairs:
        remap[gi] = oi
    g_fg = gl[fg]
    mapped = np.where(g_fg >= 0, remap[np.clip(g_fg, 0, None)], -1)
    o_fg = np.asarray(o_fg).astype(np.int64)
    exempt = band | tie
    unmatched = mapped == -2
    bad = (mapped != o_fg) & ~unmatched
    return LabelCompare(len(fg), int(np.count_nonzero(bad & ~exempt)), int(band.sum()), int(tie.sum()),
                        int(np.count_nonzero(bad & exempt)), int(unmatched.sum()))


def load_precision1024():
    """The stored oracle result of the 1024x1024 precision workload
    (tests/golden/precision1024_oracle.npz, written by make_precision1024.py
    from oracle/ alone): a dict of modes, mode_counts, fg_labels, band, tie,
    bandwidth and stats."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "precision1024_oracle.npz")
    z = np.load(path)
    n = int(z["n_fg"])
    return {"modes": z["modes"], "mode_counts": z["mode_counts"], "fg_labels": z["fg_labels"].astype(np.int64),
            "band": np.unpackbits(z["band"])[:n].astype(bool), "tie": np.unpackbits(z["tie"])[:n].astype(bool),
            "bandwidth": float(z["bandwidth"]), "stats": json.loads(bytes(z["stats"]).decode())}
