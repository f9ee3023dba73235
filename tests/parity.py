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
    gl = np.asarray(gpu_labels).reshape(-1).astype(np.int64)
    ol = np.asarray(res.labels).reshape(-1)
    fg = res.fg
    bg_ok = np.all(gl[np.setdiff1d(np.arange(len(gl)), fg)] == -1)
    assert bg_ok, "background pixels must be labelled -1"
    remap = np.full(max(1, gl.max() + 1), -2, np.int64)
    for gi, oi in match.pairs:
        remap[gi] = oi
    g_fg = gl[fg]
    mapped = np.where(g_fg >= 0, remap[np.clip(g_fg, 0, None)], -1)
    o_fg = ol[fg]
    band = np.abs(res.best - thr) < BAND
    tie = np.abs(res.best - res.second) < BAND
    exempt = band | tie
    unmatched = mapped == -2
    bad = (mapped != o_fg) & ~unmatched
    return LabelCompare(len(fg), int(np.count_nonzero(bad & ~exempt)), int(band.sum()), int(tie.sum()),
                        int(np.count_nonzero(bad & exempt)), int(unmatched.sum()))
