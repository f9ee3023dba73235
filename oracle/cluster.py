"""Alg. 2 under the online seed optimisation policy, in FP64 (oracle side;
test infrastructure only).

Control flow, in the paper's terms (Sec. 3.2, Fig. 3: the CPU steers the seed
count, the GPU iterates the seeds):

1. Foreground vectors in raster order, normalised (Eq. 1); r = n / (H W).
2. Seed order: the keyed permutation of ``seed_order``.
3. Rounds.  Round seeds are the first N - N_used positions of the seed order
   whose pixels are neither covered by a mode nor used as a seed before.  They
   are iterated in parallel with early stopping (Sec. 3.2.3); converged
   endpoints are pruned against all modes kept so far (Alg. 2); pixels within
   h of a new mode become covered.  Then I = number of modes, N_min from
   Eq. 19, and N doubles while N < L * N_min (Sec. 3.2.4).  The rounds end when
   no pixel is left to seed or N >= L * N_min.
4. The next frame's N is N - N_min when N > H * N_min (Sec. 3.2.4).
5. Every foreground vector takes its most similar mode (Alg. 2).

Reading (not in the paper): coverage and "seeds only from pixels not yet
covered" follow the online policy as stated for this hot path; a used seed
leaves the pool whether or not it converged, so the rounds always end.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

from . import meanshift as ms
from . import osop
from .seed_order import seed_order


@dataclasses.dataclass
class Params:
    bandwidth: float = 0.1         # h (Sec. 4.1 Design, Sec. 4.2)
    conv_tol: Optional[float] = None  # None: h / 1000 (Sec. 3.2.1)
    gamma: float = 0.9             # Sec. 3.2.3
    n_initial: int = 128           # Sec. 3.2.4
    big_l: float = 2.0             # Sec. 3.2.4
    big_h: float = 8.0             # Sec. 3.2.4
    p_target: float = 0.99         # Sec. 3.2.2
    max_iter: int = 100
    max_rounds: int = 32
    seed: int = 0
    n_state_in: int = 0            # N carried from the previous frame; <= 0: n_initial

    @property
    def tol(self) -> float:
        return self.conv_tol if (self.conv_tol is not None and self.conv_tol > 0) \
            else self.bandwidth / 1000.0


@dataclasses.dataclass
class RoundLog:
    seeds: np.ndarray        # foreground ordinals of this round's seeds
    positions: np.ndarray    # their positions in the seed order
    endpoints: np.ndarray
    converged: np.ndarray
    iters: np.ndarray
    counts: np.ndarray       # window counts at converged endpoints (-1 otherwise)
    accepted: List[int]      # indices (into this round's seeds) that became modes
    steps: int
    n_seeds_after: int       # N after the controller ran
    n_min: Optional[float]


@dataclasses.dataclass
class Result:
    modes: np.ndarray        # (K, D) FP64 unit rows, in acceptance order
    mode_counts: np.ndarray  # window count of each mode
    labels: np.ndarray       # (H*W,) int64, -1 on background
    fg: np.ndarray           # raster indices of the foreground
    x: np.ndarray            # (n, D) normalised foreground vectors
    best: np.ndarray         # (n,) similarity to the assigned mode
    second: np.ndarray       # (n,) second-best similarity
    rounds: List[RoundLog]
    stats: dict


def cluster(emb: np.ndarray, mask: Optional[np.ndarray], params: Params) -> Result:
    """Cluster one frame.  ``emb`` is (H, W, D) (or (P, D)); ``mask`` is (H, W)
    (or (P,)), nonzero for foreground, or None for all pixels."""
    emb = np.asarray(emb)
    dim = emb.shape[-1]
    rows = emb.reshape(-1, dim)
    n_pix = rows.shape[0]
    fg = ms.foreground(mask, n_pix)
    n = len(fg)
    thr = 1.0 - params.bandwidth
    stats = dict(n_fg=n, rounds=0, seeds_used=0, iterations_total=0, n_discarded=0,
                 n_uncovered=0, n_state_out=0, seed_pixel_updates=0, n_min=float("nan"))
    n_seeds = params.n_state_in if params.n_state_in > 0 else params.n_initial
    if n == 0:
        stats["n_state_out"] = n_seeds
        return Result(np.zeros((0, dim)), np.zeros(0, np.int64), np.full(n_pix, -1, np.int64), fg,
                      np.zeros((0, dim)), np.zeros(0), np.zeros(0), [], stats)
    x = ms.normalise(rows[fg])
    r = n / n_pix
    order = seed_order(n, params.seed)
    uncovered = np.ones(n, bool)
    used = np.zeros(n, bool)
    modes: List[np.ndarray] = []
    mode_counts: List[int] = []
    n_used = 0
    nmin: Optional[float] = None
    cursor = 0  # every position before it is used or covered
    logs: List[RoundLog] = []
    for _ in range(params.max_rounds):
        want = n_seeds - n_used
        pos = []
        j = cursor
        while len(pos) < want and j < n:
            p = order[j]
            if uncovered[p] and not used[p]:
                pos.append(j)
            j += 1
        if want > 0:
            cursor = j
        if not pos:
            break
        pos = np.array(pos, np.int64)
        seeds = order[pos]
        used[seeds] = True
        n_used += len(seeds)
        stats["rounds"] += 1
        stats["seeds_used"] += len(seeds)
        it = ms.iterate(x, seeds, thr, params.tol, params.gamma, params.max_iter)
        stats["iterations_total"] += it["steps"]
        stats["seed_pixel_updates"] += it["updates"]
        conv = it["converged"]
        stats["n_discarded"] += int((~conv).sum())
        cidx = np.flatnonzero(conv)
        counts = np.full(len(seeds), -1, np.int64)
        counts[cidx] = ms.window_counts(it["endpoints"][cidx], x, thr)
        kept = np.array(modes) if modes else np.zeros((0, dim))
        acc_local = ms.prune(it["endpoints"][cidx], counts[cidx], pos[cidx], kept, thr)
        accepted = [int(cidx[a]) for a in acc_local]
        new_modes = it["endpoints"][accepted]
        for a in accepted:
            modes.append(it["endpoints"][a])
            mode_counts.append(int(counts[a]))
        uncovered &= ~ms.covered_by(x, new_modes, thr)
        # Controller (Sec. 3.2.4).
        left = bool(np.any(uncovered & ~used))
        go_on = False
        if left:
            if len(modes) == 0:
                n_seeds *= 2
                go_on = True
            else:
                nmin = osop.n_min(params.p_target, len(modes), r)
                if osop.wants_more_seeds(n_seeds, nmin, params.big_l):
                    n_seeds *= 2
                    go_on = True
        if len(modes) > 0:
            nmin = osop.n_min(params.p_target, len(modes), r)
        logs.append(RoundLog(seeds, pos, it["endpoints"], conv, it["iters"], counts, accepted,
                             it["steps"], n_seeds, nmin))
        if not go_on:
            break
    m = np.array(modes) if modes else np.zeros((0, dim))
    lab, best, second = ms.assign(x, m)
    labels = np.full(n_pix, -1, np.int64)
    labels[fg] = lab
    stats["n_uncovered"] = int(np.count_nonzero(best < thr))
    stats["n_min"] = float(nmin) if nmin is not None else float("nan")
    stats["n_state_out"] = osop.next_frame_seeds(n_seeds, nmin, params.big_h)
    return Result(m, np.array(mode_counts, np.int64), labels, fg, x, best, second, logs, stats)


def lockstep(emb: np.ndarray, mask: Optional[np.ndarray], seeds_fg: np.ndarray, params: Params):
    """One round of the seed iteration on an explicit seed list (foreground
    ordinals), plus window counts at the converged endpoints, with the margin
    bookkeeping of ``meanshift.iterate(trace=True)`` and ``end_margin``, the
    window margin at each endpoint."""
    emb = np.asarray(emb)
    dim = emb.shape[-1]
    rows = emb.reshape(-1, dim)
    fg = ms.foreground(mask, rows.shape[0])
    x = ms.normalise(rows[fg])
    thr = 1.0 - params.bandwidth
    it = ms.iterate(x, np.asarray(seeds_fg), thr, params.tol, params.gamma, params.max_iter, trace=True)
    counts = np.full(len(seeds_fg), -1, np.int64)
    c = np.flatnonzero(it["converged"])
    counts[c] = ms.window_counts(it["endpoints"][c], x, thr)
    it["counts"] = counts
    it["end_margin"] = ms.window_margin(np.nan_to_num(it["endpoints"]), x, thr)
    it["x"] = x
    return it


def mode_error(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """1 - cos between matching rows, in FP64."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    na = np.linalg.norm(a, axis=1)
    nb = np.linalg.norm(b, axis=1)
    return 1.0 - np.sum(a * b, axis=1) / (na * nb)


__all__ = ["Params", "Result", "RoundLog", "cluster", "lockstep", "mode_error", "math"]
