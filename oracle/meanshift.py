"""Cosine flat-kernel mean shift in FP64 (oracle side; test infrastructure only).

Definitions followed, with the readings used where the paper is loose:

* Eq. 1 / Eq. 9: cosine similarity s = a.b / (|a||b|), cosine distance d = 1 - s.
  Rows are normalised once, so s is a plain dot product.
* Eq. 3 / Eq. 11: the kernel is flat, k = 1 when d <= h, else 0.  With unit rows
  that is s >= 1 - h (boundary included).
* Eq. 8 / Eq. 10: the new centre is the mean of the window members.  Eq. 10 is
  printed as a mean of distances; it is read as the kernel-weighted mean over
  all vectors, sum_i k_h(y, x_i) x_i / sum_i k_h(y, x_i), which is Eq. 8's mean
  without a neighbour search (Sec. 3.2.1).  The centre is renormalised every
  step; the 1/m factor then cancels.
* Sec. 3.2.1 convergence: the paper stops a seed once its movement between
  two iterations falls below h/1000; the movement is read as the cosine
  distance between consecutive centres, delta = 1 - y_t . y_{t+1} < tol
  (strict), and the seed stops at y_{t+1}.
* Sec. 3.2.3 early stopping: a round of iterations ends once more than gamma of
  its seeds have converged; seeds still moving are discarded.
* Alg. 2 "prune modes": greedy suppression.  Converged endpoints are visited by
  window count (descending), then seed position (ascending); one is kept when its
  similarity to every mode kept so far is below 1 - h.
* Alg. 2 assignment: every foreground vector takes its most similar mode, the
  lowest mode index on ties.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional

import numpy as np


class BadInput(ValueError):
    """A foreground embedding is zero or not finite, so it has no direction."""


def foreground(mask: Optional[np.ndarray], n_pixels: int) -> np.ndarray:
    """Raster indices of the foreground pixels (mask != 0); all pixels when the
    mask is absent."""
    if mask is None:
        return np.arange(n_pixels, dtype=np.int64)
    return np.flatnonzero(np.asarray(mask).reshape(-1) != 0).astype(np.int64)


def normalise(rows: np.ndarray) -> np.ndarray:
    """Eq. 1 denominators: divide each row by its Euclidean norm, in FP64."""
    x = np.asarray(rows, dtype=np.float64)
    if x.size and not np.all(np.isfinite(x)):
        raise BadInput("non-finite foreground embedding")
    norms = np.sqrt(np.sum(x * x, axis=1))
    if np.any(norms == 0.0):
        raise BadInput("zero-norm foreground embedding")
    return x / norms[:, None]


def _seed_block(n: int) -> int:
    # Seeds are processed in blocks only to bound memory; each seed's sums run
    # over all pixels in one matrix product, so the blocking changes nothing.
    return max(1, min(1024, 8_000_000 // max(1, n)))


def shift(y: np.ndarray, x: np.ndarray, thr: float):
    """One mean-shift step for the centres ``y`` (rows) against all vectors ``x``.

    Returns (y_next, delta, members): y_next = V / |V| with
    V = sum_i [y . x_i >= thr] x_i (Eq. 8, 10, 11), delta = 1 - y . y_next, and
    the member count of each window.  A row whose V is zero gets NaN."""
    y = np.asarray(y, dtype=np.float64)
    out = np.empty_like(y)
    delta = np.empty(len(y))
    members = np.empty(len(y), np.int64)
    blk = _seed_block(len(x))
    for a in range(0, len(y), blk):
        yb = y[a:a + blk]
        w = (yb @ x.T) >= thr
        v = w.astype(np.float64) @ x
        nv = np.sqrt(np.sum(v * v, axis=1))
        with np.errstate(invalid="ignore", divide="ignore"):
            yn = v / nv[:, None]
        out[a:a + blk] = yn
        delta[a:a + blk] = 1.0 - np.sum(yb * yn, axis=1)
        members[a:a + blk] = w.sum(axis=1)
    return out, delta, members


def window_margin(y: np.ndarray, x: np.ndarray, thr: float) -> np.ndarray:
    """Distance of the closest vector to each window's edge, min_i |y . x_i - thr|
    (bookkeeping for the comparison with lower-precision results)."""
    out = np.empty(len(y))
    blk = _seed_block(len(x))
    for a in range(0, len(y), blk):
        out[a:a + blk] = np.min(np.abs(y[a:a + blk] @ x.T - thr), axis=1)
    return out


def iterate(x: np.ndarray, seeds: np.ndarray, thr: float, tol: float, gamma: float,
            max_iter: int, trace: bool = False) -> Dict[str, np.ndarray]:
    """Parallel seed iteration of Alg. 2 with the early stop of Sec. 3.2.3.

    ``seeds`` are row indices into ``x``; each centre starts at its seed vector.
    Every iteration moves all still-active centres one step.  A centre whose
    delta falls below ``tol`` is frozen (converged).  Iteration stops after the
    step in which the number of converged centres exceeds gamma * len(seeds), when
    no centre is active, or after ``max_iter`` steps.

    With ``trace`` the result also holds, per seed, the smallest window margin
    over the centres it was evaluated at (``margin``) and the smallest
    |delta - tol| (``tol_margin``); neither changes the iteration."""
    seeds = np.asarray(seeds, dtype=np.int64)
    m = len(seeds)
    y = x[seeds].copy()
    active = np.ones(m, bool)
    conv = np.zeros(m, bool)
    iters = np.zeros(m, np.int64)
    last_delta = np.full(m, np.nan)
    updates = 0
    steps = 0
    active_per_step: List[int] = []
    margin = np.full(m, np.inf)
    tol_margin = np.full(m, np.inf)
    for _ in range(max_iter):
        idx = np.flatnonzero(active)
        if idx.size == 0:
            break
        steps += 1
        active_per_step.append(int(idx.size))
        updates += int(idx.size) * len(x)
        if trace:
            margin[idx] = np.minimum(margin[idx], window_margin(y[idx], x, thr))
        yn, delta, _ = shift(y[idx], x, thr)
        if trace:
            tol_margin[idx] = np.minimum(tol_margin[idx], np.abs(np.nan_to_num(delta, nan=np.inf) - tol))
        dead = ~np.isfinite(delta)
        iters[idx] += 1
        live = idx[~dead]
        y[live] = yn[~dead]
        last_delta[idx] = delta
        active[idx[dead]] = False
        done = live[delta[~dead] < tol]
        conv[done] = True
        active[done] = False
        if conv.sum() > gamma * m:
            break
    out = {"endpoints": y, "converged": conv, "iters": iters, "updates": updates,
           "steps": steps, "last_delta": last_delta, "active_per_step": active_per_step}
    if trace:
        out["margin"] = margin
        out["tol_margin"] = tol_margin
    return out


def window_counts(y: np.ndarray, x: np.ndarray, thr: float) -> np.ndarray:
    """Number of vectors inside each centre's window, |{i : y . x_i >= thr}|."""
    out = np.empty(len(y), np.int64)
    blk = _seed_block(len(x))
    for a in range(0, len(y), blk):
        out[a:a + blk] = ((y[a:a + blk] @ x.T) >= thr).sum(axis=1)
    return out


def prune(endpoints: np.ndarray, counts: np.ndarray, positions: np.ndarray,
          kept: np.ndarray, thr: float) -> List[int]:
    """Greedy mode pruning (Alg. 2 "Prune modes").

    Candidates are visited by window count (descending), then seed position
    (ascending).  A candidate is accepted when its similarity to every mode in
    ``kept`` and to every candidate accepted before it is below ``thr``.
    Returns the accepted candidate indices in acceptance order."""
    order = sorted(range(len(endpoints)), key=lambda j: (-int(counts[j]), int(positions[j])))
    modes = [row for row in np.asarray(kept, dtype=np.float64).reshape(-1, endpoints.shape[1])]
    accepted = []
    for j in order:
        y = endpoints[j]
        if all(float(y @ m) < thr for m in modes):
            modes.append(y)
            accepted.append(j)
    return accepted


def covered_by(x: np.ndarray, modes: np.ndarray, thr: float) -> np.ndarray:
    """Vectors inside the window of at least one of ``modes``."""
    if len(modes) == 0:
        return np.zeros(len(x), bool)
    cov = np.zeros(len(x), bool)
    for a in range(0, len(modes), 256):
        cov |= np.max(x @ modes[a:a + 256].T, axis=1) >= thr
    return cov


def assign(x: np.ndarray, modes: np.ndarray):
    """Alg. 2 assignment: label = argmax_k x . m_k (lowest k on ties), with the
    best and second-best similarities for the exempt-band bookkeeping."""
    n = len(x)
    if len(modes) == 0:
        return (np.full(n, -1, np.int64), np.full(n, -np.inf), np.full(n, -np.inf))
    s = x @ np.asarray(modes, dtype=np.float64).T
    lab = np.argmax(s, axis=1)
    best = s[np.arange(n), lab]
    if s.shape[1] > 1:
        second = np.partition(s, -2, axis=1)[:, -2]
    else:
        second = np.full(n, -np.inf)
    return lab.astype(np.int64), best, second


def classic(x: np.ndarray, thr: float, tol: float, max_iter: int):
    """Alg. 1 by plain Python loops, for tiny inputs only: every vector is a
    seed and is shifted until its cosine step falls below ``tol``.  Returns
    the endpoint and iteration count of every start vector."""
    n, dim = x.shape
    pts = [list(map(float, r)) for r in x]
    ends, its = [], []
    for g in range(n):
        y = list(pts[g])
        k = 0
        while k < max_iter:
            k += 1
            acc = [0.0] * dim
            for p in pts:
                s = 0.0
                for a, b in zip(y, p):
                    s += a * b
                if s >= thr:
                    for d in range(dim):
                        acc[d] += p[d]
            norm = math.sqrt(sum(v * v for v in acc))
            yn = [v / norm for v in acc]
            step = 1.0 - sum(a * b for a, b in zip(y, yn))
            y = yn
            if step < tol:
                break
        ends.append(y)
        its.append(k)
    return np.array(ends), np.array(its)
