"""Unrolled mean shift and its gradient with respect to the embeddings, in FP64
(oracle side; test infrastructure only).

The differentiable form runs T steps of the cosine flat-kernel step (Eq. 8,
9, 11, renormalised every step as in the forward method) from given seeds,
with no freezing and no early stop, so every seed takes exactly T steps:

    x_i = e_i / |e_i|                      (Eq. 1: rows normalised once)
    y_0 = x_seed
    V_t = sum_i [y_{t-1} . x_i >= 1 - h] x_i,   y_t = V_t / |V_t|

and returns y_T.  The gradient of a loss L(y_T) with respect to the raw
embeddings e follows from the chain rule.  The window weights are a step
function of y_{t-1} . x_i, whose derivative is zero wherever no similarity
sits exactly on the threshold, so y_t does not depend on y_{t-1} there and
only the last step's direct dependence on the members survives:

    dL/dV_T = (I - y_T y_T^T) dL/dy_T / |V_T|
    dL/dx_i = sum_j [y_{T-1,j} . x_i >= 1 - h] dL/dV_T,j
    dL/de_i = (I - x_i x_i^T) dL/dx_i / |e_i|

This is the exact derivative almost everywhere (not a surrogate); finite
differences agree with it when no similarity of any step lies within the
perturbation of the threshold (``margin`` reports the smallest distance).
"""
from __future__ import annotations

from typing import Tuple

import numpy as np


def _normalise_rows(e: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    e = np.asarray(e, np.float64)
    n = np.linalg.norm(e, axis=1)
    return e / n[:, None], n


def forward(e: np.ndarray, seeds: np.ndarray, h: float, steps: int):
    """T = ``steps`` unrolled steps.  e: (n, D) raw foreground embeddings;
    seeds: indices into the rows of e.  Returns (y_T, y_{T-1}, |V_T|, margin),
    margin being the smallest |y_{t-1} . x_i - (1 - h)| over all steps."""
    if steps < 1:
        raise ValueError("steps must be >= 1")
    x, _ = _normalise_rows(e)
    thr = 1.0 - h
    y = x[np.asarray(seeds, np.int64)]
    margin = np.inf
    y_prev = y
    vnorm = None
    for _ in range(steps):
        s = y @ x.T
        margin = min(margin, float(np.min(np.abs(s - thr))))
        w = (s >= thr).astype(np.float64)
        v = w @ x
        vnorm = np.linalg.norm(v, axis=1)
        y_prev = y
        y = v / vnorm[:, None]
    return y, y_prev, vnorm, margin


def grad(e: np.ndarray, seeds: np.ndarray, h: float, steps: int, g: np.ndarray) -> np.ndarray:
    """dL/de (n, D) for dL/dy_T = g (m, D), at the unrolled forward above."""
    x, en = _normalise_rows(e)
    y, y_prev, vnorm, _ = forward(e, seeds, h, steps)
    g = np.asarray(g, np.float64)
    gv = (g - np.sum(g * y, axis=1, keepdims=True) * y) / vnorm[:, None]
    w = (y_prev @ x.T >= 1.0 - h).astype(np.float64)
    gx = w.T @ gv
    ge = (gx - np.sum(gx * x, axis=1, keepdims=True) * x) / en[:, None]
    return ge


def loss(e: np.ndarray, seeds: np.ndarray, h: float, steps: int, targets: np.ndarray) -> float:
    """L = sum_j y_T,j . target_j, the loss the differentiation workload uses."""
    y, _, _, _ = forward(e, seeds, h, steps)
    return float(np.sum(y * np.asarray(targets, np.float64)))
