"""Online seed optimisation policy, closed forms (oracle side; test infrastructure only).

Sec. 3.2.2 models a seed's landing cell as a draw with probability r/I per
instance (Eq. 12, Eq. 13).  With N seeds, every one of the I instances receives
at least one seed with probability Eq. 14; Eq. 19 inverts Eq. 14 for the
smallest N reaching a target probability P.  Sec. 3.2.4 then drives N: start at
N_initial = 128, double while N < L * N_min, and when N > H * N_min carry
N - N_min to the next frame (L = 2, H = 8).
"""
from __future__ import annotations

import math
from typing import Optional


def p_all_seeded(n_seeds: float, n_inst: float, r: float) -> float:
    """Eq. 14: probability that each of ``n_inst`` equal instances holds at
    least one of ``n_seeds`` seeds, when a seed lands in a given instance with
    probability r / I."""
    if n_inst <= 0:
        return 1.0
    q = 1.0 - r / n_inst
    return (1.0 - q ** n_seeds) ** n_inst


def p_upper_half(n_seeds: float, n_inst: float) -> float:
    """Eq. 15's right-hand side: the r/I of Eq. 14 replaced by 1/(2I)."""
    return p_all_seeded(n_seeds, n_inst, 0.5)


def n_min(p_target: float, n_inst: int, r: float) -> Optional[float]:
    """Eq. 19: N_min = ln(1 - exp(ln(P) / I)) / ln(1 - r / I).

    Returns None when there is no instance yet (I = 0) and 1.0 when r / I >= 1
    (a single seed then lands in "every" instance)."""
    if n_inst <= 0:
        return None
    ratio = r / n_inst
    if ratio >= 1.0:
        return 1.0
    return math.log(1.0 - math.exp(math.log(p_target) / n_inst)) / math.log(1.0 - ratio)


def wants_more_seeds(n_seeds: int, nmin: Optional[float], big_l: float) -> bool:
    """Sec. 3.2.4 doubling test: more seeds are needed while N < L * N_min (or
    while no instance has been found)."""
    if nmin is None:
        return True
    return n_seeds < big_l * nmin


def next_frame_seeds(n_seeds: int, nmin: Optional[float], big_h: float) -> int:
    """Sec. 3.2.4 reduction for the next frame: N - N_min when N > H * N_min,
    N_min rounded up to a whole seed; otherwise N unchanged."""
    if nmin is None or not (n_seeds > big_h * nmin):
        return n_seeds
    return n_seeds - int(math.ceil(nmin))
