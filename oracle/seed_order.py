"""Seed order (oracle side; test infrastructure only).

Alg. 2 draws its seeds uniformly at random from the vector set.  Here the draw is a
keyed pseudo-random permutation ``pi`` of the foreground ordinals 0..n-1:
position ``j`` of the seed order holds foreground ordinal ``pi(j)``.  A round
takes the first positions whose pixels are still eligible.

Construction (all published definitions, written out here independently of the
GPU library):

* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): state += 0x9E3779B97F4A7C15,
  output = mix64(state) with the two xor-shift-multiply steps and a final
  xor-shift.  The four round keys are the first four outputs of SplitMix64
  seeded with ``seed``.
* A 4-round balanced Feistel network (Luby and Rackoff 1988) on 2b-bit words,
  round function ``F_r(R) = mix64(R xor K_r) mod 2^b``.  ``b`` is the smallest
  half-width with ``2^(2b) >= n`` (at least 1).
* Cycle walking (Black and Rogaway 2002) turns the permutation of
  ``[0, 2^(2b))`` into one of ``[0, n)``: re-encrypt until the value is < n.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
MUL1 = 0xBF58476D1CE4E5B9
MUL2 = 0x94D049BB133111EB
ROUNDS = 4


def mix64(z: int) -> int:
    """SplitMix64 output function on a Python integer."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * MUL1) & MASK64
    z = ((z ^ (z >> 27)) * MUL2) & MASK64
    return z ^ (z >> 31)


def splitmix64_stream(seed: int, count: int):
    """First ``count`` outputs of SplitMix64 seeded with ``seed``."""
    state = seed & MASK64
    out = []
    for _ in range(count):
        state = (state + GOLDEN) & MASK64
        out.append(mix64(state))
    return out


def half_bits(n: int) -> int:
    k = 0
    while (1 << k) < n:
        k += 1
    return max(1, (k + 1) // 2)


def feistel_encrypt(x: int, b: int, keys) -> int:
    mask = (1 << b) - 1
    left, right = x >> b, x & mask
    for key in keys:
        left, right = right, left ^ (mix64(right ^ key) & mask)
    return (left << b) | right


def position_to_ordinal(j: int, n: int, seed: int) -> int:
    """pi(j) for one position, by cycle walking (pure Python)."""
    b = half_bits(n)
    keys = splitmix64_stream(seed, ROUNDS)
    y = feistel_encrypt(j, b, keys)
    while y >= n:
        y = feistel_encrypt(y, b, keys)
    return y


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(MUL1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(MUL2)
    return z ^ (z >> np.uint64(31))


def seed_order(n: int, seed: int) -> np.ndarray:
    """pi(0..n-1) as an int64 array (vectorised form of position_to_ordinal)."""
    if n <= 0:
        return np.zeros(0, np.int64)
    b = half_bits(n)
    mask = np.uint64((1 << b) - 1)
    keys = [np.uint64(k) for k in splitmix64_stream(seed, ROUNDS)]

    def enc(x):
        left, right = x >> np.uint64(b), x & mask
        for key in keys:
            left, right = right, left ^ (_mix64_np(right ^ key) & mask)
        return (left << np.uint64(b)) | right

    y = enc(np.arange(n, dtype=np.uint64))
    todo = y >= np.uint64(n)
    while np.any(todo):
        y[todo] = enc(y[todo])
        todo = y >= np.uint64(n)
    return y.astype(np.int64)
