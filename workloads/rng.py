"""SplitMix64 counter-based generator (Steele, Lea and Flood, OOPSLA 2014).

Every synthetic input in this repository is drawn from this generator so that a
workload is fully named by its seed. The k-th output of a stream started at
``seed`` is ``mix(seed + (k + 1) * GAMMA)`` with

    GAMMA = 0x9E3779B97F4A7C15
    mix(z): z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
            z = (z ^ (z >> 27)) * 0x94D049BB133111EB
            return z ^ (z >> 31)

all arithmetic modulo 2**64. A 64-bit output x becomes a double in [0, 1) as
(x >> 11) * 2**-53, which is exact.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


class SplitMix64:
    """Sequential stream; ``next_u64(n)`` returns the next n outputs."""

    def __init__(self, seed: int):
        self.state = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        self.count = 0  # number of outputs drawn so far

    def next_u64(self, n: int) -> np.ndarray:
        k = np.arange(1, n + 1, dtype=np.uint64) + np.uint64(self.count)
        with np.errstate(over="ignore"):
            z = self.state + k * GAMMA
            out = _mix(z)
        self.count += n
        return out

    def uniform(self, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
        """n doubles uniform in [lo, hi): lo + (hi - lo) * u, u = (x >> 11) 2^-53."""
        u = (self.next_u64(n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        return lo + (hi - lo) * u

    def choice_without_replacement(self, n_total: int, k: int) -> np.ndarray:
        """k distinct indices in [0, n_total): the first k of a Fisher-Yates shuffle
        driven by this stream (index i swaps with i + floor(u * (n_total - i)))."""
        if k > n_total:
            raise ValueError("k > n_total")
        perm = np.arange(n_total, dtype=np.int64)
        u = self.uniform(k)
        for i in range(k):
            j = i + int(u[i] * (n_total - i))
            perm[i], perm[j] = perm[j], perm[i]
        return perm[:k].copy()
