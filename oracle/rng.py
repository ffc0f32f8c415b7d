"""Counter-based splitmix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014; the 64-bit finaliser constants of Vigna's
published splitmix64).  Output k (k = 0, 1, ...) of the stream seeded with s is
    z = s + (k + 1) * 0x9E3779B97F4A7C15            (mod 2^64)
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z = z ^ (z >> 31)
and a double in [-1, 1) is 2 * (z >> 11) * 2^-53 - 1.
Used for the power-iteration start vector, which the method draws itself.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int) -> np.ndarray:
    """First n outputs of the stream seeded with `seed` (uint64 array)."""
    with np.errstate(over="ignore"):
        k = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed % (1 << 64)) + k * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed: int, n: int) -> np.ndarray:
    """n doubles in [-1, 1) from the stream."""
    z = splitmix64(seed, n)
    return 2.0 * (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) - 1.0
