"""Counter-based SplitMix64 (Steele, Lea and Flood, OOPSLA 2014).

Output k (k = 0, 1, ...) of the stream with seed s is mix(s + (k+1) * G)
with G = 0x9E3779B97F4A7C15 and mix the SplitMix64 finaliser.  Vectorised
over k with numpy's wrapping uint64 arithmetic.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

BASE_SEED = 2505020719


def mix64(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _fnv1a64(tag: str) -> int:
    h = 0xCBF29CE484222325
    for ch in tag.encode():
        h ^= ch
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def substream(tag: str, seed: int = BASE_SEED) -> int:
    """Seed of the named sub-stream (one per workload, system and purpose)."""
    s = np.uint64((seed ^ _fnv1a64(tag)) & 0xFFFFFFFFFFFFFFFF)
    return int(mix64(s))


def raw(seed: int, count: int, start: int = 0) -> np.ndarray:
    k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(np.uint64(seed) + k * GOLDEN)


def uniform01(seed: int, count: int, start: int = 0) -> np.ndarray:
    """(z >> 11) * 2^-53, in [0, 1)."""
    return (raw(seed, count, start) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def uniform(seed: int, count: int, lo: float, hi: float, start: int = 0) -> np.ndarray:
    return lo + (hi - lo) * uniform01(seed, count, start)


def normal(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Box-Muller on consecutive pairs of outputs 2k, 2k+1 (cosine branch)."""
    u = uniform01(seed, 2 * count, 2 * start)
    u1 = 1.0 - u[0::2]  # in (0, 1]
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def integers(seed: int, count: int, lo: int, hi: int, start: int = 0) -> np.ndarray:
    """Uniform integers in [lo, hi] (inclusive), by scaling uniform01."""
    u = uniform01(seed, count, start)
    return lo + np.minimum((u * (hi - lo + 1)).astype(np.int64), hi - lo)
