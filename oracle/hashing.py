"""32-bit integer mixing used for aggregation priorities (oracle).

The finaliser of Austin Appleby's MurmurHash3 (public domain): xor-shift by
16, multiply by 0x85ebca6b, xor-shift by 13, multiply by 0xc2b2ae35,
xor-shift by 16, all modulo 2^32.  Pure integer arithmetic, so every
implementation produces identical priorities.
"""
from __future__ import annotations

import numpy as np

GOLDEN32 = 0x9E3779B9


def fmix32(h):
    h = np.asarray(h, dtype=np.uint64) & np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(16)
    h = (h * np.uint64(0x85EBCA6B)) & np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(13)
    h = (h * np.uint64(0xC2B2AE35)) & np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(16)
    return h


def level_seed(level: int) -> int:
    return (GOLDEN32 * (level + 1)) & 0xFFFFFFFF


def priority_key(n: int, level: int) -> np.ndarray:
    """Total order on nodes: (fmix32(i xor seed(level)), i) compared
    lexicographically, packed as one unsigned 64-bit key."""
    i = np.arange(n, dtype=np.uint64)
    h = fmix32(i ^ np.uint64(level_seed(level)))
    return (h << np.uint64(32)) | i
