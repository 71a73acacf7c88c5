"""Counter-based random numbers for dropout masks (test infrastructure only).

Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC 2011): a 4 x 32-bit counter and a 2 x 32-bit key; ten rounds,
each multiplying counter words 0 and 2 by the constants 0xD2511F53 and
0xCD9E8D57, swapping and xoring the high halves with the other words and the
key, and bumping the key by the Weyl constants 0x9E3779B9, 0xBB67AE85 between
rounds.  Written here from that definition, vectorised over counters in
uint64 numpy arithmetic; the HIP path implements the same generator on its
own.  Pinned by the generator's published known-answer vectors
(tests/golden/philox4x32_10_kat.json).
"""
from __future__ import annotations

import numpy as np

M32 = np.uint64(0xFFFFFFFF)
_MUL0, _MUL1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)


def philox4x32_10(ctr, key):
    """ctr: uint array [..., 4]; key: (k0, k1).  Returns uint64 array [..., 4]
    holding the four 32-bit output words."""
    c = [np.asarray(ctr, dtype=np.uint64)[..., i] & M32 for i in range(4)]
    k0, k1 = np.uint64(key[0]) & M32, np.uint64(key[1]) & M32
    for r in range(10):
        if r > 0:
            k0, k1 = (k0 + _W0) & M32, (k1 + _W1) & M32
        p0 = _MUL0 * c[0]
        p1 = _MUL1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & M32
        hi1, lo1 = p1 >> np.uint64(32), p1 & M32
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=-1)


def keep_threshold(rate: float) -> int:
    """Integer threshold of a dropout rate given as a float32 value: an element
    is kept when its 32-bit draw is >= floor(rate * 2^32)."""
    return min(int(np.floor(np.float64(np.float32(rate)) * 4294967296.0)), 0xFFFFFFFF)


def dropout_mask(seed: int, offset: int, subop: int, n_idx: int, channels: int, rate: float):
    """Dropout multipliers [n_idx, channels] (float64): 0 for a dropped element,
    1 / (1 - rate) for a kept one.  Element e = idx * channels + c draws word 0
    of Philox4x32-10 at counter (e, subop, offset_lo, offset_hi) under key
    (seed_lo, seed_hi)."""
    e = np.arange(n_idx * channels, dtype=np.uint64)
    ctr = np.stack([e, np.full_like(e, subop), np.full_like(e, offset & 0xFFFFFFFF),
                    np.full_like(e, (offset >> 32) & 0xFFFFFFFF)], axis=-1)
    w = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))[..., 0]
    keep = w >= np.uint64(keep_threshold(rate))
    scale = 1.0 / (1.0 - np.float64(np.float32(rate)))
    return (keep.astype(np.float64) * scale).reshape(n_idx, channels)
