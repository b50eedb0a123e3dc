"""Counter-based random numbers for the stochastic LOD drop (Eq. 7).

Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11): a 4 x 32-bit counter is mixed with a 2 x 32-bit key
by ten rounds of two 32x32->64-bit multiplies with the round keys bumped by
the Weyl constants between rounds.  Written here from that published
definition with Python integers (vectorised with numpy uint64); the GPU side
has its own implementation.

A Gaussian's draw for view v at step s with seed (k0, k1) uses counter
(gid, v, s, 0); u = (first output word >> 8) * 2^-24 is exact in binary32.

Pins: published known-answer vectors and a uniformity check
(`tests/test_oracle_lod.py`).
"""

from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    c0, c1, c2, c3 = (np.asarray(x, np.uint64) for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, np.uint64)
    k1 = np.asarray(k1, np.uint64)
    m = np.uint64(MASK)
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(W0)) & m
            k1 = (k1 + np.uint64(W1)) & m
        p0 = np.uint64(M0) * c0
        p1 = np.uint64(M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & m
        hi1, lo1 = p1 >> np.uint64(32), p1 & m
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return [x.astype(np.uint32) for x in (c0, c1, c2, c3)]


def uniform(gid, view, step, seed):
    """U[0, 1) draw in binary32 for each Gaussian index in `gid`."""
    gid = np.asarray(gid, np.uint64)
    s = int(seed) & 0xFFFFFFFFFFFFFFFF
    out = philox4x32_10(gid, np.full_like(gid, view), np.full_like(gid, step), np.zeros_like(gid),
                        s & MASK, s >> 32)
    return (out[0] >> np.uint32(8)).astype(np.float32) * np.float32(2.0 ** -24)
