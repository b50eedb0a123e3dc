"""Depth order of contributors and per-tile contributor lists.

Eq. (2) composites the Gaussians covering a pixel front to back.  The paper
does not say how ties are broken; reading: ascending (depth bits, Gaussian id),
where the depth bits are the binary32 pattern of the camera-space depth p_z
(positive, so the unsigned pattern orders like the value).  A tile's list is
the restriction of that order to the survivors whose footprint rectangle
contains the tile; the key of a (tile, Gaussian) pair is (tile, depth bits, id).

Pins: `tile_lists` == the brute-force Python `sorted` of key tuples
(`tests/test_oracle_order.py`).
"""

from __future__ import annotations

import numpy as np


def global_order(ids, depth_bits):
    """Survivor ids sorted by (depth bits, id); `depth_bits` is indexed by id."""
    ids = np.asarray(ids, np.int64)
    db = np.asarray(depth_bits)[ids].astype(np.uint64)
    o = np.lexsort((ids, db))
    return ids[o]


def expand_pairs(ids, x0, x1, y0, y1, gx):
    """(tile, id) pairs of every survivor `ids` over its rectangle [x0,x1)x[y0,y1)."""
    ids = np.asarray(ids, np.int64)
    nx = (x1[ids] - x0[ids]).astype(np.int64)
    ny = (y1[ids] - y0[ids]).astype(np.int64)
    cnt = nx * ny
    rep = np.repeat(np.arange(ids.size), cnt)
    start = np.concatenate([[0], np.cumsum(cnt)[:-1]]) if ids.size else np.zeros(0, np.int64)
    off = np.arange(int(cnt.sum()), dtype=np.int64) - np.repeat(start, cnt)
    tx = x0[ids][rep].astype(np.int64) + off % nx[rep]
    ty = y0[ids][rep].astype(np.int64) + off // nx[rep]
    return ty * gx + tx, ids[rep]


def tile_lists(ids, depth_bits, x0, x1, y0, y1, gx, gy):
    """Returns (tile_start (gx*gy+1,), gid_sorted) so that the list of tile t is
    gid_sorted[tile_start[t]:tile_start[t+1]], ordered by (depth bits, id)."""
    tile, gid = expand_pairs(ids, x0, x1, y0, y1, gx)
    db = np.asarray(depth_bits, np.uint64)[gid]
    o = np.lexsort((gid, db, tile))
    tile, gid = tile[o], gid[o]
    counts = np.bincount(tile, minlength=gx * gy)
    start = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return start, gid


def tile_lists_bruteforce(ids, depth_bits, x0, x1, y0, y1, gx, gy):
    """Same as `tile_lists` by enumerating tuples and Python's `sorted`."""
    keys = []
    for i in ids:
        i = int(i)
        for ty in range(int(y0[i]), int(y1[i])):
            for tx in range(int(x0[i]), int(x1[i])):
                keys.append((ty * gx + tx, int(depth_bits[i]), i))
    keys = sorted(keys)
    counts = [0] * (gx * gy)
    for t, _, _ in keys:
        counts[t] += 1
    start = [0]
    for c in counts:
        start.append(start[-1] + c)
    return np.asarray(start, np.int64), np.asarray([k[2] for k in keys], np.int64)
