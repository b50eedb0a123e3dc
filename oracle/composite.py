"""Front-to-back alpha blending of Eq. (2), FP64.

For a pixel sampled at integer coordinates (x, y) and contributors i in depth
order (see `order`), with 2D mean (u_i, v_i), inverse 2D covariance
(conic) Q_i = [[A, B], [B, C]], opacity o_i and colour c_i:
    d = (u_i - x, v_i - y);  power = -0.5 (A dx^2 + C dy^2) - B dx dy
    skip i if -power > cutoff                   (Mahalanobis cut, reading)
    alpha = min(alpha_max, o_i exp(power));  skip i if alpha < alpha_min
    T' = T (1 - alpha);  stop before i if T' < t_min
    C += c_i alpha T;  T = T'
Output C + T bg, the final transmittance T and the number of contributors.
Eq. (2) is the sum C = sum_i c_i alpha_i prod_{j<i} (1 - alpha_j); the skips,
clamp and stop are the standard 3DGS numerical rules, whose constants the paper
does not give (readings; defaults alpha_min = 1/255, alpha_max = 0.99,
t_min = 1e-4, cutoff = 4.5).

`composite` is vectorised over pixels and sequential over contributors; it
also flags pixels where any evaluated decision quantity lies within relative
`delta` of its threshold (binary32 and FP64 may decide those differently).
`composite_scalar` is the same definition as plain Python loops, for tiny
inputs (pinned equal in `tests/test_oracle_composite.py`).
"""

from __future__ import annotations

import math

import numpy as np


def composite(xs, ys, order, u, v, conic, opac, rgb, params, delta=1e-4, track=None):
    """xs, ys: (P,) pixel coordinates.  `order`: contributor ids in blending
    order; u, v, opac (N,), conic (N,3), rgb (N,3) indexed by id.  FP64.

    With a dict `track`, also records per Gaussian id whether it was blended
    into at least one pixel (`track["took"]`, a set) and whether it was
    evaluated at a pixel whose decisions lie in the guard band
    (`track["uncertain"]`, a set): the rendering-derived visibility."""
    xs = np.asarray(xs, np.float64)
    ys = np.asarray(ys, np.float64)
    P = xs.size
    C = np.zeros((P, 3))
    T = np.ones(P)
    done = np.zeros(P, bool)
    flag = np.zeros(P, bool)
    ncon = np.zeros(P, np.int64)
    cut, amin, amax, tmin = (params["cutoff"], params["alpha_min"], params["alpha_max"],
                             params["t_min"])
    for i in order:
        dx = float(u[i]) - xs
        dy = float(v[i]) - ys
        A, B, Cc = (float(q) for q in conic[i])
        power = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy
        live = ~done
        cut_i = -power > cut
        flag |= live & (np.abs(-power - cut) <= delta * cut)
        raw = float(opac[i]) * np.exp(power)
        alpha = np.minimum(amax, raw)
        ev = live & ~cut_i
        small = alpha < amin
        flag |= ev & (np.abs(alpha - amin) <= delta * amin)
        Tn = T * (1.0 - alpha)
        act = ev & ~small
        flag |= act & (np.abs(Tn - tmin) <= delta * tmin)
        stop = act & (Tn < tmin)
        con = act & ~stop
        if track is not None:
            if con.any():
                track["took"].add(int(i))
            if (ev & flag).any():
                track["uncertain"].add(int(i))
        C += np.where(con[:, None], np.asarray(rgb[i], np.float64)[None, :] * (alpha * T)[:, None], 0.0)
        T = np.where(con, Tn, T)
        ncon += con
        done |= stop
    bg = np.asarray(params["bg"], np.float64)
    return C + T[:, None] * bg[None, :], T, ncon, flag


def composite_scalar(x, y, order, u, v, conic, opac, rgb, params, took=None):
    """One pixel, plain Python floats and loops (brute force); ids blended
    into the pixel are added to the set `took` when one is given."""
    Cr = [0.0, 0.0, 0.0]
    T = 1.0
    n = 0
    for i in order:
        dx = float(u[i]) - x
        dy = float(v[i]) - y
        A, B, Cc = (float(q) for q in conic[i])
        power = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy
        if -power > params["cutoff"]:
            continue
        alpha = min(params["alpha_max"], float(opac[i]) * math.exp(power))
        if alpha < params["alpha_min"]:
            continue
        Tn = T * (1.0 - alpha)
        if Tn < params["t_min"]:
            break
        for ch in range(3):
            Cr[ch] += float(rgb[i][ch]) * alpha * T
        T = Tn
        n += 1
        if took is not None:
            took.add(int(i))
    return [Cr[ch] + T * params["bg"][ch] for ch in range(3)], T, n
