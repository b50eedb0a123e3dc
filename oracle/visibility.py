"""Temporal-visibility state (Sec. 3.3 "Temporal separation", Eqs. 5-6).

Every Gaussian carries a temporal visibility v = (v_s, v_e), initially (-1, 1),
and a point life l = (l_s, l_e), initially (1, -1).  After rendering time t with
visible mask M_t (Eq. 5):  l_s <- min(l_s, t), l_e <- max(l_e, t) where M_t[i].
After all training times (Eq. 6):  v_s <- l_s - 0.1, v_e <- l_e + 0.1.
New points start visible at all times, and the visibility is reset to all
visible periodically.

Readings: arithmetic in binary32 (the state's storage type) with the margin
rounded to f32 once; FOLD keeps the point life; RESET restores both v and l to
their initial values.  UPDATE over several views is order independent (min and
max commute).

Pins: the worked lifecycle in `tests/golden/visibility_lifecycle.txt`
(hand-computed from Eqs. 5-6) and the invariants in
`tests/test_oracle_visibility.py`.
"""

from __future__ import annotations

import numpy as np

F = np.float32


def initial(n):
    return (np.full(n, -1.0, F), np.full(n, 1.0, F), np.full(n, 1.0, F), np.full(n, -1.0, F))


def update(life_s, life_e, masks, ts):
    """Eq. (5) for every view v of a batch: masks (V, N) bool, ts (V,) f32."""
    ls = np.array(life_s, F)
    le = np.array(life_e, F)
    for m, t in zip(masks, ts):
        t = F(t)
        m = np.asarray(m, bool)
        ls = np.where(m, np.minimum(ls, t), ls)
        le = np.where(m, np.maximum(le, t), le)
    return ls.astype(F), le.astype(F)


def fold(life_s, life_e, margin=0.1):
    """Eq. (6): v_s = l_s - margin, v_e = l_e + margin (binary32)."""
    mg = F(margin)
    return (np.asarray(life_s, F) - mg).astype(F), (np.asarray(life_e, F) + mg).astype(F)


def reset(n):
    """Periodic reset: every Gaussian visible at all times again."""
    return initial(n)
