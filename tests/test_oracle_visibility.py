"""Pins of the temporal-visibility state (Eqs. 5-6)."""

import os

import numpy as np

import scenes
from oracle import decide32, visibility

GOLD = os.path.join(os.path.dirname(__file__), "golden", "visibility_lifecycle.txt")


def _golden():
    masks, ts, life, vis = [], [], None, None
    for line in open(GOLD):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "mask":
            ts.append(float(f[1]))
            masks.append([bool(int(x)) for x in f[2:]])
        elif f[0] == "life":
            life = np.asarray([float(x) for x in f[1:]]).reshape(-1, 2)
        elif f[0] == "vis":
            vis = np.asarray([float(x) for x in f[1:]]).reshape(-1, 2)
    return np.asarray(masks), np.asarray(ts, np.float32), life, vis


def test_golden_lifecycle():
    masks, ts, life, vis = _golden()
    vs, ve, ls, le = visibility.initial(3)
    ls, le = visibility.update(ls, le, masks, ts)
    np.testing.assert_allclose(np.stack([ls, le], 1), life, atol=0)
    vs, ve = visibility.fold(ls, le)
    np.testing.assert_allclose(np.stack([vs, ve], 1), vis, atol=1e-7)


def test_update_idempotent_and_commutative():
    rng = np.random.default_rng(1)
    m = rng.random((6, 500)) < 0.3
    t = rng.uniform(-1, 1, 6).astype(np.float32)
    _, _, ls, le = visibility.initial(500)
    a = visibility.update(ls, le, m, t)
    b = visibility.update(*a, m, t)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    perm = rng.permutation(6)
    c = visibility.update(ls, le, m[perm], t[perm])
    np.testing.assert_array_equal(a[0], c[0])
    np.testing.assert_array_equal(a[1], c[1])
    for v in range(6):
        assert np.all(a[0][m[v]] <= t[v]) and np.all(t[v] <= a[1][m[v]])


def test_fold_is_sound_for_the_temporal_filter():
    """After UPDATE over every timestep and FOLD, a Gaussian that was in M at
    time tau passes the temporal test at tau: the filter skips only Gaussians
    that were not visible (Sec. 3.3)."""
    c = scenes.make_config(2, scale_n=0.02)
    p = dict(c.params, temporal=False)
    masks, ts = [], []
    for v in range(0, 50, 7):
        d = decide32.project_cull32(c.scene, c.views.W[v], c.views.K[v], c.views.wh[v],
                                    int(c.views.tstep[v]), p)
        masks.append(d["visible"])
        ts.append(d["t"])
    _, _, ls, le = visibility.initial(c.scene.n)
    ls, le = visibility.update(ls, le, masks, ts)
    vs, ve = visibility.fold(ls, le)
    for m, t in zip(masks, ts):
        assert np.all((vs <= t) & (t <= ve) | ~m)
    never = ~np.any(masks, 0)
    assert np.all(vs[never] > ve[never])       # the empty interval (0.9, -0.9)


def test_reset_restores_initial_state():
    vs, ve, ls, le = visibility.reset(4)
    np.testing.assert_array_equal(vs, -1)
    np.testing.assert_array_equal(ve, 1)
    np.testing.assert_array_equal(ls, 1)
    np.testing.assert_array_equal(le, -1)
