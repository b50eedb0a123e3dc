"""Pins of the stochastic adaptive-LOD drop (Eq. 7) and its random numbers."""

import math
import os

import numpy as np
import pytest

import scenes
from oracle import decide32, rng

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        out = rng.philox4x32_10(*v[:6])
        assert [int(x) for x in out] == v[6:], line


def test_uniform_is_uniform():
    u = rng.uniform(np.arange(200_000), 3, 7, 12345)
    assert u.dtype == np.float32 and u.min() >= 0 and u.max() < 1
    hist = np.histogram(u, bins=20, range=(0, 1))[0]
    exp = len(u) / 20
    chi2 = ((hist - exp) ** 2 / exp).sum()
    assert chi2 < 45.3          # 99.99% point of chi^2 with 19 d.o.f.
    # different views / steps / seeds give independent-looking streams
    u2 = rng.uniform(np.arange(200_000), 4, 7, 12345)
    assert abs(np.corrcoef(u, u2)[0, 1]) < 0.01


def test_drop_probability_closed_form():
    """p(0) = 0.01, p(d >= D) = p_max, linear and increasing in between."""
    pmax, D = 0.8, 50.0
    d = np.asarray([0.0, 12.5, 25.0, 50.0, 80.0, 1e4], np.float32)
    p = decide32.lod_drop_probability32(d, pmax, D)
    np.testing.assert_allclose(p, [0.01, 0.01 + 0.79 / 4, 0.01 + 0.79 / 2, 0.8, 0.8, 0.8],
                               rtol=1e-6)
    assert np.all(np.diff(p) >= 0)


def test_deterministic_limit():
    """p_max = 1 and D -> 0+ drops every sub-threshold Gaussian, which is the
    deterministic LOD cull."""
    c = scenes.make_config(2, scale_n=0.02)
    v = 20
    args = (c.scene, c.views.W[v], c.views.K[v], c.views.wh[v], int(c.views.tstep[v]))
    a = decide32.project_cull32(*args, scenes.default_params(lod=True, lod_r=1.0))
    b = decide32.project_cull32(*args, scenes.default_params(
        lod=True, lod_r=1.0, lod_stochastic=True, lod_pmax=1.0, lod_D=1e-30, seed=9))
    np.testing.assert_array_equal(a["surv"], b["surv"])


def test_empirical_drop_rate():
    """Among sub-threshold visible Gaussians the dropped fraction matches the
    mean of p(depth) within a binomial 99.99% interval."""
    c = scenes.make_config(2, scale_n=0.1)
    v = 10
    p = scenes.default_params(lod=True, lod_r=2.0, lod_stochastic=True, lod_pmax=0.9,
                              lod_D=60.0, seed=31, step=4)
    d = decide32.project_cull32(c.scene, c.views.W[v], c.views.K[v], c.views.wh[v],
                                int(c.views.tstep[v]), p)
    sub = d["visible"] & (d["lam_raw"] <= np.float32(4.0))
    probs = decide32.lod_drop_probability32(d["pz"][sub], 0.9, 60.0).astype(np.float64)
    dropped = (sub & ~d["surv"]).sum()
    n = sub.sum()
    assert n > 1000
    mean, sd = probs.sum(), math.sqrt((probs * (1 - probs)).sum())
    assert abs(dropped - mean) <= 4.0 * sd
