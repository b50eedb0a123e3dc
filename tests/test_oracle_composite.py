"""Closed forms, invariants and brute force for the blending of Eq. (2)."""

import math

import numpy as np
import pytest

import scenes
from oracle import composite as comp
from oracle import render

P = scenes.default_params()


def _g(u, v, conic, o, rgb):
    return (np.asarray(u, float), np.asarray(v, float), np.asarray(conic, float),
            np.asarray(o, float), np.asarray(rgb, float))


def test_single_gaussian_closed_form():
    u, v, con, o, rgb = _g([3.2], [4.7], [[0.5, 0.1, 0.8]], [0.7], [[0.2, 0.5, 0.9]])
    xs, ys = np.array([3.0, 4.0, 2.0]), np.array([5.0, 4.0, 3.0])
    C, T, n, _ = comp.composite(xs, ys, [0], u, v, con, o, rgb, P)
    for j in range(3):
        dx, dy = 3.2 - xs[j], 4.7 - ys[j]
        pw = -0.5 * (0.5 * dx * dx + 0.8 * dy * dy) - 0.1 * dx * dy
        a = min(0.99, 0.7 * math.exp(pw))
        if -pw > 4.5 or a < 1 / 255:
            a = 0.0
        np.testing.assert_allclose(C[j], np.asarray([0.2, 0.5, 0.9]) * a, atol=1e-15)
        assert T[j] == pytest.approx(1 - a, abs=1e-15)


def test_two_gaussians_closed_form():
    u, v, con, o, rgb = _g([1.0, 1.0], [1.0, 1.0], [[1, 0, 1], [1, 0, 1]], [0.6, 0.5],
                           [[1, 0, 0], [0, 1, 0]])
    C, T, n, _ = comp.composite(np.array([1.0]), np.array([1.0]), [0, 1], u, v, con, o, rgb, P)
    np.testing.assert_allclose(C[0], [0.6, 0.5 * 0.4, 0.0], atol=1e-15)
    assert T[0] == pytest.approx(0.4 * 0.5) and n[0] == 2


def test_alpha_clamp_and_early_stop():
    # opacity 1 clamps to 0.99; after two such layers T = 1e-4 would be hit by the third
    k = 5
    u, v, con, o, rgb = _g([0.0] * k, [0.0] * k, [[1, 0, 1]] * k, [1.0] * k, [[1, 1, 1]] * k)
    C, T, n, _ = comp.composite(np.array([0.0]), np.array([0.0]), list(range(k)), u, v, con, o, rgb, P)
    # T after 1: 0.01, after 2: 1e-4 (not < 1e-4, kept), third would give 1e-6 < 1e-4: stop
    assert n[0] == 2
    assert T[0] == pytest.approx(1e-4, rel=1e-12)
    assert C[0, 0] == pytest.approx(0.99 + 0.99 * 0.01)


@pytest.mark.parametrize("seed", range(5))
def test_scalar_equals_vectorised_micro(seed):
    scene, views = scenes.micro_scene(seed, n=25, width=20, height=16)
    o = render.render_view(scene, views, 0, scenes.default_params(tile=8))
    d = o["dec"]
    conic = np.stack([d["conic_a"], d["conic_b"], d["conic_c"]], 1).astype(float)
    for y in range(16):
        for x in range(20):
            c, T, n = comp.composite_scalar(float(x), float(y), o["order"], d["u"], d["v"], conic,
                                            scene.opacity, o["rgb"], P)
            np.testing.assert_allclose(o["image"][:, y, x], c, atol=1e-12)
            assert abs(o["T"][y, x] - T) < 1e-12 and o["ncon"][y, x] == n


def test_scalar_equals_vectorised_config1_sample():
    c = scenes.make_config(1)
    o = render.render_view(c.scene, c.views, 1, c.params)
    d = o["dec"]
    conic = np.stack([d["conic_a"], d["conic_b"], d["conic_c"]], 1).astype(float)
    rng = np.random.default_rng(0)
    for _ in range(60):
        x, y = int(rng.integers(64)), int(rng.integers(64))
        col, T, n = comp.composite_scalar(float(x), float(y), o["order"], d["u"], d["v"], conic,
                                          c.scene.opacity, o["rgb"], c.params)
        np.testing.assert_allclose(o["image"][:, y, x], col, atol=1e-12)


def test_transmittance_invariants_config1():
    c = scenes.make_config(1)
    for v in range(3):
        o = render.render_view(c.scene, c.views, v, c.params)
        T = o["T"]
        assert np.all(T <= 1.0) and np.all(T >= c.params["t_min"])
        cmax = o["rgb"][o["ids"]].max()
        assert np.all(o["image"].max(0) <= cmax * (1 - T) + 1e-12)
        assert o["flag"].mean() < 0.01


def test_region_equals_full_image():
    c = scenes.make_config(1)
    full = render.render_view(c.scene, c.views, 0, c.params)
    part = render.render_view(c.scene, c.views, 0, c.params, region=(16, 32, 32, 48))
    np.testing.assert_allclose(part["image"], full["image"][:, 32:48, 16:32], atol=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_rendering_visibility_equals_brute_force(seed):
    """The rendering-derived visibility (Gaussians blended into at least one
    pixel) equals the union over pixels of the scalar loop's contributors,
    and is a subset of the survivors (M_t and the LOD test)."""
    scene, views = scenes.micro_scene(seed, n=40, width=20, height=16, n_inst=1)
    p = scenes.default_params(tile=8)
    took, unc = render.raster_visible(scene, views, 0, p)
    o = render.render_view(scene, views, 0, p)
    d = o["dec"]
    conic = np.stack([d["conic_a"], d["conic_b"], d["conic_c"]], 1).astype(float)
    brute = set()
    for y in range(16):
        for x in range(20):
            comp.composite_scalar(float(x), float(y), o["order"], d["u"], d["v"], conic,
                                  scene.opacity, o["rgb"], p, took=brute)
    np.testing.assert_array_equal(np.nonzero(took)[0], np.asarray(sorted(brute), dtype=np.int64))
    assert not np.any(took & ~d["surv"])
    assert took.sum() > 0


def test_rendering_visibility_hidden_gaussian():
    """A Gaussian behind an opaque stack is inside the frustum (in M_t) but
    never blended: the rendering-derived visibility leaves it out."""
    # three opacity-1 layers (alpha clamps to 0.99) then a fourth: T after two
    # layers is 1e-4, so the third and fourth are never blended at the centre
    u, v, con, o, rgb = _g([0.0] * 4, [0.0] * 4, [[1, 0, 1]] * 4, [1.0] * 4, [[1, 1, 1]] * 4)
    tr = {"took": set(), "uncertain": set()}
    comp.composite(np.array([0.0]), np.array([0.0]), [0, 1, 2, 3], u, v, con, o, rgb, P, track=tr)
    assert tr["took"] == {0, 1}
