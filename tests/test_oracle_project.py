"""Closed-form and property pins of the projection (Eq. 1) and the footprint."""

import math

import numpy as np
import pytest

import scenes
from oracle import decide32, project64


def one_gaussian(mean, sigma, quat=(1.0, 0.0, 0.0, 0.0)):
    """A single static isotropic Gaussian and a camera at the origin looking +x."""
    c = scenes.make_config(1)
    s = c.scene
    s1 = scenes.Scene(
        mean=np.asarray([mean], np.float32), scale=np.full((1, 3), sigma, np.float32),
        quat=np.asarray([quat], np.float32), opacity=np.asarray([0.8], np.float32),
        sh=np.zeros((1, 1, 3), np.float32), inst=np.zeros(1, np.int32),
        vis_s=np.full(1, -1, np.float32), vis_e=np.full(1, 1, np.float32),
        life_s=np.ones(1, np.float32), life_e=-np.ones(1, np.float32),
        pose=s.pose[:, :1].copy(), sh_degree=0)
    return s1, c.views


@pytest.mark.parametrize("z,sigma", [(5.0, 0.1), (12.0, 0.3), (40.0, 0.05)])
def test_isotropic_on_axis_closed_form(z, sigma):
    """World (z, 0, 0) is on the optical axis of the +x camera at depth z:
    Sigma'_raw = diag((f sigma / z)^2, (f sigma / z)^2), (u, v) = (c_x, c_y),
    R = ceil(3 sqrt((f sigma/z)^2 + eps))."""
    s1, views = one_gaussian((z, 0.0, 0.0), sigma, quat=(0.3, -0.5, 0.2, 0.7))
    p = scenes.default_params()
    f = 64.0
    sigma = float(np.float32(sigma))          # the stored (binary32) value
    e = (f * sigma / z) ** 2
    d = project64.project64(s1, views.W[0], views.K[0], views.wh[0], 0, p)
    np.testing.assert_allclose(d["cov2d"][0], np.diag([e, e]), rtol=1e-12, atol=1e-14)
    assert d["u"][0] == pytest.approx(32.0, abs=1e-12)
    assert d["v"][0] == pytest.approx(32.0, abs=1e-12)
    assert d["rad"][0] == math.ceil(3 * math.sqrt(e + 0.3))
    d32 = decide32.project_cull32(s1, views.W[0], views.K[0], views.wh[0], 0, p)
    np.testing.assert_allclose([d32["a_raw"][0], d32["c_raw"][0]], [e, e], rtol=2e-6)
    assert abs(d32["b"][0]) < 1e-6 * e
    assert d32["rad"][0] == math.ceil(3 * math.sqrt(e + 0.3))


@pytest.mark.parametrize("X,Y,Z", [(2.0, 0.0, 8.0), (0.0, -1.5, 6.0), (1.0, 2.0, 10.0)])
def test_isotropic_off_axis_closed_form(X, Y, Z):
    """Camera coordinates (X, Y, Z) (world (Z, -X, -Y)), isotropic sigma:
    Sigma' = sigma^2 J J^T with J = [[f/Z, 0, -f X/Z^2], [0, f/Z, -f Y/Z^2]]."""
    sigma = 0.2
    s1, views = one_gaussian((Z, -X, -Y), sigma)
    p = scenes.default_params(jac_clamp=float("inf"))
    f = 64.0
    sigma = float(np.float32(sigma))
    J = np.array([[f / Z, 0, -f * X / Z ** 2], [0, f / Z, -f * Y / Z ** 2]])
    ref = sigma ** 2 * J @ J.T
    d = project64.project64(s1, views.W[0], views.K[0], views.wh[0], 0, p)
    np.testing.assert_allclose(d["cov2d"][0], ref, rtol=1e-12, atol=1e-14)
    assert d["u"][0] == pytest.approx(f * X / Z + 32, abs=1e-12)
    assert d["v"][0] == pytest.approx(f * Y / Z + 32, abs=1e-12)
    d32 = decide32.project_cull32(s1, views.W[0], views.K[0], views.wh[0], 0, p)
    np.testing.assert_allclose([d32["a_raw"][0], d32["b"][0], d32["c_raw"][0]],
                               [ref[0, 0], ref[0, 1], ref[1, 1]], rtol=1e-5, atol=1e-7)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("tile", [8, 16, 32])
def test_cutoff_ellipse_inside_rect(seed, tile):
    """Every integer pixel where -power <= cutoff lies in a tile of the rect,
    so the image does not depend on the tile size (binary32 values, FP64 test)."""
    scene, views = scenes.micro_scene(seed, n=40, width=70, height=50, n_inst=1)
    p = scenes.default_params(tile=tile)
    d = decide32.project_cull32(scene, views.W[0], views.K[0], views.wh[0], 0, p)
    ys, xs = np.mgrid[0:50, 0:70]
    xs, ys = xs.ravel().astype(np.float64), ys.ravel().astype(np.float64)
    checked = 0
    for i in np.nonzero(d["visible"])[0]:
        dx = float(d["u"][i]) - xs
        dy = float(d["v"][i]) - ys
        A, B, C = (float(d["conic_a"][i]), float(d["conic_b"][i]), float(d["conic_c"][i]))
        inside = -(-0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy) <= p["cutoff"]
        tx, ty = (xs // tile).astype(int), (ys // tile).astype(int)
        in_rect = (tx >= d["x0"][i]) & (tx < d["x1"][i]) & (ty >= d["y0"][i]) & (ty < d["y1"][i])
        assert np.all(in_rect[inside])
        checked += int(inside.sum())
    assert checked > 0


def test_lod_special_cases():
    c = scenes.make_config(2, scale_n=0.02)
    v = 10
    args = (c.scene, c.views.W[v], c.views.K[v], c.views.wh[v], int(c.views.tstep[v]))
    prev = None
    for r in (0.0, 0.5, 1.0, 2.0, 4.0):
        d = decide32.project_cull32(*args, scenes.default_params(lod=True, lod_r=r))
        if r == 0.0:
            np.testing.assert_array_equal(d["surv"], d["visible"])
        else:
            assert not np.any(d["surv"] & ~prev)       # S(r2) subset of S(r1)
        prev = d["surv"]
    assert prev.sum() < d["visible"].sum()


def test_lambda_max_of_diagonal():
    a = np.asarray([1.0, 4.0, 2.5, 0.3], np.float32)
    c = np.asarray([3.0, 0.5, 2.5, 7.0], np.float32)
    lam = decide32.lam_max32(a, c, a * c)
    np.testing.assert_array_equal(lam, np.maximum(a, c))
