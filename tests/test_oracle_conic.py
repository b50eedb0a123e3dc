"""Pins of the inverse 2D covariance (the conic), the cross term of the
Mahalanobis power (Eq. 1, Eq. 2) and the clamp of the EWA Jacobian.

Every expected value here is built without the oracle's own helpers: the
rotation comes from scipy's `Rotation`, the 2D covariance from the Jacobian
written out in closed form, and the inverse from `np.linalg.inv`.  A sign slip
on the off-diagonal term, a factor 2 on the cross term or a transposed
operand anywhere in the oracle fails one of these."""

import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import scenes
from oracle import composite, decide32, grad, project64

F_PX = 64.0   # focal length of the tiny workload's camera (64x64, c = 32)
C_PX = 32.0
# world -> camera rotation of that camera (at the origin, looking along +x,
# OpenCV axes): camera x = -world y, camera y = -world z, camera z = world x
R_W = np.array([[0.0, -1.0, 0.0], [0.0, 0.0, -1.0], [1.0, 0.0, 0.0]])


def single(cam_xyz, scale, quat_wxyz, opacity=0.8):
    """One static Gaussian at camera coordinates `cam_xyz`, SH degree 0 with
    zero coefficients (colour 0.5 in every channel)."""
    c = scenes.make_config(1)
    X, Y, Z = cam_xyz
    s1 = scenes.Scene(
        mean=np.asarray([[Z, -X, -Y]], np.float32), scale=np.asarray([scale], np.float32),
        quat=np.asarray([quat_wxyz], np.float32), opacity=np.asarray([opacity], np.float32),
        sh=np.zeros((1, 1, 3), np.float32), inst=np.zeros(1, np.int32),
        vis_s=np.full(1, -1, np.float32), vis_e=np.full(1, 1, np.float32),
        life_s=np.ones(1, np.float32), life_e=-np.ones(1, np.float32),
        pose=c.scene.pose[:, :1].copy(), sh_degree=0)
    return s1, c.views


def closed_form_cov2d(s1, clamp=math.inf):
    """Sigma'_raw = J R_W Sigma R_W^T J^T in FP64 from the stored binary32
    inputs, Sigma = R diag(s)^2 R^T with R from scipy (quaternion given
    scalar-last to scipy), J the EWA Jacobian with x~ = clamp(X/Z, +-l) Z."""
    w, x, y, z = (float(q) for q in s1.quat[0])
    R = Rotation.from_quat([x, y, z, w]).as_matrix()
    s = s1.scale[0].astype(np.float64)
    Sig = R @ np.diag(s * s) @ R.T
    mw = s1.mean[0].astype(np.float64)
    X, Y, Z = R_W @ mw
    Sc = R_W @ Sig @ R_W.T
    lim = clamp * (0.5 * 64.0 / F_PX)
    xt = min(max(X / Z, -lim), lim) * Z
    yt = min(max(Y / Z, -lim), lim) * Z
    J = np.array([[F_PX / Z, 0.0, -F_PX * xt / Z ** 2], [0.0, F_PX / Z, -F_PX * yt / Z ** 2]])
    return J @ Sc @ J.T, (F_PX * X / Z + C_PX, F_PX * Y / Z + C_PX)


# a strongly anisotropic Gaussian rotated about all three axes, so that the
# 2D covariance has a large off-diagonal term of either sign
CASES = [
    ((0.4, -0.3, 6.0), (0.6, 0.08, 0.2), (0.8, 0.3, -0.2, 0.45)),
    ((-0.5, 0.2, 7.5), (0.05, 0.5, 0.3), (0.2, -0.6, 0.5, 0.58)),
]


def off_diagonal_pixels(u, v, n=3):
    """Integer pixels around (u, v) with both offsets nonzero, in all four
    sign quadrants."""
    off = [k for k in range(-n, n + 1) if k != 0]
    xs, ys = np.meshgrid([round(u) + k for k in off], [round(v) + k for k in off])
    xs, ys = xs.ravel().astype(np.float64), ys.ravel().astype(np.float64)
    keep = (np.abs(xs - u) > 0.25) & (np.abs(ys - v) > 0.25)
    return xs[keep], ys[keep]


def expected_alpha(inv, u, v, xs, ys, o):
    """o exp(-1/2 d^T inv d) with d = (u - x, v - y), d^T inv d written as a
    quadratic form through numpy's matmul."""
    d = np.stack([u - xs, v - ys], 1)
    q = np.einsum("pi,ij,pj->p", d, inv, d)
    return o * np.exp(-0.5 * q)


@pytest.mark.parametrize("case", CASES)
def test_conic_is_inverse_of_dilated_cov(case):
    cam, scale, quat = case
    s1, views = single(cam, scale, quat)
    p = scenes.default_params(jac_clamp=float("inf"))
    cov, (u, v) = closed_form_cov2d(s1)
    assert abs(cov[0, 1]) > 0.2 * math.sqrt(cov[0, 0] * cov[1, 1])  # a real cross term
    inv = np.linalg.inv(cov + p["eps2d"] * np.eye(2))
    d64 = project64.project64(s1, views.W[0], views.K[0], views.wh[0], 0, p)
    np.testing.assert_allclose(d64["cov2d"][0], cov, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(d64["conic"][0], [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-11)
    d32 = decide32.project_cull32(s1, views.W[0], views.K[0], views.wh[0], 0, p)
    got = [float(d32["conic_a"][0]), float(d32["conic_b"][0]), float(d32["conic_c"][0])]
    np.testing.assert_allclose(got, [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=2e-5,
                               atol=2e-6 * np.abs(inv).max())
    pt = grad.to_torch_params(s1, requires_grad=False)
    _, _, conic_t, _, _ = grad.project_t(pt, np.array([0]), s1.inst, views.W[0], views.K[0],
                                         views.wh[0], pt["pose"][0], p, 0)
    np.testing.assert_allclose(conic_t[0].numpy(), [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-11)


@pytest.mark.parametrize("case", CASES)
def test_blended_alpha_matches_quadratic_form(case):
    """At off-diagonal pixels a single Gaussian's contribution is
    c o exp(-1/2 d^T Sigma'_d^-1 d): through `composite` (fed the closed-form
    conic), through the scalar loop, and through the autograd forward."""
    cam, scale, quat = case
    s1, views = single(cam, scale, quat, opacity=0.8)
    o = float(s1.opacity[0])          # the stored (binary32) value
    p = scenes.default_params(jac_clamp=float("inf"))
    cov, (u, v) = closed_form_cov2d(s1)
    inv = np.linalg.inv(cov + p["eps2d"] * np.eye(2))
    xs, ys = off_diagonal_pixels(u, v)
    ref = expected_alpha(inv, u, v, xs, ys, o)
    live = (ref >= p["alpha_min"]) & (ref < p["alpha_max"])
    q = -2.0 * np.log(ref / o)
    live &= 0.5 * q <= p["cutoff"]
    assert live.sum() >= 6 and np.any((xs - u) * (ys - v) > 0) and np.any((xs - u) * (ys - v) < 0)
    xs, ys, ref = xs[live], ys[live], ref[live]
    conic = np.array([[inv[0, 0], inv[0, 1], inv[1, 1]]])
    rgb = np.full((1, 3), 0.5)
    C, T, n, _ = composite.composite(xs, ys, [0], np.array([u]), np.array([v]), conic,
                                     np.array([o]), rgb, p)
    np.testing.assert_allclose(C[:, 0], 0.5 * ref, rtol=1e-12)
    np.testing.assert_allclose(T, 1.0 - ref, rtol=1e-12)
    for k in range(len(xs)):
        Cs, Ts, _ = composite.composite_scalar(xs[k], ys[k], [0], [u], [v], conic, [o], rgb, p)
        assert Cs[0] == pytest.approx(0.5 * ref[k], rel=1e-12)
    pt = grad.to_torch_params(s1, requires_grad=False)
    img, _ = grad.render_t(pt, s1, views, 0, np.array([0]), p)
    got = img[0].numpy()[ys.astype(int), xs.astype(int)]
    np.testing.assert_allclose(got, 0.5 * ref, rtol=1e-10)
    # the binary32 conic and mean of the decision layer give the same alpha to
    # binary32 accuracy (Eq. 2 as the GPU evaluates it)
    d32 = decide32.project_cull32(s1, views.W[0], views.K[0], views.wh[0], 0, p)
    c32 = np.array([[d32["conic_a"][0], d32["conic_b"][0], d32["conic_c"][0]]], np.float64)
    C32, _, _, _ = composite.composite(xs, ys, [0], d32["u"].astype(np.float64),
                                       d32["v"].astype(np.float64), c32, np.array([o]), rgb, p)
    np.testing.assert_allclose(C32[:, 0], 0.5 * ref, rtol=1e-4)


@pytest.mark.parametrize("cam", [(9.0, 1.0, 10.0), (-1.2, -8.5, 10.0), (8.0, 7.0, 9.0)])
def test_jacobian_clamp_closed_form(cam):
    """Beyond 1.3 x the half-FOV tangent the Jacobian uses x~ = l_x p_z
    (likewise y): Sigma'_raw equals the closed form with the clamped tangent,
    and differs from the unclamped one."""
    s1, views = single(cam, (0.3, 0.1, 0.2), (0.9, 0.1, -0.3, 0.2))
    p = scenes.default_params()
    assert p["jac_clamp"] == pytest.approx(1.3)
    cov_c, _ = closed_form_cov2d(s1, clamp=1.3)
    cov_u, _ = closed_form_cov2d(s1)
    assert np.abs(cov_c - cov_u).max() > 1e-3 * np.abs(cov_u).max()
    X, Y, Z = cam
    assert max(abs(X), abs(Y)) / Z > 1.3 * 0.5          # the clamp is active
    d64 = project64.project64(s1, views.W[0], views.K[0], views.wh[0], 0, p)
    np.testing.assert_allclose(d64["cov2d"][0], cov_c, rtol=1e-12, atol=1e-14)
    d32 = decide32.project_cull32(s1, views.W[0], views.K[0], views.wh[0], 0, p)
    np.testing.assert_allclose([d32["a_raw"][0], d32["b"][0], d32["c_raw"][0]],
                               [cov_c[0, 0], cov_c[0, 1], cov_c[1, 1]], rtol=2e-5,
                               atol=2e-6 * np.abs(cov_c).max())
    inv = np.linalg.inv(cov_c + p["eps2d"] * np.eye(2))
    pt = grad.to_torch_params(s1, requires_grad=False)
    _, _, conic_t, _, _ = grad.project_t(pt, np.array([0]), s1.inst, views.W[0], views.K[0],
                                         views.wh[0], pt["pose"][0], p, 0)
    np.testing.assert_allclose(conic_t[0].numpy(), [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-11)


def test_jacobian_clamp_derivative_matches_finite_differences():
    """With the clamp active the tangent is constant in the mean, so the
    derivative of the conic runs only through 1/p_z and the rotation: the
    autograd gradient equals central differences of the closed form."""
    s1, views = single((9.0, 1.0, 10.0), (0.3, 0.1, 0.2), (0.9, 0.1, -0.3, 0.2))
    p = scenes.default_params()
    pt = grad.to_torch_params(s1, requires_grad=True)
    _, _, conic_t, _, _ = grad.project_t(pt, np.array([0]), s1.inst, views.W[0], views.K[0],
                                         views.wh[0], pt["pose"][0], p, 0)
    wts = torch.tensor([0.7, -1.3, 0.4], dtype=torch.float64)
    (conic_t[0] * wts).sum().backward()
    g = pt["mean"].grad.numpy()[0]

    def f(m):
        s2 = scenes.Scene(**{**s1.__dict__, "mean": m.astype(np.float64)[None, :]})
        cov, _ = closed_form_cov2d(s2, clamp=1.3)
        inv = np.linalg.inv(cov + p["eps2d"] * np.eye(2))
        return float(np.dot([inv[0, 0], inv[0, 1], inv[1, 1]], wts.numpy()))

    m0 = s1.mean[0].astype(np.float64)
    fd = np.zeros(3)
    for k in range(3):
        h = 1e-6 * max(1.0, abs(m0[k]))
        e = np.zeros(3)
        e[k] = h
        fd[k] = (f(m0 + e) - f(m0 - e)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9 * np.abs(fd).max())
