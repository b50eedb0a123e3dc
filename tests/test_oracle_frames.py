"""Pins of oracle.frames and of the instance-camera identity (Sec. 3.3)."""

import numpy as np
import pytest

import scenes
from oracle import frames, project64


def test_time_norm_end_points():
    assert frames.time_norm(0, 50) == np.float32(-1.0)
    assert frames.time_norm(49, 50) == np.float32(1.0)
    assert frames.time_norm(0, 1) == np.float32(0.0)
    assert frames.time_norm(1, 3) == np.float32(0.0)
    assert frames.time_norm(2, 5) == np.float32(0.0)


def test_static_slot_is_the_view_camera():
    c = scenes.make_config(1)
    P = frames.instance_cameras64(c.views.W[1], c.scene.pose[1])
    np.testing.assert_array_equal(P[0], c.views.W[1].astype(np.float64))


def test_instance_camera_is_composition():
    rng = np.random.default_rng(5)
    for _ in range(20):
        W = np.zeros((3, 4))
        W[:, :3] = np.linalg.qr(rng.normal(size=(3, 3)))[0]
        W[:, 3] = rng.normal(size=3)
        G = np.zeros((4, 3, 4))
        for k in range(4):
            G[k, :, :3] = np.linalg.qr(rng.normal(size=(3, 3)))[0]
            G[k, :, 3] = rng.normal(size=3) * 10
        P = frames.instance_cameras64(W, G)
        ref = (frames.as_h(W) @ frames.as_h(G))[:, :3, :]
        np.testing.assert_allclose(P, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("seed", range(6))
def test_instance_route_equals_transform_then_project(seed):
    """W_{t,i} = W_t W_{t,i2g}: projecting local means with the instance camera
    gives the conventional transform-then-project result (FP64, 1e-12)."""
    scene, views = scenes.micro_scene(seed, n=30, n_inst=2, sh_degree=2)
    p = scenes.default_params(jac_clamp=float("inf"))
    for v in range(views.n_views):
        a = project64.project64(scene, views.W[v], views.K[v], views.wh[v], int(views.tstep[v]), p)
        b = project64.project64(scene, views.W[v], views.K[v], views.wh[v], int(views.tstep[v]), p,
                                route="instance")
        for key in ("u", "v", "pz"):
            np.testing.assert_allclose(a[key], b[key], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(a["cov2d"], b["cov2d"], rtol=1e-11, atol=1e-12)
        # the viewing direction uses R^T as the inverse rotation; the f32 poses
        # are orthonormal only to ~1e-7, which bounds the agreement here
        np.testing.assert_allclose(a["dir"], b["dir"], rtol=0, atol=1e-6)


def test_quaternion_round_trip_and_product():
    rng = np.random.default_rng(3)
    q = rng.normal(size=(200, 4))
    R = frames.quat_to_rot64(q)
    np.testing.assert_allclose(np.einsum("nij,nkj->nik", R, R), np.broadcast_to(np.eye(3), R.shape),
                               atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-12)
    q2 = frames.rot_to_quat64(R)
    qn = q / np.linalg.norm(q, axis=1, keepdims=True)
    qn = qn * np.sign(qn[:, :1])
    np.testing.assert_allclose(q2, qn, atol=1e-12)
    a, b = rng.normal(size=(50, 4)), rng.normal(size=(50, 4))
    np.testing.assert_allclose(frames.quat_to_rot64(frames.quat_mul64(a, b)),
                               frames.quat_to_rot64(a) @ frames.quat_to_rot64(b), atol=1e-12)
