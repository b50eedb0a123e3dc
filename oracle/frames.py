"""Frames: rendering time, instance cameras and the conventional transform.

FP64 throughout; the only binary32 step is the single rounding of a composed
camera to f32, which is where the streamlined route hands the camera to the
per-Gaussian projection.

Pins: `tests/test_oracle_frames.py` (instance camera == transform-then-project,
identity slot, time end points, quaternion<->matrix round trip).
"""

from __future__ import annotations

import numpy as np


def time_norm(tau, n_timesteps) -> np.float32:
    """Sec. 3.3 "Temporal separation": the rendering time of the whole scene is
    normalised to [-1, 1].  Reading: timestep tau of T maps to -1 + 2 tau/(T-1)
    (T = 1 maps to 0).  Computed in FP64, rounded once to f32."""
    T = int(n_timesteps)
    if T <= 1:
        return np.float32(0.0)
    return np.float32(-1.0 + 2.0 * float(tau) / float(T - 1))


def as_h(m34):
    """3x4 -> 4x4 homogeneous (FP64)."""
    m34 = np.asarray(m34, np.float64)
    out = np.zeros(m34.shape[:-2] + (4, 4))
    out[..., :3, :] = m34
    out[..., 3, 3] = 1.0
    return out


def instance_cameras64(W34, pose34):
    """Sec. 3.3 "Instance-specific projection": the extrinsic of instance i at
    time t is W_{t,i} = W_t W_{t,i2g}.  `W34` is the 3x4 world->camera matrix of
    one view, `pose34` the (K+1, 3, 4) local->world poses of that view's
    timestep (slot 0 = identity for static Gaussians).

    The product is written out with the summation over j = 0..3 in ascending
    order, so that a binary32 rounding of the result is reproducible.
    Returns the (K+1, 3, 4) FP64 products."""
    W = np.asarray(W34, np.float64)
    G = as_h(pose34)                      # (K+1, 4, 4)
    Wh = as_h(W)
    out = np.zeros(G.shape[:-2] + (3, 4))
    for r in range(3):
        for c in range(4):
            acc = Wh[r, 0] * G[..., 0, c]
            acc = acc + Wh[r, 1] * G[..., 1, c]
            acc = acc + Wh[r, 2] * G[..., 2, c]
            acc = acc + Wh[r, 3] * G[..., 3, c]
            out[..., r, c] = acc
    return out


def camera_centre64(P34):
    """Centre of a camera [R | t] in the frame it maps from: c = -R^T t."""
    P = np.asarray(P34, np.float64)
    R, t = P[..., :3, :3], P[..., :3, 3]
    return -np.einsum("...ji,...j->...i", R, t)


def transform_to_world64(mean, R_G, t_G):
    """Sec. 3.1: the conventional pipeline moves an instance Gaussian to the
    world frame, mu_g = R_G mu + t_G, Sigma_g = R_G Sigma R_G^T (FP64)."""
    return np.einsum("nij,nj->ni", R_G, mean) + t_G


def quat_to_rot64(q):
    """Hamilton unit quaternion (w, x, y, z) -> rotation matrix (FP64).
    The input is normalised first."""
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def rot_to_quat64(R):
    """Rotation matrix -> unit quaternion (w, x, y, z), FP64, w >= 0 branch
    chosen by the largest of (trace, R00, R11, R22) (Shepperd's method)."""
    R = np.asarray(R, np.float64)
    out = np.empty(R.shape[:-2] + (4,))
    flat_R = R.reshape(-1, 3, 3)
    flat_o = out.reshape(-1, 4)
    for i, m in enumerate(flat_R):
        tr = m[0, 0] + m[1, 1] + m[2, 2]
        cand = [tr, m[0, 0], m[1, 1], m[2, 2]]
        b = int(np.argmax(cand))
        if b == 0:
            s = np.sqrt(1.0 + tr) * 2.0
            q = [0.25 * s, (m[2, 1] - m[1, 2]) / s, (m[0, 2] - m[2, 0]) / s, (m[1, 0] - m[0, 1]) / s]
        elif b == 1:
            s = np.sqrt(1.0 + m[0, 0] - m[1, 1] - m[2, 2]) * 2.0
            q = [(m[2, 1] - m[1, 2]) / s, 0.25 * s, (m[0, 1] + m[1, 0]) / s, (m[0, 2] + m[2, 0]) / s]
        elif b == 2:
            s = np.sqrt(1.0 + m[1, 1] - m[0, 0] - m[2, 2]) * 2.0
            q = [(m[0, 2] - m[2, 0]) / s, (m[0, 1] + m[1, 0]) / s, 0.25 * s, (m[1, 2] + m[2, 1]) / s]
        else:
            s = np.sqrt(1.0 + m[2, 2] - m[0, 0] - m[1, 1]) * 2.0
            q = [(m[1, 0] - m[0, 1]) / s, (m[0, 2] + m[2, 0]) / s, (m[1, 2] + m[2, 1]) / s, 0.25 * s]
        q = np.asarray(q)
        if q[0] < 0:
            q = -q
        flat_o[i] = q
    return out


def quat_mul64(a, b):
    """Hamilton product a (x) b of (..., 4) quaternions (w, x, y, z)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    w1, x1, y1, z1 = np.moveaxis(a, -1, 0)
    w2, x2, y2, z2 = np.moveaxis(b, -1, 0)
    return np.stack([
        w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
        w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
        w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
        w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2,
    ], axis=-1)
