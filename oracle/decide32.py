"""The streamlined per-view front end in IEEE binary32 with one fixed order.

Sec. 3.3 lists the per-view steps: select the Gaussians whose temporal
visibility interval contains t; project them with the camera of their
instance, W_{t,i} = W_t W_{t,i2g}; keep those inside the view frustum, which
gives the visible mask M_t; cull those whose 2D scale is at most the LOD
threshold r.  Eq. (1) gives the projection (mean and EWA covariance).

Every discrete decision of these steps (temporal pass, depth test, positive
determinant, footprint rectangle, LOD test, depth key) is taken here in
binary32 because that is the precision the GPU kernels decide in.  The order
of operations is written out term by term below; numpy float32 array
arithmetic rounds every + - * / sqrt to nearest-even and never fuses a
multiply-add, so the result of each expression is fully determined.  The
FP64 route in `project64` is the value layer these decisions are checked
against (`tests/test_oracle_decide.py`): away from thresholds both agree.

Canonical order (s = tile size, p = camera-space mean, q = quaternion):
  camera      P = round32(W (x) G) from FP64, rows summed j = 0..3
  temporal    pass = (v_s <= t) and (t <= v_e)
  mean        p_r = ((P_r0 mu_x + P_r1 mu_y) + P_r2 mu_z) + P_r3
  depth       z_near < p_z < z_far
  plain route mu <- ((G_r0 mu_x + G_r1 mu_y) + G_r2 mu_z) + G_r3,
              R <- R_G R(q) with entries (G_i0 R_0j + G_i1 R_1j) + G_i2 R_2j,
              and the camera is W_t itself
  quaternion  n = sqrt(((w w + x x) + y y) + z z); q <- q / n (each comp.)
  rotation    R00 = 1 - 2 (yy + zz), R01 = 2 (xy - wz), R02 = 2 (xz + wy),
              R10 = 2 (xy + wz), R11 = 1 - 2 (xx + zz), R12 = 2 (yz - wx),
              R20 = 2 (xz - wy), R21 = 2 (yz + wx), R22 = 1 - 2 (xx + yy)
  3D cov      M = R diag(s); S_ij = (M_i0 M_j0 + M_i1 M_j1) + M_i2 M_j2
  Jacobian    tx = p_x / p_z, l_x = jc * ((w/2) / f_x), tc = clamp(tx, +-l_x)
              J00 = f_x / p_z, J02 = -((f_x tc) / p_z)   (same for y)
  A = J R_c   A_0j = J00 R_0j + J02 R_2j, A_1j = J11 R_1j + J12 R_2j
  B = A S     B_ij = (A_i0 S_0j + A_i1 S_1j) + A_i2 S_2j
  2D cov      C_il = (B_i0 A_l0 + B_i1 A_l1) + B_i2 A_l2, (a, b, c) = (C00, C01, C11)
  dilated     a_d = a + eps, c_d = c + eps, det = a_d c_d - b b
  lambda_max  m = 0.5 (a + c), lam = m + sqrt(max(m m - det, 0))
  radius      R = ceil(3 sqrt(lam_d))
  2D mean     u = f_x tx + c_x, v = f_y ty + c_y
  rect        x0 = clamp(floor((u - R) / s), 0, gx), x1 = clamp(floor((u + R)/s) + 1, 0, gx)
  mask        M = pass and depth and det > 0 and x1 > x0 and y1 > y0
  LOD         keep = not (lod and r > 0 and lam_raw <= r r)
  conic       (c_d / det, (-b) / det, a_d / det)
  depth key   the bit pattern of p_z as an unsigned 32-bit integer

Parity: pinned (see `tests/test_oracle_decide.py`, `tests/test_oracle_project.py`).
"""

from __future__ import annotations

import numpy as np

from . import frames

F = np.float32


def _f(x):
    return np.float32(x)


def rot32(quat):
    """Rotation of the normalised quaternion (w, x, y, z), binary32, as a 3x3
    nested list of (N,) arrays in the canonical order."""
    w, x, y, z = quat[:, 0], quat[:, 1], quat[:, 2], quat[:, 3]
    n = np.sqrt(((w * w + x * x) + y * y) + z * z)
    w, x, y, z = w / n, x / n, y / n, z / n
    xx, yy, zz = x * x, y * y, z * z
    xy, xz, yz = x * y, x * z, y * z
    wx, wy, wz = w * x, w * y, w * z
    one, two = _f(1.0), _f(2.0)
    return [[one - two * (yy + zz), two * (xy - wz), two * (xz + wy)],
            [two * (xy + wz), one - two * (xx + zz), two * (yz - wx)],
            [two * (xz - wy), two * (yz + wx), one - two * (xx + yy)]]


def transform32(mean, quat, pose34):
    """The conventional transform in binary32 (plain route, Sec. 3.1):
    mu_g = R_G mu + t_G and R_g = R_G R(q), rows summed in order.
    `pose34` is (N, 3, 4) f32.  Returns (mu_g (N,3), R_g nested 3x3)."""
    R = pose34[:, :, :3]
    t = pose34[:, :, 3]
    mx, my, mz = mean[:, 0], mean[:, 1], mean[:, 2]
    mg = np.stack([((R[:, r, 0] * mx + R[:, r, 1] * my) + R[:, r, 2] * mz) + t[:, r]
                   for r in range(3)], axis=1)
    Rq = rot32(quat)
    Rg = [[(R[:, i, 0] * Rq[0][j] + R[:, i, 1] * Rq[1][j]) + R[:, i, 2] * Rq[2][j]
           for j in range(3)] for i in range(3)]
    return mg.astype(F), Rg


def lam_max32(a, c, det):
    m = _f(0.5) * (a + c)
    disc = m * m - det
    return m + np.sqrt(np.maximum(disc, _f(0.0)))


def lod_drop_probability32(depth, pmax, D):
    """Eq. (7): p = p_max + (p_max - 0.01) min(0, (d - D) / D), binary32 in
    this order."""
    d = np.asarray(depth, F)
    t1 = d - _f(D)
    t2 = t1 / _f(D)
    t3 = np.minimum(_f(0.0), t2)
    return _f(pmax) + (_f(pmax) - _f(0.01)) * t3


def project_cull32(scene, W34, Kv, wh, tau, params, plain=False, view_index=0):
    """Decisions and projected attributes of one view, binary32.

    Returns a dict of (N,) arrays (values of Gaussians that fail an earlier
    test are meaningless and masked by the boolean fields):
      pass_t, depth_ok, visible (= M_t), surv (= M_t and LOD keep),
      px, py, pz, u, v, a_raw, b, c_raw, a, c, det, lam_d, lam_raw, rad,
      x0, x1, y0, y1 (int32 tile rect), conic_a/b/c, depth_bits (uint32),
    plus `cam` (K+1, 3, 4) f32, `cam64`, `t` (f32 time) and for the plain
    route `mean_g`, `rot_g`."""
    N = scene.n
    T = scene.n_timesteps
    t = frames.time_norm(tau, T)
    pose = np.asarray(scene.pose[tau], F)
    cam64 = frames.instance_cameras64(W34, pose)
    cam = cam64.astype(F)
    k = scene.inst
    out = {"t": t, "cam": cam, "cam64": cam64}
    if plain:
        mean, Rq = transform32(scene.mean, scene.quat, pose[k])
        P = np.broadcast_to(cam[0], (N, 3, 4))
        out["mean_g"], out["rot_g"] = mean, Rq
    else:
        mean = scene.mean
        Rq = rot32(scene.quat)
        P = cam[k]

    with np.errstate(all="ignore"):
        if params.get("temporal", False):
            pass_t = (scene.vis_s <= t) & (t <= scene.vis_e)
        else:
            pass_t = np.ones(N, bool)

        mx, my, mz = mean[:, 0], mean[:, 1], mean[:, 2]
        R = P[:, :, :3]
        tr = P[:, :, 3]
        p = [((R[:, r, 0] * mx + R[:, r, 1] * my) + R[:, r, 2] * mz) + tr[:, r] for r in range(3)]
        px, py, pz = p
        depth_ok = (_f(params["z_near"]) < pz) & (pz < _f(params["z_far"]))

        s = [scene.scale[:, 0], scene.scale[:, 1], scene.scale[:, 2]]
        M = [[Rq[i][j] * s[j] for j in range(3)] for i in range(3)]
        S = [[None] * 3 for _ in range(3)]
        for i in range(3):
            for j in range(i, 3):
                S[i][j] = (M[i][0] * M[j][0] + M[i][1] * M[j][1]) + M[i][2] * M[j][2]
                S[j][i] = S[i][j]

        one = _f(1.0)
        fx, fy, cx, cy = (_f(Kv[0]), _f(Kv[1]), _f(Kv[2]), _f(Kv[3]))
        W_, H_ = int(wh[0]), int(wh[1])
        tx = px / pz
        ty = py / pz
        jc = _f(params["jac_clamp"])
        lx = jc * ((_f(0.5) * _f(W_)) / fx)
        ly = jc * ((_f(0.5) * _f(H_)) / fy)
        txc = np.minimum(np.maximum(tx, -lx), lx)
        tyc = np.minimum(np.maximum(ty, -ly), ly)
        j00 = fx / pz
        j02 = -((fx * txc) / pz)
        j11 = fy / pz
        j12 = -((fy * tyc) / pz)
        A0 = [j00 * R[:, 0, j] + j02 * R[:, 2, j] for j in range(3)]
        A1 = [j11 * R[:, 1, j] + j12 * R[:, 2, j] for j in range(3)]
        A = [A0, A1]
        B = [[(A[i][0] * S[0][j] + A[i][1] * S[1][j]) + A[i][2] * S[2][j] for j in range(3)]
             for i in range(2)]

        def C(i, l):
            return (B[i][0] * A[l][0] + B[i][1] * A[l][1]) + B[i][2] * A[l][2]

        a_raw, b, c_raw = C(0, 0), C(0, 1), C(1, 1)
        eps = _f(params["eps2d"])
        a = a_raw + eps
        c = c_raw + eps
        det = a * c - b * b
        det_raw = a_raw * c_raw - b * b
        lam_d = lam_max32(a, c, det)
        lam_raw = lam_max32(a_raw, c_raw, det_raw)
        rad = np.ceil(_f(3.0) * np.sqrt(lam_d))
        u = fx * tx + cx
        v = fy * ty + cy

        ts = int(params["tile"])
        sf = _f(ts)
        gx = (W_ + ts - 1) // ts
        gy = (H_ + ts - 1) // ts

        def clampi(val, hi):
            return np.minimum(np.maximum(val, _f(0.0)), _f(hi))

        x0f = clampi(np.floor((u - rad) / sf), gx)
        x1f = clampi(np.floor((u + rad) / sf) + one, gx)
        y0f = clampi(np.floor((v - rad) / sf), gy)
        y1f = clampi(np.floor((v + rad) / sf) + one, gy)
        # NaN (only possible where depth_ok is False) is mapped to an empty rect
        bad = ~np.isfinite(x0f) | ~np.isfinite(x1f) | ~np.isfinite(y0f) | ~np.isfinite(y1f)
        x0 = np.where(bad, 0, x0f).astype(np.int32)
        x1 = np.where(bad, 0, x1f).astype(np.int32)
        y0 = np.where(bad, 0, y0f).astype(np.int32)
        y1 = np.where(bad, 0, y1f).astype(np.int32)

        visible = pass_t & depth_ok & (det > _f(0.0)) & (x1 > x0) & (y1 > y0)
        r = _f(params["lod_r"])
        if params.get("lod", False) and r > 0:
            drop = lam_raw <= r * r
            if params.get("lod_stochastic", False):
                # Eq. (7): a sub-threshold Gaussian is dropped with probability
                # p(depth); the draw is the counter-based generator of `rng`
                from . import rng
                p = lod_drop_probability32(pz, params["lod_pmax"], params["lod_D"])
                draw = rng.uniform(np.arange(N), view_index, params.get("step", 0),
                                   params.get("seed", 0))
                drop = drop & (draw < p)
            keep = ~drop
        else:
            keep = np.ones(N, bool)
        surv = visible & keep

        conic_a = c / det
        conic_b = (-b) / det
        conic_c = a / det
        depth_bits = pz.astype(F).view(np.uint32)

    out.update(dict(
        pass_t=pass_t, depth_ok=depth_ok, visible=visible, surv=surv, keep=keep,
        px=px, py=py, pz=pz, u=u, v=v, a_raw=a_raw, b=b, c_raw=c_raw, a=a, c=c,
        det=det, lam_d=lam_d, lam_raw=lam_raw, rad=rad,
        x0=x0, x1=x1, y0=y0, y1=y1, gx=gx, gy=gy,
        conic_a=conic_a, conic_b=conic_b, conic_c=conic_c, depth_bits=depth_bits))
    return out
