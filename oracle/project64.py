"""The conventional route in FP64 (Sec. 3.1, Eq. 1): every instance Gaussian is
first moved to the world frame with its pose W_{t,i2g}, then every Gaussian is
projected with the view's W_t and K_t.

This is the value layer.  It takes its own decisions in FP64; those agree with
the binary32 decisions of `decide32` except within rounding distance of a
threshold (`tests/test_oracle_decide.py` counts the exceptions).

Pins: single isotropic Gaussian on the optical axis (closed form), instance
camera route == this route to 1e-12 (the identity stated for instance-specific
projection in Sec. 3.3), footprint rectangle contains the cutoff ellipse.
"""

from __future__ import annotations

import numpy as np

from . import frames


def project64(scene, W34, Kv, wh, tau, params, route="conventional"):
    """Returns a dict of FP64 (N,) arrays: px, py, pz, u, v, cov2d (N,2,2) raw,
    cov2d_d dilated, det_d, lam_d, lam_raw, rad, rect (x0,x1,y0,y1), conic (N,3),
    visible (FP64 decision), keep, surv, dir (N,3) unit viewing direction in the
    instance-local frame, and t.

    route = "conventional": transform to world, project with W_t.
    route = "instance":     project local means with P = W_t G (FP64)."""
    N = scene.n
    t = float(frames.time_norm(tau, scene.n_timesteps))
    pose = np.asarray(scene.pose[tau], np.float64)          # (K+1, 3, 4)
    k = scene.inst
    mean = scene.mean.astype(np.float64)
    Rl = frames.quat_to_rot64(scene.quat)                    # local rotation
    s = scene.scale.astype(np.float64)
    Sig = np.einsum("nij,nj,nkj->nik", Rl, s * s, Rl)        # R diag(s^2) R^T
    W = np.asarray(W34, np.float64)

    if route == "conventional":
        RG, tG = pose[k, :, :3], pose[k, :, 3]
        mg = frames.transform_to_world64(mean, RG, tG)
        Sg = np.einsum("nij,njk,nlk->nil", RG, Sig, RG)
        Rc = np.broadcast_to(W[:, :3], (N, 3, 3))
        tc = np.broadcast_to(W[:, 3], (N, 3))
        p = np.einsum("nij,nj->ni", Rc, mg) + tc
        Sc = np.einsum("nij,njk,nlk->nil", Rc, Sg, Rc)
        cw = frames.camera_centre64(W)
        dir_ = np.einsum("nji,nj->ni", RG, mg - cw)         # back to local frame
    else:
        P = frames.instance_cameras64(W, pose)[k]
        Rc, tc = P[:, :, :3], P[:, :, 3]
        p = np.einsum("nij,nj->ni", Rc, mean) + tc
        Sc = np.einsum("nij,njk,nlk->nil", Rc, Sig, Rc)
        cen = frames.camera_centre64(P)
        dir_ = mean - cen
    dir_ = dir_ / np.linalg.norm(dir_, axis=1, keepdims=True)

    fx, fy, cx, cy = [float(x) for x in Kv]
    Wd, Hd = int(wh[0]), int(wh[1])
    px, py, pz = p[:, 0], p[:, 1], p[:, 2]
    with np.errstate(all="ignore"):
        lx = params["jac_clamp"] * (0.5 * Wd / fx)
        ly = params["jac_clamp"] * (0.5 * Hd / fy)
        tx, ty = px / pz, py / pz
        txc, tyc = np.clip(tx, -lx, lx), np.clip(ty, -ly, ly)
        J = np.zeros((N, 2, 3))
        J[:, 0, 0] = fx / pz
        J[:, 0, 2] = -fx * txc / pz
        J[:, 1, 1] = fy / pz
        J[:, 1, 2] = -fy * tyc / pz
        cov = np.einsum("nij,njk,nlk->nil", J, Sc, J)
        eps = params["eps2d"]
        cov_d = cov + eps * np.eye(2)
        det_d = cov_d[:, 0, 0] * cov_d[:, 1, 1] - cov_d[:, 0, 1] ** 2
        det_r = cov[:, 0, 0] * cov[:, 1, 1] - cov[:, 0, 1] ** 2

        def lam(c, d):
            m = 0.5 * (c[:, 0, 0] + c[:, 1, 1])
            return m + np.sqrt(np.maximum(m * m - d, 0.0))

        lam_d, lam_raw = lam(cov_d, det_d), lam(cov, det_r)
        rad = np.ceil(3.0 * np.sqrt(lam_d))
        u = fx * tx + cx
        v = fy * ty + cy
        ts = int(params["tile"])
        gx, gy = (Wd + ts - 1) // ts, (Hd + ts - 1) // ts
        x0 = np.clip(np.floor((u - rad) / ts), 0, gx)
        x1 = np.clip(np.floor((u + rad) / ts) + 1, 0, gx)
        y0 = np.clip(np.floor((v - rad) / ts), 0, gy)
        y1 = np.clip(np.floor((v + rad) / ts) + 1, 0, gy)
        x0, x1, y0, y1 = [np.nan_to_num(q).astype(np.int64) for q in (x0, x1, y0, y1)]
        conic = np.stack([cov_d[:, 1, 1] / det_d, -cov_d[:, 0, 1] / det_d,
                          cov_d[:, 0, 0] / det_d], axis=1)
        if params.get("temporal", False):
            pass_t = (scene.vis_s.astype(np.float64) <= t) & (t <= scene.vis_e.astype(np.float64))
        else:
            pass_t = np.ones(N, bool)
        depth_ok = (params["z_near"] < pz) & (pz < params["z_far"])
        visible = pass_t & depth_ok & (det_d > 0) & (x1 > x0) & (y1 > y0)
        r = params["lod_r"]
        if params.get("lod", False) and r > 0:
            keep = ~(lam_raw <= r * r)
        else:
            keep = np.ones(N, bool)
    return dict(t=t, p=p, px=px, py=py, pz=pz, u=u, v=v, cov2d=cov, cov2d_d=cov_d,
                det_d=det_d, lam_d=lam_d, lam_raw=lam_raw, rad=rad, x0=x0, x1=x1, y0=y0,
                y1=y1, conic=conic, pass_t=pass_t, depth_ok=depth_ok, visible=visible,
                keep=keep, surv=visible & keep, dir=dir_, gx=gx, gy=gy, Sc=Sc)
