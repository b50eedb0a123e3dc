"""Reference gradients: torch-CPU FP64 autograd through the conventional route.

The paper optimises the scene by rendering and comparing with the images
(Sec. 3, "reconstruction"); it does not write the derivatives out.  The
reference gradient is the derivative of the forward definition with every
discrete decision frozen: the survivor set and its depth order (taken from
the binary32 decisions, the ones the GPU takes), and per pixel the Mahalanobis
cut, the alpha_min skip, the early stop and the clamps (taken in FP64 here).

The forward restates Eq. (1) and Eq. (2) directly:
  mu_g = R_G mu + t_G,  Sigma = R(q) diag(s)^2 R(q)^T,  Sigma_g = R_G Sigma R_G^T
  p = W mu_g,  Sigma' = J R_W Sigma_g R_W^T J^T + eps I,  u = f p_x/p_z + c
  alpha_i = min(alpha_max, o_i exp(power_i)),  T_i = prod_{j<i} (1 - alpha_j)
  C = sum_i c_i alpha_i T_i + T bg
The loss of a batch of views is the sum over views of the mean absolute error
against the view's target image (per channel and pixel).

Pose gradients: dL/dG for the 3x4 pose G_{tau,k} of every instance slot
k >= 1, and its 6-DoF form under the right perturbation G exp(xi^),
xi = (rho, omega):  M = G~^T D (D = dL/dG~ padded with a zero row),
d rho = M[0:3, 3],  d omega = (M21 - M12, M02 - M20, M10 - M01).

Pins: `tests/test_oracle_grad.py` checks every gradient against FP64 central
finite differences of the same forward (samples whose decisions change
between theta - h and theta + h are skipped) and the 6-DoF form against finite
differences through the matrix exponential.
"""

from __future__ import annotations

import numpy as np
import torch

from . import frames, sh

TD = torch.float64


def _quat_rot(q):
    q = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)


def project_t(params_t, ids, inst, W34, Kv, wh, pose_tau, rp, sh_degree, route="instance"):
    """Differentiable projection + colour of Gaussians `ids`.  Geometry follows
    the conventional route; the viewing direction of the colour is taken in the
    instance frame either as mu - c_{t,i} with c_{t,i} the centre of the
    instance camera P = W G (route "instance", the streamlined definition) or
    as R_G^T (mu_g - c_W) (route "conventional").  Both are the same function
    on rigid poses; as functions of the twelve raw pose entries they differ off
    the rotation manifold, so the raw pose gradient depends on the route while
    its 6-DoF form does not.
    Returns u, v, conic (n,3), opac, rgb (n,3) (torch FP64)."""
    mean, scale, quat, opac, shc = (params_t[k] for k in ("mean", "scale", "quat", "opacity", "sh"))
    idx = torch.as_tensor(ids, dtype=torch.long)
    k = torch.as_tensor(inst[ids], dtype=torch.long)
    G = pose_tau[k]                                       # (n,3,4)
    RG, tG = G[:, :, :3], G[:, :, 3]
    mu = mean[idx]
    mg = torch.einsum("nij,nj->ni", RG, mu) + tG
    Rl = _quat_rot(quat[idx])
    s2 = scale[idx] ** 2
    Sig = torch.einsum("nij,nj,nkj->nik", Rl, s2, Rl)
    Sg = RG @ Sig @ RG.transpose(1, 2)
    W = torch.as_tensor(np.asarray(W34, np.float64))
    Rc, tc = W[:, :3], W[:, 3]
    p = mg @ Rc.T + tc
    Sc = Rc @ Sg @ Rc.T
    fx, fy, cx, cy = [float(x) for x in Kv]
    px, py, pz = p[:, 0], p[:, 1], p[:, 2]
    lx = rp["jac_clamp"] * (0.5 * float(wh[0]) / fx)
    ly = rp["jac_clamp"] * (0.5 * float(wh[1]) / fy)
    txc = torch.clamp(px / pz, -lx, lx)
    tyc = torch.clamp(py / pz, -ly, ly)
    zero = torch.zeros_like(pz)
    J = torch.stack([torch.stack([fx / pz, zero, -fx * txc / pz], -1),
                     torch.stack([zero, fy / pz, -fy * tyc / pz], -1)], -2)
    cov = J @ Sc @ J.transpose(1, 2)
    a = cov[:, 0, 0] + rp["eps2d"]
    b = cov[:, 0, 1]
    c = cov[:, 1, 1] + rp["eps2d"]
    det = a * c - b * b
    conic = torch.stack([c / det, -b / det, a / det], -1)
    u = fx * px / pz + cx
    v = fy * py / pz + cy
    if route == "instance":
        Rcam = Rc @ RG                                     # (n,3,3) rotation of P = W G
        tcam = torch.einsum("ij,nj->ni", Rc, tG) + tc      # translation of P
        cen = -torch.einsum("nji,nj->ni", Rcam, tcam)      # -R_P^T t_P
        dv = mu - cen
    else:
        cw = torch.as_tensor(frames.camera_centre64(np.asarray(W34, np.float64)))
        dv = torch.einsum("nji,nj->ni", RG, mg - cw)
    dv = dv / torch.linalg.norm(dv, dim=-1, keepdim=True)
    rgb, raw = sh.colour(shc[idx], dv, sh_degree, xp=torch)
    return u, v, conic, opac[idx], rgb


def composite_t(xs, ys, u, v, conic, opac, rgb, rp, decisions=None):
    """Eq. (2) for all pixels at once: T_i = prod_{j<i}(1 - alpha_j) over the
    active contributors, truncated at the first early stop (decisions detached).
    If `decisions` is a list, the (act, excluded) masks are appended to it."""
    dx = u[:, None] - xs[None, :]
    dy = v[:, None] - ys[None, :]
    A, B, C = conic[:, 0:1], conic[:, 1:2], conic[:, 2:3]
    power = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy        # (n, P)
    alpha = torch.clamp(opac[:, None] * torch.exp(power), max=rp["alpha_max"])
    with torch.no_grad():
        act = (-power <= rp["cutoff"]) & (alpha >= rp["alpha_min"])
    a_act = torch.where(act, alpha, torch.zeros_like(alpha))
    one_m = 1.0 - a_act
    T_incl = torch.cumprod(one_m, dim=0)
    T_before = torch.cat([torch.ones_like(T_incl[:1]), T_incl[:-1]], 0)
    with torch.no_grad():
        stop = act & (T_incl < rp["t_min"])
        excluded = torch.cumsum(stop.to(torch.int64), 0) > 0
    if decisions is not None:
        decisions.append((act, excluded, alpha.detach() >= rp["alpha_max"]))
    w = torch.where(excluded, torch.zeros_like(a_act), a_act * T_before)   # (n, P)
    Cimg = w.T @ rgb                                                       # (P, 3)
    keep = ~excluded
    T_final = torch.where(keep, one_m, torch.ones_like(one_m)).prod(0)
    bg = torch.as_tensor(np.asarray(rp["bg"], np.float64))
    return Cimg + T_final[:, None] * bg[None, :], T_final


def to_torch_params(scene, requires_grad=True):
    p = {
        "mean": scene.mean, "scale": scene.scale, "quat": scene.quat,
        "opacity": scene.opacity, "sh": scene.sh, "pose": scene.pose,
    }
    return {k: torch.tensor(np.asarray(v, np.float64), dtype=TD, requires_grad=requires_grad)
            for k, v in p.items()}


def render_t(params_t, scene, views, v, order_ids, rp, region=None, decisions=None,
             route="instance"):
    """Differentiable image (3, h, w) of view v over contributors `order_ids`."""
    w, h = int(views.wh[v, 0]), int(views.wh[v, 1])
    x0, y0, x1, y1 = (0, 0, w, h) if region is None else region
    ys, xs = np.mgrid[y0:y1, x0:x1]
    xs_t = torch.as_tensor(xs.ravel().astype(np.float64))
    ys_t = torch.as_tensor(ys.ravel().astype(np.float64))
    tau = int(views.tstep[v])
    if len(order_ids) == 0:
        img = torch.zeros((xs_t.numel(), 3), dtype=TD) + torch.as_tensor(np.asarray(rp["bg"], np.float64))
        T = torch.ones(xs_t.numel(), dtype=TD)
    else:
        u, vv, conic, opac, rgb = project_t(params_t, order_ids, scene.inst, views.W[v], views.K[v],
                                            views.wh[v], params_t["pose"][tau], rp, scene.sh_degree,
                                            route)
        img, T = composite_t(xs_t, ys_t, u, vv, conic, opac, rgb, rp, decisions)
    return img.T.reshape(3, y1 - y0, x1 - x0), T.reshape(y1 - y0, x1 - x0)


def l1_loss_t(img, target):
    return (img - torch.as_tensor(np.asarray(target, np.float64))).abs().mean()


def loss_and_grads(scene, views, view_ids, orders, rp, targets, route="instance"):
    """Sum over views of mean-L1 and its FP64 gradients.

    orders[v] are the contributor ids of view v in blending order (frozen
    decisions).  Returns (loss, images, grads dict of numpy arrays)."""
    pt = to_torch_params(scene)
    loss = torch.zeros((), dtype=TD)
    imgs = {}
    for v in view_ids:
        img, T = render_t(pt, scene, views, v, np.asarray(orders[v]), rp, route=route)
        imgs[v] = (img.detach().numpy(), T.detach().numpy())
        loss = loss + l1_loss_t(img, targets[v])
    loss.backward()
    return float(loss.detach()), imgs, _grads_of(pt, scene)


def _grads_of(pt, scene):
    g = {k: (t.grad.numpy().copy() if t.grad is not None else np.zeros(t.shape))
         for k, t in pt.items()}
    g["pose"][:, 0] = 0.0            # slot 0 is the fixed identity of static Gaussians
    g["pose6"] = pose6(scene.pose, g["pose"])
    return g


def image_vjp(scene, views, rp, parts, route="instance"):
    """Gradients of sum_parts <dC, image of view v over region>: the backward
    of the image for a given dL/dC that is zero outside the regions.

    parts: list of (v, region (x0, y0, x1, y1), contributor ids of the region
    in blending order, dC (3, y1 - y0, x1 - x0)).  Returns the grads dict."""
    pt = to_torch_params(scene)
    total = torch.zeros((), dtype=TD)
    for v, region, order_ids, dC in parts:
        img, _ = render_t(pt, scene, views, v, np.asarray(order_ids), rp, region=region,
                          route=route)
        total = total + (img * torch.as_tensor(np.asarray(dC, np.float64))).sum()
    if total.requires_grad:
        total.backward()
    return _grads_of(pt, scene)


def pose6(pose34, dpose34):
    """6-DoF gradient (rho, omega) of the right perturbation G exp(xi^)."""
    G = frames.as_h(pose34)
    D = np.zeros_like(G)
    D[..., :3, :] = dpose34
    M = np.einsum("...ji,...jk->...ik", G, D)
    out = np.zeros(np.shape(pose34)[:-2] + (6,))
    out[..., 0:3] = M[..., 0:3, 3]
    out[..., 3] = M[..., 2, 1] - M[..., 1, 2]
    out[..., 4] = M[..., 0, 2] - M[..., 2, 0]
    out[..., 5] = M[..., 1, 0] - M[..., 0, 1]
    return out
