"""Pin of the reference gradient: FP64 autograd == FP64 central differences."""

import numpy as np
import pytest
import scipy.linalg
import torch

import scenes
from oracle import frames, grad, render


def _setup(seed, n=12, sh_degree=2):
    scene, views = scenes.micro_scene(seed, n=n, width=20, height=16, n_inst=2, sh_degree=sh_degree)
    p = scenes.default_params(tile=8)
    orders = {v: render.render_view(scene, views, v, p, with_image=False) for v in range(views.n_views)}
    orders = {v: __import__("oracle.order", fromlist=["x"]).global_order(o["ids"], o["dec"]["depth_bits"])
              for v, o in orders.items()}
    rng = np.random.default_rng(seed)
    tg = {v: rng.uniform(0, 1, (3, 16, 20)) for v in range(views.n_views)}
    return scene, views, p, orders, tg


def _loss(scene, views, p, orders, tg, over=None):
    pt = grad.to_torch_params(scene, requires_grad=False)
    if over is not None:
        over(pt)
    dec = []
    with torch.no_grad():
        L = 0.0
        for v in orders:
            img, _ = grad.render_t(pt, scene, views, v, orders[v], p, decisions=dec)
            L += float(grad.l1_loss_t(img, tg[v]))
            # also freeze the sign of every residual (|.| is not smooth at 0)
            dec.append((img - torch.as_tensor(tg[v])).sign())
    return L, dec


def _same(d1, d2):
    for a, b in zip(d1, d2):
        a = a if isinstance(a, tuple) else (a,)
        b = b if isinstance(b, tuple) else (b,)
        for x, y in zip(a, b):
            if not torch.equal(x, y):
                return False
    return True


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_autograd_matches_central_differences(seed):
    scene, views, p, orders, tg = _setup(seed)
    loss, _, g = grad.loss_and_grads(scene, views, list(orders), orders, p, tg)
    L0, d0 = _loss(scene, views, p, orders, tg)
    assert abs(L0 - loss) < 1e-12
    rng = np.random.default_rng(100 + seed)
    checked = 0
    for key, shape in (("mean", scene.mean.shape), ("scale", scene.scale.shape),
                       ("quat", scene.quat.shape), ("opacity", scene.opacity.shape),
                       ("sh", scene.sh.shape), ("pose", scene.pose.shape)):
        for _ in range(8):
            idx = tuple(int(rng.integers(s)) for s in shape)
            if key == "pose" and idx[1] == 0:
                continue
            base = float(np.asarray(getattr(scene, key), np.float64)[idx])
            h = 1e-6 * max(1.0, abs(base))

            def setter(delta):
                def f(pt):
                    pt[key][idx] = pt[key][idx] + delta
                return f

            Lp, dp = _loss(scene, views, p, orders, tg, setter(h))
            Lm, dm = _loss(scene, views, p, orders, tg, setter(-h))
            if not (_same(d0, dp) and _same(d0, dm)):
                continue
            fd = (Lp - Lm) / (2 * h)
            an = g[key][idx]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(an)) + 1e-9, (key, idx, fd, an)
            checked += 1
    assert checked >= 25


def test_pose6_matches_exponential_map_differences():
    seed = 4
    scene, views, p, orders, tg = _setup(seed, n=15)
    _, _, g = grad.loss_and_grads(scene, views, list(orders), orders, p, tg)
    G = frames.as_h(scene.pose)
    for tau, k in ((0, 1), (1, 2), (1, 1)):
        for j in range(6):
            h = 1e-6
            vals = []
            for sgn in (1, -1):
                xi = np.zeros(6)
                xi[j] = sgn * h
                hat = np.zeros((4, 4))
                rho, om = xi[:3], xi[3:]
                hat[:3, :3] = [[0, -om[2], om[1]], [om[2], 0, -om[0]], [-om[1], om[0], 0]]
                hat[:3, 3] = rho
                Gn = G[tau, k] @ scipy.linalg.expm(hat)

                def f(pt, Gn=Gn):
                    pt["pose"][tau, k] = torch.as_tensor(Gn[:3, :])
                vals.append(_loss(scene, views, p, orders, tg, f)[0])
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - g["pose6"][tau, k, j]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9


def test_routes_agree_on_6dof_pose_gradient():
    """Instance-frame direction through P = W G vs R_G^T (mu_g - c_W): the same
    function on rigid poses, so every gradient but the raw pose one agrees,
    and the 6-DoF pose gradients agree."""
    scene, views, p, orders, tg = _setup(5, n=15, sh_degree=3)
    _, _, a = grad.loss_and_grads(scene, views, list(orders), orders, p, tg, route="instance")
    _, _, b = grad.loss_and_grads(scene, views, list(orders), orders, p, tg, route="conventional")
    for k in ("mean", "scale", "quat", "opacity", "sh", "pose6"):
        np.testing.assert_allclose(a[k], b[k], rtol=1e-5, atol=1e-7 * np.abs(b[k]).max())
    assert np.abs(a["pose"] - b["pose"]).max() > 1e-9     # raw pose gradients differ


@pytest.mark.parametrize("seed", [0, 1])
def test_image_vjp_is_the_region_backward(seed):
    """image_vjp over regions that tile the view, with dC = dL/dC of the
    mean-L1 loss (sign(C - target) / (3 w h)), gives the L1 loss gradients;
    splitting the view into regions with each region's Mahalanobis-cut
    candidates changes nothing (the pre-filter drops only Gaussians that are
    skipped at every pixel of the region)."""
    from oracle import order
    scene, views, p, orders, tg = _setup(seed)
    _, imgs, g = grad.loss_and_grads(scene, views, list(orders), orders, p, tg)
    parts = []
    for v in orders:
        img = imgs[v][0]
        dC = np.sign(img - tg[v]) / img.size
        o = render.render_view(scene, views, v, p, with_image=False)
        for reg in ((0, 0, 11, 16), (11, 0, 20, 9), (11, 9, 20, 16)):
            cand = render.region_candidates(o["dec"], o["ids"], reg, p)
            parts.append((v, reg, order.global_order(cand, o["dec"]["depth_bits"]),
                          dC[:, reg[1]:reg[3], reg[0]:reg[2]]))
    g2 = grad.image_vjp(scene, views, p, parts)
    for k in ("mean", "scale", "quat", "opacity", "sh", "pose", "pose6"):
        np.testing.assert_allclose(g2[k], g[k], rtol=1e-10, atol=1e-14, err_msg=k)
