"""GPU parity at the states and shapes the benchmark times, against the oracle.

* the 2M-Gaussian 1080p corridor at full size, in the folded temporal state
  of Sec. 3.3 / Eqs. (5)-(6) (UPDATE over all 50 timesteps, then FOLD, which
  rejects whole 256-Gaussian blocks), rendered one view per call exactly as
  the benchmark does: the folded state itself, N_t, M_t, survivor sets,
  records and every tile list bit for bit; pixels on sampled regions; the
  backward of one region (dL/dC zero elsewhere) against the oracle's FP64
  vector-Jacobian product, element by element;
* one timestep of the six-camera rig (uneven 1920x1080 / 1550x2048 /
  2048x1550 views in one batch, more than 65535 tiles at 16 px, so the tile
  partition takes three radix passes) against the oracle view by view;
* the torch.autograd.Function wrapper against the direct backward and the
  oracle.
"""

import numpy as np
import pytest

import scenes
from oracle import decide32, order, render, visibility
from oracle import grad as ograd

from gpu_util import banner, check_pixels, check_view, compare_grads, gpu_region_grads, image_np, \
    make_renderer, mask_bits, needs_gpu, oracle_region_grads, records, T_np

pytestmark = [pytest.mark.gpu, needs_gpu]

torch = pytest.importorskip("torch")

KEYS = ("mean", "scale", "quat", "opacity", "sh", "pose", "pose6")


def oracle_fold(scene, views, params, view_ids):
    """Point life after UPDATE over `view_ids` with the temporal filter off
    (Eq. 5), and the visibility intervals after FOLD (Eq. 6), in the oracle."""
    p = dict(params, temporal=False)
    ls, le = scene.life_s.copy(), scene.life_e.copy()
    for v in view_ids:
        d = decide32.project_cull32(scene, views.W[v], views.K[v], views.wh[v],
                                    int(views.tstep[v]), p, view_index=v)
        ls, le = visibility.update(ls, le, d["visible"][None], np.float32([d["t"]]))
    vs, ve = visibility.fold(ls, le)
    return ls, le, vs, ve


def with_state(scene, vs, ve):
    sc = scene.copy()
    sc.vis_s = np.asarray(vs, np.float32).copy()
    sc.vis_e = np.asarray(ve, np.float32).copy()
    return sc


def instance_region(d, wh, size=32):
    """A size x size region around the projection of the survivor of an
    instance (slot >= 1) nearest the image centre (the centre if none)."""
    w, h = int(wh[0]), int(wh[1])
    cx, cy = w / 2, h / 2
    ids = np.nonzero(d["surv"] & (d["inst"] > 0))[0] if "inst" in d else np.zeros(0, int)
    if ids.size:
        k = ids[np.argmin((d["u"][ids] - cx) ** 2 + (d["v"][ids] - cy) ** 2)]
        cx, cy = float(d["u"][k]), float(d["v"][k])
    x0 = int(np.clip(round(cx) - size // 2, 0, w - size))
    y0 = int(np.clip(round(cy) - size // 2, 0, h - size))
    return (x0, y0, x0 + size, y0 + size)


def test_corridor_2m_folded_state():
    from paper_2503_08217_amd import S3R_VIS_FOLD, S3R_VIS_UPDATE
    from paper_2503_08217_amd.renderer import Renderer
    c = scenes.make_config(3)
    n = c.scene.n
    banner(f"corridor-2M: oracle warm-up over {c.views.n_views} views")
    ls, le, vs, ve = oracle_fold(c.scene, c.views, c.params, range(c.views.n_views))

    banner("corridor-2M: GPU warm-up (UPDATE per view, then FOLD)")
    r = Renderer(c.scene, c.views.subset([c.timed_views[0]]), c.params, cap_surv=n // 2,
                 cap_dup=2 * n)
    hs = r.prepare_views([c.views.subset([v]) for v in range(c.views.n_views)])
    r.set_flags(temporal=False)
    for h in hs:
        r.use_views(h)
        r.project_cull()
        r.update_visibility(S3R_VIS_UPDATE)
    r.update_visibility(S3R_VIS_FOLD)
    torch.cuda.synchronize()
    for name, ref in (("life_s", ls), ("life_e", le), ("vis_s", vs), ("vis_e", ve)):
        np.testing.assert_array_equal(getattr(r, name).cpu().numpy(), ref, err_msg=name)
    del hs
    r.set_flags(temporal=True)
    sc = with_state(c.scene, vs, ve)

    rng = np.random.default_rng(3)
    for vi in (c.timed_views[2], c.timed_views[5]):
        views1 = c.views.subset([vi])
        r.use_views(r.prepare_views([views1])[0])
        fit = r.fit_capacity()
        assert fit["ovf_surv"] == 0 and fit["ovf_dup"] == 0 and fit["spin"] == 0, fit
        r.forward()
        rec = records(r)
        banner(f"corridor-2M view {vi}: {rec['n']} records, {fit['n_dup']} pairs, "
               f"N_t {int(rec['stats'][0][0])}")
        centre = (944, 524, 976, 556)          # the vanishing point: the longest lists
        o = check_view(sc, views1, c.params, r, rec, 0, region=centre, full_lists=True)
        d = o["dec"]
        # the folded state rejects whole blocks, whose geometry k_cull never
        # reads, and splits others
        pt = d["pass_t"]
        blocks = np.pad(pt, (0, (-n) % 256)).reshape(-1, 256)
        assert (~blocks.any(1)).sum() > 100 and (blocks.any(1) & ~blocks.all(1)).sum() > 10
        assert 0.2 * n < pt.sum() < 0.98 * n
        corner = (1888, 1048, 1920, 1080)     # the ragged last tile row
        x0 = int(rng.integers(0, 1920 - 32))
        y0 = int(rng.integers(0, 1080 - 32))
        for reg in (corner, (x0, y0, x0 + 32, y0 + 32)):
            oo = render.render_view(sc, views1, 0, c.params, region=reg)
            img = image_np(r, 0)[:, reg[1]:reg[3], reg[0]:reg[2]]
            T = T_np(r, 0)[reg[1]:reg[3], reg[0]:reg[2]]
            check_pixels(oo, img, T, c.params, float(sc.opacity.max()), tag=f"view {vi} {reg}")
        # backward of one region around an instance
        d = dict(d, inst=sc.inst)
        reg = instance_region(d, views1.wh[0])
        dC = rng.uniform(-1.0, 1.0, (3, reg[3] - reg[1], reg[2] - reg[0])) / 1024.0
        g = gpu_region_grads(r, [(0, reg, dC)])
        ref = oracle_region_grads(sc, views1, c.params, [(0, reg, dC)])
        assert np.abs(ref["mean"]).max() > 0
        compare_grads(g, ref, KEYS, tag=f"corridor-2M view {vi} region {reg}")


def test_rig_timestep_uneven_views():
    """Six cameras of one timestep in one batch (z_far 120 m, so the folded
    state of a surround rig rejects Gaussians; with z_far = inf every
    Gaussian lies in some camera's frustum at every time)."""
    c = scenes.make_config(4, scale_n=0.02)
    p = dict(c.params, z_far=120.0)
    banner(f"rig: oracle warm-up over {c.views.n_views} views, N={c.scene.n}")
    _, _, vs, ve = oracle_fold(c.scene, c.views, p, range(c.views.n_views))
    sc = with_state(c.scene, vs, ve)
    idx = [i for i in range(c.views.n_views) if c.views.tstep[i] == 21]
    views = c.views.subset(idx)
    assert len(idx) == 6 and len({tuple(x) for x in views.wh.tolist()}) == 3
    r = make_renderer(sc, views, p)
    assert r.total_tiles > 65535
    rec = records(r)
    st = rec["stats"]
    banner(f"rig: {r.total_tiles} tiles, {rec['n']} records, N_t/N {st[:, 0].mean() / sc.n:.3f}")
    assert 0 < st[:, 0].max() < sc.n
    outs = []
    for v in range(6):
        w, h = int(views.wh[v, 0]), int(views.wh[v, 1])
        corner = (w - 40, h - 40, w, h)      # ragged tiles at 1080 and 1550
        o = check_view(sc, views, p, r, rec, v, region=corner, full_lists=True)
        outs.append(o)
        reg = (w // 2 - 16, h // 2 - 16, w // 2 + 16, h // 2 + 16)
        oo = render.render_view(sc, views, v, p, region=reg)
        check_pixels(oo, image_np(r, v)[:, reg[1]:reg[3], reg[0]:reg[2]],
                     T_np(r, v)[reg[1]:reg[3], reg[0]:reg[2]], p, float(sc.opacity.max()),
                     tag=f"rig view {v} centre")
    rng = np.random.default_rng(4)
    parts = []
    for v in (0, 1, 3):
        d = dict(outs[v]["dec"], inst=sc.inst)
        reg = instance_region(d, views.wh[v])
        parts.append((v, reg, rng.uniform(-1.0, 1.0, (3, 32, 32)) / 1024.0))
    g = gpu_region_grads(r, parts)
    ref = oracle_region_grads(sc, views, p, parts)
    compare_grads(g, ref, KEYS, tag="rig regions")


def test_render_fn_autograd():
    """torch.autograd through RenderFn gives the direct backward's gradients
    (the loss computed by torch on the returned image) and the oracle's; a
    backward after another forward of the same renderer raises."""
    from paper_2503_08217_amd.renderer import render as render_fn
    c = scenes.make_config(1)
    tg = scenes.targets(1, c.views)
    r = make_renderer(c.scene, c.views, c.params)
    target = torch.as_tensor(np.concatenate([t.ravel() for t in tg])).cuda()
    params = r.parameters()
    for t in params:
        t.requires_grad_(True)
        t.grad = None
    img = render_fn(r, *params)
    loss = torch.zeros((), device=img.device, dtype=torch.float32)
    for v in range(r.V):
        o, npx = int(r.poff_np[v]), int(r.wh_np[v, 0] * r.wh_np[v, 1])
        loss = loss + (img[3 * o: 3 * (o + npx)] - target[3 * o: 3 * (o + npx)]).abs().mean()
    loss.backward()
    auto = {k: t.grad.detach().cpu().numpy().astype(np.float64)
            for k, t in zip(("mean", "scale", "quat", "opacity", "sh", "pose"), params)}
    for t in params:
        t.requires_grad_(False)
    # the direct calls: forward, the library's L1 loss, backward
    r.forward()
    r.l1_loss(target)
    r.raster_bwd()
    torch.cuda.synchronize()
    direct = dict(mean=r.g_mean, scale=r.g_scale, quat=r.g_quat, opacity=r.g_opacity, sh=r.g_sh,
                  pose=r.g_pose)
    for k, t in direct.items():
        a, b = auto[k].ravel(), t.cpu().numpy().astype(np.float64).ravel()
        assert np.abs(a - b).max() <= 1e-5 * max(np.abs(b).max(), 1e-12), k
    orders = {}
    for v in range(3):
        o = render.render_view(c.scene, c.views, v, c.params, with_image=False)
        orders[v] = order.global_order(o["ids"], o["dec"]["depth_bits"])
    lref, _, ref = ograd.loss_and_grads(c.scene, c.views, [0, 1, 2], orders, c.params, tg)
    assert abs(float(loss) - lref) <= 1e-4 * abs(lref)
    auto["pose"] = auto["pose"].reshape(ref["pose"].shape)
    compare_grads(auto, ref, ("mean", "scale", "quat", "opacity", "sh", "pose"), tag="RenderFn")
    # a forward in between invalidates the stored transmittance
    for t in params:
        t.requires_grad_(True)
    img = render_fn(r, *params)
    r.forward()
    with pytest.raises(RuntimeError):
        img.sum().backward()
    for t in params:
        t.requires_grad_(False)
        t.grad = None
    with pytest.raises(ValueError):
        render_fn(r, r.mean.clone(), *params[1:])
    assert mask_bits(r).shape[0] == r.V
