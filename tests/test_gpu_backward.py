"""GPU gradients vs the oracle's FP64 autograd (1e-3 per tensor normwise and
element by element relative to the entry plus the tensor's rms), and the
temporal-visibility update vs the oracle (exact)."""

import numpy as np
import pytest

import scenes
from oracle import grad as ograd
from oracle import render, visibility

from gpu_util import banner, compare_grads, gpu_region_grads, make_renderer, mask_bits, needs_gpu, \
    oracle_region_grads, poison_grads

pytestmark = [pytest.mark.gpu, needs_gpu]

torch = pytest.importorskip("torch")


def flat_targets(tg):
    return torch.as_tensor(np.concatenate([t.ravel() for t in tg])).cuda().contiguous()


def gpu_grads(r, tg_list):
    r.forward()
    r.l1_loss(flat_targets(tg_list))
    poison_grads(r)
    r.raster_bwd()
    torch.cuda.synchronize()
    g = dict(mean=r.g_mean, scale=r.g_scale, quat=r.g_quat, opacity=r.g_opacity, sh=r.g_sh,
             pose=r.g_pose.view(r.T, r.S, 3, 4), pose6=r.g_pose6)
    return float(r.loss_v[:r.V].sum()), {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}


def compare(g, ref, keys, rel=1e-3, tag=""):
    compare_grads(g, ref, keys, rel=rel, tag=tag)


def oracle_grads(scene, views, params, tg, plain=False):
    orders = {}
    for v in range(views.n_views):
        o = render.render_view(scene, views, v, params, plain=plain, with_image=False)
        from oracle import order
        orders[v] = order.global_order(o["ids"], o["dec"]["depth_bits"])
    return ograd.loss_and_grads(scene, views, list(range(views.n_views)), orders, params, tg,
                                route="conventional" if plain else "instance")


KEYS = ("mean", "scale", "quat", "opacity", "sh", "pose", "pose6")


@pytest.mark.parametrize("plain", [False, True])
def test_grads_config1(plain):
    c = scenes.make_config(1)
    tg = scenes.targets(1, c.views)
    banner(f"grads config1 plain={plain}")
    r = make_renderer(c.scene, c.views, c.params, plain=plain)
    loss, g = gpu_grads(r, tg)
    lref, _, ref = oracle_grads(c.scene, c.views, c.params, tg, plain=plain)
    assert abs(loss - lref) <= 1e-4 * abs(lref)
    compare(g, ref, KEYS)


@pytest.mark.parametrize("seed", range(4))
def test_grads_micro(seed):
    scene, views = scenes.micro_scene(seed, n=60, width=40, height=30, n_inst=2,
                                      sh_degree=seed % 4)
    p = scenes.default_params(tile=16)
    rng = np.random.default_rng(seed)
    tg = [rng.uniform(0, 1, (3, 30, 40)).astype(np.float32) for _ in range(views.n_views)]
    banner(f"grads micro seed={seed}")
    r = make_renderer(scene, views, p)
    loss, g = gpu_grads(r, tg)
    lref, _, ref = oracle_grads(scene, views, p, tg)
    assert abs(loss - lref) <= 1e-4 * abs(lref)
    compare(g, ref, KEYS)


def test_visibility_update_fold_reset():
    c = scenes.make_config(2, scale_n=0.05)
    p = dict(c.params, temporal=True)
    views = c.views.subset([3, 19, 33, 47])
    banner("visibility lifecycle")
    r = make_renderer(c.scene, views, p)
    r.forward()
    masks = mask_bits(r)
    from paper_2503_08217_amd import S3R_VIS_FOLD, S3R_VIS_RESET, S3R_VIS_UPDATE
    r.update_visibility(S3R_VIS_UPDATE)
    t = r.t_norm.cpu().numpy()
    ls, le = visibility.update(c.scene.life_s, c.scene.life_e, masks, t)
    np.testing.assert_array_equal(r.life_s.cpu().numpy(), ls)
    np.testing.assert_array_equal(r.life_e.cpu().numpy(), le)
    r.update_visibility(S3R_VIS_UPDATE)      # idempotent
    np.testing.assert_array_equal(r.life_s.cpu().numpy(), ls)
    r.update_visibility(S3R_VIS_FOLD)
    vs, ve = visibility.fold(ls, le)
    np.testing.assert_array_equal(r.vis_s.cpu().numpy(), vs)
    np.testing.assert_array_equal(r.vis_e.cpu().numpy(), ve)
    # after the fold every Gaussian in M at time t passes the temporal test at t
    r.forward()
    m2 = mask_bits(r)
    np.testing.assert_array_equal(m2, masks)
    r.update_visibility(S3R_VIS_RESET)
    np.testing.assert_array_equal(r.vis_s.cpu().numpy(), -1.0)
    np.testing.assert_array_equal(r.life_e.cpu().numpy(), -1.0)


def test_grads_single_view_config2_subset():
    """One view per batch takes the exclusive (non-atomic) accumulation path."""
    c = scenes.make_config(2, scale_n=0.02)
    views = c.views.subset([12])
    tg = scenes.targets(2, views)
    banner("grads single view")
    r = make_renderer(c.scene, views, c.params)
    loss, g = gpu_grads(r, tg)
    lref, _, ref = oracle_grads(c.scene, views, c.params, tg)
    assert abs(loss - lref) <= 1e-4 * abs(lref)
    compare(g, ref, KEYS)


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_grads_long_lists_all_tiles(tile):
    """Thousands of faint Gaussians: pixels keep accumulating for hundreds to
    thousands of list entries, so the backward replays several LDS windows
    per tile (windows of 128 / 512 / 2048 entries for tiles 8 / 16 / 32) and
    every window flush, wave count and tile shape is checked against the
    oracle's gradients, over a batch of two views."""
    scene, views = scenes.micro_scene(5, n=4000, width=64, height=48, n_inst=2, sh_degree=1,
                                      spread=0.35)
    rng = np.random.default_rng(17)
    scene.opacity[:] = rng.uniform(0.005, 0.02, scene.opacity.shape).astype(np.float32)
    p = scenes.default_params(tile=tile)
    tg = [rng.uniform(0, 1, (3, 48, 64)).astype(np.float32) for _ in range(views.n_views)]
    banner(f"grads long lists tile={tile}")
    r = make_renderer(scene, views, p)
    loss, g = gpu_grads(r, tg)
    last = r.last[: r.total_px].cpu().numpy()
    assert last.max() > {8: 128, 16: 512, 32: 2048}[tile], last.max()
    lref, _, ref = oracle_grads(scene, views, p, tg)
    assert abs(loss - lref) <= 1e-4 * abs(lref)
    compare(g, ref, KEYS)


def test_sparse_gradient_mode_matches_dense():
    """S3R_GRAD_SPARSE clears only the rows the previous call wrote: over a
    sequence of batches (two views each, so Gaussians repeat in the row list)
    every call's gradients equal those of the dense mode: the same rows are
    exactly zero (no stale row survives) and the values agree to float
    rounding (the raster backward's float atomics complete in varying order)."""
    c = scenes.make_config(2, scale_n=0.02)
    batches = [[5, 20], [35, 12], [44, 2], [5, 20]]
    first = c.views.subset(batches[0])
    banner("sparse gradient mode")
    rs = make_renderer(c.scene, first, dict(c.params, grad_sparse=True))
    rd = make_renderer(c.scene, first, c.params)
    rs.zero_grads()
    hs = rs.prepare_views([c.views.subset(b) for b in batches])
    hd = rd.prepare_views([c.views.subset(b) for b in batches])
    for b, h1, h2 in zip(batches, hs, hd):
        tg = flat_targets(scenes.targets(2, c.views.subset(b)))
        for r, h in ((rs, h1), (rd, h2)):
            r.use_views(h)
            r.forward()
            r.l1_loss(tg)
            r.raster_bwd()
        torch.cuda.synchronize()
        for k in ("g_mean", "g_scale", "g_quat", "g_opacity", "g_sh"):
            gs = getattr(rs, k).cpu().numpy().reshape(rs.n, -1)
            gd = getattr(rd, k).cpu().numpy().reshape(rd.n, -1)
            np.testing.assert_array_equal(np.any(gs != 0, 1), np.any(gd != 0, 1),
                                          err_msg=f"{k} rows batch {b}")
            np.testing.assert_allclose(gs, gd, rtol=1e-4, atol=1e-6 * np.abs(gd).max(),
                                       err_msg=f"{k} batch {b}")
        np.testing.assert_allclose(rs.g_pose.cpu().numpy(), rd.g_pose.cpu().numpy(), rtol=1e-5,
                                   atol=1e-7)


def test_grads_records_spanning_reduce_workgroups():
    """Six Gaussians cover more than 4096 tiles each (960x540 view, 8 px
    tiles, 8160 tiles), so each record's per-pair gradient slots contain at
    least one whole workgroup of the per-record slot sum (2048 slots per
    workgroup) and are combined across workgroups; dL/dC is non-zero on 80
    scattered 8x8 tiles of both views, so slots all along those records
    carry gradient.  Checked element by element against the oracle."""
    scene, views = scenes.micro_scene(21, n=200, width=960, height=540, n_inst=1, sh_degree=1)
    scene.scale[:6] = 1.2
    p = scenes.default_params(tile=8)
    banner("grads of records spanning reduce workgroups")
    r = make_renderer(scene, views, p)
    rect = r.rec_rect[: r.read_counters()["n_surv"]].cpu().numpy()
    area = (rect[:, 2] - rect[:, 0]) * (rect[:, 3] - rect[:, 1])
    assert (area > 2 * 2048).sum() >= 2, area.max()
    rng = np.random.default_rng(8)
    parts = []
    for v in range(views.n_views):
        for _ in range(40):
            tx, ty = int(rng.integers(0, 120)), int(rng.integers(0, 67))
            reg = (8 * tx, 8 * ty, 8 * tx + 8, 8 * ty + 8)
            parts.append((v, reg, rng.uniform(-1.0, 1.0, (3, 8, 8)) / 64.0))
    g = gpu_region_grads(r, parts)
    ref = oracle_region_grads(scene, views, p, parts)
    compare(g, ref, KEYS, tag="spanning records")


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_deterministic_gradients_bitwise(tile):
    """S3R_DETERMINISTIC_GRADS: repeated backward calls (and a repeated
    forward + backward) give bitwise equal gradients of every tensor, which
    also match the oracle -- on a scene whose large Gaussians cover thousands
    of tiles, so per-record sums cross runs and workgroups of the slot sum,
    and a tile's waves all add into the same window entries."""
    scene, views = scenes.micro_scene(21, n=200, width=960, height=540, n_inst=1, sh_degree=1)
    scene.scale[:6] = 1.2
    p = dict(scenes.default_params(tile=tile), deterministic=True)
    banner(f"deterministic gradients tile={tile}")
    r = make_renderer(scene, views, p)
    rng = np.random.default_rng(9)
    parts = []
    for v in range(views.n_views):
        for _ in range(24):
            tx, ty = int(rng.integers(0, 960 // 8)), int(rng.integers(0, 540 // 8))
            reg = (8 * tx, 8 * ty, 8 * tx + 8, 8 * ty + 8)
            parts.append((v, reg, rng.uniform(-1.0, 1.0, (3, 8, 8)) / 64.0))
    runs = [gpu_region_grads(r, parts) for _ in range(2)]
    r.forward()
    runs.append(gpu_region_grads(r, parts))
    for k in KEYS:
        for o in runs[1:]:
            np.testing.assert_array_equal(o[k], runs[0][k], err_msg=f"{k} not reproducible")
    ref = oracle_region_grads(scene, views, p, parts)
    compare(runs[0], ref, KEYS, tag=f"deterministic tile {tile}")
