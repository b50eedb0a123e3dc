"""A whole batched training step captured in a HIP graph replays exactly like
the eager step (several replays, eager work and synchronisation in between)."""

import numpy as np
import pytest

import scenes

from gpu_util import banner, make_renderer, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]

torch = pytest.importorskip("torch")


def snapshot(r):
    torch.cuda.synchronize()
    return dict(color=r.color.cpu().numpy(), T=r.T_final.cpu().numpy(),
                loss=r.loss_v.cpu().numpy(), g_mean=r.g_mean.cpu().numpy(),
                g_sh=r.g_sh.cpu().numpy(), g_pose=r.g_pose.cpu().numpy(),
                life_s=r.life_s.cpu().numpy(), life_e=r.life_e.cpu().numpy())


def test_graph_replay_matches_eager():
    c = scenes.make_config(4, scale_n=0.01)
    idx = [i for i in range(c.views.n_views) if 20 <= c.views.tstep[i] <= 21]
    views = c.views.subset(idx)
    tg = scenes.targets(4, views)
    target = torch.as_tensor(np.concatenate([t.ravel() for t in tg])).cuda()
    banner(f"graph capture of a {len(idx)}-view step")
    r = make_renderer(c.scene, views, c.params)
    r.step(target)
    ref = snapshot(r)
    g = r.capture_step(target)
    for rep in range(3):
        # eager work in between: a forward of the same batch, then a sync
        r.forward()
        torch.cuda.synchronize()
        g.replay()
        out = snapshot(r)
        np.testing.assert_array_equal(out["color"], ref["color"], err_msg=f"replay {rep}")
        np.testing.assert_array_equal(out["T"], ref["T"])
        np.testing.assert_allclose(out["loss"], ref["loss"], rtol=1e-6)
        for k in ("g_mean", "g_sh", "g_pose"):
            scale = np.abs(ref[k]).max() + 1e-30
            np.testing.assert_allclose(out[k] / scale, ref[k] / scale, atol=1e-5, err_msg=k)
        np.testing.assert_array_equal(out["life_s"], ref["life_s"])
        np.testing.assert_array_equal(out["life_e"], ref["life_e"])


def test_autotuner_picks_a_shape_that_renders_the_same_image():
    """The library-side autotuner times every (tile, sort, forward waves per
    workgroup, binning) candidate on a step of an uneven batch, then the
    fine-tile counts at the fastest, requires each to render the same image
    bit for bit, and leaves the knobs at the fastest; the renderer it
    returns renders that image too."""
    from paper_2503_08217_amd import _abi as A
    from paper_2503_08217_amd.renderer import Renderer
    c = scenes.make_config(4, scale_n=0.01)
    idx = [i for i in range(c.views.n_views) if c.views.tstep[i] == 21]
    views = c.views.subset(idx)
    tg = scenes.targets(4, views)
    target = torch.as_tensor(np.concatenate([t.ravel() for t in tg])).cuda()
    banner("autotune")
    try:
        r, res = Renderer.autotuned(c.scene, views, c.params, target, tiles=(8, 16, 32),
                                    raster_waves=(1, 16), fine_tiles=(0, 160, 4096), reps=2)
        table, best = res["table"], res["best"]
        assert len(table) == 3 * (2 * 2 + 2) + 2
        assert best["ms"] == min(row["ms"] for row in table)
        knobs = A.get_tuning()
        assert knobs["raster_waves"] == best["raster_waves"]
        assert knobs["bin_max_tiles"] == (12288 if best["binning"] else 0)
        assert knobs["fine_tiles"] == best["fine_tiles"]
        r.forward()
        ref = make_renderer(c.scene, views, c.params)
        ref.forward()
        np.testing.assert_array_equal(r.color.cpu().numpy(), ref.color.cpu().numpy())
    finally:
        A.set_tuning(**{k: -1 for k in A.TUNE_KNOBS})
