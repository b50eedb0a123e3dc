"""s3r_project_cull_noalloc (the fixed-scratch variant for callers that cannot
allocate) against s3r_project_cull with a caller workspace, through the C ABI:
two calls in a row on one device, the second on a smaller input (fewer
Gaussians and views), every output bit-identical."""

import numpy as np
import pytest

import scenes

from gpu_util import banner, make_renderer, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]

torch = pytest.importorskip("torch")

from paper_2503_08217_amd import _abi as A  # noqa: E402


def poison(r):
    """Outputs of project_cull start from garbage so that an entry the call
    does not write shows up."""
    for t in (r.cam, r.cen, r.t_norm, r.rec_geo, r.rec_conic, r.rec_rgb):
        t.fill_(float("nan"))
    for t in (r.mask, r.surv, r.rec_gid, r.rec_view, r.rec_rect, r.rec_npairs, r.rec_pair,
              r.counters, r.stats, r.bstat):
        t.fill_(-7)


def outputs(r):
    torch.cuda.synchronize()
    n = int(r.counters[0].item())
    nblk = (r.n + 255) // 256
    o = {k: getattr(r, k).cpu().numpy().copy() for k in ("cam", "cen", "t_norm", "mask", "surv",
                                                         "stats")}
    o["counters"] = r.counters[:4].cpu().numpy().copy()
    o["bstat"] = r.bstat[: nblk * r.V * A.BSTAT].cpu().numpy().copy()
    for k in ("rec_gid", "rec_view", "rec_geo", "rec_conic", "rec_rgb", "rec_rect", "rec_npairs",
              "rec_pair"):
        o[k] = getattr(r, k)[:n].cpu().numpy().copy()
    return o


def assert_same(a, b, what):
    assert a.keys() == b.keys()
    for k in a:
        x, y = a[k], b[k]
        assert x.shape == y.shape, (what, k)
        np.testing.assert_array_equal(x.view(np.uint8), y.view(np.uint8), err_msg=f"{what}: {k}")


def folded(r):
    """A folded temporal state from an UPDATE over the renderer's views."""
    from paper_2503_08217_amd import S3R_VIS_FOLD, S3R_VIS_UPDATE
    r.set_flags(temporal=False)
    r.project_cull()
    r.update_visibility(S3R_VIS_UPDATE)
    r.update_visibility(S3R_VIS_FOLD)
    r.set_flags(temporal=True)


def test_noalloc_matches_workspace_entry_point():
    big_cfg = scenes.make_config(2)
    big_views = big_cfg.views.subset([3, 17, 30, 44])
    small_scene, small_views = scenes.micro_scene(3, n=700, width=70, height=50, n_inst=2,
                                                  sh_degree=2)
    banner("no-alloc project_cull: 240k Gaussians x 4 views, then 700 x 2")
    rb = make_renderer(big_cfg.scene, big_views, big_cfg.params)
    folded(rb)
    rs = make_renderer(small_scene, small_views, scenes.default_params(tile=8, temporal=True,
                                                                       lod=True, lod_r=0.5))
    ref = {}
    for name, r in (("big", rb), ("small", rs)):
        poison(r)
        r.project_cull()
        ref[name] = outputs(r)
        assert ref[name]["counters"][0] > 0 and ref[name]["counters"][1] == 0
    # two calls in a row of the fixed-scratch entry point, the second smaller
    for name, r in (("big", rb), ("small", rs)):
        poison(r)
        r.project_cull_noalloc()
        assert_same(outputs(r), ref[name], name)
    # and once more on the big input after the small one
    poison(rb)
    rb.project_cull_noalloc()
    assert_same(outputs(rb), ref["big"], "big again")
    # a whole forward from the fixed-scratch projection renders the same image
    rb.sort()
    rb.raster_fwd()
    img_noalloc = rb.color.cpu().numpy().copy()
    rb.forward()
    np.testing.assert_array_equal(rb.color.cpu().numpy(), img_noalloc)

