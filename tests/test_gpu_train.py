"""The epoch lifecycle on the GPU: loss decreases, FOLD makes the temporal
filter sound for the rendered times, RESET restores all-visible, appended
Gaussians start visible."""

import numpy as np
import pytest

import scenes

from gpu_util import banner, make_renderer, mask_bits, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]

torch = pytest.importorskip("torch")


def test_epoch_lifecycle():
    from paper_2503_08217_amd.train import Trainer
    c = scenes.make_config(2, scale_n=0.02)
    p = dict(c.params, temporal=True, lod=True, lod_r=1.0)
    taus = [3, 12, 21, 30, 39, 48]
    batches = [c.views.subset([t]) for t in taus]
    tg = scenes.targets(2, c.views, taus)
    targets = [torch.as_tensor(t.ravel()).cuda() for t in tg]
    banner("training lifecycle")
    r = make_renderer(c.scene, batches[0], p)
    tr = Trainer(r, batches, targets, reset_every=3)
    recs = [tr.epoch(e) for e in range(3)]
    assert recs[0]["action"] == "fold" and recs[2]["action"] == "reset"
    assert recs[1]["loss"] < recs[0]["loss"]
    # after the first fold the filter passed fewer Gaussians than before it
    assert recs[1]["temporal_pass"] < recs[0]["temporal_pass"]
    # the last epoch reset: everything visible again
    np.testing.assert_array_equal(tr.r.vis_s.cpu().numpy(), -1.0)
    np.testing.assert_array_equal(tr.r.vis_e.cpu().numpy(), 1.0)
    # fold soundness: after an epoch and a fold, every Gaussian in M at a
    # rendered time passes the temporal test at that time
    rec = tr.epoch(3)
    assert rec["action"] == "fold"
    r = tr.r
    for h in tr.handles:
        r.use_views(h)
        r.set_flags(temporal=False)
        r.project_cull()
        m = mask_bits(r)[0]
        t = float(r.t_norm.cpu().numpy()[0])
        vs, ve = r.vis_s.cpu().numpy(), r.vis_e.cpu().numpy()
        assert np.all((vs[m] <= t) & (t <= ve[m]))
    r.set_flags(temporal=True)


def test_appended_gaussians_start_visible():
    from paper_2503_08217_amd.train import Trainer
    c = scenes.make_config(1)
    p = dict(c.params, temporal=True)
    batches = [c.views.subset([v]) for v in range(3)]
    tg = scenes.targets(1, c.views)
    targets = [torch.as_tensor(t.ravel()).cuda() for t in tg]
    banner("append")
    r = make_renderer(c.scene, batches[0], p)
    tr = Trainer(r, batches, targets, reset_every=0)
    tr.epoch(0)
    extra = scenes.make_config(1).scene
    n0 = tr.r.n
    tr.append_gaussians(extra)
    assert tr.r.n == n0 + extra.n
    vs = tr.r.vis_s.cpu().numpy()
    np.testing.assert_array_equal(vs[n0:], -1.0)
    np.testing.assert_array_equal(tr.r.vis_e.cpu().numpy()[n0:], 1.0)
    tr.r.fit_capacity()
    rec = tr.epoch(1)
    assert np.isfinite(rec["loss"])
