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


def test_lifecycle_matches_oracle():
    """Four epochs of training (Adam moves the Gaussians between steps) with
    a fold after epochs 0, 1, 3 and a reset after epoch 2: at every step the
    oracle takes the visibility decisions from the parameters the GPU
    rendered with and its own temporal state, and M_t must match bit for
    bit; its UPDATE (Eq. 5) per step and FOLD (Eq. 6) or RESET per epoch must
    give the GPU's point life and visibility intervals bit for bit after
    every epoch."""
    from oracle import decide32, visibility
    from paper_2503_08217_amd.train import Trainer
    c = scenes.make_config(2, scale_n=0.02)
    p = dict(c.params, temporal=True, lod=True, lod_r=1.0)
    taus = [2, 9, 17, 25, 33, 41, 49]
    batches = [c.views.subset([t]) for t in taus]
    tg = scenes.targets(2, c.views, taus)
    targets = [torch.as_tensor(t.ravel()).cuda() for t in tg]
    banner("training lifecycle against the oracle")
    r = make_renderer(c.scene, batches[0], p)
    tr = Trainer(r, batches, targets, reset_every=3)
    st = dict(life_s=c.scene.life_s.copy(), life_e=c.scene.life_e.copy(),
              vis_s=c.scene.vis_s.copy(), vis_e=c.scene.vis_e.copy())
    sc = c.scene.copy()
    trajectory = []

    def on_step(rr):
        for k in ("mean", "scale", "quat", "opacity"):
            setattr(sc, k, getattr(rr, k).cpu().numpy().reshape(getattr(sc, k).shape).copy())
        sc.vis_s, sc.vis_e = st["vis_s"], st["vis_e"]
        tau = int(rr.tstep_np[0])
        d = decide32.project_cull32(sc, rr._vs["W"].cpu().numpy().reshape(3, 4),
                                    rr._vs["K"].cpu().numpy()[0], rr.wh_np[0], tau, p)
        np.testing.assert_array_equal(mask_bits(rr)[0], d["visible"], err_msg=f"M_t tau {tau}")
        assert int(rr.stats[0, 0]) == int(d["pass_t"].sum())
        st["life_s"], st["life_e"] = visibility.update(st["life_s"], st["life_e"],
                                                       d["visible"][None], [d["t"]])

    for e in range(4):
        rec = tr.epoch(e, on_step=on_step)
        if rec["action"] == "fold":
            st["vis_s"], st["vis_e"] = visibility.fold(st["life_s"], st["life_e"])
        else:
            st["vis_s"], st["vis_e"], st["life_s"], st["life_e"] = visibility.reset(sc.n)
        for k in ("life_s", "life_e", "vis_s", "vis_e"):
            np.testing.assert_array_equal(getattr(tr.r, k).cpu().numpy(), st[k],
                                          err_msg=f"{k} after epoch {e}")
        trajectory.append((rec["action"], rec["temporal_pass"]))
    banner(f"temporal-pass fraction per epoch: {trajectory}")
    assert trajectory[0][1] == 1.0 and trajectory[1][1] < 1.0 and trajectory[3][1] == 1.0
