"""A minimal reconstruction loop around the per-view step, exercising the
temporal-visibility lifecycle of Sec. 3.3 over epochs.

Every training step renders a batch of views, backpropagates the L1 loss and
updates the point life l with the batch's visible masks (Eq. 5).  At the end
of an epoch, once every training time has been rendered, the visibility is
folded from the point life (Sec. 3.3, Eq. 6); every `reset_every` epochs it is instead
reset to visible at all times.  Gaussians appended during training start
visible at all times.  Parameters are updated with Adam on the activated
quantities (scale is kept positive, opacity inside (0, 1)); the optimiser is
not part of the rendering path and runs as plain tensor arithmetic.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import _abi as A


def epoch_action(epoch: int, reset_every: int) -> str:
    """What happens to the visibility state at the end of epoch `epoch`
    (0-based): "reset" every `reset_every` epochs, "fold" otherwise."""
    if reset_every > 0 and (epoch + 1) % reset_every == 0:
        return "reset"
    return "fold"


@dataclass
class Adam:
    lr: dict
    b1: float = 0.9
    b2: float = 0.999
    eps: float = 1e-15
    t: int = 0
    m: dict = field(default_factory=dict)
    v: dict = field(default_factory=dict)

    def step(self, params: dict, grads: dict):
        self.t += 1
        for k, p in params.items():
            g = grads[k]
            if k not in self.m:
                self.m[k] = torch.zeros_like(p)
                self.v[k] = torch.zeros_like(p)
            m, v = self.m[k], self.v[k]
            m.mul_(self.b1).add_(g, alpha=1 - self.b1)
            v.mul_(self.b2).addcmul_(g, g, value=1 - self.b2)
            mh = m / (1 - self.b1 ** self.t)
            vh = v / (1 - self.b2 ** self.t)
            p.sub_(self.lr[k] * mh / (vh.sqrt() + self.eps))


class Trainer:
    """Epochs over `batches` (a list of view batches of equal shape) with
    per-view targets; `renderer` is a Renderer built on the first batch."""

    def __init__(self, renderer, batches, targets, lr=None, reset_every=3):
        self.r = renderer
        self.handles = renderer.prepare_views(batches)
        self.targets = targets
        self.reset_every = reset_every
        lr = lr or dict(mean=1e-3, scale=5e-4, quat=1e-3, opacity=5e-3, sh=2.5e-3)
        self.opt = Adam(lr)
        self.history = []

    def params(self):
        r = self.r
        return dict(mean=r.mean, scale=r.scale, quat=r.quat, opacity=r.opacity, sh=r.sh)

    def grads(self):
        r = self.r
        return dict(mean=r.g_mean, scale=r.g_scale, quat=r.g_quat, opacity=r.g_opacity,
                    sh=r.g_sh)

    def epoch(self, e, on_step=None):
        """One pass over the batches, then FOLD or RESET.  `on_step(r)`, if
        given, runs after each batch's step (forward, backward, point-life
        update) and before the optimiser moves the parameters, so it sees the
        parameters and the visible mask that step used."""
        r = self.r
        losses, visible = [], []
        for h, tg in zip(self.handles, self.targets):
            r.use_views(h)
            r.step(tg)
            if on_step is not None:
                on_step(r)
            self.opt.step(self.params(), self.grads())
            with torch.no_grad():
                r.scale.clamp_(min=1e-4)
                r.opacity.clamp_(1e-3, 0.999)
            losses.append(float(r.loss_v[: r.V].sum()))
            visible.append(float(r.stats[:, 0].float().mean()) / max(1, r.n))
        action = epoch_action(e, self.reset_every)
        r.update_visibility(A.S3R_VIS_RESET if action == "reset" else A.S3R_VIS_FOLD)
        torch.cuda.synchronize()
        rec = dict(epoch=e, loss=float(np.mean(losses)), temporal_pass=float(np.mean(visible)),
                   action=action)
        self.history.append(rec)
        return rec

    def append_gaussians(self, scene_new):
        """Append Gaussians (same SH degree); they start visible at all times
        (Sec. 3.3) and the renderer's buffers are rebuilt for the larger N."""
        r = self.r
        keep = {k: getattr(r, k).detach().cpu().numpy() for k in
                ("mean", "scale", "quat", "opacity", "sh", "inst", "vis_s", "vis_e",
                 "life_s", "life_e")}
        n_new = int(scene_new.mean.shape[0])
        cat = {k: np.concatenate([keep[k], np.asarray(getattr(scene_new, k)).reshape(
            (n_new,) + keep[k].shape[1:])]) for k in keep}
        cat["vis_s"][-n_new:] = -1.0
        cat["vis_e"][-n_new:] = 1.0
        cat["life_s"][-n_new:] = 1.0
        cat["life_e"][-n_new:] = -1.0

        class _S:
            pass
        s = _S()
        for k, v in cat.items():
            setattr(s, k, v)
        s.pose = r.pose.view(r.T, r.S, 3, 4).cpu().numpy()
        s.sh_degree = r.sh_degree
        from .renderer import Renderer
        batches = [h for h in self.handles]
        self.r = Renderer(s, _ViewsOf(batches[0]), r.params, device=r.dev,
                          cap_surv=r.cap_surv + n_new * r.V, cap_dup=r.cap_dup + 64 * n_new)
        self.handles = [self.r._upload_views(_ViewsOf(h)) for h in batches]
        self.opt = Adam(self.opt.lr)


class _ViewsOf:
    """Views-like adapter over an uploaded view set (host arrays kept there)."""

    def __init__(self, vs):
        self.W = vs["W"].cpu().numpy().reshape(-1, 3, 4)
        self.K = vs["K"].cpu().numpy()
        self.wh = vs["wh_np"]
        self.tstep = vs["tstep_np"]

    @property
    def n_views(self):
        return int(self.W.shape[0])
