"""Throughput of the per-view fwd+bwd step: streamlined vs plain, same GPU.

Workload (default): the 2M-Gaussian, 1 km corridor with 30 instances,
1920x1080 forward camera, SH degree 3, LOD threshold 1 px, temporal
visibility on after a warm-up pass (UPDATE over all 50 timesteps, then FOLD).
A step is one view: project/cull, sort, raster, L1 loss, backward and the
point-life update.  Steps cycle over 8 evenly spaced timesteps.  The plain
(conventional) pipeline -- transform every Gaussian to the world frame,
project everything, no temporal filter, no LOD -- is timed the same way on
the same GPU.

Prints one JSON line.  Only one GPU is used (--gpus above 1 is refused).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_renderer(cfg, plain, torch):
    from paper_2503_08217_amd.renderer import Renderer
    import scenes
    c = cfg
    params = dict(c.params)
    if plain:
        params.update(temporal=False, lod=False, lod_r=0.0)
    first = c.views.subset([c.timed_views[0]])
    r = Renderer(c.scene, first, params, plain=plain, cap_surv=max(1024, c.scene.n // 2),
                 cap_dup=max(4096, 2 * c.scene.n))
    return r


def warmup_temporal(r, cfg, torch):
    """Temporal-visibility state after one pass over every timestep (Eq. 5),
    folded into visibility intervals (Eq. 6)."""
    from paper_2503_08217_amd import S3R_VIS_FOLD, S3R_VIS_UPDATE
    handles = r.prepare_views([cfg.views.subset([v]) for v in range(cfg.views.n_views)])
    saved = dict(r.params)
    r.set_flags(temporal=False)
    for h in handles:
        r.use_views(h)
        r.project_cull()
        r.update_visibility(S3R_VIS_UPDATE)
    r.update_visibility(S3R_VIS_FOLD)
    r.set_flags(**saved)
    torch.cuda.synchronize()


def time_steps(r, handles, targets, steps, warmup, torch):
    ev = {}

    def mark(name):
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        ev.setdefault(name, []).append(e)

    for i in range(warmup):
        h = i % len(handles)
        r.use_views(handles[h])
        r.step(targets[h])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        h = i % len(handles)
        r.use_views(handles[h])
        mark("a")
        if r.plain:
            r.plain_transform()
        r.project_cull()
        mark("b")
        r.sort()
        mark("c")
        r.raster_fwd()
        mark("d")
        r.l1_loss(targets[h])
        r.zero_grads()
        mark("e")
        r.raster_bwd()
        mark("f")
        if not r.plain:
            from paper_2503_08217_amd import S3R_VIS_UPDATE
            r.update_visibility(S3R_VIS_UPDATE)
        mark("g")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    seg = {}
    names = ["a", "b", "c", "d", "e", "f", "g"]
    labels = ["project", "sort", "raster_fwd", "loss", "backward", "visibility"]
    for j, lab in enumerate(labels):
        s, e = ev[names[j]], ev[names[j + 1]]
        seg[lab] = float(np.mean([s[i].elapsed_time(e[i]) for i in range(steps)]))
    return (t1 - t0), seg


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              "(the path would shard views across GPUs; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import scenes

    t_gen = time.perf_counter()
    cfg = scenes.make_config(a.config)
    log(f"config {a.config} ({cfg.name}) generated in {time.perf_counter() - t_gen:.1f}s, "
        f"N={cfg.scene.n}")
    tg_np = scenes.targets(a.config, cfg.views, cfg.timed_views)
    targets = [torch.as_tensor(t.ravel()).cuda().contiguous() for t in tg_np]

    results = {}
    for plain in ([False] if a.no_plain else [False, True]):
        name = "plain" if plain else "streamlined"
        r = build_renderer(cfg, plain, torch)
        if cfg.warmup_fold and not plain:
            warmup_temporal(r, cfg, torch)
            log("temporal warm-up done")
        handles = r.prepare_views([cfg.views.subset([v]) for v in cfg.timed_views])
        # size capacities on the heaviest timed view
        for h in handles:
            r.use_views(h)
            r.fit_capacity()
        handles = r.prepare_views([cfg.views.subset([v]) for v in cfg.timed_views])
        stats = []
        for h in handles:
            r.use_views(h)
            r.forward()
            torch.cuda.synchronize()
            stats.append(r.stats.cpu().numpy()[0].tolist())
        log(f"{name}: per-view [N_t, N_f, N_r, N_dup] = {stats}")
        elapsed, seg = time_steps(r, handles, targets, a.steps, a.warmup, torch)
        vps = a.steps / elapsed
        log(f"{name}: {vps:.1f} views/s, {1000 * elapsed / a.steps:.3f} ms/step, segments(ms)={seg}")
        results[name] = dict(views_per_s=vps, ms_per_step=1000 * elapsed / a.steps, seg=seg,
                             stats=stats)
        del r
        torch.cuda.empty_cache()

    s = results["streamlined"]
    out = {
        "metric": "fwd+bwd views/s at 1080p, 2M Gaussians: streamlined vs plain, same GPU",
        "value": s["views_per_s"],
        "unit": "views/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": s["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg.name, "gaussians": int(cfg.scene.n), "instances": 30,
                   "resolution": "1920x1080", "views_per_step": 1, "sh_degree": 3,
                   "lod_r_px": 1.0, "temporal": "on (after warm-up fold)"},
        "segments_ms": s["seg"],
    }
    if "plain" in results:
        out["plain_views_per_s"] = results["plain"]["views_per_s"]
        out["speedup_vs_plain"] = s["views_per_s"] / results["plain"]["views_per_s"]
        out["plain_segments_ms"] = results["plain"]["seg"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
