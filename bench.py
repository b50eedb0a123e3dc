"""Throughput of the per-view fwd+bwd step: streamlined vs plain, same GPU.

Workload (default, the 2M-Gaussian corridor): 1.7M static Gaussians along a
1 km corridor plus 30 instances of 10k, 1920x1080 forward camera, SH degree 3,
LOD threshold 1 px, temporal visibility on after one warm-up pass (UPDATE over
all 50 timesteps, then FOLD).  A step renders one view: project/cull, sort,
raster, L1 loss against a seeded target, backward, point-life update.  Steps
cycle over 8 evenly spaced timesteps.  The plain (conventional) pipeline --
transform every Gaussian to the world frame, project all of them, no temporal
filter and no LOD -- runs the same steps on the same GPU.

Inputs are resident in HBM before the timed region; the timed region is the K
steps between two synchronisations.  Every kernel of the timed steps is
bracketed by HIP events on its stream (the library's opt-in profiler); the
kernel with the largest total time is the one the roofline entry describes.

Prints one JSON line on stdout.  Only one GPU is used (--gpus above 1 is
refused).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
METRIC = "fwd+bwd views/s at 1080p, 2M Gaussians: streamlined vs plain, same GPU"

# algorithmic work per unit (see the design notes): FP32 operations of Eq. (2)
# and its derivative per evaluated (pixel, entry) pair -- an entry whose
# cutoff box meets the pixel's sub-tile, while the pixel still blends -- as
# counted by the forward's work census
FLOP_FWD_PAIR = 22.0     # blending: offsets, quadratic form, o exp(power), clamp,
                         # tests, transmittance and colour update (+1 exp)
FLOP_BWD_PAIR = 60.0     # the backward replay of a pair (+1 exp, +1 rcp)
# the same work itemised: 15 FLOP per evaluated pair (the exponent), and per
# blended pair 8 (forward) or 25 (backward: T recovery, dL/dalpha, dL/dpower,
# five conic moments, opacity and colour gradients)
FLOP_EVAL = 15.0
FLOP_FWD_BLEND = 8.0
FLOP_BWD_BLEND = 25.0
REC_BYTES = 72           # record written per survivor (gid, view, geo, conic, rgb, rect)
GEOM_BYTES = 44          # mean, scale, quat, instance id of a Gaussian that passes


# source files whose change invalidates a kernel's measured HBM traffic
KERNEL_SOURCES = {
    "raster_bwd": ("backward.hip", "common.hpp", "internal.hpp"),
    "raster_fwd": ("raster.hip", "common.hpp", "internal.hpp"),
    "project": ("project.hip", "common.hpp", "internal.hpp"),
    "records": ("project.hip", "common.hpp", "internal.hpp"),
    "radix": ("sort.hip", "common.hpp", "internal.hpp"),
    "project_bwd": ("backward.hip", "common.hpp", "internal.hpp"),
}


# kernels of steps a1-a8 (instance cameras through tile ranges)
PCS_KERNELS = ("compose", "project", "block_offsets", "records", "scan", "emit_pairs", "radix",
               "tile_ranges", "tile_order", "tile_sort", "tile_sort_merge",
               "tile_bin")


def sources_digest(kernel):
    """Digest of the kernel's source files and the compiler flags."""
    from paper_2503_08217_amd.build import FLAGS
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, ()):
        with open(os.path.join(ROOT, "paper_2503_08217_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(FLAGS).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the PMC summary under profiles/
    (FETCH_SIZE + WRITE_SIZE scaled by a copy-kernel calibration), or None when
    there is none or the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    d = re.search(r"sources_sha256_16:\s*([0-9a-f]+)", text)
    if not m or not d or d.group(1) != sources_digest(kernel):
        return None
    return float(m.group(1))


def copy_calibration(mib, torch):
    """A plain device copy of known size (`mib` MiB read and written), run
    twice, whose FETCH_SIZE / WRITE_SIZE readings calibrate the counters."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy calibration: {mib} MiB copied twice")
    del src, dst
    torch.cuda.empty_cache()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_renderer(cfg, plain):
    """The streamlined renderer clears only the gradient rows its previous
    backward wrote (sparse gradient mode); the plain route keeps dense
    world-frame gradient arrays, as the conventional pipeline does."""
    from paper_2503_08217_amd.renderer import Renderer
    params = dict(cfg.params, grad_sparse=not plain)
    if plain:
        params.update(temporal=False, lod=False, lod_r=0.0)
    first = cfg.views.subset([cfg.timed_views[0]])
    return Renderer(cfg.scene, first, params, plain=plain, cap_surv=max(1024, cfg.scene.n // 2),
                    cap_dup=max(4096, 2 * cfg.scene.n))


def warmup_temporal(r, cfg, torch, source="frustum"):
    """Temporal-visibility state after one pass over every timestep (Eq. 5),
    folded into visibility intervals (Eq. 6).  `source` picks the visibility
    that updates the point life: the frustum mask M_t, or "raster", the
    Gaussians blended into at least one pixel (needs a full forward)."""
    from paper_2503_08217_amd import S3R_VIS_FOLD, S3R_VIS_UPDATE
    handles = r.prepare_views([cfg.views.subset([v]) for v in range(cfg.views.n_views)])
    saved = dict(r.params)
    r.set_flags(temporal=False)
    for h in handles:
        r.use_views(h)
        if source == "raster":
            r.fit_capacity()
        else:
            r.project_cull()
        r.update_visibility(S3R_VIS_UPDATE, source=source)
    r.update_visibility(S3R_VIS_FOLD)
    r.set_flags(**saved)
    torch.cuda.synchronize()


def view_units(r, handles, targets, torch):
    """Per timed view: stats and the algorithmic units of each kernel (the
    forward's work census: evaluated and blended (pixel, entry) pairs)."""
    out = []
    for h, tg in zip(handles, targets):
        r.use_views(h)
        cen = r.work_census()
        torch.cuda.synchronize()
        st = r.stats.cpu().numpy()[0].astype(np.int64)
        last = r.last[: r.total_px].to(torch.int64).sum().item()
        out.append(dict(N_t=int(st[0]), N_f=int(st[1]), N_r=int(st[2]), N_dup=int(st[3]),
                        pairs_last=int(last), pairs_eval=cen["evaluated"],
                        pairs_blend=cen["blended"]))
    return out


def timed(r, handles, targets, steps, warmup, torch, profile=True):
    """Warm-up steps with every kernel timed (this picks the dominant kernel),
    then the timed region: `steps` steps with only the dominant kernel
    bracketed by HIP events.  Returns (seconds, {kernel: (ms, launches)} of
    the profiled warm-up steps, the handle index of each of those steps,
    (dominant name, ms, launches) of the timed region).  The first warm-up
    step carries one-time costs and is left out of the table when there are
    more."""
    from paper_2503_08217_amd import _abi
    lib = _abi.load()
    _abi.check(lib.s3r_profile_reset(), "profile reset")
    _abi.check(lib.s3r_profile_only(-1), "profile only")
    _abi.check(lib.s3r_profile_enable(1), "profile enable")
    profiled = []
    for i in range(warmup):
        h = i % len(handles)
        r.use_views(handles[h])
        r.step(targets[h])
        profiled.append(h)
        if i == 0 and warmup > 1:
            # first launches carry one-time costs: they do not pick the
            # dominant kernel
            torch.cuda.synchronize()
            _abi.check(lib.s3r_profile_reset(), "profile reset")
            profiled = []
    torch.cuda.synchronize()
    table = _abi.profile_table()
    dom = max(table.items(), key=lambda kv: kv[1][0])[0]
    _abi.check(lib.s3r_profile_reset(), "profile reset")
    _abi.check(lib.s3r_profile_only(_abi.profile_id(dom)), "profile only")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        h = i % len(handles)
        r.use_views(handles[h])
        r.step(targets[h])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    live = _abi.profile_table()
    _abi.check(lib.s3r_profile_enable(0), "profile disable")
    _abi.check(lib.s3r_profile_only(-1), "profile only")
    return t1 - t0, table, profiled, (dom,) + tuple(live.get(dom, (0.0, 0)))


def kernel_roofline(name, total_ms, launches, units, steps, sh_degree, n):
    """Algorithmic work of the timed steps for kernel `name` -> (bound,
    achieved, peak, unit, basis, extra)."""
    nviews = len(units)
    # the timed steps cycle over the views: work of step i is that of view i % nviews
    per = [units[i % nviews] for i in range(steps)]
    sh_bytes = 12 * (sh_degree + 1) ** 2
    sec = total_ms * 1e-3
    if name in ("raster_bwd", "raster_fwd"):
        fwd = name == "raster_fwd"
        per_pair = FLOP_FWD_PAIR if fwd else FLOP_BWD_PAIR
        blend = FLOP_FWD_BLEND if fwd else FLOP_BWD_BLEND
        ev = sum(u["pairs_eval"] for u in per)
        bl = sum(u["pairs_blend"] for u in per)
        last = sum(u["pairs_last"] for u in per)
        work = ev * per_pair

        def model(flop, what):
            return {"achieved": flop / sec / 1e12, "frac": flop / sec / 1e12 / FP32_PEAK_TFLOPS,
                    "work": what}
        extra = {"pairs_per_launch": {"list_entries_to_last": last / steps, "evaluated": ev / steps,
                                      "blended": bl / steps},
                 "flop_per_launch": work / steps,
                 "other_models": {
                     "per_blended_pair": model(bl * per_pair, f"{per_pair:.0f} FLOP per blended pair"),
                     "itemised": model(FLOP_EVAL * ev + blend * bl,
                                       f"{FLOP_EVAL:.0f} FLOP per evaluated + {blend:.0f} per "
                                       "blended pair"),
                     "per_list_entry": model(last * per_pair,
                                             f"{per_pair:.0f} FLOP per list entry up to each "
                                             "pixel's last contributor (counts entries the "
                                             "cutoff box skips: an upper bound)")}}
        return "alu", work / sec / 1e12, FP32_PEAK_TFLOPS, "TFLOP/s", \
            (f"{per_pair:.0f} FLOP + 1 exp per evaluated (pixel, entry) pair (work census of "
             "the forward)"), extra
    if name == "project":
        b = sum(8 * n + GEOM_BYTES * u["N_t"] + n / 8 + (4 + sh_bytes + REC_BYTES) * u["N_r"]
                for u in per)
        return "hbm", b / sec / 1e9, HBM_PEAK_GBS, "GB/s", \
            "8 N + 44 N_t + N/8 + (4 + 12(L+1)^2 + 72) N_r bytes", {}
    if name == "radix":
        passes = launches // steps // 2
        b = sum((8 + 24) * passes * u["N_dup"] for u in per)
        return "hbm", b / sec / 1e9, HBM_PEAK_GBS, "GB/s", \
            "per radix pass 8 B read (histogram) + 12 B read + 12 B written per pair", {}
    if name == "records":
        b = sum((GEOM_BYTES + 4 + sh_bytes + REC_BYTES + 4) * u["N_r"] for u in per)
        return "hbm", b / sec / 1e9, HBM_PEAK_GBS, "GB/s", \
            "(44 + 4 + 12(L+1)^2 + 76) N_r bytes", {}
    if name == "project_bwd":
        b = sum((48 + 4 + 2 * sh_bytes + 40 + 48) * u["N_r"] for u in per)
        return "hbm", b / sec / 1e9, HBM_PEAK_GBS, "GB/s", \
            "(read 48 + 4 + 12(L+1)^2 + g2d 48, write 40 + 12(L+1)^2) N_r bytes", {}
    return None


def pcs_span(r, handles, torch, reps=3):
    """Wall time on the GPU of steps a1-a8 (s3r_project_cull + s3r_sort) per
    call, launch gaps included, between two events on the renderer's stream;
    mean over `reps` passes over the handles."""
    ev = []
    for _ in range(reps):
        for h in handles:
            r.use_views(h)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            r.project_cull()
            r.sort()
            e1.record()
            ev.append((e0, e1))
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in ev]))


def pcs_batch_bytes(batch, sh_degree, n):
    """Algorithmic HBM bytes of project/cull/sort for one batch of views (a
    list of per-view units): every Gaussian's visibility interval once, the
    geometry of the Gaussians that pass the temporal test (counted for the
    view where most pass: a lower bound on the union), per view the M_t bits,
    SH + opacity + record of each survivor, and every (tile, record) pair
    written once and read + written once by a sort."""
    sh_bytes = 12 * (sh_degree + 1) ** 2
    return (8 * n + GEOM_BYTES * max(u["N_t"] for u in batch)
            + sum(n / 8 + (4 + sh_bytes + REC_BYTES) * u["N_r"] + 36 * u["N_dup"] for u in batch))


def pcs_bytes(units, view_ids, sh_degree, n):
    """pcs_batch_bytes over one-view steps rendering units[i] for i in view_ids."""
    return sum(pcs_batch_bytes([units[i]], sh_degree, n) for i in view_ids)


def cpu_baseline(cfg, n_tiles_sample=160):
    """The oracle as it stands, on a bounded sample of one view of the same
    workload: the binary32 decision layer and colours over all N Gaussians,
    then FP64 blending + autograd backward of `n_tiles_sample` random 16x16
    tiles, scaled to a whole view."""
    import torch

    from oracle import grad as ograd
    from oracle import order, render
    threads = len(os.sched_getaffinity(0))
    torch.set_num_threads(threads)
    v = cfg.timed_views[len(cfg.timed_views) // 2]
    t0 = time.perf_counter()
    o = render.render_view(cfg.scene, cfg.views, v, cfg.params, with_image=False)
    t_dec = time.perf_counter() - t0
    d = o["dec"]
    w, h = int(cfg.views.wh[v, 0]), int(cfg.views.wh[v, 1])
    ts = int(cfg.params["tile"])
    gx, gy = (w + ts - 1) // ts, (h + ts - 1) // ts
    rng = np.random.default_rng(7)
    pt = ograd.to_torch_params(cfg.scene)
    t1 = time.perf_counter()
    tg = np.asarray(rng.uniform(0, 1, (3, ts, ts)))
    for _ in range(n_tiles_sample):
        tx, ty = int(rng.integers(gx)), int(rng.integers(gy))
        reg = (tx * ts, ty * ts, min(w, tx * ts + ts), min(h, ty * ts + ts))
        ids = o["ids"]
        uu, vv = d["u"][ids].astype(np.float64), d["v"][ids].astype(np.float64)
        ddx = np.maximum(0.0, np.maximum(reg[0] - uu, uu - (reg[2] - 1)))
        ddy = np.maximum(0.0, np.maximum(reg[1] - vv, vv - (reg[3] - 1)))
        lim = 2.0 * cfg.params["cutoff"] * d["lam_d"][ids].astype(np.float64) * 1.0001
        cand = order.global_order(ids[ddx * ddx + ddy * ddy <= lim], d["depth_bits"])
        img, _ = ograd.render_t(pt, cfg.scene, cfg.views, v, cand, cfg.params, region=reg)
        loss = ograd.l1_loss_t(img, tg[:, : reg[3] - reg[1], : reg[2] - reg[0]])
        loss.backward()
    t_tiles = time.perf_counter() - t1
    per_view = t_dec + t_tiles / n_tiles_sample * gx * gy
    return {"value": 1.0 / per_view, "unit": "views/s", "cores": int(torch.get_num_threads()),
            "kind": "oracle",
            "sample": (f"one {w}x{h} view of the same workload: binary32 decisions + SH colours over "
                       f"all {cfg.scene.n} Gaussians without the temporal pre-filter (same survivors, "
                       f"more projections; {t_dec:.1f}s, single-threaded numpy), FP64 "
                       f"blending + autograd backward of {n_tiles_sample} random {ts}x{ts} tiles "
                       f"({t_tiles:.1f}s, torch CPU), scaled to the view's {gx * gy} tiles")}


def lod_temporal_sweep(cfg, targets, torch, steps=16):
    """views/s of the streamlined step over LOD threshold x temporal filter."""
    r = make_renderer(cfg, plain=False)
    warmup_temporal(r, cfg, torch)
    handles = r.prepare_views([cfg.views.subset([v]) for v in cfg.timed_views])
    out = []
    for temporal in (True, False):
        for lod_r in (0.0, 0.5, 1.0, 2.0):
            r.set_flags(temporal=temporal, lod=lod_r > 0, lod_r=lod_r)
            for h in handles:
                r.use_views(h)
                r.fit_capacity()
            handles = r.prepare_views([cfg.views.subset([v]) for v in cfg.timed_views])
            for i in range(4):
                r.use_views(handles[i % len(handles)])
                r.step(targets[i % len(handles)])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(steps):
                r.use_views(handles[i % len(handles)])
                r.step(targets[i % len(handles)])
            torch.cuda.synchronize()
            vps = steps / (time.perf_counter() - t0)
            st = []
            for h in handles:
                r.use_views(h)
                r.forward()
                torch.cuda.synchronize()
                st.append(r.stats.cpu().numpy()[0].tolist())
            mean = np.mean(np.asarray(st, np.float64), 0)
            out.append({"lod_r": lod_r, "temporal": temporal, "views_per_s": vps,
                        "mean_N_t": mean[0], "mean_N_r": mean[2], "mean_N_dup": mean[3]})
            log(f"sweep lod_r={lod_r} temporal={temporal}: {vps:.1f} views/s, "
                f"N_t {mean[0]:.0f} N_r {mean[2]:.0f} N_dup {mean[3]:.0f}")
    del r
    torch.cuda.empty_cache()
    return out


def scale_up(torch, lengths, steps=16):
    """Per-view fwd+bwd time as the corridor grows at constant density and
    camera (1700 static Gaussians per metre, 30 instances per km, one frame
    every 20 m), streamlined vs plain: the paper's scale-up experiment."""
    import scenes
    out = []
    for L in lengths:
        t0 = time.perf_counter()
        cfg = scenes.make_scaleup(L)
        tg_np = scenes.targets(cfg.cfg, cfg.views, cfg.timed_views)
        targets = [torch.as_tensor(t.ravel()).cuda().contiguous() for t in tg_np]
        row = {"length_m": L, "gaussians": int(cfg.scene.n), "timesteps": int(cfg.views.n_views),
               "generated_s": time.perf_counter() - t0}
        for plain in (False, True):
            r = make_renderer(cfg, plain)
            if not plain:
                warmup_temporal(r, cfg, torch)
            handles = r.prepare_views([cfg.views.subset([v]) for v in cfg.timed_views])
            for h in handles:
                r.use_views(h)
                r.fit_capacity()
            handles = r.prepare_views([cfg.views.subset([v]) for v in cfg.timed_views])
            units = view_units(r, handles, targets, torch)
            for i in range(4):
                r.use_views(handles[i % len(handles)])
                r.step(targets[i % len(handles)])
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for i in range(steps):
                r.use_views(handles[i % len(handles)])
                r.step(targets[i % len(handles)])
            torch.cuda.synchronize()
            ms = 1000 * (time.perf_counter() - t1) / steps
            mean = {k: float(np.mean([u[k] for u in units])) for k in ("N_t", "N_r", "N_dup")}
            row["plain" if plain else "streamlined"] = dict(ms_per_view=ms, **mean)
            del r
            torch.cuda.empty_cache()
        log(f"scale-up {L:6.0f} m, N={row['gaussians']}: streamlined "
            f"{row['streamlined']['ms_per_view']:.3f} ms/view (N_t {row['streamlined']['N_t']:.0f},"
            f" N_r {row['streamlined']['N_r']:.0f}), plain {row['plain']['ms_per_view']:.3f} ms/view")
        out.append(row)
    return out


def visibility_sources(cfg, targets, torch, steps=16):
    """The two readings of the visibility the rendering process yields: the
    frustum mask M_t and the Gaussians blended into at least one pixel.  Each
    drives the warm-up UPDATE and FOLD; reported: Gaussians passing the
    temporal test per timed view, and views/s of the streamlined step."""
    out = {}
    for source in ("frustum", "raster"):
        from paper_2503_08217_amd.renderer import Renderer
        params = dict(cfg.params, grad_sparse=True, raster_mask=(source == "raster"),
                      visibility_source=source)
        first = cfg.views.subset([cfg.timed_views[0]])
        r = Renderer(cfg.scene, first, params, cap_surv=max(1024, cfg.scene.n // 2),
                     cap_dup=max(4096, 2 * cfg.scene.n))
        warmup_temporal(r, cfg, torch, source=source)
        handles = r.prepare_views([cfg.views.subset([v]) for v in cfg.timed_views])
        for h in handles:
            r.use_views(h)
            r.fit_capacity()
        handles = r.prepare_views([cfg.views.subset([v]) for v in cfg.timed_views])
        units = view_units(r, handles, targets, torch)
        for i in range(4):
            r.use_views(handles[i % len(handles)])
            r.step(targets[i % len(handles)])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            r.use_views(handles[i % len(handles)])
            r.step(targets[i % len(handles)])
        torch.cuda.synchronize()
        vps = steps / (time.perf_counter() - t0)
        out[source] = {"views_per_s": vps,
                       "mean_N_t": float(np.mean([u["N_t"] for u in units])),
                       "mean_N_r": float(np.mean([u["N_r"] for u in units]))}
        log(f"visibility source {source}: {vps:.1f} views/s, N_t {out[source]['mean_N_t']:.0f}, "
            f"N_r {out[source]['mean_N_r']:.0f}")
        del r
        torch.cuda.empty_cache()
    return out


def lifecycle(cfg, torch, epochs=6, reset_every=3):
    """The temporal-visibility lifecycle over training epochs (Sec. 3.3,
    Eqs. 5-6): every epoch renders all timesteps one view per step (forward,
    L1 loss, backward, point-life update, Adam), then folds the visibility,
    or resets it every `reset_every` epochs.  Returns per epoch the action,
    the mean loss and the mean fraction of Gaussians passing the temporal
    test."""
    import scenes
    from paper_2503_08217_amd.train import Trainer
    r = make_renderer(cfg, plain=False)
    r.zero_grads()
    views = list(range(cfg.views.n_views))
    batches = [cfg.views.subset([v]) for v in views]
    targets = [torch.as_tensor(t.ravel()).cuda() for t in scenes.targets(cfg.cfg, cfg.views, views)]
    tr = Trainer(r, batches, targets, reset_every=reset_every)
    out = []
    for e in range(epochs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec = tr.epoch(e)
        rec["ms_per_step"] = 1000 * (time.perf_counter() - t0) / len(views)
        out.append(rec)
        log(f"lifecycle epoch {e}: loss {rec['loss']:.5f}, temporal pass "
            f"{rec['temporal_pass']:.3f}, then {rec['action']} ({rec['ms_per_step']:.2f} ms/step "
            f"incl. Adam)")
    del tr, r, targets
    torch.cuda.empty_cache()
    return out


def batched_graph(cfg, torch, replays, tiles, sorts=("tiles", "global"), waves=(1, 4)):
    """Batched multi-view step (all timed views of the workload in one batch)
    captured in a HIP graph.  With more than one candidate, the tile size,
    sort mode and forward waves per workgroup come from the library's
    autotuner (eager steps timed per candidate, same image required); the
    chosen shape is then captured and replayed `replays` times."""
    from paper_2503_08217_amd import S3R_VIS_FOLD, S3R_VIS_UPDATE
    from paper_2503_08217_amd import _abi
    from paper_2503_08217_amd.autotune import autotune
    from paper_2503_08217_amd.renderer import Renderer
    import scenes
    views = cfg.views.subset(cfg.timed_views)
    tg = scenes.targets(cfg.cfg, views)
    target = torch.as_tensor(np.concatenate([t.ravel() for t in tg])).cuda()
    del tg
    # temporal state: one pass over every timestep with the rig of one timestep
    rig = sorted(set(int(t) for t in cfg.views.tstep))
    per_t = [np.nonzero(cfg.views.tstep == t)[0] for t in rig]
    warm = Renderer(cfg.scene, cfg.views.subset(per_t[0]), dict(cfg.params, temporal=False),
                    cap_surv=max(1024, cfg.scene.n // 4), cap_dup=max(4096, cfg.scene.n))
    hs = warm.prepare_views([cfg.views.subset(ix) for ix in per_t])
    for h in hs:
        warm.use_views(h)
        warm.project_cull()
        warm.update_visibility(S3R_VIS_UPDATE)
    warm.update_visibility(S3R_VIS_FOLD)
    torch.cuda.synchronize()
    vis_s, vis_e = warm.vis_s.clone(), warm.vis_e.clone()
    del warm, hs
    torch.cuda.empty_cache()
    caps = dict(cap_surv=max(1024, cfg.scene.n // 2), cap_dup=max(4096, 2 * cfg.scene.n))
    base = dict(cfg.params, grad_sparse=True)
    tune = None
    if len(tiles) * len(sorts) * len(waves) > 1:
        tune = autotune(cfg.scene, views, base, target, tiles=tiles, sorts=sorts,
                        raster_waves=waves, reps=5, vis=(vis_s, vis_e), log=log, **caps)
        choice = tune["best"]
    else:
        choice = dict(tile=tiles[0], sort=sorts[0], raster_waves=waves[0], binning=True)
        _abi.set_tuning(raster_waves=waves[0])
    params = dict(base, tile=choice["tile"], sort=choice["sort"])
    r = Renderer(cfg.scene, views, params, **caps)
    r.vis_s.copy_(vis_s)
    r.vis_e.copy_(vis_e)
    c = r.fit_capacity()
    g = r.capture_step(target, update_visibility=True)
    times = []
    for i in range(replays):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        times.append((e0, e1))
    torch.cuda.synchronize()
    ms = np.asarray([a.elapsed_time(b) for a, b in times])
    st = r.stats.cpu().numpy()
    # a few eager steps with every kernel timed: per-kernel breakdown and
    # the project/cull/sort share of HBM peak for this batch
    lib = _abi.load()
    _abi.check(lib.s3r_profile_reset(), "profile reset")
    _abi.check(lib.s3r_profile_only(-1), "profile only")
    _abi.check(lib.s3r_profile_enable(1), "profile enable")
    prof_steps = 3
    for _ in range(prof_steps):
        r.step(target)
    torch.cuda.synchronize()
    table = _abi.profile_table()
    _abi.check(lib.s3r_profile_enable(0), "profile disable")
    units = [dict(N_t=int(x[0]), N_f=int(x[1]), N_r=int(x[2]), N_dup=int(x[3])) for x in st]
    pcs_ms = sum(table[k][0] for k in PCS_KERNELS if k in table) / prof_steps
    pcs_b = pcs_batch_bytes(units, cfg.scene.sh_degree, cfg.scene.n)
    res = {"tile": choice["tile"], "sort": choice["sort"], "raster_waves": choice["raster_waves"],
           "binning": choice["binning"], "p50_ms": float(np.percentile(ms, 50)),
           "p99_ms": float(np.percentile(ms, 99)), "mean_ms": float(ms.mean()),
           "views_per_s": views.n_views / (ms.mean() * 1e-3),
           "temporal_pass_fraction": float(st[:, 0].mean() / cfg.scene.n),
           "frustum_visible_fraction": float(st[:, 1].mean() / cfg.scene.n),
           "records": c["n_surv"], "pairs": c["n_dup"],
           "gaussians_per_s": cfg.scene.n * views.n_views / (ms.mean() * 1e-3),
           "project_cull_sort_hbm": {"achieved": pcs_b / (pcs_ms * 1e-3) / 1e9,
                                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": pcs_b / (pcs_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                     "ms_per_step": pcs_ms, "bytes": pcs_b},
           "kernels_us_per_step": {k: 1000 * v[0] / prof_steps for k, v in table.items()}}
    log(f"batched {cfg.name} tile {choice['tile']} sort {choice['sort']} waves "
        f"{choice['raster_waves']}: p50 {res['p50_ms']:.2f} ms, p99 {res['p99_ms']:.2f} ms, "
        f"{res['views_per_s']:.1f} views/s, N_t/N {res['temporal_pass_fraction']:.3f}, N_f/N "
        f"{res['frustum_visible_fraction']:.3f}, project/cull/sort "
        f"{res['project_cull_sort_hbm']['ms_per_step']:.3f} ms at "
        f"{100 * res['project_cull_sort_hbm']['frac']:.1f}% of HBM peak")
    for k, v in sorted(res["kernels_us_per_step"].items(), key=lambda kv: -kv[1])[:12]:
        log(f"   {k:22s} {v:9.1f} us/step")
    del g, r
    torch.cuda.empty_cache()
    _abi.set_tuning(**{k: -1 for k in _abi.TUNE_KNOBS})
    return {"workload": cfg.name, "views_per_batch": views.n_views, "replays": replays,
            "best": res, "autotune": tune["table"] if tune else None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tile", type=int, default=16, choices=(8, 16, 32))
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the LOD threshold x temporal filter grid")
    ap.add_argument("--replays", type=int, default=100)
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched 24-view graph replays of the rig and city workloads")
    ap.add_argument("--batched-replays", type=int, default=30)
    ap.add_argument("--no-lifecycle", action="store_true",
                    help="skip the training epochs with fold / reset of the visibility")
    ap.add_argument("--scale-up", action="store_true",
                    help="per-view time vs corridor length (125 m .. 3 km), then exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run a plain copy of this many MiB first (for counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported here "
              "(views would be sharded across GPUs with a gradient all-reduce)", file=sys.stderr)
        sys.exit(2)

    import torch

    import scenes

    if a.copy_calibration > 0:
        copy_calibration(a.copy_calibration, torch)
    if a.scale_up:
        rows = scale_up(torch, (125.0, 250.0, 500.0, 1000.0, 2000.0, 3000.0), steps=a.steps)
        print(json.dumps({"metric": "per-view fwd+bwd ms vs corridor length, streamlined vs plain",
                          "unit": "ms/view", "data": "synthetic", "rows": rows}), flush=True)
        return
    t_gen = time.perf_counter()
    cfg = scenes.make_config(a.config)
    cfg.params["tile"] = a.tile
    if a.config in (4, 5):
        out = batched_graph(cfg, torch, a.replays, (8, 16, 32))
        out["metric"] = "batched fwd+bwd step, hipGraph replay"
        print(json.dumps(out), flush=True)
        return
    log(f"config {a.config} ({cfg.name}) generated in {time.perf_counter() - t_gen:.1f}s, "
        f"N={cfg.scene.n}, tile {a.tile}")
    tg_np = scenes.targets(a.config, cfg.views, cfg.timed_views)
    targets = [torch.as_tensor(t.ravel()).cuda().contiguous() for t in tg_np]

    results = {}
    for plain in ([False] if a.no_plain else [False, True]):
        name = "plain" if plain else "streamlined"
        r = make_renderer(cfg, plain)
        if cfg.warmup_fold and not plain:
            warmup_temporal(r, cfg, torch)
            log("temporal warm-up done")
        handles = r.prepare_views([cfg.views.subset([v]) for v in cfg.timed_views])
        for h in handles:
            r.use_views(h)
            r.fit_capacity()
        handles = r.prepare_views([cfg.views.subset([v]) for v in cfg.timed_views])
        units = view_units(r, handles, targets, torch)
        log(f"{name}: per view (N_t, N_f, N_r, N_dup, evaluated, blended) "
            f"{[(u['N_t'], u['N_f'], u['N_r'], u['N_dup'], u['pairs_eval'], u['pairs_blend']) for u in units]}")
        span = pcs_span(r, handles, torch)
        elapsed, table, profiled, live = timed(r, handles, targets, a.steps, a.warmup, torch)
        vps = a.steps / elapsed
        log(f"{name}: {vps:.1f} views/s, {1000 * elapsed / a.steps:.3f} ms/step; dominant "
            f"{live[0]} {1000 * live[1] / max(live[2], 1):.1f} us x {live[2]} (timed region); "
            f"project/cull/sort span {1000 * span:.1f} us per view")
        for k, (ms, cnt) in sorted(table.items(), key=lambda kv: -kv[1][0]):
            log(f"   {k:22s} {1000 * ms / cnt:9.1f} us x {cnt}  (warm-up)")
        results[name] = dict(vps=vps, ms=1000 * elapsed / a.steps, table=table, units=units,
                             live=live, profiled=profiled, span=span)
        del r
        torch.cuda.empty_cache()

    s = results["streamlined"]
    table, units, profiled = s["table"], s["units"], s["profiled"]
    dname, dms, dcnt = s["live"]
    rl = kernel_roofline(dname, dms, dcnt, units, a.steps, cfg.scene.sh_degree, cfg.scene.n)
    roof = None
    if rl:
        bound, ach, peak, unit, basis, extra = rl
        roof = {"bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
                "traffic": measured_traffic(dname, cfg.name), "kernel": dname,
                "avg_us": 1000 * dms / dcnt, "work": basis,
                "sources_sha256_16": sources_digest(dname), **extra}
    # the profiled warm-up steps (every kernel timed) give the project/cull/sort
    # kernel time; bytes are those of the views those steps rendered
    npro = max(len(profiled), 1)
    pcs_ms = sum(table[k][0] for k in PCS_KERNELS if k in table)
    pcs_b = pcs_bytes(units, profiled, cfg.scene.sh_degree, cfg.scene.n)
    pcs_gbs = pcs_b / (pcs_ms * 1e-3) / 1e9
    span_b = pcs_bytes(units, range(len(units)), cfg.scene.sh_degree, cfg.scene.n) / len(units)
    span_gbs = span_b / (s["span"] * 1e-3) / 1e9
    wh = cfg.views.wh[cfg.timed_views[0]]
    out = {
        "metric": METRIC,
        "value": s["vps"],
        "unit": "views/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": s["ms"],
        "gaussians_per_s": cfg.scene.n * s["vps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg.name, "gaussians": int(cfg.scene.n),
                   "instances": int(cfg.scene.n_slots - 1),
                   "resolution": f"{int(wh[0])}x{int(wh[1])}", "views_per_step": 1,
                   "sh_degree": int(cfg.scene.sh_degree), "tile": int(cfg.params["tile"]),
                   "lod_r_px": float(cfg.params["lod_r"]) if cfg.params.get("lod") else 0.0,
                   "temporal": ("on (after warm-up fold)" if cfg.params.get("temporal")
                                and cfg.warmup_fold else
                                "on" if cfg.params.get("temporal") else "off")},
        "roofline": roof,
        "project_cull_sort_hbm": {
            "achieved": pcs_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": pcs_gbs / HBM_PEAK_GBS, "ms_per_step": pcs_ms / npro,
            "bytes_per_step": pcs_b / npro, "profiled_steps": npro,
            "basis": "algorithmic bytes of the profiled warm-up steps / the sum of their a1-a8 "
                     "kernel times (HIP events around each launch)",
            "span": {"achieved": span_gbs, "frac": span_gbs / HBM_PEAK_GBS,
                     "ms_per_view": s["span"],
                     "basis": "mean algorithmic bytes per timed view / GPU time from the first "
                              "a1 launch to the end of the last a8 launch (gaps included)"}},
        "kernels_us_per_step_warmup": {k: 1000 * ms / npro for k, (ms, cnt) in table.items()},
        "launches_per_step_warmup": {k: cnt / npro for k, (ms, cnt) in table.items()},
    }
    if "plain" in results:
        p = results["plain"]
        out["plain_views_per_s"] = p["vps"]
        out["speedup_vs_plain"] = s["vps"] / p["vps"]
        npp = max(len(p["profiled"]), 1)
        out["plain_kernels_us_per_step_warmup"] = {k: 1000 * ms / npp
                                                   for k, (ms, cnt) in p["table"].items()}
    if not a.no_sweep and a.config == 3:
        out["sweep"] = lod_temporal_sweep(cfg, targets, torch)
        out["visibility_source"] = visibility_sources(cfg, targets, torch)
    if not a.no_lifecycle and a.config == 3:
        out["lifecycle"] = lifecycle(cfg, torch)
    if not a.no_batched and a.config == 3:
        # the batched workloads at one tile and sort mode (the full search:
        # --config 4 / --config 5)
        del targets
        torch.cuda.empty_cache()
        out["batched"] = {}
        for cid, tile in ((4, 16), (5, 32)):
            t0 = time.perf_counter()
            bc = scenes.make_config(cid)
            log(f"config {cid} ({bc.name}) generated in {time.perf_counter() - t0:.1f}s")
            res = batched_graph(bc, torch, a.batched_replays, (tile,), ("tiles",), (1,))
            out["batched"][bc.name] = res["best"]
            del bc
            torch.cuda.empty_cache()
    if not a.no_cpu:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(cfg)
        log(f"cpu baseline {out['cpu_baseline']['value']:.5f} views/s "
            f"({time.perf_counter() - t0:.1f}s)")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
