"""Launch-shape autotuner of the per-view step.

`autotune` times one whole training step (forward, L1 loss, backward,
point-life update) of a batch of views for every candidate of

* the tile edge (8, 16, 32 px): changes the lists, the sort and both
  rasterizers' work decomposition,
* the sort mode ("tiles": binning or tile partition plus per-list depth
  sorts; "global": one radix sort over (tile, depth) keys),
* the forward rasterizer's waves per workgroup (S3R_TUNE_RASTER_WAVES: one
  8x8 sub-tile per workgroup, or all of a tile's sub-tiles together),
* the tile binning limit (S3R_TUNE_BIN_MAX_TILES: LDS binning, or the radix
  tile partition),

then, at the fastest of those, the number of longest tiles the forward
rasterizes in 4x4 blocks (S3R_TUNE_FINE_TILES), and keeps the fastest.  Every candidate must render the same image bit for
bit (the Mahalanobis cutoff makes images independent of the tile size, and
the launch shapes change no arithmetic); a candidate that does not is an
error, not a choice.  The project/cull workgroup shape is fixed by the
per-256-Gaussian-block layout of S3RProjected.bstat and is not searched.
"""

from __future__ import annotations

import itertools
import time

import numpy as np
import torch

from . import _abi as A


def _time_step(r, target, reps, warm=2):
    for _ in range(warm):
        r.step(target, update_visibility=False)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        r.step(target, update_visibility=False)
        e1.record()
        ms.append((e0, e1))
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ms]))


def autotune(scene, views, params, target, *, tiles=(8, 16, 32), sorts=("tiles", "global"),
             raster_waves=(1, 4, 16), binning=(True, False), fine_tiles=(0, 64, 160, 256, 1024),
             reps=5, vis=None, device="cuda", cap_surv=None, cap_dup=None, log=None):
    """Time every candidate launch shape on a step of `views`; returns
    {"best": {...}, "table": [...]} (times in ms, median of `reps`).

    `target` is the flat target image of the batch (the layout of
    Renderer.color); `vis` = (vis_s, vis_e) device tensors to start every
    candidate from the same temporal state.  The knobs are left at the best
    candidate's values (`apply(best)` sets them again later); `params`
    entries "tile" and "sort" of the best candidate are in best["params"]."""
    from .renderer import Renderer
    table = []
    ref_img = None
    old = A.get_tuning()
    default_fine = A.get_tuning()["fine_tiles"]

    def renderer(tile):
        r = Renderer(scene, views, dict(params, tile=int(tile)), device=device, cap_surv=cap_surv,
                     cap_dup=cap_dup)
        if vis is not None:
            r.vis_s.copy_(vis[0])
            r.vis_e.copy_(vis[1])
        c = r.fit_capacity()
        if c["spin"] or c["ovf_surv"] or c["ovf_dup"]:
            raise A.S3RError(f"capacities did not fit for tile {tile}: {c}")
        return r

    def measure(r, cand):
        nonlocal ref_img
        apply(cand)
        r.set_flags(sort=cand["sort"])
        r.forward()
        torch.cuda.synchronize()
        img = r.color.detach().cpu().numpy().copy()
        if ref_img is None:
            ref_img = img
        elif not np.array_equal(img, ref_img):
            raise A.S3RError(f"candidate {cand} renders a different image")
        t0 = time.perf_counter()
        ms = _time_step(r, target, reps)
        row = dict(cand, ms=ms, tuning_s=time.perf_counter() - t0)
        table.append(row)
        if log:
            log(f"autotune {cand}: {ms:.3f} ms/step")
        return row

    try:
        for tile in tiles:
            r = renderer(tile)
            for sort, waves, binned in itertools.product(sorts, raster_waves, binning):
                if sort == "global" and not binned:
                    continue  # the binning limit only matters to the tile sort
                measure(r, dict(tile=int(tile), sort=sort, raster_waves=int(waves),
                                binning=bool(binned), fine_tiles=default_fine))
            del r
            torch.cuda.empty_cache()
        best = min(table, key=lambda row: row["ms"])
        rest = [f for f in fine_tiles if f != default_fine]
        if rest:
            r = renderer(best["tile"])
            for f in rest:
                cand = {k: best[k] for k in ("tile", "sort", "raster_waves", "binning")}
                measure(r, dict(cand, fine_tiles=int(f)))
            del r
            torch.cuda.empty_cache()
    except Exception:
        A.set_tuning(**old)
        raise
    best = min(table, key=lambda row: row["ms"])
    best = dict(best, params=dict(params, tile=best["tile"], sort=best["sort"]))
    apply(best)
    return {"best": best, "table": table}


def apply(best):
    """Set the launch-shape knobs of an autotune result."""
    A.set_tuning(raster_waves=best["raster_waves"], bin_max_tiles=-1 if best["binning"] else 0,
                 fine_tiles=best.get("fine_tiles", -1))
