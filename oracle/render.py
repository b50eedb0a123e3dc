"""Per-view driver of the oracle: decisions (binary32), colours and blending (FP64).

render_view follows the per-view steps of Sec. 3.3 in the paper's order:
temporal selection, instance-specific projection, frustum test (M_t), LOD
cull, colour query for the survivors only, and alpha blending (Eq. 2).  The
decisions come from `decide32`; colours are FP64 SH of the instance-local
viewing direction; blending is FP64 on the binary32 projected attributes
(the same values the GPU rasterises).
"""

from __future__ import annotations

import numpy as np

from . import composite as comp
from . import decide32, frames, order, sh


def view_pixels(w, h, region=None):
    """Integer pixel coordinates of a whole view or of region (x0, y0, x1, y1)."""
    x0, y0, x1, y1 = (0, 0, w, h) if region is None else region
    ys, xs = np.mgrid[y0:y1, x0:x1]
    return xs.ravel().astype(np.float64), ys.ravel().astype(np.float64)


def survivor_colours(scene, d, ids):
    """FP64 colour of Gaussians `ids` from the direction mu - c_{t,i} in the
    instance-local frame (c_{t,i} the camera centre seen from instance i)."""
    cen = frames.camera_centre64(d["cam64"])            # (K+1, 3)
    k = scene.inst[ids]
    dv = scene.mean[ids].astype(np.float64) - cen[k]
    dv /= np.linalg.norm(dv, axis=1, keepdims=True)
    rgb, raw = sh.colour(scene.sh[ids].astype(np.float64), dv, scene.sh_degree)
    return rgb, raw, dv


def region_candidates(d, ids, region, params):
    """The survivors `ids` that can pass the Mahalanobis cut somewhere in
    region (x0, y0, x1, y1).  The others are skipped at every pixel of the
    region, so leaving them out changes nothing there:
    -power >= |d|^2 / (2 lam_max) > cutoff when |d|^2 > 2 cutoff lam_max."""
    if not ids.size:
        return ids
    x0, y0, x1, y1 = region
    uu = d["u"][ids].astype(np.float64)
    vv = d["v"][ids].astype(np.float64)
    ddx = np.maximum(0.0, np.maximum(x0 - uu, uu - (x1 - 1)))
    ddy = np.maximum(0.0, np.maximum(y0 - vv, vv - (y1 - 1)))
    lim = 2.0 * params["cutoff"] * d["lam_d"][ids].astype(np.float64) * 1.0001 + 1e-9
    return ids[ddx * ddx + ddy * ddy <= lim]


def render_view(scene, views, v, params, plain=False, region=None, with_image=True,
                delta=1e-4):
    W34, Kv, wh, tau = views.W[v], views.K[v], views.wh[v], int(views.tstep[v])
    d = decide32.project_cull32(scene, W34, Kv, wh, tau, params, plain=plain, view_index=v)
    ids = np.nonzero(d["surv"])[0]
    N = scene.n
    rgb = np.zeros((N, 3))
    rgb_s, raw_s, _ = survivor_colours(scene, d, ids)
    rgb[ids] = rgb_s
    out = dict(dec=d, ids=ids, rgb=rgb, rgb_raw=raw_s)
    if not with_image:
        return out
    w, h = int(wh[0]), int(wh[1])
    xs, ys = view_pixels(w, h, region)
    cand = ids if region is None else region_candidates(d, ids, region, params)
    ordr = order.global_order(cand, d["depth_bits"])
    conic = np.stack([d["conic_a"], d["conic_b"], d["conic_c"]], 1).astype(np.float64)
    C, T, ncon, flag = comp.composite(xs, ys, ordr, d["u"].astype(np.float64),
                                      d["v"].astype(np.float64), conic,
                                      scene.opacity.astype(np.float64), rgb, params, delta=delta)
    if region is None:
        out["image"] = C.T.reshape(3, h, w)
        out["T"] = T.reshape(h, w)
        out["ncon"] = ncon.reshape(h, w)
        out["flag"] = flag.reshape(h, w)
    else:
        rw, rh = region[2] - region[0], region[3] - region[1]
        out["image"] = C.T.reshape(3, rh, rw)
        out["T"] = T.reshape(rh, rw)
        out["ncon"] = ncon.reshape(rh, rw)
        out["flag"] = flag.reshape(rh, rw)
    out["order"] = ordr
    return out


def raster_visible(scene, views, v, params, plain=False):
    """Rendering-derived visibility of view v: the Gaussians blended into at
    least one pixel (one reading of the visibility that the Fig. 1 caption
    attributes to the rendering process), plus those whose status rests on a
    guard-band decision.  Returns (took, uncertain) as boolean (N,) arrays."""
    tr = {"took": set(), "uncertain": set()}
    W34, Kv, wh, tau = views.W[v], views.K[v], views.wh[v], int(views.tstep[v])
    d = decide32.project_cull32(scene, W34, Kv, wh, tau, params, plain=plain, view_index=v)
    ids = np.nonzero(d["surv"])[0]
    rgb = np.zeros((scene.n, 3))
    if ids.size:
        rgb[ids] = survivor_colours(scene, d, ids)[0]
    xs, ys = view_pixels(int(wh[0]), int(wh[1]))
    ordr = order.global_order(ids, d["depth_bits"])
    conic = np.stack([d["conic_a"], d["conic_b"], d["conic_c"]], 1).astype(np.float64)
    comp.composite(xs, ys, ordr, d["u"].astype(np.float64), d["v"].astype(np.float64), conic,
                   scene.opacity.astype(np.float64), rgb, params, track=tr)
    took = np.zeros(scene.n, bool)
    unc = np.zeros(scene.n, bool)
    took[list(tr["took"])] = True
    unc[list(tr["uncertain"])] = True
    return took, unc


def tile_lists_of(d, ids, params):
    """Per-tile contributor lists of one view's survivors (see `order`)."""
    return order.tile_lists(ids, d["depth_bits"], d["x0"], d["x1"], d["y0"], d["y1"],
                            d["gx"], d["gy"])
