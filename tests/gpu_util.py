"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and read its outputs back in the oracle's terms."""

from __future__ import annotations

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP device")


def banner(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def make_renderer(scene, views, params, plain=False, **kw):
    from paper_2503_08217_amd.renderer import Renderer
    r = Renderer(scene, views, params, plain=plain, **kw)
    c = r.fit_capacity()
    assert c["spin"] == 0 and c["ovf_surv"] == 0 and c["ovf_dup"] == 0, c
    return r


def check_view(scene, views, params, r, rec, v, plain=False, region=None, full_lists=True):
    """View v of the GPU batch in `r` (records `rec`) against the oracle:
    M_t, survivors, record fields and (optionally) the full tile lists bit
    for bit, colours within 1e-5, pixels of `region` (the whole view if None)
    by `check_pixels`.  Returns the oracle's output."""
    from oracle import render
    o = render.render_view(scene, views, v, params, plain=plain, region=region)
    d = o["dec"]
    gm = mask_bits(r)[v]
    np.testing.assert_array_equal(gm, d["visible"], err_msg=f"M_t view {v}")
    sel = rec["view"] == v
    gid = rec["gid"][sel]
    assert np.all(np.diff(gid) > 0), "records of a view must be in Gaussian order"
    np.testing.assert_array_equal(gid, np.nonzero(d["surv"])[0], err_msg=f"survivors view {v}")
    geo = rec["geo"][sel]
    np.testing.assert_array_equal(geo[:, 0].view(np.uint32), d["u"][gid].view(np.uint32))
    np.testing.assert_array_equal(geo[:, 1].view(np.uint32), d["v"][gid].view(np.uint32))
    np.testing.assert_array_equal(geo[:, 3].view(np.uint32), d["depth_bits"][gid])
    np.testing.assert_array_equal(geo[:, 2], scene.opacity[gid])
    rect = rec["rect"][sel]
    np.testing.assert_array_equal(rect[:, 0], d["x0"][gid])
    np.testing.assert_array_equal(rect[:, 1], d["y0"][gid])
    np.testing.assert_array_equal(rect[:, 2], d["x1"][gid])
    np.testing.assert_array_equal(rect[:, 3], d["y1"][gid])
    con = rec["conic"][sel][:, :3]
    ref = np.stack([d["conic_a"], d["conic_b"], d["conic_c"]], 1)[gid]
    np.testing.assert_array_equal(con.view(np.uint32), ref.view(np.uint32))
    np.testing.assert_allclose(rec["rgb"][sel][:, :3], o["rgb"][gid], atol=1e-5, rtol=0)
    st = rec["stats"][v]
    assert st[1] == d["visible"].sum() and st[2] == d["surv"].sum()
    if params.get("temporal"):
        assert st[0] == d["pass_t"].sum()
    if full_lists:
        a = render.tile_lists_of(d, np.nonzero(d["surv"])[0], params)
        g = tile_lists_gpu(r, rec)[v]
        np.testing.assert_array_equal(g[0], a[0])
        np.testing.assert_array_equal(g[1], a[1])
    img = image_np(r, v)
    T = T_np(r, v)
    if region is not None:
        x0, y0, x1, y1 = region
        img = img[:, y0:y1, x0:x1]
        T = T[y0:y1, x0:x1]
    check_pixels(o, img, T, params, float(scene.opacity.max()), tag=f"view {v}")
    return o


def poison_grads(r):
    """The backward writes every gradient entry: start from NaN so that an
    entry it skipped shows up."""
    for t in (r.g_mean, r.g_scale, r.g_quat, r.g_opacity, r.g_sh, r.g_pose, r.g_pose6,
              r.g_mean_w, r.g_rot_w):
        if t is not None:
            t.fill_(float("nan"))


def mask_bits(r):
    """(V, N) bool from the GPU M_t words."""
    m = r.mask.cpu().numpy().view(np.uint32)
    bits = np.unpackbits(m.view(np.uint8).reshape(r.V, -1), axis=1, bitorder="little")
    return bits[:, : r.n].astype(bool)


def records(r):
    """Dict of numpy arrays of the first n_surv records."""
    c = r.read_counters()
    n = c["n_surv"]
    return dict(
        n=n, counters=c,
        gid=r.rec_gid[:n].cpu().numpy(), view=r.rec_view[:n].cpu().numpy(),
        geo=r.rec_geo[:n].cpu().numpy(), conic=r.rec_conic[:n].cpu().numpy(),
        rgb=r.rec_rgb[:n].cpu().numpy(), rect=r.rec_rect[:n].cpu().numpy(),
        stats=r.stats.cpu().numpy())


def tile_lists_gpu(r, rec):
    """Per view: (tile_start local to the view, gid list) from the GPU bins."""
    ts = r.tile_start.cpu().numpy().astype(np.int64)
    vals = r.vals.cpu().numpy().view(np.uint32).astype(np.int64)
    out = []
    for v in range(r.V):
        a, b = int(r.toff_np[v]), int(r.toff_np[v + 1])
        st = ts[a:b + 1] - ts[a]
        ids = rec["gid"][vals[ts[a]:ts[b]]]
        out.append((st, ids))
    return out


def image_np(r, v):
    return r.image(v).cpu().numpy()


def T_np(r, v):
    return r.view_slice(r.T_final, v).cpu().numpy()


def compare_grads(g, ref, keys, rel=1e-3, tag=""):
    """GPU gradients `g` vs the oracle's `ref`, per tensor: normwise
    |a - b|_2 <= rel |b|_2, and element by element |a_i - b_i| <= rel (|b_i| +
    rms of the non-zero b), so that a few wrong entries cannot hide under the
    norm (the rms is taken over the entries that carry gradient: most rows
    of a scene belong to Gaussians no pixel sees).  Prints the normwise error
    and the 99th percentile of the relative error of the elements above 1%
    of the tensor's largest magnitude."""
    for k in keys:
        a = np.asarray(g[k], np.float64).ravel()
        b = np.asarray(ref[k], np.float64).ravel()
        assert np.all(np.isfinite(a)), (tag, k, "non-finite GPU gradient")
        nb = np.linalg.norm(b)
        err = np.linalg.norm(a - b)
        assert err <= rel * max(nb, 1e-12), (tag, k, "normwise", err, nb)
        rms = nb / np.sqrt(max(int(np.count_nonzero(b)), 1))
        ee = np.abs(a - b)
        bound = rel * (np.abs(b) + rms)
        bad = ee > bound + 1e-30
        assert not bad.any(), (tag, k, "elementwise", int(bad.sum()), int(np.argmax(ee - bound)),
                               float(ee.max()), float(rms))
        big = np.abs(b) > 0.01 * np.abs(b).max() if b.size and np.abs(b).max() > 0 else None
        p99 = float(np.percentile(ee[big] / np.abs(b[big]), 99)) if big is not None and big.any() \
            else 0.0
        banner(f"{tag} grad {k}: rel-norm {err / max(nb, 1e-12):.2e}, p99 rel {p99:.2e}")


def flagged_pixel_bound(params, opac_max, cmax):
    """Largest change of a pixel caused by binary32 and FP64 taking one
    blending decision differently (a decision in the guard band) plus one
    early stop: a flipped Mahalanobis cut or alpha_min skip changes one alpha
    by at most da = max(alpha_min, o_max exp(-cutoff)), which moves that
    Gaussian's term by <= da c_max T and every later term by a factor within
    da / (1 - da), <= 2 da / (1 - da) c_max in total; a flipped early stop
    drops or keeps the rest of the list, worth <= t_min (1 + 1e-4) c_max."""
    import math
    da = max(params["alpha_min"], opac_max * math.exp(-params["cutoff"]))
    return (2.0 * da / (1.0 - da) + params["t_min"] * (1.0 + 1e-4)) * cmax


def check_pixels(o, img, T, params, opac_max, tag=""):
    """Blended pixels and transmittance against the oracle output `o` of the
    same region: unflagged pixels within 1e-4 absolute, flagged ones within
    `flagged_pixel_bound` of the largest survivor colour (plus the
    background); returns the flagged count."""
    ok = ~o["flag"]
    err = np.abs(img - o["image"])
    assert err[:, ok].max(initial=0) <= 1e-4, (tag, err[:, ok].max())
    cmax = max(1e-6, float(o["rgb"].max()), float(np.max(params["bg"])))
    fb = flagged_pixel_bound(params, opac_max, cmax)
    assert err.max(initial=0) <= fb, (tag, err.max(), fb)
    assert np.abs(T - o["T"])[ok].max(initial=0) <= 1e-4, tag
    nflag = int(o["flag"].sum())
    banner(f"{tag} pixels: max err {err[:, ok].max(initial=0):.2e} unflagged, "
           f"{err.max(initial=0):.2e} overall (bound {fb:.3f}), flagged {nflag} of {ok.size}")
    return nflag


def gpu_region_grads(r, parts):
    """Backward of the GPU renderer's last forward with dL/dC = dC on the
    regions of `parts` [(view in batch, region, dC)] (summed where regions
    overlap) and zero elsewhere."""
    dc = torch.zeros(3 * r.total_px, device=r.dev, dtype=torch.float32)
    for v, (x0, y0, x1, y1), dC in parts:
        w, h = int(r.wh_np[v, 0]), int(r.wh_np[v, 1])
        o = int(r.poff_np[v])
        dc[3 * o: 3 * o + 3 * w * h].view(3, h, w)[:, y0:y1, x0:x1] += \
            torch.as_tensor(np.asarray(dC, np.float32), device=r.dev)
    poison_grads(r)
    r.raster_bwd(dc)
    torch.cuda.synchronize()
    g = dict(mean=r.g_mean, scale=r.g_scale, quat=r.g_quat, opacity=r.g_opacity, sh=r.g_sh,
             pose=r.g_pose.view(r.T, r.S, 3, 4), pose6=r.g_pose6)
    return {k: t.cpu().numpy().astype(np.float64) for k, t in g.items()}


def oracle_region_grads(scene, views, params, parts):
    """The oracle's FP64 gradients of sum <dC, image region> over `parts`
    [(view, region, dC)], each region over its candidates in blending order."""
    from oracle import grad as ograd
    from oracle import order, render
    op = []
    for v, reg, dC in parts:
        o = render.render_view(scene, views, v, params, with_image=False)
        cand = render.region_candidates(o["dec"], o["ids"], reg, params)
        op.append((v, reg, order.global_order(cand, o["dec"]["depth_bits"]), dC))
    return ograd.image_vjp(scene, views, params, op)
