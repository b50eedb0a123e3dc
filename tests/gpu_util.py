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
