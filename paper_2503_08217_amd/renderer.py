"""Device buffers and calls of the per-view rendering step (PyTorch for memory
and streams only; every step runs in libs3r.so).

`Renderer` owns the device copies of a scene and of a batch of views plus all
capacity-sized buffers, and exposes the C entry points one by one
(`project_cull`, `sort`, `raster_fwd`, `l1_loss`, `raster_bwd`,
`update_visibility`, `plain_transform`, `plain_transform_bwd`) and composed
(`forward`, `step`).  `RenderFn` wraps forward/backward as a
torch.autograd.Function.
"""

from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import _abi as A

# lists of this many entries or more take the per-tile sort's slow path
TILE_SORT_MAX = 16384


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def tile_layout(wh, tile):
    """Exclusive prefixes of tiles and pixels per view (host bookkeeping)."""
    wh = np.asarray(wh, np.int64).reshape(-1, 2)
    g = ((wh[:, 0] + tile - 1) // tile) * ((wh[:, 1] + tile - 1) // tile)
    toff = np.concatenate([[0], np.cumsum(g)]).astype(np.int32)
    poff = np.concatenate([[0], np.cumsum(wh[:, 0] * wh[:, 1])]).astype(np.int64)
    return toff, poff


class Renderer:
    def __init__(self, scene, views, params, *, device="cuda", plain=False, cap_surv=None,
                 cap_dup=None, requires_grad=False):
        A.load()
        self.dev = torch.device(device)
        self.params = dict(params)
        self._max_list = None  # longest tile list seen by fit_capacity
        self.plain = bool(plain)
        self.V = int(views.n_views)
        self.n = int(scene.mean.shape[0])
        self.T = int(scene.pose.shape[0])
        self.S = int(scene.pose.shape[1])
        self.sh_degree = int(scene.sh_degree)
        self.B = (self.sh_degree + 1) ** 2
        d = self.dev
        f32 = torch.float32

        def up(x, dt=f32):
            return torch.as_tensor(np.ascontiguousarray(x)).to(device=d, dtype=dt).contiguous()

        self.mean = up(scene.mean)
        self.scale = up(scene.scale)
        self.quat = up(scene.quat)
        self.opacity = up(scene.opacity)
        self.sh = up(scene.sh).reshape(self.n, self.B, 3)
        self.inst = up(scene.inst, torch.int32)
        self.vis_s = up(scene.vis_s)
        self.vis_e = up(scene.vis_e)
        self.life_s = up(scene.life_s)
        self.life_e = up(scene.life_e)
        self.pose = up(np.asarray(scene.pose).reshape(self.T, self.S, 12))
        self._fwd_gen = 0  # raster forwards so far (the backward replays the last one)
        self.set_views(views)
        self.cap_surv = int(cap_surv) if cap_surv else max(1, self.n * self.V)
        self.cap_dup = int(cap_dup) if cap_dup else max(1024, 4 * self.cap_surv)
        self._alloc()

    # ------------------------------------------------------------------ views
    def _upload_views(self, views):
        d = self.dev
        tile = int(self.params["tile"])
        vs = {}
        vs["wh_np"] = np.asarray(views.wh, np.int32).reshape(-1, 2)
        vs["tstep_np"] = np.asarray(views.tstep, np.int32)
        toff, poff = tile_layout(vs["wh_np"], tile)
        vs["toff_np"], vs["poff_np"] = toff, poff
        vs["total_tiles"] = int(toff[-1])
        vs["total_px"] = int(poff[-1])
        vs["W"] = torch.as_tensor(np.asarray(views.W, np.float32).reshape(-1, 12)).to(d).contiguous()
        vs["K"] = torch.as_tensor(np.asarray(views.K, np.float32).reshape(-1, 4)).to(d).contiguous()
        vs["wh"] = torch.as_tensor(vs["wh_np"]).to(d).contiguous()
        vs["tstep"] = torch.as_tensor(vs["tstep_np"]).to(d).contiguous()
        vs["tile_offset"] = torch.as_tensor(toff).to(d).contiguous()
        vs["px_offset"] = torch.as_tensor(poff).to(d).contiguous()
        ts = sorted(set(int(t) for t in vs["tstep_np"]))
        vs["plain_ts"] = np.asarray(ts, np.int32)
        slot = np.asarray([ts.index(int(t)) for t in vs["tstep_np"]], np.int32)
        vs["plain_slot"] = torch.as_tensor(slot).to(d).contiguous()
        vs["c_views"] = A.S3RViews(
            _ptr(vs["W"]), _ptr(vs["K"]), _ptr(vs["wh"]), _ptr(vs["tstep"]), _ptr(vs["tile_offset"]),
            _ptr(vs["px_offset"]), _ptr(vs["plain_slot"]), int(len(vs["wh_np"])), vs["total_tiles"],
            vs["total_px"])
        vs["c_ts"] = (C.c_int32 * len(ts))(*ts)
        return vs

    def _use(self, vs):
        self._vs = vs
        for k in ("wh_np", "tstep_np", "toff_np", "poff_np", "total_tiles", "total_px", "W", "K",
                  "wh", "tstep", "tile_offset", "px_offset", "plain_ts", "plain_slot", "c_views",
                  "c_ts"):
            setattr(self, k, vs[k])

    def set_views(self, views):
        self._use(self._upload_views(views))

    def prepare_views(self, view_sets):
        """Upload several batches of views (each no larger than the first one
        the buffers were sized for); returns handles for `use_views`."""
        out = []
        for views in view_sets:
            vs = self._upload_views(views)
            if (vs["total_tiles"] > self.total_tiles or vs["total_px"] > self.total_px
                    or len(vs["wh_np"]) != self.V or len(vs["plain_ts"]) > len(self.plain_ts)):
                raise ValueError("view set larger than the allocated buffers")
            out.append(vs)
        return out

    def use_views(self, handle):
        self._use(handle)

    # ---------------------------------------------------------------- buffers
    def _alloc(self):
        d, f32, i32 = self.dev, torch.float32, torch.int32
        V, S, n = self.V, self.S, self.n
        cs, cd = self.cap_surv, self.cap_dup
        self.mask_words = ((n + 63) // 64) * 2
        self.cam = torch.zeros(V, S, 12, device=d, dtype=f32)
        self.cen = torch.zeros(V, S, 4, device=d, dtype=f32)
        self.t_norm = torch.zeros(V, device=d, dtype=f32)
        self.mask = torch.zeros(V, self.mask_words, device=d, dtype=i32)
        self.rec_gid = torch.zeros(cs, device=d, dtype=i32)
        self.rec_view = torch.zeros(cs, device=d, dtype=i32)
        self.rec_geo = torch.zeros(cs, 4, device=d, dtype=f32)
        self.rec_conic = torch.zeros(cs, 4, device=d, dtype=f32)
        self.rec_rgb = torch.zeros(cs, 4, device=d, dtype=f32)
        self.rec_rect = torch.zeros(cs, 4, device=d, dtype=i32)
        self.counters = torch.zeros(16, device=d, dtype=i32)
        self.stats = torch.zeros(V, 4, device=d, dtype=i32)
        self.rec_npairs = torch.zeros(cs, device=d, dtype=i32)
        self.surv = torch.zeros(V, self.mask_words, device=d, dtype=i32)
        self.bstat = torch.zeros((n + 255) // 256 * V * A.BSTAT + 4, device=d, dtype=i32)
        self.tile_count = torch.zeros(self.total_tiles, device=d, dtype=i32)
        self.tile_start = torch.zeros(self.total_tiles + 1, device=d, dtype=i32)
        self.tile_order = torch.zeros(max(1, self.total_tiles), device=d, dtype=i32)
        self.vals = torch.zeros(cd, device=d, dtype=i32)
        self.rec_pair = torch.zeros(cs + 1, device=d, dtype=i32)
        self.color = torch.zeros(3 * self.total_px, device=d, dtype=f32)
        self.T_final = torch.zeros(self.total_px, device=d, dtype=f32)
        self.last = torch.zeros(self.total_px, device=d, dtype=i32)
        # optional rendering-derived visibility (Gaussians blended into a pixel)
        if self.params.get("raster_mask", False):
            self.m_raster = torch.zeros(V, self.mask_words, device=d, dtype=i32)
            self.rec_taken = torch.zeros(max(1, cs), device=d, dtype=i32)
        else:
            self.m_raster = self.rec_taken = None
        self.census = torch.zeros(2, device=d, dtype=torch.int64)
        self.d_color = torch.zeros(3 * self.total_px, device=d, dtype=f32)
        self.loss_v = torch.zeros(max(V, 4), device=d, dtype=f32)
        n_ts = len(self.plain_ts)
        if self.plain:
            self.mean_w = torch.zeros(n_ts, n, 3, device=d, dtype=f32)
            self.rot_w = torch.zeros(n_ts, n, 9, device=d, dtype=f32)
        else:
            self.mean_w = self.rot_w = None
        # gradients
        self.g_mean = torch.zeros(n, 3, device=d, dtype=f32)
        self.g_scale = torch.zeros(n, 3, device=d, dtype=f32)
        self.g_quat = torch.zeros(n, 4, device=d, dtype=f32)
        self.g_opacity = torch.zeros(n, device=d, dtype=f32)
        self.g_sh = torch.zeros(n, self.B, 3, device=d, dtype=f32)
        self.g_pose = torch.zeros(self.T, S, 12, device=d, dtype=f32)
        self.g_pose6 = torch.zeros(self.T, S, 6, device=d, dtype=f32)
        # rows written by the last backward (sparse gradient mode)
        self.g_rows = torch.zeros(max(1, cs), device=d, dtype=i32)
        self.g_n_rows = torch.zeros(4, device=d, dtype=i32)
        if self.plain:
            self.g_mean_w = torch.zeros(n_ts, n, 3, device=d, dtype=f32)
            self.g_rot_w = torch.zeros(n_ts, n, 9, device=d, dtype=f32)
        else:
            self.g_mean_w = self.g_rot_w = None
        # workspaces
        lib = A.load()
        z = A.S3RSizes(n, V, self.total_tiles, cs, cd, S, 0)
        self.ws = {}
        for which in (A.S3R_WS_PROJECT, A.S3R_WS_SORT, A.S3R_WS_BACKWARD):
            nb = C.c_size_t(0)
            A.check(lib.s3r_workspace_size(C.byref(z), which, C.byref(nb)), "s3r_workspace_size")
            self.ws[which] = (torch.zeros(max(256, nb.value), device=d, dtype=torch.uint8),
                              nb.value)
        self._build_structs()

    def _build_structs(self):
        self.c_params = self.make_params()
        self.c_scene = A.S3RScene(
            _ptr(self.mean), _ptr(self.scale), _ptr(self.quat), _ptr(self.opacity), _ptr(self.sh),
            _ptr(self.inst), _ptr(self.vis_s), _ptr(self.vis_e), _ptr(self.pose), _ptr(self.mean_w),
            _ptr(self.rot_w), self.n, self.sh_degree, self.S, self.T, 0)
        self.c_proj = A.S3RProjected(
            _ptr(self.cam), _ptr(self.cen), _ptr(self.t_norm), _ptr(self.mask), _ptr(self.rec_gid),
            _ptr(self.rec_view), _ptr(self.rec_geo), _ptr(self.rec_conic), _ptr(self.rec_rgb),
            _ptr(self.rec_rect), _ptr(self.counters), _ptr(self.stats), _ptr(self.rec_npairs),
            _ptr(self.surv), _ptr(self.bstat), _ptr(self.rec_pair))
        self.c_bins = A.S3RBins(_ptr(self.tile_count), _ptr(self.tile_start), _ptr(self.vals),
                                _ptr(self.tile_order))
        self.c_img = A.S3RImage(_ptr(self.color), _ptr(self.T_final), _ptr(self.last),
                                _ptr(self.m_raster), _ptr(self.rec_taken), self.n, None)
        self.c_img_census = A.S3RImage(_ptr(self.color), _ptr(self.T_final), _ptr(self.last),
                                       _ptr(self.m_raster), _ptr(self.rec_taken), self.n,
                                       _ptr(self.census))
        self.c_grads = A.S3RGrads(
            _ptr(self.g_mean), _ptr(self.g_scale), _ptr(self.g_quat), _ptr(self.g_opacity),
            _ptr(self.g_sh), _ptr(self.g_pose), _ptr(self.g_pose6), _ptr(self.g_mean_w),
            _ptr(self.g_rot_w), _ptr(self.g_rows), _ptr(self.g_n_rows))

    def make_params(self):
        p = self.params
        flags = 0
        if p.get("temporal", False):
            flags |= A.S3R_TEMPORAL
        if p.get("lod", False):
            flags |= A.S3R_LOD
        if self.plain:
            flags |= A.S3R_PLAIN
        if p.get("lod_stochastic", False):
            flags |= A.S3R_LOD_STOCHASTIC
        if p.get("grad_sparse", False):
            flags |= A.S3R_GRAD_SPARSE
        if p.get("deterministic", False):
            flags |= A.S3R_DETERMINISTIC_GRADS
        # sort mode: "tiles" (tile partition + per-list depth sort) is fastest
        # while lists stay short; "auto" takes it when every list seen by the
        # last capacity fit held fewer than TILE_SORT_MAX entries
        sort = p.get("sort") or "auto"
        if sort not in ("tiles", "global", "auto"):
            raise ValueError(f"sort must be 'tiles', 'global' or 'auto', not {sort!r}")
        if sort == "auto":
            sort = "tiles" if (self._max_list is not None and
                               self._max_list < TILE_SORT_MAX) else "global"
        if sort == "tiles":
            flags |= A.S3R_SORT_TILES
        bg = (C.c_float * 3)(*[float(x) for x in p["bg"]])
        return A.S3RParams(int(p["tile"]), flags, float(p["lod_r"]), float(p["z_near"]),
                           float(p["z_far"]), float(p["eps2d"]), float(p["alpha_min"]),
                           float(p["alpha_max"]), float(p["t_min"]), float(p["cutoff"]),
                           float(p["jac_clamp"]), bg, self.cap_surv, self.cap_dup,
                           int(p.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF,
                           float(p.get("lod_pmax", 1.0)), float(p.get("lod_D", 1.0)),
                           int(p.get("step", 0)) & 0xFFFFFFFF, 0)

    def set_flags(self, **over):
        """Change parameters; the longest list seen so far is forgotten (the
        next fit_capacity measures it again for the "auto" sort mode)."""
        self.params.update(over)
        self._max_list = None
        self.c_params = self.make_params()

    # ------------------------------------------------------------ entry points
    def plain_transform(self):
        A.check(A.load().s3r_plain_transform(C.byref(self.c_scene), self.c_ts, len(self.plain_ts),
                                             _ptr(self.mean_w), _ptr(self.rot_w), _stream()),
                "s3r_plain_transform")

    def project_cull(self):
        ws, nb = self.ws[A.S3R_WS_PROJECT]
        A.check(A.load().s3r_project_cull(C.byref(self.c_scene), C.byref(self.c_views),
                                          C.byref(self.c_params), C.byref(self.c_proj), _ptr(ws),
                                          nb, _stream()), "s3r_project_cull")

    def project_cull_noalloc(self):
        """s3r_project_cull with the library's fixed scratch instead of a
        workspace (no device allocation in the call)."""
        A.check(A.load().s3r_project_cull_noalloc(C.byref(self.c_scene), C.byref(self.c_views),
                                                  C.byref(self.c_params), C.byref(self.c_proj),
                                                  _stream()), "s3r_project_cull_noalloc")

    def sort(self):
        ws, nb = self.ws[A.S3R_WS_SORT]
        A.check(A.load().s3r_sort(C.byref(self.c_scene), C.byref(self.c_proj), C.byref(self.c_views),
                                  C.byref(self.c_params), C.byref(self.c_bins), _ptr(ws), nb,
                                  _stream()), "s3r_sort")

    def raster_fwd(self, census=False):
        """Eq. (2) for every view.  With census=True the call also adds its
        evaluated and blended (pixel, entry) pair counts to `self.census`."""
        self._fwd_gen += 1
        img = self.c_img_census if census else self.c_img
        A.check(A.load().s3r_raster_fwd(C.byref(self.c_proj), C.byref(self.c_bins),
                                        C.byref(self.c_views), C.byref(self.c_params),
                                        C.byref(img), _stream()), "s3r_raster_fwd")

    def work_census(self):
        """Forward of the current batch with the work census: returns the
        (pixel, entry) pairs evaluated (cutoff box met, pixel still blending)
        and blended, summed over the batch.  The census is taken with every
        tile in 8x8 sub-tiles (the raster backward's decomposition), so the
        evaluated count does not depend on S3R_TUNE_FINE_TILES."""
        self.census.zero_()
        if self.plain:
            self.plain_transform()
        self.project_cull()
        self.sort()
        old = A.set_tuning(fine_tiles=0)
        try:
            self.raster_fwd(census=True)
        finally:
            A.set_tuning(**old)
        c = self.census.cpu().numpy()
        return dict(evaluated=int(c[0]), blended=int(c[1]))

    def l1_loss(self, target):
        A.check(A.load().s3r_l1_loss(C.byref(self.c_img), _ptr(target), C.byref(self.c_views),
                                     _ptr(self.loss_v), _ptr(self.d_color), _stream()),
                "s3r_l1_loss")

    def zero_grads(self):
        """Clear every gradient array and the sparse-mode row list.  The
        backward writes the gradients itself; this is only for starting over
        (and required once before the first sparse-mode backward)."""
        for t in (self.g_mean, self.g_scale, self.g_quat, self.g_opacity, self.g_sh, self.g_pose,
                  self.g_pose6, self.g_mean_w, self.g_rot_w, self.g_n_rows):
            if t is not None:
                t.zero_()

    def raster_bwd(self, d_color=None):
        dc = self.d_color if d_color is None else d_color
        ws, nb = self.ws[A.S3R_WS_BACKWARD]
        A.check(A.load().s3r_raster_bwd(C.byref(self.c_scene), C.byref(self.c_views),
                                        C.byref(self.c_params), C.byref(self.c_proj),
                                        C.byref(self.c_bins), C.byref(self.c_img), _ptr(dc),
                                        C.byref(self.c_grads), _ptr(ws), nb, _stream()),
                "s3r_raster_bwd")
        if self.plain:
            A.check(A.load().s3r_plain_transform_bwd(C.byref(self.c_scene), self.c_ts,
                                                     len(self.plain_ts), C.byref(self.c_grads),
                                                     _stream()), "s3r_plain_transform_bwd")

    def update_visibility(self, mode, margin=None, source=None):
        """Eqs. (5)-(6).  The UPDATE uses the frustum mask M_t, or with
        source="raster" the rendering-derived one of the last forward."""
        m = float(self.params.get("margin", 0.1) if margin is None else margin)
        src = source or self.params.get("visibility_source", "frustum")
        mask = self.m_raster if src == "raster" else self.mask
        if mask is None:
            raise ValueError("rendering-derived visibility needs raster_mask=True")
        A.check(A.load().s3r_update_visibility(
            _ptr(self.life_s), _ptr(self.life_e), _ptr(self.vis_s), _ptr(self.vis_e),
            _ptr(mask), _ptr(self.t_norm), self.V, self.n, int(mode), m, _stream()),
            "s3r_update_visibility")

    # --------------------------------------------------------------- composed
    def forward(self):
        if self.plain:
            self.plain_transform()
        self.project_cull()
        self.sort()
        self.raster_fwd()

    def step(self, target, update_visibility=True):
        """One training step of the batch: forward, L1 loss, backward and
        point-life update (Eq. 5)."""
        self.forward()
        self.l1_loss(target)
        self.raster_bwd()
        if update_visibility and not self.plain:
            self.update_visibility(A.S3R_VIS_UPDATE)

    def capture_step(self, target, update_visibility=True):
        """Record one whole `step` (forward, loss, backward, point-life update)
        into a HIP graph; `graph.replay()` then runs it with one launch.  The
        library records only kernel nodes (its buffers are zeroed by fill
        kernels, never memset nodes) and allocates nothing, so the captured
        step reuses this renderer's buffers on every replay."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.step(target, update_visibility)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            self.step(target, update_visibility)
        torch.cuda.synchronize()
        return graph

    @classmethod
    def autotuned(cls, scene, views, params, target, *, vis=None, **kw):
        """A renderer of `views` with the tile size, sort mode and launch
        shapes that ran one training step fastest (autotune.autotune; every
        candidate must render the same image).  Returns (renderer, result)."""
        from .autotune import autotune
        res = autotune(scene, views, params, target, vis=vis, **kw)
        r = cls(scene, views, res["best"]["params"], device=kw.get("device", "cuda"),
                cap_surv=kw.get("cap_surv"), cap_dup=kw.get("cap_dup"))
        if vis is not None:
            r.vis_s.copy_(vis[0])
            r.vis_e.copy_(vis[1])
        r.fit_capacity()
        return r, res

    # ---------------------------------------------------------------- helpers
    def parameters(self):
        """The scene parameters as the renderer's own device tensors, in the
        argument order of `RenderFn` / `render` (mean, scale, quat, opacity,
        sh, pose).  They alias the buffers the library reads, so an
        optimiser step on them changes what the next forward renders."""
        return (self.mean, self.scale, self.quat, self.opacity, self.sh, self.pose)

    def read_counters(self):
        torch.cuda.synchronize()
        c = self.counters.cpu().numpy()
        return dict(n_surv=int(c[A.CNT_SURV]), ovf_surv=int(c[A.CNT_OVF_SURV]),
                    n_dup=int(c[A.CNT_DUP]), ovf_dup=int(c[A.CNT_OVF_DUP]),
                    spin=int(c[A.CNT_SPIN]))

    def fit_capacity(self, margin=1.25):
        """Run the forward once and grow the capacities until nothing overflows."""
        for _ in range(8):
            self.forward()
            c = self.read_counters()
            if c["spin"]:
                raise A.S3RError("a bounded device wait gave up")
            need_s = c["n_surv"] + c["ovf_surv"]
            need_d = c["n_dup"] + c["ovf_dup"]
            if c["ovf_surv"] == 0 and c["ovf_dup"] == 0:
                longest = int(self.tile_count[: self.total_tiles].max().item())
                self._max_list = max(self._max_list or 0, longest)
                c["max_list"] = longest
                self.c_params = self.make_params()
                return c
            self.cap_surv = max(self.cap_surv, int(math.ceil(need_s * margin)) + 1024)
            self.cap_dup = max(self.cap_dup, int(math.ceil(need_d * margin)) + 4096)
            self._alloc()
        raise A.S3RError("capacities did not converge")

    def image(self, v):
        """(3, h, w) view of the colour buffer for view v."""
        w, h = int(self.wh_np[v, 0]), int(self.wh_np[v, 1])
        o = int(self.poff_np[v])
        return self.color[3 * o: 3 * o + 3 * w * h].view(3, h, w)

    def view_slice(self, buf, v, channels=1):
        w, h = int(self.wh_np[v, 0]), int(self.wh_np[v, 1])
        o = int(self.poff_np[v])
        return buf[channels * o: channels * (o + w * h)].view(*(() if channels == 1 else (channels,)), h, w)


class RenderFn(torch.autograd.Function):
    """Images of every view of `renderer` (its colour buffer, planar per view)
    as a function of the scene parameters.

    The library reads the parameters from the renderer's own buffers, so the
    tensors passed in must be exactly those (`Renderer.parameters()`); they
    are passed so that autograd tracks them.  The backward replays the
    forward from its stored final transmittance and last contributors, so it
    must follow its own forward: a backward after another raster forward of
    the same renderer raises instead of returning gradients of the wrong
    image."""

    @staticmethod
    def forward(ctx, renderer, mean, scale, quat, opacity, sh, pose):
        for mine, given, name in zip(renderer.parameters(), (mean, scale, quat, opacity, sh, pose),
                                     ("mean", "scale", "quat", "opacity", "sh", "pose")):
            if given.data_ptr() != mine.data_ptr() or given.shape != mine.shape:
                raise ValueError(f"RenderFn: `{name}` is not the renderer's own {name} buffer")
        renderer.forward()
        ctx.renderer = renderer
        ctx.gen = renderer._fwd_gen
        return renderer.color.clone()

    @staticmethod
    def backward(ctx, d_color):
        r = ctx.renderer
        if r._fwd_gen != ctx.gen:
            raise RuntimeError("RenderFn.backward: the renderer ran another forward since this "
                               "image was rendered; its stored transmittance belongs to that one")
        r.raster_bwd(d_color.contiguous())
        return (None, r.g_mean.clone(), r.g_scale.clone(), r.g_quat.clone(),
                r.g_opacity.clone(), r.g_sh.clone(), r.g_pose.view(r.T, r.S, 12).clone())


def render(renderer, *params):
    """`RenderFn.apply(renderer, *params)`: the differentiable image of the
    renderer's views (params default to `renderer.parameters()`)."""
    return RenderFn.apply(renderer, *(params or renderer.parameters()))
