/*
 * s3r.h -- C ABI of the MI355X (gfx950) per-view Gaussian rendering library
 * for streamlined street-scene reconstruction (S3R-GS, arXiv 2503.08217).
 *
 * One call of each entry point processes a batch of V views (V >= 1, possibly
 * of different sizes and timesteps).  The steps follow Sec. 3.3 of the paper:
 * temporal-visibility selection, instance-specific projection, frustum test
 * giving the visible mask M_t, adaptive-LOD cull, colour query of the
 * survivors, alpha blending (Eq. 2) and the point-life / temporal-visibility
 * update (Eqs. 5-6); plus the backward pass of the blending and projection.
 * The conventional pipeline the paper compares against (Sec. 3.1: transform
 * every instance Gaussian to the world frame, then project everything) is
 * available as the "plain" route through s3r_plain_transform and the
 * S3R_PLAIN flag, sharing every other kernel.
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Struct arguments are host memory, read during the call, not retained.
 *    Every array they point to is DEVICE memory owned by the caller.
 *  - The library never allocates, frees or synchronises; it enqueues kernels on
 *    the caller's `stream` (a hipStream_t passed as void*; NULL = default
 *    stream) and returns.  All calls can be captured in a hipGraph.
 *  - Float arrays are IEEE binary32; every array must be 16-byte aligned
 *    (S3R_E_ALIGN otherwise).
 *  - Return value: S3R_OK (0) or a negative S3R_E_* code; no exception
 *    crosses the ABI.  s3r_status_string() names a code.  Errors detected on
 *    the host leave all outputs untouched.
 *  - Data-dependent sizes (survivor count, number of (tile, Gaussian) pairs)
 *    stay on the device.  If they exceed the capacities in S3RParams the
 *    device sets an overflow counter (S3RProjected.counters[S3R_CNT_OVF_*]),
 *    drops the excess consistently and the caller re-runs with larger buffers.
 *
 * Gaussian layout (structure of arrays, N Gaussians, static ones first, each
 * instance's Gaussians contiguous):
 *   mean[N][3]      position, instance-local for instance Gaussians
 *   scale[N][3]     per-axis standard deviation (activated)
 *   quat[N][4]      rotation quaternion (w, x, y, z), need not be normalised
 *   opacity[N]      in (0, 1) (activated)
 *   sh[N][B][3]     real SH coefficients, B = (L+1)^2, L = sh_degree <= 3
 *   inst[N]         0 = static, k in 1..S-1 = instance k
 *   vis_s[N], vis_e[N]   temporal visibility interval
 *   pose[T][S][12]  row-major 3x4 local->world pose of slot k at timestep tau
 *                   (slot 0 must be the identity)
 * Views (V views):
 *   W[V][12]        row-major 3x4 world->camera extrinsic (OpenCV axes)
 *   K[V][4]         fx, fy, cx, cy; pixel (x, y) is sampled at integer (x, y)
 *   wh[V][2]        width, height
 *   tstep[V]        timestep index tau in [0, T)
 *   tile_offset[V+1]  exclusive prefix of tiles per view, gx*gy with
 *                     gx = ceil(w/tile), gy = ceil(h/tile)
 *   px_offset[V+1]    exclusive prefix of w*h
 */
#ifndef S3R_H
#define S3R_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define S3R_ABI_VERSION 2


enum {
  S3R_OK = 0,
  S3R_E_NULL = -1,      /* a required pointer is NULL                     */
  S3R_E_ALIGN = -2,     /* a pointer is not 16-byte aligned               */
  S3R_E_SIZE = -3,      /* a size is out of range (n, views, degree, tile) */
  S3R_E_WORKSPACE = -4, /* workspace smaller than s3r_workspace_size()    */
  S3R_E_HIP = -5,       /* a kernel launch failed                          */
  S3R_E_ARG = -6,       /* an argument value is invalid                    */
  S3R_E_SCRATCH = -7    /* the problem needs more than the fixed scratch of
                           s3r_project_cull_noalloc                         */
};

/* S3RParams.flags */
enum {
  S3R_TEMPORAL = 1, /* apply the temporal-visibility test (Sec. 3.3)       */
  S3R_LOD = 2,      /* apply the LOD cull with threshold lod_r (Sec. 3.3)  */
  S3R_PLAIN = 4,    /* project the world-frame arrays of s3r_plain_transform
                       with the view camera (conventional route, Sec. 3.1) */
  S3R_LOD_STOCHASTIC = 8, /* Eq. (7): drop a sub-threshold Gaussian with
                       probability p = p_max + (p_max - 0.01) min(0, (d - D)/D)
                       instead of always (needs S3R_LOD)                   */
  S3R_GRAD_SPARSE = 16, /* s3r_raster_bwd clears only the gradient rows it
                       wrote on the previous call (S3RGrads.rows) instead of
                       the whole arrays; streamlined route only            */
  S3R_SORT_TILES = 32, /* s3r_sort bins the pairs by tile (or partitions them
                       by radix passes over the tile bits) and orders each
                       list by depth in registers / LDS: fastest when lists
                       are short (a few thousand entries, as with the LOD
                       cull); lists of 16384 entries or more take a slow
                       one-workgroup path.  Without the flag a radix sort over
                       all key bits orders every list, whatever its length.
                       Both give the same order.                            */
  S3R_DETERMINISTIC_GRADS = 64 /* s3r_raster_bwd sums every gradient in a fixed
                       order (per-wave window copies added in wave order,
                       per-record slot sums in emission order with no
                       atomics, camera gradients in 2^-32 fixed point), so two
                       calls on the same inputs give bitwise equal gradients;
                       slower.  Streamlined route only (with S3R_PLAIN:
                       S3R_E_ARG).                                          */
};

/* modes of s3r_update_visibility */
enum { S3R_VIS_UPDATE = 0, S3R_VIS_FOLD = 1, S3R_VIS_RESET = 2 };

/* indices into S3RProjected.counters (device int32[16]) */
enum {
  S3R_CNT_SURV = 0,     /* number of survivor records written            */
  S3R_CNT_OVF_SURV = 1, /* survivors dropped for lack of capacity        */
  S3R_CNT_DUP = 2,      /* number of (tile, record) pairs                 */
  S3R_CNT_OVF_DUP = 3,  /* pairs dropped for lack of capacity             */
  S3R_CNT_SPIN = 4,     /* reserved, always 0: no kernel waits on another
                           workgroup                                        */
  S3R_CNT_TICKET = 5,   /* reserved                                        */
  S3R_CNT_TICKET2 = 6,  /* reserved                                        */
  S3R_CNT_PAIRS = 7     /* (tile, record) pairs of every survivor, before the
                           capacities (saturates at 2^31 - 1)               */
};

typedef struct S3RParams {
  int32_t tile;       /* tile edge in pixels: 8, 16 or 32                   */
  uint32_t flags;     /* S3R_TEMPORAL | S3R_LOD | S3R_PLAIN                 */
  float lod_r;        /* LOD threshold r in pixels (Sec. 3.3, "Adaptive LOD") */
  float z_near, z_far;
  float eps2d;        /* low-pass added to the 2D covariance (px^2)         */
  float alpha_min, alpha_max, t_min; /* skip (> 0), clamp (in (0, 1)), stop (> 0) */
  float cutoff;       /* skip where the Mahalanobis power is below -cutoff  */
  float jac_clamp;    /* EWA Jacobian clamp, multiple of the half FOV tangent */
  float bg[3];        /* background colour                                  */
  int64_t cap_surv;   /* capacity of the survivor-record arrays             */
  int64_t cap_dup;    /* capacity of the (tile, record) pair arrays         */
  /* stochastic LOD drop (S3R_LOD_STOCHASTIC): the draw of Gaussian i in view v
     is Philox4x32-10 with counter (i, v, step, 0) and key (seed low, seed
     high); u = (first word >> 8) 2^-24 and the Gaussian is dropped if u < p */
  uint64_t seed;
  float lod_pmax;     /* p_max of Eq. (7)                                   */
  float lod_D;        /* D of Eq. (7), camera-space depth                   */
  uint32_t step;      /* training-step counter of the draw                  */
  uint32_t pad_;
} S3RParams;

typedef struct S3RScene {
  const float* mean;
  const float* scale;
  const float* quat;
  const float* opacity;
  const float* sh;
  const int32_t* inst;
  const float* vis_s;
  const float* vis_e;
  const float* pose;
  /* plain route only (S3R_PLAIN): world-frame arrays written by
     s3r_plain_transform, [n_plain_slots][N][3] and [n_plain_slots][N][9]   */
  const float* mean_w;
  const float* rot_w;
  int64_t n;          /* number of Gaussians, < 2^31                        */
  int32_t sh_degree;  /* 0..3                                               */
  int32_t n_slots;    /* S = number of instances + 1                        */
  int32_t n_timesteps;/* T                                                  */
  int32_t pad_;
} S3RScene;

typedef struct S3RViews {
  const float* W;
  const float* K;
  const int32_t* wh;
  const int32_t* tstep;
  const int32_t* tile_offset;
  const int64_t* px_offset;
  const int32_t* plain_slot; /* [V] world-frame array slot of each view (plain route) */
  int32_t n_views;           /* 1..64                                              */
  int32_t total_tiles;       /* tile_offset[V], host copy                          */
  int64_t total_px;          /* px_offset[V], host copy                            */
} S3RViews;

typedef struct S3RProjected {
  /* written by s3r_project_cull */
  float* cam;         /* [V][S][12] instance cameras P = W G, binary32        */
  float* cen;         /* [V][S][4]  camera centre seen from each slot's frame */
  float* t_norm;      /* [V] normalised rendering time in [-1, 1]             */
  uint32_t* mask;     /* [V][ceil(N/64)*2] bit i of view v = M_t[i]           */
  int32_t* rec_gid;   /* [cap_surv] Gaussian index of each survivor record    */
  int32_t* rec_view;  /* [cap_surv] view of each record                       */
  float* rec_geo;     /* [cap_surv][4] u, v, opacity, depth                   */
  float* rec_conic;   /* [cap_surv][4] inverse 2D covariance A, B, C, and the
                         x half-width of the box that holds the pixels which
                         can pass the Mahalanobis cut (3e38: unbounded)     */
  float* rec_rgb;     /* [cap_surv][4] r, g, b, and that box's y half-width   */
  int32_t* rec_rect;  /* [cap_surv][4] tile rect x0, y0, x1, y1 (view-local)  */
  int32_t* counters;  /* [16] see S3R_CNT_*                                   */
  int32_t* stats;     /* [V][4] N_t (temporal pass), N_f (= |M_t|), N_r (records),
                         N_dup (pairs, written by s3r_sort)                     */
  int32_t* rec_npairs;/* [cap_surv] number of tiles each record covers          */
  uint32_t* surv;     /* [V][ceil(N/64)*2] bit i of view v: Gaussian i has a record
                         (M_t and kept by the LOD test); same layout as mask     */
  int32_t* bstat;     /* [ceil(N/256)][V][8] per block of 256 Gaussians and view:
                         temporal passes, M_t count, records, first record,
                         (tile, record) pairs, first pair, 2 unused.  The
                         records of a batch are ordered by (block, view, Gaussian);
                         s3r_raster_bwd uses this to find each Gaussian's records */
  int32_t* rec_pair;  /* [cap_surv] index of each record's first (record, tile)
                         pair in emission order: a record emits the tiles of
                         its rectangle row by row, records in record order, so
                         the pair of record r and tile (tx, ty) is rec_pair[r] +
                         (ty - y0) (x1 - x0) + (tx - x0).  s3r_sort bins the
                         pairs by it and s3r_raster_bwd gives every pair its
                         own gradient slot by it */
} S3RProjected;

typedef struct S3RBins {
  int32_t* tile_count; /* [total_tiles] number of records covering each tile */
  int32_t* tile_start; /* [total_tiles+1] start of each tile's list          */
  uint32_t* vals;      /* [cap_dup] record index of each list entry, sorted  */
  int32_t* tile_order; /* [total_tiles] tiles by descending list length (the
                          rasterizer's launch order; ties in tile order)      */
} S3RBins;

typedef struct S3RImage {
  float* color;   /* per view v: [3][h][w] planar at offset 3*px_offset[v]   */
  float* T_final; /* [total_px] transmittance after the last contributor     */
  int32_t* last;  /* [total_px] 1 + list position of the last contributor    */
  /* optional rendering-derived visibility (NULL m_raster: not produced): bit i
     of view v is set when Gaussian i was blended into at least one pixel of
     view v -- a second reading of the visibility the rendering process gives
     (Sec. 3.3), usable as the `mask` of s3r_update_visibility.  rec_taken is
     per-record scratch [cap_surv]; n is the scene's N (sizes m_raster). */
  uint32_t* m_raster; /* [V][ceil(N/64)*2], layout of S3RProjected.mask     */
  int32_t* rec_taken;
  int64_t n;
  /* optional work census (NULL: not counted), two device counters that
     s3r_raster_fwd adds to (the caller clears them): [0] the evaluated
     (pixel, list entry) pairs -- a pixel still blending and an entry whose
     Mahalanobis cutoff box meets the pixel's 8x8 sub-tile, so Eq. (2)'s
     exponent is computed -- and [1] the blended ones (the entry contributed
     to the pixel).  One atomic per wave and counter: for measurement runs. */
  uint64_t* census;
} S3RImage;

typedef struct S3RGrads {
  /* written (=) by s3r_raster_bwd: every entry, zero where a Gaussian has no
     record, so the caller never zeroes them; `pose` is zeroed, then summed */
  float* mean;    /* [N][3] */
  float* scale;   /* [N][3] */
  float* quat;    /* [N][4] */
  float* opacity; /* [N]    */
  float* sh;      /* [N][B][3] */
  float* pose;    /* [T][S][12] dL/d(3x4 pose); slot 0 left untouched        */
  float* pose6;   /* [T][S][6]  right-perturbation (rho, omega) form of `pose`,
                     overwritten from the accumulated `pose` (optional, may be NULL) */
  /* plain route only: world-frame gradients, [n_plain_slots][N][3] / [..][9] */
  float* mean_w;
  float* rot_w;
  /* S3R_GRAD_SPARSE only: rows[0 .. *n_rows) lists Gaussians whose rows of
     mean / scale / quat / opacity / sh may be nonzero (written by the
     previous call; entries of -1 are ignored).  A call clears those rows,
     writes its own, and replaces the list: one entry per record, the
     Gaussian for the record that is its Gaussian's first in the batch, -1
     for the others.  Before the first
     call the caller zeroes the arrays once and sets *n_rows = 0; between
     calls it must not write the arrays.  [cap_surv] and [1], device. */
  int32_t* rows;
  int32_t* n_rows;
} S3RGrads;

/* Sizes used to plan workspaces. */
typedef struct S3RSizes {
  int64_t n;
  int32_t n_views;
  int32_t total_tiles;
  int64_t cap_surv;
  int64_t cap_dup;
  int32_t n_slots;
  int32_t pad_;
} S3RSizes;

enum { S3R_WS_PROJECT = 0, S3R_WS_SORT = 1, S3R_WS_BACKWARD = 2 };

/* Bytes of device workspace entry point `which` needs (S3R_WS_*). */
int s3r_workspace_size(const S3RSizes* sizes, int32_t which, size_t* bytes);

/*
 * s3r_project_cull -- Sec. 3.3 steps 1-3 and the colour query, per view:
 *   instance cameras W_{t,i} = W_t W_{t,i2g} (Sec. 3.3 "Instance-specific
 *   projection"; composed in FP64, rounded once), normalised time t,
 *   temporal selection v_s <= t <= v_e (Sec. 3.3 "Temporal separation"),
 *   projection of mean and covariance (Eq. 1, EWA), frustum test -> M_t,
 *   LOD cull of Gaussians whose 2D scale is at most lod_r (Sec. 3.3 "Adaptive
 *   LOD", drop probability 1), SH colour of the survivors only.
 * Writes one record per (view, surviving Gaussian), ordered by Gaussian block
 * then view then Gaussian index (so record index increases with the Gaussian
 * index within a view), each record's first (tile, record) pair, M_t bits and
 * stats; counters[S3R_CNT_DUP] / [S3R_CNT_OVF_DUP] get the pairs kept (those
 * of the kept records, at most cap_dup) and dropped.
 * `ws` must hold s3r_workspace_size(S3R_WS_PROJECT) bytes.
 */
int s3r_project_cull(const S3RScene* scene, const S3RViews* views, const S3RParams* params,
                     S3RProjected* out, void* ws, size_t ws_bytes, void* stream);

/*
 * s3r_project_cull_noalloc -- s3r_project_cull without a workspace argument,
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, outputs and errors otherwise; it calls no allocating routine.
 * Its scratch is a fixed 4 MiB device array in the library, one per device
 * (held until the process ends, its address looked up on the first call on
 * each device).  A problem whose workspace, s3r_workspace_size(
 * S3R_WS_PROJECT), exceeds 4 MiB is rejected with S3R_E_SCRATCH before
 * anything is enqueued; 4 MiB holds e.g. 100M Gaussians x 24 views or 20M x 64.
 * Every call on a device shares that device's scratch: calls that overlap in
 * time on one device (different streams, or several threads) race and must
 * be serialised by the caller.  Nothing in the scratch needs clearing between
 * calls (each call writes what it reads).
 */
int s3r_project_cull_noalloc(const S3RScene* scene, const S3RViews* views,
                             const S3RParams* params, S3RProjected* out, void* stream);

/*
 * s3r_sort -- builds per-tile contributor lists ordered by (depth bits,
 * Gaussian index), the blending order of Eq. (2), bit-exactly, from the
 * (tile, record) pairs of s3r_project_cull (proj->rec_pair): keyed (tile <<
 * 32 | depth bits) in record order and sorted by a stable radix sort -- or,
 * with S3R_SORT_TILES, binned by tile and each list sorted on (depth bits,
 * record index) (a stable radix partition on the tile bits and a sort on
 * (depth bits, position) when the batch has more tiles than the binning
 * holds), which gives the same lists.  Also writes the rasterizers' launch
 * order and stats[v][3].  Reads the records of s3r_project_cull (only
 * scene->n is read from `scene`); `ws` holds s3r_workspace_size(S3R_WS_SORT)
 * bytes.
 */
int s3r_sort(const S3RScene* scene, const S3RProjected* proj, const S3RViews* views,
             const S3RParams* params, S3RBins* bins, void* ws, size_t ws_bytes, void* stream);

/*
 * s3r_raster_fwd -- front-to-back alpha blending of Eq. (2) for every pixel of
 * every view in one launch: Mahalanobis cut, alpha = min(alpha_max,
 * o exp(power)), skip below alpha_min, stop before T would fall below t_min.
 */
int s3r_raster_fwd(const S3RProjected* proj, const S3RBins* bins, const S3RViews* views,
                   const S3RParams* params, S3RImage* img, void* stream);

/*
 * s3r_l1_loss -- per-view mean absolute error against `target` (same layout
 * as S3RImage.color), loss[v] written, and its gradient d_color.
 */
int s3r_l1_loss(const S3RImage* img, const float* target, const S3RViews* views,
                float* loss, float* d_color, void* stream);

/*
 * s3r_raster_bwd -- gradient of the blending (replayed back to front from
 * T_final and `last`) and of the projection, colour and instance cameras
 * (chain of Eq. 1 and the SH colour), written to `g` (every per-Gaussian
 * entry; no caller-side zeroing).  The projection gradient is gathered per
 * Gaussian over the views of the batch, using `proj->surv` and `proj->bstat`
 * to find each Gaussian's records; the blending gradients of each (record,
 * tile) pair go to the pair's own slot in `ws` (found from proj->rec_pair
 * and the record's tile rectangle) and are summed per record, so no
 * gradient atomics contend across tiles.  Pose gradients are chained through
 * W_{t,i} = W_t W_{t,i2g} and also given in 6-DoF form.  In the plain route
 * the world-frame gradients g->mean_w / g->rot_w (every slot of the batch)
 * are written instead of mean / quat; s3r_plain_transform_bwd finishes them.
 */
int s3r_raster_bwd(const S3RScene* scene, const S3RViews* views, const S3RParams* params,
                   const S3RProjected* proj, const S3RBins* bins, const S3RImage* img,
                   const float* d_color, S3RGrads* g, void* ws, size_t ws_bytes, void* stream);

/*
 * s3r_update_visibility -- Eqs. (5)-(6).  UPDATE: for every view v of the
 * batch whose M_t bit is set, l_s = min(l_s, t_v), l_e = max(l_e, t_v).
 * FOLD: v_s = l_s - margin, v_e = l_e + margin.  RESET: v = (-1, 1),
 * l = (1, -1).  `mask` and `t_norm` are those of S3RProjected (UPDATE only).
 */
int s3r_update_visibility(float* life_s, float* life_e, float* vis_s, float* vis_e,
                          const uint32_t* mask, const float* t_norm, int32_t n_views,
                          int64_t n, int32_t mode, float margin, void* stream);

/*
 * s3r_plain_transform -- the conventional local->global transform of Sec. 3.1
 * for the baseline route: for each of the n_ts timesteps in `tsteps` (host
 * array), mean_w = R_G mean + t_G and rot_w = R_G R(q) for every Gaussian,
 * written to out_mean_w[n_ts][N][3] and out_rot_w[n_ts][N][9].
 */
int s3r_plain_transform(const S3RScene* scene, const int32_t* tsteps, int32_t n_ts,
                        float* out_mean_w, float* out_rot_w, void* stream);

/*
 * s3r_plain_transform_bwd -- chains world-frame gradients (S3RGrads.mean_w,
 * rot_w) back to local mean / quat (written) and to the poses of the n_ts
 * timesteps (added to g->pose).
 */
int s3r_plain_transform_bwd(const S3RScene* scene, const int32_t* tsteps, int32_t n_ts,
                            S3RGrads* g, void* stream);

/*
 * Launch-shape knobs, process-wide (every device, every later call; a value
 * is read when a call enqueues its kernels, so a captured graph keeps the
 * values of its capture).  None changes any result: every path gives the
 * same records, lists, images and gradients, bit for bit.  Calls that set
 * knobs while other threads enqueue work race with them.
 *   S3R_TUNE_OFFSET_FUSE_MAX  the per-(block, view) record/pair offset scan
 *       of s3r_project_cull runs in two launches while it has at most this
 *       many chunks of 1024 entries, in three beyond (0..1024, default 1024)
 *   S3R_TUNE_SCAN_FUSE_MAX    the same for the library's other prefix scans
 *       (radix histograms; chunks of 4096 entries)
 *   S3R_TUNE_BIN_MAX_TILES    with S3R_SORT_TILES, batches of at most this
 *       many tiles are binned through LDS histograms, larger ones partitioned
 *       by radix passes (0..12288, default 12288; 0: always partition)
 *   S3R_TUNE_RASTER_WAVES     waves per workgroup of s3r_raster_fwd: 1 (each
 *       8x8 sub-tile its own workgroup, default) or the tile's sub-tiles
 *       together (TILE^2 / 64; the value is clamped to that)
 *   S3R_TUNE_FINE_TILES       s3r_raster_fwd gives the first this many tiles
 *       of the launch order (the longest lists; rounded down to a multiple of
 *       32) one wave per 4x4 pixel block instead of one per 8x8 sub-tile
 *       (0..1048576, default 160)
 * s3r_set_tuning(knob, negative value) restores the default.  Errors:
 * S3R_E_ARG for an unknown knob or a value out of range.
 */
enum {
  S3R_TUNE_OFFSET_FUSE_MAX = 0,
  S3R_TUNE_SCAN_FUSE_MAX = 1,
  S3R_TUNE_BIN_MAX_TILES = 2,
  S3R_TUNE_RASTER_WAVES = 3,
  S3R_TUNE_FINE_TILES = 4,
  S3R_TUNE_COUNT = 5
};
int s3r_set_tuning(int32_t knob, int32_t value);
int s3r_get_tuning(int32_t knob, int32_t* value);

/*
 * Opt-in per-kernel timing (tracing): when enabled, every kernel the library
 * enqueues is bracketed by HIP events on its stream.  s3r_profile_read()
 * waits for the recorded events and returns the accumulated milliseconds and
 * launch count of kernel `id` (0 <= id < s3r_profile_kernels(), named by
 * s3r_profile_name()).  Not for use while a stream is being captured.
 */
int s3r_profile_enable(int on);
int s3r_profile_only(int32_t id); /* >= 0: time kernel `id` only; -1: every kernel */
int s3r_profile_reset(void);
int s3r_profile_read(int32_t id, double* total_ms, int64_t* count);
const char* s3r_profile_name(int32_t id);
int s3r_profile_kernels(void);

int s3r_abi_version(void);
const char* s3r_status_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* S3R_H */
