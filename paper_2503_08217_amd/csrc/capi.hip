// extern "C" entry points: argument validation, workspace carving, launches.
#include <algorithm>
#include <atomic>
#include <mutex>

#include "internal.hpp"

using namespace s3r;

// Fixed device scratch of s3r_project_cull_noalloc (the block-offset scan's
// chunk sums and per-view chunk statistics).  Each device holds its own copy
// for the life of the process; every call on a device reuses it.
constexpr size_t kScratchBytes = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace s3r {
namespace {
// defaults, and the largest value, of the launch-shape knobs
constexpr int kTuneDefault[S3R_TUNE_COUNT] = {1024, 1024, 12288, 1, 160};
constexpr int kTuneMax[S3R_TUNE_COUNT] = {1024, 1024, 12288, 16, 1 << 20};
std::atomic<int> g_tune[S3R_TUNE_COUNT] = {{kTuneDefault[0]}, {kTuneDefault[1]},
                                           {kTuneDefault[2]}, {kTuneDefault[3]},
                                           {kTuneDefault[4]}};
}  // namespace
int tune(int knob) { return g_tune[knob].load(std::memory_order_relaxed); }
}  // namespace s3r

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

// Device address of the current device's `scratch`, looked up once per
// device (the array's name is only a host-side stand-in).
int scratch_base(char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return S3R_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return S3R_E_HIP;
    g_scratch[dev] = static_cast<char*>(p);
  }
  *out = g_scratch[dev];
  return S3R_OK;
}

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

#define S3R_REQUIRE(p)                    \
  do {                                    \
    if ((p) == nullptr) return S3R_E_NULL; \
    if (!aligned16(p)) return S3R_E_ALIGN; \
  } while (0)

#define S3R_HIP(expr)                         \
  do {                                        \
    if ((expr) != hipSuccess) return S3R_E_HIP; \
  } while (0)

struct WsProject {
  int32_t* chunk_sum;
  long long* chunk_sum_p;
  int32_t* chunk_stat;
};
struct WsSort {
  uint64_t* keys;
  uint64_t* keys_alt;
  uint32_t* vals;
  uint32_t* vals_alt;
  int32_t* hist;
  int32_t* sums;
  int32_t* misc;
  int32_t* order_cnt;
  int32_t* bin_count;   // [total_tiles] pairs per tile (binning path)
  int32_t* bin_cursor;  // [total_tiles] next free slot of each tile's list
};
struct WsBwd {
  float4* g2d;
  float4* part;
  int2* tile_cut;
  float* d_cam;
  unsigned long long* d_cam_fx;
  int32_t* carry_rec;
  float* carry_g;
};

size_t ws_project(const S3RSizes& z, WsProject* w, char* base) {
  const int nchunk = offset_chunks(project_blocks(z.n), (int)z.n_views);
  size_t off = 0;
  if (w) w->chunk_sum = reinterpret_cast<int32_t*>(base + off);
  off += align_up((size_t)nchunk * 4 + 16);
  if (w) w->chunk_sum_p = reinterpret_cast<long long*>(base + off);
  off += align_up((size_t)nchunk * 8 + 16);
  if (w) w->chunk_stat = reinterpret_cast<int32_t*>(base + off);
  off += align_up((size_t)nchunk * z.n_views * 12 + 16);
  return off;
}

size_t ws_sort(const S3RSizes& z, WsSort* w, char* base) {
  size_t off = 0;
  if (w) w->keys = reinterpret_cast<uint64_t*>(base + off);
  off += align_up((size_t)z.cap_dup * 8);
  if (w) w->keys_alt = reinterpret_cast<uint64_t*>(base + off);
  off += align_up((size_t)z.cap_dup * 8);
  if (w) w->vals = reinterpret_cast<uint32_t*>(base + off);
  off += align_up((size_t)z.cap_dup * 4);
  if (w) w->vals_alt = reinterpret_cast<uint32_t*>(base + off);
  off += align_up((size_t)z.cap_dup * 4);
  const size_t hw = sort_hist_words(z.cap_dup);
  if (w) w->hist = reinterpret_cast<int32_t*>(base + off);
  off += align_up(hw * 4 + 4);
  const int64_t sb = std::max<int64_t>(scan_blocks(z.cap_surv), scan_blocks((int64_t)hw));
  if (w) w->sums = reinterpret_cast<int32_t*>(base + off);
  off += align_up((size_t)sb * 4 + 4);
  if (w) w->misc = reinterpret_cast<int32_t*>(base + off);
  off += align_up(64);
  if (w) w->order_cnt = reinterpret_cast<int32_t*>(base + off);
  off += align_up(order_count_words(z.total_tiles) * 4);
  if (w) w->bin_count = reinterpret_cast<int32_t*>(base + off);
  off += align_up((size_t)z.total_tiles * 4 + 4);
  if (w) w->bin_cursor = reinterpret_cast<int32_t*>(base + off);
  off += align_up((size_t)z.total_tiles * 4 + 4);
  return off;
}

size_t ws_bwd(const S3RSizes& z, WsBwd* w, char* base) {
  size_t off = 0;
  if (w) w->g2d = reinterpret_cast<float4*>(base + off);
  off += align_up((size_t)z.cap_surv * 48);
  if (w) w->part = reinterpret_cast<float4*>(base + off);
  off += align_up((size_t)z.cap_dup * 48);
  if (w) w->tile_cut = reinterpret_cast<int2*>(base + off);
  off += align_up((size_t)z.total_tiles * 8 + 8);
  if (w) w->d_cam = reinterpret_cast<float*>(base + off);
  off += align_up((size_t)z.n_views * z.n_slots * 48 + 16);
  if (w) w->d_cam_fx = reinterpret_cast<unsigned long long*>(base + off);
  off += align_up((size_t)z.n_views * z.n_slots * 96 + 16);
  // one carry-in and one carry-out per workgroup of the per-record sum
  const size_t nwg = (size_t)(z.cap_dup + 2047) / 2048 + 1;
  if (w) w->carry_rec = reinterpret_cast<int32_t*>(base + off);
  off += align_up(2 * nwg * 4);
  if (w) w->carry_g = reinterpret_cast<float*>(base + off);
  off += align_up(2 * nwg * 9 * 4);
  return off;
}

KParams kparams(const S3RParams& p) {
  KParams k;
  k.tile = p.tile;
  k.flags = p.flags;
  k.lod_r = p.lod_r;
  k.z_near = p.z_near;
  k.z_far = p.z_far;
  k.eps2d = p.eps2d;
  k.alpha_min = p.alpha_min;
  k.alpha_max = p.alpha_max;
  k.t_min = p.t_min;
  k.cutoff = p.cutoff;
  k.jac_clamp = p.jac_clamp;
  k.bg0 = p.bg[0];
  k.bg1 = p.bg[1];
  k.bg2 = p.bg[2];
  k.cap_surv = p.cap_surv;
  k.cap_dup = p.cap_dup;
  k.seed = p.seed;
  k.lod_pmax = p.lod_pmax;
  k.lod_D = p.lod_D;
  k.step = p.step;
  return k;
}

int check_params(const S3RParams* p) {
  if (!p) return S3R_E_NULL;
  if (p->tile != 8 && p->tile != 16 && p->tile != 32) return S3R_E_SIZE;
  if (p->cap_surv <= 0 || p->cap_surv >= (int64_t(1) << 31)) return S3R_E_SIZE;
  if (p->cap_dup <= 0 || p->cap_dup >= (int64_t(1) << 31)) return S3R_E_SIZE;
  if (!(p->alpha_min > 0.f) || !(p->alpha_max > 0.f) || !(p->alpha_max < 1.f) ||
      !(p->t_min > 0.f))
    return S3R_E_ARG;
  if ((p->flags & S3R_LOD_STOCHASTIC) && !(p->lod_D > 0.f)) return S3R_E_ARG;
  return S3R_OK;
}

int check_views(const S3RViews* v) {
  if (!v) return S3R_E_NULL;
  if (v->n_views < 1 || v->n_views > kMaxViews) return S3R_E_SIZE;
  if (v->total_tiles < 1 || v->total_px < 1) return S3R_E_SIZE;
  S3R_REQUIRE(v->W);
  S3R_REQUIRE(v->K);
  S3R_REQUIRE(v->wh);
  S3R_REQUIRE(v->tstep);
  S3R_REQUIRE(v->tile_offset);
  S3R_REQUIRE(v->px_offset);
  return S3R_OK;
}

int check_scene(const S3RScene* s, bool plain) {
  if (!s) return S3R_E_NULL;
  if (s->n < 0 || s->n >= (int64_t(1) << 31)) return S3R_E_SIZE;
  if (s->sh_degree < 0 || s->sh_degree > 3) return S3R_E_SIZE;
  if (s->n_slots < 1 || s->n_timesteps < 1) return S3R_E_SIZE;
  S3R_REQUIRE(s->mean);
  S3R_REQUIRE(s->scale);
  S3R_REQUIRE(s->quat);
  S3R_REQUIRE(s->opacity);
  S3R_REQUIRE(s->sh);
  S3R_REQUIRE(s->inst);
  S3R_REQUIRE(s->pose);
  if (plain) {
    S3R_REQUIRE(s->mean_w);
    S3R_REQUIRE(s->rot_w);
  }
  return S3R_OK;
}

S3RSizes sizes_of(const S3RScene* s, const S3RViews* v, const S3RParams* p) {
  S3RSizes z{};
  z.n = s ? s->n : 0;
  z.n_views = v->n_views;
  z.total_tiles = v->total_tiles;
  z.cap_surv = p->cap_surv;
  z.cap_dup = p->cap_dup;
  z.n_slots = s ? s->n_slots : 1;
  return z;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }


int check_project_args(const S3RScene* scene, const S3RViews* views, const S3RParams* params,
                       const S3RProjected* out) {
  int rc = check_params(params);
  if (rc) return rc;
  const bool plain = (params->flags & S3R_PLAIN) != 0;
  if ((rc = check_scene(scene, plain))) return rc;
  if ((rc = check_views(views))) return rc;
  if (!out) return S3R_E_NULL;
  if ((params->flags & S3R_TEMPORAL)) {
    S3R_REQUIRE(scene->vis_s);
    S3R_REQUIRE(scene->vis_e);
  }
  if (plain) S3R_REQUIRE(views->plain_slot);
  if ((uint64_t)scene->n * (uint64_t)views->n_views >= (uint64_t(1) << 32)) return S3R_E_SIZE;
  S3R_REQUIRE(out->cam);
  S3R_REQUIRE(out->cen);
  S3R_REQUIRE(out->t_norm);
  S3R_REQUIRE(out->mask);
  S3R_REQUIRE(out->rec_gid);
  S3R_REQUIRE(out->rec_view);
  S3R_REQUIRE(out->rec_geo);
  S3R_REQUIRE(out->rec_conic);
  S3R_REQUIRE(out->rec_rgb);
  S3R_REQUIRE(out->rec_rect);
  S3R_REQUIRE(out->counters);
  S3R_REQUIRE(out->stats);
  S3R_REQUIRE(out->rec_npairs);
  S3R_REQUIRE(out->surv);
  S3R_REQUIRE(out->bstat);
  S3R_REQUIRE(out->rec_pair);
  return S3R_OK;
}

// a1-a5 on `st` with the workspace carved into `w` (arguments validated)
int project_cull_launch(const S3RScene* scene, const S3RViews* views, const S3RParams* params,
                        S3RProjected* out, const WsProject& w, hipStream_t st) {
  const int nblk = project_blocks(scene->n);
  S3R_HIP(launch_compose(views->W, views->tstep, scene->pose, scene->n_slots, scene->n_timesteps,
                         views->n_views, out->cam, out->cen, out->t_norm, out->counters,
                         out->stats, st));
  ProjArgs a{};
  a.mean = scene->mean;
  a.scale = scene->scale;
  a.quat = scene->quat;
  a.opac = scene->opacity;
  a.sh = scene->sh;
  a.inst = scene->inst;
  a.vis_s = scene->vis_s;
  a.vis_e = scene->vis_e;
  a.pose = scene->pose;
  a.mean_w = scene->mean_w;
  a.rot_w = scene->rot_w;
  a.n = (int)scene->n;
  a.sh_deg = scene->sh_degree;
  a.n_slots = scene->n_slots;
  a.n_ts = scene->n_timesteps;
  a.Kv = views->K;
  a.wh = views->wh;
  a.tstep = views->tstep;
  a.tile_offset = views->tile_offset;
  a.plain_slot = views->plain_slot;
  a.nv = views->n_views;
  a.cam = out->cam;
  a.cen = out->cen;
  a.t_norm = out->t_norm;
  a.mask = out->mask;
  a.mask_words = ((scene->n + 63) / 64) * 2;
  a.rec_gid = out->rec_gid;
  a.rec_view = out->rec_view;
  a.rec_geo = reinterpret_cast<float4*>(out->rec_geo);
  a.rec_conic = reinterpret_cast<float4*>(out->rec_conic);
  a.rec_rgb = reinterpret_cast<float4*>(out->rec_rgb);
  a.rec_rect = reinterpret_cast<int4*>(out->rec_rect);
  a.rec_npairs = out->rec_npairs;
  a.counters = out->counters;
  a.surv = out->surv;
  a.bstat = out->bstat;
  a.rec_pair = out->rec_pair;
  a.chunk_sum = w.chunk_sum;
  a.chunk_sum_p = w.chunk_sum_p;
  a.chunk_stat = w.chunk_stat;
  a.nblk = nblk;
  a.kp = kparams(*params);
  S3R_HIP(launch_project(a, out->stats, st));
  return S3R_OK;
}

}  // namespace

extern "C" {

int s3r_abi_version(void) { return S3R_ABI_VERSION; }

int s3r_set_tuning(int32_t knob, int32_t value) {
  if (knob < 0 || knob >= S3R_TUNE_COUNT) return S3R_E_ARG;
  if (value < 0) value = kTuneDefault[knob];
  if (value > kTuneMax[knob] || (knob == S3R_TUNE_RASTER_WAVES && value < 1)) return S3R_E_ARG;
  g_tune[knob].store(value, std::memory_order_relaxed);
  return S3R_OK;
}

int s3r_get_tuning(int32_t knob, int32_t* value) {
  if (knob < 0 || knob >= S3R_TUNE_COUNT) return S3R_E_ARG;
  if (!value) return S3R_E_NULL;
  *value = tune(knob);
  return S3R_OK;
}

const char* s3r_status_string(int code) {
  switch (code) {
    case S3R_OK: return "ok";
    case S3R_E_NULL: return "a required pointer is NULL";
    case S3R_E_ALIGN: return "a pointer is not 16-byte aligned";
    case S3R_E_SIZE: return "a size is out of range";
    case S3R_E_WORKSPACE: return "workspace too small";
    case S3R_E_HIP: return "HIP kernel launch failed";
    case S3R_E_ARG: return "invalid argument value";
    case S3R_E_SCRATCH:
      return "problem too large for the fixed scratch of the no-allocation entry point";
    default: return "unknown status";
  }
}

int s3r_workspace_size(const S3RSizes* z, int32_t which, size_t* bytes) {
  if (!z || !bytes) return S3R_E_NULL;
  if (z->n < 0 || z->n_views < 1 || z->n_views > kMaxViews || z->total_tiles < 0 ||
      z->cap_surv < 0 || z->cap_dup < 0 || z->n_slots < 1)
    return S3R_E_SIZE;
  switch (which) {
    case S3R_WS_PROJECT: *bytes = ws_project(*z, nullptr, nullptr); break;
    case S3R_WS_SORT: *bytes = ws_sort(*z, nullptr, nullptr); break;
    case S3R_WS_BACKWARD: *bytes = ws_bwd(*z, nullptr, nullptr); break;
    default: return S3R_E_ARG;
  }
  return S3R_OK;
}

int s3r_project_cull(const S3RScene* scene, const S3RViews* views, const S3RParams* params,
                     S3RProjected* out, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_project_args(scene, views, params, out);
  if (rc) return rc;
  const S3RSizes z = sizes_of(scene, views, params);
  if (!ws && ws_bytes) return S3R_E_NULL;
  if (ws_bytes < ws_project(z, nullptr, nullptr) || !ws) return S3R_E_WORKSPACE;
  if (!aligned16(ws)) return S3R_E_ALIGN;
  WsProject w;
  ws_project(z, &w, static_cast<char*>(ws));
  return project_cull_launch(scene, views, params, out, w, as_stream(stream));
}

int s3r_project_cull_noalloc(const S3RScene* scene, const S3RViews* views,
                             const S3RParams* params, S3RProjected* out, void* stream) {
  int rc = check_project_args(scene, views, params, out);
  if (rc) return rc;
  const S3RSizes z = sizes_of(scene, views, params);
  if (ws_project(z, nullptr, nullptr) > kScratchBytes) return S3R_E_SCRATCH;
  char* base = nullptr;
  if ((rc = scratch_base(&base))) return rc;
  WsProject w;
  ws_project(z, &w, base);
  return project_cull_launch(scene, views, params, out, w, as_stream(stream));
}

int s3r_sort(const S3RScene* scene, const S3RProjected* proj, const S3RViews* views,
             const S3RParams* params, S3RBins* bins, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_params(params);
  if (rc) return rc;
  if ((rc = check_views(views))) return rc;
  if (!scene || !proj || !bins) return S3R_E_NULL;
  if (scene->n < 0 || scene->n >= (int64_t(1) << 31)) return S3R_E_SIZE;
  S3R_REQUIRE(proj->rec_geo);
  S3R_REQUIRE(proj->rec_rect);
  S3R_REQUIRE(proj->counters);
  S3R_REQUIRE(proj->stats);
  S3R_REQUIRE(proj->rec_view);
  S3R_REQUIRE(proj->rec_npairs);
  S3R_REQUIRE(bins->tile_count);
  S3R_REQUIRE(bins->tile_start);
  S3R_REQUIRE(bins->tile_order);
  S3R_REQUIRE(bins->vals);
  S3R_REQUIRE(proj->rec_pair);
  const S3RSizes z = sizes_of(nullptr, views, params);
  if (!ws || ws_bytes < ws_sort(z, nullptr, nullptr)) return S3R_E_WORKSPACE;
  if (!aligned16(ws)) return S3R_E_ALIGN;
  WsSort w;
  ws_sort(z, &w, static_cast<char*>(ws));
  SortArgs a{};
  a.rec_rect = reinterpret_cast<const int4*>(proj->rec_rect);
  a.rec_geo = reinterpret_cast<const float4*>(proj->rec_geo);
  a.rec_view = proj->rec_view;
  a.rec_npairs = proj->rec_npairs;
  a.nv = views->n_views;
  a.total_tiles = views->total_tiles;
  a.tile = params->tile;
  a.by_tile = (params->flags & S3R_SORT_TILES) != 0;
  a.tile_offset = views->tile_offset;
  a.wh = views->wh;
  a.counters = proj->counters;
  a.stats = proj->stats;
  a.tile_count = bins->tile_count;
  a.tile_start = bins->tile_start;
  a.tile_order = bins->tile_order;
  a.pair_off = proj->rec_pair;
  a.bin_count = w.bin_count;
  a.bin_cursor = w.bin_cursor;
  a.keys = w.keys;
  a.keys_alt = w.keys_alt;
  a.vals0 = w.vals;
  a.vals1 = w.vals_alt;
  a.vals_out = bins->vals;
  a.hist = w.hist;
  a.scan_sums = w.sums;
  a.misc = w.misc;
  a.order_cnt = w.order_cnt;
  a.cap_dup = params->cap_dup;
  a.cap_surv = params->cap_surv;
  S3R_HIP(launch_sort(a, as_stream(stream)));
  return S3R_OK;
}

int s3r_raster_fwd(const S3RProjected* proj, const S3RBins* bins, const S3RViews* views,
                   const S3RParams* params, S3RImage* img, void* stream) {
  int rc = check_params(params);
  if (rc) return rc;
  if ((rc = check_views(views))) return rc;
  if (!proj || !bins || !img) return S3R_E_NULL;
  S3R_REQUIRE(proj->rec_geo);
  S3R_REQUIRE(proj->rec_conic);
  S3R_REQUIRE(proj->rec_rgb);
  S3R_REQUIRE(proj->counters);
  S3R_REQUIRE(bins->tile_start);
  S3R_REQUIRE(bins->tile_order);
  S3R_REQUIRE(bins->vals);
  S3R_REQUIRE(img->color);
  S3R_REQUIRE(img->T_final);
  S3R_REQUIRE(img->last);
  RasterArgs a{};
  a.rec_geo = reinterpret_cast<const float4*>(proj->rec_geo);
  a.rec_conic = reinterpret_cast<const float4*>(proj->rec_conic);
  a.rec_rgb = reinterpret_cast<const float4*>(proj->rec_rgb);
  a.tile_start = bins->tile_start;
  a.tile_order = bins->tile_order;
  a.vals = bins->vals;
  a.tile_offset = views->tile_offset;
  a.px_offset = views->px_offset;
  a.wh = views->wh;
  a.counters = proj->counters;
  a.nv = views->n_views;
  a.total_tiles = views->total_tiles;
  a.color = img->color;
  a.T_final = img->T_final;
  a.last = img->last;
  a.kp = kparams(*params);
  if (img->census) {
    if ((reinterpret_cast<uintptr_t>(img->census) & 7u) != 0) return S3R_E_ALIGN;
    a.census = reinterpret_cast<unsigned long long*>(img->census);
  }
  const hipStream_t st = as_stream(stream);
  const int64_t mw = ((img->n + 63) / 64) * 2;
  if (img->m_raster) {
    S3R_REQUIRE(img->rec_taken);
    S3R_REQUIRE(proj->rec_gid);
    S3R_REQUIRE(proj->rec_view);
    if (img->n < 0 || img->n >= (int64_t(1) << 31)) return S3R_E_SIZE;
    a.rec_taken = img->rec_taken;
    S3R_HIP(launch_zero(img->rec_taken, (size_t)params->cap_surv * 4, img->m_raster,
                        (size_t)views->n_views * mw * 4, nullptr, 0, nullptr, 0, st));
  }
  S3R_HIP(launch_raster_fwd(a, st));
  if (img->m_raster)
    S3R_HIP(launch_raster_mask(img->rec_taken, proj->rec_gid, proj->rec_view, proj->counters,
                               params->cap_surv, mw, img->m_raster, st));
  return S3R_OK;
}

int s3r_l1_loss(const S3RImage* img, const float* target, const S3RViews* views, float* loss,
                float* d_color, void* stream) {
  int rc = check_views(views);
  if (rc) return rc;
  if (!img) return S3R_E_NULL;
  S3R_REQUIRE(img->color);
  S3R_REQUIRE(target);
  S3R_REQUIRE(loss);
  S3R_REQUIRE(d_color);
  S3R_HIP(launch_l1_loss(img->color, target, views->px_offset, views->wh, views->n_views,
                         views->total_px, loss, d_color, as_stream(stream)));
  return S3R_OK;
}

int s3r_raster_bwd(const S3RScene* scene, const S3RViews* views, const S3RParams* params,
                   const S3RProjected* proj, const S3RBins* bins, const S3RImage* img,
                   const float* d_color, S3RGrads* g, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_params(params);
  if (rc) return rc;
  const bool plain = (params->flags & S3R_PLAIN) != 0;
  if ((rc = check_scene(scene, plain))) return rc;
  if ((rc = check_views(views))) return rc;
  if (!proj || !bins || !img || !g) return S3R_E_NULL;
  if (plain) S3R_REQUIRE(views->plain_slot);
  S3R_REQUIRE(d_color);
  S3R_REQUIRE(img->T_final);
  S3R_REQUIRE(img->last);
  S3R_REQUIRE(proj->cam);
  S3R_REQUIRE(proj->cen);
  S3R_REQUIRE(proj->rec_gid);
  S3R_REQUIRE(proj->rec_view);
  S3R_REQUIRE(proj->rec_geo);
  S3R_REQUIRE(proj->rec_conic);
  S3R_REQUIRE(proj->rec_rgb);
  S3R_REQUIRE(proj->rec_rect);
  S3R_REQUIRE(proj->counters);
  S3R_REQUIRE(proj->surv);
  S3R_REQUIRE(proj->bstat);
  S3R_REQUIRE(bins->tile_start);
  S3R_REQUIRE(bins->tile_order);
  S3R_REQUIRE(bins->vals);
  S3R_REQUIRE(proj->rec_pair);
  S3R_REQUIRE(g->scale);
  S3R_REQUIRE(g->opacity);
  S3R_REQUIRE(g->sh);
  S3R_REQUIRE(g->pose);
  if (plain) {
    S3R_REQUIRE(g->mean_w);
    S3R_REQUIRE(g->rot_w);
  } else {
    S3R_REQUIRE(g->mean);
    S3R_REQUIRE(g->quat);
  }
  if (g->pose6 && !aligned16(g->pose6)) return S3R_E_ALIGN;
  const bool det = (params->flags & S3R_DETERMINISTIC_GRADS) != 0;
  if (det && plain) return S3R_E_ARG;
  const bool sparse = (params->flags & S3R_GRAD_SPARSE) != 0 && !plain;
  if (sparse) {
    S3R_REQUIRE(g->rows);
    S3R_REQUIRE(g->n_rows);
  }
  const S3RSizes z = sizes_of(scene, views, params);
  if (!ws || ws_bytes < ws_bwd(z, nullptr, nullptr)) return S3R_E_WORKSPACE;
  if (!aligned16(ws)) return S3R_E_ALIGN;
  WsBwd w;
  ws_bwd(z, &w, static_cast<char*>(ws));
  const hipStream_t st = as_stream(stream);
  const KParams kp = kparams(*params);

  BwdArgs b{};
  b.rec_geo = reinterpret_cast<const float4*>(proj->rec_geo);
  b.rec_conic = reinterpret_cast<const float4*>(proj->rec_conic);
  b.rec_rgb = reinterpret_cast<const float4*>(proj->rec_rgb);
  b.rec_gid = proj->rec_gid;
  b.rec_view = proj->rec_view;
  b.tile_start = bins->tile_start;
  b.tile_order = bins->tile_order;
  b.vals = bins->vals;
  b.tile_offset = views->tile_offset;
  b.px_offset = views->px_offset;
  b.wh = views->wh;
  b.counters = proj->counters;
  b.T_final = img->T_final;
  b.last = img->last;
  b.d_color = d_color;
  b.nv = views->n_views;
  b.total_tiles = views->total_tiles;
  b.rec_pair = proj->rec_pair;
  b.rec_rect = reinterpret_cast<const int4*>(proj->rec_rect);
  b.part = w.part;
  b.tile_cut = w.tile_cut;
  // (the fixed-point sums of the deterministic mode are cleared as floats:
  // two per 64-bit sum)
  b.zero_a = det ? reinterpret_cast<float*>(w.d_cam_fx) : w.d_cam;
  b.n_zero_a = (int64_t)views->n_views * scene->n_slots * 12 * (det ? 2 : 1);
  b.carry_rec = w.carry_rec;
  b.carry_g = w.carry_g;
  b.zero_b = g->pose;
  b.n_zero_b = (int64_t)scene->n_timesteps * scene->n_slots * 12;
  b.g2d = w.g2d;
  b.kp = kp;
  {
    // every gradient output is written by this call: clear the dense arrays
    // (Gaussians without records keep these zeros), the per-record gradient
    // slots and the camera and pose accumulators -- in the sparse mode the
    // rows the previous call wrote instead of the dense arrays, all in one
    // launch
    const size_t N = (size_t)scene->n;
    const size_t B = (size_t)(scene->sh_degree + 1) * (scene->sh_degree + 1);
    if (sparse) {
      S3R_HIP(launch_clear_rows(g->rows, g->n_rows, scene->n, (int)B, g->mean, g->scale, g->quat,
                                g->opacity, g->sh, params->cap_surv,
                                reinterpret_cast<const uint32_t*>(proj->surv),
                                ((scene->n + 63) / 64) * 2, views->n_views, b, st));
    } else {
      void* ps[5] = {g->scale, g->opacity, g->sh, plain ? nullptr : g->mean,
                     plain ? nullptr : g->quat};
      const size_t bs[5] = {N * 12, N * 4, N * B * 12, N * 12, N * 16};
      S3R_HIP(launch_zero_n(ps, bs, 5, st));
      S3R_HIP(launch_zero_g2d(b, st));
    }
  }
  S3R_HIP(launch_raster_bwd(b, st));

  ProjBwdArgs p{};
  p.mean = scene->mean;
  p.scale = scene->scale;
  p.quat = scene->quat;
  p.opac = scene->opacity;
  p.sh = scene->sh;
  p.inst = scene->inst;
  p.pose = scene->pose;
  p.mean_w = scene->mean_w;
  p.rot_w = scene->rot_w;
  p.n = (int)scene->n;
  p.sh_deg = scene->sh_degree;
  p.n_slots = scene->n_slots;
  p.n_ts = scene->n_timesteps;
  p.Kv = views->K;
  p.wh = views->wh;
  p.tstep = views->tstep;
  p.plain_slot = views->plain_slot;
  p.nv = views->n_views;
  p.cam = proj->cam;
  p.cen = proj->cen;
  p.rec_gid = proj->rec_gid;
  p.rec_view = proj->rec_view;
  p.counters = proj->counters;
  p.surv = proj->surv;
  p.bstat = proj->bstat;
  p.mask_words = ((scene->n + 63) / 64) * 2;
  p.g2d = w.g2d;
  p.d_mean = g->mean;
  p.d_scale = g->scale;
  p.d_quat = g->quat;
  p.d_opac = g->opacity;
  p.d_sh = g->sh;
  p.d_mean_w = g->mean_w;
  p.d_rot_w = g->rot_w;
  p.d_cam = w.d_cam;
  p.d_cam_fx = det ? w.d_cam_fx : nullptr;
  p.d_pose = g->pose;
  p.kp = kp;
  p.rows = sparse ? g->rows : nullptr;
  p.n_rows = sparse ? g->n_rows : nullptr;
  S3R_HIP(launch_project_bwd(p, st));
  if (det)
    S3R_HIP(launch_pose_bwd_det(views->W, views->tstep, scene->pose, w.d_cam_fx, views->n_views,
                                scene->n_slots, scene->n_timesteps, g->pose, g->pose6, st));
  else if (!plain)
    S3R_HIP(launch_pose_bwd(views->W, views->tstep, scene->pose, w.d_cam, views->n_views,
                            scene->n_slots, scene->n_timesteps, g->pose, g->pose6, st));
  return S3R_OK;
}

int s3r_update_visibility(float* life_s, float* life_e, float* vis_s, float* vis_e,
                          const uint32_t* mask, const float* t_norm, int32_t n_views, int64_t n,
                          int32_t mode, float margin, void* stream) {
  if (n < 0 || n >= (int64_t(1) << 31)) return S3R_E_SIZE;
  if (mode != S3R_VIS_UPDATE && mode != S3R_VIS_FOLD && mode != S3R_VIS_RESET) return S3R_E_ARG;
  S3R_REQUIRE(life_s);
  S3R_REQUIRE(life_e);
  if (mode != S3R_VIS_UPDATE) {
    S3R_REQUIRE(vis_s);
    S3R_REQUIRE(vis_e);
  } else {
    if (n_views < 1 || n_views > kMaxViews) return S3R_E_SIZE;
    S3R_REQUIRE(mask);
    S3R_REQUIRE(t_norm);
  }
  S3R_HIP(launch_visibility(life_s, life_e, vis_s, vis_e, mask, t_norm, n_views, n, mode, margin,
                            as_stream(stream)));
  return S3R_OK;
}

int s3r_plain_transform(const S3RScene* scene, const int32_t* tsteps, int32_t n_ts,
                        float* out_mean_w, float* out_rot_w, void* stream) {
  if (!scene || !tsteps) return S3R_E_NULL;
  if (scene->n < 0 || scene->n >= (int64_t(1) << 31)) return S3R_E_SIZE;
  if (n_ts < 1 || n_ts > kMaxViews) return S3R_E_SIZE;
  for (int s = 0; s < n_ts; ++s)
    if (tsteps[s] < 0 || tsteps[s] >= scene->n_timesteps) return S3R_E_ARG;
  S3R_REQUIRE(scene->mean);
  S3R_REQUIRE(scene->quat);
  S3R_REQUIRE(scene->inst);
  S3R_REQUIRE(scene->pose);
  S3R_REQUIRE(out_mean_w);
  S3R_REQUIRE(out_rot_w);
  S3R_HIP(launch_plain_transform(scene->mean, scene->quat, scene->inst, scene->pose,
                                 (int)scene->n, scene->n_slots, tsteps, n_ts, out_mean_w,
                                 out_rot_w, as_stream(stream)));
  return S3R_OK;
}

int s3r_plain_transform_bwd(const S3RScene* scene, const int32_t* tsteps, int32_t n_ts,
                            S3RGrads* g, void* stream) {
  if (!scene || !tsteps || !g) return S3R_E_NULL;
  if (scene->n < 0 || scene->n >= (int64_t(1) << 31)) return S3R_E_SIZE;
  if (n_ts < 1 || n_ts > kMaxViews) return S3R_E_SIZE;
  for (int s = 0; s < n_ts; ++s)
    if (tsteps[s] < 0 || tsteps[s] >= scene->n_timesteps) return S3R_E_ARG;
  S3R_REQUIRE(scene->mean);
  S3R_REQUIRE(scene->quat);
  S3R_REQUIRE(scene->inst);
  S3R_REQUIRE(scene->pose);
  S3R_REQUIRE(g->mean);
  S3R_REQUIRE(g->quat);
  S3R_REQUIRE(g->pose);
  S3R_REQUIRE(g->mean_w);
  S3R_REQUIRE(g->rot_w);
  if (g->pose6 && !aligned16(g->pose6)) return S3R_E_ALIGN;
  const hipStream_t st = as_stream(stream);
  S3R_HIP(launch_plain_transform_bwd(scene->mean, scene->quat, scene->inst, scene->pose,
                                     (int)scene->n, scene->n_slots, tsteps, n_ts, g->mean_w,
                                     g->rot_w, g->mean, g->quat, g->pose, g->pose6, st));
  S3R_HIP(launch_pose_bwd(nullptr, nullptr, scene->pose, nullptr, 0, scene->n_slots,
                          scene->n_timesteps, g->pose, g->pose6, st));
  return S3R_OK;
}

}  // extern "C"
