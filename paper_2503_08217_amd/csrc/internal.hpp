// Kernel argument blocks and host launchers shared between the translation
// units of the library (not part of the public ABI).
#pragma once

#include "common.hpp"

namespace s3r {

// kernels timed by the opt-in profiler (names in profile.hip)
enum KernelId {
  K_COMPOSE, K_PLAIN_TRANSFORM, K_PROJECT, K_STATS, K_RECORDS, K_SCAN, K_EMIT, K_RADIX,
  K_TILE_RANGES, K_TILE_ORDER, K_TILE_SORT, K_TILE_SORT_MERGE, K_TILE_BIN,
  K_RASTER_FWD, K_L1, K_ZERO_G2D, K_RASTER_BWD, K_PAIR_REDUCE, K_PROJECT_BWD,
  K_POSE_BWD, K_POSE6, K_PLAIN_TRANSFORM_BWD, K_VISIBILITY, K_ZERO, K_COUNT
};
// current value of launch-shape knob S3R_TUNE_* (capi.hip)
int tune(int knob);
void prof_begin(int id, hipStream_t st);
void prof_end(int id, hipStream_t st);
#define S3R_LAUNCH(ID, ...)        \
  do {                             \
    ::s3r::prof_begin(ID, st);     \
    hipLaunchKernelGGL(__VA_ARGS__); \
    ::s3r::prof_end(ID, st);       \
  } while (0)

struct ProjArgs {
  // scene
  const float* mean;
  const float* scale;
  const float* quat;
  const float* opac;
  const float* sh;
  const int32_t* inst;
  const float* vis_s;
  const float* vis_e;
  const float* pose;
  const float* mean_w;
  const float* rot_w;
  int n, sh_deg, n_slots, n_ts;
  // views
  const float* Kv;
  const int32_t* wh;
  const int32_t* tstep;
  const int32_t* tile_offset;
  const int32_t* plain_slot;
  int nv;
  // per-view products of k_compose
  const float* cam;
  const float* cen;
  const float* t_norm;
  // outputs
  uint32_t* mask;
  uint32_t* surv;  // survivor bits, same layout as mask (workspace)
  int64_t mask_words;
  int32_t* rec_gid;
  int32_t* rec_view;
  float4* rec_geo;
  float4* rec_conic;
  float4* rec_rgb;
  int4* rec_rect;
  int32_t* rec_npairs;
  int32_t* counters;
  int32_t* rec_pair;  // first (tile, record) pair of each record, emission order
  // per (block, view), kBstat ints: N_t, N_f, N_r, first record, pairs,
  // first pair
  int32_t* bstat;
  // workspace: per chunk of (block, view) entries, the record and pair count
  // sums (then their offsets) and per-view partial stats
  int32_t* chunk_sum;
  long long* chunk_sum_p;
  int32_t* chunk_stat;
  uint64_t* flags;
  int nblk;
  KParams kp;
};

struct RasterArgs {
  const float4* rec_geo;
  const float4* rec_conic;
  const float4* rec_rgb;
  const int32_t* tile_start;
  const int32_t* tile_order;
  const uint32_t* vals;
  const int32_t* tile_offset;
  const int64_t* px_offset;
  const int32_t* wh;
  const int32_t* counters;
  int nv, total_tiles;
  float* color;
  float* T_final;
  int32_t* last;
  int32_t* rec_taken;  // optional: record blended into some pixel (rendering-derived M_t)
  unsigned long long* census;  // optional: evaluated and blended (pixel, entry) pairs
  KParams kp;
};

struct BwdArgs {
  // forward state
  const float4* rec_geo;
  const float4* rec_conic;
  const float4* rec_rgb;
  const int32_t* rec_gid;
  const int32_t* rec_view;
  const int32_t* tile_start;
  const int32_t* tile_order;
  const uint32_t* vals;
  const int32_t* tile_offset;
  const int64_t* px_offset;
  const int32_t* wh;
  const int32_t* counters;
  const float* T_final;
  const int32_t* last;
  const float* d_color;
  int nv, total_tiles;
  // first pair of each record in emission order and the records' tile
  // rectangles: the slot of a (record, tile) pair in `part`
  const int32_t* rec_pair;
  const int4* rec_rect;
  // small accumulators the g2d clear also zeroes (nullable)
  float* zero_a;
  int64_t n_zero_a;
  float* zero_b;
  int64_t n_zero_b;
  // per-pair 2D gradients (workspace, [cap_dup][12] floats), summed per
  // record into g2d ([cap_surv][12] floats, every record written)
  float4* part;
  // per tile: the first list entry the backward did not replay (record,
  // depth bits), or record -1 when it replayed the whole list (workspace)
  int2* tile_cut;
  float4* g2d;
  // S3R_DETERMINISTIC_GRADS: per workgroup of the per-record sum, the record
  // running in (2 w) and the one handed on (2 w + 1) with their partial sums
  int32_t* carry_rec;
  float* carry_g;
  KParams kp;
};

struct ProjBwdArgs {
  const float* mean;
  const float* scale;
  const float* quat;
  const float* opac;
  const float* sh;
  const int32_t* inst;
  const float* pose;
  const float* mean_w;
  const float* rot_w;
  int n, sh_deg, n_slots, n_ts;
  const float* Kv;
  const int32_t* wh;
  const int32_t* tstep;
  const int32_t* plain_slot;
  int nv;
  const float* cam;
  const float* cen;
  const int32_t* rec_gid;
  const int32_t* rec_view;
  const int32_t* counters;
  const uint32_t* surv;   // [V][mask_words] survivor bits
  const int32_t* bstat;   // [nblk][V][kBstat] per-block counts and first record
  int64_t mask_words;
  const float4* g2d;
  // gradients (written)
  float* d_mean;
  float* d_scale;
  float* d_quat;
  float* d_opac;
  float* d_sh;
  float* d_mean_w;
  float* d_rot_w;
  int32_t* rows;   // sparse gradient mode: [cap_surv] owner Gaussian or -1
  int32_t* n_rows;  // (null in the dense mode)
  float* d_cam;    // [V][S][12] workspace
  unsigned long long* d_cam_fx;  // [V][S][12] S3R_DETERMINISTIC_GRADS: fixed point, 2^-32 units
  float* d_pose;   // [T][S][12] (plain route: colour-direction part)
  KParams kp;
};

// project.hip
hipError_t launch_compose(const float* W, const int32_t* tstep, const float* pose, int S, int T,
                          int nv, float* cam, float* cen, float* t_norm, int32_t* counters,
                          int32_t* stats, hipStream_t st);
hipError_t launch_plain_transform(const float* mean, const float* quat, const int32_t* inst,
                                  const float* pose, int n, int S, const int32_t* tsteps, int n_ts,
                                  float* mean_w, float* rot_w, hipStream_t st);
// Gaussians per projection workgroup: records are ordered by (block, view,
// Gaussian) and the per-(block, view) survivor counts give each block's
// first record
constexpr int kProjBlock = 256;
constexpr int kBstat = 8;  // ints per (256-Gaussian block, view) entry of S3RProjected.bstat
constexpr int kProjWaves = kProjBlock / kWave;
int project_blocks(int64_t n);
int offset_chunks(int64_t nblk, int nv);
hipError_t launch_project(const ProjArgs& a, int32_t* stats, hipStream_t st);

// util.hip
// zero up to 8 device buffers (16-byte aligned) with one kernel
hipError_t launch_zero_n(void* const* ps, const size_t* bytes, int count, hipStream_t st);
hipError_t launch_zero(void* p0, size_t b0, void* p1, size_t b1, void* p2, size_t b2, void* p3,
                       size_t b3, hipStream_t st);

// sort.hip
int scan_blocks(int64_t n);
struct SortArgs {
  const int4* rec_rect;
  const float4* rec_geo;
  const int32_t* rec_view;
  const int32_t* rec_npairs;
  int nv, total_tiles, tile;
  bool by_tile;  // S3R_SORT_TILES: tile partition + per-list depth sort
  const int32_t* tile_offset;
  const int32_t* wh;
  int32_t* counters;
  int32_t* stats;
  int32_t* tile_count;
  int32_t* tile_start;
  int32_t* tile_order;
  // workspace
  const int32_t* pair_off;  // [cap_surv] first pair of each record (s3r_project_cull)
  uint64_t* keys;      // [cap_dup]
  uint64_t* keys_alt;  // [cap_dup]
  uint32_t* vals0;     // [cap_dup]: emitted values
  uint32_t* vals1;     // [cap_dup]: the other buffer of the partition passes
  uint32_t* vals_out;  // [cap_dup]: the sorted lists (S3RBins.vals)
  int32_t* hist;       // [256 * scan_blocks(cap_dup)]
  int32_t* scan_sums;
  int32_t* misc;       // [0] total pairs, [1] histogram total, [2] histogram length
  int32_t* order_cnt;  // [order_count_words] per (bucket, chunk) tile counts
  int32_t* bin_count;  // [total_tiles] pairs per tile (binning path)
  int32_t* bin_cursor; // [total_tiles] next free slot of each list (binning path)
  int64_t cap_dup, cap_surv;
};
int sort_passes(int total_tiles, bool by_tile);
size_t sort_hist_words(int64_t cap_dup);
size_t order_count_words(int total_tiles);
hipError_t launch_sort(const SortArgs& a, hipStream_t st);

// raster.hip
hipError_t launch_raster_fwd(const RasterArgs& a, hipStream_t st);
hipError_t launch_raster_mask(const int32_t* rec_taken, const int32_t* rec_gid,
                              const int32_t* rec_view, const int32_t* counters, int64_t cap,
                              int64_t mask_words, uint32_t* m_raster, hipStream_t st);
hipError_t launch_l1_loss(const float* color, const float* target, const int64_t* px_offset,
                          const int32_t* wh, int nv, int64_t total_px, float* loss,
                          float* d_color, hipStream_t st);

// backward.hip
hipError_t launch_zero_g2d(const BwdArgs& a, hipStream_t st);
hipError_t launch_raster_bwd(const BwdArgs& a, hipStream_t st);
hipError_t launch_project_bwd(const ProjBwdArgs& a, hipStream_t st);
// (also clears what launch_zero_g2d clears: a.g2d, a.zero_a, a.zero_b)
hipError_t launch_clear_rows(const int32_t* rows, const int32_t* n_rows, int64_t n, int B,
                             float* mean, float* scale, float* quat, float* opac, float* sh,
                             int64_t cap, const uint32_t* surv, int64_t mask_words, int nv,
                             const BwdArgs& a, hipStream_t st);

hipError_t launch_pose_bwd_det(const float* W, const int32_t* tstep, const float* pose,
                               const unsigned long long* d_cam_fx, int nv, int S, int T,
                               float* d_pose, float* d_pose6, hipStream_t st);
hipError_t launch_pose_bwd(const float* W, const int32_t* tstep, const float* pose,
                           const float* d_cam, int nv, int S, int T, float* d_pose,
                           float* d_pose6, hipStream_t st);
hipError_t launch_plain_transform_bwd(const float* mean, const float* quat, const int32_t* inst,
                                      const float* pose, int n, int S, const int32_t* tsteps,
                                      int n_ts, const float* d_mean_w, const float* d_rot_w,
                                      float* d_mean, float* d_quat, float* d_pose,
                                      float* d_pose6, hipStream_t st);

// visibility.hip
hipError_t launch_visibility(float* life_s, float* life_e, float* vis_s, float* vis_e,
                             const uint32_t* mask, const float* t_norm, int nv, int64_t n,
                             int mode, float margin, hipStream_t st);

}  // namespace s3r
