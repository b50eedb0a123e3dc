// Front-to-back alpha blending of Eq. (2) over every tile of every view in
// one launch.
//
// One thread per pixel; each wave64 owns an 8x8 sub-tile of its tile and
// walks the tile's sorted list independently of the other waves (no LDS, no
// barriers), so every wave is a workgroup of its own and a wave slot freed
// by a short sub-tile takes the next one at once (a workgroup of the whole
// tile would wait for four free slots on one CU).  Workgroups are dealt
// round-robin to the chip's kXcds dies, each with its own L2; the sub-tiles
// of a tile take workgroup ids congruent modulo kXcds, so they run on one die
// and read the tile's records through one L2, and tiles start in their
// launch order.  A batch of 64 entries is fetched
// lane-parallel; entries whose cutoff box misses the sub-tile (no pixel there
// could pass the Mahalanobis cut) are dropped with one ballot, and the rest
// are broadcast from their lane into scalar registers and blended in list
// order.  A wave stops once all its pixels reached the transmittance floor.
// Pixels are sampled at integer coordinates (x, y).
#include "internal.hpp"

namespace s3r {

template <int TS, int WPG>
__global__ __launch_bounds__(kWave * WPG)
__attribute__((amdgpu_waves_per_eu(8))) void k_raster_fwd(RasterArgs a) {
  constexpr int NW = RasterShape<TS>::NW;
  constexpr int G = NW / WPG;  // workgroups per tile
  // id = kXcds (G q + g) + x  ->  tile rank kXcds q + x, sub-tiles g WPG ..
  // g WPG + WPG - 1 (one per wave)
  const int xcd = (int)(blockIdx.x % kXcds), k = (int)(blockIdx.x / kXcds);
  const int rank = (k / G) * kXcds + xcd;
  if (rank >= a.total_tiles) return;  // padding of the last group of tiles
  const int lane = threadIdx.x % kWave;
  const int tid = ((k % G) * WPG + (int)(threadIdx.x / kWave)) * kWave + lane;  // pixel slot
  const int t = a.tile_order[rank];
  const int v = find_view(a.tile_offset, a.nv, t);
  const int lt = t - a.tile_offset[v];
  const int W = a.wh[2 * v], H = a.wh[2 * v + 1];
  const int gx = (W + TS - 1) / TS;
  int ox, oy, sx, sy;
  raster_pixel<TS>(tid, ox, oy, sx, sy);
  const int tx0 = (lt % gx) * TS, ty0 = (lt / gx) * TS;
  const int px = tx0 + ox, py = ty0 + oy;
  const float fxp = (float)px, fyp = (float)py;
  const float sub_x = (float)(tx0 + sx), sub_y = (float)(ty0 + sy);
  const bool inside = (px < W) && (py < H);
  const int64_t s = a.tile_start[t];
  const int64_t e = min((int64_t)a.tile_start[t + 1], a.kp.cap_dup);

  float T = 1.0f, cr = 0.f, cg = 0.f, cb = 0.f;
  bool done = !inside;
  int last = 0;
  unsigned long long n_eval = 0, n_blend = 0;  // work census (optional)
  // Each wave walks the tile's list on its own, 64 entries at a time: lane l
  // holds entry b0 + l, one ballot keeps the entries whose cutoff box meets
  // the wave's sub-tile, and those are broadcast lane by lane.  Loads are
  // pipelined: record ids two batches ahead, record fields one batch ahead.
  const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
  uint32_t rn = (s + lane < e) ? a.vals[s + lane] : 0u;
  float4 gn = zero4, cn = zero4, kn = zero4;
  if (s + lane < e) {
    gn = a.rec_geo[rn];
    cn = a.rec_conic[rn];
    kn = a.rec_rgb[rn];
  }
  uint32_t rcur = rn;  // record ids of the batch being blended
  rn = (s + kWave + lane < e) ? a.vals[s + kWave + lane] : 0u;
  for (int64_t b0 = s; b0 < e; b0 += kWave) {
    if (ballot(!done) == 0ull) break;
    const float4 g = gn, c = cn, col = kn;
    const uint32_t rb = rcur;
    const bool valid = b0 + lane < e;
    if (b0 + kWave + lane < e) {
      gn = a.rec_geo[rn];
      cn = a.rec_conic[rn];
      kn = a.rec_rgb[rn];
    }
    rcur = rn;
    rn = (b0 + 2 * kWave + lane < e) ? a.vals[b0 + 2 * kWave + lane] : 0u;
    const bool near =
        valid && box_hits(cutoff_box(g.x, g.y, c.x, c.y, c.z, a.kp.cutoff), sub_x, sub_y);
    uint64_t m = ballot(near);
    while (m != 0ull) {
      const int j = __builtin_ctzll(m);
      m &= m - 1ull;
      const float u = bcast(g.x, j), vv = bcast(g.y, j), o = bcast(g.z, j);
      const float A = bcast(c.x, j), B = bcast(c.y, j), C = bcast(c.z, j);
      const Blend bl = blend_eval(u, vv, A, B, C, o, fxp, fyp, a.kp);
      if (a.census) n_eval += __popcll(ballot(!done));
      const bool hit = bl.hit && !done;
      if (ballot(hit) == 0ull) continue;  // no pixel of the wave takes it
      const float kr = bcast(col.x, j), kg = bcast(col.y, j), kb = bcast(col.z, j);
      const float Tn = T * (1.0f - bl.alpha);
      const bool stop = Tn < a.kp.t_min;  // this entry would push T under the floor
      const bool take = hit && !stop;
      if (a.census) n_blend += __popcll(ballot(take));
      done = done || (hit && stop);
      const float w = bl.alpha * T;
      cr = take ? fmaf(kr, w, cr) : cr;
      cg = take ? fmaf(kg, w, cg) : cg;
      cb = take ? fmaf(kb, w, cb) : cb;
      T = take ? Tn : T;
      last = take ? (int)(b0 - s) + j + 1 : last;
      // rendering-derived visibility: mark the record (every writer stores 1)
      if (a.rec_taken && ballot(take) != 0ull && lane == 0)
        a.rec_taken[__builtin_amdgcn_readlane(rb, j)] = 1;
    }
  }
  if (a.census && lane == 0) {
    atomicAdd(a.census, n_eval);
    atomicAdd(a.census + 1, n_blend);
  }
  if (inside) {
    const int64_t npx = (int64_t)W * H;
    const int64_t p = (int64_t)py * W + px;
    const int64_t base = 3 * a.px_offset[v];
    a.color[base + p] = fmaf(T, a.kp.bg0, cr);
    a.color[base + npx + p] = fmaf(T, a.kp.bg1, cg);
    a.color[base + 2 * npx + p] = fmaf(T, a.kp.bg2, cb);
    a.T_final[a.px_offset[v] + p] = T;
    a.last[a.px_offset[v] + p] = last;
  }
}

// M_raster bits from the records the rasterizer marked (one atomic per record;
// a (view, Gaussian) pair has at most one record)
__global__ __launch_bounds__(256) void k_raster_mask(const int32_t* __restrict__ rec_taken,
                                                     const int32_t* __restrict__ rec_gid,
                                                     const int32_t* __restrict__ rec_view,
                                                     const int32_t* __restrict__ counters,
                                                     int64_t cap, int64_t mask_words,
                                                     uint32_t* __restrict__ m_raster) {
  const int64_t n = min((int64_t)counters[S3R_CNT_SURV], cap);
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    if (!rec_taken[r]) continue;
    const int i = rec_gid[r];
    atomicOr(m_raster + (size_t)rec_view[r] * mask_words + (i >> 5), 1u << (i & 31));
  }
}

hipError_t launch_raster_mask(const int32_t* rec_taken, const int32_t* rec_gid,
                              const int32_t* rec_view, const int32_t* counters, int64_t cap,
                              int64_t mask_words, uint32_t* m_raster, hipStream_t st) {
  const int64_t want = (cap + 255) / 256;
  const int grid = (int)(want < 2048 ? (want > 0 ? want : 1) : 2048);
  S3R_LAUNCH(K_RASTER_FWD, k_raster_mask, dim3(grid), dim3(256), 0, st, rec_taken, rec_gid,
             rec_view, counters, cap, mask_words, m_raster);
  return hipGetLastError();
}

template <int TS, int WPG>
static void launch_fwd_shape(const RasterArgs& a, unsigned groups, hipStream_t st) {
  constexpr int NW = RasterShape<TS>::NW;
  const dim3 grid(groups * kXcds * (unsigned)(NW / WPG));
  S3R_LAUNCH(K_RASTER_FWD, (k_raster_fwd<TS, WPG>), grid, dim3(kWave * WPG), 0, st, a);
}

// waves per workgroup: the largest power of two up to the knob and the tile's
// sub-tile count
template <int TS>
static void launch_fwd_tile(const RasterArgs& a, unsigned groups, hipStream_t st) {
  constexpr int NW = RasterShape<TS>::NW;
  const int want = min(tune(S3R_TUNE_RASTER_WAVES), NW);
  if constexpr (NW >= 16) {
    if (want >= 16) return launch_fwd_shape<TS, 16>(a, groups, st);
    if (want >= 8) return launch_fwd_shape<TS, 8>(a, groups, st);
  }
  if constexpr (NW >= 4) {
    if (want >= 4) return launch_fwd_shape<TS, 4>(a, groups, st);
    if (want >= 2) return launch_fwd_shape<TS, 2>(a, groups, st);
  }
  launch_fwd_shape<TS, 1>(a, groups, st);
}

hipError_t launch_raster_fwd(const RasterArgs& a, hipStream_t st) {
  if (a.total_tiles <= 0) return hipSuccess;
  // tiles padded to a multiple of kXcds; the sub-tiles of a tile take
  // workgroup ids congruent modulo kXcds (one L2)
  const unsigned groups = ((unsigned)a.total_tiles + kXcds - 1) / kXcds;
  switch (a.kp.tile) {
    case 8: launch_fwd_tile<8>(a, groups, st); break;
    case 16: launch_fwd_tile<16>(a, groups, st); break;
    case 32: launch_fwd_tile<32>(a, groups, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-view mean absolute error and its gradient
// ---------------------------------------------------------------------------
// Each workgroup takes one contiguous range of pixels, so a thread's view
// changes rarely; per-thread sums are reduced over the wave when its lanes
// share a view, then per workgroup, and a workgroup adds one value per view it
// touched to the loss (few same-address atomics: they serialise).
// 1024 threads per workgroup: the ~512 workgroups of a 1080p view then fill
// every wave slot of the chip, with one 4-pixel group per thread
constexpr int kL1Threads = 1024;

__device__ __forceinline__ float l1_sign(float d, float inv) {
  return d > 0.f ? inv : (d < 0.f ? -inv : 0.f);
}

__global__ __launch_bounds__(kL1Threads) void k_l1(const float* __restrict__ color,
                                            const float* __restrict__ target,
                                            const int64_t* __restrict__ pxo,
                                            const int32_t* __restrict__ wh, int nv, int64_t total,
                                            int64_t chunk, float* __restrict__ loss,
                                            float* __restrict__ dcol) {
  __shared__ float s_loss[kMaxViews];
  for (int v = threadIdx.x; v < nv; v += blockDim.x) s_loss[v] = 0.f;
  // with every view's pixel count a multiple of 4, planes and view offsets
  // are 16-byte aligned and a thread takes 4 pixels with float4 accesses
  bool vec = true;
  for (int v = 0; v < nv; ++v) vec = vec && (((int64_t)wh[2 * v] * wh[2 * v + 1]) % 4 == 0);
  __syncthreads();
  const int step = vec ? 4 : 1;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = min(total, lo + chunk);
  int cur = 0;
  while (cur + 1 < nv && pxo[cur + 1] <= lo) ++cur;
  int64_t vend = cur + 1 < nv ? pxo[cur + 1] : total;
  int64_t npx = (int64_t)wh[2 * cur] * wh[2 * cur + 1];
  int64_t vb = pxo[cur];
  float inv = 1.0f / (3.0f * (float)npx);
  float acc = 0.f;
  for (int64_t i = lo + (int64_t)threadIdx.x * step; i < hi; i += (int64_t)blockDim.x * step) {
    if (i >= vend) {
      atomicAdd(&s_loss[cur], acc);
      acc = 0.f;
      while (cur + 1 < nv && pxo[cur + 1] <= i) ++cur;
      vend = cur + 1 < nv ? pxo[cur + 1] : total;
      npx = (int64_t)wh[2 * cur] * wh[2 * cur + 1];
      vb = pxo[cur];
      inv = 1.0f / (3.0f * (float)npx);
    }
    const int64_t loc = i - vb;
    float a = 0.f;
    if (vec) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int64_t q = (3 * vb + c * npx + loc) / 4;
        const float4 x = reinterpret_cast<const float4*>(color)[q];
        const float4 t = reinterpret_cast<const float4*>(target)[q];
        const float4 d = make_float4(x.x - t.x, x.y - t.y, x.z - t.z, x.w - t.w);
        a += (fabsf(d.x) + fabsf(d.y)) + (fabsf(d.z) + fabsf(d.w));
        reinterpret_cast<float4*>(dcol)[q] =
            make_float4(l1_sign(d.x, inv), l1_sign(d.y, inv), l1_sign(d.z, inv), l1_sign(d.w, inv));
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int64_t q = 3 * vb + c * npx + loc;
        const float d = color[q] - target[q];
        a += fabsf(d);
        dcol[q] = l1_sign(d, inv);
      }
    }
    acc += a * inv;
  }
  const int c0 = __shfl(cur, 0, kWave);
  if (ballot(cur != c0) == 0ull) {
    acc = wave_sum_dpp(acc);
    if ((threadIdx.x % kWave) == kWave - 1) atomicAdd(&s_loss[cur], acc);
  } else {
    atomicAdd(&s_loss[cur], acc);
  }
  __syncthreads();
  for (int v = threadIdx.x; v < nv; v += blockDim.x)
    if (s_loss[v] != 0.f) atomicAdd(loss + v, s_loss[v]);
}

hipError_t launch_l1_loss(const float* color, const float* target, const int64_t* px_offset,
                          const int32_t* wh, int nv, int64_t total_px, float* loss,
                          float* d_color, hipStream_t st) {
  hipError_t e = launch_zero(loss, (size_t)nv * 4, nullptr, 0, nullptr, 0, nullptr, 0, st);
  if (e != hipSuccess) return e;
  if (total_px <= 0) return hipGetLastError();
  // about 512 workgroups of kL1Threads threads, each over a contiguous range
  // (a multiple of 1024 pixels, so 4-pixel groups never straddle chunks)
  const int64_t chunk = max((int64_t)256 * 8, ((total_px + 511) / 512 + 1023) / 1024 * 1024);
  const int64_t grid = (total_px + chunk - 1) / chunk;
  S3R_LAUNCH(K_L1, k_l1, dim3((unsigned)grid), dim3(kL1Threads), 0, st, color, target, px_offset, wh, nv,
             total_px, chunk, loss, d_color);
  return hipGetLastError();
}

}  // namespace s3r
