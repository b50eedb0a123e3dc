// Front-to-back alpha blending of Eq. (2) over every tile of every view in
// one launch.
//
// One thread per pixel; each wave64 owns an 8x8 sub-tile of its tile and
// walks the tile's sorted list independently of the other waves (no
// barriers), so every wave is a workgroup of its own and a wave slot freed
// by a short sub-tile takes the next one at once (a workgroup of the whole
// tile would wait for four free slots on one CU).  Workgroups are dealt
// round-robin to the chip's kXcds dies, each with its own L2; the sub-tiles
// of a tile take workgroup ids congruent modulo kXcds, so they run on one die
// and read the tile's records through one L2, and tiles start in their
// launch order.  A batch of 64 entries is fetched
// lane-parallel; entries whose cutoff box misses the sub-tile (no pixel there
// could pass the Mahalanobis cut) are dropped with one ballot, and the rest
// are compacted into wave-private LDS rows and blended in list order, each
// read back with one broadcast load per field (no per-field lane reads on
// the vector ALU, which bounds this kernel).  A wave stops once all its
// pixels reached the transmittance floor.
// Pixels are sampled at integer coordinates (x, y).
#include "internal.hpp"

namespace s3r {

constexpr int kFwdRun = 4;  // consecutive launch-order tiles per XCD

template <int TS, int WPG, bool EXTRA>
__global__ __launch_bounds__(kWave * WPG)
__attribute__((amdgpu_waves_per_eu(8))) void k_raster_fwd(RasterArgs a, int n_fine) {
  constexpr int NW = RasterShape<TS>::NW;
  constexpr int G = NW / WPG;                    // workgroups per tile (8x8 sub-tiles)
  constexpr int GF = (TS / 4) * (TS / 4) / WPG;  // workgroups per tile (4x4 blocks)
  // the entries of the batch being blended that meet the wave's pixels,
  // compacted in list order (wave-private: written and read by one wave)
  __shared__ float4 s_geo[WPG][kWave];  // u, v, opacity, record id (bits)
  __shared__ float4 s_con[WPG][kWave];  // conic A, B, C, -
  __shared__ float4 s_rgb[WPG][kWave];  // colour, list position (bits)
  // The n_fine first tiles of the launch order (the longest lists; n_fine is
  // a multiple of kXcds kFwdRun) take one wave per 4x4 block, 16 lanes busy: a wave
  // then walks only the entries near its block, which shortens the longest
  // waves of the launch.  The other tiles take one wave per 8x8 sub-tile.
  // id = kXcds (G q + g) + x  ->  the q-th tile of XCD x, waves g WPG ..
  // g WPG + WPG - 1 (ids of the 4x4 part first, GF in place of G); an XCD
  // takes runs of kFwdRun consecutive launch-order ranks (neighbouring tiles
  // of a length bucket share records in its L2), the runs dealt round-robin
  // to the XCDs, so the longest lists still start first on every XCD
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const unsigned fine_ids = (unsigned)n_fine * GF;
  const bool fine = blockIdx.x < fine_ids;
  const unsigned id = fine ? blockIdx.x : blockIdx.x - fine_ids;
  const int xcd = (int)(id % kXcds), k = (int)(id / kXcds);
  const int per = fine ? GF : G;
  const int q = k / per;
  const int rank = (fine ? 0 : n_fine) + (q / kFwdRun) * (kXcds * kFwdRun) + xcd * kFwdRun +
                   q % kFwdRun;
  if (rank >= (fine ? n_fine : a.total_tiles)) return;  // padding of the last round
  const int sub = (k % per) * WPG + wv;  // the wave's sub-tile or block
  const int t = a.tile_order[rank];
  const int v = find_view(a.tile_offset, a.nv, t);
  const int lt = t - a.tile_offset[v];
  const int W = a.wh[2 * v], H = a.wh[2 * v + 1];
  const int gx = (W + TS - 1) / TS;
  int ox, oy, sx, sy;
  if (fine) {
    sx = 4 * (sub % (TS / 4));
    sy = 4 * (sub / (TS / 4));
    ox = sx + lane % 4;
    oy = sy + (lane / 4) % 4;
  } else {
    raster_pixel<TS>(sub * kWave + lane, ox, oy, sx, sy);
  }
  const float ext = fine ? 3.f : 7.f;  // the wave's pixels: [sub, sub + ext]^2
  const int tx0 = (lt % gx) * TS, ty0 = (lt / gx) * TS;
  const int px = tx0 + ox, py = ty0 + oy;
  const float fxp = (float)px, fyp = (float)py;
  const float sub_x = (float)(tx0 + sx), sub_y = (float)(ty0 + sy);
  const bool inside = (px < W) && (py < H) && (!fine || lane < 16);
  const int64_t s = a.tile_start[t];
  const int64_t e = min((int64_t)a.tile_start[t + 1], a.kp.cap_dup);

  float T = 1.0f, cr = 0.f, cg = 0.f, cb = 0.f;
  bool done = !inside;
  int last = 0;
  unsigned long long n_eval = 0, n_blend = 0;  // work census (optional)
  // Each wave walks the tile's list on its own, 64 entries at a time: lane l
  // holds entry b0 + l, one ballot keeps the entries whose cutoff box meets
  // the wave's sub-tile, and those are compacted into the wave's LDS rows and
  // read back one by one (a broadcast read: every lane the same address).
  // Loads are pipelined: record ids two batches ahead, record fields one
  // batch ahead.
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
    // (a 4x4 block's box test is nearly as tight as the square test, which
    // then costs more than the entries it drops: coarse waves only)
    const bool near =
        valid && box_hits(cutoff_box(g.x, g.y, make_float2(c.w, col.w)), sub_x, sub_y, ext) &&
        (fine || square_may_hit(g.x, g.y, c.x, c.y, c.z, g.z, sub_x, sub_y, ext, a.kp));
    const uint64_t m = ballot(near);
    const int n = __popcll(m);
    if (near) {
      const int slot = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
      s_geo[wv][slot] = make_float4(g.x, g.y, g.z, __int_as_float((int)rb));
      s_con[wv][slot] = c;
      // colour, and the entry's 1-based list position (the pixel's `last`
      // once it blends the entry)
      s_rgb[wv][slot] = make_float4(col.x, col.y, col.z, __int_as_float((int)(b0 - s) + lane + 1));
    }
    // (the batch's entries are blended to the end even if every pixel of the
    // wave stops on the way: a per-entry exit test costs more than the rare
    // tail it saves)
    for (int j = 0; j < n; ++j) {
      const float4 eg = s_geo[wv][j], ec = s_con[wv][j], ek = s_rgb[wv][j];
      const Blend bl = blend_eval(eg.x, eg.y, ec.x, ec.y, ec.z, eg.z, fxp, fyp, a.kp);
      if (EXTRA && a.census) n_eval += __popcll(ballot(!done));
      const bool hit = bl.hit && !done;
      const float Tn = T * (1.0f - bl.alpha);
      const bool stop = Tn < a.kp.t_min;  // this entry would push T under the floor
      const bool take = hit && !stop;
      done = done || (hit && stop);
      const float w = take ? bl.alpha * T : 0.f;
      cr = fmaf(ek.x, w, cr);
      cg = fmaf(ek.y, w, cg);
      cb = fmaf(ek.z, w, cb);
      T = take ? Tn : T;
      last = take ? __float_as_int(ek.w) : last;
      if (EXTRA) {
        if (a.census) n_blend += __popcll(ballot(take));
        // rendering-derived visibility: mark the record (every writer stores 1)
        if (a.rec_taken && ballot(take) != 0ull && lane == 0)
          a.rec_taken[__float_as_int(eg.w)] = 1;
      }
    }
  }
  if (EXTRA && a.census && lane == 0) {
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
static void launch_fwd_shape(const RasterArgs& a, hipStream_t st) {
  constexpr int NW = RasterShape<TS>::NW, NB = (TS / 4) * (TS / 4);
  // tiles in 4x4 blocks: a multiple of kXcds kFwdRun, at most the tile count
  const int n_fine =
      min(tune(S3R_TUNE_FINE_TILES), a.total_tiles) / (kXcds * kFwdRun) * (kXcds * kFwdRun);
  // the other tiles padded to whole rounds of kXcds kFwdRun
  const unsigned round = kXcds * kFwdRun;
  const unsigned groups = ((unsigned)(a.total_tiles - n_fine) + round - 1) / round * kFwdRun;
  const dim3 grid((unsigned)n_fine * (NB / WPG) + groups * kXcds * (unsigned)(NW / WPG));
  if (a.census || a.rec_taken)
    S3R_LAUNCH(K_RASTER_FWD, (k_raster_fwd<TS, WPG, true>), grid, dim3(kWave * WPG), 0, st, a,
               n_fine);
  else
    S3R_LAUNCH(K_RASTER_FWD, (k_raster_fwd<TS, WPG, false>), grid, dim3(kWave * WPG), 0, st, a,
               n_fine);
}

// waves per workgroup: the largest power of two up to the knob and the tile's
// sub-tile count
template <int TS>
static void launch_fwd_tile(const RasterArgs& a, hipStream_t st) {
  constexpr int NW = RasterShape<TS>::NW;
  const int want = min(tune(S3R_TUNE_RASTER_WAVES), NW);
  if constexpr (NW >= 16) {
    if (want >= 16) return launch_fwd_shape<TS, 16>(a, st);
    if (want >= 8) return launch_fwd_shape<TS, 8>(a, st);
  }
  if constexpr (NW >= 4) {
    if (want >= 4) return launch_fwd_shape<TS, 4>(a, st);
    if (want >= 2) return launch_fwd_shape<TS, 2>(a, st);
  }
  launch_fwd_shape<TS, 1>(a, st);
}

hipError_t launch_raster_fwd(const RasterArgs& a, hipStream_t st) {
  if (a.total_tiles <= 0) return hipSuccess;
  // the waves of a tile take workgroup ids congruent modulo kXcds (one L2)
  switch (a.kp.tile) {
    case 8: launch_fwd_tile<8>(a, st); break;
    case 16: launch_fwd_tile<16>(a, st); break;
    case 32: launch_fwd_tile<32>(a, st); break;
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
