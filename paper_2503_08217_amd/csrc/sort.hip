// Per-tile contributor lists in the blending order of Eq. (2).
//
// The order is ascending (depth bits, Gaussian index) within every tile.  A
// record's index increases with the Gaussian index within a view and every
// tile belongs to one view, so the 64-bit key (depth bits << 32 | record) is
// unique and sorts exactly like (depth, Gaussian index).  Instead of a global
// radix sort over (tile, depth, id) the lists are built as buckets:
//   1. k_bin<count>: each workgroup takes the records of one view from a
//      chunk of Gaussian blocks and counts the tiles they cover in an LDS
//      histogram, then adds the touched bins to the global tile counts (one
//      global atomic per touched tile per chunk, so crowded tiles near the
//      horizon cost no more than quiet ones)
//   2. exclusive scan of the tile counts (single pass, decoupled look-back)
//   3. k_bin<emit>: the same histogram reserves each touched tile's range with
//      one global atomic; every key then takes its slot with an LDS atomic
//   4. one workgroup per tile sorts its bucket in LDS (bitonic network);
//      buckets larger than the LDS tile are sorted in 4096-key chunks by many
//      workgroups and merged with merge-path passes, also spread over the GPU.
#include "internal.hpp"

namespace s3r {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

int scan_blocks(int64_t n) { return (int)((n + kScanTile - 1) / kScanTile); }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t t = __shfl_up(x, o, kWave);
    if (lane >= o) x += t;
  }
  return x;
}

// exclusive scan of tile_count -> tile_start, total written to counters
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(
    const int32_t* __restrict__ cnt, int n, int32_t* __restrict__ start,
    uint64_t* __restrict__ flags, int32_t* __restrict__ counters, int64_t cap_dup, int nblk) {
  __shared__ int s_vb;
  __shared__ uint32_t s_wsum[kScanThreads / kWave];
  __shared__ uint32_t s_excl;
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  if (tid == 0) s_vb = atomicAdd(&counters[S3R_CNT_TICKET2], 1);
  __syncthreads();
  const int vb = s_vb;
  const int64_t base = (int64_t)vb * kScanTile + (int64_t)tid * kScanItems;
  uint32_t v[kScanItems];
  uint32_t tsum = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const int64_t idx = base + q;
    v[q] = idx < n ? (uint32_t)cnt[idx] : 0u;
    tsum += v[q];
  }
  const uint32_t incl = wave_incl_scan(tsum);
  if (lane == kWave - 1) s_wsum[wave] = incl;
  __syncthreads();
  if (wave == 0) {
    uint32_t agg_l = 0;
    if (lane == 0) {
      for (int w = 0; w < kScanThreads / kWave; ++w) agg_l += s_wsum[w];
      st_release(flags + vb, ((uint64_t)(vb == 0 ? 2u : 1u) << 32) | agg_l);
    }
    const uint32_t agg = __shfl(agg_l, 0, kWave);
    uint32_t excl = 0;
    if (vb > 0) excl = lookback(flags, vb, counters + S3R_CNT_SPIN);
    if (lane == 0) {
      if (vb > 0) st_release(flags + vb, (2ull << 32) | (uint64_t)(excl + agg));
      s_excl = excl;
      if (vb == nblk - 1) {
        const int64_t total = (int64_t)excl + agg;
        start[n] = (int32_t)total;
        counters[S3R_CNT_DUP] = (int32_t)(total < cap_dup ? total : cap_dup);
        counters[S3R_CNT_OVF_DUP] = (int32_t)(total > cap_dup ? total - cap_dup : 0);
      }
    }
  }
  __syncthreads();
  uint32_t run = s_excl + (incl - tsum);
  for (int w = 0; w < wave; ++w) run += s_wsum[w];
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const int64_t idx = base + q;
    if (idx < n) start[idx] = (int32_t)run;
    run += v[q];
  }
}

__global__ void k_dup_stats(const int32_t* __restrict__ start, const int32_t* __restrict__ toff,
                            int nv, int32_t* __restrict__ stats) {
  const int v = threadIdx.x;
  if (v < nv) stats[v * 4 + 3] = start[toff[v + 1]] - start[toff[v]];
}

// ---------------------------------------------------------------------------
// binning: LDS histogram of the tiles covered by one view's records of a chunk
// of Gaussian blocks, processed in windows of kBinWindow tiles
// ---------------------------------------------------------------------------
constexpr int kBinThreads = 256;
constexpr int kBinWindow = 8192;
constexpr int kChunkBlocks = 16;

template <bool EMIT>
__global__ __launch_bounds__(kBinThreads) void k_bin(SortArgs a) {
  __shared__ uint32_t hist[kBinWindow];
  __shared__ uint16_t touched[kBinWindow];
  __shared__ int n_touched;
  __shared__ int s_start[kChunkBlocks], s_pref[kChunkBlocks + 1];
  const int tid = threadIdx.x;
  const int v = blockIdx.y;
  const int b0 = blockIdx.x * kChunkBlocks;
  const int b1 = min(b0 + kChunkBlocks, a.nblk);
  if (tid == 0) {
    // the chunk's records of view v, as one index range over its blocks
    int run = 0;
    for (int b = b0; b < b0 + kChunkBlocks; ++b) {
      s_pref[b - b0] = run;
      int cnt = 0, st = 0;
      if (b < b1) {
        const int4 info = reinterpret_cast<const int4*>(a.blocks)[(size_t)b * a.nv + v];
        const int64_t room = a.cap_surv - info.w;
        cnt = (int)min((int64_t)info.z, room > 0 ? room : 0);
        st = info.w;
      }
      s_start[b - b0] = st;
      run += cnt;
    }
    s_pref[kChunkBlocks] = run;
  }
  __syncthreads();
  const int total = s_pref[kChunkBlocks];
  const int W = a.wh[2 * v], H = a.wh[2 * v + 1];
  const int gx = (W + a.tile - 1) / a.tile;
  const int gy = (H + a.tile - 1) / a.tile;
  const int ntiles = gx * gy;
  const int tb = a.tile_offset[v];
  for (int w0 = 0; w0 < ntiles; w0 += kBinWindow) {
    const int w1 = min(w0 + kBinWindow, ntiles);
    for (int i = tid; i < w1 - w0; i += kBinThreads) hist[i] = 0u;
    if (tid == 0) n_touched = 0;
    __syncthreads();
    for (int j = tid; j < total; j += kBinThreads) {
      {
        int b = 0;
        while (s_pref[b + 1] <= j) ++b;
        const int4 rc = a.rec_rect[s_start[b] + (j - s_pref[b])];
        const int ty0 = max(rc.y, w0 / gx), ty1 = min(rc.w, (w1 + gx - 1) / gx);
        for (int ty = ty0; ty < ty1; ++ty) {
          for (int tx = rc.x; tx < rc.z; ++tx) {
            const int tl = ty * gx + tx;
            if (tl < w0 || tl >= w1) continue;
            const uint32_t old = atomicAdd(&hist[tl - w0], 1u);
            if (old == 0u) touched[atomicAdd(&n_touched, 1)] = (uint16_t)(tl - w0);
          }
        }
      }
    }
    __syncthreads();
    const int nt = n_touched;
    if (!EMIT) {
      for (int k = tid; k < nt; k += kBinThreads) {
        const int tl = touched[k];
        atomicAdd(a.tile_count + tb + w0 + tl, (int)hist[tl]);
      }
    } else {
      for (int k = tid; k < nt; k += kBinThreads) {
        const int tl = touched[k];
        const int t = tb + w0 + tl;
        hist[tl] = (uint32_t)a.tile_start[t] + (uint32_t)atomicAdd(a.cursor + t, (int)hist[tl]);
      }
      __syncthreads();
      for (int j = tid; j < total; j += kBinThreads) {
        {
          int b = 0;
          while (s_pref[b + 1] <= j) ++b;
          const int r = s_start[b] + (j - s_pref[b]);
          const int4 rc = a.rec_rect[r];
          const uint64_t key = ((uint64_t)__float_as_uint(a.rec_geo[r].w) << 32) | (uint32_t)r;
          const int ty0 = max(rc.y, w0 / gx), ty1 = min(rc.w, (w1 + gx - 1) / gx);
          for (int ty = ty0; ty < ty1; ++ty) {
            for (int tx = rc.x; tx < rc.z; ++tx) {
              const int tl = ty * gx + tx;
              if (tl < w0 || tl >= w1) continue;
              const uint32_t pos = atomicAdd(&hist[tl - w0], 1u);
              if ((int64_t)pos < a.cap_dup) a.keys[pos] = key;
            }
          }
        }
      }
    }
    __syncthreads();
  }
  (void)gy;
}

// ---------------------------------------------------------------------------
// per-tile sort
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortCap = 4096;  // keys sorted in LDS at once (32 KiB)
constexpr int kMergePer = kSortCap / kSortThreads;  // outputs per thread in a merge pass

__device__ __forceinline__ void bitonic_lds(uint64_t* sk, int P) {
  const int tid = threadIdx.x;
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < (P >> 1); i += kSortThreads) {
        const int lo = 2 * i - (i & (j - 1));
        const int hi = lo + j;
        const bool up = (lo & k) == 0;
        const uint64_t x = sk[lo], y = sk[hi];
        if ((x > y) == up) {
          sk[lo] = y;
          sk[hi] = x;
        }
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ int next_pow2(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// tiles up to kSortCap keys are sorted here; larger ones are listed for the
// chunked path (big[0] = count, big[4 + i] = tile)
__global__ __launch_bounds__(kSortThreads) void k_tile_sort(const int32_t* __restrict__ start,
                                                            const uint64_t* __restrict__ keys,
                                                            uint32_t* __restrict__ vals,
                                                            int32_t* __restrict__ big,
                                                            int64_t cap_dup) {
  __shared__ uint64_t sk[kSortCap];
  const int t = blockIdx.x;
  const int64_t s = start[t];
  const int64_t e = min((int64_t)start[t + 1], cap_dup);
  if (e <= s) return;
  const int n = (int)(e - s);
  if (n == 1) {
    if (threadIdx.x == 0) vals[s] = (uint32_t)keys[s];
    return;
  }
  if (n > kSortCap) {
    if (threadIdx.x == 0) big[4 + atomicAdd(big, 1)] = t;
    return;
  }
  const int P = next_pow2(n);
  for (int i = threadIdx.x; i < P; i += kSortThreads) sk[i] = i < n ? keys[s + i] : ~0ull;
  __syncthreads();
  bitonic_lds(sk, P);
  for (int i = threadIdx.x; i < n; i += kSortThreads) vals[s + i] = (uint32_t)sk[i];
}

__device__ __forceinline__ int log2_ceil(int x) {
  int p = 0;
  while ((1 << p) < x) ++p;
  return p;
}

// chunk offsets of the big tiles: off[i] = sum_{j<i} ceil(n_j / kSortCap);
// big[1] = total chunks, big[2] = merge passes the largest tile needs
__global__ __launch_bounds__(256) void k_big_prefix(const int32_t* __restrict__ start,
                                                    int32_t* __restrict__ big, int total_tiles,
                                                    int64_t cap_dup) {
  __shared__ uint32_t s_w[4];
  __shared__ int s_pass[4];
  const int nbig = big[0];
  int32_t* list = big + 4;
  int32_t* off = big + 4 + total_tiles;
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const int per = (nbig + 255) / 256;
  const int i0 = tid * per, i1 = min(nbig, i0 + per);
  uint32_t sum = 0;
  int passes = 0;
  for (int i = i0; i < i1; ++i) {
    const int t = list[i];
    const int n = (int)(min((int64_t)start[t + 1], cap_dup) - start[t]);
    const int c = (n + kSortCap - 1) / kSortCap;
    sum += c;
    passes = max(passes, log2_ceil(c));
  }
  const uint32_t incl = wave_incl_scan(sum);
  int pm = passes;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) pm = max(pm, __shfl_xor(pm, o, kWave));
  if (lane == kWave - 1) s_w[wave] = incl;
  if (lane == 0) s_pass[wave] = pm;
  __syncthreads();
  uint32_t run = incl - sum;
  for (int w = 0; w < wave; ++w) run += s_w[w];
  for (int i = i0; i < i1; ++i) {
    off[i] = (int32_t)run;
    const int t = list[i];
    const int n = (int)(min((int64_t)start[t + 1], cap_dup) - start[t]);
    run += (n + kSortCap - 1) / kSortCap;
  }
  if (tid == 0) {
    uint32_t tot = 0;
    int pmax = 0;
    for (int w = 0; w < 4; ++w) {
      tot += s_w[w];
      pmax = max(pmax, s_pass[w]);
    }
    off[nbig] = (int32_t)tot;
    big[1] = (int32_t)tot;
    big[2] = pmax;
  }
}

struct BigItem {
  int64_t s;  // first key of the tile
  int n;      // keys in the tile
  int c;      // chunk (segment) index within the tile
};

__device__ __forceinline__ BigItem big_item(const int32_t* __restrict__ start,
                                            const int32_t* __restrict__ big, int total_tiles,
                                            int64_t cap_dup, int w) {
  const int nbig = big[0];
  const int32_t* off = big + 4 + total_tiles;
  int lo = 0, hi = nbig - 1;
  while (lo < hi) {  // last i with off[i] <= w
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= w) lo = mid;
    else hi = mid - 1;
  }
  const int t = big[4 + lo];
  BigItem it;
  it.s = start[t];
  it.n = (int)(min((int64_t)start[t + 1], cap_dup) - it.s);
  it.c = w - off[lo];
  return it;
}

__global__ __launch_bounds__(kSortThreads) void k_big_chunks(const int32_t* __restrict__ start,
                                                             const int32_t* __restrict__ big,
                                                             int total_tiles, int64_t cap_dup,
                                                             uint64_t* __restrict__ keys) {
  __shared__ uint64_t sk[kSortCap];
  const int total = big[1];
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const BigItem it = big_item(start, big, total_tiles, cap_dup, w);
    uint64_t* src = keys + it.s + (int64_t)it.c * kSortCap;
    const int m = min(kSortCap, it.n - it.c * kSortCap);
    const int P = next_pow2(m);
    for (int i = threadIdx.x; i < P; i += kSortThreads) sk[i] = i < m ? src[i] : ~0ull;
    __syncthreads();
    bitonic_lds(sk, P);
    for (int i = threadIdx.x; i < m; i += kSortThreads) src[i] = sk[i];
    __syncthreads();
  }
}

// merge pass p: sorted runs of kSortCap << p keys -> runs of twice that;
// a tile whose keys already form one run is left alone
__global__ __launch_bounds__(kSortThreads) void k_big_merge(const int32_t* __restrict__ start,
                                                            const int32_t* __restrict__ big,
                                                            int total_tiles, int64_t cap_dup,
                                                            int pass, uint64_t* __restrict__ k0,
                                                            uint64_t* __restrict__ k1) {
  if (pass >= big[2]) return;
  const int total = big[1];
  const int width = kSortCap << pass;
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const BigItem it = big_item(start, big, total_tiles, cap_dup, w);
    if (width >= it.n) continue;
    const uint64_t* src = ((pass & 1) ? k1 : k0) + it.s;
    uint64_t* dst = ((pass & 1) ? k0 : k1) + it.s;
    int o = it.c * kSortCap + threadIdx.x * kMergePer;
    const int end = min(it.n, o + kMergePer);
    if (o >= end) continue;
    const int p0 = (o / (2 * width)) * (2 * width);
    const int a0 = p0, a1 = min(p0 + width, it.n);
    const int b0 = a1, b1 = min(p0 + 2 * width, it.n);
    const int la = a1 - a0, lb = b1 - b0;
    const int d = o - p0;
    int lo = max(0, d - lb), hi = min(d, la);
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (src[a0 + mid] < src[b0 + d - mid - 1]) lo = mid + 1;
      else hi = mid;
    }
    int i = lo, j = d - lo;
    while (o < end) {
      const bool take_a = (j >= lb) || (i < la && src[a0 + i] < src[b0 + j]);
      dst[o++] = take_a ? src[a0 + i++] : src[b0 + j++];
    }
  }
}

__global__ __launch_bounds__(kSortThreads) void k_big_final(const int32_t* __restrict__ start,
                                                            const int32_t* __restrict__ big,
                                                            int total_tiles, int64_t cap_dup,
                                                            const uint64_t* __restrict__ k0,
                                                            const uint64_t* __restrict__ k1,
                                                            uint32_t* __restrict__ vals) {
  const int total = big[1];
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const BigItem it = big_item(start, big, total_tiles, cap_dup, w);
    const int passes = log2_ceil((it.n + kSortCap - 1) / kSortCap);
    const uint64_t* src = ((passes & 1) ? k1 : k0) + it.s;
    const int c0 = it.c * kSortCap, c1 = min(it.n, c0 + kSortCap);
    for (int i = c0 + threadIdx.x; i < c1; i += kSortThreads) vals[it.s + i] = (uint32_t)src[i];
  }
}

size_t sort_big_words(int total_tiles) { return 8 + 2 * (size_t)total_tiles; }

hipError_t launch_sort(const SortArgs& a, hipStream_t st) {
  const int nscan = scan_blocks(a.total_tiles);
  hipError_t e = launch_zero(a.scan_flags, (size_t)nscan * 8, a.cursor, (size_t)a.total_tiles * 4,
                             a.counters + S3R_CNT_TICKET2, 4, a.tile_count,
                             (size_t)a.total_tiles * 4, st);
  if (e != hipSuccess) return e;
  e = launch_zero(a.big, 16, nullptr, 0, nullptr, 0, nullptr, 0, st);
  if (e != hipSuccess) return e;
  const dim3 bgrid((a.nblk + kChunkBlocks - 1) / kChunkBlocks, a.nv);
  if (a.nblk > 0) S3R_LAUNCH(K_BIN_COUNT, k_bin<false>, bgrid, dim3(kBinThreads), 0, st, a);
  S3R_LAUNCH(K_SCAN_TILES, k_scan_tiles, dim3(nscan), dim3(kScanThreads), 0, st, a.tile_count,
                     a.total_tiles, a.tile_start, a.scan_flags, a.counters, a.cap_dup, nscan);
  S3R_LAUNCH(K_DUP_STATS, k_dup_stats, dim3(1), dim3(64), 0, st, a.tile_start, a.tile_offset, a.nv,
                     a.stats);
  if (a.nblk > 0) S3R_LAUNCH(K_BIN_EMIT, k_bin<true>, bgrid, dim3(kBinThreads), 0, st, a);
  S3R_LAUNCH(K_TILE_SORT, k_tile_sort, dim3(a.total_tiles), dim3(kSortThreads), 0, st, a.tile_start,
                     a.keys, a.vals, a.big, a.cap_dup);
  S3R_LAUNCH(K_BIG_PREFIX, k_big_prefix, dim3(1), dim3(256), 0, st, a.tile_start, a.big, a.total_tiles,
                     a.cap_dup);
  const int grid = 1024;
  S3R_LAUNCH(K_BIG_CHUNKS, k_big_chunks, dim3(grid), dim3(kSortThreads), 0, st, a.tile_start, a.big,
                     a.total_tiles, a.cap_dup, a.keys);
  int max_pass = 0;
  while (((int64_t)kSortCap << max_pass) < a.cap_dup) ++max_pass;
  for (int p = 0; p < max_pass; ++p)
    S3R_LAUNCH(K_BIG_MERGE, k_big_merge, dim3(grid), dim3(kSortThreads), 0, st, a.tile_start, a.big,
                       a.total_tiles, a.cap_dup, p, a.keys, a.keys_alt);
  S3R_LAUNCH(K_BIG_FINAL, k_big_final, dim3(grid), dim3(kSortThreads), 0, st, a.tile_start, a.big,
                     a.total_tiles, a.cap_dup, a.keys, a.keys_alt, a.vals);
  return hipGetLastError();
}

}  // namespace s3r
