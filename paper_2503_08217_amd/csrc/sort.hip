// Per-tile contributor lists in the blending order of Eq. (2).
//
// The order is ascending (depth bits, Gaussian index) within every tile.  A
// record's index increases with the Gaussian index within a view and every
// tile belongs to one view, so the 64-bit key (depth bits << 32 | record) is
// unique and sorts exactly like (depth, Gaussian index).  Instead of a global
// radix sort over (tile, depth, id) the lists are built as buckets:
//   1. exclusive scan of the per-tile pair counts (single pass, look-back)
//   2. every record scatters its key into the buckets of the tiles it covers
//   3. one workgroup per tile sorts its bucket in LDS (bitonic network); a
//      bucket larger than the LDS tile is sorted in chunks and merged with
//      merge-path passes by the same workgroup.
// Each pair is written once and read/written once by the per-tile sort.
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

// every record scatters (depth bits << 32 | record) into its tiles' buckets
__global__ __launch_bounds__(256) void k_emit(const int4* __restrict__ rect,
                                              const float4* __restrict__ geo,
                                              const int32_t* __restrict__ view,
                                              const int32_t* __restrict__ toff,
                                              const int32_t* __restrict__ wh, int tile,
                                              const int32_t* __restrict__ start,
                                              int32_t* __restrict__ cursor,
                                              const int32_t* __restrict__ counters,
                                              uint64_t* __restrict__ keys, int64_t cap_dup) {
  const int nrec = counters[S3R_CNT_SURV];
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nrec; r += gridDim.x * blockDim.x) {
    const int4 rc = rect[r];
    const int v = view[r];
    const uint64_t key = ((uint64_t)__float_as_uint(geo[r].w) << 32) | (uint32_t)r;
    const int gx = (wh[2 * v] + tile - 1) / tile;
    const int tb = toff[v];
    for (int ty = rc.y; ty < rc.w; ++ty) {
      for (int tx = rc.x; tx < rc.z; ++tx) {
        const int t = tb + ty * gx + tx;
        const int64_t pos = (int64_t)start[t] + atomicAdd(cursor + t, 1);
        if (pos < cap_dup) keys[pos] = key;
      }
    }
  }
}

constexpr int kSortThreads = 256;
constexpr int kSortCap = 4096;  // keys sorted in LDS at once (32 KiB)

__device__ __forceinline__ void bitonic_lds(uint64_t* sk, int P) {
  const int tid = threadIdx.x;
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < (P >> 1); i += kSortThreads) {
        const int lo = 2 * i - (i & (j - 1));
        const int hi = lo + j;
        const bool up = (lo & k) == 0;
        const uint64_t a = sk[lo], b = sk[hi];
        if ((a > b) == up) {
          sk[lo] = b;
          sk[hi] = a;
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

// sort keys[s, s+n) in chunks of kSortCap (in place)
__device__ void sort_chunks(uint64_t* keys, int n, uint64_t* sk) {
  for (int c0 = 0; c0 < n; c0 += kSortCap) {
    const int m = min(kSortCap, n - c0);
    const int P = next_pow2(m);
    for (int i = threadIdx.x; i < P; i += kSortThreads) sk[i] = i < m ? keys[c0 + i] : ~0ull;
    __syncthreads();
    bitonic_lds(sk, P);
    for (int i = threadIdx.x; i < m; i += kSortThreads) keys[c0 + i] = sk[i];
    __syncthreads();
  }
}

// one merge pass: runs of width w in src -> runs of 2w in dst
__device__ void merge_pass(const uint64_t* src, uint64_t* dst, int n, int w) {
  const int per = (n + kSortThreads - 1) / kSortThreads;
  int o = threadIdx.x * per;
  const int end = min(n, o + per);
  while (o < end) {
    const int p0 = (o / (2 * w)) * (2 * w);
    const int a0 = p0, a1 = min(p0 + w, n);
    const int b0 = a1, b1 = min(p0 + 2 * w, n);
    const int la = a1 - a0, lb = b1 - b0;
    const int d = o - p0;
    int lo = max(0, d - lb), hi = min(d, la);
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (src[a0 + mid] < src[b0 + d - mid - 1]) lo = mid + 1;
      else hi = mid;
    }
    int i = lo, j = d - lo;
    const int stop = min(end, b1);
    while (o < stop) {
      const bool take_a = (j >= lb) || (i < la && src[a0 + i] < src[b0 + j]);
      dst[o++] = take_a ? src[a0 + i++] : src[b0 + j++];
    }
  }
}

__global__ __launch_bounds__(kSortThreads) void k_tile_sort(const int32_t* __restrict__ start,
                                                            uint64_t* __restrict__ keys,
                                                            uint64_t* __restrict__ keys_alt,
                                                            uint32_t* __restrict__ vals,
                                                            int64_t cap_dup) {
  __shared__ uint64_t sk[kSortCap];
  const int t = blockIdx.x;
  const int64_t s64 = start[t];
  const int64_t e64 = min((int64_t)start[t + 1], cap_dup);
  if (e64 <= s64) return;
  const int64_t s = s64;
  const int n = (int)(e64 - s64);
  if (n == 1) {
    if (threadIdx.x == 0) vals[s] = (uint32_t)keys[s];
    return;
  }
  if (n <= kSortCap) {
    const int P = next_pow2(n);
    for (int i = threadIdx.x; i < P; i += kSortThreads) sk[i] = i < n ? keys[s + i] : ~0ull;
    __syncthreads();
    bitonic_lds(sk, P);
    for (int i = threadIdx.x; i < n; i += kSortThreads) vals[s + i] = (uint32_t)sk[i];
    return;
  }
  uint64_t* src = keys + s;
  uint64_t* dst = keys_alt + s;
  sort_chunks(src, n, sk);
  for (int w = kSortCap; w < n; w <<= 1) {
    merge_pass(src, dst, n, w);
    __syncthreads();
    uint64_t* tmp = src;
    src = dst;
    dst = tmp;
  }
  for (int i = threadIdx.x; i < n; i += kSortThreads) vals[s + i] = (uint32_t)src[i];
}

hipError_t launch_sort(const int32_t* tile_count, int total_tiles, const int32_t* tile_offset,
                       int nv, const int32_t* wh, int tile, const int4* rec_rect,
                       const float4* rec_geo, const int32_t* rec_view, int32_t* counters,
                       int32_t* stats, int32_t* tile_start, uint32_t* vals, uint64_t* keys,
                       uint64_t* keys_alt, int32_t* cursor, uint64_t* scan_flags,
                       int64_t cap_dup, int64_t cap_surv, hipStream_t st) {
  const int nblk = scan_blocks(total_tiles);
  hipError_t e = launch_zero(scan_flags, (size_t)nblk * 8, cursor, (size_t)total_tiles * 4,
                             counters + S3R_CNT_TICKET2, 4, nullptr, 0, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_tiles, dim3(nblk), dim3(kScanThreads), 0, st, tile_count, total_tiles,
                     tile_start, scan_flags, counters, cap_dup, nblk);
  hipLaunchKernelGGL(k_dup_stats, dim3(1), dim3(64), 0, st, tile_start, tile_offset, nv, stats);
  const int64_t want = (cap_surv + 255) / 256;
  const int grid = (int)(want < 2048 ? (want > 0 ? want : 1) : 2048);
  hipLaunchKernelGGL(k_emit, dim3(grid), dim3(256), 0, st, rec_rect, rec_geo, rec_view,
                     tile_offset, wh, tile, tile_start, cursor, counters, keys, cap_dup);
  hipLaunchKernelGGL(k_tile_sort, dim3(total_tiles), dim3(kSortThreads), 0, st, tile_start, keys,
                     keys_alt, vals, cap_dup);
  return hipGetLastError();
}

}  // namespace s3r
