// Per-tile contributor lists in the blending order of Eq. (2).
//
// A list entry is a (tile, record) pair.  s3r_project_cull gives every
// record its first pair in emission order (a record emits the tiles of its
// rectangle row by row, records in record order, and records of a view are
// in Gaussian order); ordering every tile's list by (depth bits, record)
// gives the order the oracle defines -- (depth, Gaussian index) -- bit for
// bit.
//
// With S3R_SORT_TILES and at most kBinMaxTiles tiles (a batch of one 1080p
// view at 16 px has 8160):
//   1. k_bin_count / k_bin_scan / k_bin_place: pairs counted per tile in LDS
//      histograms, list starts and the launch order from one scan, pairs
//      written into their lists as keys (depth bits << 32 | record)
//   2. k_tile_sort_*: each list sorted on that key with bitonic networks
//      (registers, LDS between waves; long lists in chunks merged by rank;
//      lists too long for LDS in place in global memory)
// Otherwise:
//   1. k_emit_pairs: keys (global tile << 32 | depth bits) in record order,
//      every thread a run of consecutive pairs, stored coalesced through LDS
//   2. least-significant-digit radix passes, 8 bits each: block histograms ->
//      scan of the digit-major histogram matrix (sized by the pair count on
//      the device, not by the capacity) -> stable scatter, where each wave
//      ranks its keys by matching digits with eight ballots.  The passes
//      cover all key bits, or with S3R_SORT_TILES only the tile bits (a stable
//      partition that leaves every list in emission order)
//   3. tile ranges from where the tile changes between neighbouring keys; the
//      tiles' launch order (descending list length)
//   4. with S3R_SORT_TILES, k_tile_sort_*: each list sorted by (depth bits,
//      position in the list)
// No kernel waits on another workgroup and none uses a contended atomic.
#include "internal.hpp"

namespace s3r {

// ---------------------------------------------------------------------------
// generic exclusive scan of int32 (reduce-then-scan), n on the host or device
// ---------------------------------------------------------------------------
constexpr int kST = 256;
constexpr int kSI = 16;
constexpr int kSTile = kST * kSI;

int scan_blocks(int64_t n) { return (int)((n + kSTile - 1) / kSTile); }

__device__ __forceinline__ int64_t dev_n(const int32_t* n_dev, int64_t n_host) {
  return n_dev ? (int64_t)*n_dev : n_host;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t t = __shfl_up(x, o, kWave);
    if (lane >= o) x += t;
  }
  return x;
}

// exclusive scan of the 256 thread values of a block; returns the block total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t& excl) {
  __shared__ uint32_t s_w[kST / kWave];
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  const uint32_t incl = wave_incl_scan(x);
  if (lane == kWave - 1) s_w[wave] = incl;
  __syncthreads();
  uint32_t run = incl - x, tot = 0;
  for (int w = 0; w < kST / kWave; ++w) {
    if (w < wave) run += s_w[w];
    tot += s_w[w];
  }
  __syncthreads();
  excl = run;
  return tot;
}

__global__ __launch_bounds__(kST) void k_scan_reduce(const int32_t* __restrict__ in,
                                                     const int32_t* n_dev, int64_t n_host,
                                                     int32_t* __restrict__ sums) {
  const int64_t n = dev_n(n_dev, n_host);
  const int64_t base = (int64_t)blockIdx.x * kSTile + (int64_t)threadIdx.x * kSI;
  uint32_t s = 0;
#pragma unroll
  for (int q = 0; q < kSI; ++q)
    if (base + q < n) s += (uint32_t)in[base + q];
  uint32_t excl;
  const uint32_t tot = block_excl_scan(s, excl);
  if (threadIdx.x == 0) sums[blockIdx.x] = (int32_t)tot;
}

// one workgroup: exclusive scan of the block sums in place, total -> *total
__global__ __launch_bounds__(1024) void k_scan_top(int32_t* __restrict__ sums, int nb,
                                                   int32_t* __restrict__ total) {
  __shared__ uint32_t s_w[16];
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const int per = (nb + 1023) / 1024;
  const int e0 = tid * per, e1 = min(nb, e0 + per);
  uint32_t s = 0;
  for (int e = e0; e < e1; ++e) s += (uint32_t)sums[e];
  uint32_t incl = wave_incl_scan(s);
  if (lane == kWave - 1) s_w[wave] = incl;
  __syncthreads();
  uint32_t run = incl - s;
  for (int w = 0; w < wave; ++w) run += s_w[w];
  for (int e = e0; e < e1; ++e) {
    const uint32_t v = (uint32_t)sums[e];
    sums[e] = (int32_t)run;
    run += v;
  }
  if (tid == 1023) *total = (int32_t)run;
}

// kPrefix: sums[] holds the raw block sums and each block adds up those
// before it itself (at most kScanFuseMax of them), in place of k_scan_top;
// the last block then stores the total
template <bool kPrefix>
__global__ __launch_bounds__(kST) void k_scan_down(const int32_t* __restrict__ in,
                                                   const int32_t* n_dev, int64_t n_host,
                                                   const int32_t* __restrict__ sums,
                                                   int32_t* __restrict__ out,
                                                   int32_t* __restrict__ total) {
  const int64_t n = dev_n(n_dev, n_host);
  const int64_t base = (int64_t)blockIdx.x * kSTile + (int64_t)threadIdx.x * kSI;
  uint32_t v[kSI], s = 0;
#pragma unroll
  for (int q = 0; q < kSI; ++q) {
    v[q] = (base + q < n) ? (uint32_t)in[base + q] : 0u;
    s += v[q];
  }
  uint32_t before;
  if (kPrefix) {
    uint32_t p = 0;
    for (int q = threadIdx.x; q < (int)blockIdx.x; q += kST) p += (uint32_t)sums[q];
    uint32_t unused;
    before = block_excl_scan(p, unused);
  } else {
    before = (uint32_t)sums[blockIdx.x];
  }
  uint32_t excl;
  const uint32_t mine = block_excl_scan(s, excl);
  if (kPrefix && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
    *total = (int32_t)(before + mine);
  uint32_t run = before + excl;
#pragma unroll
  for (int q = 0; q < kSI; ++q) {
    if (base + q < n) out[base + q] = (int32_t)run;
    run += v[q];
  }
}

// up to this many blocks, each block of the down sweep sums the block sums
// before it (a few KB from L2) instead of a third launch scanning them
constexpr int kScanFuseMax = 1024;

static hipError_t scan_i32(const int32_t* in, const int32_t* n_dev, int64_t n_cap, int32_t* out,
                           int32_t* sums, int32_t* total, hipStream_t st) {
  const int nb = scan_blocks(n_cap) > 0 ? scan_blocks(n_cap) : 1;
  S3R_LAUNCH(K_SCAN, k_scan_reduce, dim3(nb), dim3(kST), 0, st, in, n_dev, n_cap, sums);
  if (nb <= min(kScanFuseMax, tune(S3R_TUNE_SCAN_FUSE_MAX))) {
    S3R_LAUNCH(K_SCAN, k_scan_down<true>, dim3(nb), dim3(kST), 0, st, in, n_dev, n_cap, sums, out,
               total);
  } else {
    S3R_LAUNCH(K_SCAN, k_scan_top, dim3(1), dim3(1024), 0, st, sums, nb, total);
    S3R_LAUNCH(K_SCAN, k_scan_down<false>, dim3(nb), dim3(kST), 0, st, in, n_dev, n_cap, sums,
               out, nullptr);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// pair emission
// ---------------------------------------------------------------------------
constexpr int kEmitRun = 8;  // consecutive pairs per thread
constexpr int kEmitThreads = 256;
constexpr int kEmitBlock = kEmitThreads * kEmitRun;  // pairs per workgroup pass
constexpr int kEmitPad = kEmitRun + 1;  // a thread's LDS row, padded against bank conflicts

// Each thread finds the record of its first pair by binary search and walks
// its run of kEmitRun pairs; the runs are staged in LDS and the workgroup
// then stores the kEmitBlock pairs lane-consecutively (whole cache lines,
// where run-per-lane stores would leave lines partly written).
__global__ __launch_bounds__(kEmitThreads) void k_emit_pairs(SortArgs a) {
  __shared__ uint64_t s_key[kEmitThreads * kEmitPad];
  __shared__ uint32_t s_val[kEmitThreads * kEmitPad];
  const int nrec = a.counters[S3R_CNT_SURV];
  const int64_t ndup = min((int64_t)a.counters[S3R_CNT_DUP], a.cap_dup);
  const int tid = threadIdx.x;
  // the loop bounds are uniform over the workgroup (it holds barriers)
  for (int64_t P = (int64_t)blockIdx.x * kEmitBlock; P < ndup;
       P += (int64_t)gridDim.x * kEmitBlock) {
    const int64_t p0 = P + (int64_t)tid * kEmitRun;
    if (p0 < ndup) {
      // last record whose first pair is at or before p0
      int lo = 0, hi = nrec - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.pair_off[mid] <= p0) lo = mid;
        else hi = mid - 1;
      }
      int r = lo;
      int64_t next = (r + 1 < nrec) ? (int64_t)a.pair_off[r + 1] : ndup;
      int4 rc = a.rec_rect[r];
      int v = a.rec_view[r];
      uint32_t db = __float_as_uint(a.rec_geo[r].w);
      int gx = (a.wh[2 * v] + a.tile - 1) / a.tile;
      const int64_t p1 = min(ndup, p0 + kEmitRun);
      for (int64_t p = p0; p < p1; ++p) {
        while (p >= next) {
          ++r;
          next = (r + 1 < nrec) ? (int64_t)a.pair_off[r + 1] : ndup;
          rc = a.rec_rect[r];
          v = a.rec_view[r];
          db = __float_as_uint(a.rec_geo[r].w);
          gx = (a.wh[2 * v] + a.tile - 1) / a.tile;
        }
        const int j = (int)(p - a.pair_off[r]);
        const int w = rc.z - rc.x;
        const int tx = rc.x + j % w;
        const int ty = rc.y + j / w;
        const uint32_t t = (uint32_t)(a.tile_offset[v] + ty * gx + tx);
        const int slot = tid * kEmitPad + (int)(p - p0);
        s_key[slot] = ((uint64_t)t << 32) | db;
        s_val[slot] = (uint32_t)r;
      }
    }
    __syncthreads();
    // pair P + e lives in row e / kEmitRun, column e % kEmitRun
#pragma unroll
    for (int m = 0; m < kEmitRun; ++m) {
      const int e = tid + kEmitThreads * m;
      if (P + e < ndup) {
        const int slot = (e / kEmitRun) * kEmitPad + e % kEmitRun;
        a.keys[P + e] = s_key[slot];
        a.vals0[P + e] = s_val[slot];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits, 4096 keys per workgroup
// ---------------------------------------------------------------------------
constexpr int kRT = 256;
constexpr int kRI = 16;
constexpr int kRTile = kRT * kRI;
constexpr int kRWaves = kRT / kWave;

// lanes whose 8-bit digit equals this lane's (among valid lanes)
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
  uint64_t eq = ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bb = ballot(bit);
    eq &= bit ? bb : ~bb;
  }
  return eq;
}

// The histogram is digit-major over the blocks that hold keys (nb of them,
// from the device-side key count), so the scan that follows covers 256 nb
// counts however large the capacity; its length is left in *hist_len.
__global__ __launch_bounds__(kRT) void k_radix_hist(const uint64_t* __restrict__ keys,
                                                    const int32_t* __restrict__ n_dev,
                                                    int shift, int32_t* __restrict__ hist,
                                                    int32_t* __restrict__ hist_len) {
  __shared__ uint32_t h[kRWaves][256];
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const int64_t n = *n_dev;
  const int nb = (int)((n + kRTile - 1) / kRTile);
  if (blockIdx.x == 0 && tid == 0) *hist_len = 256 * nb;
  if ((int)blockIdx.x >= nb) return;  // uniform over the workgroup
  for (int q = tid; q < kRWaves * 256; q += kRT) (&h[0][0])[q] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRTile;
  {
    for (int k = 0; k < kRI; ++k) {
      const int64_t idx = base + (int64_t)k * kRT + tid;
      const bool valid = idx < n;
      const uint32_t d = valid ? (uint32_t)(keys[idx] >> shift) & 255u : 0u;
      const uint64_t eq = match_digit(d, valid);
      if (valid && (eq & ((1ull << lane) - 1ull)) == 0ull) h[wave][d] += __popcll(eq);
    }
  }
  __syncthreads();
  uint32_t s = 0;
  for (int w = 0; w < kRWaves; ++w) s += h[w][tid];
  hist[(size_t)tid * nb + blockIdx.x] = (int32_t)s;
}

__global__ __launch_bounds__(kRT) void k_radix_scatter(const uint64_t* __restrict__ kin,
                                                       const uint32_t* __restrict__ vin,
                                                       uint64_t* __restrict__ kout,
                                                       uint32_t* __restrict__ vout,
                                                       const int32_t* __restrict__ n_dev,
                                                       int shift,
                                                       const int32_t* __restrict__ off) {
  __shared__ uint16_t cnt[kRI][kRWaves][256];
  __shared__ uint32_t s_base[256];
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const int64_t n = *n_dev;
  const int64_t nb = (n + kRTile - 1) / kRTile;
  const int64_t base = (int64_t)blockIdx.x * kRTile;
  if (base >= n) return;
  for (int q = tid; q < kRI * kRWaves * 256; q += kRT) (&cnt[0][0][0])[q] = 0;
  __syncthreads();
  uint64_t key[kRI];
  uint32_t val[kRI];
  uint32_t rank[kRI];
  const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int k = 0; k < kRI; ++k) {
    const int64_t idx = base + (int64_t)k * kRT + tid;
    const bool valid = idx < n;
    key[k] = valid ? kin[idx] : 0ull;
    val[k] = valid ? vin[idx] : 0u;
    const uint32_t d = (uint32_t)(key[k] >> shift) & 255u;
    const uint64_t eq = match_digit(d, valid);
    rank[k] = __popcll(eq & lt);
    if (valid && rank[k] == 0u) cnt[k][wave][d] = (uint16_t)__popcll(eq);
  }
  __syncthreads();
  // per digit: running count over the (item, wave) slots in key order
  {
    const int d = tid;
    uint32_t run = 0;
    for (int k = 0; k < kRI; ++k)
      for (int w = 0; w < kRWaves; ++w) {
        const uint32_t c = cnt[k][w][d];
        cnt[k][w][d] = (uint16_t)run;
        run += c;
      }
    s_base[d] = (uint32_t)off[(size_t)d * nb + blockIdx.x];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kRI; ++k) {
    const int64_t idx = base + (int64_t)k * kRT + tid;
    if (idx < n) {
      const uint32_t d = (uint32_t)(key[k] >> shift) & 255u;
      const uint32_t pos = s_base[d] + cnt[k][wave][d] + rank[k];
      kout[pos] = key[k];
      vout[pos] = val[k];
    }
  }
}

// ---------------------------------------------------------------------------
// tile ranges and per-view pair counts
// ---------------------------------------------------------------------------
// List ranges from the partitioned keys in one streaming pass: key i opens
// the lists of the tiles t in (tile(i - 1), tile(i)] at position i, with
// tile(-1) = -1 and tile(n) = total_tiles, so every start[t], t <= total_tiles,
// is written exactly once.  The lengths (start differences) are written by
// k_order_count, which reads them anyway.
__global__ __launch_bounds__(256) void k_tile_ranges(const uint64_t* __restrict__ keys,
                                                     const int32_t* __restrict__ n_dev,
                                                     int total_tiles,
                                                     int32_t* __restrict__ start) {
  const int64_t n = *n_dev;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int lo = i == 0 ? -1 : (int)(keys[i - 1] >> 32);
    const int hi = i == n ? total_tiles : min((int)(keys[i] >> 32), total_tiles);
    for (int t = lo + 1; t <= hi; ++t) start[t] = (int32_t)i;
  }
}

// Launch order of the rasterizer: tiles by descending list length, so the
// longest lists (whose waves set the critical path) start first.  Lengths are
// bucketed by their binary logarithm (empty lists last) and the order within
// a bucket is the tile order: a stable counting sort over chunks of
// kOrderChunk tiles (per-chunk bucket counts, a one-workgroup scan over
// (bucket, chunk), per-chunk placement).  The top kernel also writes each
// view's number of (tile, record) pairs.
constexpr int kOrderBuckets = 17;
constexpr int kOrderThreads = 256;
constexpr int kOrderPer = 4;
constexpr int kOrderChunk = kOrderThreads * kOrderPer;

__device__ __forceinline__ int order_bucket(const int32_t* start, int t) {
  const int len = start[t + 1] - start[t];
  return len <= 0 ? kOrderBuckets - 1 : 15 - min(15, 31 - __builtin_clz((unsigned)len));
}

__global__ __launch_bounds__(kOrderThreads) void k_order_count(const int32_t* __restrict__ start,
                                                              int total_tiles, int nchunk,
                                                              int32_t* __restrict__ cnt,
                                                              int32_t* __restrict__ len) {
  __shared__ int s_c[kOrderBuckets];
  const int tid = threadIdx.x, c = blockIdx.x;
  if (tid < kOrderBuckets) s_c[tid] = 0;
  __syncthreads();
  for (int m = 0; m < kOrderPer; ++m) {
    const int t = c * kOrderChunk + m * kOrderThreads + tid;
    if (t < total_tiles) {
      len[t] = start[t + 1] - start[t];
      atomicAdd(&s_c[order_bucket(start, t)], 1);
    }
  }
  __syncthreads();
  if (tid < kOrderBuckets) cnt[tid * nchunk + c] = s_c[tid];  // bucket-major
}

__global__ __launch_bounds__(1024) void k_order_top(int32_t* __restrict__ cnt, int n,
                                                    const int32_t* __restrict__ start,
                                                    const int32_t* __restrict__ toff, int nv,
                                                    int32_t* __restrict__ stats) {
  __shared__ int s_w[1024 / kWave];
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const int per = (n + 1023) / 1024;
  const int e0 = min(n, tid * per), e1 = min(n, e0 + per);
  int sum = 0;
  for (int e = e0; e < e1; ++e) sum += cnt[e];
  int incl = sum;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  if (lane == kWave - 1) s_w[wave] = incl;
  __syncthreads();
  int run = incl - sum;
  for (int w = 0; w < wave; ++w) run += s_w[w];
  for (int e = e0; e < e1; ++e) {
    const int x = cnt[e];
    cnt[e] = run;
    run += x;
  }
  if (tid < nv) stats[tid * 4 + 3] = start[toff[tid + 1]] - start[toff[tid]];
}

__global__ __launch_bounds__(kOrderThreads) void k_order_place(const int32_t* __restrict__ start,
                                                              int total_tiles, int nchunk,
                                                              const int32_t* __restrict__ cnt,
                                                              int32_t* __restrict__ order) {
  // per (bucket, thread) counts of the chunk, scanned in (bucket, thread) order
  __shared__ int s_c[kOrderBuckets * kOrderThreads];
  __shared__ int s_w[kOrderThreads / kWave];
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave, c = blockIdx.x;
  const int t0 = c * kOrderChunk + tid * kOrderPer;  // this thread's consecutive tiles
  int bk[kOrderPer];
  for (int b = 0; b < kOrderBuckets; ++b) s_c[b * kOrderThreads + tid] = 0;
#pragma unroll
  for (int m = 0; m < kOrderPer; ++m) {
    const int t = t0 + m;
    bk[m] = t < total_tiles ? order_bucket(start, t) : -1;
    if (bk[m] >= 0) s_c[bk[m] * kOrderThreads + tid] += 1;
  }
  __syncthreads();
  // thread i scans entries i*17 .. i*17+16 of the linear (bucket, thread) order
  int sum = 0;
  for (int k = 0; k < kOrderBuckets; ++k) sum += s_c[tid * kOrderBuckets + k];
  int incl = sum;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  if (lane == kWave - 1) s_w[wave] = incl;
  __syncthreads();
  int run = incl - sum;
  for (int w = 0; w < wave; ++w) run += s_w[w];
  __syncthreads();
  for (int k = 0; k < kOrderBuckets; ++k) {
    const int x = s_c[tid * kOrderBuckets + k];
    s_c[tid * kOrderBuckets + k] = run;
    run += x;
  }
  __syncthreads();
  // in-chunk position = scanned (bucket, thread) entry minus the chunk-local
  // start of the bucket; global position = the (bucket, chunk) offset plus it
  __shared__ int s_base[kOrderBuckets];
  if (tid < kOrderBuckets) s_base[tid] = s_c[tid * kOrderThreads];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < kOrderPer; ++m) {
    if (bk[m] < 0) continue;
    const int b = bk[m];
    const int in_chunk = s_c[b * kOrderThreads + tid] - s_base[b];
    s_c[b * kOrderThreads + tid] += 1;
    order[cnt[b * nchunk + c] + in_chunk] = t0 + m;
  }
}

// ---------------------------------------------------------------------------
// tile binning (S3R_SORT_TILES while a tile histogram fits in LDS)
// ---------------------------------------------------------------------------
// Each workgroup takes kBinBlock consecutive pairs (in emission order) and
// counts them per tile in an LDS histogram; k_bin_count adds the non-zero
// bins to the global counts, and k_bin_place takes each tile's list start
// from an exclusive scan of the counts, claims, per non-zero bin, a block of
// slots of the tile's list with one atomic on its fill counter and writes each
// pair there as the key (depth bits << 32 | record).  One more workgroup of
// the placement launch writes the list starts and lengths and the launch
// order.  The order inside a list is
// left arbitrary: the per-list sort orders it by that key, whose record part
// is the Gaussian order within a view, so the lists come out exactly as a
// stable sort would leave them.  Same-address atomics are one per tile and
// workgroup, never one per pair.
constexpr int kBinThreads = 1024;
constexpr int kBinRun = 4;  // consecutive pairs per thread
constexpr int kBinBlock = kBinThreads * kBinRun;
constexpr int kBinMaxTiles = 12288;  // a 48 KB histogram: two workgroups per CU

// the pairs [p0, p1) of this thread (inside the workgroup's window):
// f(global tile, record, depth bits)
template <class F>
__device__ __forceinline__ void walk_pairs(const SortArgs& a, const int* s_pair, int r0, int nw,
                                           int64_t p0, int64_t p1, F&& f) {
  int lo = 0, hi = nw - 1;  // last window record whose first pair is at or before p0
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_pair[mid] <= p0) lo = mid;
    else hi = mid - 1;
  }
  int i = lo;
  int64_t first = s_pair[i], next = s_pair[i + 1];
  int r = r0 + i;
  int4 rc = a.rec_rect[r];
  int v = a.rec_view[r];
  uint32_t db = __float_as_uint(a.rec_geo[r].w);
  int gx = (a.wh[2 * v] + a.tile - 1) / a.tile;
  int tb = a.tile_offset[v];
  for (int64_t p = p0; p < p1; ++p) {
    while (p >= next) {
      ++i;
      first = next;
      next = s_pair[i + 1];
      r = r0 + i;
      rc = a.rec_rect[r];
      v = a.rec_view[r];
      db = __float_as_uint(a.rec_geo[r].w);
      gx = (a.wh[2 * v] + a.tile - 1) / a.tile;
      tb = a.tile_offset[v];
    }
    const int j = (int)(p - first);
    const int w = rc.z - rc.x;
    f(tb + (rc.y + j / w) * gx + rc.x + j % w, r, db);
  }
}

// the per-tile counts and fill counters start at zero
__global__ __launch_bounds__(256) void k_bin_zero(int32_t* __restrict__ c, int32_t* __restrict__ f,
                                                  int n) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    c[t] = 0;
    f[t] = 0;
  }
}

__global__ __launch_bounds__(kBinThreads) void k_bin_count(SortArgs a) {
  __shared__ int s_h[kBinMaxTiles];
  __shared__ int s_pair[kBinBlock + 2];
  __shared__ int s_red[2 * kBinThreads / kWave];
  const int nrec = a.counters[S3R_CNT_SURV];
  const int64_t ndup = min((int64_t)a.counters[S3R_CNT_DUP], a.cap_dup);
  const int64_t P = (int64_t)blockIdx.x * kBinBlock;
  if (P >= ndup || nrec <= 0) return;  // uniform over the workgroup
  const int tid = threadIdx.x;
  for (int t = tid; t < a.total_tiles; t += kBinThreads) s_h[t] = 0;
  const int64_t Pe = min(ndup, P + kBinBlock);
  int nw;
  const int r0 = record_window<kBinThreads>(a.pair_off, nrec, P, Pe, s_pair, s_red, &nw);
  const int64_t p0 = P + (int64_t)tid * kBinRun;
  const int64_t p1 = min(Pe, p0 + kBinRun);
  if (p0 < p1)
    walk_pairs(a, s_pair, r0, nw, p0, p1, [&](int t, int, uint32_t) { atomicAdd(&s_h[t], 1); });
  __syncthreads();
  for (int t = tid; t < a.total_tiles; t += kBinThreads)
    if (s_h[t] != 0) atomicAdd(&a.bin_count[t], s_h[t]);
}

// tiles per thread in the placement launch's scans of the counts (thread t
// takes tiles t kBinTpt .. t kBinTpt + kBinTpt - 1)
constexpr int kBinTpt = kBinMaxTiles / kBinThreads;
static_assert(kBinTpt * kBinThreads == kBinMaxTiles, "whole tile runs per thread");

// exclusive scan of x over the workgroup in thread order; the total out
__device__ __forceinline__ int bin_block_scan(int x, int* s_w, int& total) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int incl = wave_inclusive_scan(x);
  if (lane == kWave - 1) s_w[wave] = incl;
  __syncthreads();
  int base = 0;
  total = 0;
  for (int w = 0; w < kBinThreads / kWave; ++w) {
    if (w < wave) base += s_w[w];
    total += s_w[w];
  }
  __syncthreads();
  return base + incl - x;
}

__device__ __forceinline__ int order_bucket(int c) {
  return c <= 0 ? kOrderBuckets - 1 : 15 - min(15, 31 - __builtin_clz((unsigned)c));
}

// The last workgroup of the placement launch: list lengths and starts
// (exclusive scan of the counts), each view's pair count, and the
// rasterizers' launch order -- tiles by descending binary logarithm of the
// list length (empty lists last), tile order within a bucket -- with the
// bucket starts the per-list sorts read (order_cnt[b * nchunk], nchunk tile
// chunks of kOrderChunk).  s_c holds kOrderBuckets x kBinThreads counters.
__device__ __forceinline__ void bin_lists(const SortArgs& a, int nchunk, int* s_c, int* s_w,
                                          int* s_v, int* s_toff) {
  const int tid = threadIdx.x;
  const int T = a.total_tiles;
  const int t0 = tid * kBinTpt;
  for (int v = tid; v < a.nv; v += kBinThreads) s_v[v] = 0;
  for (int v = tid; v <= a.nv; v += kBinThreads) s_toff[v] = a.tile_offset[v];
  for (int b = 0; b < kOrderBuckets; ++b) s_c[b * kBinThreads + tid] = 0;
  int c[kBinTpt], sum = 0;
#pragma unroll
  for (int k = 0; k < kBinTpt; ++k) {
    c[k] = t0 + k < T ? a.bin_count[t0 + k] : 0;
    sum += c[k];
  }
  int total;
  int run = bin_block_scan(sum, s_w, total);
  int v = 0, vsum = 0;
#pragma unroll
  for (int k = 0; k < kBinTpt; ++k) {
    const int t = t0 + k;
    if (t < T) {
      a.tile_count[t] = c[k];
      a.tile_start[t] = run;
      run += c[k];
      while (s_toff[v + 1] <= t) {
        if (vsum) atomicAdd(&s_v[v], vsum);
        vsum = 0;
        ++v;
      }
      vsum += c[k];
      s_c[order_bucket(c[k]) * kBinThreads + tid] += 1;
    }
  }
  if (vsum) atomicAdd(&s_v[v], vsum);
  if (tid == 0) a.tile_start[T] = total;
  __syncthreads();
  // (bucket, thread) offsets: thread i scans the kOrderBuckets consecutive
  // entries i * kOrderBuckets .. of the bucket-major linear order
  int bsum = 0;
  for (int k = 0; k < kOrderBuckets; ++k) bsum += s_c[tid * kOrderBuckets + k];
  int btot;
  int brun = bin_block_scan(bsum, s_w, btot);
  for (int k = 0; k < kOrderBuckets; ++k) {
    const int x = s_c[tid * kOrderBuckets + k];
    s_c[tid * kOrderBuckets + k] = brun;
    brun += x;
  }
  __syncthreads();
  if (tid < kOrderBuckets) a.order_cnt[tid * nchunk] = s_c[tid * kBinThreads];
  if (tid < a.nv) a.stats[tid * 4 + 3] = s_v[tid];
  __syncthreads();  // (the bucket starts are read before the cursors below move)
#pragma unroll
  for (int k = 0; k < kBinTpt; ++k) {
    const int t = t0 + k;
    if (t < T) a.tile_order[s_c[order_bucket(c[k]) * kBinThreads + tid]++] = t;
  }
}

// Workgroup 0 runs bin_lists (dispatched first, it overlaps the placement);
// workgroups 1 .. gridDim.x - 1 place the pairs.  A placing workgroup takes
// each tile's list start from a scan of the counts over its waves: wave w
// holds tiles w kBinTpt kWave + k kWave + lane (k < kBinTpt), so its loads
// and slot claims are lane-consecutive.  LDS: the placing workgroups' tile
// histogram and record window share one array with bin_lists' counters.
constexpr int kBinLds = (kBinMaxTiles + kBinBlock + 2 > kOrderBuckets * kBinThreads)
                            ? kBinMaxTiles + kBinBlock + 2
                            : kOrderBuckets * kBinThreads;

__global__ __launch_bounds__(kBinThreads) void k_bin_place(SortArgs a, int nchunk) {
  __shared__ int s_mem[kBinLds];
  __shared__ int s_red[2 * kBinThreads / kWave];
  __shared__ int s_w[kBinThreads / kWave];
  __shared__ int s_v[kMaxViews];
  __shared__ int s_toff[kMaxViews + 1];
  if (blockIdx.x == 0) {  // uniform over the workgroup
    bin_lists(a, nchunk, s_mem, s_w, s_v, s_toff);
    return;
  }
  int* s_h = s_mem;
  int* s_pair = s_mem + kBinMaxTiles;
  const int nrec = a.counters[S3R_CNT_SURV];
  const int64_t ndup = min((int64_t)a.counters[S3R_CNT_DUP], a.cap_dup);
  const int64_t P = (int64_t)(blockIdx.x - 1) * kBinBlock;
  if (P >= ndup || nrec <= 0) return;  // uniform over the workgroup
  const int tid = threadIdx.x;
  const int T = a.total_tiles;
  for (int t = tid; t < T; t += kBinThreads) s_h[t] = 0;
  const int64_t Pe = min(ndup, P + kBinBlock);
  int nw;
  const int r0 = record_window<kBinThreads>(a.pair_off, nrec, P, Pe, s_pair, s_red, &nw);
  const int64_t p0 = P + (int64_t)tid * kBinRun;
  const int64_t p1 = min(Pe, p0 + kBinRun);
  if (p0 < p1)
    walk_pairs(a, s_pair, r0, nw, p0, p1, [&](int t, int, uint32_t) { atomicAdd(&s_h[t], 1); });
  // list starts of this thread's tiles, then this workgroup's block of slots
  // in every list it touches
  const int lane = tid % kWave, wave = tid / kWave;
  const int tw = wave * kBinTpt * kWave + lane;  // this thread's tile of round k: tw + k kWave
  int ex[kBinTpt], carry = 0;
#pragma unroll
  for (int k = 0; k < kBinTpt; ++k) {
    const int t = tw + k * kWave;
    const int c = t < T ? a.bin_count[t] : 0;
    const int incl = wave_inclusive_scan(c);
    ex[k] = carry + incl - c;
    carry += __builtin_amdgcn_readlane(incl, kWave - 1);
  }
  if (lane == 0) s_w[wave] = carry;
  __syncthreads();  // (also orders the histogram above before the claims)
  int wbase = 0;
  for (int w = 0; w < wave; ++w) wbase += s_w[w];
  int h[kBinTpt], base[kBinTpt];
#pragma unroll
  for (int k = 0; k < kBinTpt; ++k) h[k] = tw + k * kWave < T ? s_h[tw + k * kWave] : 0;
#pragma unroll
  for (int k = 0; k < kBinTpt; ++k)
    base[k] = h[k] != 0 ? atomicAdd(&a.bin_cursor[tw + k * kWave], h[k]) : 0;
#pragma unroll
  for (int k = 0; k < kBinTpt; ++k)
    if (h[k] != 0) s_h[tw + k * kWave] = wbase + ex[k] + base[k];
  __syncthreads();
  if (p0 < p1)
    walk_pairs(a, s_pair, r0, nw, p0, p1, [&](int t, int r, uint32_t db) {
      const int slot = atomicAdd(&s_h[t], 1);
      a.keys[slot] = ((uint64_t)db << 32) | (uint32_t)r;
    });
}

// ---------------------------------------------------------------------------
// per-tile depth order
// ---------------------------------------------------------------------------
// A list of n entries is sorted on the composite key (depth bits << 32 |
// position in the list), which orders equal depths by emission position as a
// stable sort would.  The network is the bitonic sorter written so that every
// merge compares an element with its mirror image in the first step and with
// the element j places on in the later steps; all comparators put the smaller
// key at the lower index, so keys padded at the end with the largest value
// never move and lengths need not be powers of two.
//
// Inside a wave the keys live in registers: lane l holds positions l E .. l E
// + E - 1, steps at distance below E are register compare-swaps and longer
// ones exchange keys with the partner lane (shuffles); only steps between
// waves go through LDS.
//
// Size classes follow the binary-logarithm buckets of the launch order (lists
// by descending length), so each longer class is a prefix of that order:
//   tiny  (< kTsTiny entries): one wave per list, E = 1 .. 8 keys per lane
//   small (< kTsChunk): four waves per list, 8 keys per lane
//   large (< kTsLarge): chunks of kTsChunk entries sorted like small lists by
//         separate workgroups, then merged in LDS by rank (an entry's place
//         is its place in its chunk plus the entries below it in the others)
//   huge  (>= kTsLarge): one workgroup, in global memory
constexpr int kTsTiny = 512;
constexpr int kTsChunk = 2048;
constexpr int kTsLarge = 16384;
constexpr int kTsMaxChunks = kTsLarge / kTsChunk;
constexpr int kTsChunkBlocks = 1024;
constexpr int kTsE = 8;                    // keys per lane of the small class
constexpr int kTsWaveKeys = kWave * kTsE;  // 512: keys per wave

__device__ __forceinline__ int next_pow2(int n) {
  int m = 1;
  while (m < n) m <<= 1;
  return m;
}

// lower element of comparator q at distance j (a zero bit inserted at log2 j)
__device__ __forceinline__ int cmp_lower(int q, int j) { return ((q & ~(j - 1)) << 1) | (q & (j - 1)); }

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int mask) {
  const int lo = __shfl_xor((int)(uint32_t)v, mask, kWave);
  const int hi = __shfl_xor((int)(uint32_t)(v >> 32), mask, kWave);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// step (K, J) of the network on a wave's 64 E register keys
template <int E, int K, int J>
__device__ __forceinline__ void net_step(uint64_t (&x)[E], int lane) {
  constexpr bool flip = J == K / 2;
  if constexpr (J < E) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int f = flip ? (e ^ (K - 1)) : (e ^ J);
      if (f > e) {
        const uint64_t a = x[e], b = x[f];
        x[e] = b < a ? b : a;
        x[f] = b < a ? a : b;
      }
    }
  } else {
    // partner lane and, in a mirror step, the mirrored register
    constexpr int lmask = flip ? (K / E - 1) : (J / E);
    constexpr int hb = flip ? (K / (2 * E)) : (J / E);
    const bool lower = (lane & hb) == 0;
    uint64_t y[E];
#pragma unroll
    for (int e = 0; e < E; ++e) y[e] = shfl_xor64(x[flip ? (E - 1 - e) : e], lmask);
    // the lower lane keeps the smaller key, the upper the larger (keys are
    // distinct but for the padding, where either choice is the same value)
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = ((y[e] < x[e]) == lower) ? y[e] : x[e];
  }
}

// steps J, J/2, .., 1 of a merge of size K
template <int E, int K, int J>
struct NetMerge {
  __device__ __forceinline__ static void run(uint64_t (&x)[E], int lane) {
    net_step<E, K, J>(x, lane);
    NetMerge<E, K, J / 2>::run(x, lane);
  }
};
template <int E, int K>
struct NetMerge<E, K, 0> {
  __device__ __forceinline__ static void run(uint64_t (&)[E], int) {}
};
// all merges of sizes 2 .. K
template <int E, int K>
struct NetSort {
  __device__ __forceinline__ static void run(uint64_t (&x)[E], int lane) {
    NetSort<E, K / 2>::run(x, lane);
    NetMerge<E, K, K / 2>::run(x, lane);
  }
};
template <int E>
struct NetSort<E, 1> {
  __device__ __forceinline__ static void run(uint64_t (&)[E], int) {}
};

__device__ __forceinline__ void list_of(const int32_t* start, const int32_t* order, int i,
                                        int64_t cap, int64_t& s0, int& n) {
  const int t = order[i];
  s0 = start[t];
  n = (int)(min((int64_t)start[t + 1], cap) - s0);
}

// keys [at + base, at + base + 64 E) of this wave's lanes, the largest key
// past len.  Binned lists (direct) hold their sort keys (depth bits << 32 |
// record) already; partitioned ones hold (tile << 32 | depth bits) and become
// composite keys (depth bits << 32 | position, positions from pos0).
template <int E>
__device__ __forceinline__ void load_keys(uint64_t (&x)[E], const uint64_t* __restrict__ keys,
                                          int64_t at, int base, int len, uint32_t pos0, int lane,
                                          bool direct) {
  uint64_t d[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = base + lane * E + e;
    d[e] = p < len ? keys[at + p] : ~0ull;
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = base + lane * E + e;
    x[e] = (p >= len || direct) ? d[e] : (((uint64_t)(uint32_t)d[e] << 32) | (pos0 + (uint32_t)p));
  }
}

// the list entry (record index) of a sorted key
__device__ __forceinline__ uint32_t entry_of(uint64_t x, const uint32_t* __restrict__ vin,
                                             int64_t s0, bool direct) {
  return direct ? (uint32_t)x : vin[s0 + (uint32_t)x];
}

// vout[s0 + p] = vin[s0 + position of sorted key p] for this lane's keys
template <int E>
__device__ __forceinline__ void gather_keys(const uint64_t (&x)[E], const uint32_t* __restrict__ vin,
                                            uint32_t* __restrict__ vout, int64_t s0, int base,
                                            int n, int lane, bool direct) {
  uint32_t r[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = base + lane * E + e;
    r[e] = p < n ? entry_of(x[e], vin, s0, direct) : 0u;
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = base + lane * E + e;
    if (p < n) vout[s0 + p] = r[e];
  }
}

template <int E>
__device__ __forceinline__ void sort_tiny(const uint64_t* __restrict__ keys,
                                          const uint32_t* __restrict__ vin,
                                          uint32_t* __restrict__ vout, int64_t s0, int n,
                                          int lane, bool direct) {
  uint64_t x[E];
  load_keys<E>(x, keys, s0, 0, n, 0u, lane, direct);
  NetSort<E, kWave * E>::run(x, lane);
  gather_keys<E>(x, vin, vout, s0, 0, n, lane, direct);
}

// list i of the launch order if it is tiny (fewer than kTsTiny entries), by
// one wave
__device__ __forceinline__ void tiny_list(const uint64_t* __restrict__ keys,
                                          const uint32_t* __restrict__ vin,
                                          uint32_t* __restrict__ vout,
                                          const int32_t* __restrict__ start,
                                          const int32_t* __restrict__ order, int i, int64_t cap,
                                          bool direct, int lane) {
  int64_t s0;
  int n;
  list_of(start, order, i, cap, s0, n);
  if (n >= kTsTiny || n <= 0) return;
  if (n == 1) {
    if (lane == 0) vout[s0] = direct ? (uint32_t)keys[s0] : vin[s0];
  } else if (n <= kWave) {
    sort_tiny<1>(keys, vin, vout, s0, n, lane, direct);
  } else if (n <= 2 * kWave) {
    sort_tiny<2>(keys, vin, vout, s0, n, lane, direct);
  } else if (n <= 4 * kWave) {
    sort_tiny<4>(keys, vin, vout, s0, n, lane, direct);
  } else {
    sort_tiny<8>(keys, vin, vout, s0, n, lane, direct);
  }
}

// Launch-order positions where the lists drop below kTsLarge, kTsChunk and
// kTsTiny entries: the starts of the corresponding length buckets, read from
// the (bucket, chunk) offsets of the launch-order sort.
__device__ __forceinline__ void class_bounds(const int32_t* ocnt, int nchunk, int& h, int& l,
                                             int& t) {
  h = ocnt[2 * nchunk];  // lengths >= 2^14
  l = ocnt[5 * nchunk];  // lengths >= 2^11
  t = ocnt[7 * nchunk];  // lengths >= 2^9
}

// LDS slot of network position p in the steps between waves: inside each
// wave's 512 positions, key e of lane l goes to e 64 + l, so the 64 lanes of
// a store, of a load at p ^ j (j >= 512: the same lane and key of another
// wave) and of a load at p ^ (k - 1) (lane 63 - l, key 7 - e) touch
// consecutive slots (no bank conflicts; lane-major, a lane's eight keys were
// 64 bytes apart)
__device__ __forceinline__ int ts_swz(int p) {
  return (p & ~(kTsWaveKeys - 1)) | ((p & (kTsE - 1)) * kWave) | ((p / kTsE) & (kWave - 1));
}

// small lists, the chunks of large lists, then the tiny lists.  Work items
// are the kTsMaxChunks chunks of every large list, then one item per small
// list.  Each wave sorts its 512 keys in registers; merges of 1024 and 2048
// keys take their steps between waves through LDS.  A small list is written
// out, a large list's chunk goes back in place as sorted composite keys.
// After its items every wave sorts tiny lists, one at a time, starting from
// the workgroups numbered last (those with no item when the items are fewer
// than the workgroups).  Launched with kTsChunkBlocks workgroups of 256.
__global__ __launch_bounds__(256) void k_tile_sort(uint64_t* __restrict__ keys,
                                                          const uint32_t* __restrict__ vin,
                                                          uint32_t* __restrict__ vout,
                                                          const int32_t* __restrict__ start,
                                                          const int32_t* __restrict__ order,
                                                          const int32_t* __restrict__ ocnt,
                                                          int nchunk, int total_tiles,
                                                          int64_t cap, bool direct) {
  __shared__ uint64_t s[kTsChunk];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int base = wave * kTsWaveKeys;
  int lh, ll, lt;
  class_bounds(ocnt, nchunk, lh, ll, lt);
  const int64_t n_large_items = (int64_t)kTsMaxChunks * (ll - lh);
  const int64_t n_items = n_large_items + (lt - ll);
  for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    int i, c;
    if (item < n_large_items) {
      i = lh + (int)(item / kTsMaxChunks);
      c = (int)(item % kTsMaxChunks);
    } else {
      i = ll + (int)(item - n_large_items);
      c = 0;
    }
    int64_t s0;
    int n;
    list_of(start, order, i, cap, s0, n);
    const int c0 = c * kTsChunk;
    if (c0 >= n) continue;
    const int len = min(kTsChunk, n - c0);
    uint64_t x[kTsE];
    load_keys<kTsE>(x, keys, s0 + c0, base, len, (uint32_t)c0, lane, direct);
    NetSort<kTsE, kTsWaveKeys>::run(x, lane);
    const int mtop = next_pow2(len);  // merges above this size leave the keys in place
    for (int k = 2 * kTsWaveKeys; k <= mtop; k <<= 1) {
      for (int j = k >> 1; j >= kTsWaveKeys; j >>= 1) {
#pragma unroll
        for (int e = 0; e < kTsE; ++e) s[ts_swz(base + lane * kTsE + e)] = x[e];
        __syncthreads();
#pragma unroll
        for (int e = 0; e < kTsE; ++e) {
          const int p = base + lane * kTsE + e;
          const int q = (j == (k >> 1)) ? (p ^ (k - 1)) : (p ^ j);
          const uint64_t y = s[ts_swz(q)];
          x[e] = ((y < x[e]) == (p < q)) ? y : x[e];
        }
        __syncthreads();
      }
      NetMerge<kTsE, 4 * kTsChunk, kTsWaveKeys / 2>::run(x, lane);
    }
    if (n < kTsChunk) {
      gather_keys<kTsE>(x, vin, vout, s0, base, n, lane, direct);
    } else {
#pragma unroll
      for (int e = 0; e < kTsE; ++e) {
        const int p = base + lane * kTsE + e;
        if (p < len) keys[s0 + c0 + p] = x[e];
      }
    }
  }
  constexpr int kWpg = 256 / kWave;
  const int gw = ((int)gridDim.x - 1 - (int)blockIdx.x) * kWpg + wave;
  for (int i = lt + gw; i < total_tiles; i += (int)gridDim.x * kWpg)
    tiny_list(keys, vin, vout, start, order, i, cap, direct, lane);
}

// lists of kTsLarge entries or more: the same network on the keys in global
// memory (rewritten in place as composite keys), by one workgroup
__device__ void sort_list_global(uint64_t* __restrict__ keys, const uint32_t* __restrict__ vin,
                                 uint32_t* __restrict__ vout, int64_t s0, int n, bool direct) {
  uint64_t* g = keys + s0;
  if (!direct)
    for (int q = threadIdx.x; q < n; q += blockDim.x)
      g[q] = ((uint64_t)(uint32_t)g[q] << 32) | (uint32_t)q;
  __syncthreads();
  const int m = next_pow2(n);
  for (int k = 2; k <= m; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int q = threadIdx.x; q < (m >> 1); q += blockDim.x) {
        const int a = cmp_lower(q, j);
        const int b = (j == (k >> 1)) ? (a ^ (k - 1)) : (a + j);
        if (b >= n) continue;  // the padded partner holds the largest key
        const uint64_t x = g[a], y = g[b];
        if (y < x) {
          g[a] = y;
          g[b] = x;
        }
      }
      __syncthreads();
    }
  }
  for (int q = threadIdx.x; q < n; q += blockDim.x) vout[s0 + q] = entry_of(g[q], vin, s0, direct);
  __syncthreads();
}

// large lists: rank merge of their sorted chunks.  Work items are slices of
// kTsMergeSlice entries of every large list, so the longest list is placed by
// several workgroups at once; each stages the whole list in LDS and walks the
// binary searches of its entries in step (fixed-step, branch-free lower
// bounds), so their LDS reads overlap.  The first items are the huge lists,
// one workgroup each (sort_list_global).
constexpr int kTsMergeSlice = 2048;
constexpr int kTsMergeBlocks = 512;

__global__ __launch_bounds__(1024) void k_tile_sort_merge(uint64_t* __restrict__ keys,
                                                          const uint32_t* __restrict__ vin,
                                                          uint32_t* __restrict__ vout,
                                                          const int32_t* __restrict__ start,
                                                          const int32_t* __restrict__ order,
                                                          const int32_t* __restrict__ ocnt,
                                                          int nchunk, int64_t cap, bool direct) {
  constexpr int NTH = 1024, EL = kTsLarge / NTH, E = kTsMergeSlice / NTH;
  constexpr int SLICES = kTsLarge / kTsMergeSlice;
  __shared__ uint64_t s[kTsLarge];
  int lh, ll, lt;
  class_bounds(ocnt, nchunk, lh, ll, lt);
  const int64_t n_items = lh + (int64_t)SLICES * (ll - lh);
  for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    int64_t s0;
    int n;
    if (item < lh) {
      list_of(start, order, (int)item, cap, s0, n);
      sort_list_global(keys, vin, vout, s0, n, direct);
      continue;
    }
    const int i = lh + (int)((item - lh) / SLICES);
    const int q0 = (int)((item - lh) % SLICES) * kTsMergeSlice;
    list_of(start, order, i, cap, s0, n);
    if (q0 >= n) continue;
    uint64_t v[EL];
#pragma unroll
    for (int e = 0; e < EL; ++e) {
      const int q = threadIdx.x + e * NTH;
      v[e] = q < n ? keys[s0 + q] : ~0ull;
    }
#pragma unroll
    for (int e = 0; e < EL; ++e) {
      const int q = threadIdx.x + e * NTH;
      if (q < n) s[q] = v[e];
    }
    __syncthreads();
    const int nc = (n + kTsChunk - 1) / kTsChunk;
    const int qe = min(n, q0 + kTsMergeSlice);
    uint64_t x[E];
    int pos[E], own[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int q = q0 + threadIdx.x + e * NTH;
      x[e] = q < qe ? s[q] : ~0ull;
      own[e] = q / kTsChunk;
      pos[e] = q % kTsChunk;
    }
    for (int d = 0; d < nc; ++d) {
      const int base = d * kTsChunk, len = min(kTsChunk, n - base);
      int lo[E];
#pragma unroll
      for (int e = 0; e < E; ++e) lo[e] = 0;
      // entries of chunk d below x: the largest lo with s[base + lo - 1] < x
      for (int step = kTsChunk; step > 0; step >>= 1) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int t = lo[e] + step;
          if (own[e] != d && t <= len && s[base + t - 1] < x[e]) lo[e] = t;
        }
      }
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (own[e] != d) pos[e] += lo[e];
    }
    uint32_t r[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int q = q0 + threadIdx.x + e * NTH;
      r[e] = q < qe ? entry_of(x[e], vin, s0, direct) : 0u;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int q = q0 + threadIdx.x + e * NTH;
      if (q < qe) vout[s0 + pos[e]] = r[e];
    }
    __syncthreads();
  }
}


int sort_passes(int total_tiles, bool by_tile) {
  int tb = 1;
  while ((1ll << tb) < (long long)total_tiles + 1) ++tb;
  return by_tile ? (tb + 7) / 8 : (32 + tb + 7) / 8;
}

size_t sort_hist_words(int64_t cap_dup) { return (size_t)256 * scan_blocks(cap_dup); }

size_t order_count_words(int total_tiles) {
  return (size_t)kOrderBuckets * ((total_tiles + kOrderChunk - 1) / kOrderChunk) + 4;
}

hipError_t launch_sort(const SortArgs& a, hipStream_t st) {
  const int nchunk = (a.total_tiles + kOrderChunk - 1) / kOrderChunk;
  // pairs in emission order come from s3r_project_cull (a.pair_off, the pair
  // count in counters[S3R_CNT_DUP]); launch grids are sized by the capacity
  // and workgroups past the pair count return at once
  const int64_t bin_grid = (a.cap_dup + kBinBlock - 1) / kBinBlock;
  const bool binned =
      a.by_tile && a.total_tiles <= min(kBinMaxTiles, tune(S3R_TUNE_BIN_MAX_TILES));
  const uint64_t* parted = a.keys;
  const uint32_t* pvals = a.vals0;
  if (binned) {
    // 1. pairs per tile, 2. pairs into their lists as (depth bits << 32 |
    // record) keys, the list starts and the launch order by the placement
    // launch's last workgroup
    S3R_LAUNCH(K_TILE_BIN, k_bin_zero, dim3((a.total_tiles + 255) / 256), dim3(256), 0, st,
               a.bin_count, a.bin_cursor, a.total_tiles);
    S3R_LAUNCH(K_TILE_BIN, k_bin_count, dim3((unsigned)(bin_grid > 0 ? bin_grid : 1)),
               dim3(kBinThreads), 0, st, a);
    S3R_LAUNCH(K_TILE_BIN, k_bin_place, dim3((unsigned)((bin_grid > 0 ? bin_grid : 0) + 1)),
               dim3(kBinThreads), 0, st, a, nchunk);
  } else {
    // radix passes over the tile bits only (then a depth sort per list) or
    // over all key bits; the values of a full sort end in the caller's array
    const int passes = sort_passes(a.total_tiles, a.by_tile);
    const int shift0 = a.by_tile ? 32 : 0;
    const int nblk = scan_blocks(a.cap_dup) > 0 ? scan_blocks(a.cap_dup) : 1;
    uint64_t* kb[2] = {a.keys, a.keys_alt};
    uint32_t* vb[2] = {a.vals0, a.vals1};
    if (!a.by_tile) vb[passes & 1] = a.vals_out;
    // 1. emit (tile, depth) keys in record order
    {
      SortArgs ea = a;
      ea.vals0 = vb[0];
      const int64_t want = (a.cap_dup + kEmitBlock - 1) / kEmitBlock;
      const int grid = (int)(want < 4096 ? (want > 0 ? want : 1) : 4096);
      S3R_LAUNCH(K_EMIT, k_emit_pairs, dim3(grid), dim3(kEmitThreads), 0, st, ea);
    }
    // 2. radix passes
    for (int p = 0; p < passes; ++p) {
      const int shift = shift0 + 8 * p;
      const int src = p & 1, dst = src ^ 1;
      S3R_LAUNCH(K_RADIX, k_radix_hist, dim3(nblk), dim3(kRT), 0, st, kb[src],
                 a.counters + S3R_CNT_DUP, shift, a.hist, a.misc + 2);
      hipError_t e = scan_i32(a.hist, a.misc + 2, (int64_t)256 * nblk, a.hist, a.scan_sums,
                              a.misc + 1, st);
      if (e != hipSuccess) return e;
      S3R_LAUNCH(K_RADIX, k_radix_scatter, dim3(nblk), dim3(kRT), 0, st, kb[src], vb[src],
                 kb[dst], vb[dst], a.counters + S3R_CNT_DUP, shift, a.hist);
    }
    parted = kb[passes & 1];
    pvals = vb[passes & 1];
    // 3. tile ranges and the launch order
    {
      const int64_t want = (a.cap_dup + 1 + 255) / 256;
      const int grid = (int)(want < 1024 ? want : 1024);
      S3R_LAUNCH(K_TILE_RANGES, k_tile_ranges, dim3(grid), dim3(256), 0, st, parted,
                 a.counters + S3R_CNT_DUP, a.total_tiles, a.tile_start);
    }
    if (nchunk > 0)
      S3R_LAUNCH(K_TILE_ORDER, k_order_count, dim3(nchunk), dim3(kOrderThreads), 0, st,
                 a.tile_start, a.total_tiles, nchunk, a.order_cnt, a.tile_count);
    S3R_LAUNCH(K_TILE_ORDER, k_order_top, dim3(1), dim3(1024), 0, st, a.order_cnt,
               kOrderBuckets * nchunk, a.tile_start, a.tile_offset, a.nv, a.stats);
    if (nchunk > 0)
      S3R_LAUNCH(K_TILE_ORDER, k_order_place, dim3(nchunk), dim3(kOrderThreads), 0, st,
                 a.tile_start, a.total_tiles, nchunk, a.order_cnt, a.tile_order);
  }
  // 4. depth order inside every list, written to the caller's value array
  if (a.by_tile) {
    uint64_t* keys = const_cast<uint64_t*>(parted);
    S3R_LAUNCH(K_TILE_SORT, k_tile_sort, dim3(kTsChunkBlocks), dim3(256), 0, st, keys,
               pvals, a.vals_out, a.tile_start, a.tile_order, a.order_cnt, nchunk,
               a.total_tiles, a.cap_dup, binned);
    S3R_LAUNCH(K_TILE_SORT_MERGE, k_tile_sort_merge, dim3(kTsMergeBlocks), dim3(1024), 0, st,
               keys, pvals, a.vals_out, a.tile_start, a.tile_order, a.order_cnt, nchunk,
               a.cap_dup, binned);
  }
  return hipGetLastError();
}

}  // namespace s3r
