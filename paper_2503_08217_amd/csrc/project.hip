// Front end of the per-view step (Sec. 3.3): instance cameras, temporal
// selection, projection (Eq. 1), frustum mask M_t, LOD cull, SH colour of the
// survivors, and compaction of the survivors into records.
//
// Kernels, none of which waits on another workgroup or uses a contended
// atomic:
//   k_cull           each workgroup owns 256 consecutive Gaussians and loops
//                    over the batch's views (a Gaussian's 44 bytes of geometry
//                    are read once per batch); decisions become M_t bits and
//                    survivor bits through wave ballots, plus per-(block,
//                    view) counts of records and of (tile, record) pairs
//   k_off_*          exclusive scans of the counts (chunk sums, one small
//                    top scan, chunk rescans) give the first record and the
//                    first pair of every (block, view)
//   k_records        one wave per Gaussian block: its survivors (only,
//                    packed densely over the lanes) re-project, query their
//                    colour and write their record at base + rank within the
//                    block, with the record's first pair in emission order
// Records come out ordered by Gaussian block, then view, then Gaussian.
#include "internal.hpp"

namespace s3r {

// ---------------------------------------------------------------------------
// a1: instance cameras P_{v,k} = W_v G_{tau_v,k} (FP64, rounded once) and the
//     normalised time of each view.
// ---------------------------------------------------------------------------
__global__ void k_compose(const float* __restrict__ W, const int32_t* __restrict__ tstep,
                          const float* __restrict__ pose, int S, int T, int nv,
                          float* __restrict__ cam, float* __restrict__ cen,
                          float* __restrict__ t_norm, int32_t* __restrict__ counters,
                          int32_t* __restrict__ stats) {
  const int v = blockIdx.x;
  const int tau = clampi(tstep[v], 0, T - 1);
  // the call's device counters and this view's statistics start at zero
  if (threadIdx.x < 4) stats[4 * v + threadIdx.x] = 0;
  if (v == 0 && threadIdx.x < 16) counters[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    t_norm[v] = (T > 1) ? (float)(-1.0 + (2.0 * (double)tau) / (double)(T - 1)) : 0.0f;
  }
  double w[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) w[q] = (double)W[v * 12 + q];
  for (int k = threadIdx.x; k < S; k += blockDim.x) {
    const float* G = pose + ((size_t)tau * S + k) * 12;
    double g[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) g[q] = (double)G[q];
    double P[12];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double acc = w[r * 4 + 0] * g[0 * 4 + c];
        acc = acc + w[r * 4 + 1] * g[1 * 4 + c];
        acc = acc + w[r * 4 + 2] * g[2 * 4 + c];
        acc = acc + w[r * 4 + 3] * (c == 3 ? 1.0 : 0.0);
        P[r * 4 + c] = acc;
      }
    }
    float* o = cam + ((size_t)v * S + k) * 12;
#pragma unroll
    for (int q = 0; q < 12; ++q) o[q] = (float)P[q];
    float* ce = cen + ((size_t)v * S + k) * 4;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double s = (P[0 * 4 + j] * P[3] + P[1 * 4 + j] * P[7]) + P[2 * 4 + j] * P[11];
      ce[j] = (float)(-s);
    }
    ce[3] = 0.0f;
  }
}

// ---------------------------------------------------------------------------
// p1: conventional local->global transform (plain route): for each timestep
//     slot s, mean_w = R_G mean + t_G and rot_w = R_G R(q).
// ---------------------------------------------------------------------------
struct TsList {
  int32_t tau[kMaxViews];
};

__global__ __launch_bounds__(256) void k_plain_transform(
    const float* __restrict__ mean, const float* __restrict__ quat,
    const int32_t* __restrict__ inst, const float* __restrict__ pose, int n, int S, TsList ts,
    int n_ts, float* __restrict__ mean_w, float* __restrict__ rot_w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float mx = mean[3 * i], my = mean[3 * i + 1], mz = mean[3 * i + 2];
  const float4 q = reinterpret_cast<const float4*>(quat)[i];
  float Rq[9];
  quat_rot(q.x, q.y, q.z, q.w, Rq);
  const int k = clampi(inst[i], 0, S - 1);
  for (int s = 0; s < n_ts; ++s) {
    const float* G = pose + ((size_t)ts.tau[s] * S + k) * 12;
    float g[12];
#pragma unroll
    for (int t = 0; t < 12; ++t) g[t] = G[t];
    float* mw = mean_w + ((size_t)s * n + i) * 3;
    mw[0] = ((g[0] * mx + g[1] * my) + g[2] * mz) + g[3];
    mw[1] = ((g[4] * mx + g[5] * my) + g[6] * mz) + g[7];
    mw[2] = ((g[8] * mx + g[9] * my) + g[10] * mz) + g[11];
    float* rw = rot_w + ((size_t)s * n + i) * 9;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        rw[r * 3 + c] = (g[r * 4 + 0] * Rq[0 * 3 + c] + g[r * 4 + 1] * Rq[1 * 3 + c]) +
                        g[r * 4 + 2] * Rq[2 * 3 + c];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// a2-a5: temporal test, projection, M_t, LOD, colour, compaction.
// ---------------------------------------------------------------------------
struct Loaded {
  float mx, my, mz;
  float R[9];  // the Gaussian's rotation (local, or world for the plain route)
  float s0, s1, s2;
  int k;
};

__device__ __forceinline__ void load_camera(const float* __restrict__ cam, int v, int S, int slot,
                                            float P[12]) {
  const float4* c4 = reinterpret_cast<const float4*>(cam + ((size_t)v * S + slot) * 12);
  float4 a = c4[0], b = c4[1], c = c4[2];
  P[0] = a.x; P[1] = a.y; P[2] = a.z; P[3] = a.w;
  P[4] = b.x; P[5] = b.y; P[6] = b.z; P[7] = b.w;
  P[8] = c.x; P[9] = c.y; P[10] = c.z; P[11] = c.w;
}

__device__ __forceinline__ void load_gaussian(const ProjArgs& a, int i, bool need, bool plain,
                                              Loaded& g) {
  g.mx = g.my = g.mz = 0.f;
  g.s0 = g.s1 = g.s2 = 0.f;
  g.k = 0;
#pragma unroll
  for (int t = 0; t < 9; ++t) g.R[t] = 0.f;
  if (!need) return;
  g.mx = a.mean[3 * i]; g.my = a.mean[3 * i + 1]; g.mz = a.mean[3 * i + 2];
  g.s0 = a.scale[3 * i]; g.s1 = a.scale[3 * i + 1]; g.s2 = a.scale[3 * i + 2];
  g.k = clampi(a.inst[i], 0, a.n_slots - 1);
  if (!plain) {
    const float4 q = reinterpret_cast<const float4*>(a.quat)[i];
    quat_rot(q.x, q.y, q.z, q.w, g.R);
  }
}

__device__ __forceinline__ void view_geometry(const ProjArgs& a, int v, const Loaded& g,
                                              bool plain, int i, Loaded& eff, float P[12],
                                              float& fx, float& fy, float& cx, float& cy, int& W,
                                              int& H) {
  const float4 kv = reinterpret_cast<const float4*>(a.Kv)[v];
  fx = kv.x; fy = kv.y; cx = kv.z; cy = kv.w;
  W = a.wh[2 * v];
  H = a.wh[2 * v + 1];
  eff = g;
  if (plain) {
    const int slot = a.plain_slot[v];
    const float* mw = a.mean_w + ((size_t)slot * a.n + i) * 3;
    eff.mx = mw[0]; eff.my = mw[1]; eff.mz = mw[2];
    const float* rw = a.rot_w + ((size_t)slot * a.n + i) * 9;
#pragma unroll
    for (int t = 0; t < 9; ++t) eff.R[t] = rw[t];
    load_camera(a.cam, v, a.n_slots, 0, P);
  } else {
    load_camera(a.cam, v, a.n_slots, g.k, P);
  }
}

// Phase A: decisions of every (view, Gaussian) of the block.  Writes the M_t
// bits, the survivor bits and the block's per-view counts (N_t, N_f, N_r).
__global__ __launch_bounds__(kProjBlock) void k_cull(ProjArgs a) {
  __shared__ int s_cnt[kMaxViews][kProjWaves][4];
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = tid % kWave;
  const int vb = blockIdx.x;
  const int i = vb * kProjBlock + tid;
  const bool valid = i < a.n;
  const bool plain = (a.kp.flags & S3R_PLAIN) != 0;
  const bool temporal = (a.kp.flags & S3R_TEMPORAL) != 0;

  // temporal selection first: a Gaussian whose interval excludes every view's
  // time is never read further (Sec. 3.3, select before projecting)
  uint64_t pass_bits = 0;
  if (valid) {
    if (temporal) {
      const float vs = a.vis_s[i];
      const float ve = a.vis_e[i];
      for (int v = 0; v < a.nv; ++v) {
        const float t = a.t_norm[v];
        if ((vs <= t) && (t <= ve)) pass_bits |= 1ull << v;
      }
    } else {
      pass_bits = (a.nv >= 64) ? ~0ull : ((1ull << a.nv) - 1ull);
    }
  }
  Loaded g;
  load_gaussian(a, i, pass_bits != 0, plain, g);

  for (int v = 0; v < a.nv; ++v) {
    const bool pass_t = (pass_bits >> v) & 1ull;
    bool vis = false, surv = false;
    int npairs = 0;  // tiles of the footprint rectangle of a survivor
    if (pass_t) {
      Loaded e;
      float P[12], fx, fy, cx, cy;
      int W, H;
      view_geometry(a, v, g, plain, i, e, P, fx, fy, cx, cy, W, H);
      // a Gaussian behind the camera (or beyond z_far) fails M_t on its depth
      // alone: skip the covariance, eigenvalue and rectangle (most pairs of a
      // surround rig; the decision is the same one project_canonical takes)
      if (depth_pass(cam_depth(P, e.mx, e.my, e.mz), a.kp)) {
        Proj o;
        project_canonical(P, e.mx, e.my, e.mz, e.R, e.s0, e.s1, e.s2, fx, fy, cx, cy, W, H, a.kp,
                          o, i, v);
        vis = o.visible;
        surv = vis && o.keep;
        npairs = surv ? (o.x1 - o.x0) * (o.y1 - o.y0) : 0;
      }
    }
    const uint64_t bt = ballot(pass_t);
    const uint64_t bf = ballot(vis);
    const uint64_t bs = ballot(surv);
    const int wp = bs != 0ull ? (int)wave_sum_u32((uint32_t)npairs) : 0;
    if (lane == 0) {
      const int gw = vb * kProjWaves + wave;
      if ((int64_t)gw * kWave < a.n) {
        uint32_t* m = a.mask + (size_t)v * a.mask_words + 2 * (size_t)gw;
        m[0] = (uint32_t)bf;
        m[1] = (uint32_t)(bf >> 32);
        uint32_t* sb = a.surv + (size_t)v * a.mask_words + 2 * (size_t)gw;
        sb[0] = (uint32_t)bs;
        sb[1] = (uint32_t)(bs >> 32);
      }
      s_cnt[v][wave][0] = __popcll(bt);
      s_cnt[v][wave][1] = __popcll(bf);
      s_cnt[v][wave][2] = __popcll(bs);
      s_cnt[v][wave][3] = wp;
    }
  }
  __syncthreads();
  for (int v = tid; v < a.nv; v += kProjBlock) {
    int nt = 0, nf = 0, nr = 0, np = 0;
    for (int w = 0; w < kProjWaves; ++w) {
      nt += s_cnt[v][w][0];
      nf += s_cnt[v][w][1];
      nr += s_cnt[v][w][2];
      np += s_cnt[v][w][3];
    }
    int32_t* bs = a.bstat + ((size_t)vb * a.nv + v) * kBstat;
    bs[0] = nt; bs[1] = nf; bs[2] = nr; bs[4] = np;
  }
}

// Exclusive scans of the per-(block, view) record and pair counts in (block,
// view) order -> first record and first pair of each (block, view); totals
// -> counters and stats.  Over chunks of kOffChunk entries: chunk sums (and
// per-view partial stats), then each chunk rescanned with its offsets, the
// sums of the chunk sums before it -- added up by the chunk itself when there
// are at most kOffFuseMax chunks, else scanned by one workgroup in between.
// Pair sums are 64-bit (a batch may hold more pairs than any capacity).  No
// contended atomics.
constexpr int kOffChunk = 1024;
constexpr int kOffThreads = 256;
constexpr int kOffPer = kOffChunk / kOffThreads;

__device__ __forceinline__ long long shfl_up64(long long v, int o) {
  const int lo = __shfl_up((int)(uint32_t)(uint64_t)v, o, kWave);
  const int hi = __shfl_up((int)(uint32_t)((uint64_t)v >> 32), o, kWave);
  return (long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// exclusive scan of (x, y) over the workgroup in thread order; totals out
__device__ __forceinline__ void block_exclusive_scan2(int x, long long y, int* s_w,
                                                      long long* s_w64, int& ex, long long& ey,
                                                      int& total, long long& total64) {
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  int ix = x;
  long long iy = y;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int tx = __shfl_up(ix, o, kWave);
    const long long ty = shfl_up64(iy, o);
    if (lane >= o) {
      ix += tx;
      iy += ty;
    }
  }
  if (lane == kWave - 1) {
    s_w[wave] = ix;
    s_w64[wave] = iy;
  }
  __syncthreads();
  int bx = 0;
  long long by = 0;
  total = 0;
  total64 = 0;
  for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
    if (w < wave) {
      bx += s_w[w];
      by += s_w64[w];
    }
    total += s_w[w];
    total64 += s_w64[w];
  }
  __syncthreads();
  ex = bx + ix - x;
  ey = by + iy - y;
}

__global__ __launch_bounds__(kOffThreads) void k_off_reduce(const int32_t* __restrict__ bstat,
                                                           int64_t total, int nv,
                                                           int32_t* __restrict__ csum,
                                                           long long* __restrict__ csum_p,
                                                           int32_t* __restrict__ cstat) {
  __shared__ int s_w[kOffThreads / kWave];
  __shared__ long long s_w64[kOffThreads / kWave];
  __shared__ int s_stat[kMaxViews][3];
  const int tid = threadIdx.x;
  const int64_t c = blockIdx.x;
  for (int q = tid; q < nv * 3; q += kOffThreads) s_stat[q / 3][q % 3] = 0;
  __syncthreads();
  int sum = 0;
  long long psum = 0;
  for (int m = 0; m < kOffPer; ++m) {
    const int64_t e = c * kOffChunk + (int64_t)m * kOffThreads + tid;
    if (e < total) {
      const int4 bs = reinterpret_cast<const int4*>(bstat)[e * (kBstat / 4)];
      const int v = (int)(e % nv);
      sum += bs.z;
      psum += bstat[e * kBstat + 4];
      if (bs.x) atomicAdd(&s_stat[v][0], bs.x);
      if (bs.y) atomicAdd(&s_stat[v][1], bs.y);
      if (bs.z) atomicAdd(&s_stat[v][2], bs.z);
    }
  }
  int ex, tot;
  long long ey, tot64;
  block_exclusive_scan2(sum, psum, s_w, s_w64, ex, ey, tot, tot64);
  if (tid == 0) {
    csum[c] = tot;
    csum_p[c] = tot64;
  }
  for (int q = tid; q < nv * 3; q += kOffThreads) cstat[(c * nv + q / 3) * 3 + q % 3] = s_stat[q / 3][q % 3];
}

// survivor and pair totals -> counters (records beyond cap_surv dropped; the
// pairs are settled by k_records, which knows the last kept record's pairs)
__device__ __forceinline__ void store_totals(int32_t* counters, long long surv, long long pairs,
                                             int64_t cap_surv) {
  counters[S3R_CNT_SURV] = (int32_t)min(surv, (long long)cap_surv);
  counters[S3R_CNT_OVF_SURV] = (int32_t)max(0ll, surv - (long long)cap_surv);
  counters[S3R_CNT_PAIRS] = (int32_t)min(pairs, (long long)INT32_MAX);
}

__global__ __launch_bounds__(1024) void k_off_top(int32_t* __restrict__ csum,
                                                  long long* __restrict__ csum_p, int nchunk,
                                                  int nv, const int32_t* __restrict__ cstat,
                                                  int32_t* __restrict__ counters,
                                                  int32_t* __restrict__ stats, int64_t cap_surv) {
  __shared__ int s_w[1024 / kWave];
  __shared__ long long s_w64[1024 / kWave];
  const int tid = threadIdx.x;
  const int per = (nchunk + 1023) / 1024;
  const int c0 = min(nchunk, tid * per), c1 = min(nchunk, c0 + per);
  int sum = 0;
  long long psum = 0;
  for (int c = c0; c < c1; ++c) {
    sum += csum[c];
    psum += csum_p[c];
  }
  int run, tot;
  long long run64, tot64;
  block_exclusive_scan2(sum, psum, s_w, s_w64, run, run64, tot, tot64);
  for (int c = c0; c < c1; ++c) {
    const int x = csum[c];
    const long long y = csum_p[c];
    csum[c] = run;
    csum_p[c] = run64;
    run += x;
    run64 += y;
  }
  if (tid == 0) store_totals(counters, tot, tot64, cap_surv);
  for (int q = tid; q < nv * 3; q += 1024) {
    int acc = 0;
    for (int c = 0; c < nchunk; ++c) acc += cstat[((int64_t)c * nv + q / 3) * 3 + q % 3];
    stats[(q / 3) * 4 + (q % 3)] = acc;
  }
}

// kPrefix (at most kOffFuseMax chunks): in place of k_off_top, each chunk
// adds up the chunk sums before it, the chunks share out the per-view
// statistics, and the last chunk stores the totals
constexpr int kOffFuseMax = 1024;

template <bool kPrefix>
__global__ __launch_bounds__(kOffThreads) void k_off_down(int32_t* __restrict__ bstat,
                                                         int64_t total,
                                                         const int32_t* __restrict__ csum,
                                                         const long long* __restrict__ csum_p,
                                                         int64_t cap_surv, int nchunk, int nv,
                                                         const int32_t* __restrict__ cstat,
                                                         int32_t* __restrict__ counters,
                                                         int32_t* __restrict__ stats) {
  __shared__ int s_w[kOffThreads / kWave];
  __shared__ long long s_w64[kOffThreads / kWave];
  const int tid = threadIdx.x;
  const int64_t c = blockIdx.x;
  int before;
  long long before_p;
  if (kPrefix) {
    int p = 0;
    long long pp = 0;
    for (int q = tid; q < (int)c; q += kOffThreads) {
      p += csum[q];
      pp += csum_p[q];
    }
    int ex;
    long long ey;
    block_exclusive_scan2(p, pp, s_w, s_w64, ex, ey, before, before_p);
    // statistic q of the views (3 per view) is summed over the chunks by
    // chunk q mod nchunk
    for (int q = (int)c; q < nv * 3; q += nchunk) {
      int acc = 0;
      for (int k = tid; k < nchunk; k += kOffThreads)
        acc += cstat[((int64_t)k * nv + q / 3) * 3 + q % 3];
      int all, ex2;
      long long ey2, all64;
      block_exclusive_scan2(acc, 0ll, s_w, s_w64, ex2, ey2, all, all64);
      if (tid == 0) stats[(q / 3) * 4 + (q % 3)] = all;
    }
  } else {
    before = csum[c];
    before_p = csum_p[c];
  }
  // thread t takes the kOffPer consecutive entries c*kOffChunk + t*kOffPer + m
  int cnt[kOffPer], pc[kOffPer];
  int sum = 0;
  long long psum = 0;
#pragma unroll
  for (int m = 0; m < kOffPer; ++m) {
    const int64_t e = c * kOffChunk + (int64_t)tid * kOffPer + m;
    cnt[m] = e < total ? bstat[e * kBstat + 2] : 0;
    pc[m] = e < total ? bstat[e * kBstat + 4] : 0;
    sum += cnt[m];
    psum += pc[m];
  }
  int ex, tot;
  long long ey, tot64;
  block_exclusive_scan2(sum, psum, s_w, s_w64, ex, ey, tot, tot64);
  int64_t run = (int64_t)before + ex;
  long long run_p = before_p + ey;
  if (kPrefix && c == (int64_t)gridDim.x - 1 && tid == 0)
    store_totals(counters, (long long)before + tot, before_p + tot64, cap_surv);
#pragma unroll
  for (int m = 0; m < kOffPer; ++m) {
    const int64_t e = c * kOffChunk + (int64_t)tid * kOffPer + m;
    if (e < total) {
      bstat[e * kBstat + 3] = (int32_t)min(run, cap_surv);
      bstat[e * kBstat + 5] = (int32_t)min(run_p, (long long)INT32_MAX);
    }
    run += cnt[m];
    run_p += pc[m];
  }
}

// Phase C: records of the survivors, at the slots given by the block offsets.
// Position of the k-th (0-based) set bit of x (k < popcount(x)).
__device__ __forceinline__ int select_bit(uint64_t x, int k) {
  int pos = 0;
#pragma unroll
  for (int sft = 32; sft >= 1; sft >>= 1) {
    const uint64_t lo = x & ((1ull << sft) - 1ull);
    const int c = __popcll(lo);
    if (k >= c) {
      k -= c;
      x >>= sft;
      pos += sft;
    } else {
      x = lo;
    }
  }
  return pos;
}

// The block's survivors of all views are processed densely: survivor k of
// view v (in Gaussian order) is item prefix[v] + k of the block, and lane l
// of the block's one wave takes items l, l + 64, ...  Lanes are not tied to
// Gaussians: only a few per cent of a block's (Gaussian, view) pairs survive,
// so a 256-thread workgroup would leave three of its four waves idle while
// holding their slots.
constexpr int kRecThreads = kWave;
// (at most 128 VGPRs, no spills: four waves per SIMD)
__global__ __launch_bounds__(kRecThreads)
__attribute__((amdgpu_waves_per_eu(4))) void k_records(ProjArgs a) {
  __shared__ uint64_t s_w[kMaxViews][kProjWaves];
  __shared__ int s_pre[kMaxViews + 1];
  __shared__ int s_carry[kMaxViews];  // pairs of the view's items already placed
  __shared__ int s_base[kMaxViews];   // carry minus the scan at the view's first lane
  const int tid = threadIdx.x;
  const int vb = blockIdx.x;
  const bool plain = (a.kp.flags & S3R_PLAIN) != 0;
  for (int v = tid; v < a.nv; v += kRecThreads) s_carry[v] = 0;
  for (int q = tid; q < a.nv * kProjWaves; q += kRecThreads) {
    const int v = q / kProjWaves, w = q % kProjWaves;
    const int gw = vb * kProjWaves + w;
    uint64_t word = 0;
    if ((int64_t)gw * kWave < a.n) {
      const uint32_t* sb = a.surv + (size_t)v * a.mask_words + 2 * (size_t)gw;
      word = ((uint64_t)sb[1] << 32) | sb[0];
    }
    s_w[v][w] = word;
  }
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int v = 0; v < a.nv; ++v) {
      s_pre[v] = run;
      for (int w = 0; w < kProjWaves; ++w) run += __popcll(s_w[v][w]);
    }
    s_pre[a.nv] = run;
  }
  __syncthreads();
  const int total = s_pre[a.nv];
  const int B = (a.sh_deg + 1) * (a.sh_deg + 1);
  const int n_keep = a.counters[S3R_CNT_SURV];  // records kept (min(survivors, cap_surv))
  const int lane = tid;
  // survivor `item` of the block (survivors in (view, Gaussian) order):
  // its view, its record slot and its Gaussian
  auto locate = [&](int item, int& v, int64_t& slot, int& i) {
    v = 0;
    while (s_pre[v + 1] <= item) ++v;
    const int k = item - s_pre[v];
    slot = (int64_t)a.bstat[((size_t)vb * a.nv + v) * kBstat + 3] + k;
    int w = 0, kk = k;
    while (kk >= __popcll(s_w[v][w])) {
      kk -= __popcll(s_w[v][w]);
      ++w;
    }
    i = vb * kProjBlock + w * kWave + select_bit(s_w[v][w], kk);
  };
  // pass 1: projection and the geometric part of the records (and each
  // record's pair count)
  for (int item = lane; item < total; item += kRecThreads) {
    int v, i;
    int64_t slot;
    locate(item, v, slot, i);
    if (slot >= a.kp.cap_surv) continue;
    Loaded g;
    load_gaussian(a, i, true, plain, g);
    Loaded e;
    float P[12], fx, fy, cx, cy;
    int W, H;
    view_geometry(a, v, g, plain, i, e, P, fx, fy, cx, cy, W, H);
    Proj o;
    project_canonical(P, e.mx, e.my, e.mz, e.R, e.s0, e.s1, e.s2, fx, fy, cx, cy, W, H, a.kp, o,
                      i, v);
    a.rec_gid[slot] = i;
    a.rec_view[slot] = v;
    a.rec_geo[slot] = make_float4(o.u, o.v, a.opac[i], o.pz);
    {
      // the conic, and the cutoff box's x half-width (the y one goes with
      // the colour in pass 2)
      const float A = o.c / o.det, Bc = (-o.b) / o.det, C = o.a / o.det;
      a.rec_conic[slot] = make_float4(A, Bc, C, cutoff_half(A, Bc, C, a.kp.cutoff).x);
    }
    a.rec_rect[slot] = make_int4(o.x0, o.y0, o.x1, o.y1);
    a.rec_npairs[slot] = (o.x1 - o.x0) * (o.y1 - o.y0);
  }
  // pass 2 (each item on the lane that wrote it): first pairs and colours.
  // The loop bound is uniform over the wave (it holds a wave scan).
  for (int it0 = 0; it0 < total; it0 += kRecThreads) {
    const int item = it0 + lane;
    const bool live = item < total;
    int v = 0, i = 0;
    int64_t slot = INT64_MAX;
    if (live) locate(item, v, slot, i);
    const bool kept = live && slot < a.kp.cap_surv;
    const int npairs = kept ? a.rec_npairs[slot] : 0;
    // first pair of each item: its (block, view)'s first pair plus the pairs
    // of the view's items before it -- a scan over the wave in item order,
    // rebased at the first lane of each view's run and carried across
    // iterations in LDS (records past cap_surv are a suffix: their zeros
    // change no kept record's first pair)
    const int incl = wave_inclusive_scan(npairs);
    const int excl = incl - npairs;
    const bool run_start = live && (lane == 0 || item == s_pre[v]);
    const bool run_end = live && (lane == kWave - 1 || item + 1 == s_pre[v + 1]);
    if (run_start) s_base[v] = s_carry[v] - excl;
    __syncthreads();
    const int first_pair = live ? a.bstat[((size_t)vb * a.nv + v) * kBstat + 5] + s_base[v] + excl
                                : 0;
    if (run_end) s_carry[v] = s_base[v] + incl;
    __syncthreads();
    if (!kept) continue;
    // the last kept record settles the pair counters: pairs beyond it, or
    // beyond cap_dup, are dropped
    if (slot == n_keep - 1) {
      const int64_t all = a.counters[S3R_CNT_PAIRS];
      const int64_t kept_pairs = min((int64_t)first_pair + npairs, a.kp.cap_dup);
      a.counters[S3R_CNT_DUP] = (int32_t)kept_pairs;
      a.counters[S3R_CNT_OVF_DUP] = (int32_t)max((int64_t)0, all - kept_pairs);
    }
    a.rec_pair[slot] = first_pair;

    // viewing direction in the instance-local frame
    const int kslot = clampi(a.inst[i], 0, a.n_slots - 1);
    float dx, dy, dz;
    if (plain) {
      const float* mw = a.mean_w + ((size_t)a.plain_slot[v] * a.n + i) * 3;
      const float4 cw = reinterpret_cast<const float4*>(a.cen)[(size_t)v * a.n_slots];
      const float wx = mw[0] - cw.x, wy = mw[1] - cw.y, wz = mw[2] - cw.z;
      const float* G = a.pose + ((size_t)clampi(a.tstep[v], 0, a.n_ts - 1) * a.n_slots + kslot) * 12;
      dx = (G[0] * wx + G[4] * wy) + G[8] * wz;
      dy = (G[1] * wx + G[5] * wy) + G[9] * wz;
      dz = (G[2] * wx + G[6] * wy) + G[10] * wz;
    } else {
      const float4 ce = reinterpret_cast<const float4*>(a.cen)[(size_t)v * a.n_slots + kslot];
      dx = a.mean[3 * i] - ce.x;
      dy = a.mean[3 * i + 1] - ce.y;
      dz = a.mean[3 * i + 2] - ce.z;
    }
    const float nrm = sqrtf((dx * dx + dy * dy) + dz * dz);
    dx = dx / nrm; dy = dy / nrm; dz = dz / nrm;
    float Y[16];
    sh_basis(a.sh_deg, dx, dy, dz, Y);
    float f[48];
    load_sh(a.sh + (size_t)i * B * 3, B, f);
    float r = 0.f, gg = 0.f, bb = 0.f;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if (q < B) {
        r = fmaf(Y[q], f[3 * q], r);
        gg = fmaf(Y[q], f[3 * q + 1], gg);
        bb = fmaf(Y[q], f[3 * q + 2], bb);
      }
    }
    r = fmaxf(r + 0.5f, 0.f);
    gg = fmaxf(gg + 0.5f, 0.f);
    bb = fmaxf(bb + 0.5f, 0.f);

    const float4 cq = a.rec_conic[slot];  // (written by this lane in pass 1)
    a.rec_rgb[slot] = make_float4(r, gg, bb, cutoff_half(cq.x, cq.y, cq.z, a.kp.cutoff).y);
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hipError_t launch_compose(const float* W, const int32_t* tstep, const float* pose, int S, int T,
                          int nv, float* cam, float* cen, float* t_norm, int32_t* counters,
                          int32_t* stats, hipStream_t st) {
  S3R_LAUNCH(K_COMPOSE, k_compose, dim3(nv), dim3(128), 0, st, W, tstep, pose, S, T, nv, cam, cen,
             t_norm, counters, stats);
  return hipGetLastError();
}

hipError_t launch_plain_transform(const float* mean, const float* quat, const int32_t* inst,
                                  const float* pose, int n, int S, const int32_t* tsteps, int n_ts,
                                  float* mean_w, float* rot_w, hipStream_t st) {
  TsList ts;
  for (int s = 0; s < kMaxViews; ++s) ts.tau[s] = s < n_ts ? tsteps[s] : 0;
  const int grid = (n + 255) / 256;
  if (grid > 0)
    S3R_LAUNCH(K_PLAIN_TRANSFORM, k_plain_transform, dim3(grid), dim3(256), 0, st, mean, quat, inst, pose, n,
                       S, ts, n_ts, mean_w, rot_w);
  return hipGetLastError();
}

int project_blocks(int64_t n) { return (int)((n + kProjBlock - 1) / kProjBlock); }

int offset_chunks(int64_t nblk, int nv) {
  return (int)((nblk * nv + kOffChunk - 1) / kOffChunk);
}

hipError_t launch_project(const ProjArgs& a, int32_t* stats, hipStream_t st) {
  if (a.nblk > 0) S3R_LAUNCH(K_PROJECT, k_cull, dim3(a.nblk), dim3(kProjBlock), 0, st, a);
  const int64_t total = (int64_t)a.nblk * a.nv;
  const int nchunk = offset_chunks(a.nblk, a.nv);
  if (nchunk > 0)
    S3R_LAUNCH(K_STATS, k_off_reduce, dim3(nchunk), dim3(kOffThreads), 0, st, a.bstat, total, a.nv,
               a.chunk_sum, a.chunk_sum_p, a.chunk_stat);
  if (nchunk > 0 && nchunk <= min(kOffFuseMax, tune(S3R_TUNE_OFFSET_FUSE_MAX))) {
    // counters and statistics start at zero (k_compose), so no chunks, no launch
    S3R_LAUNCH(K_STATS, k_off_down<true>, dim3(nchunk), dim3(kOffThreads), 0, st, a.bstat, total,
               a.chunk_sum, a.chunk_sum_p, a.kp.cap_surv, nchunk, a.nv, a.chunk_stat, a.counters,
               stats);
  } else if (nchunk > 0) {
    S3R_LAUNCH(K_STATS, k_off_top, dim3(1), dim3(1024), 0, st, a.chunk_sum, a.chunk_sum_p, nchunk,
               a.nv, a.chunk_stat, a.counters, stats, a.kp.cap_surv);
    S3R_LAUNCH(K_STATS, k_off_down<false>, dim3(nchunk), dim3(kOffThreads), 0, st, a.bstat, total,
               a.chunk_sum, a.chunk_sum_p, a.kp.cap_surv, nchunk, a.nv, a.chunk_stat, a.counters,
               stats);
  }
  if (a.nblk > 0) S3R_LAUNCH(K_RECORDS, k_records, dim3(a.nblk), dim3(kRecThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace s3r
