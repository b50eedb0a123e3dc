// Backward pass of the per-view step.
//
// k_raster_bwd replays each tile back to front from the stored final
// transmittance and the position of the last contributor, recovering
// T_i = T_{i+1} / (1 - alpha_i) instead of storing per-pixel lists.  With
// C = sum_i c_i alpha_i T_i + T_N bg and S_i = sum_{j>i} c_j alpha_j T_j:
//   dL/dc_i     = alpha_i T_i dL/dC
//   dL/dalpha_i = T_i c_i . dL/dC - (S_i + T_N bg) . dL/dC / (1 - alpha_i)
// and alpha_i = min(alpha_max, o_i exp(power_i)) chains to the 2D mean, the
// conic and the opacity.  A thread owns one pixel and a wave64 an 8x8
// sub-tile; each wave replays only the list entries up to its own last
// contributor, 64 at a time, keeping with one ballot the entries whose cutoff
// box meets its sub-tile.  A record's nine gradient components are summed
// over the wave (permlane swaps pack four sums into one register, DPP row sums
// finish) and added into an LDS slot shared by the tile's waves; the list is
// walked in windows of twice the tile's pixel count of entries, and at each
// window's end every entry stores its record's sums for this tile into the
// (record, tile) pair's own slot.  k_pair_reduce then sums each record's
// slots (no gradient atomics contend across the tiles a record covers).
//
// k_project_bwd chains those 2D gradients through the conic inverse, the EWA
// covariance J R Sigma R^T J^T (Eq. 1), the quaternion/scale parameterisation,
// the projection of the mean, the SH colour and its viewing direction, and
// into the instance cameras P = W G; k_pose_bwd maps camera gradients to the
// poses (dL/dG = W_R^T dL/dP) and k_pose6 to the 6-DoF right perturbation.
#include "internal.hpp"

namespace s3r {

// ---------------------------------------------------------------------------
// raster backward
// ---------------------------------------------------------------------------
// slot of the (record r, tile (tx, ty)) pair in emission order: a record's
// pairs are the tiles of its rectangle row by row from rec_pair[r]
__device__ __forceinline__ int64_t pair_slot(const int32_t* __restrict__ rec_pair,
                                             const int4* __restrict__ rec_rect, uint32_t r, int tx,
                                             int ty) {
  const int4 rc = rec_rect[r];
  return (int64_t)rec_pair[r] + (int64_t)(ty - rc.y) * (rc.z - rc.x) + (tx - rc.x);
}

// window of list entries whose sums a tile keeps in LDS; the deterministic
// variant keeps one copy per wave (summed in wave order at the flush), in at
// most 36 KB
template <int TS, bool DET>
struct BwdWindow {
  static constexpr int NW = RasterShape<TS>::NW;
  static constexpr int WIN_DET = 512 / NW < 64 ? 64 : 512 / NW;
  static constexpr int WIN = DET && WIN_DET < RasterShape<TS>::WIN ? WIN_DET : RasterShape<TS>::WIN;
  static constexpr int COPIES = DET ? NW : 1;
};

constexpr int kBwdRun = 4;  // consecutive launch-order tiles per XCD

template <int TS, bool DET>
// (64 VGPRs: eight waves per SIMD)
__global__ __launch_bounds__(RasterShape<TS>::NT)
__attribute__((amdgpu_waves_per_eu(8))) void k_raster_bwd(BwdArgs a) {
  constexpr int NT = RasterShape<TS>::NT, NW = RasterShape<TS>::NW;
  constexpr int WIN = BwdWindow<TS, DET>::WIN;
  constexpr int COPIES = BwdWindow<TS, DET>::COPIES;
  // per list entry of the window [w0, w0 + WIN), summed over the tile's waves
  // (atomically, or per wave when DET): moments m_x, m_y, m_xx, m_xy, m_yy,
  // then d opacity and d rgb
  __shared__ float s_g[COPIES][WIN][9];
  __shared__ int s_max[NW];
  const int tid = threadIdx.x;
  const int lane = tid % kWave, wave = tid / kWave;
  // launch-order rank of this workgroup's tile: runs of kBwdRun consecutive
  // ranks (neighbouring tiles of a length bucket, which share records) on one
  // XCD, the runs dealt round-robin to the XCDs (so the longest lists still
  // start first on every XCD); the grid is padded to whole rounds
  const int kb = (int)(blockIdx.x / kXcds);
  const int rank = (kb / kBwdRun) * (kXcds * kBwdRun) + (int)(blockIdx.x % kXcds) * kBwdRun +
                   kb % kBwdRun;
  if (rank >= a.total_tiles) return;  // padding (uniform over the workgroup)
  const int t = a.tile_order[rank];
  const int v = find_view(a.tile_offset, a.nv, t);
  const int lt = t - a.tile_offset[v];
  const int W = a.wh[2 * v], H = a.wh[2 * v + 1];
  const int gx = (W + TS - 1) / TS;
  int ox, oy, sx, sy;
  raster_pixel<TS>(tid, ox, oy, sx, sy);
  const int tcx = lt % gx, tcy = lt / gx;
  const int tx0 = tcx * TS, ty0 = tcy * TS;
  const int px = tx0 + ox, py = ty0 + oy;
  const float fxp = (float)px, fyp = (float)py;
  const float sub_x = (float)(tx0 + sx), sub_y = (float)(ty0 + sy);
  const int64_t s = a.tile_start[t];
  const int64_t e = min((int64_t)a.tile_start[t + 1], a.kp.cap_dup);
  const int64_t npx = (int64_t)W * H;
  const int64_t base = 3 * a.px_offset[v];

  float T = 1.f, dCr = 0.f, dCg = 0.f, dCb = 0.f;
  int last = 0;
  if (px < W && py < H) {
    const int64_t p = (int64_t)py * W + px;
    T = a.T_final[a.px_offset[v] + p];
    last = a.last[a.px_offset[v] + p];
    dCr = a.d_color[base + p];
    dCg = a.d_color[base + npx + p];
    dCb = a.d_color[base + 2 * npx + p];
  }
  // sd = (S_i + T_N bg) . dL/dC, S_i the colour blended behind entry i: only
  // this dot product enters dL/dalpha, so it is accumulated directly, each
  // replayed entry adding (c . dL/dC) alpha T
  float sd = T * (a.kp.bg0 * dCr + a.kp.bg1 * dCg + a.kp.bg2 * dCb);
  // each wave replays its own list prefix (entries up to its last contributor)
  int mw = last;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mw = max(mw, __shfl_xor(mw, o, kWave));
  mw = __builtin_amdgcn_readfirstlane(mw);
  if (lane == 0) s_max[wave] = mw;
  for (int k = tid; k < COPIES * WIN * 9; k += NT) (&s_g[0][0][0])[k] = 0.f;
  __syncthreads();
  int nrep = 0;
  for (int w = 0; w < NW; ++w) nrep = max(nrep, s_max[w]);
  const int64_t tile_end = min(e, s + (int64_t)nrep);
  const int64_t wave_end = min(e, s + (int64_t)mw);

  // Batches are the 64-entry blocks [s + 64 m, s + 64 m + 64) of the list and
  // windows the WIN-entry blocks [s + WIN k, s + WIN k + WIN); both are walked
  // back to front.  Inside a window every wave replays its batches (those
  // below its own end) and adds each record's wave total into the shared
  // window slot, stored to the (record, tile) pair slots at the window's end.
  // Loads are pipelined: record ids two batches ahead, record fields one
  // batch ahead.
  constexpr int BPW = WIN / kWave;  // batches per window
  const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
  int mb = (int)((wave_end - s + kWave - 1) / kWave) - 1;  // next batch of this wave
  uint32_t rn = 0u;
  float4 gn = zero4, cn = zero4, kn = zero4;
  if (mb >= 0) {
    const int64_t i0 = s + (int64_t)mb * kWave + lane;
    if (i0 < wave_end) {
      rn = a.vals[i0];
      gn = a.rec_geo[rn];
      cn = a.rec_conic[rn];
      kn = a.rec_rgb[rn];
    }
    rn = mb >= 1 ? a.vals[s + (int64_t)(mb - 1) * kWave + lane] : 0u;
  }
  const int nwin = (int)((tile_end - s + WIN - 1) / WIN);
  for (int wi = nwin - 1; wi >= 0; --wi) {
    const int64_t w0 = s + (int64_t)wi * WIN;
    const int64_t w_end = min(tile_end, w0 + WIN);
    for (; mb >= wi * BPW; --mb) {
      const int64_t b0 = s + (int64_t)mb * kWave;
      const bool valid = b0 + lane < wave_end;
      const float4 g = gn, c = cn, col = kn;
      if (mb >= 1) {
        gn = a.rec_geo[rn];
        cn = a.rec_conic[rn];
        kn = a.rec_rgb[rn];
      }
      rn = mb >= 2 ? a.vals[b0 - 2 * kWave + lane] : 0u;
      const bool near =
          valid && box_hits(cutoff_box(g.x, g.y, make_float2(c.w, col.w)), sub_x, sub_y) &&
          square_may_hit(g.x, g.y, c.x, c.y, c.z, g.z, sub_x, sub_y, 7.f, a.kp);
      uint64_t m = ballot(near);
      while (m != 0ull) {
        const int j = 63 - __builtin_clzll(m);  // back to front
        m &= ~(1ull << j);
        const float u = bcast(g.x, j), vv = bcast(g.y, j), o = bcast(g.z, j);
        const float A = bcast(c.x, j), B = bcast(c.y, j), C = bcast(c.z, j);
        const int pos = (int)(b0 - s) + j;
        const Blend bl = blend_eval(u, vv, A, B, C, o, fxp, fyp, a.kp);
        const bool contrib = bl.hit && (pos < last);
        if (ballot(contrib) == 0ull) continue;
        // (the colour is broadcast only for entries some pixel of the wave takes)
        const float kr = bcast(col.x, j), kg = bcast(col.y, j), kb = bcast(col.z, j);
        const float one_m = 1.0f - bl.alpha;
        const float rinv = __builtin_amdgcn_rcpf(one_m);  // one_m >= 1 - alpha_max
        const float Tb = T * rinv;
        const float wgt = contrib ? bl.alpha * Tb : 0.f;
        // gradient arithmetic (no decision depends on it) in fused form
        const float cdot = fmaf(kb, dCb, fmaf(kg, dCg, kr * dCr));
        const float dal = fmaf(Tb, cdot, -sd * rinv);
        // alpha clamped at alpha_max carries no gradient to o and the conic
        const bool open = contrib && (bl.raw <= a.kp.alpha_max);
        const float dpow = open ? dal * bl.alpha : 0.f;
        const float g_o = open ? dal * bl.ex : 0.f;
        // d power / d(u, v, A, B, C) are linear in the conic, so the wave sums
        // the moments dpow (dx, dy, dx^2, dx dy, dy^2) and the conic is applied
        // once per record when the window is flushed
        const float dx = u - fxp;
        const float dy = vv - fyp;
        const float m_x = dpow * dx, m_y = dpow * dy;
        const float m_xx = m_x * dx, m_xy = m_x * dy, m_yy = m_y * dy;
        sd = fmaf(cdot, wgt, sd);
        T = contrib ? Tb : T;
        // window slot q of the record receives, in order, m_x, m_y, m_xx, m_xy
        // (from s1), m_yy, o, r, g (from s2) and b (from sb)
        if (DET) {
          // this wave's own copy: one writer per entry and component
          const float s1 = wave_sum4(m_x, m_y, m_xx, m_xy);
          const float s2 = wave_sum4(m_yy, g_o, wgt * dCr, wgt * dCg);
          const float sb = wave_sum_dpp(wgt * dCb);
          if ((lane & 15) == 15) {
            const int row = lane >> 4;
            const int q = ((row & 1) << 1) | (row >> 1);
            float* G = s_g[wave][(int)(b0 - w0) + j];
            G[q] = s1;
            G[4 + q] = s2;
            if (row == 3) G[8] = sb;
          }
        } else {
          // the LDS slot adds sb's four row partials: the two row
          // broadcasts of a full wave sum cost more issue slots than three
          // more lanes of the slot's atomic add
          const float s1 = wave_sum4(m_x, m_y, m_xx, m_xy);
          const float s2 = wave_sum4(m_yy, g_o, wgt * dCr, wgt * dCg);
          const float sb = row_sum(wgt * dCb);
          if ((lane & 15) == 15) {
            const int row = lane >> 4;
            const int q = ((row & 1) << 1) | (row >> 1);
            float* G = s_g[0][(int)(b0 - w0) + j];
            atomicAdd(G + q, s1);
            atomicAdd(G + 4 + q, s2);
            atomicAdd(G + 8, sb);
          }
        }
      }
    }
    __syncthreads();
    // each entry of the window writes its record's nine sums for this tile
    // into the pair's own slot (zeros where nothing blended): no two tiles
    // share a slot, so no atomics reach global memory here
    for (int k = tid; k < (int)(w_end - w0); k += NT) {
      float gv[9];
      bool any = false;
#pragma unroll
      for (int q = 0; q < 9; ++q) gv[q] = 0.f;
      for (int c = 0; c < COPIES; ++c) {  // wave order
        float* G = s_g[c][k];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          gv[q] += G[q];
          G[q] = 0.f;
        }
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) any |= (gv[q] != 0.f);
      const uint32_t r = a.vals[w0 + k];
      float4 o0 = zero4, o1 = zero4, o2 = zero4;
      if (any) {
        const float4 c = a.rec_conic[r];
        // moments -> d(u, v, A, B, C): -(A mx + B my), -(B mx + C my),
        // -mxx / 2, -mxy, -myy / 2; then d opacity and d rgb
        o0 = make_float4(-(c.x * gv[0] + c.y * gv[1]), -(c.y * gv[0] + c.z * gv[1]), -0.5f * gv[2],
                         -gv[3]);
        o1 = make_float4(-0.5f * gv[4], gv[5], gv[6], gv[7]);
        o2 = make_float4(gv[8], 0.f, 0.f, 0.f);
      }
      float4* P = a.part + 3 * pair_slot(a.rec_pair, a.rec_rect, r, tcx, tcy);
      P[0] = o0;
      P[1] = o1;
      P[2] = o2;
    }
    __syncthreads();
  }
  // the first entry not replayed: it and every later entry of the list (later
  // in (depth, record) order) keep no slot and read as zero gradients
  if (tid == 0) {
    int2 cut = make_int2(-1, 0);
    if (tile_end < e) {
      const uint32_t r = a.vals[tile_end];
      cut = make_int2((int)r, (int)__float_as_uint(a.rec_geo[r].w));
    }
    a.tile_cut[t] = cut;
  }
}

// Sum of the per-pair gradients of each record (pairs are contiguous per
// record in emission order).  A pair counts only if its tile's backward
// replayed it, i.e. if it precedes the tile's cut in the list order (depth
// bits, then record index: the order of the stable sort).  A workgroup takes
// kPairSlabs slabs of kPairThreads consecutive pairs, one pair per lane: the
// records of the workgroup's pairs are staged in LDS (record_window), each
// lane finds its own there, and loads its pair's partial (coalesced over the
// lanes) only if the pair was replayed.  Lanes of one record are adjacent: a segmented
// scan over the wave leaves each record's sum in its last lane, which stores
// it when the record lies wholly in the wave and otherwise adds it to an LDS
// slot (the slot of the wave-chunk where the record begins, or the carry-in
// slot for a record begun before the workgroup; only the last record begun in
// a chunk can run past it, so slots are not shared).  The slots are stored at
// the end, or added atomically for the (at most two) records that cross the
// workgroup's bounds; g2d must be zero beforehand for those.
constexpr int kPairThreads = 256;
constexpr int kPairRun = 8;    // pairs per thread of the deterministic sum
constexpr int kPairSlabs = 4;  // slabs per workgroup of the atomic sum
constexpr int kPairViews = 64; // views whose tile offsets and widths are staged in LDS
constexpr int kPairGrid = 2048; // workgroups of the atomic sum at most

// one step of a segmented inclusive scan: lanes add the DPP source lane's
// values when it holds the same key (keys ascend over the lanes, so the
// source's partial sum lies wholly in the lane's own segment); a lane whose
// source is outside its row, or whose row the mask leaves out, reads key -2
template <int CTRL, int ROW_MASK, int N>
__device__ __forceinline__ void seg_scan_step(int key, float (&v)[N]) {
  const int ks = __builtin_amdgcn_update_dpp(-2, key, CTRL, ROW_MASK, 0xf, false);
  const bool take = ks == key;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    const float x = __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(v[q]), CTRL, ROW_MASK, 0xf, false));
    if (take) v[q] += x;
  }
}

// inclusive sums over the runs of equal keys of a wave (keys >= -1, ascending)
template <int N>
__device__ __forceinline__ void wave_segmented_scan(int key, float (&v)[N]) {
  seg_scan_step<0x111, 0xf>(key, v);  // row_shr:1
  seg_scan_step<0x112, 0xf>(key, v);  // row_shr:2
  seg_scan_step<0x114, 0xf>(key, v);  // row_shr:4
  seg_scan_step<0x118, 0xf>(key, v);  // row_shr:8
  seg_scan_step<0x142, 0xa>(key, v);  // row_bcast:15 into rows 1 and 3
  seg_scan_step<0x143, 0xc>(key, v);  // row_bcast:31 into rows 2 and 3
}

__global__ __launch_bounds__(kPairThreads) void k_pair_reduce(BwdArgs a) {
  constexpr int S = kPairSlabs, NP = kPairThreads * S, NC = NP / kWave + 1;
  __shared__ int s_pair[NP + 2];
  __shared__ int s_red[2 * kPairThreads / kWave];
  __shared__ float s_acc[NC][9];
  __shared__ int s_rec[NC];
  __shared__ int2 s_view[kPairViews];  // (first tile, tiles per row)
  const int nrec = a.counters[S3R_CNT_SURV];
  const int64_t ndup = a.counters[S3R_CNT_DUP];
  if (nrec <= 0) return;  // uniform over the grid
  const int tid = threadIdx.x, lane = lane_id();
  const bool vlds = a.nv <= kPairViews;
  if (vlds && tid < a.nv)
    s_view[tid] = make_int2(a.tile_offset[tid], (a.wh[2 * tid] + a.kp.tile - 1) / a.kp.tile);
  // the grid is capped (the pair count is known only on the device): a
  // workgroup takes every gridDim.x-th group of slabs
  for (int64_t P0 = (int64_t)blockIdx.x * NP; P0 < ndup; P0 += (int64_t)gridDim.x * NP) {
    const int64_t Pe = min(ndup, P0 + (int64_t)NP);
    const int64_t wb0 = P0 + (int64_t)(tid - lane);  // the wave's first pair in slab 0
    float g[S][9];
    bool live[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
      live[k] = wb0 + (int64_t)k * kPairThreads + lane < Pe;
#pragma unroll
      for (int q = 0; q < 9; ++q) g[k][q] = 0.f;
    }
    for (int k = tid; k < NC * 9; k += kPairThreads) (&s_acc[0][0])[k] = 0.f;
    for (int k = tid; k < NC; k += kPairThreads) s_rec[k] = -1;
    int nw;  // (record_window ends with a barrier: the LDS above is visible after it)
    const int r0 = record_window<kPairThreads>(a.rec_pair, nrec, P0, Pe, s_pair, s_red, &nw);
    // last window record whose first pair is at or before p (s_pair[0] <= P0)
    int idx[S];
#pragma unroll
    for (int k = 0; k < S; ++k) idx[k] = 0;
    int step = 1;
    while (2 * step < nw) step *= 2;
    for (; step > 0; step >>= 1) {  // uniform over the workgroup
#pragma unroll
      for (int k = 0; k < S; ++k) {
        const int64_t p = wb0 + (int64_t)k * kPairThreads + lane;
        const int t = idx[k] + step;
        if (t < nw && s_pair[t] <= p) idx[k] = t;
      }
    }
    int4 rc[S];
    int rv[S];
    uint32_t db[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
      if (!live[k]) continue;
      const int r = r0 + idx[k];
      rc[k] = a.rec_rect[r];
      rv[k] = a.rec_view[r];
      db[k] = __float_as_uint(a.rec_geo[r].w);
    }
#pragma unroll
    for (int k = 0; k < S; ++k) {
      if (!live[k]) continue;
      const int64_t p = wb0 + (int64_t)k * kPairThreads + lane;
      const int v = rv[k];
      const int2 vw = vlds ? s_view[v]
                           : make_int2(a.tile_offset[v], (a.wh[2 * v] + a.kp.tile - 1) / a.kp.tile);
      const int j = (int)(p - s_pair[idx[k]]), w = rc[k].z - rc[k].x;
      const int tx = rc[k].x + j % w, ty = rc[k].y + j / w;
      const int2 cut = a.tile_cut[vw.x + ty * vw.y + tx];
      const uint32_t dc = (uint32_t)cut.y;
      const int r = r0 + idx[k];
      if (cut.x < 0 || db[k] < dc || (db[k] == dc && r < cut.x)) {  // replayed: load its partial
        const float4 x0 = a.part[3 * p], x1 = a.part[3 * p + 1], x2 = a.part[3 * p + 2];
        g[k][0] = x0.x; g[k][1] = x0.y; g[k][2] = x0.z; g[k][3] = x0.w;
        g[k][4] = x1.x; g[k][5] = x1.y; g[k][6] = x1.z; g[k][7] = x1.w;
        g[k][8] = x2.x;
      }
    }
#pragma unroll
    for (int k = 0; k < S; ++k) {
      const int64_t wb = wb0 + (int64_t)k * kPairThreads;
      if (wb >= Pe) break;  // uniform over the wave
      const int key = live[k] ? idx[k] : -1;
      wave_segmented_scan(key, g[k]);  // each record's sum in its last lane of the wave
      const int kn = __shfl_down(key, 1, kWave);
      if (live[k] && (lane == kWave - 1 || kn != key)) {
        const int64_t f = s_pair[key], e = s_pair[key + 1];
        if (f >= wb && e <= wb + kWave) {
          const int r = r0 + key;
          a.g2d[3 * (size_t)r] = make_float4(g[k][0], g[k][1], g[k][2], g[k][3]);
          a.g2d[3 * (size_t)r + 1] = make_float4(g[k][4], g[k][5], g[k][6], g[k][7]);
          a.g2d[3 * (size_t)r + 2] = make_float4(g[k][8], 0.f, 0.f, 0.f);
        } else {
          const int slot = f < P0 ? 0 : 1 + (int)((f - P0) / kWave);
          s_rec[slot] = key;
#pragma unroll
          for (int q = 0; q < 9; ++q) atomicAdd(&s_acc[slot][q], g[k][q]);
        }
      }
    }
    __syncthreads();
    if (tid < NC && s_rec[tid] >= 0) {
      const int key = s_rec[tid], r = r0 + key;
      const int64_t f = s_pair[key], e = s_pair[key + 1];
      if (f >= P0 && e <= Pe) {
        const float* x = s_acc[tid];
        a.g2d[3 * (size_t)r] = make_float4(x[0], x[1], x[2], x[3]);
        a.g2d[3 * (size_t)r + 1] = make_float4(x[4], x[5], x[6], x[7]);
        a.g2d[3 * (size_t)r + 2] = make_float4(x[8], 0.f, 0.f, 0.f);
      } else {
        float* D = reinterpret_cast<float*>(a.g2d + 3 * (size_t)r);
#pragma unroll
        for (int q = 0; q < 9; ++q)
          if (s_acc[tid][q] != 0.f) atomicAdd(D + q, s_acc[tid][q]);
      }
    }
    __syncthreads();  // the next group rewrites the LDS read above
  }
}

// S3R_DETERMINISTIC_GRADS: the same sums, with the pairs of every record
// added in emission order and no atomics -- inside a run by its thread,
// across the runs of a workgroup by the thread where the record begins (its
// owner), across workgroups by k_pair_reduce_carry from the partial sums
// each workgroup leaves for the record running into it (carry-in) and for the
// record it began that runs on past it (carry-out).
__global__ __launch_bounds__(kPairThreads) void k_pair_reduce_det(BwdArgs a) {
  __shared__ float s_head[kPairThreads][9];  // a run's first segment, of a record begun before it
  __shared__ int s_head_rec[kPairThreads];
  __shared__ float s_tail[kPairThreads][9];  // a run's last segment, of a record that runs on
  __shared__ int s_tail_rec[kPairThreads];
  constexpr int NP = kPairThreads * kPairRun;
  __shared__ int s_pair[NP + 2];
  __shared__ int s_red[2 * kPairThreads / kWave];
  const int nrec = a.counters[S3R_CNT_SURV];
  const int64_t ndup = min((int64_t)a.counters[S3R_CNT_DUP], a.kp.cap_dup);
  const int64_t P0 = (int64_t)blockIdx.x * NP;
  if (P0 >= ndup || nrec <= 0) return;  // uniform over the workgroup
  const int64_t Pend = min(ndup, P0 + (int64_t)NP);
  const int tid = threadIdx.x;
  s_head_rec[tid] = -1;
  s_tail_rec[tid] = -1;
  int nw;
  const int r0 = record_window<kPairThreads>(a.rec_pair, nrec, P0, Pend, s_pair, s_red, &nw);
  const int64_t p0 = P0 + (int64_t)tid * kPairRun;
  const int64_t p1 = min(ndup, p0 + kPairRun);
  if (p0 < p1) {
    int lo = 0, hi = nw - 1;  // last window record whose first pair is at or before p0
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_pair[mid] <= p0) lo = mid;
      else hi = mid - 1;
    }
    int r = r0 + lo - 1;
    int64_t first = 0, next = s_pair[lo];
    int4 rc = make_int4(0, 0, 1, 1);
    int tx = 0, ty = 0, gx = 1, tbase = 0;
    uint32_t db = 0u;
    float acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = 0.f;
    for (int64_t p = p0; p < p1; ++p) {
      if (p >= next) {
        do {
          ++r;
          first = next;
          next = s_pair[r - r0 + 1];
        } while (p >= next);
        rc = a.rec_rect[r];
        const int v = a.rec_view[r];
        db = __float_as_uint(a.rec_geo[r].w);
        gx = (a.wh[2 * v] + a.kp.tile - 1) / a.kp.tile;
        tbase = a.tile_offset[v];
        const int j = (int)(p - first), w = rc.z - rc.x;
        tx = rc.x + j % w;
        ty = rc.y + j / w;
      }
      const int2 cut = a.tile_cut[tbase + ty * gx + tx];
      const uint32_t dc = (uint32_t)cut.y;
      if (cut.x < 0 || db < dc || (db == dc && r < cut.x)) {
        const float4 x0 = a.part[3 * p], x1 = a.part[3 * p + 1], x2 = a.part[3 * p + 2];
        acc[0] += x0.x; acc[1] += x0.y; acc[2] += x0.z; acc[3] += x0.w;
        acc[4] += x1.x; acc[5] += x1.y; acc[6] += x1.z; acc[7] += x1.w;
        acc[8] += x2.x;
      }
      if (++tx == rc.z) {
        tx = rc.x;
        ++ty;
      }
      if (p + 1 < p1 && p + 1 < next) continue;
      // the segment of record r in this run ends at p
      const bool before = first < p0, on = min(next, ndup) > p1;
      if (!before && !on) {
        a.g2d[3 * (size_t)r] = make_float4(acc[0], acc[1], acc[2], acc[3]);
        a.g2d[3 * (size_t)r + 1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
        a.g2d[3 * (size_t)r + 2] = make_float4(acc[8], 0.f, 0.f, 0.f);
      } else if (before) {
        s_head_rec[tid] = r;
#pragma unroll
        for (int q = 0; q < 9; ++q) s_head[tid][q] = acc[q];
      } else {
        s_tail_rec[tid] = r;
#pragma unroll
        for (int q = 0; q < 9; ++q) s_tail[tid][q] = acc[q];
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) acc[q] = 0.f;
    }
  }
  __syncthreads();
  const int64_t wg = blockIdx.x;
  if (tid == 0) a.carry_rec[2 * wg + 1] = -1;
  // owners: a record begun in this run, summed over the runs that follow
  const int r = s_tail_rec[tid];
  if (r >= 0) {
    float sum[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) sum[q] = s_tail[tid][q];
    for (int u = tid + 1; u < kPairThreads && s_head_rec[u] == r; ++u)
#pragma unroll
      for (int q = 0; q < 9; ++q) sum[q] += s_head[u][q];
    const int64_t end = min((int64_t)s_pair[r - r0 + 1], ndup);
    if (end <= Pend) {
      a.g2d[3 * (size_t)r] = make_float4(sum[0], sum[1], sum[2], sum[3]);
      a.g2d[3 * (size_t)r + 1] = make_float4(sum[4], sum[5], sum[6], sum[7]);
      a.g2d[3 * (size_t)r + 2] = make_float4(sum[8], 0.f, 0.f, 0.f);
    } else {
      a.carry_rec[2 * wg + 1] = r;
#pragma unroll
      for (int q = 0; q < 9; ++q) a.carry_g[(2 * wg + 1) * 9 + q] = sum[q];
    }
  }
  // carry-in: the record running into this workgroup, summed over its runs here
  if (tid == 0) {
    const int rin = s_head_rec[0];
    a.carry_rec[2 * wg] = rin;
    if (rin >= 0) {
      float sum[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) sum[q] = 0.f;
      for (int u = 0; u < kPairThreads && s_head_rec[u] == rin; ++u)
#pragma unroll
        for (int q = 0; q < 9; ++q) sum[q] += s_head[u][q];
#pragma unroll
      for (int q = 0; q < 9; ++q) a.carry_g[2 * wg * 9 + q] = sum[q];
    }
  }
}

// one thread per workgroup of k_pair_reduce_det: the record it began and
// handed on is completed with the carry-ins of the workgroups that follow,
// in order
__global__ __launch_bounds__(256) void k_pair_reduce_carry(BwdArgs a, int64_t nb) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ndup = min((int64_t)a.counters[S3R_CNT_DUP], a.kp.cap_dup);
  const int64_t per = (int64_t)kPairThreads * kPairRun;
  const int64_t active = min(nb, (ndup + per - 1) / per);
  if (w >= active || a.counters[S3R_CNT_SURV] <= 0) return;
  const int r = a.carry_rec[2 * w + 1];
  if (r < 0) return;
  float sum[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) sum[q] = a.carry_g[(2 * w + 1) * 9 + q];
  for (int64_t u = w + 1; u < active && a.carry_rec[2 * u] == r; ++u)
#pragma unroll
    for (int q = 0; q < 9; ++q) sum[q] += a.carry_g[2 * u * 9 + q];
  a.g2d[3 * (size_t)r] = make_float4(sum[0], sum[1], sum[2], sum[3]);
  a.g2d[3 * (size_t)r + 1] = make_float4(sum[4], sum[5], sum[6], sum[7]);
  a.g2d[3 * (size_t)r + 2] = make_float4(sum[8], 0.f, 0.f, 0.f);
}

// ---------------------------------------------------------------------------
// projection / colour backward
// ---------------------------------------------------------------------------
// dL/dq (raw quaternion) from dL/dR of R(q / |q|)
__device__ __forceinline__ void quat_rot_bwd(float4 q, const float dR[9], float dq[4]) {
  const float n = sqrtf(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
  const float w = q.x / n, x = q.y / n, y = q.z / n, z = q.w / n;
  const float dw = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  const float dx = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] +
                          z * dR[6] + w * dR[7] - 2.f * x * dR[8]);
  const float dy = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] -
                          w * dR[6] + z * dR[7] - 2.f * y * dR[8]);
  const float dz = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] +
                          y * dR[5] + x * dR[6] + y * dR[7]);
  const float dot = w * dw + x * dx + y * dy + z * dz;
  dq[0] = (dw - w * dot) / n;
  dq[1] = (dx - x * dot) / n;
  dq[2] = (dy - y * dot) / n;
  dq[3] = (dz - z * dot) / n;
}

// 2^32: the unit of the fixed-point camera-gradient sums of the deterministic
// mode (integer additions commute, so their order cannot change the result)
constexpr double kFixedScale = 4294967296.0;

// Sum 12 values over the lanes of a wave that share a key (key < 0: none)
// and add them to dst + key * 12 -- or, with fx, to the fixed-point sums
// fx + key * 12 (deterministic whatever order the waves add in).
__device__ __forceinline__ void wave_segmented_add(int key, const float val[12], float* dst,
                                                   unsigned long long* fx = nullptr) {
  const int lane = lane_id();
  uint64_t todo = ballot(key >= 0);
  while (todo) {
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const int lk = __builtin_amdgcn_readlane(key, leader);
    const bool mine = (key == lk);
    const uint64_t grp = ballot(mine);
    // twelve independent DPP reductions (no LDS round trips), totals in
    // lane 63, then the twelve atomics
    float s[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) s[q] = wave_sum_dpp(mine ? val[q] : 0.f);
    if (lane == kWave - 1) {
#pragma unroll
      for (int q = 0; q < 12; ++q) {
        if (fx)
          atomicAdd(fx + (size_t)lk * 12 + q,
                    (unsigned long long)(long long)__double2ll_rn((double)s[q] * kFixedScale));
        else
          atomicAdd(dst + (size_t)lk * 12 + q, s[q]);
      }
    }
    todo &= ~grp;
  }
}

// bit of Gaussian i in a [ceil(N/64)*2] word mask (word i / 32, bit i % 32)
__device__ __forceinline__ bool mask_bit(const uint32_t* m, int i) {
  return (m[i >> 5] >> (i & 31)) & 1u;
}

// Gradient of the projection, colour and instance cameras, gathered per
// Gaussian.  One thread per record; the record that is its Gaussian's first
// in the batch (the owner) does the work: it walks the later views, finds
// the Gaussian's record in each view where it survived (records are ordered
// by (block of 256 Gaussians, view, Gaussian), so the slot is the block's
// first record of that view plus the Gaussian's rank among the block's
// survivors), chains each record's 2D gradient back through Eq. (1) and the
// SH colour, sums over views (SH coefficients in the Gaussian's own rows),
// and writes the Gaussian's gradients once: no per-Gaussian atomics.  With
// one view per batch every record is an owner.  The entry point zeroes the
// dense gradient arrays first, so Gaussians without records cost nothing
// here.  Camera gradients are summed per wave over lanes of the same (view,
// instance) before their atomics.
__device__ __forceinline__ void project_bwd_owner(const ProjBwdArgs& a, int r0, int nrec) {
  const bool plain = (a.kp.flags & S3R_PLAIN) != 0;
  const int B = (a.sh_deg + 1) * (a.sh_deg + 1);
  int i = 0, v0 = 0;
  bool active = r0 < nrec;
  if (active) {
    i = a.rec_gid[r0];
    v0 = a.rec_view[r0];
    // the owner is the Gaussian's record in the first view where it survived
    for (int v = 0; v < v0; ++v)
      if (mask_bit(a.surv + (size_t)v * a.mask_words, i)) {
        active = false;
        break;
      }
  }
  const int k = active ? clampi(a.inst[i], 0, a.n_slots - 1) : 0;
  const int vb = i / kProjBlock, wave = (i % kProjBlock) / kWave, bit = i % kWave;
  // sparse gradient mode: the owners' Gaussians are the rows this call writes
  if (a.rows && r0 < nrec) a.rows[r0] = active ? i : -1;

  // the Gaussian's parameters (local frame)
  float mx = 0.f, my = 0.f, mz = 0.f, sc[3] = {1.f, 1.f, 1.f}, Rl[9];
  float4 q = make_float4(1.f, 0.f, 0.f, 0.f);
  if (active) {
    mx = a.mean[3 * i]; my = a.mean[3 * i + 1]; mz = a.mean[3 * i + 2];
    sc[0] = a.scale[3 * i]; sc[1] = a.scale[3 * i + 1]; sc[2] = a.scale[3 * i + 2];
    q = reinterpret_cast<const float4*>(a.quat)[i];
  }
  // d_sh is summed in place (this thread owns the Gaussian's entries): the
  // first record writes, later ones add; Gaussians without records keep the
  // zeros the caller side of the launch wrote
  float* dsh = a.d_sh + (size_t)i * B * 3;
  const bool vec_sh = ((3 * B) & 3) == 0;
  bool first = true;
  quat_rot(q.x, q.y, q.z, q.w, Rl);
  // plain route: world-frame gradients (zeroed by the entry point) are
  // summed in place per timestep slot; this thread owns the Gaussian's rows
  // accumulated over the views
  float acc_mu[3] = {0.f, 0.f, 0.f}, acc_sc[3] = {0.f, 0.f, 0.f}, acc_R[9], acc_o = 0.f;
#pragma unroll
  for (int t = 0; t < 9; ++t) acc_R[t] = 0.f;

  for (int v = 0; v < a.nv; ++v) {
    // this Gaussian's record in view v, if it has one
    int64_t r = r0;
    bool has = active && v == v0;
    if (active && v > v0 && mask_bit(a.surv + (size_t)v * a.mask_words, i)) {
      const int first = a.bstat[((size_t)vb * a.nv + v) * kBstat + 3];
      int before = 0;
      for (int w = 0; w <= wave; ++w) {
        const uint32_t* sb = a.surv + (size_t)v * a.mask_words + 2 * ((size_t)vb * kProjWaves + w);
        uint64_t word = ((uint64_t)sb[1] << 32) | sb[0];
        if (w == wave) word &= (1ull << bit) - 1ull;
        before += __popcll(word);
      }
      r = (int64_t)first + before;
      has = r < a.kp.cap_surv;
    }
    int cam_key = -1;
    float dcam[12];
#pragma unroll
    for (int t = 0; t < 12; ++t) dcam[t] = 0.f;
    if (has) {
      const int tau = clampi(a.tstep[v], 0, a.n_ts - 1);
      const float4 G0 = a.g2d[3 * (size_t)r], G1 = a.g2d[3 * (size_t)r + 1],
                   G2 = a.g2d[3 * (size_t)r + 2];
      const float du = G0.x, dv = G0.y, dA = G0.z, dB = G0.w, dC = G1.x, dO = G1.y;
      const float drgb[3] = {G1.z, G1.w, G2.x};
      const float4 kv = reinterpret_cast<const float4*>(a.Kv)[v];
      const float fx = kv.x, fy = kv.y;
      const int Wd = a.wh[2 * v], Hd = a.wh[2 * v + 1];

      // ---- forward recompute ----
      float px_m = mx, py_m = my, pz_m = mz, Rg[9];
      int slot = 0;
      if (plain) {
        slot = a.plain_slot[v];
        const float* mw = a.mean_w + ((size_t)slot * a.n + i) * 3;
        px_m = mw[0]; py_m = mw[1]; pz_m = mw[2];
        const float* rw = a.rot_w + ((size_t)slot * a.n + i) * 9;
#pragma unroll
        for (int t = 0; t < 9; ++t) Rg[t] = rw[t];
      } else {
#pragma unroll
        for (int t = 0; t < 9; ++t) Rg[t] = Rl[t];
      }
      float P[12];
      {
        const float4* c4 =
            reinterpret_cast<const float4*>(a.cam + ((size_t)v * a.n_slots + (plain ? 0 : k)) * 12);
        const float4 c0 = c4[0], c1 = c4[1], c2 = c4[2];
        P[0] = c0.x; P[1] = c0.y; P[2] = c0.z; P[3] = c0.w;
        P[4] = c1.x; P[5] = c1.y; P[6] = c1.z; P[7] = c1.w;
        P[8] = c2.x; P[9] = c2.y; P[10] = c2.z; P[11] = c2.w;
      }
      const float px = ((P[0] * px_m + P[1] * py_m) + P[2] * pz_m) + P[3];
      const float py = ((P[4] * px_m + P[5] * py_m) + P[6] * pz_m) + P[7];
      const float pz = ((P[8] * px_m + P[9] * py_m) + P[10] * pz_m) + P[11];
      float M[9];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) M[ii * 3 + jj] = Rg[ii * 3 + jj] * sc[jj];
      float S[9];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
          S[ii * 3 + jj] = M[ii * 3] * M[jj * 3] + M[ii * 3 + 1] * M[jj * 3 + 1] +
                           M[ii * 3 + 2] * M[jj * 3 + 2];
      const float tx = px / pz, ty = py / pz;
      const float lx = a.kp.jac_clamp * ((0.5f * (float)Wd) / fx);
      const float ly = a.kp.jac_clamp * ((0.5f * (float)Hd) / fy);
      const bool clx = (tx < -lx) || (tx > lx);
      const bool cly = (ty < -ly) || (ty > ly);
      const float txc = fminf(fmaxf(tx, -lx), lx);
      const float tyc = fminf(fmaxf(ty, -ly), ly);
      const float iz = 1.f / pz;
      const float J00 = fx * iz, J02 = -fx * txc * iz, J11 = fy * iz, J12 = -fy * tyc * iz;
      float A[6];
#pragma unroll
      for (int jj = 0; jj < 3; ++jj) {
        A[jj] = J00 * P[jj] + J02 * P[8 + jj];
        A[3 + jj] = J11 * P[4 + jj] + J12 * P[8 + jj];
      }
      float AS[6];  // A Sigma
#pragma unroll
      for (int ii = 0; ii < 2; ++ii)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
          AS[ii * 3 + jj] = A[ii * 3] * S[jj] + A[ii * 3 + 1] * S[3 + jj] + A[ii * 3 + 2] * S[6 + jj];
      const float ca = AS[0] * A[0] + AS[1] * A[1] + AS[2] * A[2] + a.kp.eps2d;
      const float cb = AS[0] * A[3] + AS[1] * A[4] + AS[2] * A[5];
      const float cc = AS[3] * A[3] + AS[4] * A[4] + AS[5] * A[5] + a.kp.eps2d;
      const float det = ca * cc - cb * cb;
      const float id2 = 1.f / (det * det);

      // ---- conic -> 2D covariance ----
      const float d_a = (-cc * cc * dA + cb * cc * dB - cb * cb * dC) * id2;
      const float d_b = (2.f * cb * cc * dA - (det + 2.f * cb * cb) * dB + 2.f * ca * cb * dC) * id2;
      const float d_c = (-cb * cb * dA + ca * cb * dB - ca * ca * dC) * id2;
      // symmetric G' = [[d_a, d_b/2], [d_b/2, d_c]]
      const float g00 = d_a, g01 = 0.5f * d_b, g11 = d_c;
      // dSigma = A^T G' A (3x3)
      float GA[6];  // G' A
#pragma unroll
      for (int jj = 0; jj < 3; ++jj) {
        GA[jj] = g00 * A[jj] + g01 * A[3 + jj];
        GA[3 + jj] = g01 * A[jj] + g11 * A[3 + jj];
      }
      float dS[9];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) dS[ii * 3 + jj] = A[ii] * GA[jj] + A[3 + ii] * GA[3 + jj];
      // dA = 2 G' A Sigma
      float dAm[6];
#pragma unroll
      for (int ii = 0; ii < 2; ++ii)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
          dAm[ii * 3 + jj] = 2.f * (GA[ii * 3] * S[jj] + GA[ii * 3 + 1] * S[3 + jj] +
                                    GA[ii * 3 + 2] * S[6 + jj]);
      // A = J R_c
      float dRc[9];
#pragma unroll
      for (int jj = 0; jj < 3; ++jj) {
        dRc[jj] = J00 * dAm[jj];
        dRc[3 + jj] = J11 * dAm[3 + jj];
        dRc[6 + jj] = J02 * dAm[jj] + J12 * dAm[3 + jj];
      }
      const float dJ00 = dAm[0] * P[0] + dAm[1] * P[1] + dAm[2] * P[2];
      const float dJ02 = dAm[0] * P[8] + dAm[1] * P[9] + dAm[2] * P[10];
      const float dJ11 = dAm[3] * P[4] + dAm[4] * P[5] + dAm[5] * P[6];
      const float dJ12 = dAm[3] * P[8] + dAm[4] * P[9] + dAm[5] * P[10];
      float dpx = du * fx * iz;
      float dpy = dv * fy * iz;
      float dpz = -(du * fx * px + dv * fy * py) * iz * iz;
      dpz += -(dJ00 * fx + dJ11 * fy) * iz * iz;
      // J02 = -fx txc / pz, txc = clamp(px / pz)
      dpz += dJ02 * fx * txc * iz * iz;
      dpz += dJ12 * fy * tyc * iz * iz;
      if (!clx) {
        dpx += dJ02 * (-fx * iz * iz);
        dpz += dJ02 * (fx * iz) * (px * iz * iz);
      }
      if (!cly) {
        dpy += dJ12 * (-fy * iz * iz);
        dpz += dJ12 * (fy * iz) * (py * iz * iz);
      }
      // Sigma = M M^T, M = R diag(s)
      float dM[9];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
          dM[ii * 3 + jj] = 2.f * (dS[ii * 3] * M[jj] + dS[ii * 3 + 1] * M[3 + jj] +
                                   dS[ii * 3 + 2] * M[6 + jj]);
      float dRg[9];
#pragma unroll
      for (int jj = 0; jj < 3; ++jj) {
        acc_sc[jj] += Rg[jj] * dM[jj] + Rg[3 + jj] * dM[3 + jj] + Rg[6 + jj] * dM[6 + jj];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) dRg[ii * 3 + jj] = dM[ii * 3 + jj] * sc[jj];
      }
      // p = R_c mu + tau
      float dmu[3], dtau[3] = {dpx, dpy, dpz};
#pragma unroll
      for (int jj = 0; jj < 3; ++jj) dmu[jj] = P[jj] * dpx + P[4 + jj] * dpy + P[8 + jj] * dpz;
      const float mm[3] = {px_m, py_m, pz_m};
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) dRc[ii * 3 + jj] += dtau[ii] * mm[jj];

      // ---- colour ----
      float dl[3], w3[3] = {0.f, 0.f, 0.f};
      const float* Gp = nullptr;
      if (plain) {
        const float4 cw = reinterpret_cast<const float4*>(a.cen)[(size_t)v * a.n_slots];
        w3[0] = px_m - cw.x; w3[1] = py_m - cw.y; w3[2] = pz_m - cw.z;
        Gp = a.pose + ((size_t)tau * a.n_slots + k) * 12;
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) dl[jj] = Gp[jj] * w3[0] + Gp[4 + jj] * w3[1] + Gp[8 + jj] * w3[2];
      } else {
        const float4 ce = reinterpret_cast<const float4*>(a.cen)[(size_t)v * a.n_slots + k];
        dl[0] = mx - ce.x; dl[1] = my - ce.y; dl[2] = mz - ce.z;
      }
      const float nrm = sqrtf(dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2]);
      const float dir[3] = {dl[0] / nrm, dl[1] / nrm, dl[2] / nrm};
      float Y[16];
      sh_basis(a.sh_deg, dir[0], dir[1], dir[2], Y);
      float f[48];
      load_sh(a.sh + (size_t)i * B * 3, B, f);
      float raw[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        if (b < B) {
          raw[0] += Y[b] * f[3 * b];
          raw[1] += Y[b] * f[3 * b + 1];
          raw[2] += Y[b] * f[3 * b + 2];
        }
      }
      float dr[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) dr[c] = raw[c] >= 0.f ? drgb[c] : 0.f;
      float gb[16];
#pragma unroll
      for (int b = 0; b < 16; ++b)
        gb[b] = (b < B) ? f[3 * b] * dr[0] + f[3 * b + 1] * dr[1] + f[3 * b + 2] * dr[2] : 0.f;
      // dL/df_{b,c} = Y_b dr_c, element 3 b + c
      if (vec_sh) {
        float4* d4 = reinterpret_cast<float4*>(dsh);
#pragma unroll
        for (int t = 0; t < 12; ++t) {
          if (4 * t < 3 * B) {
            float4 x = first ? make_float4(0.f, 0.f, 0.f, 0.f) : d4[t];
            x.x += Y[(4 * t) / 3] * dr[(4 * t) % 3];
            x.y += Y[(4 * t + 1) / 3] * dr[(4 * t + 1) % 3];
            x.z += Y[(4 * t + 2) / 3] * dr[(4 * t + 2) % 3];
            x.w += Y[(4 * t + 3) / 3] * dr[(4 * t + 3) % 3];
            d4[t] = x;
          }
        }
      } else {
#pragma unroll
        for (int t = 0; t < 48; ++t)
          if (t < 3 * B) dsh[t] = (first ? 0.f : dsh[t]) + Y[t / 3] * dr[t % 3];
      }
      first = false;
      float ddir[3];
      sh_basis_grad(a.sh_deg, dir[0], dir[1], dir[2], gb, ddir[0], ddir[1], ddir[2]);
      const float dd = dir[0] * ddir[0] + dir[1] * ddir[1] + dir[2] * ddir[2];
      float ddl[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) ddl[c] = (ddir[c] - dir[c] * dd) / nrm;

      acc_o += dO;
      if (plain) {
        // dl = R_G^T w, w = mu_w - c_w; this thread owns (slot, i)
        float dw[3];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii)
          dw[ii] = Gp[ii * 4] * ddl[0] + Gp[ii * 4 + 1] * ddl[1] + Gp[ii * 4 + 2] * ddl[2];
        float* dmw = a.d_mean_w + ((size_t)slot * a.n + i) * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) dmw[c] += dmu[c] + dw[c];
        float* drw = a.d_rot_w + ((size_t)slot * a.n + i) * 9;
#pragma unroll
        for (int t = 0; t < 9; ++t) drw[t] += dRg[t];
        if (k > 0) {
          // dR_G[j][i] += w_j ddl_i (rotation part of the pose)
#pragma unroll
          for (int jj = 0; jj < 3; ++jj)
#pragma unroll
            for (int ii = 0; ii < 3; ++ii) dcam[jj * 4 + ii] = w3[jj] * ddl[ii];
          cam_key = tau * a.n_slots + k;
        }
      } else {
        // d = mu - cen, cen = -R_c^T tau
#pragma unroll
        for (int c = 0; c < 3; ++c) acc_mu[c] += dmu[c] + ddl[c];
#pragma unroll
        for (int t = 0; t < 9; ++t) acc_R[t] += dRg[t];
        const float dcen[3] = {-ddl[0], -ddl[1], -ddl[2]};
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) {
#pragma unroll
          for (int jj = 0; jj < 3; ++jj) dRc[ii * 3 + jj] += -P[ii * 4 + 3] * dcen[jj];
          dtau[ii] += -(P[ii * 4] * dcen[0] + P[ii * 4 + 1] * dcen[1] + P[ii * 4 + 2] * dcen[2]);
        }
        if (k > 0) {
#pragma unroll
          for (int ii = 0; ii < 3; ++ii) {
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) dcam[ii * 4 + jj] = dRc[ii * 3 + jj];
            dcam[ii * 4 + 3] = dtau[ii];
          }
          cam_key = v * a.n_slots + k;
        }
      }
    }
    wave_segmented_add(cam_key, dcam, plain ? a.d_pose : a.d_cam, plain ? nullptr : a.d_cam_fx);
  }

  if (first) return;  // not an owner: nothing to write
  a.d_opac[i] = acc_o;
#pragma unroll
  for (int c = 0; c < 3; ++c) a.d_scale[3 * i + c] = acc_sc[c];
  if (!plain) {
#pragma unroll
    for (int c = 0; c < 3; ++c) a.d_mean[3 * i + c] = acc_mu[c];
    float dq[4];
    quat_rot_bwd(q, acc_R, dq);
    reinterpret_cast<float4*>(a.d_quat)[i] = make_float4(dq[0], dq[1], dq[2], dq[3]);
  }
}

// (at most 256 VGPRs, no spills: two waves per SIMD instead of one)
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(2))) void k_project_bwd(ProjBwdArgs a) {
  const int nrec = (int)min((int64_t)a.counters[S3R_CNT_SURV], a.kp.cap_surv);
  const int stride = gridDim.x * blockDim.x;
  for (int base = blockIdx.x * blockDim.x; base < nrec; base += stride)
    project_bwd_owner(a, base + (int)threadIdx.x, nrec);
  if (a.n_rows && blockIdx.x == 0 && threadIdx.x == 0) *a.n_rows = nrec;
}

// 6-DoF form of one pose gradient D (3x4) at pose G: M = G~^T D,
// rho = M[0:3,3], omega = (M21 - M12, M02 - M20, M10 - M01)
__device__ __forceinline__ void pose6_of(const float* __restrict__ G, const float (&D)[12],
                                         float* __restrict__ o) {
  float M[12];  // rows 0..2 of G~^T D: M[i][c] = sum_r G[r][i] D[r][c]
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      M[i * 4 + c] = G[0 * 4 + i] * D[0 * 4 + c] + G[1 * 4 + i] * D[1 * 4 + c] +
                     G[2 * 4 + i] * D[2 * 4 + c];
  o[0] = M[3]; o[1] = M[7]; o[2] = M[11];
  o[3] = M[2 * 4 + 1] - M[1 * 4 + 2];
  o[4] = M[0 * 4 + 2] - M[2 * 4 + 0];
  o[5] = M[1 * 4 + 0] - M[0 * 4 + 1];
}

// One thread per (timestep, slot): dL/dG_{tau,k} = sum over the batch's views
// v at timestep tau, in view order, of W_R^T dL/dP_{v,k}, written whole (no
// atomics), and with d_pose6 its 6-DoF form.  Slot 0 (static Gaussians) has
// no pose: its rows are left at the zeros the call wrote.  The camera
// gradients are float sums, or with kFixed the fixed-point sums of the
// deterministic mode.
template <bool kFixed>
__global__ void k_pose_bwd(const float* __restrict__ W, const int32_t* __restrict__ tstep,
                           const void* __restrict__ d_cam_any, int nv, int S, int T,
                           const float* __restrict__ pose, float* __restrict__ d_pose,
                           float* __restrict__ d_pose6) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= T * S) return;
  const int tau = idx / S, k = idx % S;
  if (k == 0) {
    if (d_pose6 != nullptr)
#pragma unroll
      for (int c = 0; c < 6; ++c) d_pose6[(size_t)idx * 6 + c] = 0.f;
    return;
  }
  float g[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) g[q] = 0.f;
  for (int v = 0; v < nv; ++v) {
    if (clampi(tstep[v], 0, T - 1) != tau) continue;
    const float* w = W + v * 12;
    const size_t c0 = ((size_t)v * S + k) * 12;
    float dP[12];
#pragma unroll
    for (int q = 0; q < 12; ++q)
      dP[q] = kFixed
                  ? (float)((double)(long long)static_cast<const unsigned long long*>(d_cam_any)[c0 + q] /
                            kFixedScale)
                  : static_cast<const float*>(d_cam_any)[c0 + q];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        g[r * 4 + c] += w[0 * 4 + r] * dP[0 * 4 + c] + w[1 * 4 + r] * dP[1 * 4 + c] +
                        w[2 * 4 + r] * dP[2 * 4 + c];
  }
  float* dG = d_pose + (size_t)idx * 12;
#pragma unroll
  for (int q = 0; q < 12; ++q) dG[q] = g[q];
  if (d_pose6 != nullptr) pose6_of(pose + (size_t)idx * 12, g, d_pose6 + (size_t)idx * 6);
}

// 6-DoF form of pose gradients summed elsewhere (plain route)
__global__ void k_pose6(const float* __restrict__ pose, const float* __restrict__ d_pose, int TS_,
                        int S, float* __restrict__ d_pose6) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= TS_) return;
  float* o = d_pose6 + (size_t)idx * 6;
  if (idx % S == 0) {  // slot 0 (static Gaussians) has no pose
#pragma unroll
    for (int c = 0; c < 6; ++c) o[c] = 0.f;
    return;
  }
  float D[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) D[q] = d_pose[(size_t)idx * 12 + q];
  pose6_of(pose + (size_t)idx * 12, D, o);
}

// plain route: world-frame gradients -> local mean / quaternion and poses
struct TsList2 {
  int32_t tau[kMaxViews];
};

__global__ __launch_bounds__(256) void k_plain_transform_bwd(
    const float* __restrict__ mean, const float* __restrict__ quat,
    const int32_t* __restrict__ inst, const float* __restrict__ pose, int n, int S, TsList2 ts,
    int n_ts, const float* __restrict__ d_mean_w, const float* __restrict__ d_rot_w,
    float* __restrict__ d_mean, float* __restrict__ d_quat, float* __restrict__ d_pose) {
  const int stride = gridDim.x * blockDim.x;
  for (int base = blockIdx.x * blockDim.x; base < n; base += stride) {
    const int i = base + threadIdx.x;
    const bool active = i < n;
    const int k = active ? clampi(inst[i], 0, S - 1) : 0;
    float mu[3] = {0.f, 0.f, 0.f};
    float4 q = make_float4(1.f, 0.f, 0.f, 0.f);
    float Rq[9];
    if (active) {
      mu[0] = mean[3 * i]; mu[1] = mean[3 * i + 1]; mu[2] = mean[3 * i + 2];
      q = reinterpret_cast<const float4*>(quat)[i];
    }
    quat_rot(q.x, q.y, q.z, q.w, Rq);
    float dmu[3] = {0.f, 0.f, 0.f}, dRq[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) dRq[t] = 0.f;
    for (int sl = 0; sl < n_ts; ++sl) {
      float dG[12];
#pragma unroll
      for (int t = 0; t < 12; ++t) dG[t] = 0.f;
      int key = -1;
      if (active) {
        const float* G = pose + ((size_t)ts.tau[sl] * S + k) * 12;
        const float* dmw = d_mean_w + ((size_t)sl * n + i) * 3;
        const float* drw = d_rot_w + ((size_t)sl * n + i) * 9;
        float gm[3] = {dmw[0], dmw[1], dmw[2]}, gr[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) gr[t] = drw[t];
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
          dmu[jj] += G[jj] * gm[0] + G[4 + jj] * gm[1] + G[8 + jj] * gm[2];
#pragma unroll
          for (int cc = 0; cc < 3; ++cc)
            dRq[jj * 3 + cc] += G[jj] * gr[cc] + G[4 + jj] * gr[3 + cc] + G[8 + jj] * gr[6 + cc];
        }
        if (k > 0) {
#pragma unroll
          for (int r = 0; r < 3; ++r) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
              dG[r * 4 + c] = gm[r] * mu[c] + gr[r * 3] * Rq[c * 3] + gr[r * 3 + 1] * Rq[c * 3 + 1] +
                              gr[r * 3 + 2] * Rq[c * 3 + 2];
            dG[r * 4 + 3] = gm[r];
          }
          key = ts.tau[sl] * S + k;
        }
      }
      wave_segmented_add(key, dG, d_pose);
    }
    if (active) {
      float dq[4];
      quat_rot_bwd(q, dRq, dq);
#pragma unroll
      for (int c = 0; c < 3; ++c) d_mean[3 * i + c] = dmu[c];
#pragma unroll
      for (int c = 0; c < 4; ++c) d_quat[4 * i + c] = dq[c];
    }
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
// zero the per-record gradient slots of the records that exist, and the two
// small accumulators of the call (camera and pose gradients)
__global__ __launch_bounds__(256) void k_zero_g2d(float4* __restrict__ g2d,
                                                  const int32_t* __restrict__ counters,
                                                  float* __restrict__ za, int64_t na,
                                                  float* __restrict__ zb, int64_t nb) {
  const int64_t n = 3 * (int64_t)counters[S3R_CNT_SURV];
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i < n; i += stride) g2d[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  if (za)
    for (int64_t i = i0; i < na; i += stride) za[i] = 0.f;
  if (zb)
    for (int64_t i = i0; i < nb; i += stride) zb[i] = 0.f;
}

hipError_t launch_zero_g2d(const BwdArgs& a, hipStream_t st) {
  S3R_LAUNCH(K_ZERO_G2D, k_zero_g2d, dim3(1024), dim3(256), 0, st, a.g2d, a.counters, a.zero_a,
             a.n_zero_a, a.zero_b, a.n_zero_b);
  return hipGetLastError();
}

// (the gradient slots and accumulators are cleared before this launch, by
// launch_zero_g2d or launch_clear_rows)
hipError_t launch_raster_bwd(const BwdArgs& a, hipStream_t st) {
  if (a.total_tiles <= 0) return hipGetLastError();
  const bool det = (a.kp.flags & S3R_DETERMINISTIC_GRADS) != 0;
  const unsigned round = kXcds * kBwdRun;
  const dim3 grid(((unsigned)a.total_tiles + round - 1) / round * round);
  switch (a.kp.tile) {
    case 8:
      if (det) S3R_LAUNCH(K_RASTER_BWD, (k_raster_bwd<8, true>), grid, dim3(64), 0, st, a);
      else S3R_LAUNCH(K_RASTER_BWD, (k_raster_bwd<8, false>), grid, dim3(64), 0, st, a);
      break;
    case 16:
      if (det) S3R_LAUNCH(K_RASTER_BWD, (k_raster_bwd<16, true>), grid, dim3(256), 0, st, a);
      else S3R_LAUNCH(K_RASTER_BWD, (k_raster_bwd<16, false>), grid, dim3(256), 0, st, a);
      break;
    case 32:
      if (det) S3R_LAUNCH(K_RASTER_BWD, (k_raster_bwd<32, true>), grid, dim3(1024), 0, st, a);
      else S3R_LAUNCH(K_RASTER_BWD, (k_raster_bwd<32, false>), grid, dim3(1024), 0, st, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  {
    const int64_t per = (int64_t)kPairThreads * (det ? kPairRun : kPairSlabs);
    const int64_t nb = (a.kp.cap_dup + per - 1) / per;
    const dim3 g((unsigned)(nb > 0 ? (det ? nb : min(nb, (int64_t)kPairGrid)) : 1));
    if (det) {
      S3R_LAUNCH(K_PAIR_REDUCE, k_pair_reduce_det, g, dim3(kPairThreads), 0, st, a);
      S3R_LAUNCH(K_PAIR_REDUCE, k_pair_reduce_carry, dim3((unsigned)((nb + 255) / 256 > 0 ? (nb + 255) / 256 : 1)),
                 dim3(256), 0, st, a, nb);
    } else {
      S3R_LAUNCH(K_PAIR_REDUCE, k_pair_reduce, g, dim3(kPairThreads), 0, st, a);
    }
  }
  return hipGetLastError();
}

// plain route: clear the world-frame gradients of every timestep slot of the
// batch (slots = 1 + the largest plain_slot of the views)
__global__ __launch_bounds__(256) void k_zero_plain_w(const int32_t* __restrict__ plain_slot,
                                                      int nv, int64_t n, float4* __restrict__ mw,
                                                      float4* __restrict__ rw) {
  int ns = 0;
  for (int v = 0; v < nv; ++v) ns = max(ns, plain_slot[v] + 1);
  const int64_t n_mw = ns * n * 3 / 4, n_rw = ns * n * 9 / 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n_mw; j += stride) mw[j] = z;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n_rw; j += stride) rw[j] = z;
  // tails (ns * n * 3 and ns * n * 9 need not be multiples of 4)
  if (blockIdx.x == 0 && threadIdx.x < 4) {
    float* m = reinterpret_cast<float*>(mw);
    float* r = reinterpret_cast<float*>(rw);
    const int64_t tm = 4 * n_mw + threadIdx.x, tr = 4 * n_rw + threadIdx.x;
    if (tm < ns * n * 3) m[tm] = 0.f;
    if (tr < ns * n * 9) r[tr] = 0.f;
  }
}

// Sparse gradient mode: clear the rows the previous call wrote, and record
// the Gaussians whose rows this call writes (its records' Gaussians); the
// same launch clears the per-record gradient slots and the two small
// accumulators, as k_zero_g2d does in the dense mode.
// kClearLanes consecutive lanes clear one listed row: its SH coefficients
// as contiguous 16-byte stores (whole cache lines), and one lane each its
// mean, scale, quaternion and opacity.  A row whose Gaussian survives in a
// view of this call is skipped when every survivor got a record: the
// projection backward then writes that row whole (it owns the Gaussian).
constexpr int kClearLanes = 16;

__global__ __launch_bounds__(256) void k_clear_rows(const int32_t* __restrict__ rows,
                                                    const int32_t* __restrict__ n_rows, int64_t n,
                                                    int B, float* __restrict__ mean,
                                                    float* __restrict__ scale,
                                                    float* __restrict__ quat,
                                                    float* __restrict__ opac,
                                                    float* __restrict__ sh,
                                                    const uint32_t* __restrict__ surv,
                                                    int64_t mask_words, int nv,
                                                    const int32_t* __restrict__ counters,
                                                    float4* __restrict__ g2d,
                                                    float* __restrict__ za, int64_t na,
                                                    float* __restrict__ zb, int64_t nb) {
  const int64_t cnt = *n_rows;
  const bool all_kept = counters[S3R_CNT_OVF_SURV] == 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ng = 3 * (int64_t)counters[S3R_CNT_SURV];
    for (int64_t j = i0; j < ng; j += stride) g2d[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (za)
      for (int64_t j = i0; j < na; j += stride) za[j] = 0.f;
    if (zb)
      for (int64_t j = i0; j < nb; j += stride) zb[j] = 0.f;
  }
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < cnt * kClearLanes;
       q += stride) {
    const int i = rows[q / kClearLanes];
    const int sub = (int)(q % kClearLanes);
    if (i < 0 || i >= n) continue;
    if (all_kept) {
      bool rewritten = false;
      for (int v = 0; v < nv && !rewritten; ++v)
        rewritten = (surv[(size_t)v * mask_words + (i >> 5)] >> (i & 31)) & 1u;
      if (rewritten) continue;
    }
    float* s = sh + (size_t)i * 3 * B;
    if (((3 * B) & 3) == 0) {
      float4* s4 = reinterpret_cast<float4*>(s);
      for (int t = sub; t < (3 * B) / 4; t += kClearLanes) s4[t] = make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
      for (int t = sub; t < 3 * B; t += kClearLanes) s[t] = 0.f;
    }
    if (sub < 3) {
      mean[3 * (size_t)i + sub] = 0.f;
      scale[3 * (size_t)i + sub] = 0.f;
    } else if (sub == 3) {
      reinterpret_cast<float4*>(quat)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    } else if (sub == 4) {
      opac[i] = 0.f;
    }
  }
}

hipError_t launch_clear_rows(const int32_t* rows, const int32_t* n_rows, int64_t n, int B,
                             float* mean, float* scale, float* quat, float* opac, float* sh,
                             int64_t cap, const uint32_t* surv, int64_t mask_words, int nv,
                             const BwdArgs& a, hipStream_t st) {
  // (at least the dense mode's 1024 workgroups for the per-record slots)
  const int64_t want = (cap * kClearLanes + 255) / 256;
  const int grid = (int)(want < 2048 ? (want > 1024 ? want : 1024) : 2048);
  S3R_LAUNCH(K_ZERO, k_clear_rows, dim3(grid), dim3(256), 0, st, rows, n_rows, n, B, mean, scale,
             quat, opac, sh, surv, mask_words, nv, a.counters, a.g2d, a.zero_a, a.n_zero_a,
             a.zero_b, a.n_zero_b);
  return hipGetLastError();
}

hipError_t launch_project_bwd(const ProjBwdArgs& a, hipStream_t st) {
  if ((a.kp.flags & S3R_PLAIN) != 0)
    S3R_LAUNCH(K_ZERO, k_zero_plain_w, dim3(2048), dim3(256), 0, st, a.plain_slot, a.nv,
               (int64_t)a.n, reinterpret_cast<float4*>(a.d_mean_w),
               reinterpret_cast<float4*>(a.d_rot_w));
  const int64_t want = (a.kp.cap_surv + 255) / 256;
  const int grid = (int)(want < 4096 ? (want > 0 ? want : 1) : 4096);
  S3R_LAUNCH(K_PROJECT_BWD, k_project_bwd, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_pose_bwd_det(const float* W, const int32_t* tstep, const float* pose,
                               const unsigned long long* d_cam_fx, int nv, int S, int T,
                               float* d_pose, float* d_pose6, hipStream_t st) {
  const int ts = T * S;
  if (ts > 0)
    S3R_LAUNCH(K_POSE_BWD, k_pose_bwd<true>, dim3((ts + 127) / 128), dim3(128), 0, st, W, tstep,
               d_cam_fx, nv, S, T, pose, d_pose, d_pose6);
  return hipGetLastError();
}

hipError_t launch_pose_bwd(const float* W, const int32_t* tstep, const float* pose,
                           const float* d_cam, int nv, int S, int T, float* d_pose,
                           float* d_pose6, hipStream_t st) {
  const int ts = T * S;
  if (ts <= 0) return hipGetLastError();
  if (d_cam != nullptr)
    S3R_LAUNCH(K_POSE_BWD, k_pose_bwd<false>, dim3((ts + 127) / 128), dim3(128), 0, st, W, tstep,
               d_cam, nv, S, T, pose, d_pose, d_pose6);
  else if (d_pose6 != nullptr)
    S3R_LAUNCH(K_POSE6, k_pose6, dim3((ts + 127) / 128), dim3(128), 0, st, pose, d_pose, ts, S,
               d_pose6);
  return hipGetLastError();
}

hipError_t launch_plain_transform_bwd(const float* mean, const float* quat, const int32_t* inst,
                                      const float* pose, int n, int S, const int32_t* tsteps,
                                      int n_ts, const float* d_mean_w, const float* d_rot_w,
                                      float* d_mean, float* d_quat, float* d_pose,
                                      float* d_pose6, hipStream_t st) {
  TsList2 ts;
  for (int s = 0; s < kMaxViews; ++s) ts.tau[s] = s < n_ts ? tsteps[s] : 0;
  const int64_t want = ((int64_t)n + 255) / 256;
  const int grid = (int)(want < 4096 ? (want > 0 ? want : 1) : 4096);
  S3R_LAUNCH(K_PLAIN_TRANSFORM_BWD, k_plain_transform_bwd, dim3(grid), dim3(256), 0, st, mean, quat, inst, pose,
                     n, S, ts, n_ts, d_mean_w, d_rot_w, d_mean, d_quat, d_pose);
  return hipGetLastError();
}

}  // namespace s3r
