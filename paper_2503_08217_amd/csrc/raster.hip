// Front-to-back alpha blending of Eq. (2) over every tile of every view in
// one launch.
//
// One workgroup per tile; a 16x16 tile is a single wave64 whose lanes own four
// pixels each, so every record read from LDS is blended into four pixels.
// The tile's sorted list is consumed in batches: each lane stages one record
// (mean, conic, opacity, colour) in LDS, then every lane blends the whole
// batch into its pixels.  The loop ends as soon as every pixel of the tile
// has reached the transmittance floor.  Pixels are sampled at integer
// coordinates (x, y).
#include "internal.hpp"

namespace s3r {

template <int TS>
__global__ __launch_bounds__(RasterShape<TS>::NT) void k_raster_fwd(RasterArgs a) {
  using Sh = RasterShape<TS>;
  constexpr int NT = Sh::NT, PPT = Sh::PPT, ROWS = Sh::ROWS;
  __shared__ float4 s_geo[NT];  // u, v, opacity
  __shared__ float4 s_con[NT];  // A, B, C
  __shared__ float4 s_rgb[NT];
  const int tid = threadIdx.x;
  const int t = blockIdx.x;
  const int v = find_view(a.tile_offset, a.nv, t);
  const int lt = t - a.tile_offset[v];
  const int W = a.wh[2 * v], H = a.wh[2 * v + 1];
  const int gx = (W + TS - 1) / TS;
  const int px = (lt % gx) * TS + tid % TS;
  const int py0 = (lt / gx) * TS + tid / TS;
  const float fxp = (float)px;
  const int64_t s = a.tile_start[t];
  const int64_t e = min((int64_t)a.tile_start[t + 1], a.kp.cap_dup);

  float T[PPT], cr[PPT], cg[PPT], cb[PPT];
  int last[PPT];
  bool done[PPT];
  bool all_done = true;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    T[k] = 1.f;
    cr[k] = cg[k] = cb[k] = 0.f;
    last[k] = 0;
    done[k] = !(px < W && py0 + k * ROWS < H);
    all_done = all_done && done[k];
  }
  for (int64_t b0 = s; b0 < e; b0 += NT) {
    if (__syncthreads_count(all_done) == NT) break;
    const int64_t idx = b0 + tid;
    if (idx < e) {
      const uint32_t r = a.vals[idx];
      s_geo[tid] = a.rec_geo[r];
      s_con[tid] = a.rec_conic[r];
      s_rgb[tid] = a.rec_rgb[r];
    }
    __syncthreads();
    const int nb = (int)min((int64_t)NT, e - b0);
    if (!all_done) {
      for (int j = 0; j < nb; ++j) {
        const float4 g = s_geo[j];
        const float4 c = s_con[j];
        bool any = false;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          if (done[k]) continue;
          const Blend bl = blend_eval(g.x, g.y, c.x, c.y, c.z, g.z, fxp,
                                      (float)(py0 + k * ROWS), a.kp);
          if (!bl.hit) continue;
          const float Tn = T[k] * (1.0f - bl.alpha);
          if (Tn < a.kp.t_min) {
            done[k] = true;
            continue;
          }
          const float4 col = s_rgb[j];
          const float w = bl.alpha * T[k];
          cr[k] = fmaf(col.x, w, cr[k]);
          cg[k] = fmaf(col.y, w, cg[k]);
          cb[k] = fmaf(col.z, w, cb[k]);
          T[k] = Tn;
          last[k] = (int)(b0 - s) + j + 1;
          any = true;
        }
        (void)any;
        bool dn = true;
#pragma unroll
        for (int k = 0; k < PPT; ++k) dn = dn && done[k];
        if (dn) {
          all_done = true;
          break;
        }
      }
    }
  }
  const int64_t npx = (int64_t)W * H;
  const int64_t base = 3 * a.px_offset[v];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int py = py0 + k * ROWS;
    if (px < W && py < H) {
      const int64_t p = (int64_t)py * W + px;
      a.color[base + p] = fmaf(T[k], a.kp.bg0, cr[k]);
      a.color[base + npx + p] = fmaf(T[k], a.kp.bg1, cg[k]);
      a.color[base + 2 * npx + p] = fmaf(T[k], a.kp.bg2, cb[k]);
      a.T_final[a.px_offset[v] + p] = T[k];
      a.last[a.px_offset[v] + p] = last[k];
    }
  }
}

hipError_t launch_raster_fwd(const RasterArgs& a, hipStream_t st) {
  if (a.total_tiles <= 0) return hipSuccess;
  switch (a.kp.tile) {
    case 8:
      S3R_LAUNCH(K_RASTER_FWD, k_raster_fwd<8>, dim3(a.total_tiles), dim3(RasterShape<8>::NT), 0,
                 st, a);
      break;
    case 16:
      S3R_LAUNCH(K_RASTER_FWD, k_raster_fwd<16>, dim3(a.total_tiles), dim3(RasterShape<16>::NT),
                 0, st, a);
      break;
    case 32:
      S3R_LAUNCH(K_RASTER_FWD, k_raster_fwd<32>, dim3(a.total_tiles), dim3(RasterShape<32>::NT),
                 0, st, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-view mean absolute error and its gradient
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_l1(const float* __restrict__ color,
                                            const float* __restrict__ target,
                                            const int64_t* __restrict__ pxo,
                                            const int32_t* __restrict__ wh, int nv, int64_t total,
                                            float* __restrict__ loss, float* __restrict__ dcol) {
  __shared__ float s_loss[kMaxViews];
  for (int v = threadIdx.x; v < nv; v += blockDim.x) s_loss[v] = 0.f;
  __syncthreads();
  int cur = -1;
  float acc = 0.f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    int v = 0;
    while (v + 1 < nv && pxo[v + 1] <= i) ++v;
    if (v != cur) {
      if (cur >= 0) atomicAdd(&s_loss[cur], acc);
      cur = v;
      acc = 0.f;
    }
    const int64_t npx = (int64_t)wh[2 * v] * wh[2 * v + 1];
    const int64_t loc = i - pxo[v];
    const float inv = 1.0f / (3.0f * (float)npx);
    float a = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t q = 3 * pxo[v] + c * npx + loc;
      const float d = color[q] - target[q];
      a += fabsf(d);
      dcol[q] = d > 0.f ? inv : (d < 0.f ? -inv : 0.f);
    }
    acc += a * inv;
  }
  if (cur >= 0) atomicAdd(&s_loss[cur], acc);
  __syncthreads();
  for (int v = threadIdx.x; v < nv; v += blockDim.x)
    if (s_loss[v] != 0.f) atomicAdd(loss + v, s_loss[v]);
}

hipError_t launch_l1_loss(const float* color, const float* target, const int64_t* px_offset,
                          const int32_t* wh, int nv, int64_t total_px, float* loss,
                          float* d_color, hipStream_t st) {
  hipError_t e = launch_zero(loss, (size_t)nv * 4, nullptr, 0, nullptr, 0, nullptr, 0, st);
  if (e != hipSuccess) return e;
  int64_t grid = (total_px + 255) / 256;
  if (grid > 1024) grid = 1024;
  if (grid > 0)
    S3R_LAUNCH(K_L1, k_l1, dim3((unsigned)grid), dim3(256), 0, st, color, target, px_offset, wh,
                       nv, total_px, loss, d_color);
  return hipGetLastError();
}

}  // namespace s3r
