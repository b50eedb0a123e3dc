// Front-to-back alpha blending of Eq. (2) over every tile of every view in
// one launch.
//
// One workgroup per tile, one thread per pixel; each wave64 owns an 8x8
// sub-tile of the 16x16 tile.  The tile's sorted list is consumed in
// batches: each thread stages one record (mean, conic, opacity, colour and the
// bounding box of its cutoff ellipse) in LDS, then every wave blends the batch
// into its pixels, skipping -- uniformly across the wave -- records whose box
// misses its sub-tile (no pixel there could pass the Mahalanobis cut).  The
// loop ends as soon as every pixel of the tile has reached the transmittance
// floor.  Pixels are sampled at integer coordinates (x, y).
#include "internal.hpp"

namespace s3r {

template <int TS>
__global__ __launch_bounds__(RasterShape<TS>::NT) void k_raster_fwd(RasterArgs a) {
  constexpr int NT = RasterShape<TS>::NT;
  __shared__ float4 s_geo[NT];  // u, v, opacity
  __shared__ float4 s_con[NT];  // A, B, C
  __shared__ float4 s_rgb[NT];
  __shared__ float4 s_box[NT];  // cutoff bounding box
  const int tid = threadIdx.x;
  const int t = blockIdx.x;
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
  for (int64_t b0 = s; b0 < e; b0 += NT) {
    if (__syncthreads_count(done) == NT) break;
    const int64_t idx = b0 + tid;
    if (idx < e) {
      const uint32_t r = a.vals[idx];
      const float4 g = a.rec_geo[r];
      const float4 c = a.rec_conic[r];
      s_geo[tid] = g;
      s_con[tid] = c;
      s_rgb[tid] = a.rec_rgb[r];
      s_box[tid] = cutoff_box(g.x, g.y, c.x, c.y, c.z, a.kp.cutoff);
    }
    __syncthreads();
    const int nb = (int)min((int64_t)NT, e - b0);
    // the wave walks the batch while any of its pixels is still open
    if (ballot(!done) != 0ull) {
      for (int j = 0; j < nb; ++j) {
        if (!box_hits(s_box[j], sub_x, sub_y)) continue;  // uniform across the wave
        if (done) continue;
        const float4 g = s_geo[j];
        const float4 c = s_con[j];
        const Blend bl = blend_eval(g.x, g.y, c.x, c.y, c.z, g.z, fxp, fyp, a.kp);
        if (!bl.hit) continue;
        const float Tn = T * (1.0f - bl.alpha);
        if (Tn < a.kp.t_min) {
          done = true;
          continue;
        }
        const float4 col = s_rgb[j];
        const float w = bl.alpha * T;
        cr = fmaf(col.x, w, cr);
        cg = fmaf(col.y, w, cg);
        cb = fmaf(col.z, w, cb);
        T = Tn;
        last = (int)(b0 - s) + j + 1;
      }
    }
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
