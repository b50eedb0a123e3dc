// Device-side building blocks shared by the gfx950 kernels.
//
// Everything here is compiled with -ffp-contract=off and correctly rounded
// binary32 division and square root, so the projection below evaluates each
// expression exactly in the order it is written: every decision it feeds
// (depth test, determinant sign, footprint rectangle, LOD test, depth key) is
// reproducible bit for bit.  Rasterisation code that wants fused multiply-adds
// asks for them explicitly with fmaf().
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/s3r.h"

namespace s3r {

constexpr int kWave = 64;
// dies (XCDs) of the chip, each with its own L2; consecutive workgroup ids are
// dealt to them round-robin
constexpr int kXcds = 8;
constexpr int kMaxViews = 64;

// ---------------------------------------------------------------------------
// wave-level primitives (wave64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
// value of x in lane j (j wave-uniform), as a scalar operand
__device__ __forceinline__ float bcast(float x, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), j));
}

// number of set bits of `mask` below this lane
__device__ __forceinline__ int lane_rank(uint64_t mask) {
  uint32_t lo = __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u);
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), lo);
}

// Sum over the 64 lanes with DPP row operations; the total is valid in lane 63.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float x) {
  const int y = __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, true);
  return x + __int_as_float(y);
}
__device__ __forceinline__ float wave_sum_dpp(float x) {
  x = dpp_add<0xB1, 0xf>(x);   // quad_perm [1,0,3,2]
  x = dpp_add<0x4E, 0xf>(x);   // quad_perm [2,3,0,1]
  x = dpp_add<0x124, 0xf>(x);  // row_ror:4
  x = dpp_add<0x128, 0xf>(x);  // row_ror:8  -> every lane holds its row's sum
  x = dpp_add<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x = dpp_add<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

// Four wave-wide sums at once: a permlane32 swap pairs x with y and z with w
// (each register then holds one value's half-sums in lanes 0-31 and the
// other's in lanes 32-63), a permlane16 swap pairs the two results, and DPP
// row sums finish.  On return every lane of row k (lanes 16k..16k+15) holds
// the wave total of x (k = 0), z (k = 1), y (k = 2) or w (k = 3).
__device__ __forceinline__ float wave_sum4(float x, float y, float z, float w) {
  const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                  false);
  const auto q = __builtin_amdgcn_permlane32_swap(__float_as_uint(z), __float_as_uint(w), false,
                                                  false);
  const float xy = __uint_as_float(p[0]) + __uint_as_float(p[1]);
  const float zw = __uint_as_float(q[0]) + __uint_as_float(q[1]);
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(xy), __float_as_uint(zw), false,
                                                  false);
  float s = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  s = dpp_add<0xB1, 0xf>(s);   // quad_perm [1,0,3,2]
  s = dpp_add<0x4E, 0xf>(s);   // quad_perm [2,3,0,1]
  s = dpp_add<0x124, 0xf>(s);  // row_ror:4
  s = dpp_add<0x128, 0xf>(s);  // row_ror:8
  return s;
}

// sum over each 16-lane row, in every lane of the row
__device__ __forceinline__ float row_sum(float s) {
  s = dpp_add<0xB1, 0xf>(s);   // quad_perm [1,0,3,2]
  s = dpp_add<0x4E, 0xf>(s);   // quad_perm [2,3,0,1]
  s = dpp_add<0x124, 0xf>(s);  // row_ror:4
  s = dpp_add<0x128, 0xf>(s);  // row_ror:8
  return s;
}

// inclusive prefix sum over the 64 lanes (DPP: row shifts, then row
// broadcasts across rows; no LDS)
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_add_i32(int x) {
  return x + __builtin_amdgcn_update_dpp(0, x, CTRL, ROW_MASK, 0xf, false);
}
__device__ __forceinline__ int wave_inclusive_scan(int x) {
  x = dpp_add_i32<0x111, 0xf>(x);  // row_shr:1
  x = dpp_add_i32<0x112, 0xf>(x);  // row_shr:2
  x = dpp_add_i32<0x114, 0xf>(x);  // row_shr:4
  x = dpp_add_i32<0x118, 0xf>(x);  // row_shr:8
  x = dpp_add_i32<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x = dpp_add_i32<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

// wave total, in every lane (DPP scan, then lane 63: no LDS round trips)
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readlane(wave_inclusive_scan((int)v), kWave - 1);
}

// ---------------------------------------------------------------------------
// parameters copied by value into every kernel
// ---------------------------------------------------------------------------
struct KParams {
  int tile;
  uint32_t flags;
  float lod_r, z_near, z_far, eps2d, alpha_min, alpha_max, t_min, cutoff, jac_clamp;
  float bg0, bg1, bg2;
  int64_t cap_surv, cap_dup;
  uint64_t seed;
  float lod_pmax, lod_D;
  uint32_t step;
};

// Philox4x32-10 (Salmon et al., SC'11): first output word of counter
// (c0, c1, c2, c3) under key (k0, k1).
__device__ __forceinline__ uint32_t philox_first(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
  }
  return c0;
}

// ---------------------------------------------------------------------------
// canonical binary32 projection of one Gaussian into one view
// ---------------------------------------------------------------------------
struct Proj {
  float px, py, pz;
  float u, v;
  float a_raw, b, c_raw;  // undilated 2D covariance
  float a, c, det;        // dilated entries and determinant
  float lam_raw;
  int x0, y0, x1, y1;     // tile rectangle [x0,x1) x [y0,y1)
  bool depth_ok, visible, keep;
};

// Unit quaternion (w,x,y,z) -> rotation, normalising first.
__device__ __forceinline__ void quat_rot(float w, float x, float y, float z, float R[9]) {
  float n = sqrtf(((w * w + x * x) + y * y) + z * z);
  w = w / n; x = x / n; y = y / n; z = z / n;
  float xx = x * x, yy = y * y, zz = z * z;
  float xy = x * y, xz = x * z, yz = y * z;
  float wx = w * x, wy = w * y, wz = w * z;
  R[0] = 1.0f - 2.0f * (yy + zz); R[1] = 2.0f * (xy - wz); R[2] = 2.0f * (xz + wy);
  R[3] = 2.0f * (xy + wz); R[4] = 1.0f - 2.0f * (xx + zz); R[5] = 2.0f * (yz - wx);
  R[6] = 2.0f * (xz - wy); R[7] = 2.0f * (yz + wx); R[8] = 1.0f - 2.0f * (xx + yy);
}

__device__ __forceinline__ float lam_max(float a, float c, float det) {
  float m = 0.5f * (a + c);
  float disc = m * m - det;
  return m + sqrtf(fmaxf(disc, 0.0f));
}

__device__ __forceinline__ float clamp_nan(float v, float hi) {
  // clamp to [0, hi], propagating NaN like numpy's maximum/minimum
  return (v != v) ? v : fminf(fmaxf(v, 0.0f), hi);
}

// Rg: the Gaussian's rotation (row-major 3x3), s: its scales, P: camera 3x4
// (row-major), mean: position in the frame P maps from.
// camera-space depth of a mean, in the canonical operation order, and the
// depth test it must pass (the first condition of M_t)
__device__ __forceinline__ float cam_depth(const float P[12], float mx, float my, float mz) {
  return ((P[8] * mx + P[9] * my) + P[10] * mz) + P[11];
}
__device__ __forceinline__ bool depth_pass(float pz, const KParams& kp) {
  return (kp.z_near < pz) && (pz < kp.z_far);
}

__device__ __forceinline__ void project_canonical(const float P[12], float mx, float my, float mz,
                                                  const float Rg[9], float s0, float s1, float s2,
                                                  float fx, float fy, float cx, float cy, int W,
                                                  int H, const KParams& kp, Proj& o, int gid = 0,
                                                  int view = 0) {
  o.px = ((P[0] * mx + P[1] * my) + P[2] * mz) + P[3];
  o.py = ((P[4] * mx + P[5] * my) + P[6] * mz) + P[7];
  o.pz = cam_depth(P, mx, my, mz);
  o.depth_ok = depth_pass(o.pz, kp);

  float M[9];
  M[0] = Rg[0] * s0; M[1] = Rg[1] * s1; M[2] = Rg[2] * s2;
  M[3] = Rg[3] * s0; M[4] = Rg[4] * s1; M[5] = Rg[5] * s2;
  M[6] = Rg[6] * s0; M[7] = Rg[7] * s1; M[8] = Rg[8] * s2;
  float S00 = (M[0] * M[0] + M[1] * M[1]) + M[2] * M[2];
  float S01 = (M[0] * M[3] + M[1] * M[4]) + M[2] * M[5];
  float S02 = (M[0] * M[6] + M[1] * M[7]) + M[2] * M[8];
  float S11 = (M[3] * M[3] + M[4] * M[4]) + M[5] * M[5];
  float S12 = (M[3] * M[6] + M[4] * M[7]) + M[5] * M[8];
  float S22 = (M[6] * M[6] + M[7] * M[7]) + M[8] * M[8];

  float tx = o.px / o.pz;
  float ty = o.py / o.pz;
  float lx = kp.jac_clamp * ((0.5f * (float)W) / fx);
  float ly = kp.jac_clamp * ((0.5f * (float)H) / fy);
  float txc = fminf(fmaxf(tx, -lx), lx);
  float tyc = fminf(fmaxf(ty, -ly), ly);
  float j00 = fx / o.pz;
  float j02 = -((fx * txc) / o.pz);
  float j11 = fy / o.pz;
  float j12 = -((fy * tyc) / o.pz);

  float A00 = j00 * P[0] + j02 * P[8];
  float A01 = j00 * P[1] + j02 * P[9];
  float A02 = j00 * P[2] + j02 * P[10];
  float A10 = j11 * P[4] + j12 * P[8];
  float A11 = j11 * P[5] + j12 * P[9];
  float A12 = j11 * P[6] + j12 * P[10];

  float B00 = (A00 * S00 + A01 * S01) + A02 * S02;
  float B01 = (A00 * S01 + A01 * S11) + A02 * S12;
  float B02 = (A00 * S02 + A01 * S12) + A02 * S22;
  float B10 = (A10 * S00 + A11 * S01) + A12 * S02;
  float B11 = (A10 * S01 + A11 * S11) + A12 * S12;
  float B12 = (A10 * S02 + A11 * S12) + A12 * S22;

  o.a_raw = (B00 * A00 + B01 * A01) + B02 * A02;
  o.b = (B00 * A10 + B01 * A11) + B02 * A12;
  o.c_raw = (B10 * A10 + B11 * A11) + B12 * A12;
  o.a = o.a_raw + kp.eps2d;
  o.c = o.c_raw + kp.eps2d;
  o.det = o.a * o.c - o.b * o.b;
  float det_raw = o.a_raw * o.c_raw - o.b * o.b;
  float lam_d = lam_max(o.a, o.c, o.det);
  o.lam_raw = lam_max(o.a_raw, o.c_raw, det_raw);
  float rad = ceilf(3.0f * sqrtf(lam_d));
  o.u = fx * tx + cx;
  o.v = fy * ty + cy;

  const int ts = kp.tile;
  const float sf = (float)ts;
  const int gx = (W + ts - 1) / ts;
  const int gy = (H + ts - 1) / ts;
  float x0f = clamp_nan(floorf((o.u - rad) / sf), (float)gx);
  float x1f = clamp_nan(floorf((o.u + rad) / sf) + 1.0f, (float)gx);
  float y0f = clamp_nan(floorf((o.v - rad) / sf), (float)gy);
  float y1f = clamp_nan(floorf((o.v + rad) / sf) + 1.0f, (float)gy);
  bool bad = (x0f != x0f) || (x1f != x1f) || (y0f != y0f) || (y1f != y1f);
  o.x0 = bad ? 0 : (int)x0f;
  o.x1 = bad ? 0 : (int)x1f;
  o.y0 = bad ? 0 : (int)y0f;
  o.y1 = bad ? 0 : (int)y1f;
  o.visible = o.depth_ok && (o.det > 0.0f) && (o.x1 > o.x0) && (o.y1 > o.y0);
  const float r = kp.lod_r;
  const bool lod = (kp.flags & S3R_LOD) && (r > 0.0f);
  bool drop = lod && (o.lam_raw <= r * r);
  if (drop && (kp.flags & S3R_LOD_STOCHASTIC)) {
    // Eq. (7): drop probability grows with depth from 0.01 to p_max at D
    const float t1 = o.pz - kp.lod_D;
    const float t2 = t1 / kp.lod_D;
    const float t3 = fminf(0.0f, t2);
    const float p = kp.lod_pmax + (kp.lod_pmax - 0.01f) * t3;
    const uint32_t x = philox_first((uint32_t)gid, (uint32_t)view, kp.step, 0u,
                                    (uint32_t)kp.seed, (uint32_t)(kp.seed >> 32));
    const float u = (float)(x >> 8) * 5.9604644775390625e-08f;
    drop = u < p;
  }
  o.keep = !drop;
}

// ---------------------------------------------------------------------------
// real spherical harmonics, degree <= 3 (3DGS sign convention)
// ---------------------------------------------------------------------------
constexpr float kC0 = 0.28209479177387814f;
constexpr float kC1 = 0.4886025119029199f;
constexpr float kC2_0 = 1.0925484305920792f;
constexpr float kC2_1 = -1.0925484305920792f;
constexpr float kC2_2 = 0.31539156525252005f;
constexpr float kC2_3 = -1.0925484305920792f;
constexpr float kC2_4 = 0.5462742152960396f;
constexpr float kC3_0 = -0.5900435899266435f;
constexpr float kC3_1 = 2.890611442640554f;
constexpr float kC3_2 = -0.4570457994644658f;
constexpr float kC3_3 = 0.3731763325901154f;
constexpr float kC3_4 = -0.4570457994644658f;
constexpr float kC3_5 = 1.445305721320277f;
constexpr float kC3_6 = -0.5900435899266435f;

__device__ __forceinline__ void sh_basis(int deg, float x, float y, float z, float Y[16]) {
  Y[0] = kC0;
  if (deg < 1) return;
  Y[1] = -kC1 * y; Y[2] = kC1 * z; Y[3] = -kC1 * x;
  if (deg < 2) return;
  float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = kC2_0 * (x * y);
  Y[5] = kC2_1 * (y * z);
  Y[6] = kC2_2 * (2.0f * zz - xx - yy);
  Y[7] = kC2_3 * (x * z);
  Y[8] = kC2_4 * (xx - yy);
  if (deg < 3) return;
  Y[9] = kC3_0 * y * (3.0f * xx - yy);
  Y[10] = kC3_1 * (x * y) * z;
  Y[11] = kC3_2 * y * (4.0f * zz - xx - yy);
  Y[12] = kC3_3 * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
  Y[13] = kC3_4 * x * (4.0f * zz - xx - yy);
  Y[14] = kC3_5 * z * (xx - yy);
  Y[15] = kC3_6 * x * (xx - 3.0f * yy);
}

// d(sum_b g_b Y_b)/d(x,y,z) for per-basis weights g_b.
__device__ __forceinline__ void sh_basis_grad(int deg, float x, float y, float z, const float g[16],
                                              float& dx, float& dy, float& dz) {
  dx = 0.f; dy = 0.f; dz = 0.f;
  if (deg < 1) return;
  dy += -kC1 * g[1]; dz += kC1 * g[2]; dx += -kC1 * g[3];
  if (deg < 2) return;
  float xx = x * x, yy = y * y, zz = z * z;
  dx += kC2_0 * y * g[4]; dy += kC2_0 * x * g[4];
  dy += kC2_1 * z * g[5]; dz += kC2_1 * y * g[5];
  dx += -2.0f * kC2_2 * x * g[6]; dy += -2.0f * kC2_2 * y * g[6]; dz += 4.0f * kC2_2 * z * g[6];
  dx += kC2_3 * z * g[7]; dz += kC2_3 * x * g[7];
  dx += 2.0f * kC2_4 * x * g[8]; dy += -2.0f * kC2_4 * y * g[8];
  if (deg < 3) return;
  dx += kC3_0 * 6.0f * x * y * g[9]; dy += kC3_0 * (3.0f * xx - 3.0f * yy) * g[9];
  dx += kC3_1 * y * z * g[10]; dy += kC3_1 * x * z * g[10]; dz += kC3_1 * x * y * g[10];
  dx += kC3_2 * (-2.0f * x * y) * g[11]; dy += kC3_2 * (4.0f * zz - xx - 3.0f * yy) * g[11];
  dz += kC3_2 * 8.0f * y * z * g[11];
  dx += kC3_3 * (-6.0f * x * z) * g[12]; dy += kC3_3 * (-6.0f * y * z) * g[12];
  dz += kC3_3 * (6.0f * zz - 3.0f * xx - 3.0f * yy) * g[12];
  dx += kC3_4 * (4.0f * zz - 3.0f * xx - yy) * g[13]; dy += kC3_4 * (-2.0f * x * y) * g[13];
  dz += kC3_4 * 8.0f * x * z * g[13];
  dx += kC3_5 * 2.0f * x * z * g[14]; dy += kC3_5 * (-2.0f * y * z) * g[14];
  dz += kC3_5 * (xx - yy) * g[14];
  dx += kC3_6 * (3.0f * xx - 3.0f * yy) * g[15]; dy += kC3_6 * (-6.0f * x * y) * g[15];
}

// ---------------------------------------------------------------------------
// blending of one (pixel, record) pair -- shared by the forward and the
// backward so that both take every skip / clamp / stop decision identically
// ---------------------------------------------------------------------------
struct Blend {
  float power, ex, raw, alpha;
  bool hit;  // passes the Mahalanobis cut and alpha_min
};

__device__ __forceinline__ Blend blend_eval(float u, float v, float A, float Bc, float C, float o,
                                            float px, float py, const KParams& kp) {
  // evaluated without branches: the exponential is taken even past the cut
  // (its value is then unused), so a wave needs no divergent control flow
  Blend b;
  const float dx = u - px;
  const float dy = v - py;
  b.power = fmaf(-0.5f, fmaf(A * dx, dx, C * dy * dy), -Bc * dx * dy);
  b.ex = __expf(b.power);
  b.raw = o * b.ex;
  // min(alpha_max, raw) as one v_med3 clamp to [0, alpha_max]: raw is finite
  // (the power of a positive-definite conic exceeds zero by at most a
  // rounding error), equal to the minimum for raw >= 0, and for raw < 0 (a
  // negative opacity) both fall below alpha_min, so no pixel takes the entry
  b.alpha = __builtin_amdgcn_fmed3f(b.raw, 0.0f, kp.alpha_max);
  b.hit = !(-b.power > kp.cutoff) && !(b.alpha < kp.alpha_min);
  return b;
}

// Rasterizer layout: one thread per pixel, each wave64 owns an 8x8 sub-tile
// (a 16x16 tile is four waves).  Lane l of wave w covers pixel
// (8 (w % (TS/8)) + l % 8, 8 (w / (TS/8)) + l / 8) of the tile.
template <int TS>
struct RasterShape {
  static constexpr int NT = TS * TS;
  static constexpr int SUB = TS / 8;  // sub-tiles per row
  static constexpr int NW = NT / 64;
  // list entries whose gradients the raster backward accumulates in LDS at
  // once (36 B each; 18 KB for a 16x16 tile keeps eight workgroups per CU)
  static constexpr int WIN = 2 * NT;
};
template <int TS>
__device__ __forceinline__ void raster_pixel(int tid, int& ox, int& oy, int& sx, int& sy) {
  const int w = tid / 64, l = tid % 64;
  sx = 8 * (w % RasterShape<TS>::SUB);
  sy = 8 * (w / RasterShape<TS>::SUB);
  ox = sx + (l % 8);
  oy = sy + (l / 8);
}

// Half-widths of the bounding box of the pixels where a record can pass the
// Mahalanobis cut.  -power <= cutoff means d^T Q d <= 2 cutoff (Q the conic),
// an ellipse whose extent along x is sqrt(2 cutoff (Q^-1)_xx) =
// sqrt(2 cutoff C / det Q).  The rasterizer's binary32 evaluation of the form
// differs from the exact one by at most ~30 u kappa relative (u = 2^-24,
// kappa = condition of Q, bounded above by (A + C)^2 / det); the box is grown
// by that margin so that skipping records outside it never removes a pixel
// the blend test would keep, and is unbounded (3e38) when Q is too
// ill-conditioned for the bound to be useful.  k_records stores them with
// the record (the conic's and the colour's fourth component), so the
// rasterizers' per-wave tests take no division or square root.
__device__ __forceinline__ float2 cutoff_half(float A, float B, float C, float cutoff) {
  const float det = A * C - B * B;
  const float tr = A + C;
  const float kap = tr * tr / det;
  if (!(det > 0.f) || !(kap < 1.0e5f)) return make_float2(3.0e38f, 3.0e38f);
  const float grow = 2.f * cutoff * (1.002f + 64.f * 5.9604645e-8f * kap) / det;
  return make_float2(sqrtf(grow * C) + 0.01f, sqrtf(grow * A) + 0.01f);
}
__device__ __forceinline__ float4 cutoff_box(float u, float v, float2 h) {
  return make_float4(u - h.x, u + h.x, v - h.y, v + h.y);
}
// the box meets the pixel square [x0, x0 + ext] x [y0, y0 + ext]
__device__ __forceinline__ bool box_hits(float4 b, float x0, float y0, float ext = 7.f) {
  return (b.y >= x0) && (b.x <= x0 + ext) && (b.w >= y0) && (b.z <= y0 + ext);
}

// q = A dx^2 + 2 B dx dy + C dy^2 at dx on the segment dy in [dyl, dyh], at
// the segment's minimising dy (rC = 1 / C to about an ulp: a dy off the
// minimiser by e raises q by C e^2, far inside the caller's margin)
__device__ __forceinline__ float edge_min_q(float dx, float dyl, float dyh, float A, float B,
                                            float C, float rC) {
  const float dy = fminf(fmaxf(-B * dx * rC, dyl), dyh);
  return (A * dx) * dx + (2.f * B * dx) * dy + (C * dy) * dy;
}

// Can any pixel (x, y) of the square [x0, x0 + ext]^2 pass blend_eval's two
// tests (-power <= cutoff, alpha >= alpha_min) for a record at (u, v) with
// conic (A, B, C) and opacity o?  False only when none can.  blend_eval's
// power is -q/2 with q = A dx^2 + 2 B dx dy + C dy^2 (dx = u - x, dy = v - y);
// the minimum of q over the square is 0 when (u, v) lies in it and otherwise
// lies on an edge facing (u, v) -- the x-edge on (u, v)'s side when u is
// outside [x0, x0 + ext], the y-edge likewise: q is convex, and at a minimum
// inside an edge whose line (u, v) does not cross q would fall into the
// square -- so the least of those (at most) two edges' minima; the edge
// taken when (u, v) is within an edge's range is harmless (its minimum is
// not below the square's).  The binary32 power of
// the kernel and this minimum each differ from the exact values by a few
// units of rounding relative to A dx^2 + C dy^2 <= q / (1 - rho), rho =
// |B| / sqrt(A C) < 1 for a positive-definite conic, so the minimum is
// lowered by 64 u / (1 - rho) relative (u = 2^-24) before the tests, and
// conics with rho > 0.999 are never skipped.  The alpha test allows the
// exponential and the opacity product a relative error of 2^-16.
__device__ __forceinline__ bool square_may_hit(float u, float v, float A, float B, float C,
                                               float o, float x0, float y0, float ext,
                                               const KParams& kp) {
  const float dxl = u - (x0 + ext), dxh = u - x0;
  const float dyl = v - (y0 + ext), dyh = v - y0;
  if (dxl <= 0.f && dxh >= 0.f && dyl <= 0.f && dyh >= 0.f)
    return o * 1.0000153f >= kp.alpha_min;  // alpha <= o e^(rounding) there
  const float rho = fabsf(B) * __builtin_amdgcn_rsqf(A * C);
  if (!(A > 0.f) || !(C > 0.f) || !(rho <= 0.999f)) return true;
  const float rA = __builtin_amdgcn_rcpf(A), rC = __builtin_amdgcn_rcpf(C);
  const float dxe = dxl > 0.f ? dxl : dxh;  // u right of the square: its right edge
  const float dye = dyl > 0.f ? dyl : dyh;
  const float q = fminf(edge_min_q(dxe, dyl, dyh, A, B, C, rC), edge_min_q(dye, dxl, dxh, C, B, A, rA));
  // 64 u / (1 - rho), the reciprocal rounded down by at most a few ulp
  const float qlo = q * (1.f - 3.8148e-6f * __builtin_amdgcn_rcpf(1.f - rho));
  const float pmax = -0.5f * qlo;                             // >= every pixel's power
  if (-pmax > kp.cutoff) return false;
  return o * __expf(pmax) * 1.0000153f >= kp.alpha_min;
}

// The records holding the pairs [P, Pe) of a workgroup of NTH threads (each
// record has at least one pair, so at most Pe - P of them): their first pairs
// (pair_off, non-decreasing) are staged in s_pair[0 .. nw) and s_pair[nw] is
// the first pair after them.  The two record searches run cooperatively, NTH
// probes per round (about three rounds of parallel loads instead of a chain
// of dependent ones per thread).  Returns the first record; *nw_out gets nw.
// s_pair holds Pe - P + 2 ints, s_red 2 NTH / 64.
template <int NTH>
__device__ __forceinline__ int record_window(const int32_t* __restrict__ pair_off, int nrec,
                                             int64_t P, int64_t Pe, int* s_pair, int* s_red,
                                             int* nw_out) {
  const int tid = threadIdx.x, wave = tid / kWave;
  constexpr int NW = NTH / kWave;
  int lo0 = 0, hi0 = nrec - 1, lo1 = 0, hi1 = nrec - 1;  // last record with first pair <= P, <= Pe - 1
  while (hi0 > lo0 || hi1 > lo1) {  // uniform over the workgroup
    const int st0 = (hi0 - lo0 + NTH) / NTH;
    const int st1 = (hi1 - lo1 + NTH) / NTH;
    const int i0 = lo0 + tid * st0, i1 = lo1 + tid * st1;
    const bool ok0 = i0 <= hi0 && pair_off[i0] <= P;
    const bool ok1 = i1 <= hi1 && pair_off[i1] <= Pe - 1;
    // first pairs are non-decreasing: the probes that pass form a prefix
    const uint64_t b0 = ballot(ok0), b1 = ballot(ok1);
    if ((tid % kWave) == 0) {
      s_red[wave] = __popcll(b0);
      s_red[NW + wave] = __popcll(b1);
    }
    __syncthreads();
    int c0 = 0, c1 = 0;
    for (int w = 0; w < NW; ++w) {
      c0 += s_red[w];
      c1 += s_red[NW + w];
    }
    __syncthreads();
    lo0 += (c0 - 1) * st0;
    hi0 = min(hi0, lo0 + st0 - 1);
    lo1 += (c1 - 1) * st1;
    hi1 = min(hi1, lo1 + st1 - 1);
  }
  const int nw = lo1 - lo0 + 1;
  for (int i = tid; i <= nw; i += NTH)
    s_pair[i] = (lo0 + i < nrec) ? pair_off[lo0 + i] : INT32_MAX;
  __syncthreads();
  *nw_out = nw;
  return lo0;
}

// SH coefficients of one Gaussian (B*3 floats) into registers; 16-byte loads
// when the per-Gaussian stride keeps them aligned (degrees 1 and 3)
__device__ __forceinline__ void load_sh(const float* __restrict__ f, int B, float out[48]) {
  const int nf = 3 * B;
  if ((nf & 3) == 0) {
    const float4* f4 = reinterpret_cast<const float4*>(f);
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      if (4 * q < nf) {
        const float4 x = f4[q];
        out[4 * q] = x.x; out[4 * q + 1] = x.y; out[4 * q + 2] = x.z; out[4 * q + 3] = x.w;
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < 48; ++q)
      if (q < nf) out[q] = f[q];
  }
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

__device__ __forceinline__ int find_view(const int32_t* __restrict__ tile_offset, int nv, int t) {
  int v = 0;
  while (v + 1 < nv && tile_offset[v + 1] <= t) ++v;
  return v;
}

}  // namespace s3r
