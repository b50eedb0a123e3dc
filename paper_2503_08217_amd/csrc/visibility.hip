// Temporal-visibility state update (Sec. 3.3 "Temporal separation"):
//   UPDATE (Eq. 5): l_s = min(l_s, t_v), l_e = max(l_e, t_v) for every view v
//                   of the batch whose M_t bit is set;
//   FOLD   (Eq. 6): v_s = l_s - margin, v_e = l_e + margin;
//   RESET:          v = (-1, 1), l = (1, -1).
// One thread per Gaussian loops over the batch's mask bits, so no atomics are
// needed and the result does not depend on the order of the views.
#include "internal.hpp"

namespace s3r {

__global__ __launch_bounds__(256) void k_visibility(float* __restrict__ life_s,
                                                    float* __restrict__ life_e,
                                                    float* __restrict__ vis_s,
                                                    float* __restrict__ vis_e,
                                                    const uint32_t* __restrict__ mask,
                                                    const float* __restrict__ t_norm, int nv,
                                                    int64_t n, int64_t words, int mode,
                                                    float margin) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (mode == S3R_VIS_UPDATE) {
    uint64_t bits = 0;
    for (int v = 0; v < nv; ++v)
      if ((mask[(size_t)v * words + (i >> 5)] >> (i & 31)) & 1u) bits |= 1ull << v;
    if (!bits) return;
    float ls = life_s[i], le = life_e[i];
    for (int v = 0; v < nv; ++v) {
      if ((bits >> v) & 1ull) {
        const float t = t_norm[v];
        ls = fminf(ls, t);
        le = fmaxf(le, t);
      }
    }
    life_s[i] = ls;
    life_e[i] = le;
  } else if (mode == S3R_VIS_FOLD) {
    vis_s[i] = life_s[i] - margin;
    vis_e[i] = life_e[i] + margin;
  } else {
    vis_s[i] = -1.0f;
    vis_e[i] = 1.0f;
    life_s[i] = 1.0f;
    life_e[i] = -1.0f;
  }
}

hipError_t launch_visibility(float* life_s, float* life_e, float* vis_s, float* vis_e,
                             const uint32_t* mask, const float* t_norm, int nv, int64_t n,
                             int mode, float margin, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t words = ((n + 63) / 64) * 2;
  const int64_t grid = (n + 255) / 256;
  S3R_LAUNCH(K_VISIBILITY, k_visibility, dim3((unsigned)grid), dim3(256), 0, st, life_s, life_e, vis_s,
                     vis_e, mask, t_norm, nv, n, words, mode, margin);
  return hipGetLastError();
}

}  // namespace s3r
