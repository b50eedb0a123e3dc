// Zero-fill of device buffers with a kernel (capturable in a hipGraph as a
// kernel node; no memset nodes are recorded).
#include "internal.hpp"

namespace s3r {

struct ZeroList {
  uint32_t* p[4];
  size_t words[4];
};

__global__ void k_zero(ZeroList z) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    uint32_t* p = z.p[b];
    const size_t n = z.words[b];
    for (size_t i = t0; i < n; i += stride) p[i] = 0u;
  }
}

hipError_t launch_zero(void* p0, size_t b0, void* p1, size_t b1, void* p2, size_t b2, void* p3,
                       size_t b3, hipStream_t st) {
  ZeroList z;
  void* ps[4] = {p0, p1, p2, p3};
  size_t bs[4] = {b0, b1, b2, b3};
  size_t most = 0;
  for (int b = 0; b < 4; ++b) {
    z.p[b] = static_cast<uint32_t*>(ps[b]);
    z.words[b] = ps[b] ? bs[b] / 4 : 0;
    if (z.words[b] > most) most = z.words[b];
  }
  if (most == 0) return hipSuccess;
  size_t blocks = (most + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  S3R_LAUNCH(K_ZERO, k_zero, dim3((unsigned)blocks), dim3(256), 0, st, z);
  return hipGetLastError();
}

}  // namespace s3r
