// Zero-fill of device buffers with a kernel (capturable in a hipGraph as a
// kernel node; no memset nodes are recorded).
#include "internal.hpp"

namespace s3r {

constexpr int kZeroMax = 8;
struct ZeroList {
  uint32_t* p[kZeroMax];
  size_t words[kZeroMax];
};

// Buffers are 16-byte aligned (the ABI requires it): 16-byte stores for the
// bulk, 4-byte stores for a tail of fewer than four words.
__global__ void k_zero(ZeroList z) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
  for (int b = 0; b < kZeroMax; ++b) {
    uint32_t* p = z.p[b];
    const size_t n = z.words[b];
    uint4* p4 = reinterpret_cast<uint4*>(p);
    const size_t n4 = n / 4;
    for (size_t i = t0; i < n4; i += stride) p4[i] = make_uint4(0u, 0u, 0u, 0u);
    for (size_t i = 4 * n4 + t0; i < n; i += stride) p[i] = 0u;
  }
}

hipError_t launch_zero_n(void* const* ps, const size_t* bytes, int count, hipStream_t st) {
  ZeroList z;
  size_t most = 0;
  for (int b = 0; b < kZeroMax; ++b) {
    const bool use = b < count && ps[b] != nullptr;
    z.p[b] = use ? static_cast<uint32_t*>(ps[b]) : nullptr;
    z.words[b] = use ? bytes[b] / 4 : 0;
    if (z.words[b] > most) most = z.words[b];
  }
  if (most == 0) return hipSuccess;
  size_t blocks = (most / 4 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 8192) blocks = 8192;
  S3R_LAUNCH(K_ZERO, k_zero, dim3((unsigned)blocks), dim3(256), 0, st, z);
  return hipGetLastError();
}

hipError_t launch_zero(void* p0, size_t b0, void* p1, size_t b1, void* p2, size_t b2, void* p3,
                       size_t b3, hipStream_t st) {
  void* ps[4] = {p0, p1, p2, p3};
  const size_t bs[4] = {b0, b1, b2, b3};
  return launch_zero_n(ps, bs, 4, st);
}

}  // namespace s3r
