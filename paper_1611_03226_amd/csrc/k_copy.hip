// Plain device-to-device stream copy: the bandwidth and traffic-counter
// reference against which the actor kernels are measured.  16-byte loads
// and stores, four independent accesses per thread per iteration.
#include "common.h"

namespace dfh {

__global__ __launch_bounds__(256) void k_stream_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                     int64_t n) {
  // each workgroup copies one span of 1024 vectors (four per thread)
  const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  if (base + 768 < n) {
    const uint4 a = src[base], b = src[base + 256], c = src[base + 512], d = src[base + 768];
    dst[base] = a;
    dst[base + 256] = b;
    dst[base + 512] = c;
    dst[base + 768] = d;
  } else {
    for (int64_t i = base; i < n; i += 256) dst[i] = src[i];
  }
}

hipError_t launch_stream_copy(const void *src, void *dst, int64_t bytes, hipStream_t s) {
  const int64_t n = bytes / 16;
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 1023) / 1024;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, s, (const uint4 *)src, (uint4 *)dst, n);
  return hipGetLastError();
}

}  // namespace dfh
