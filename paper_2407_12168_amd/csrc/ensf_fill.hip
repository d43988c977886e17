// Two small copy kernels of the host side: zero-fill of a device range, and a host-to-device
// copy of a few kilobytes carried in the kernel arguments.  Both replace hipMemsetAsync /
// hipMemcpyAsync where a caller may capture the enqueued work in a graph or may not own
// pinned host memory.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>

#include "ensf_run.h"

namespace ensf {

namespace {

constexpr int kPayloadWords = 512;   // 2 KiB of kernel arguments per copy launch

struct Payload {
  uint32_t w[kPayloadWords];
};

__global__ __launch_bounds__(256) void k_fill_zero(uint32_t* p, int64_t n_words) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n4 = n_words >> 2;
  if (i < n4) reinterpret_cast<uint4*>(p)[i] = make_uint4(0u, 0u, 0u, 0u);
  if (i < (n_words & 3)) p[4 * n4 + i] = 0u;
}

__global__ __launch_bounds__(kPayloadWords) void k_put_words(uint32_t* dst, int n_words,
                                                             Payload pl) {
  const int i = threadIdx.x;
  if (i < n_words) dst[i] = pl.w[i];
}

}  // namespace

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if ((reinterpret_cast<uintptr_t>(p) & 15) != 0 || (bytes & 3) != 0) return hipErrorInvalidValue;
  const int64_t n_words = (int64_t)(bytes / 4);
  const int64_t threads = ((n_words >> 2) > 3 ? (n_words >> 2) : 3);
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<uint32_t*>(p), n_words);
  return hipGetLastError();
}

hipError_t launch_put_bytes(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if ((reinterpret_cast<uintptr_t>(dst) & 3) != 0 || (bytes & 3) != 0) return hipErrorInvalidValue;
  const uint32_t* w = static_cast<const uint32_t*>(src);
  uint32_t* d = static_cast<uint32_t*>(dst);
  size_t left = bytes / 4;
  while (left > 0) {
    const int n = (int)(left < (size_t)kPayloadWords ? left : (size_t)kPayloadWords);
    Payload pl;
    std::memcpy(pl.w, w, (size_t)n * 4);
    hipLaunchKernelGGL(k_put_words, dim3(1), dim3(kPayloadWords), 0, s, d, n, pl);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    w += n;
    d += n;
    left -= (size_t)n;
  }
  return hipSuccess;
}

}  // namespace ensf
