// Measured matrix-core issue rate of the device (ensf_measure_mfma_rate): the attainable
// dense MFMA throughput under the card's own clock and power limits, against which the
// analysis kernels' issued throughput can be read beside the published peak.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ensf.h"
#include "ensf_internal.h"

namespace ensf {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;

constexpr int kBlocks = 2048, kThreads = 256, kChains = 8;

// Every wave runs `iters` rounds of kChains independent accumulator chains of the MFMA the
// analysis uses for the form (32x32x16 BF16 or 32x32x2 FP32); operands stay in registers.
template <int PREC>
__global__ __launch_bounds__(kThreads) void k_mfma_rate(float* out, int iters, float seed) {
  f32x16_t acc[kChains];
#pragma unroll
  for (int a = 0; a < kChains; ++a)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[a][r] = 0.0f;
  const float s = seed + (float)threadIdx.x * 1e-3f;
  bf16x8_t x, y;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    x[i] = (__bf16)(s + i);
    y[i] = (__bf16)(s - i);
  }
  const float fx = s, fy = 0.5f * s;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int a = 0; a < kChains; ++a) {
      if constexpr (PREC == kFP32)
        acc[a] = __builtin_amdgcn_mfma_f32_32x32x2f32(fx, fy, acc[a], 0, 0, 0);
      else
        acc[a] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, acc[a], 0, 0, 0);
    }
  }
  float t = 0.0f;
#pragma unroll
  for (int a = 0; a < kChains; ++a)
#pragma unroll
    for (int r = 0; r < 16; ++r) t += acc[a][r];
  out[(int64_t)blockIdx.x * kThreads + threadIdx.x] = t;
}

}  // namespace
}  // namespace ensf

extern "C" ensf_status ensf_measure_mfma_rate(int32_t precision, double* tflops, void* stream) {
  using namespace ensf;
  if (!tflops || (precision != ENSF_PREC_FP32 && precision != ENSF_PREC_BF16X3 &&
                  precision != ENSF_PREC_BF16))
    return ENSF_EINVAL;
  *tflops = 0.0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&out, (size_t)kBlocks * kThreads * sizeof(float));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // about 1 ms per launch at the published peaks; 20 warm-up launches bring the clocks to
  // their loaded state, then 100 back-to-back launches (about 0.1 s) are timed together, so
  // the rate is the sustained one, as the analysis (hundreds of milliseconds of dense MFMA
  // work) sees it
  const bool f32 = precision == ENSF_PREC_FP32;
  const int iters = f32 ? 500 : 1000;
  constexpr int kWarm = 20, kTimed = 100;
  const double flops = (double)kBlocks * (kThreads / 64) * iters * kChains *
                       (f32 ? 2.0 * 32 * 32 * 2 : 2.0 * 32 * 32 * 16);
  auto launch = [&]() {
    if (f32)
      hipLaunchKernelGGL(k_mfma_rate<kFP32>, dim3(kBlocks), dim3(kThreads), 0, s, out, iters, 1.0f);
    else
      hipLaunchKernelGGL(k_mfma_rate<kBF16>, dim3(kBlocks), dim3(kThreads), 0, s, out, iters, 1.0f);
    return hipGetLastError();
  };
  for (int rep = 0; rep < kWarm && e == hipSuccess; ++rep) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int rep = 0; rep < kTimed && e == hipSuccess; ++rep) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  const double rate = ms > 0.0f ? kTimed * flops / ((double)ms * 1e-3) / 1e12 : 0.0;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (out) (void)hipFree(out);
  if (e != hipSuccess) {
    record_hip_error(e);
    return ENSF_EHIP;
  }
  *tflops = rate;
  return ENSF_OK;
}
