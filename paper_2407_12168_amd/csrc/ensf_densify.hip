// Observation densification (eqs. 2 and 5), deterministic for any order of the
// observations and any number of duplicates:
//   A[e] = sum_{m : idx_m = e} y_m / sigma_o^2,   B[e] = #{m : idx_m = e} / sigma_o^2.
// The sums of y are formed exactly in 64-bit fixed point with integer atomics (integer
// addition is associative, so the result does not depend on the order in which the device
// adds the terms), then scaled by 1 / sigma_o^2 in FP64 and rounded once to FP32.
//
// Fixed-point scale: with |y_m| < 2^E for every observation (E from the largest |y|, found
// with an integer atomic max on the float bits) and n_obs <= 2^L, the scale 2^s with
// s = 62 - L - E keeps every partial sum below 2^62 in magnitude; each term is rounded to
// a multiple of 2^-s, i.e. to about 2^-(62 - L) of the largest |y|.
//
// Indices outside [0, d) and non-finite values are counted (reported as bad observations)
// and skipped.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ensf_internal.h"

namespace ensf {

namespace {

__device__ __forceinline__ bool obs_ok(int64_t e, float y, int64_t d) {
  return e >= 0 && e < d && isfinite(y);
}

// Pass 1: largest |y| over the valid observations (float bits of non-negative finite values
// order like the unsigned integers), and the count of invalid ones.
__global__ void k_obs_max(const int32_t* idx, const float* val, int64_t n_obs, int64_t d,
                          unsigned long long* maxbits, unsigned long long* bad_obs) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_obs) return;
  const int64_t e = idx[m];
  const float y = val[m];
  if (!obs_ok(e, y, d)) {
    atomicAdd(bad_obs, 1ull);
    return;
  }
  atomicMax(maxbits, (unsigned long long)__float_as_uint(fabsf(y)));
}

// Scale exponent s of the fixed point (see the file comment); 0 when every |y| is 0.
__device__ __forceinline__ int obs_scale(unsigned long long maxbits, int log2_n) {
  const float mx = __uint_as_float((uint32_t)maxbits);
  if (!(mx > 0.0f)) return 0;
  int E;
  (void)frexpf(mx, &E);          // mx = f 2^E, f in [0.5, 1): every |y| < 2^E
  return 62 - log2_n - E;
}

// Pass 2: exact fixed-point sums and counts per component.
__global__ void k_obs_accumulate(const int32_t* idx, const float* val, int64_t n_obs, int64_t d,
                                 int log2_n, const unsigned long long* maxbits,
                                 long long* acc, int32_t* cnt) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_obs) return;
  const int64_t e = idx[m];
  const float y = val[m];
  if (!obs_ok(e, y, d)) return;
  const int s = obs_scale(*maxbits, log2_n);
  atomicAdd(reinterpret_cast<unsigned long long*>(acc + e),
            (unsigned long long)llrint(ldexp((double)y, s)));
  atomicAdd(cnt + e, 1);
}

// Pass 3: A and B per component.  cnt aliases B (an int32 count read and replaced by the
// same thread).
__global__ void k_obs_finish(const long long* acc, int64_t d, int log2_n,
                             const unsigned long long* maxbits, double inv_sig2, float* A,
                             float* B) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d) return;
  const int32_t c = reinterpret_cast<const int32_t*>(B)[e];
  if (c == 0) return;                      // A and B stay 0
  const int s = obs_scale(*maxbits, log2_n);
  A[e] = (float)(ldexp((double)acc[e], -s) * inv_sig2);
  B[e] = (float)((double)c * inv_sig2);
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

int ceil_log2(int64_t n) {
  int l = 0;
  while ((int64_t(1) << l) < n) ++l;
  return l;
}

}  // namespace

// A and B must be zero and ob_acc (ldz + 1 entries) too when this is enqueued.
hipError_t launch_densify(const ProbDev& p, unsigned long long* bad_obs, hipStream_t s) {
  if (p.n_obs <= 0) return hipSuccess;
  const int l = ceil_log2(p.n_obs);
  unsigned long long* maxbits = reinterpret_cast<unsigned long long*>(p.ob_acc + p.ldz);
  int32_t* cnt = reinterpret_cast<int32_t*>(p.B);
  hipLaunchKernelGGL(k_obs_max, dim3(blocks_for(p.n_obs, 256)), dim3(256), 0, s, p.obs_idx,
                     p.obs_val, p.n_obs, p.d, maxbits, bad_obs);
  hipLaunchKernelGGL(k_obs_accumulate, dim3(blocks_for(p.n_obs, 256)), dim3(256), 0, s,
                     p.obs_idx, p.obs_val, p.n_obs, p.d, l, maxbits, p.ob_acc, cnt);
  hipLaunchKernelGGL(k_obs_finish, dim3(blocks_for(p.d, 256)), dim3(256), 0, s, p.ob_acc, p.d, l,
                     maxbits, p.inv_sig2_d, p.A, p.B);
  return hipGetLastError();
}

}  // namespace ensf
