// GPU SQG (nonlinear Eady) model, pseudo-spectral in FP64: hipFFT for the transforms,
// this file's kernels for the inversion, spectral derivatives, the advection product,
// dealiasing, RK4 bookkeeping and the exact hyperdiffusion factor.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cmath>
#include <map>

#include "../../include/ensf_sqg.h"
#include "ensf_internal.h"

namespace {

struct SqgParams {
  int n, nh, batch;
  double k1, shear, dt, efold, kcut, relax;
  int order;
};

__device__ __forceinline__ void wavenumbers(const SqgParams& p, int iy, int ix, double& kx,
                                            double& ky, bool& keep) {
  const int iys = iy < p.n / 2 ? iy : iy - p.n;
  kx = ix * p.k1;
  ky = iys * p.k1;
  keep = (fabs((double)iys) < p.n / 3.0) && ((double)ix < p.n / 3.0);   // 2/3 rule
}

// u, v, d/dx theta, d/dy theta of both levels (spectral, scaled by 1/n^2 for the inverse)
__global__ void k_sqg_derivs(SqgParams p, const double2* __restrict__ ts, double2* __restrict__ d4) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t plane = (int64_t)p.n * p.nh;
  if (idx >= (int64_t)p.batch * plane) return;
  const int64_t b = idx / plane, r = idx % plane;
  const int iy = (int)(r / p.nh), ix = (int)(r % p.nh);
  double kx, ky;
  bool keep;
  wavenumbers(p, iy, ix, kx, ky, keep);
  const double K = sqrt(kx * kx + ky * ky);
  const double it = K > 0 ? 1.0 / (K * tanh(K)) : 0.0;
  const double is = K > 0 ? 1.0 / (K * sinh(K)) : 0.0;
  const double2 t0 = ts[(b * 2 + 0) * plane + r], t1 = ts[(b * 2 + 1) * plane + r];
  const double sc = 1.0 / ((double)p.n * p.n);
  const double2 p0 = make_double2(-t0.x * it + t1.x * is, -t0.y * it + t1.y * is);
  const double2 p1 = make_double2(-t0.x * is + t1.x * it, -t0.y * is + t1.y * it);
  for (int L = 0; L < 2; ++L) {
    const double2 ps = L == 0 ? p0 : p1, th = L == 0 ? t0 : t1;
    double2 out[4];
    out[0] = make_double2(ky * ps.y * sc, -ky * ps.x * sc);    // u = -i ky psi
    out[1] = make_double2(-kx * ps.y * sc, kx * ps.x * sc);    // v = i kx psi
    out[2] = make_double2(-kx * th.y * sc, kx * th.x * sc);    // i kx theta
    out[3] = make_double2(-ky * th.y * sc, ky * th.x * sc);    // i ky theta
    for (int q = 0; q < 4; ++q) d4[(((int64_t)q * p.batch + b) * 2 + L) * plane + r] = out[q];
  }
}

// advective tendency on the grid: (U_i + u) d theta/dx + v (d theta/dy - shear)
__global__ void k_sqg_adv(SqgParams p, const double* __restrict__ r4, double* __restrict__ adv) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n2 = (int64_t)p.n * p.n;
  const int64_t per_q = (int64_t)p.batch * 2 * n2;
  if (idx >= per_q) return;
  const int L = (int)((idx / n2) % 2);
  const double U = L == 0 ? -0.5 * p.shear : 0.5 * p.shear;
  const double u = r4[idx], v = r4[per_q + idx], tx = r4[2 * per_q + idx], ty = r4[3 * per_q + idx];
  adv[idx] = (U + u) * tx + v * (ty - p.shear);
}

// RK4 stage bookkeeping with the dealiased tendency k = -mask * FFT(adv)
__global__ void k_sqg_stage(SqgParams p, const double2* __restrict__ advh, double2* __restrict__ th,
                            double2* __restrict__ ts, double2* __restrict__ kacc, int stage) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t plane = (int64_t)p.n * p.nh;
  if (idx >= (int64_t)p.batch * 2 * plane) return;
  const int64_t r = idx % plane;
  const int iy = (int)(r / p.nh), ix = (int)(r % p.nh);
  double kx, ky;
  bool keep;
  wavenumbers(p, iy, ix, kx, ky, keep);
  const double2 a = advh[idx];
  const double2 k = keep ? make_double2(-a.x, -a.y) : make_double2(0.0, 0.0);
  const double2 t = th[idx];
  if (stage == 0) {
    kacc[idx] = k;
    ts[idx] = make_double2(t.x + 0.5 * p.dt * k.x, t.y + 0.5 * p.dt * k.y);
  } else if (stage == 1 || stage == 2) {
    const double2 c = kacc[idx];
    kacc[idx] = make_double2(c.x + 2.0 * k.x, c.y + 2.0 * k.y);
    const double h = stage == 1 ? 0.5 * p.dt : p.dt;
    ts[idx] = make_double2(t.x + h * k.x, t.y + h * k.y);
  } else {
    const double2 c = kacc[idx];
    const double K = sqrt(kx * kx + ky * ky);
    const double diff = isinf(p.efold) ? 0.0 : p.dt / p.efold * pow(K / p.kcut, (double)p.order);
    const double hyper = exp(-diff) * exp(-p.dt / p.relax);
    const double2 nt = make_double2((t.x + p.dt / 6.0 * (c.x + k.x)) * hyper,
                                    (t.y + p.dt / 6.0 * (c.y + k.y)) * hyper);
    th[idx] = nt;
    ts[idx] = nt;
  }
}

// initial spectral state: masked forward transform
__global__ void k_sqg_mask_copy(SqgParams p, const double2* __restrict__ src, double2* __restrict__ th,
                                double2* __restrict__ ts) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t plane = (int64_t)p.n * p.nh;
  if (idx >= (int64_t)p.batch * 2 * plane) return;
  const int64_t r = idx % plane;
  double kx, ky;
  bool keep;
  wavenumbers(p, (int)(r / p.nh), (int)(r % p.nh), kx, ky, keep);
  const double2 v = keep ? src[idx] : make_double2(0.0, 0.0);
  th[idx] = v;
  ts[idx] = v;
}

template <typename T>
__global__ void k_to_double(const T* __restrict__ in, double* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)in[i];
}

template <typename T>
__global__ void k_from_double(const double* __restrict__ in, T* __restrict__ out, int64_t n,
                              double scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (T)(in[i] * scale);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

ensf_status fail(hipError_t e) {
  ensf::record_hip_error(e);
  return e == hipErrorOutOfMemory ? ENSF_ENOMEM : ENSF_EHIP;
}

#define HIP_TRY(expr)                         \
  do {                                        \
    hipError_t _e = (expr);                   \
    if (_e != hipSuccess) return fail(_e);    \
  } while (0)
#define FFT_TRY(expr)                                   \
  do {                                                  \
    if ((expr) != HIPFFT_SUCCESS) return ENSF_EHIP;     \
  } while (0)

}  // namespace

struct ensf_sqg {
  int n = 0, nh = 0, max_batch = 0, device = 0, order = 8;
  double lx = 20.0, shear = 1.0, dt = 0.025, efold = 0.25, relax = INFINITY;
  double2 *th = nullptr, *ts = nullptr, *kacc = nullptr, *d4 = nullptr, *advh = nullptr;
  double *r4 = nullptr, *adv = nullptr, *state = nullptr;
  std::map<int, hipfftHandle> z2d, d2z;   // plans keyed by the number of fields
};

namespace {

ensf_status plan_for(std::map<int, hipfftHandle>& cache, int n, int fields, hipfftType type,
                     hipfftHandle* out) {
  auto it = cache.find(fields);
  if (it != cache.end()) {
    *out = it->second;
    return ENSF_OK;
  }
  hipfftHandle h;
  int dims[2] = {n, n};
  FFT_TRY(hipfftPlanMany(&h, 2, dims, nullptr, 1, 0, nullptr, 1, 0, type, fields));
  cache[fields] = h;
  *out = h;
  return ENSF_OK;
}

SqgParams params(const ensf_sqg* s, int batch) {
  SqgParams p;
  p.n = s->n;
  p.nh = s->nh;
  p.batch = batch;
  p.k1 = 2.0 * M_PI / s->lx;
  p.shear = s->shear;
  p.dt = s->dt;
  p.efold = s->efold;
  p.kcut = 2.0 / 3.0 * p.k1 * (s->n / 2);
  p.order = s->order;
  p.relax = s->relax;
  return p;
}

// advances s->state (batch, 2, n, n) in place by n_steps
ensf_status run_chunk(ensf_sqg* s, int batch, int n_steps, hipStream_t st) {
  const SqgParams p = params(s, batch);
  const int64_t spec = (int64_t)batch * 2 * s->n * s->nh;
  hipfftHandle fwd2, inv2, inv8;
  ensf_status rc = plan_for(s->d2z, s->n, 2 * batch, HIPFFT_D2Z, &fwd2);
  if (rc == ENSF_OK) rc = plan_for(s->z2d, s->n, 2 * batch, HIPFFT_Z2D, &inv2);
  if (rc == ENSF_OK) rc = plan_for(s->z2d, s->n, 8 * batch, HIPFFT_Z2D, &inv8);
  if (rc != ENSF_OK) return rc;
  FFT_TRY(hipfftSetStream(fwd2, st));
  FFT_TRY(hipfftSetStream(inv2, st));
  FFT_TRY(hipfftSetStream(inv8, st));
  FFT_TRY(hipfftExecD2Z(fwd2, s->state, reinterpret_cast<hipfftDoubleComplex*>(s->advh)));
  hipLaunchKernelGGL(k_sqg_mask_copy, dim3(nblk(spec)), dim3(256), 0, st, p, s->advh, s->th, s->ts);
  HIP_TRY(hipGetLastError());
  const int64_t phys = (int64_t)batch * 2 * s->n * s->n;
  for (int step = 0; step < n_steps; ++step) {
    for (int stage = 0; stage < 4; ++stage) {
      hipLaunchKernelGGL(k_sqg_derivs, dim3(nblk((int64_t)batch * s->n * s->nh)), dim3(256), 0, st,
                         p, s->ts, s->d4);
      HIP_TRY(hipGetLastError());
      FFT_TRY(hipfftExecZ2D(inv8, reinterpret_cast<hipfftDoubleComplex*>(s->d4), s->r4));
      hipLaunchKernelGGL(k_sqg_adv, dim3(nblk(phys)), dim3(256), 0, st, p, s->r4, s->adv);
      HIP_TRY(hipGetLastError());
      FFT_TRY(hipfftExecD2Z(fwd2, s->adv, reinterpret_cast<hipfftDoubleComplex*>(s->advh)));
      hipLaunchKernelGGL(k_sqg_stage, dim3(nblk(spec)), dim3(256), 0, st, p, s->advh, s->th,
                         s->ts, s->kacc, stage);
      HIP_TRY(hipGetLastError());
    }
  }
  FFT_TRY(hipfftExecZ2D(inv2, reinterpret_cast<hipfftDoubleComplex*>(s->th), s->state));
  return ENSF_OK;
}

template <typename T>
ensf_status run_any(ensf_sqg* s, const T* d_in, T* d_out, int batch, int n_steps, void* stream) {
  if (!s || !d_in || !d_out || batch < 1 || n_steps < 0) return ENSF_EINVAL;
  ensf::clear_stale_hip_error();
  HIP_TRY(hipSetDevice(s->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t per = 2LL * s->n * s->n;
  const double inv = 1.0 / ((double)s->n * s->n);
  for (int b0 = 0; b0 < batch; b0 += s->max_batch) {
    const int nb = std::min(s->max_batch, batch - b0);
    hipLaunchKernelGGL(k_to_double<T>, dim3(nblk(nb * per)), dim3(256), 0, st, d_in + b0 * per,
                       s->state, nb * per);
    HIP_TRY(hipGetLastError());
    ensf_status rc = run_chunk(s, nb, n_steps, st);
    if (rc != ENSF_OK) return rc;
    hipLaunchKernelGGL(k_from_double<T>, dim3(nblk(nb * per)), dim3(256), 0, st, s->state,
                       d_out + b0 * per, nb * per, inv);
    HIP_TRY(hipGetLastError());
  }
  return ENSF_OK;
}

}  // namespace

extern "C" {

ensf_status ensf_sqg_create(int32_t n, double lx, double shear, double dt, int32_t diff_order,
                            double diff_efold, double relax_time, int32_t max_batch,
                            int32_t device, ensf_sqg** out) {
  if (!out) return ENSF_EINVAL;
  *out = nullptr;
  if (n < 8 || n % 2 || !(lx > 0) || !(dt > 0) || diff_order < 2 || !(diff_efold > 0) ||
      !(relax_time > 0) || max_batch < 1)
    return ENSF_EINVAL;
  ensf::clear_stale_hip_error();
  HIP_TRY(hipSetDevice(device));
  ensf_sqg* s = new ensf_sqg();
  s->n = n;
  s->nh = n / 2 + 1;
  s->lx = lx;
  s->shear = shear;
  s->dt = dt;
  s->order = diff_order;
  s->efold = diff_efold;
  s->relax = relax_time;
  s->max_batch = max_batch;
  s->device = device;
  const size_t spec = (size_t)max_batch * 2 * n * s->nh * sizeof(double2);
  const size_t phys = (size_t)max_batch * 2 * n * n * sizeof(double);
  hipError_t e = hipSuccess;
  for (double2** p : {&s->th, &s->ts, &s->kacc, &s->advh})
    if (e == hipSuccess) e = hipMalloc(p, spec);
  if (e == hipSuccess) e = hipMalloc(&s->d4, 4 * spec);
  if (e == hipSuccess) e = hipMalloc(&s->r4, 4 * phys);
  if (e == hipSuccess) e = hipMalloc(&s->adv, phys);
  if (e == hipSuccess) e = hipMalloc(&s->state, phys);
  if (e != hipSuccess) {
    ensf_sqg_destroy(s);
    return fail(e);
  }
  *out = s;
  return ENSF_OK;
}

ensf_status ensf_sqg_run(ensf_sqg* s, const double* d_in, double* d_out, int32_t batch,
                         int32_t n_steps, void* stream) {
  return run_any<double>(s, d_in, d_out, batch, n_steps, stream);
}

ensf_status ensf_sqg_run_f32(ensf_sqg* s, const float* d_in, float* d_out, int32_t batch,
                             int32_t n_steps, void* stream) {
  return run_any<float>(s, d_in, d_out, batch, n_steps, stream);
}

ensf_status ensf_sqg_destroy(ensf_sqg* s) {
  if (!s) return ENSF_OK;
  (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : s->z2d) (void)hipfftDestroy(kv.second);
  for (auto& kv : s->d2z) (void)hipfftDestroy(kv.second);
  for (void* p : {(void*)s->th, (void*)s->ts, (void*)s->kacc, (void*)s->advh, (void*)s->d4,
                  (void*)s->r4, (void*)s->adv, (void*)s->state})
    if (p) (void)hipFree(p);
  delete s;
  return ENSF_OK;
}

}  // extern "C"
