// ensf_analysis_noalloc: the analysis in a statically allocated device buffer.
//
// `scratch` below is a file-scope device array.  In host code its name is only a host-side
// stand-in: the device address of each GPU's copy comes from hipGetSymbolAddress, looked up
// once per device (with that device current) on the first call there, and only that address
// is handed to kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/ensf.h"
#include "ensf_internal.h"
#include "ensf_run.h"

namespace {

static __device__ __align__(256) unsigned char scratch[ENSF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use).
hipError_t scratch_on(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

extern "C" ensf_status ensf_analysis_noalloc(const ensf_options* opt, const float* d_prior,
                                             int32_t n_members, int64_t dim, float* d_post,
                                             int32_t n_particles, const int32_t* d_obs_idx,
                                             const float* d_obs_val, int64_t n_obs,
                                             float obs_sigma, int32_t n_steps, uint64_t seed,
                                             uint32_t filter_id, unsigned long long* d_counters,
                                             void* stream) {
  ensf_options o;
  ensf_default_options(&o);
  if (opt) o = *opt;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) {
    ensf::record_hip_error(e != hipSuccess ? e : hipErrorNoDevice);
    return ENSF_EHIP;
  }
  if (o.device < 0 || o.device >= ndev || o.device >= kMaxDevices) return ENSF_EINVAL;
  const ensf_problem p{d_prior, n_members, dim, d_post, n_particles, d_obs_idx, d_obs_val,
                       n_obs, obs_sigma, n_steps, seed, filter_id};
  // size check first: an oversized problem is rejected before anything touches the device
  const size_t need = ensf::workspace_bytes(o, p);
  if (need == 0) return ENSF_EINVAL;
  if (need > ENSF_NOALLOC_SCRATCH_BYTES) return ENSF_ESCRATCH;
  e = hipSetDevice(o.device);
  void* ws = nullptr;
  if (e == hipSuccess) e = scratch_on(o.device, &ws);
  if (e != hipSuccess) {
    ensf::record_hip_error(e);
    return ENSF_EHIP;
  }
  return ensf::run_in_workspace(o, p, static_cast<char*>(ws), ENSF_NOALLOC_SCRATCH_BYTES,
                                d_counters, reinterpret_cast<hipStream_t>(stream));
}
