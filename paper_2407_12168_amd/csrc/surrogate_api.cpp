// Host side of the convolutional forecast surrogate: parameter layout, workspace,
// forward / backward orchestration and Adam.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "../../include/ensf_surrogate.h"
#include "ensf_internal.h"
#include "surrogate_internal.h"

using namespace ensf::sg;

namespace {

constexpr int kRows = 8;            // output rows per workgroup
constexpr int kChunkPixels = 2048;  // pixels per weight-gradient partial (one workgroup each)

inline int pad_ch(int c) { return c <= 32 ? 32 : 64; }

ensf_status hip_fail(hipError_t e) {
  ensf::record_hip_error(e);
  return e == hipErrorOutOfMemory ? ENSF_ENOMEM : ENSF_EHIP;
}

#define HIP_TRY(expr)                          \
  do {                                         \
    hipError_t _e = (expr);                    \
    if (_e != hipSuccess) return hip_fail(_e); \
  } while (0)

}  // namespace

struct ensf_surrogate {
  int c0 = 0, width = 0, L = 0, H = 0, W = 0, max_batch = 0, device = 0;
  std::vector<int> cin, cout, cinp, coutp;   // real and padded channels per layer
  std::vector<size_t> woff, boff;            // float offsets of weights / biases (GPU layout)
  std::vector<size_t> wkoff;                 // bf16 offsets of per-layer weight copies
  size_t nflat = 0, nbf = 0;
  float *d_param = nullptr, *d_grad = nullptr, *d_m = nullptr, *d_v = nullptr;
  uint16_t *d_wk = nullptr, *d_wf = nullptr;
  // activations: act[l] = input of layer l (NHWC bf16, cinp[l] channels); gd[l] = GELU' at
  // layer l's pre-activation (NHWC bf16, coutp[l]) for l < L-1, written by training forward
  // passes; du ping-pong buffers (NHWC bf16)
  std::vector<uint16_t*> act;
  std::vector<uint16_t*> gd;
  uint16_t *du0 = nullptr, *du1 = nullptr;
  float *y_tmp = nullptr, *wpart = nullptr, *bpart = nullptr, *loss_part = nullptr;
  double* d_loss = nullptr;
  int64_t step = 0;
};

namespace {

int64_t npix(const ensf_surrogate* s, int batch) { return (int64_t)batch * s->H * s->W; }
int loss_parts(const ensf_surrogate* s, int batch) { return batch * ((s->H + kRows - 1) / kRows); }
int chunks(const ensf_surrogate* s, int batch) {
  return (int)((npix(s, batch) + kChunkPixels - 1) / kChunkPixels);
}

void free_all(ensf_surrogate* s) {
  for (void* p : std::vector<void*>{s->d_param, s->d_grad, s->d_m, s->d_v, s->d_wk, s->d_wf,
                                    s->du0, s->du1, s->y_tmp, s->wpart, s->bpart, s->loss_part,
                                    s->d_loss})
    if (p) (void)hipFree(p);
  for (auto* p : s->act)
    if (p) (void)hipFree(p);
  for (auto* p : s->gd)
    if (p) (void)hipFree(p);
}

ensf_status refresh_bf16(ensf_surrogate* s, hipStream_t st) {
  for (int l = 0; l < s->L; ++l)
    HIP_TRY(launch_make_bf16_weights(s->d_param + s->woff[l], s->coutp[l], s->cinp[l],
                                     s->d_wk + s->wkoff[l], s->d_wf + s->wkoff[l], st));
  return ENSF_OK;
}

// GPU layout <-> ABI order (per layer: weight (Cout, Cin, 3, 3), bias (Cout))
void to_gpu_layout(const ensf_surrogate* s, const float* abi, std::vector<float>& flat) {
  flat.assign(s->nflat, 0.0f);
  size_t k = 0;
  for (int l = 0; l < s->L; ++l) {
    for (int co = 0; co < s->cout[l]; ++co)
      for (int ci = 0; ci < s->cin[l]; ++ci)
        for (int tap = 0; tap < 9; ++tap)
          flat[s->woff[l] + ((size_t)co * 9 + tap) * s->cinp[l] + ci] = abi[k++];
    for (int co = 0; co < s->cout[l]; ++co) flat[s->boff[l] + co] = abi[k++];
  }
}

void to_abi_order(const ensf_surrogate* s, const std::vector<float>& flat, float* abi) {
  size_t k = 0;
  for (int l = 0; l < s->L; ++l) {
    for (int co = 0; co < s->cout[l]; ++co)
      for (int ci = 0; ci < s->cin[l]; ++ci)
        for (int tap = 0; tap < 9; ++tap)
          abi[k++] = flat[s->woff[l] + ((size_t)co * 9 + tap) * s->cinp[l] + ci];
    for (int co = 0; co < s->cout[l]; ++co) abi[k++] = flat[s->boff[l] + co];
  }
}

// forward over one chunk of <= max_batch states; keep = store pre-activations (training)
ensf_status forward_chunk(ensf_surrogate* s, const float* d_x, float* d_y, int batch,
                          const float* d_target, hipStream_t st) {
  HIP_TRY(launch_pack_input(d_x, s->act[0], batch, s->c0, s->H, s->W, s->cinp[0], st));
  for (int l = 0; l < s->L; ++l) {
    ConvArgs a{};
    a.in = s->act[l];
    a.wk = s->d_wk + s->wkoff[l];
    a.bias = s->d_param + s->boff[l];
    a.batch = batch;
    a.H = s->H;
    a.W = s->W;
    a.rows = kRows;
    a.c0 = s->c0;
    if (l < s->L - 1) {
      a.gd_out = d_target ? s->gd[l] : nullptr;
      a.a_out = s->act[l + 1];
      HIP_TRY(launch_conv(s->cinp[l], s->coutp[l], 0, a, st));
    } else {
      a.x_res = d_x;
      a.y_out = d_y;
      if (d_target) {
        a.target = d_target;
        a.a_out = s->du0;
        a.loss_part = s->loss_part;
        a.grad_scale = (float)(2.0 / ((double)batch * s->c0 * s->H * s->W));
      }
      HIP_TRY(launch_conv(s->cinp[l], s->coutp[l], 1, a, st));
    }
  }
  return ENSF_OK;
}

// full gradient into s->d_grad (GPU layout) and the loss into s->d_loss
ensf_status gradient(ensf_surrogate* s, const float* d_x, const float* d_target, int batch,
                     hipStream_t st) {
  ensf_status rc = forward_chunk(s, d_x, s->y_tmp, batch, d_target, st);
  if (rc != ENSF_OK) return rc;
  HIP_TRY(launch_sum_loss(s->loss_part, loss_parts(s, batch),
                          1.0 / ((double)batch * s->c0 * s->H * s->W), s->d_loss, st));
  const int nch = chunks(s, batch);
  uint16_t* du = s->du0;
  uint16_t* du_next = s->du1;
  for (int l = s->L - 1; l >= 0; --l) {
    WgradArgs w{};
    w.du = du;
    w.in = s->act[l];
    w.part = s->wpart;
    w.batch = batch;
    w.H = s->H;
    w.W = s->W;
    w.chunk_pixels = kChunkPixels;
    HIP_TRY(launch_wgrad(s->cinp[l], s->coutp[l], w, nch, st));
    HIP_TRY(launch_reduce_wgrad(s->wpart, s->coutp[l], s->cinp[l], nch, s->d_grad + s->woff[l], st));
    HIP_TRY(launch_bias_grad(du, npix(s, batch), s->coutp[l], kChunkPixels, nch, s->bpart,
                             s->d_grad + s->boff[l], st));
    if (l > 0) {
      ConvArgs a{};
      a.in = du;
      a.wk = s->d_wf + s->wkoff[l];
      a.gd_prev = s->gd[l - 1];
      a.a_out = du_next;
      a.batch = batch;
      a.H = s->H;
      a.W = s->W;
      a.rows = kRows;
      a.c0 = s->c0;
      HIP_TRY(launch_conv(s->coutp[l], s->cinp[l], 2, a, st));
      std::swap(du, du_next);
    }
  }
  return ENSF_OK;
}

}  // namespace

extern "C" {

ensf_status ensf_surrogate_create(int32_t c0, int32_t width, int32_t layers, int32_t h,
                                  int32_t w, int32_t max_batch, uint64_t seed, int32_t device,
                                  ensf_surrogate** out) {
  if (!out) return ENSF_EINVAL;
  *out = nullptr;
  if (c0 < 1 || c0 > 32 || (width != 32 && width != 64) || layers < 2 || h < 1 || w < 32 ||
      w % 32 != 0 || max_batch < 1 || (int64_t)max_batch * h * w > INT32_MAX)
    return ENSF_EINVAL;
  if (conv_smem_bytes(64, 64, w, 1) + 1024 > 160 * 1024) return ENSF_EUNSUPPORTED;
  ensf::clear_stale_hip_error();
  HIP_TRY(hipSetDevice(device));
  ensf_surrogate* s = new ensf_surrogate();
  s->c0 = c0;
  s->width = width;
  s->L = layers;
  s->H = h;
  s->W = w;
  s->max_batch = max_batch;
  s->device = device;
  for (int l = 0; l < layers; ++l) {
    s->cin.push_back(l == 0 ? c0 : width);
    s->cout.push_back(l == layers - 1 ? c0 : width);
    s->cinp.push_back(pad_ch(s->cin.back()));
    s->coutp.push_back(pad_ch(s->cout.back()));
    s->woff.push_back(s->nflat);
    s->nflat += (size_t)9 * s->cinp.back() * s->coutp.back();
    s->boff.push_back(s->nflat);
    s->nflat += s->coutp.back();
    s->wkoff.push_back(s->nbf);
    s->nbf += (size_t)9 * s->cinp.back() * s->coutp.back();
  }
  auto fail = [&](hipError_t e) {
    free_all(s);
    delete s;
    return hip_fail(e);
  };
  const size_t F = s->nflat * sizeof(float);
  hipError_t e = hipSuccess;
  for (float** p : {&s->d_param, &s->d_grad, &s->d_m, &s->d_v})
    if (e == hipSuccess) e = hipMalloc(p, F);
  if (e == hipSuccess) e = hipMalloc(&s->d_wk, s->nbf * 2);
  if (e == hipSuccess) e = hipMalloc(&s->d_wf, s->nbf * 2);
  const int64_t P = npix(s, max_batch);
  s->act.assign(layers, nullptr);
  s->gd.assign(layers, nullptr);
  for (int l = 0; l < layers && e == hipSuccess; ++l) {
    e = hipMalloc(&s->act[l], (size_t)P * s->cinp[l] * 2);
    if (e == hipSuccess && l < layers - 1) e = hipMalloc(&s->gd[l], (size_t)P * s->coutp[l] * 2);
  }
  if (e == hipSuccess) e = hipMalloc(&s->du0, (size_t)P * 64 * 2);
  if (e == hipSuccess) e = hipMalloc(&s->du1, (size_t)P * 64 * 2);
  if (e == hipSuccess) e = hipMalloc(&s->y_tmp, (size_t)P * c0 * 4);
  if (e == hipSuccess)
    e = hipMalloc(&s->wpart, (size_t)chunks(s, max_batch) * 9 * 64 * 64 * 4);
  if (e == hipSuccess) e = hipMalloc(&s->bpart, (size_t)chunks(s, max_batch) * 64 * 4);
  if (e == hipSuccess) e = hipMalloc(&s->loss_part, (size_t)loss_parts(s, max_batch) * 4);
  if (e == hipSuccess) e = hipMalloc(&s->d_loss, sizeof(double));
  if (e == hipSuccess) e = hipMemset(s->d_grad, 0, F);
  if (e != hipSuccess) return fail(e);

  // He-normal initialisation (last layer scaled by 0.1), zero biases
  std::mt19937_64 gen(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<float> abi((size_t)ensf_surrogate_num_params(s));
  size_t k = 0;
  for (int l = 0; l < layers; ++l) {
    const double sd = std::sqrt(2.0 / (9.0 * s->cin[l])) * (l == layers - 1 ? 0.1 : 1.0);
    for (int i = 0; i < 9 * s->cin[l] * s->cout[l]; ++i) abi[k++] = (float)(sd * nd(gen));
    for (int i = 0; i < s->cout[l]; ++i) abi[k++] = 0.0f;
  }
  ensf_status st = ensf_surrogate_set_params(s, abi.data());
  if (st != ENSF_OK) {
    free_all(s);
    delete s;
    return st;
  }
  *out = s;
  return ENSF_OK;
}

int64_t ensf_surrogate_num_params(const ensf_surrogate* s) {
  if (!s) return 0;
  int64_t n = 0;
  for (int l = 0; l < s->L; ++l) n += 9LL * s->cin[l] * s->cout[l] + s->cout[l];
  return n;
}

ensf_status ensf_surrogate_set_params(ensf_surrogate* s, const float* h_params) {
  if (!s || !h_params) return ENSF_EINVAL;
  ensf::clear_stale_hip_error();
  HIP_TRY(hipSetDevice(s->device));
  std::vector<float> flat;
  to_gpu_layout(s, h_params, flat);
  HIP_TRY(hipMemcpy(s->d_param, flat.data(), s->nflat * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(s->d_m, 0, s->nflat * 4));
  HIP_TRY(hipMemset(s->d_v, 0, s->nflat * 4));
  s->step = 0;
  ensf_status st = refresh_bf16(s, nullptr);
  if (st != ENSF_OK) return st;
  HIP_TRY(hipDeviceSynchronize());
  return ENSF_OK;
}

ensf_status ensf_surrogate_get_params(ensf_surrogate* s, float* h_params) {
  if (!s || !h_params) return ENSF_EINVAL;
  ensf::clear_stale_hip_error();
  HIP_TRY(hipSetDevice(s->device));
  HIP_TRY(hipDeviceSynchronize());
  std::vector<float> flat(s->nflat);
  HIP_TRY(hipMemcpy(flat.data(), s->d_param, s->nflat * 4, hipMemcpyDeviceToHost));
  to_abi_order(s, flat, h_params);
  return ENSF_OK;
}

ensf_status ensf_surrogate_forward(ensf_surrogate* s, const float* d_x, float* d_y,
                                   int32_t batch, void* stream) {
  if (!s || !d_x || !d_y || batch < 1) return ENSF_EINVAL;
  ensf::clear_stale_hip_error();
  HIP_TRY(hipSetDevice(s->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t per = (int64_t)s->c0 * s->H * s->W;
  for (int b0 = 0; b0 < batch; b0 += s->max_batch) {
    const int nb = std::min(s->max_batch, batch - b0);
    ensf_status rc = forward_chunk(s, d_x + b0 * per, d_y + b0 * per, nb, nullptr, st);
    if (rc != ENSF_OK) return rc;
  }
  return ENSF_OK;
}

ensf_status ensf_surrogate_grad(ensf_surrogate* s, const float* d_x, const float* d_target,
                                int32_t batch, float* d_grad, double* h_loss, void* stream) {
  if (!s || !d_x || !d_target || !d_grad || batch < 1 || batch > s->max_batch) return ENSF_EINVAL;
  ensf::clear_stale_hip_error();
  HIP_TRY(hipSetDevice(s->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  ensf_status rc = gradient(s, d_x, d_target, batch, st);
  if (rc != ENSF_OK) return rc;
  HIP_TRY(hipStreamSynchronize(st));
  std::vector<float> flat(s->nflat), abi((size_t)ensf_surrogate_num_params(s));
  HIP_TRY(hipMemcpy(flat.data(), s->d_grad, s->nflat * 4, hipMemcpyDeviceToHost));
  to_abi_order(s, flat, abi.data());
  HIP_TRY(hipMemcpy(d_grad, abi.data(), abi.size() * 4, hipMemcpyHostToDevice));
  if (h_loss) HIP_TRY(hipMemcpy(h_loss, s->d_loss, sizeof(double), hipMemcpyDeviceToHost));
  return ENSF_OK;
}

ensf_status ensf_surrogate_train_step(ensf_surrogate* s, const float* d_x,
                                      const float* d_target, int32_t batch, float lr,
                                      double* h_loss, void* stream) {
  if (!s || !d_x || !d_target || batch < 1 || batch > s->max_batch || !(lr > 0.0f))
    return ENSF_EINVAL;
  ensf::clear_stale_hip_error();
  HIP_TRY(hipSetDevice(s->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  ensf_status rc = gradient(s, d_x, d_target, batch, st);
  if (rc != ENSF_OK) return rc;
  s->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  HIP_TRY(launch_adam(s->d_param, s->d_grad, s->d_m, s->d_v, (int64_t)s->nflat, lr, (float)b1,
                      (float)b2, 1e-8f, (float)(1.0 - std::pow(b1, (double)s->step)),
                      (float)(1.0 - std::pow(b2, (double)s->step)), st));
  rc = refresh_bf16(s, st);
  if (rc != ENSF_OK) return rc;
  if (h_loss) {
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipMemcpy(h_loss, s->d_loss, sizeof(double), hipMemcpyDeviceToHost));
  }
  return ENSF_OK;
}

ensf_status ensf_surrogate_destroy(ensf_surrogate* s) {
  if (!s) return ENSF_OK;
  (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();
  free_all(s);
  delete s;
  return ENSF_OK;
}

}  // extern "C"
