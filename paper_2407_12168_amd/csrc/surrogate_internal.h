// Internal interface between the surrogate's host code and its HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ensf {
namespace sg {

// Arguments of the implicit-GEMM convolution (k_conv).  MODE 0: hidden layer, writes
// a_out = bf16(GELU(u)) of the pre-activation u and, if gd_out is set (training), bf16(GELU'(u)).
// MODE 1: last layer, writes y_out = x_res + u (NCHW, c0 channels) and, when target is set,
// the loss partials and the bf16 output gradient grad_scale * (y - target) into a_out (NHWC).
// MODE 2: input gradient, a_out = bf16(acc * gd_prev).
struct ConvArgs {
  const uint16_t* in;       // NHWC bf16, CIN channels
  const uint16_t* wk;       // [COUT][9*CIN] bf16
  const float* bias;        // [COUT] or null
  uint16_t* gd_out;         // MODE 0, training: GELU' at the pre-activation (NHWC bf16)
  uint16_t* a_out;
  const uint16_t* gd_prev;  // MODE 2: the layer below's GELU' (NHWC bf16)
  const float* x_res;
  float* y_out;
  const float* target;
  float* loss_part;
  float grad_scale;
  int batch, H, W, rows, c0;
};

struct WgradArgs {
  const uint16_t* du;       // NHWC bf16, COUT channels
  const uint16_t* in;       // NHWC bf16, CIN channels
  float* part;              // [chunks][9][COUT][CIN]
  int batch, H, W, chunk_pixels;
};

// Dynamic LDS of the convolution kernel with rp output rows per step (rp = 2 where it fits).
size_t conv_smem_bytes(int cin, int cout, int W, int rp);
hipError_t launch_conv(int cin, int cout, int mode, const ConvArgs& a, hipStream_t s);
hipError_t launch_wgrad(int cin, int cout, const WgradArgs& a, int chunks, hipStream_t s);
hipError_t launch_pack_input(const float* x, uint16_t* a, int batch, int c0, int H, int W, int cp,
                             hipStream_t s);
hipError_t launch_bias_grad(const uint16_t* du, int64_t npix, int cout, int chunk_pixels,
                            int chunks, float* part, float* grad, hipStream_t s);
hipError_t launch_reduce_wgrad(const float* part, int cout, int cin, int chunks, float* grad,
                               hipStream_t s);
hipError_t launch_sum_loss(const float* part, int n, double scale, double* out, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                       float b1, float b2, float eps, float corr1, float corr2, hipStream_t s);
hipError_t launch_make_bf16_weights(const float* w, int cout, int cin, uint16_t* wk,
                                    uint16_t* wf, hipStream_t s);

}  // namespace sg
}  // namespace ensf
