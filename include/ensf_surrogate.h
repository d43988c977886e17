/*
 * ensf_surrogate.h -- C ABI of the convolutional forecast surrogate in libensf.so.
 *
 * The paper's framework forecasts every analysis member with a model that may be
 * physics-based (its SQG model, Sec. II-B) or learned (its ViT surrogate, Sec. III-B), and
 * adapts the learned model to data.  This library provides a small learned forecast model
 * trained and run by its own HIP kernels:
 *
 *   y = x + net(x),  net = six 3x3 convolutions with periodic (circular) padding,
 *   channels C0 -> width -> ... -> width -> C0, erf-GELU between layers (erf evaluated to
 *   1.5e-7, below the BF16 rounding of the activations),
 *   trained on mean squared error with Adam (FP32 master weights).
 *
 * Numerics: every convolution (forward, input gradient, weight gradient) has BF16 weight and
 * activation operands and FP32 accumulation on MFMA; the GELU derivative at each hidden
 * pre-activation is kept for the backward pass in BF16; pre-activations inside a kernel,
 * the output, the loss, the gradient sums and the optimizer state are FP32.
 *
 * Layout: states are float32 NCHW (batch x C0 x H x W), i.e. one ensemble member of the
 * analysis is one C0 x H x W block (component e = c*H*W + y*W + x).  Parameters cross
 * the ABI in the order layer 0..L-1, each as weight (Cout, Cin, 3, 3) then bias (Cout),
 * float32, host memory.  W must be a multiple of 32.
 *
 * Pointers named d_* are device pointers owned by the caller.  Calls are asynchronous on
 * the given stream (hipStream_t as void*) unless stated.
 */
#ifndef ENSF_SURROGATE_H
#define ENSF_SURROGATE_H

#include <stdint.h>

#include "ensf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ensf_surrogate ensf_surrogate;

/* Creates a surrogate for C0-channel H x W states (C0 <= 32, width in {32, 64},
   layers >= 2, W a multiple of 32, max_batch * H * W < 2^31) with workspace for batches up
   to max_batch; parameters are initialised from `seed` (He-normal, last layer scaled by 0.1,
   zero biases).  device: HIP ordinal.  Errors: ENSF_EINVAL (shape constraints above, out
   NULL), ENSF_ENOMEM, ENSF_EHIP. */
ensf_status ensf_surrogate_create(int32_t c0, int32_t width, int32_t layers, int32_t h,
                                  int32_t w, int32_t max_batch, uint64_t seed, int32_t device,
                                  ensf_surrogate** out);

/* Number of parameters (weights and biases of all layers). */
int64_t ensf_surrogate_num_params(const ensf_surrogate* s);

/* Copies parameters in (host float32, ABI order above); resets the Adam state.  Synchronous. */
ensf_status ensf_surrogate_set_params(ensf_surrogate* s, const float* h_params);

/* Copies the FP32 master parameters out (host float32, ABI order).  Synchronous. */
ensf_status ensf_surrogate_get_params(ensf_surrogate* s, float* h_params);

/* Inference: d_y = d_x + net(d_x) for `batch` states (any batch >= 1; larger batches are
   processed in chunks of max_batch).  d_y may equal d_x. */
ensf_status ensf_surrogate_forward(ensf_surrogate* s, const float* d_x, float* d_y,
                                   int32_t batch, void* stream);

/* Gradient of the mean squared error mean((x + net(x) - target)^2) over all outputs with
   respect to every parameter, written to d_grad (device float32, ABI order), and the
   loss to *h_loss (synchronous).  batch <= max_batch. */
ensf_status ensf_surrogate_grad(ensf_surrogate* s, const float* d_x, const float* d_target,
                                int32_t batch, float* d_grad, double* h_loss, void* stream);

/* One training step: gradient as above, then Adam (beta1 0.9, beta2 0.999, eps 1e-8,
   learning rate lr, bias correction with the step counter kept by the surrogate).
   If h_loss is not NULL the call synchronises and returns the batch loss. */
ensf_status ensf_surrogate_train_step(ensf_surrogate* s, const float* d_x,
                                      const float* d_target, int32_t batch, float lr,
                                      double* h_loss, void* stream);

/* Frees the surrogate.  NULL is a no-op. */
ensf_status ensf_surrogate_destroy(ensf_surrogate* s);

#ifdef __cplusplus
}
#endif
#endif /* ENSF_SURROGATE_H */
