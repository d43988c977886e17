/*
 * ensf_vit.h -- C ABI of the vision-transformer forecast surrogate in libensf.so.
 *
 * The paper's framework forecasts the analysis ensemble with a ViT surrogate of the
 * forecast model (Sec. III-B, Fig. `fig:arch`) and trains it online (Sec. I, Sec. V); its
 * Table II lists the sizes (64^2 input: patch 4, 12 layers, 8 heads, embedding 1024, MLP
 * ratio 4).  This library trains and runs such a model with its own HIP kernels:
 *
 *   tokens  h = patches W_pe^T + b_pe + pos       (p x p patches of the C x H x W state,
 *                                                  each flattened in (c, row, col) order)
 *   block   h = h + MHSA(LN1(h)) W_o^T + b_o,  h = h + GELU(LN2(h) W_1^T + b_1) W_2^T + b_2
 *           (pre-norm; softmax(q k^T / sqrt(dh)) per head; exact erf-GELU)
 *   output  y = x + unpatchify(LNf(h) W_h^T + b_h);  loss = mean((y - target)^2)
 *
 * LayerNorm uses the population variance and eps 1e-5.  Dropout and DropPath are not
 * applied.  Training is Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on FP32
 * master weights.
 *
 * Numerics: every matrix product (forward, input and weight gradients, attention) has BF16
 * operands and FP32 accumulation on MFMA; the residual stream, LayerNorm statistics, the
 * loss and the optimizer state are FP32; the GELU derivative at the MLP pre-activation is
 * kept for the backward pass in BF16.
 *
 * Parameters cross the ABI flat, float32, host memory, in this order: W_pe (D x P), b_pe (D),
 * pos (T x D); per layer ln1 gamma, beta (D), W_qkv (3D x D), b_qkv (3D), W_o (D x D),
 * b_o (D), ln2 gamma, beta (D), W_1 (F x D), b_1 (F), W_2 (D x F), b_2 (D); then lnf
 * gamma, beta (D), W_h (P x D), b_h (P).  Weights are (out, in): y = v W^T + b.
 * T = (H/p)(W/p) tokens, P = C p^2, D = embed, F = mlp_hidden.
 *
 * States are float32 NCHW (batch x C x H x W).  Pointers named d_* are device pointers owned
 * by the caller; calls are asynchronous on the given stream (hipStream_t as void*) unless
 * stated.  A surrogate must not be used by two threads at once.
 */
#ifndef ENSF_VIT_H
#define ENSF_VIT_H

#include <stdint.h>

#include "ensf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ensf_vit ensf_vit;

typedef struct {
  int32_t channels;     /* C */
  int32_t height;       /* H, a multiple of patch */
  int32_t width;        /* W, a multiple of patch */
  int32_t patch;        /* p; P = C p^2 must be a multiple of 32 */
  int32_t layers;       /* >= 1 */
  int32_t heads;        /* embed / heads (head size) a multiple of 32 */
  int32_t embed;        /* D: a multiple of 64, at most 2048 */
  int32_t mlp_hidden;   /* F: a multiple of 32 */
  int32_t max_batch;    /* states per call */
  int32_t device;       /* HIP device ordinal */
  uint64_t seed;        /* parameter initialisation */
} ensf_vit_config;

/* Creates the model with workspace for max_batch states.  T = (H/p)(W/p) must be a multiple
   of 64 and at most 1024.  Parameters are initialised from seed: N(0, 0.02) weights and
   positions (the head's scaled by 0.1), zero biases, unit LayerNorm gains.
   Errors: ENSF_EINVAL (shape constraints above), ENSF_ENOMEM, ENSF_EHIP. */
ensf_status ensf_vit_create(const ensf_vit_config* cfg, ensf_vit** out);

/* Number of parameters (the length of the flat parameter vector). */
int64_t ensf_vit_num_params(const ensf_vit* v);

/* Copies parameters in (host float32, ABI order); resets the Adam state.  Synchronous. */
ensf_status ensf_vit_set_params(ensf_vit* v, const float* h_params);

/* Copies the FP32 master parameters out (host float32, ABI order).  Synchronous. */
ensf_status ensf_vit_get_params(ensf_vit* v, float* h_params);

/* Inference: d_y = d_x + net(d_x) for `batch` states (in chunks of max_batch).  d_y must not
   overlap d_x. */
ensf_status ensf_vit_forward(ensf_vit* v, const float* d_x, float* d_y, int32_t batch,
                             void* stream);

/* Gradient of mean((x + net(x) - target)^2) over all outputs with respect to every
   parameter, written to d_grad (device float32, ABI order); the loss to *h_loss if not NULL
   (synchronises).  1 <= batch <= max_batch. */
ensf_status ensf_vit_grad(ensf_vit* v, const float* d_x, const float* d_target, int32_t batch,
                          float* d_grad, double* h_loss, void* stream);

/* One training step: the gradient as above, then Adam with learning rate lr (the step
   counter for the bias correction is kept by the model).  h_loss as above. */
ensf_status ensf_vit_train_step(ensf_vit* v, const float* d_x, const float* d_target,
                                int32_t batch, float lr, double* h_loss, void* stream);

/* Frees the model.  NULL is a no-op. */
ensf_status ensf_vit_destroy(ensf_vit* v);

#ifdef __cplusplus
}
#endif
#endif /* ENSF_VIT_H */
