/*
 * ensf.h -- C ABI of the EnSF analysis library (libensf.so, MI355X / gfx950).
 *
 * The library runs the analysis (update) step of the ensemble score filter of
 * Sec. III-A of "A Scalable Real-Time Data Assimilation Framework for Predicting
 * Turbulent Atmosphere Dynamics" (arXiv 2407.12168) on one GPU:
 *
 *   particles Z start as N(0, I) at pseudo-time t = 1 (Sec. III-A-2) and follow the
 *   Euler-Maruyama discretisation of the reverse-time SDE (eq. 7)
 *       z <- z - (b(t) z - sigma^2(t) s(z, t)) dt + sqrt(sigma^2(t) dt) xi
 *   on a uniform grid t_k = 1 - k dt, dt = 1/K, k = 0 .. K-1, with the damped
 *   posterior score (eqs. 11, 17)
 *       s(z, t) = sum_j -(z - alpha_t x_j) / beta_t^2 * w_j(z)            (eq. 15)
 *               + h(t) * grad_z log p(y | z),
 *       w_j(z)  = softmax_j( -|z - alpha_t x_j|^2 / (2 beta_t^2) )         (eqs. 12, 16)
 *   over the forecast members x_j, schedule alpha_t = 1 - t (1 - eps), beta_t^2 = t,
 *   b = d log(alpha_t)/dt, sigma^2 = d(beta_t^2)/dt - 2 b beta_t^2 (eq. 9), h(t) = 1 - t,
 *   and the Gaussian likelihood of eqs. 2 and 5 with R = obs_sigma^2 I,
 *       log p(y | z) = -sum_m (y_m - g(z[idx_m]))^2 / (2 obs_sigma^2),
 *   g = arctan (ENSF_OBS_ARCTAN) or the identity (ENSF_OBS_LINEAR).  With
 *   ensf_options.lik_step = ENSF_LIK_IMPLICIT the likelihood part of the drift is
 *   advanced linearly implicitly instead (see ensf_lik_step).
 *
 * The noise xi and the initial particles come from Philox4x32-10 (key = seed,
 * counter = (element / 4, particle, step, filter_id), step = 0xFFFFFFFF for the
 * initial draw) and the Box-Muller transform; the four words of one counter give
 * the normals of elements 4q .. 4q+3 (pairs (w0, w1) and (w2, w3)), each word mapped
 * to u = ((w >> 8) + 0.5) * 2^-24.
 *
 * Conventions
 *   - Pointers named d_* are device pointers on the context's GPU, owned by the
 *     caller; the library owns only its context and workspace.  Matrices are
 *     row-major float32: the prior X is n_members x dim, particles n_particles x dim.
 *   - Calls are asynchronous on the given stream (a hipStream_t passed as void*;
 *     NULL is the default stream): they validate, enqueue and return.  A context
 *     must not be used by two threads at once.  Calls on one context run in call
 *     order on the device even when they name different streams: a call on another
 *     stream than the previous call's makes its stream wait for that call first (the
 *     context's workspace is shared by its calls).
 *   - Observations with the same index add (independent likelihood factors).  Their sums
 *     are formed exactly in 64-bit fixed point (each value rounded to within 2^-31 of
 *     the largest |y|), so results do not depend on the order of the observations or
 *     of the device's work: runs are bit-reproducible.
 *   - Argument errors return ENSF_EINVAL synchronously and enqueue nothing.
 *     Launch failures return ENSF_EHIP.  Observations with an index outside [0, dim)
 *     or a non-finite value are skipped on the device and reported by ensf_sync_status
 *     as ENSF_EINVAL;
 *     non-finite particle values are counted and reported there as ENSF_ENONFINITE.
 */
#ifndef ENSF_H
#define ENSF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ensf_ctx ensf_ctx;

typedef enum {
  ENSF_OK = 0,
  ENSF_EINVAL = 1,        /* bad argument (null pointer, size, aliasing, sigma <= 0) */
  ENSF_ENOMEM = 2,        /* device or pinned host allocation failed */
  ENSF_EHIP = 3,          /* HIP runtime or launch error */
  ENSF_ENONFINITE = 4,    /* a particle became NaN or Inf (from ensf_sync_status) */
  ENSF_EUNSUPPORTED = 5,  /* valid request that the library does not implement */
  ENSF_ESCRATCH = 6       /* ensf_analysis_noalloc: the problem needs more than the
                             ENSF_NOALLOC_SCRATCH_BYTES of the library's static buffer */
} ensf_status;

typedef enum {
  ENSF_PREC_FP32 = 0,     /* Gram and W.X on FP32 MFMA */
  ENSF_PREC_BF16X3 = 1,   /* split BF16: hi*hi + hi*lo + lo*hi on BF16 MFMA, FP32 accumulate */
  ENSF_PREC_BF16 = 2      /* plain BF16 operands (error studies only) */
} ensf_precision;

typedef enum { ENSF_OBS_ARCTAN = 0, ENSF_OBS_LINEAR = 1 } ensf_obs_op;

/* Time stepping of the reverse SDE (eq. 7) with the posterior score of eq. 17, whose
   likelihood part is L(z) = (A_e - B_e g(z)) g'(z) per component (g the observation
   operator, A_e = sum y / sigma_o^2, B_e = count / sigma_o^2):
   EXPLICIT  Euler-Maruyama, z <- z - (b z - sigma^2 s) dt + sqrt(sigma^2 dt) xi;
   IMPLICIT  the likelihood drift sigma^2 h dt L is divided by 1 + sigma^2 h dt B_e g'(z)^2
             (linearly implicit in its Gauss-Newton curvature).  The same step without
             observations; stable when dt is not small against sigma_o^2, where the explicit
             step is not (it needs K of order 1 / sigma_o^2). */
typedef enum { ENSF_LIK_EXPLICIT = 0, ENSF_LIK_IMPLICIT = 1 } ensf_lik_step;

typedef struct {
  int32_t precision;      /* ensf_precision */
  int32_t obs_op;         /* ensf_obs_op */
  double  eps_alpha;      /* schedule floor eps in alpha_t = 1 - t (1 - eps); default 0.05 */
  double  spread_relax;   /* r in [0, 1]: relax the analysis spread toward the prior
                             spread per component (Sec. IV-A); 0 = off */
  int32_t use_graph;      /* pseudo-time loop: 0 eager launches; 1 (default) and 3 one
                             captured hipGraph; 2 one cooperative launch that runs every
                             pseudo-step with grid-wide barriers between its phases, when the
                             tile table gives the Gram 64 x 64 / W.X 128 x 32 tiles with k-step
                             32 and one LDS stage (else the graph).  All give bit-identical
                             results; the graph is the faster on MI355X. */
  int32_t device;         /* HIP device ordinal the context lives on */
  const char* tune_cache; /* JSON tile-table path for the autotuner; NULL = $ENSF_TUNE_CACHE */
  int32_t lik_step;       /* ensf_lik_step; default EXPLICIT */
  int32_t wx_sparse;      /* 1: degenerate-weight W.X (variant, default 0): per pseudo-step,
                             W.X tiles whose particles all have at most 8 weights >= 2^-30
                             compute xhat (eq. 15, weights of eq. 16) = sum of those
                             weights times their members (FP32) instead of the dense product;
                             the weights below 2^-30 are dropped (error below
                             n_members * 2^-30 * max |x|); others run dense */
} ensf_options;

/* One analysis problem of a batched call; fields as in ensf_analysis. */
typedef struct {
  const float*   d_prior;     /* n_members x dim */
  int32_t        n_members;
  int64_t        dim;
  float*         d_post;      /* n_particles x dim, must not overlap d_prior */
  int32_t        n_particles;
  const int32_t* d_obs_idx;   /* n_obs indices into [0, dim); duplicates add */
  const float*   d_obs_val;   /* n_obs observed values */
  int64_t        n_obs;
  float          obs_sigma;   /* > 0 */
  int32_t        n_steps;     /* K >= 1 */
  uint64_t       seed;
  uint32_t       filter_id;
} ensf_problem;

/* Fills *opt with the defaults (FP32, arctan, eps 0.05, no relaxation, graphs on, device 0,
   explicit step, dense W.X). */
void ensf_default_options(ensf_options* opt);

/* Creates a context on opt->device (NULL opt = defaults).  *out receives the handle.
   Errors: ENSF_EINVAL (out NULL, bad enum), ENSF_EHIP (device), ENSF_ENOMEM. */
ensf_status ensf_create(const ensf_options* opt, ensf_ctx** out);

/* Analysis step (Sec. III-A-2, eqs. 7, 11-17): writes the n_particles analysis particles
   into d_post.  d_prior is read on every pseudo-step and must stay valid and unchanged
   until the stream reaches the end of this call.  n_obs = 0 runs without observations
   (d_obs_idx / d_obs_val may then be NULL); n_obs <= 2^31 - 1.  Limits: 1 <= n_members <= 16384,
   n_particles >= 1, dim >= 1, n_steps >= 1. */
ensf_status ensf_analysis(ensf_ctx* ctx,
                          const float* d_prior, int32_t n_members, int64_t dim,
                          float* d_post, int32_t n_particles,
                          const int32_t* d_obs_idx, const float* d_obs_val, int64_t n_obs,
                          float obs_sigma, int32_t n_steps, uint64_t seed, uint32_t filter_id,
                          void* stream);

/* Many independent analyses (uneven sizes, per-problem K) in one grouped launch per
   kernel phase and pseudo-step; problems with fewer steps idle once finished.
   probs is a host array of n_problems descriptors (copied before return). */
ensf_status ensf_analysis_batched(ensf_ctx* ctx, const ensf_problem* probs,
                                  int32_t n_problems, void* stream);

/* One evaluation of the damped posterior score (eq. 17) at pseudo-time t in (0, 1] for
   given particles d_z (n_particles x dim): writes d_score (n_particles x dim) and, if
   d_weights is not NULL, the weights of eq. 16 (n_particles x n_members). */
ensf_status ensf_score(ensf_ctx* ctx,
                       const float* d_prior, int32_t n_members, int64_t dim,
                       const float* d_z, int32_t n_particles,
                       const int32_t* d_obs_idx, const float* d_obs_val, int64_t n_obs,
                       float obs_sigma, double t, float* d_score, float* d_weights,
                       void* stream);

/* The filter's standard normals for one (seed, filter_id, step, particle) and elements
   0 .. n-1 (step 0xFFFFFFFF = the initial draw).  d_raw_words, if not NULL, receives the
   4 * ceil(n / 4) raw Philox words.  Stream-ordered; no context needed. */
ensf_status ensf_rng_normal(uint64_t seed, uint32_t filter_id, uint32_t step, uint32_t particle,
                            int64_t n, float* d_out, uint32_t* d_raw_words, void* stream);

/* Per-component mean and spread (std, ddof = 1) over the n rows of d_ens (n x dim):
   d_mean and d_spread are float32[dim].  n >= 2. */
ensf_status ensf_ensemble_stats(const float* d_ens, int32_t n, int64_t dim,
                                float* d_mean, float* d_spread, void* stream);

/* Waits for the last stream used by ctx (and so for every earlier call on ctx) and reports
   device-side conditions of the calls since the previous ensf_sync_status: ENSF_EINVAL for
   invalid observations (index outside [0, dim) or non-finite value), ENSF_ENONFINITE (with
   *nonfinite_count set) for NaN/Inf particles. */
ensf_status ensf_sync_status(ensf_ctx* ctx, int64_t* nonfinite_count);

/* Times candidate kernel variants on the given problem (running it several times on
   the stream; d_post is overwritten) and records the fastest in the context's table
   and, if set, the tune_cache file.  The search is coordinate-wise: Gram tile, split-K
   scale, k-step depth and LDS stage count with the W.X variant fixed, then the W.X tile,
   k-step depth and stage count, then the Gram side again.  Cache entries map a key
   "gfx950/p<precision>/n<log2 N>/m<log2 M_p>/d<log2 d>" to
   [gram tile, W.X tile, split scale, Gram k-step, W.X k-step, Gram stages, W.X stages].
   With the environment variable ENSF_TUNE_LOG set, each timed candidate is reported on
   stderr. */
ensf_status ensf_autotune(ensf_ctx* ctx, const ensf_problem* prob, void* stream);

/* The same for a batch (an array of n_problems host descriptors, as for
   ensf_analysis_batched): candidates are timed on the whole batch and recorded under a key
   made of the largest problem's buckets and the batch size ("gfx950/p<precision>/b<log2
   n_problems>/n../m../d.."), which is the only entry a batched call consults; a batch
   without one uses the built-in heuristic. */
ensf_status ensf_autotune_batched(ensf_ctx* ctx, const ensf_problem* probs, int32_t n_problems,
                                  void* stream);

/* Phase timing: with enable = 1 the context runs the pseudo-time loop eagerly and records
   HIP events on the call's stream around every kernel launch; ensf_phase_times then
   waits for them and returns the summed durations in milliseconds of the Gram, softmax
   and W.X/update kernels (ms[0..2]) and the number of launches of each (*count), since
   the last reset (ensf_profile_phases(ctx, 1) resets). */
ensf_status ensf_profile_phases(ensf_ctx* ctx, int32_t enable);
ensf_status ensf_phase_times(ensf_ctx* ctx, double* ms, int64_t* count);

/* Measures the attainable matrix-core rate of the current device for a form's MFMA
   (v_mfma_f32_32x32x2f32 for ENSF_PREC_FP32, v_mfma_f32_32x32x16_bf16 otherwise): 2048
   workgroups of four waves, each wave eight independent accumulator chains on register
   operands, timed with HIP events on the stream over 100 back-to-back launches (about 0.1 s)
   after 20 warm-up launches.  This is the throughput the card sustains under its own clock
   and power limits, the
   ceiling for the analysis kernels' issued MFMA work beside the published peak (Sec. IV-B
   reports the analysis against the hardware it ran on).  *tflops receives TFLOP/s (dense,
   2 flops per multiply-add).  Allocates and frees 2 MiB of device memory; synchronises the
   stream.  Errors: ENSF_EINVAL (tflops NULL, bad precision), ENSF_EHIP. */
ensf_status ensf_measure_mfma_rate(int32_t precision, double* tflops, void* stream);

/* Size in bytes of the device buffer behind ensf_analysis_noalloc: one statically allocated
   array in the library's device code, held by every GPU the entry point runs on until the
   process ends. */
#define ENSF_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (code being captured into a HIP graph,
   tight serving loops, harnesses that forbid hipMalloc): ensf_analysis without a context.
   Every buffer of the analysis (workspace, descriptor and step tables, counters) is carved
   out of the library's static scratch array of ENSF_NOALLOC_SCRATCH_BYTES on the current
   device of opt->device; nothing is allocated, no memset or host-to-device copy is enqueued
   (tables travel as kernel arguments, buffers are cleared by kernels), and the pseudo-time
   loop is launched eagerly on the stream.  opt gives precision, observation operator,
   likelihood step, eps, spread relaxation, degenerate-weight W.X and device (NULL = the
   defaults of ensf_default_options); use_graph and tune_cache are ignored: tiles come from
   the built-in heuristic, the choice a context makes without a tune table, so results are
   bit-identical to ensf_analysis on such a context.  Arguments as in ensf_analysis.
   d_counters: NULL, or a caller-owned device array of two uint64 to which the call adds the
   number of non-finite particle values ([0]) and of skipped invalid observations ([1]).
   Errors: ENSF_EINVAL (as ensf_analysis), ENSF_ESCRATCH if the problem needs more than the
   scratch size (synchronously, nothing enqueued), ENSF_EHIP.  All calls on one GPU share its
   scratch array, which keeps the last call's contents: calls that can overlap on one GPU
   (other streams, other threads) race and must be serialised by the caller.  The first call
   on each device looks the array up there (hipGetSymbolAddress). */
ensf_status ensf_analysis_noalloc(const ensf_options* opt,
                                  const float* d_prior, int32_t n_members, int64_t dim,
                                  float* d_post, int32_t n_particles,
                                  const int32_t* d_obs_idx, const float* d_obs_val,
                                  int64_t n_obs, float obs_sigma, int32_t n_steps,
                                  uint64_t seed, uint32_t filter_id,
                                  unsigned long long* d_counters, void* stream);

/* Frees the context and its workspace.  NULL is a no-op. */
ensf_status ensf_destroy(ensf_ctx* ctx);

const char* ensf_status_string(ensf_status s);

/* Text of the HIP error behind the calling thread's most recent ENSF_EHIP / ENSF_ENOMEM
   (from any entry point of this library), or "" if none. */
const char* ensf_last_error_string(void);

#ifdef __cplusplus
}
#endif
#endif /* ENSF_H */
