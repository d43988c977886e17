// Internal descriptors shared by the HIP kernels and the host side of libensf.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ensf {

enum Prec : int { kFP32 = 0, kBF16X3 = 1, kBF16 = 2 };
enum ObsOp : int { kArctan = 0, kLinear = 1 };

// Rows of the particle and member dimensions and the state dimension of every workspace
// matrix are padded to multiples of the chosen tile shapes (at least 64 and 128), so
// kernels never read outside an allocation; the padding is zero.
constexpr int kMaxMembers = 16384;
// Degenerate-weight W.X: a weight row counts as sparse when at most kSparseMax of its weights
// reach kSparseTau (= 2^-30); the smaller ones (at most N of them, below FP32 resolution of a
// unit-sum row) are dropped.
constexpr int kSparseMax = 8;
constexpr float kSparseTau = 9.313225746154785e-10f;

// One analysis problem as the kernels see it (device-resident table, one entry per
// problem of a batched call).
// Per-step scalars in FP32, computed on the host in FP64 from (t, eps) exactly as the oracle
// does and rounded once (a table per problem; the kernels read it with scalar loads).
struct StepScalars {
  float alpha, inv_beta2, b, sigma2, h, dt, cnoise;
  float damp;   // sigma^2 h dt: weight of the likelihood score in the update
};

struct ProbDev {
  // caller-owned
  const float* X;           // N x d prior
  float* post;              // Mp x d output
  const int32_t* obs_idx;
  const float* obs_val;
  const float* zin;         // score mode: given particles (Mp x d)
  float* score_out;         // score mode: score (Mp x d)
  float* weights_out;       // score mode: weights (Mp x N), may be null
  // workspace
  float* Z;                 // Mp_pad x ldz particles (zero padded)
  float* Xf;                // N_pad x ldz prior copy (FP32 form)
  uint16_t* Xh;             // N_pad x ldz  bf16 hi (split forms)
  uint16_t* Xl;             // N_pad x ldz  bf16 lo
  uint16_t* XTh;            // ldz x ldn    transposed hi
  uint16_t* XTl;            // ldz x ldn    transposed lo
  float* xnorm;             // ldn  |x_j|^2
  float* A;                 // ldz  sum y / sigma^2 per component
  float* B;                 // ldz  count / sigma^2 per component
  float* part;              // S x Mp_pad x ldn split-K Gram partials
  float* W;                 // Mp_pad x ldn softmax weights (FP32 form)
  uint16_t* Wh;             // Mp_pad x ldn (split forms)
  uint16_t* Wl;
  int64_t d, ldz, n_obs, kchunk;
  int32_t N, Mp, Mp_pad, N_pad, ldn, S, K;
  uint32_t seed_lo, seed_hi, filter;
  double inv_sig2_d;         // 1 / obs_sigma^2 (0 without observations)
  int32_t obs_op;
  int32_t lik_implicit;     // 1: linearly implicit likelihood drift in the update
  double eps, t_score;
  const StepScalars* steps;   // K + 1 entries: pseudo-steps 0..K-1, then the score time
  int32_t sparse;             // 1: W.X tiles whose weight rows are sparse gather instead
  int32_t* sp_cnt;            // Mp_pad  weights >= kSparseTau per row (written by the softmax)
  int32_t* sp_idx;            // Mp_pad x kSparseMax  their members, in member order
  float* sp_w;                // Mp_pad x kSparseMax  their weights
  long long* ob_acc;          // ldz + 1: fixed-point sums of y per component, then the
                              // float bits of the largest |y| (densification)
  int32_t gram_tm, gram_tn;   // Gram tiles along particles, members
  int32_t wx_tp, wx_te;       // W.X tiles along particles, state components
};


// Prefix arrays of a grouped launch: tiles of problem f are [pre[f], pre[f+1]).
struct GroupedLaunch {
  const ProbDev* desc;
  const int32_t* pre;
  int32_t np;
  int32_t total;
};

// Kernel-shape identifiers chosen by the host (heuristic or autotuner).
// Gram tiles: particles x members.
enum GramCfg : int {
  kGram128 = 0, kGram64 = 1, kGram32 = 2, kGram256 = 3,
  kGram256x256 = 4,   // 4 waves of 128 x 128
  kGram256w = 5,      // 256 x 128 on 4 waves of 128 x 64
  kGram128e = 6,      // 128 x 128 on 8 waves of 64 x 32
  kNumGram = 7
};
// W.X tiles: state components x particles.
enum WxCfg : int {
  kWx128 = 0, kWx64 = 1, kWx32 = 2, kWx256 = 3, kWx128x256 = 4,
  kWx256w = 5,        // 256 x 128 on 4 waves of 128 x 64
  kWx128x256w = 6,    // 128 x 256 on 4 waves of 64 x 128
  kWx128e = 7,        // 128 x 128 on 8 waves of 64 x 32 (fewer registers per wave)
  kWx128f = 8,        // 128 x 128 on 8 waves of 32 x 64
  kNumWx = 9
};

// kGram256 is 256 particles x 128 members; kWx256 is 256 components x 128 particles.
inline int gram_bm(int c) {
  return c == kGram256 || c == kGram256x256 || c == kGram256w ? 256
         : c == kGram128 || c == kGram128e                  ? 128
         : c == kGram64                                     ? 64
                                                            : 32;
}
inline int gram_bn(int c) {
  return c == kGram256x256 ? 256 : c == kGram256 || c == kGram256w ? 128 : gram_bm(c);
}
inline int wx_be(int c) { return c == kWx256 || c == kWx256w ? 256 : 128; }
inline int wx_bp(int c) {
  return c == kWx128x256 || c == kWx128x256w                     ? 256
         : c == kWx128 || c == kWx256 || c == kWx256w || c == kWx128e || c == kWx128f ? 128
         : c == kWx64                              ? 64
                                                   : 32;
}
// kGram256x256 exists with a k-step of 32 only (at 64 its split-BF16 form spills).
inline bool gram_variant_exists(int cfg, int bk) { return !(cfg == kGram256x256 && bk == 64); }
// k-step depths of the MFMA main loops are template variants (32 or 64); every padding
// is a multiple of the largest.  The LDS stage count (1, or 2 = ping-pong) is a variant too.
constexpr int kMaxBK = 64;

// Remembers the HIP error behind the calling thread's latest failed call
// (ensf_last_error_string) and clears HIP's sticky last-error state.
void record_hip_error(hipError_t e);
void clear_stale_hip_error();

// Host-callable launchers (ensf_kernels.hip).
hipError_t launch_gram(int prec, int cfg, int bk, int st, const GroupedLaunch& g, int step,
                       hipStream_t s);
hipError_t launch_softmax(int prec, const GroupedLaunch& g, int step, int max_ldn, hipStream_t s);
// sparse: the degenerate-weight variant of the W.X kernel (k-step 32, one LDS stage, whatever
// bk and st say), which gathers xhat for tiles whose weight rows are all sparse.
hipError_t launch_wx(int prec, int cfg, int bk, int st, bool score_mode, bool sparse,
                     const GroupedLaunch& g, int step, unsigned long long* nonfinite,
                     hipStream_t s);
// The pseudo-time loop of a grouped launch in one cooperative launch (ensf_kernels.hip).
struct PersistArgs {
  GroupedLaunch gram, rows, wx;
  int kmax, max_ldn;
  unsigned* bar;                    // barrier arrivals, zero before the launch
  unsigned* err;                    // set when a barrier wait gave up
  unsigned long long* nonfinite;
  int spin_limit;
};
// Tile variants the persistent kernel is built for: Gram kGram64, W.X kWx32, k-step 32, one
// LDS stage, FP32 or split BF16.
bool persistent_tiles(int prec, int gram, int gram_bk, int gram_st, int wx, int wx_bk, int wx_st);
// Launches it with at most max_blocks workgroups (all co-resident; cooperative launch).
hipError_t launch_persistent(int prec, const PersistArgs& a, int max_blocks, hipStream_t s);

// Observation densification (ensf_densify.hip): deterministic A and B, any duplicates.
hipError_t launch_densify(const ProbDev& p, unsigned long long* bad_obs, hipStream_t s);
hipError_t launch_prep_rows(int prec, const ProbDev& p, hipStream_t s);
hipError_t launch_transpose(const ProbDev& p, hipStream_t s);
hipError_t launch_init_z(const ProbDev& p, hipStream_t s);
hipError_t launch_load_z(const ProbDev& p, hipStream_t s);
hipError_t launch_store_post(const ProbDev& p, hipStream_t s);
hipError_t launch_relax(const ProbDev& p, double r, hipStream_t s);
hipError_t launch_rng_normal(uint64_t seed, uint32_t filter, uint32_t step, uint32_t particle,
                             int64_t n, float* out, uint32_t* raw, hipStream_t s);
hipError_t launch_stats(const float* ens, int32_t n, int64_t d, float* mean, float* spread,
                        hipStream_t s);

}  // namespace ensf
