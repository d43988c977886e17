// HIP kernels of the EnSF analysis step for CDNA4 (gfx950).
//
// Per pseudo-step k of the reverse-time SDE (eq. 7) three grouped launches run:
//   k_gram     G = Z X^T (particles x members), split-K over the state dimension with a
//              fixed-order (deterministic) reduction: the squared distances of eq. 12 are
//              |z|^2 - 2 alpha z.x + alpha^2 |x|^2 and only z.x needs a contraction.
//   k_softmax  logits (alpha G_ij - alpha^2 |x_j|^2 / 2) / beta^2 (the |z_i|^2 term is the
//              same for every j of a row and cancels in eq. 16), row max, exp, normalise.
//   k_wx       xhat = W X on MFMA, then in the same kernel the damped posterior score of
//              eq. 17 (prior score of eq. 15 plus h(t) times the likelihood score of the
//              Gaussian of eq. 5), Philox4x32-10 + Box-Muller noise, and the
//              Euler-Maruyama update of eq. 7, written back in place.
// A launch covers the tiles of every problem of a batch; a tile finds its problem by a
// binary search over the prefix array.
//
// Operands: FP32 form on v_mfma_f32_32x32x2_f32; split-BF16 form
// (hi = bf16(x), lo = bf16(x - hi), products hi*hi + hi*lo + lo*hi) and plain BF16 on
// v_mfma_f32_32x32x16_bf16, FP32 accumulation in both.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "ensf_internal.h"
#include "mfma_tile.h"

namespace ensf {


// ----------------------------------------------------------------------------------------
// small helpers

__device__ __forceinline__ int find_problem(const int32_t* pre, int np, int tile) {
  int lo = 0, hi = np;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= tile) lo = mid; else hi = mid;
  }
  return lo;
}


__device__ __forceinline__ double step_time(const ProbDev& P, int step) {
  if (step < 0) return P.t_score;
  const double dt = 1.0 / (double)P.K;
  return 1.0 - (double)step * dt;
}

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 multiplies with the
// Weyl key schedule.
struct Words4 { uint32_t w0, w1, w2, w3; };

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32 -> 64-bit product gives both halves (a single v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    // three-input XOR in one v_bitop3_b32 (truth table 0x96: odd number of set inputs)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

__device__ __forceinline__ float u24(uint32_t r) {
  return ((float)(r >> 8) + 0.5f) * 5.9604644775390625e-08f;  // 2^-24, exact
}

// Box-Muller (1958): one pair of standard normals from two uniforms.  The radius uses the
// hardware base-2 logarithm (ln u = ln 2 * log2 u) and square root; the angle 2 pi u is
// passed in revolutions to the hardware sine and cosine, which take revolutions.
__device__ __forceinline__ void box_muller(uint32_t ra, uint32_t rb, float& n0, float& n1) {
  const float rad = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u24(ra)));
  const float rev = u24(rb);
  n0 = rad * __builtin_amdgcn_cosf(rev);
  n1 = rad * __builtin_amdgcn_sinf(rev);
}

__device__ __forceinline__ f32x4 normals4(uint32_t quad, uint32_t particle, uint32_t step,
                                           const ProbDev& P) {
  const Words4 w = philox4x32_10(quad, particle, step, P.filter, P.seed_lo, P.seed_hi);
  float a, b, c, d;
  box_muller(w.w0, w.w1, a, b);
  box_muller(w.w2, w.w3, c, d);
  return f32x4{a, b, c, d};
}

__device__ __forceinline__ uint16_t bf16_bits(__bf16 h) { return __builtin_bit_cast(uint16_t, h); }

// RNE split of an FP32 value into bf16 hi and lo (x - hi is exact in FP32).
__device__ __forceinline__ void split_bf16(float x, uint16_t& hi, uint16_t& lo) {
  const __bf16 h = (__bf16)x;
  hi = bf16_bits(h);
  lo = bf16_bits((__bf16)(x - (float)h));
}

// Damped posterior score (eq. 17) of one component given xhat = sum_j w_j x_j.
// a_e = sum y / sigma_o^2 and b_e = count / sigma_o^2 of the component (eq. 5).
// The fused multiply-adds of the score and the update are written out and the compiler may
// fuse nothing else, so every kernel that inlines them computes the same bits.
template <int OP>
__device__ __forceinline__ float posterior_score(float z, float xh, float a_e, float b_e,
                                                 const StepScalars& sc) {
#pragma clang fp contract(off)
  const float prior = fmaf(sc.alpha, xh, -z) * sc.inv_beta2;
  const float lik = (OP == kArctan)
                        ? fmaf(-b_e, atanf(z), a_e) * __builtin_amdgcn_rcpf(fmaf(z, z, 1.0f))
                        : fmaf(-b_e, z, a_e);
  return fmaf(sc.h, lik, prior);
}

// One step of the reverse-time SDE (eq. 7), backward in t, with the posterior score of
// eq. 17 split into its prior part and its likelihood part L = (A - B g(z)) g'(z).
// Explicit (Euler-Maruyama):  z - (b z - sigma^2 prior) dt + sigma^2 h dt L + c xi.
// Linearly implicit likelihood: the L term is divided by 1 + sigma^2 h dt kappa with the
// Gauss-Newton curvature kappa = B g'(z)^2, which keeps the step stable when dt is not
// small against sigma_o^2; without observations (B = 0) both are the same step.
template <int OP, bool IMPLICIT>
__device__ __forceinline__ float update_step(float z, float xh, float a_e, float b_e, float xi,
                                             const StepScalars& sc) {
#pragma clang fp contract(off)
  const float prior = fmaf(sc.alpha, xh, -z) * sc.inv_beta2;
  const float gp = (OP == kArctan) ? __builtin_amdgcn_rcpf(fmaf(z, z, 1.0f)) : 1.0f;
  const float lik = (OP == kArctan) ? fmaf(-b_e, atanf(z), a_e) * gp : fmaf(-b_e, z, a_e);
  float w = sc.damp;
  if constexpr (IMPLICIT) w *= __builtin_amdgcn_rcpf(fmaf((sc.damp * b_e) * gp, gp, 1.0f));
  const float drift = fmaf(sc.b, z, -(sc.sigma2 * prior));   // b z - sigma^2 prior
  float out = fmaf(-drift, sc.dt, z);
  out = fmaf(w, lik, out);
  return fmaf(sc.cnoise, xi, out);
}

// ----------------------------------------------------------------------------------------
// Gram: part[s][i][j] = sum_{k in chunk s} Z[i][k] X[j][k]

template <int PREC, int WGM, int WGN, int TM, int TN, int BK, int ST>
struct GramShape {
  static constexpr int BM = WGM * TM * 32, BN = WGN * TN * 32;
  using S = TileSmem<PREC, BM, BN, BK, false>;
  static constexpr bool PP = ST == 2 && 2 * S::kBytes <= kPingPongBytes;
  static constexpr int kSmem = PP ? 2 * S::kBytes : S::kBytes;
};

// One logical Gram tile (particle block x member block x split-K chunk) of a grouped launch.
template <int PREC, int WGM, int WGN, int TM, int TN, int BK, int ST>
__device__ __forceinline__ void gram_tile(const GroupedLaunch& g, int step, int tile, char* smem) {
  constexpr int NT = 64 * WGM * WGN, BM = WGM * TM * 32, BN = WGN * TN * 32;
  using S = TileSmem<PREC, BM, BN, BK, false>;
  constexpr bool PP = GramShape<PREC, WGM, WGN, TM, TN, BK, ST>::PP;
  const int f = find_problem(g.pre, g.np, tile);
  const ProbDev& P = g.desc[f];
  if (step >= P.K) return;
  const int local = tile - g.pre[f];
  const int tn = local % P.gram_tn;
  const int rest = local / P.gram_tn;
  const int tm = rest % P.gram_tm;
  const int s = rest / P.gram_tm;
  const int64_t kbeg = (int64_t)s * P.kchunk;
  const int64_t kend = min(kbeg + P.kchunk, P.ldz);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;

  f32x16_t acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

  if constexpr (PREC == kFP32) {
    F32KmajLoad<BM, NT, BK> la;
    F32KmajLoad<BN, NT, BK> lb;
    la.init(P.Z, P.ldz, m0);
    lb.init(P.Xf, P.ldz, n0);
    tile_k_loop<PREC, WGM, WGN, TM, TN, BK, PP, false>(
        smem, kbeg, kend,
        [&](int64_t kb) {
          la.load(kb);
          lb.load(kb);
        },
        [&](char* st) {
          float* sA = reinterpret_cast<float*>(st);
          la.store_rows(sA);
          lb.store_rows(sA + S::kAFloats);
        },
        acc);
  } else {
    constexpr bool LO = PREC == kBF16X3;
    F32KmajLoad<BM, NT, BK> la;
    Bf16KmajLoad<BN, NT, LO, BK> lb;
    la.init(P.Z, P.ldz, m0);
    lb.init(P.Xh, P.Xl, P.ldz, n0);
    tile_k_loop<PREC, WGM, WGN, TM, TN, BK, PP, false>(
        smem, kbeg, kend,
        [&](int64_t kb) {
          la.load(kb);
          lb.load(kb);
        },
        [&](char* st) {
          uint16_t* sAh = reinterpret_cast<uint16_t*>(st);
          la.template store_split<LO>(sAh, sAh + S::kALo, S::LDH);
          lb.store(sAh + S::kBHi, sAh + S::kBLo, S::LDH);
        },
        acc);
  }

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int64_t ldn = P.ldn;
  float* out = P.part + (int64_t)s * P.Mp_pad * ldn +
               (m0 + wm * TM * 32 + (lane >> 5) * 4) * ldn + n0 + wn * TN * 32 + (lane & 31);
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r)
        gstore(out + (a * 32 + (r >> 2) * 8 + (r & 3)) * ldn + b * 32, acc[a][b][r]);
}

template <int PREC, int WGM, int WGN, int TM, int TN, int BK, int ST>
__global__ __launch_bounds__(64 * WGM * WGN) void k_gram(GroupedLaunch g, int step) {
  __shared__ __attribute__((aligned(16)))
      char smem[GramShape<PREC, WGM, WGN, TM, TN, BK, ST>::kSmem];
  gram_tile<PREC, WGM, WGN, TM, TN, BK, ST>(g, step, xcd_remap(blockIdx.x, g.total), smem);
}

// ----------------------------------------------------------------------------------------
// Row softmax of the logits (eq. 16), one workgroup of 256 per particle row.  The split-K
// partials are summed in FP64 in a fixed order (deterministic): thread groups take
// disjoint, strided sets of splits with float4 loads, and the groups are then added in
// group order.

__device__ __forceinline__ double block_reduce_max(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  v = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) v = fmax(v, red[w]);
  return v;
}

__device__ __forceinline__ double block_reduce_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  v = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) v += red[w];
  return v;
}

// One particle row of the grouped launch, 256 threads; sL holds ldn doubles, sG 1024, red 8.
template <int PREC>
__device__ __forceinline__ void softmax_row(const GroupedLaunch& g, int step, int row, double* sL,
                                            double* sG, double* red) {
  const int f = find_problem(g.pre, g.np, row);
  const ProbDev& P = g.desc[f];
  if (step >= P.K) return;
  const int64_t i = row - g.pre[f];
  const double t = step_time(P, step);
  const double alpha = 1.0 - t * (1.0 - P.eps);
  const double inv_beta2 = 1.0 / t;
  const int N = P.N;
  const int S = P.S;
  const int nq = P.ldn >> 2;                 // quads of the padded row
  const int64_t pstride = (int64_t)P.Mp_pad * P.ldn;
  const float* prow = P.part + i * P.ldn;
  const int tid = threadIdx.x;

  // Partials s0, s0 + ds, ... < S of quad q summed in that order (FP64); the loads are
  // issued eight at a time ahead of their additions, which keep the order.
  auto sum_quads = [&](int q, int s0, int ds, double& a0, double& a1, double& a2, double& a3) {
    const float* pq = prow + 4 * q;
    int s = s0;
    for (; s + 7 * ds < S; s += 8 * ds) {
      f32x4 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        v[u] = gload(reinterpret_cast<const f32x4*>(pq + (int64_t)(s + u * ds) * pstride));
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        a0 += v[u].x; a1 += v[u].y; a2 += v[u].z; a3 += v[u].w;
      }
    }
    for (; s < S; s += ds) {
      const f32x4 v = gload(reinterpret_cast<const f32x4*>(pq + (int64_t)s * pstride));
      a0 += v.x; a1 += v.y; a2 += v.z; a3 += v.w;
    }
  };
  if (nq >= 256) {
    for (int q = tid; q < nq; q += 256) {
      double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
      sum_quads(q, 0, 1, a0, a1, a2, a3);
      sL[4 * q + 0] = a0; sL[4 * q + 1] = a1; sL[4 * q + 2] = a2; sL[4 * q + 3] = a3;
    }
  } else {
    const int G = 256 / nq;                  // split groups
    const int grp = tid / nq, q = tid % nq;
    if (grp < G) {
      double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
      sum_quads(q, grp, G, a0, a1, a2, a3);
      double* o = sG + 4 * (grp * nq + q);
      o[0] = a0; o[1] = a1; o[2] = a2; o[3] = a3;
    }
    __syncthreads();
    for (int j = tid; j < 4 * nq; j += 256) {
      double a = 0;
      for (int gg = 0; gg < G; ++gg) a += sG[4 * gg * nq + j];
      sL[j] = a;
    }
  }
  __syncthreads();

  double mx = -INFINITY;
  for (int j = tid; j < N; j += 256) {
    const double L = (alpha * sL[j] - 0.5 * alpha * alpha * (double)P.xnorm[j]) * inv_beta2;
    sL[j] = L;
    mx = fmax(mx, L);
  }
  mx = block_reduce_max(mx, red);
  double sum = 0.0;
  for (int j = tid; j < N; j += 256) {
    const double e = (double)expf((float)(sL[j] - mx));
    sL[j] = e;
    sum += e;
  }
  sum = block_reduce_sum(sum, red);
  const double inv = 1.0 / sum;
  for (int j = tid; j < P.ldn; j += 256) {
    const float w = j < N ? (float)(sL[j] * inv) : 0.0f;
    if constexpr (PREC == kFP32) {
      P.W[i * P.ldn + j] = w;
    } else {
      uint16_t h, l;
      split_bf16(w, h, l);
      P.Wh[i * P.ldn + j] = h;
      P.Wl[i * P.ldn + j] = PREC == kBF16X3 ? l : (uint16_t)0;
    }
    if (P.weights_out != nullptr && j < N) P.weights_out[i * N + j] = w;
  }
  // degenerate-weight W.X: wave 0 lists the weights >= kSparseTau in member order (ballot and
  // prefix counts per 64 members); rows with more than kSparseMax are marked by the count
  if (P.sparse && tid < 64) {
    int cnt = 0;
    for (int j0 = 0; j0 < N; j0 += 64) {
      const int j = j0 + tid;
      const float w = j < N ? (float)(sL[j] * inv) : 0.0f;
      const bool keep = w >= kSparseTau;
      const uint64_t mask = __ballot(keep);
      const int pos = cnt + __popcll(mask & ((1ull << tid) - 1ull));
      if (keep && pos < kSparseMax) {
        P.sp_idx[i * kSparseMax + pos] = j;
        P.sp_w[i * kSparseMax + pos] = w;
      }
      cnt += __popcll(mask);
    }
    if (tid == 0) P.sp_cnt[i] = cnt;
  }
}

template <int PREC>
__global__ __launch_bounds__(256) void k_softmax(GroupedLaunch g, int step) {
  extern __shared__ double sL[];            // ldn logits of the row
  __shared__ double sG[256 * 4];            // per-group partial sums (4 components each)
  __shared__ double red[8];
  softmax_row<PREC>(g, step, blockIdx.x, sL, sG, red);
}

// ----------------------------------------------------------------------------------------
// W.X with the fused score / noise / Euler-Maruyama epilogue.
// The tile computes xhat^T: BE state components (MFMA rows) x BP particles (MFMA columns),
// contraction over the padded members.  In this orientation register group r/4 of a lane
// holds four consecutive components of one particle, i.e. exactly the four normals of one
// Philox counter, so the epilogue runs from the accumulators without any exchange.

// Sparse xhat of a W.X tile in the accumulator layout: for the lane's particle i and each of
// its component quads, the sum over the row's listed members j of w_ij x_j (FP32, member
// order), read from the caller's prior (n_members x dim, row stride dim).
template <int WGN, int TM, int TN>
__device__ __forceinline__ void wx_sparse_gather(const ProbDev& P, int64_t i0, int64_t e0,
                                                 f32x16_t (&acc)[TM][TN]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const float* X = P.X;
  const int64_t d = P.d;
  const bool vec = (d & 3) == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0;
#pragma unroll
  for (int b = 0; b < TN; ++b) {
    const int64_t i = i0 + wn * TN * 32 + b * 32 + (lane & 31);
    if (i >= P.Mp) continue;
    const int cnt = P.sp_cnt[i];
    for (int s = 0; s < cnt; ++s) {
      const int j = P.sp_idx[i * kSparseMax + s];
      const float w = P.sp_w[i * kSparseMax + s];
      const float* xrow = X + (int64_t)j * d;
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int gq = 0; gq < 4; ++gq) {
          const int64_t e = e0 + wm * TM * 32 + a * 32 + gq * 8 + (lane >> 5) * 4;
          f32x4 x = {0.0f, 0.0f, 0.0f, 0.0f};
          if (vec && e + 3 < d) {
            x = gload(reinterpret_cast<const f32x4*>(xrow + e));
          } else {
            if (e < d) x.x = xrow[e];
            if (e + 1 < d) x.y = xrow[e + 1];
            if (e + 2 < d) x.z = xrow[e + 2];
            if (e + 3 < d) x.w = xrow[e + 3];
          }
          acc[a][b][gq * 4 + 0] = fmaf(w, x.x, acc[a][b][gq * 4 + 0]);
          acc[a][b][gq * 4 + 1] = fmaf(w, x.y, acc[a][b][gq * 4 + 1]);
          acc[a][b][gq * 4 + 2] = fmaf(w, x.z, acc[a][b][gq * 4 + 2]);
          acc[a][b][gq * 4 + 3] = fmaf(w, x.w, acc[a][b][gq * 4 + 3]);
        }
    }
  }
}

// Epilogue state of one W.X tile: descriptor fields and step scalars in registers.
struct WxEpi {
  float* Z;
  const float* A;
  const float* B;
  float* score_out;
  int64_t d, ldz, Mp, i0, e0;
  StepScalars sc;
  int obs_op, step;
  bool implicit, active;
  uint32_t filt, k0, k1;
};

__device__ __forceinline__ WxEpi make_wx_epi(const ProbDev& P, int step, int64_t i0, int64_t e0,
                                             bool active) {
  WxEpi E;
  E.Z = P.Z;
  E.A = P.A;
  E.B = P.B;
  E.score_out = P.score_out;
  E.d = P.d;
  E.ldz = P.ldz;
  E.Mp = P.Mp;
  E.i0 = i0;
  E.e0 = e0;
  E.sc = P.steps[step < 0 ? P.K : step];
  E.obs_op = P.obs_op;
  E.step = step;
  E.implicit = P.lik_implicit != 0;
  E.active = active;
  E.filt = P.filter;
  E.k0 = P.seed_lo;
  E.k1 = P.seed_hi;
  return E;
}

// xhat for the four consecutive components e..e+3 of particle i (one Philox counter).  SCORE
// writes the posterior score; otherwise the particle components are advanced one step in
// place.
template <bool SCORE, int OP, bool IMPLICIT>
__device__ __forceinline__ void wx_epi_elems(const WxEpi& E, int64_t i, int64_t e, f32x4 xh,
                                             unsigned int& bad) {
  if (i >= E.Mp || e >= E.d) return;
  f32x4* zp = reinterpret_cast<f32x4*>(E.Z + i * E.ldz + e);
  const f32x4 z = gload(zp);
  const f32x4 av = gload(reinterpret_cast<const f32x4*>(E.A + e));
  const f32x4 bv = gload(reinterpret_cast<const f32x4*>(E.B + e));
  const int64_t rem = E.d - e;
  if constexpr (SCORE) {
    float* so = E.score_out + i * E.d + e;
    so[0] = posterior_score<OP>(z.x, xh.x, av.x, bv.x, E.sc);
    if (rem > 1) so[1] = posterior_score<OP>(z.y, xh.y, av.y, bv.y, E.sc);
    if (rem > 2) so[2] = posterior_score<OP>(z.z, xh.z, av.z, bv.z, E.sc);
    if (rem > 3) so[3] = posterior_score<OP>(z.w, xh.w, av.w, bv.w, E.sc);
  } else {
    const Words4 w =
        philox4x32_10((uint32_t)(e >> 2), (uint32_t)i, (uint32_t)E.step, E.filt, E.k0, E.k1);
    float n0, n1, n2, n3;
    box_muller(w.w0, w.w1, n0, n1);
    box_muller(w.w2, w.w3, n2, n3);
    f32x4 zn;
    zn.x = update_step<OP, IMPLICIT>(z.x, xh.x, av.x, bv.x, n0, E.sc);
    zn.y = update_step<OP, IMPLICIT>(z.y, xh.y, av.y, bv.y, n1, E.sc);
    zn.z = update_step<OP, IMPLICIT>(z.z, xh.z, av.z, bv.z, n2, E.sc);
    zn.w = update_step<OP, IMPLICIT>(z.w, xh.w, av.w, bv.w, n3, E.sc);
    if (rem < 4) {  // ragged tail: keep the padding at zero
      zn.w = 0.0f;
      if (rem < 3) zn.z = 0.0f;
      if (rem < 2) zn.y = 0.0f;
    }
    if (!isfinite(zn.x + zn.y + zn.z + zn.w))
      bad += !isfinite(zn.x) + !isfinite(zn.y) + !isfinite(zn.z) + !isfinite(zn.w);
    gstore(zp, zn);
  }
}

// Orders a wave's LDS accesses before the ones that follow, for data exchanged between its
// own lanes: no code motion across it (fence, wave barrier) and the wave's outstanding LDS
// operations complete first (s_waitcnt lgkmcnt(0)).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_wave_barrier();
}

// The epilogue of a W.X tile.  In the accumulator layout a lane holds, per 32 x 32 block, the
// component quads Q = 2 gq + lane / 32 of particle lane % 32, so a store instruction would
// write 32-byte pieces of 32 particle rows.  Each block is therefore passed through a
// wave-private 4 KB LDS region ([particle][component], 16-byte quads XOR-permuted by the
// particle row) and read back with lane l on particle row 8 r + l / 8 and quad l % 8: eight
// consecutive lanes then cover one 128-byte line of a particle row, so every Z, A and B access
// of the epilogue is a whole line.  The per-element arithmetic is unchanged.
template <int WGN, int TM, int TN, bool SCORE, int OP, bool IMPLICIT>
__device__ __forceinline__ void wx_epilogue(const WxEpi& E, const f32x16_t (&acc)[TM][TN],
                                            float* stage, unsigned int& bad) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  float* ws = stage + wave * 1024;
  const int pw = lane & 31, q = lane & 7;
#pragma unroll
  for (int b = 0; b < TN; ++b)
#pragma unroll
    for (int a = 0; a < TM; ++a) {
#pragma unroll
      for (int gq = 0; gq < 4; ++gq) {
        const int Q = 2 * gq + (lane >> 5);
        *reinterpret_cast<f32x4*>(ws + pw * 32 + ((Q ^ (pw & 7)) << 2)) =
            f32x4{acc[a][b][gq * 4 + 0], acc[a][b][gq * 4 + 1], acc[a][b][gq * 4 + 2],
                  acc[a][b][gq * 4 + 3]};
      }
      // the wave reads what its other lanes wrote: order the LDS accesses within the wave
      wave_lds_sync();
      f32x4 xq[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int pr = r * 8 + (lane >> 3);
        xq[r] = *reinterpret_cast<const f32x4*>(ws + pr * 32 + ((q ^ (pr & 7)) << 2));
      }
      wave_lds_sync();
      const int64_t e = E.e0 + wm * TM * 32 + a * 32 + 4 * q;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = E.i0 + wn * TN * 32 + b * 32 + r * 8 + (lane >> 3);
        wx_epi_elems<SCORE, OP, IMPLICIT>(E, i, e, xq[r], bad);
      }
    }
}

template <int PREC, int WGM, int WGN, int TM, int TN, int BK, int ST>
struct WxShape {
  static constexpr int NT = 64 * WGM * WGN, BE = WGM * TM * 32, BP = WGN * TN * 32;
  using S = TileSmem<PREC, BE, BP, BK, true>;
  static constexpr bool PP = ST == 2 && 2 * S::kBytes <= kPingPongBytes;
  // the epilogue stages one 32 x 32 FP32 block per wave through the operand buffer
  static constexpr int kStage = NT / 64 * 4096;
  static constexpr int kOps = PP ? 2 * S::kBytes : S::kBytes;
  static constexpr int kSmem = kOps > kStage ? kOps : kStage;
};

// One logical W.X tile (component block x particle block) of a grouped launch.
template <int PREC, int WGM, int WGN, int TM, int TN, int BK, int ST, bool SCORE, bool SP>
__device__ __forceinline__ void wx_tile(const GroupedLaunch& g, int step, int tile,
                                        unsigned long long* nonfinite, char* smem) {
  constexpr int NT = 64 * WGM * WGN, BE = WGM * TM * 32, BP = WGN * TN * 32;
  using S = TileSmem<PREC, BE, BP, BK, true>;
  constexpr bool PP = WxShape<PREC, WGM, WGN, TM, TN, BK, ST>::PP;
  const int f = find_problem(g.pre, g.np, tile);
  const ProbDev& P = g.desc[f];
  if (!SCORE && step >= P.K) return;
  const int local = tile - g.pre[f];
  const int tp = local % P.wx_tp;           // particle tile (fastest: tiles sharing X are adjacent)
  const int te = local / P.wx_tp;
  const int64_t e0 = (int64_t)te * BE, i0 = (int64_t)tp * BP;


  f32x16_t acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

  // degenerate-weight variant: when every particle row of the tile has at most kSparseMax
  // weights >= kSparseTau (listed by the softmax), xhat is gathered from those members of
  // the FP32 prior instead of the dense product (uniform decision per tile)
  bool sparse = false;
  if constexpr (!SCORE && SP) {
    if (P.sparse) {
      int over = 0;
      for (int t = threadIdx.x; t < BP; t += NT) {
        const int64_t i = i0 + t;
        over |= (i < P.Mp && P.sp_cnt[i] > kSparseMax);
      }
      sparse = !__syncthreads_or(over);
    }
  }
  if (sparse) {
    if constexpr (SP) wx_sparse_gather<WGN, TM, TN>(P, i0, e0, acc);
  } else if constexpr (PREC == kFP32) {
    F32NmajLoad<BE, NT, BK> la;   // X rows (members) x components, components contiguous
    F32KmajLoad<BP, NT, BK> lb;   // W particles x members, members contiguous
    la.init(P.Xf, P.ldz, e0);
    lb.init(P.W, P.ldn, i0);
    tile_k_loop<PREC, WGM, WGN, TM, TN, BK, PP, true>(
        smem, 0, P.ldn,
        [&](int64_t kb) {
          la.load(kb);
          lb.load(kb);
        },
        [&](char* st) {
          float* sA = reinterpret_cast<float*>(st);
          la.store(sA, S::LDF_A);
          lb.store_rows(sA + S::kAFloats);
        },
        acc);
  } else {
    constexpr bool LO = PREC == kBF16X3;
    Bf16KmajLoad<BE, NT, LO, BK> la;   // X^T components x members
    Bf16KmajLoad<BP, NT, LO, BK> lb;   // W particles x members
    la.init(P.XTh, P.XTl, P.ldn, e0);
    lb.init(P.Wh, P.Wl, P.ldn, i0);
    tile_k_loop<PREC, WGM, WGN, TM, TN, BK, PP, true>(
        smem, 0, P.ldn,
        [&](int64_t kb) {
          la.load(kb);
          lb.load(kb);
        },
        [&](char* st) {
          uint16_t* sAh = reinterpret_cast<uint16_t*>(st);
          la.store(sAh, sAh + S::kALo, S::LDH);
          lb.store(sAh + S::kBHi, sAh + S::kBLo, S::LDH);
        },
        acc);
  }

  const WxEpi E = make_wx_epi(P, step, i0, e0, true);
  unsigned int bad = 0;
  __syncthreads();   // every wave is done with the operand tiles before the staging reuses them
  float* stage = reinterpret_cast<float*>(smem);
  // one specialised epilogue per observation operator and time-stepping variant (uniform)
  auto epilogue = [&](auto op_tag, auto impl_tag) {
    constexpr int OP = decltype(op_tag)::value;
    constexpr bool IMPL = decltype(impl_tag)::value;
    wx_epilogue<WGN, TM, TN, SCORE, OP, IMPL>(E, acc, stage, bad);
  };
  using ArcT = std::integral_constant<int, kArctan>;
  using LinT = std::integral_constant<int, kLinear>;
  using Yes = std::true_type;
  using No = std::false_type;
  if (E.obs_op == kArctan) {
    if (E.implicit && !SCORE) epilogue(ArcT{}, Yes{}); else epilogue(ArcT{}, No{});
  } else {
    if (E.implicit && !SCORE) epilogue(LinT{}, Yes{}); else epilogue(LinT{}, No{});
  }
  if (!SCORE && bad) atomicAdd(nonfinite, (unsigned long long)bad);
}

template <int PREC, int WGM, int WGN, int TM, int TN, int BK, int ST, bool SCORE, bool SP = false>
__global__ __launch_bounds__(64 * WGM * WGN) void k_wx(GroupedLaunch g, int step,
                                                       unsigned long long* nonfinite) {
  __shared__ __attribute__((aligned(16)))
      char smem[WxShape<PREC, WGM, WGN, TM, TN, BK, ST>::kSmem];
  wx_tile<PREC, WGM, WGN, TM, TN, BK, ST, SCORE, SP>(g, step, xcd_remap(blockIdx.x, g.total),
                                                     nonfinite, smem);
}

// ----------------------------------------------------------------------------------------
// The whole pseudo-time loop in one cooperative launch, for problems too small to fill the
// device, where three graph nodes per pseudo-step cost more in launch latency than their
// work.  Every pseudo-step runs the Gram tiles, the softmax rows and the W.X tiles of the
// grouped launches, each strided over the grid with the same per-tile code as the separate
// kernels (hence bit-identical results), separated by grid-wide barriers.  Tile shapes:
// Gram 64 x 64 on four waves, W.X 128 components x 32 particles on four waves, k-step 32,
// one LDS stage.

// Grid-wide barrier number n (targets n * gridDim.x arrivals on a counter that starts at 0).
// The wait is bounded: after spin_limit polls the barrier gives up and raises *err, which the
// host reports, so every workgroup always finishes.
__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned target, unsigned* err,
                                             int spin_limit) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int it = 0;
    while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++it > spin_limit) {
        __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
  }
  __syncthreads();
}

template <int PREC>
using PersistGS = GramShape<PREC, 2, 2, 1, 1, 32, 1>;
template <int PREC>
using PersistWS = WxShape<PREC, 4, 1, 1, 1, 32, 1>;

template <int PREC>
__global__ __launch_bounds__(256) void k_persistent(PersistArgs a) {
  extern __shared__ __attribute__((aligned(16))) char psmem[];
  double* sL = reinterpret_cast<double*>(psmem);     // softmax: ldn logits, 1024 group sums,
  double* sG = sL + a.max_ldn;                       // 8 reduction slots
  double* red = sG + 1024;
  const unsigned G = gridDim.x;
  unsigned n = 0;
  for (int k = 0; k < a.kmax; ++k) {
    for (int t = blockIdx.x; t < a.gram.total; t += G) {
      gram_tile<PREC, 2, 2, 1, 1, 32, 1>(a.gram, k, t, psmem);
      __syncthreads();
    }
    grid_barrier(a.bar, (++n) * G, a.err, a.spin_limit);
    for (int r = blockIdx.x; r < a.rows.total; r += G) {
      softmax_row<PREC>(a.rows, k, r, sL, sG, red);
      __syncthreads();
    }
    grid_barrier(a.bar, (++n) * G, a.err, a.spin_limit);
    for (int t = blockIdx.x; t < a.wx.total; t += G) {
      wx_tile<PREC, 4, 1, 1, 1, 32, 1, false, false>(a.wx, k, t, a.nonfinite, psmem);
      __syncthreads();
    }
    grid_barrier(a.bar, (++n) * G, a.err, a.spin_limit);
  }
}

// ----------------------------------------------------------------------------------------
// One-off kernels of an analysis

// Member row j: |x_j|^2 (FP64 accumulation) and the padded FP32 or bf16 hi/lo copy.
template <int PREC>
__global__ __launch_bounds__(256) void k_prep_rows(ProbDev P) {
  __shared__ double red[8];
  const int64_t j = blockIdx.x;
  const float* x = P.X + j * P.d;
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < P.d; e += blockDim.x) {
    const float v = x[e];
    acc += (double)v * (double)v;
    if constexpr (PREC == kFP32) {
      P.Xf[j * P.ldz + e] = v;
    } else {
      uint16_t h, l;
      split_bf16(v, h, l);
      P.Xh[j * P.ldz + e] = h;
      P.Xl[j * P.ldz + e] = PREC == kBF16X3 ? l : (uint16_t)0;
    }
  }
  acc = block_reduce_sum(acc, red);
  if (threadIdx.x == 0) P.xnorm[j] = (float)acc;
}

// XT[e][j] = X[j][e] over the padded N_pad x ldz block (bf16 hi and lo).
__global__ __launch_bounds__(256) void k_transpose(ProbDev P) {
  __shared__ uint16_t th[64][66], tl[64][66];
  const int64_t e0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    th[r][tx] = P.Xh[(j0 + r) * P.ldz + e0 + tx];
    tl[r][tx] = P.Xl[(j0 + r) * P.ldz + e0 + tx];
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    P.XTh[(e0 + r) * P.ldn + j0 + tx] = th[tx][r];
    P.XTl[(e0 + r) * P.ldn + j0 + tx] = tl[tx][r];
  }
}

// Initial particles: N(0, I) at t = 1, Philox step word 0xFFFFFFFF.
__global__ void k_init_z(ProbDev P) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  const int64_t e = q * 4;
  if (e >= P.d) return;
  const f32x4 n = normals4((uint32_t)q, (uint32_t)i, 0xFFFFFFFFu, P);
  const int64_t rem = P.d - e;
  const f32x4 v = {n.x, rem > 1 ? n.y : 0.f, rem > 2 ? n.z : 0.f, rem > 3 ? n.w : 0.f};
  *reinterpret_cast<f32x4*>(P.Z + i * P.ldz + e) = v;
}

__global__ void k_load_z(ProbDev P) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (e < P.d) P.Z[i * P.ldz + e] = P.zin[i * P.d + e];
}

__global__ void k_store_post(ProbDev P) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (e < P.d) P.post[i * P.d + e] = P.Z[i * P.ldz + e];
}

// Spread relaxation toward the prior spread per component (ddof = 1 on both sides).
__global__ void k_relax(ProbDev P, double r) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P.d) return;
  double s = 0.0, s2 = 0.0;
  for (int64_t i = 0; i < P.Mp; ++i) s += P.Z[i * P.ldz + e];
  const double mean = s / P.Mp;
  for (int64_t i = 0; i < P.Mp; ++i) {
    const double v = P.Z[i * P.ldz + e] - mean;
    s2 += v * v;
  }
  const double sd_post = sqrt(s2 / (P.Mp - 1));
  double xs = 0.0, xs2 = 0.0;
  for (int64_t j = 0; j < P.N; ++j) xs += P.X[j * P.d + e];
  const double xmean = xs / P.N;
  for (int64_t j = 0; j < P.N; ++j) {
    const double v = P.X[j * P.d + e] - xmean;
    xs2 += v * v;
  }
  const double sd_prior = sqrt(xs2 / (P.N - 1));
  const double fac = sd_post > 0.0 ? 1.0 - r + r * sd_prior / sd_post : 1.0;
  for (int64_t i = 0; i < P.Mp; ++i) {
    float* zp = P.Z + i * P.ldz + e;
    *zp = (float)(mean + ((double)*zp - mean) * fac);
  }
}

__global__ void k_stats(const float* ens, int32_t n, int64_t d, float* mean, float* spread) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d) return;
  double s = 0.0, s2 = 0.0;
  for (int64_t i = 0; i < n; ++i) s += ens[i * d + e];
  const double m = s / n;
  for (int64_t i = 0; i < n; ++i) {
    const double v = ens[i * d + e] - m;
    s2 += v * v;
  }
  mean[e] = (float)m;
  spread[e] = (float)sqrt(s2 / (n - 1));
}

__global__ void k_rng_normal(uint32_t k0, uint32_t k1, uint32_t filter, uint32_t step,
                             uint32_t particle, int64_t n, float* out, uint32_t* raw) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q * 4 >= n) return;
  const Words4 w = philox4x32_10((uint32_t)q, particle, step, filter, k0, k1);
  if (raw != nullptr) {
    raw[q * 4 + 0] = w.w0;
    raw[q * 4 + 1] = w.w1;
    raw[q * 4 + 2] = w.w2;
    raw[q * 4 + 3] = w.w3;
  }
  float v[4];
  box_muller(w.w0, w.w1, v[0], v[1]);
  box_muller(w.w2, w.w3, v[2], v[3]);
  for (int c = 0; c < 4; ++c)
    if (q * 4 + c < n) out[q * 4 + c] = v[c];
}

// ----------------------------------------------------------------------------------------
// host launchers

namespace {
inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }
}

#define ENSF_GRAM_LAUNCH(PR, WGM, WGN, TM, TN, BKV, STV)                                     \
  hipLaunchKernelGGL((k_gram<PR, WGM, WGN, TM, TN, BKV, STV>), dim3(g.total),                \
                     dim3(64 * WGM * WGN), 0, s, g, step)
#define ENSF_GRAM_CASE(PR, C, WGM, WGN, TM, TN)                                              \
  if (prec == PR && cfg == C) {                                                              \
    if (bk == 64 && st == 2)                                                                 \
      ENSF_GRAM_LAUNCH(PR, WGM, WGN, TM, TN, 64, 2);                                         \
    else if (bk == 64)                                                                       \
      ENSF_GRAM_LAUNCH(PR, WGM, WGN, TM, TN, 64, 1);                                         \
    else if (st == 2)                                                                        \
      ENSF_GRAM_LAUNCH(PR, WGM, WGN, TM, TN, 32, 2);                                         \
    else                                                                                     \
      ENSF_GRAM_LAUNCH(PR, WGM, WGN, TM, TN, 32, 1);                                         \
    return hipGetLastError();                                                                \
  }

#define ENSF_GRAM_CASE32(PR, C, WGM, WGN, TM, TN)                                            \
  if (prec == PR && cfg == C) {                                                              \
    if (bk != 32) return hipErrorInvalidValue;                                               \
    if (st == 2)                                                                             \
      ENSF_GRAM_LAUNCH(PR, WGM, WGN, TM, TN, 32, 2);                                         \
    else                                                                                     \
      ENSF_GRAM_LAUNCH(PR, WGM, WGN, TM, TN, 32, 1);                                         \
    return hipGetLastError();                                                                \
  }

#define ENSF_GRAM_ALL(PR)                 \
  ENSF_GRAM_CASE(PR, kGram128, 2, 2, 2, 2) \
  ENSF_GRAM_CASE(PR, kGram64, 2, 2, 1, 1)  \
  ENSF_GRAM_CASE(PR, kGram32, 1, 1, 1, 1)  \
  ENSF_GRAM_CASE(PR, kGram256, 4, 2, 2, 2)    \
  ENSF_GRAM_CASE32(PR, kGram256x256, 2, 2, 4, 4) \
  ENSF_GRAM_CASE(PR, kGram256w, 2, 2, 4, 2)    \
  ENSF_GRAM_CASE(PR, kGram128e, 2, 4, 2, 1)

hipError_t launch_gram(int prec, int cfg, int bk, int st, const GroupedLaunch& g, int step,
                       hipStream_t s) {
  if (g.total <= 0) return hipSuccess;
  ENSF_GRAM_ALL(kFP32)
  ENSF_GRAM_ALL(kBF16X3)
  ENSF_GRAM_ALL(kBF16)
  return hipErrorInvalidValue;
}

#define ENSF_WX_LAUNCH(PR, WGM, WGN, TM, TN, BKV, STV, SC)                                   \
  hipLaunchKernelGGL((k_wx<PR, WGM, WGN, TM, TN, BKV, STV, SC>), dim3(g.total),              \
                     dim3(64 * WGM * WGN), 0, s, g, step, nonfinite)
#define ENSF_WX_CASE(PR, C, WGM, WGN, TM, TN)                                                \
  if (prec == PR && cfg == C) {                                                              \
    if (sparse && !score_mode)                                                               \
      hipLaunchKernelGGL((k_wx<PR, WGM, WGN, TM, TN, 32, 1, false, true>), dim3(g.total),    \
                         dim3(64 * WGM * WGN), 0, s, g, step, nonfinite);                    \
    else if (score_mode)                                                                     \
      ENSF_WX_LAUNCH(PR, WGM, WGN, TM, TN, 32, 2, true);                                     \
    else if (bk == 64 && st == 2)                                                            \
      ENSF_WX_LAUNCH(PR, WGM, WGN, TM, TN, 64, 2, false);                                    \
    else if (bk == 64)                                                                       \
      ENSF_WX_LAUNCH(PR, WGM, WGN, TM, TN, 64, 1, false);                                    \
    else if (st == 2)                                                                        \
      ENSF_WX_LAUNCH(PR, WGM, WGN, TM, TN, 32, 2, false);                                    \
    else                                                                                     \
      ENSF_WX_LAUNCH(PR, WGM, WGN, TM, TN, 32, 1, false);                                    \
    return hipGetLastError();                                                                \
  }

// (components x particles) per config: 128x128, 128x64, 128x32, 256x128, 128x256, then
// 256x128 and 128x256 on four waves with larger per-wave tiles, 128x128 on eight waves (two
// wave shapes)
#define ENSF_WX_ALL(PR)                     \
  ENSF_WX_CASE(PR, kWx128, 2, 2, 2, 2)      \
  ENSF_WX_CASE(PR, kWx64, 2, 2, 2, 1)       \
  ENSF_WX_CASE(PR, kWx32, 4, 1, 1, 1)       \
  ENSF_WX_CASE(PR, kWx256, 4, 2, 2, 2)      \
  ENSF_WX_CASE(PR, kWx128x256, 2, 4, 2, 2)  \
  ENSF_WX_CASE(PR, kWx256w, 2, 2, 4, 2)     \
  ENSF_WX_CASE(PR, kWx128x256w, 2, 2, 2, 4) \
  ENSF_WX_CASE(PR, kWx128e, 2, 4, 2, 1)     \
  ENSF_WX_CASE(PR, kWx128f, 4, 2, 1, 2)

hipError_t launch_wx(int prec, int cfg, int bk, int st, bool score_mode, bool sparse,
                     const GroupedLaunch& g, int step, unsigned long long* nonfinite,
                     hipStream_t s) {
  if (g.total <= 0) return hipSuccess;
  ENSF_WX_ALL(kFP32)
  ENSF_WX_ALL(kBF16X3)
  ENSF_WX_ALL(kBF16)
  return hipErrorInvalidValue;
}

hipError_t launch_softmax(int prec, const GroupedLaunch& g, int step, int max_ldn, hipStream_t s) {
  if (g.total <= 0) return hipSuccess;
  const size_t shm = (size_t)max_ldn * sizeof(double);
  if (prec == kFP32) {
    hipLaunchKernelGGL(k_softmax<kFP32>, dim3(g.total), dim3(256), shm, s, g, step);
  } else if (prec == kBF16X3) {
    hipLaunchKernelGGL(k_softmax<kBF16X3>, dim3(g.total), dim3(256), shm, s, g, step);
  } else {
    hipLaunchKernelGGL(k_softmax<kBF16>, dim3(g.total), dim3(256), shm, s, g, step);
  }
  return hipGetLastError();
}

bool persistent_tiles(int prec, int gram, int gram_bk, int gram_st, int wx, int wx_bk,
                      int wx_st) {
  return (prec == kFP32 || prec == kBF16X3) && gram == kGram64 && gram_bk == 32 &&
         gram_st == 1 && wx == kWx32 && wx_bk == 32 && wx_st == 1;
}

hipError_t launch_persistent(int prec, const PersistArgs& a, int max_blocks, hipStream_t s) {
  auto go = [&](const void* fn, size_t ops) -> hipError_t {
    const size_t shm = std::max(ops, (size_t)(a.max_ldn + 1024 + 8) * sizeof(double));
    hipError_t e = hipSuccess;
    if (shm > 64 * 1024)
      e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, shm)) != hipSuccess)
      return e;
    const int work = std::max({a.gram.total, a.rows.total, a.wx.total});
    const int blocks = std::min({work, per_cu * prop.multiProcessorCount, max_blocks});
    if (blocks < 1) return hipErrorInvalidConfiguration;
    PersistArgs arg = a;
    void* params[] = {&arg};
    return hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(256), params, (unsigned)shm, s);
  };
  if (prec == kFP32)
    return go(reinterpret_cast<const void*>(k_persistent<kFP32>),
              std::max(PersistGS<kFP32>::kSmem, PersistWS<kFP32>::kSmem));
  if (prec == kBF16X3)
    return go(reinterpret_cast<const void*>(k_persistent<kBF16X3>),
              std::max(PersistGS<kBF16X3>::kSmem, PersistWS<kBF16X3>::kSmem));
  return hipErrorInvalidValue;
}

hipError_t set_softmax_smem_limit(size_t bytes) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_softmax<kFP32>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_softmax<kBF16X3>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k_softmax<kBF16>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_prep_rows(int prec, const ProbDev& p, hipStream_t s) {
  if (prec == kFP32)
    hipLaunchKernelGGL(k_prep_rows<kFP32>, dim3(p.N), dim3(256), 0, s, p);
  else if (prec == kBF16X3)
    hipLaunchKernelGGL(k_prep_rows<kBF16X3>, dim3(p.N), dim3(256), 0, s, p);
  else
    hipLaunchKernelGGL(k_prep_rows<kBF16>, dim3(p.N), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_transpose(const ProbDev& p, hipStream_t s) {
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)(p.ldz / 64), (unsigned)(p.N_pad / 64)),
                     dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_init_z(const ProbDev& p, hipStream_t s) {
  hipLaunchKernelGGL(k_init_z, dim3(blocks_for((p.d + 3) / 4, 256), (unsigned)p.Mp), dim3(256),
                     0, s, p);
  return hipGetLastError();
}

hipError_t launch_load_z(const ProbDev& p, hipStream_t s) {
  hipLaunchKernelGGL(k_load_z, dim3(blocks_for(p.d, 256), (unsigned)p.Mp), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_store_post(const ProbDev& p, hipStream_t s) {
  hipLaunchKernelGGL(k_store_post, dim3(blocks_for(p.d, 256), (unsigned)p.Mp), dim3(256), 0, s,
                     p);
  return hipGetLastError();
}

hipError_t launch_relax(const ProbDev& p, double r, hipStream_t s) {
  hipLaunchKernelGGL(k_relax, dim3(blocks_for(p.d, 256)), dim3(256), 0, s, p, r);
  return hipGetLastError();
}

hipError_t launch_rng_normal(uint64_t seed, uint32_t filter, uint32_t step, uint32_t particle,
                             int64_t n, float* out, uint32_t* raw, hipStream_t s) {
  const int64_t nq = (n + 3) / 4;
  hipLaunchKernelGGL(k_rng_normal, dim3(blocks_for(nq, 256)), dim3(256), 0, s,
                     (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), filter, step,
                     particle, n, out, raw);
  return hipGetLastError();
}

hipError_t launch_stats(const float* ens, int32_t n, int64_t d, float* mean, float* spread,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_stats, dim3(blocks_for(d, 256)), dim3(256), 0, s, ens, n, d, mean, spread);
  return hipGetLastError();
}

}  // namespace ensf
