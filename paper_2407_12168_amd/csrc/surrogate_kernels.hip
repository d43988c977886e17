// HIP kernels of the convolutional forecast surrogate (gfx950).
//
// Activations are NHWC bf16 with the channel count padded to CP in {32, 64} (padding is
// zero and stays zero: padded weights and biases are zero).  A 3x3 convolution with
// periodic padding is an implicit GEMM: M = pixels, N = output channels, K = 9 taps x
// input channels.  One workgroup owns one image and a band of output rows and computes RP
// rows per step on 4 * RP waves (RP = 2 where LDS allows); it keeps all weights and a ring of
// RP + 2 input rows (with a one-pixel periodic halo) in LDS, so each output row costs one new
// input row from memory, fetched during the previous step.  Wave w computes 32-pixel groups
// w % 4, + 4, ... of its row against all output channels with v_mfma_f32_32x32x16_bf16
// (FP32 accumulation).
//
// The input-gradient convolution is the same kernel run on the output gradient with the
// taps flipped and the weight matrix transposed.  The weight gradient contracts over
// pixels, which are strided in NHWC, so it stages BF16 tiles channel-major in LDS and uses
// v_mfma_f32_32x32x16_bf16; per-chunk partials are reduced in a fixed order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "surrogate_internal.h"

namespace ensf {
namespace sg {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float x) {
  return __builtin_bit_cast(uint16_t, (__bf16)x);
}
__device__ __forceinline__ float from_bf16(uint16_t h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// GELU(u) = u Phi(u) and its derivative Phi(u) + u phi(u) from one exponential.  The normal
// tail 1 - Phi(|u|) = erfc(|u| / sqrt 2) / 2 is taken from the rational form of
// Abramowitz & Stegun 7.1.26, erfc(x) = (a1 t + ... + a5 t^5) exp(-x^2) with t = 1 / (1 + p x)
// (|error| <= 1.5e-7), whose factor exp(-x^2) = exp(-u^2 / 2) is also sqrt(2 pi) phi(u); the
// exponential and the reciprocal are the hardware's.  Both results are rounded to BF16 by
// their users, far coarser than these errors.
struct GeluPair {
  float g, d;   // GELU(u), GELU'(u)
};
__device__ __forceinline__ GeluPair gelu_pair(float u) {
  const float e = __builtin_amdgcn_exp2f(-0.72134752044448170f * (u * u));  // exp(-u^2 / 2)
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * 0.70710678118654752f * fabsf(u));
  const float poly =
      t * (0.254829592f +
           t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
  const float tail = 0.5f * poly * e;               // 1 - Phi(|u|)
  const float cdf = u >= 0.0f ? 1.0f - tail : tail;
  return {u * cdf, cdf + u * (0.3989422804014327f * e)};
}

__device__ __forceinline__ int wrap(int v, int n) { return ((v % n) + n) % n; }

// NCHW float32 (c0 channels) -> NHWC bf16 with CP channels (zero padded).
__global__ void k_pack_input(const float* __restrict__ x, uint16_t* __restrict__ a, int batch,
                             int c0, int H, int W, int CP) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t npix = (int64_t)batch * H * W;
  if (p >= npix) return;
  const int64_t b = p / ((int64_t)H * W), yx = p % ((int64_t)H * W);
  // eight channels per 16-byte store (CP is 32 or 64)
  u32x4* dst = reinterpret_cast<u32x4*>(a + p * CP);
  for (int c8 = 0; c8 < CP / 8; ++c8) {
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = c8 * 8 + 2 * q;
      const uint32_t lo = c < c0 ? to_bf16(x[(b * c0 + c) * (int64_t)H * W + yx]) : 0u;
      const uint32_t hi = c + 1 < c0 ? to_bf16(x[(b * c0 + c + 1) * (int64_t)H * W + yx]) : 0u;
      w[q] = lo | (hi << 16);
    }
    dst[c8] = u32x4{w[0], w[1], w[2], w[3]};
  }
}

// ---------------------------------------------------------------------------------------
// implicit-GEMM convolution with fused epilogues

// RP output rows per step: 4 * RP waves, wave w computes row y + w / 4 (its 32-pixel groups
// w % 4, + 4, ...), with a ring of RP + 2 input rows in LDS.  RP = 2 keeps two waves per SIMD
// (one can issue MFMAs while the other waits on LDS or memory) and halves the barriers per
// row; it needs 4 input rows beside the weights in LDS, so wide rows use RP = 1.
template <int CIN, int COUT, int MODE, int RP>
__global__ __launch_bounds__(256 * RP) void k_conv(ConvArgs args) {
  constexpr int NT = 256 * RP, NS = RP + 2;
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  constexpr int LDW = 9 * CIN + 8;        // weight row (one output channel), bf16
  constexpr int LDI = CIN + 8;            // one halo pixel, bf16
  constexpr int TN = COUT / 32;
  const int H = args.H, W = args.W;
  uint16_t* sW = reinterpret_cast<uint16_t*>(smem_raw);
  uint16_t* sIn = sW + COUT * LDW;
  const int64_t row_elems = (int64_t)(W + 2) * LDI;
  __shared__ float red[4 * RP];

  const int b = blockIdx.y;
  const int y0 = blockIdx.x * args.rows;
  const int y1 = min(y0 + args.rows, H);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wrow = wave >> 2, wq = wave & 3;
  const uint16_t* in = args.in + (int64_t)b * H * W * CIN;

  // all weights -> LDS, every load of a thread issued before its stores (one memory latency
  // per workgroup instead of one per 16-byte vector)
  {
    constexpr int kWV = COUT * 9 * CIN / 8, kWPer = (kWV + NT - 1) / NT;
    u32x4 wv[kWPer];
#pragma unroll
    for (int k = 0; k < kWPer; ++k) {
      const int v = tid + k * NT;
      if (v < kWV) {
        const int co = v / (9 * CIN / 8), k8 = v % (9 * CIN / 8);
        wv[k] = *reinterpret_cast<const u32x4*>(args.wk + (int64_t)co * 9 * CIN + k8 * 8);
      }
    }
#pragma unroll
    for (int k = 0; k < kWPer; ++k) {
      const int v = tid + k * NT;
      if (v < kWV) {
        const int co = v / (9 * CIN / 8), k8 = v % (9 * CIN / 8);
        *reinterpret_cast<u32x4*>(sW + co * LDW + k8 * 8) = wv[k];
      }
    }
  }
  auto load_row = [&](int yy) {  // unwrapped row index -> ring slot yy mod NS
    const uint16_t* src = in + (int64_t)wrap(yy, H) * W * CIN;
    uint16_t* dst = sIn + wrap(yy, NS) * row_elems;
    for (int v = tid; v < (W + 2) * (CIN / 8); v += NT) {
      const int xh = v / (CIN / 8), c8 = v % (CIN / 8);
      const int xs = wrap(xh - 1, W);
      *reinterpret_cast<u32x4*>(dst + xh * LDI + c8 * 8) =
          *reinterpret_cast<const u32x4*>(src + (int64_t)xs * CIN + c8 * 8);
    }
  };
  // The next RP input rows are fetched into registers before a step's MFMAs and written to
  // their ring slots after them, so their memory latency overlaps the compute (rows of up to
  // kPf * NT 16-byte vectors; longer rows are loaded after the compute instead).
  constexpr int kPf = 8 / RP;
  const int row_vecs = (W + 2) * (CIN / 8);
  const bool prefetch = row_vecs <= kPf * NT;
  u32x4 pf[RP][kPf];
  auto fetch_row = [&](int j, int yy) {
    const uint16_t* src = in + (int64_t)wrap(yy, H) * W * CIN;
#pragma unroll
    for (int k = 0; k < kPf; ++k) {
      const int v = tid + k * NT;
      if (v < row_vecs) {
        const int xh = v / (CIN / 8), c8 = v % (CIN / 8);
        pf[j][k] = *reinterpret_cast<const u32x4*>(src + (int64_t)wrap(xh - 1, W) * CIN + c8 * 8);
      }
    }
  };
  auto commit_row = [&](int j, int yy) {
    uint16_t* dst = sIn + wrap(yy, NS) * row_elems;
#pragma unroll
    for (int k = 0; k < kPf; ++k) {
      const int v = tid + k * NT;
      if (v < row_vecs) {
        const int xh = v / (CIN / 8), c8 = v % (CIN / 8);
        *reinterpret_cast<u32x4*>(dst + xh * LDI + c8 * 8) = pf[j][k];
      }
    }
  };
  // rows y0 - 1 .. y0 + RP
  for (int yy = y0 - 1; yy <= y0 + RP; ++yy) {
    if (prefetch) {
      fetch_row(0, yy);
      commit_row(0, yy);
    } else {
      load_row(yy);
    }
  }
  __syncthreads();

  float loss_local = 0.0f;
  for (int ys = y0; ys < y1; ys += RP) {
    const bool more = ys + RP < y1;       // a next step: its new rows ys + RP + 1 .. ys + 2 RP
    if (prefetch && more)
#pragma unroll
      for (int j = 0; j < RP; ++j) fetch_row(j, ys + RP + 1 + j);
    const int y = ys + wrow;
    if (y < y1) {
      for (int g = wq; g < W / 32; g += 4) {
        f32x16_t acc[TN];
#pragma unroll
        for (int tn = 0; tn < TN; ++tn)
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[tn][r] = 0.0f;
        // the epilogue's FP32 inputs (MODE 2: the pre-activation below; MODE 1: the residual
        // and the target) are loaded before the MFMAs, so their latency overlaps them
        float pre0[TN][16], pre1[TN][16];
        if constexpr (MODE != 0) {
#pragma unroll
          for (int tn = 0; tn < TN; ++tn) {
            const int co = tn * 32 + (lane & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const int x = 32 * g + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
              const int64_t pix = ((int64_t)b * H + y) * W + x;
              pre0[tn][r] = pre1[tn][r] = 0.0f;
              if constexpr (MODE == 2) {
                pre0[tn][r] = from_bf16(args.gd_prev[pix * COUT + co]);
              } else if (co < args.c0) {
                const int64_t o = (((int64_t)b * args.c0 + co) * H + y) * W + x;
                pre0[tn][r] = args.x_res[o];
                if (args.target) pre1[tn][r] = args.target[o];
              }
            }
          }
        }
        auto tap_mfma = [&](int tap) {
          const int dy = tap / 3 - 1, dx = tap % 3 - 1;
          const uint16_t* rowp = sIn + wrap(y + dy, NS) * row_elems +
                                 (int64_t)(32 * g + (lane & 31) + dx + 1) * LDI + (lane >> 5) * 8;
#pragma unroll
          for (int c16 = 0; c16 < CIN / 16; ++c16) {
            const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(rowp + c16 * 16);
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) {
              const bf16x8_t bw = *reinterpret_cast<const bf16x8_t*>(
                  sW + (tn * 32 + (lane & 31)) * LDW + tap * CIN + c16 * 16 + (lane >> 5) * 8);
              acc[tn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bw, acc[tn], 0, 0, 0);
            }
          }
        };
        // one wave per SIMD (RP = 1) can hold every fragment of the nine taps at once; with
        // two waves per SIMD the taps are issued one at a time within the register budget
        if constexpr (RP == 1) {
#pragma unroll
          for (int tap = 0; tap < 9; ++tap) tap_mfma(tap);
        } else {
#pragma unroll 1
          for (int tap = 0; tap < 9; ++tap) tap_mfma(tap);
        }
        // epilogue: lane holds output channel co for 16 pixels of the group
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
          const int co = tn * 32 + (lane & 31);
          const float bias = (MODE != 2 && args.bias) ? args.bias[co] : 0.0f;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int x = 32 * g + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
            const int64_t pix = ((int64_t)b * H + y) * W + x;
            const float v = acc[tn][r] + bias;
            if constexpr (MODE == 0) {
              const GeluPair gp = gelu_pair(v);
              if (args.gd_out) args.gd_out[pix * COUT + co] = to_bf16(gp.d);
              args.a_out[pix * COUT + co] = to_bf16(gp.g);
            } else if constexpr (MODE == 1) {
              if (co < args.c0) {
                const int64_t o = (((int64_t)b * args.c0 + co) * H + y) * W + x;
                const float yv = pre0[tn][r] + v;
                args.y_out[o] = yv;
                if (args.target) {
                  const float diff = yv - pre1[tn][r];
                  loss_local += diff * diff;
                  args.a_out[pix * COUT + co] = to_bf16(args.grad_scale * diff);
                }
              } else if (args.target) {
                args.a_out[pix * COUT + co] = 0;
              }
            } else {
              args.a_out[pix * COUT + co] = to_bf16(v * pre0[tn][r]);
            }
          }
        }
      }
    }
    __syncthreads();                      // the rows ys - 1 .. ys + RP - 2 are no longer read
    if (more) {
#pragma unroll
      for (int j = 0; j < RP; ++j) {
        if (prefetch) commit_row(j, ys + RP + 1 + j); else load_row(ys + RP + 1 + j);
      }
      __syncthreads();
    }
  }
  if constexpr (MODE == 1) {
    if (args.loss_part) {
      for (int o = 32; o > 0; o >>= 1) loss_local += __shfl_xor(loss_local, o);
      if (lane == 0) red[wave] = loss_local;
      __syncthreads();
      if (tid == 0) {
        float t = 0.0f;
        for (int w = 0; w < 4 * RP; ++w) t += red[w];
        args.loss_part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
constexpr int kWgradThreads = 512;
constexpr int kWgradStep = 64;     // pixels per k-step of the weight gradient

// weight gradient: part[chunk][tap][co][ci] = sum_{p in chunk} du[p][co] * in[p + tap][ci]
// on v_mfma_f32_32x32x16_bf16 (the operands are the BF16 activations and output gradients;
// FP32 accumulation).  One workgroup computes all nine taps of its pixel chunk, so each k-step
// stages the output-gradient tile once and the nine shifted input tiles beside it.  The
// contraction runs over pixels, which are strided in NHWC, so each k-step of KS pixels is
// staged channel-major in LDS ([channel][pixel], rows padded to KS + 8): a thread loads eight
// channels of two consecutive pixels (two 16-byte loads) and writes the eight (pixel,
// pixel + 1) pairs as 4-byte words; a lane then reads the 8 consecutive pixels of its channel
// as one 16-byte fragment.  The 32 x 32 output blocks of one tap (COUT/32 x CIN/32 of them)
// go to as many waves; the waves left over split the taps.  A k-step's loads are issued two
// steps ahead (two register sets), so they have two steps' MFMAs to arrive in.

// HALO (W and the chunk a multiple of KS, so a k-step's pixels are KS consecutive pixels of
// one image row): the nine tap tiles are built from three input row segments of KS + 2
// pixels (rows y - 1, y, y + 1, columns x0 - 1 .. x0 + KS, periodic), each loaded once and
// written at the three column shifts; the dx = 0 copy is one pixel off the pair boundary and
// is written as 2-byte halves.  Otherwise each tap tile is loaded on its own.
template <int CIN, int COUT, bool HALO>
__global__ __launch_bounds__(kWgradThreads) void k_conv_wgrad(WgradArgs args) {
  constexpr int NT = kWgradThreads;
  constexpr int KS = kWgradStep;
  constexpr int LDK = KS + 8;             // LDS row (one channel), bf16
  constexpr int WM = COUT / 32, WN = CIN / 32, NBLK = WM * WN;
  constexpr int NGRP = NT / 64 / NBLK;    // wave groups splitting the taps
  constexpr int NTAP = (9 + NGRP - 1) / NGRP;
  __shared__ __attribute__((aligned(16))) uint16_t sA[COUT * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t sB[9 * CIN * LDK];
  const int H = args.H, W = args.W;
  const int chunk = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t npix = (int64_t)args.batch * H * W;
  const int64_t p0 = (int64_t)chunk * args.chunk_pixels;
  const int64_t p1 = min(p0 + (int64_t)args.chunk_pixels, npix);
  const int blk = wave % NBLK, grp = wave / NBLK;
  const int wm = blk / WN, wn = blk % WN;

  // staging units (pixel pair pp, channel octet c8; for B also the tap)
  constexpr int kPairs = KS / 2;
  constexpr int kPairsH = KS / 2 + 1;      // HALO: pairs of a row segment of KS + 2 pixels
  constexpr int kNA = kPairs * (COUT / 8);
  constexpr int kNB = HALO ? 3 * kPairsH * (CIN / 8) : 9 * kPairs * (CIN / 8);
  constexpr int kUA = (kNA + NT - 1) / NT, kUB = (kNB + NT - 1) / NT;
  // two register sets of staged vectors: a k-step's loads are issued two k-steps ahead (the
  // loop is unrolled by two so that each set is a fixed set of registers)
  u32x4 a0[2][kUA], a1[2][kUA], b0[2][kUB], b1[2][kUB];
  // Pixel pb + off (off < KS) of the batch shifted by the tap, with periodic wrap, from the
  // k-step's first pixel (bimg0, y00, x00): off < KS <= 2 W adds at most two rows (32-bit: the
  // host keeps batch * H * W below 2^31).
  int bimg0 = 0, y00 = 0, x00 = 0;
  auto in_row = [&](int off, int tap) {
    int bimg = bimg0, yy = y00, xx = x00 + off;
    while (xx >= W) {
      xx -= W;
      if (++yy == H) {
        yy = 0;
        ++bimg;
      }
    }
    int ys = yy + tap / 3 - 1, xs = xx + tap % 3 - 1;
    ys = ys < 0 ? ys + H : (ys >= H ? ys - H : ys);
    xs = xs < 0 ? xs + W : (xs >= W ? xs - W : xs);
    return args.in + ((int64_t)(bimg * H + ys) * W + xs) * CIN;
  };
  auto fetch = [&](auto set, int64_t pb) {
    constexpr int S = decltype(set)::value;
    {
      const int pi = (int)pb, hw = H * W;
      bimg0 = pi / hw;
      const int rem = pi - bimg0 * hw;
      y00 = rem / W;
      x00 = rem - y00 * W;
    }
#pragma unroll
    for (int k = 0; k < kUA; ++k) {
      const int v = tid + k * NT;
      if (v < kNA) {
        const int pp = v % kPairs, c8 = v / kPairs;
        const int64_t p = pb + 2 * pp;
        a0[S][k] = a1[S][k] = u32x4{0, 0, 0, 0};
        if (p < p1) a0[S][k] = *reinterpret_cast<const u32x4*>(args.du + p * COUT + c8 * 8);
        if (p + 1 < p1)
          a1[S][k] = *reinterpret_cast<const u32x4*>(args.du + (p + 1) * COUT + c8 * 8);
      }
    }
    if constexpr (HALO) {
      // pair m of row segment dyi: pixels x0 - 1 + 2m and x0 + 2m of row y + dyi - 1
#pragma unroll
      for (int k = 0; k < kUB; ++k) {
        const int v = tid + k * NT;
        if (v < kNB) {
          const int dyi = v / (kPairsH * (CIN / 8)), rem = v % (kPairsH * (CIN / 8));
          const int m = rem % kPairsH, c8 = rem / kPairsH;
          int ys = y00 + dyi - 1;
          ys = ys < 0 ? ys + H : (ys >= H ? ys - H : ys);
          int xa = x00 - 1 + 2 * m, xb = xa + 1;
          xa = xa < 0 ? xa + W : (xa >= W ? xa - W : xa);
          xb = xb >= W ? xb - W : xb;
          const uint16_t* row = args.in + (int64_t)(bimg0 * H + ys) * W * CIN + c8 * 8;
          b0[S][k] = *reinterpret_cast<const u32x4*>(row + (int64_t)xa * CIN);
          b1[S][k] = *reinterpret_cast<const u32x4*>(row + (int64_t)xb * CIN);
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < kUB; ++k) {
        const int v = tid + k * NT;
        if (v < kNB) {
          const int tap = v / (kPairs * (CIN / 8)), rem = v % (kPairs * (CIN / 8));
          const int pp = rem % kPairs, c8 = rem / kPairs;
          const int64_t p = pb + 2 * pp;
          b0[S][k] = b1[S][k] = u32x4{0, 0, 0, 0};
          if (p < p1) b0[S][k] = *reinterpret_cast<const u32x4*>(in_row(2 * pp, tap) + c8 * 8);
          if (p + 1 < p1)
            b1[S][k] = *reinterpret_cast<const u32x4*>(in_row(2 * pp + 1, tap) + c8 * 8);
        }
      }
    }
  };
  auto put_pair = [&](uint16_t* dst, const u32x4& w0, const u32x4& w1) {
    uint32_t* d = reinterpret_cast<uint32_t*>(dst);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      d[(2 * q) * (LDK / 2)] = (w0[q] & 0xFFFFu) | (w1[q] << 16);
      d[(2 * q + 1) * (LDK / 2)] = (w0[q] >> 16) | (w1[q] & 0xFFFF0000u);
    }
  };
  auto put = [&](auto set) {
    constexpr int S = decltype(set)::value;
#pragma unroll
    for (int k = 0; k < kUA; ++k) {
      const int v = tid + k * NT;
      if (v < kNA) {
        const int pp = v % kPairs, c8 = v / kPairs;
        put_pair(sA + (c8 * 8) * LDK + 2 * pp, a0[S][k], a1[S][k]);
      }
    }
    if constexpr (HALO) {
      // tile position k of tap (dyi, dx) holds segment pixel k + dx + 1: pair m is the pair at
      // k = 2m of dx = -1 and at k = 2m - 2 of dx = +1, and pixels k = 2m - 1, 2m of dx = 0
#pragma unroll
      for (int k = 0; k < kUB; ++k) {
        const int v = tid + k * NT;
        if (v < kNB) {
          const int dyi = v / (kPairsH * (CIN / 8)), rem = v % (kPairsH * (CIN / 8));
          const int m = rem % kPairsH, c8 = rem / kPairsH;
          uint16_t* base = sB + (dyi * 3) * CIN * LDK + (c8 * 8) * LDK;
          const u32x4& w0 = b0[S][k];
          const u32x4& w1 = b1[S][k];
          if (m < kPairsH - 1) put_pair(base + 2 * m, w0, w1);
          if (m >= 1) put_pair(base + 2 * CIN * LDK + 2 * m - 2, w0, w1);
          uint16_t* d0 = base + CIN * LDK;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (m >= 1) {
              d0[(2 * q) * LDK + 2 * m - 1] = (uint16_t)(w0[q] & 0xFFFFu);
              d0[(2 * q + 1) * LDK + 2 * m - 1] = (uint16_t)(w0[q] >> 16);
            }
            if (m < kPairsH - 1) {
              d0[(2 * q) * LDK + 2 * m] = (uint16_t)(w1[q] & 0xFFFFu);
              d0[(2 * q + 1) * LDK + 2 * m] = (uint16_t)(w1[q] >> 16);
            }
          }
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < kUB; ++k) {
        const int v = tid + k * NT;
        if (v < kNB) {
          const int tap = v / (kPairs * (CIN / 8)), rem = v % (kPairs * (CIN / 8));
          const int pp = rem % kPairs, c8 = rem / kPairs;
          put_pair(sB + tap * CIN * LDK + (c8 * 8) * LDK + 2 * pp, b0[S][k], b1[S][k]);
        }
      }
    }
  };

  f32x16_t acc[NTAP];
#pragma unroll
  for (int t = 0; t < NTAP; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;

  // one k-step from register set `set`, whose refill (k-step pb + 2 KS) is issued before the
  // MFMAs
  auto step = [&](auto set, int64_t pb) {
    __syncthreads();
    put(set);
    __syncthreads();
    if (pb + 2 * KS < p1) fetch(set, pb + 2 * KS);
#pragma unroll
    for (int kk = 0; kk < KS; kk += 16) {
      const int o = kk + (lane >> 5) * 8;
      const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(sA + (wm * 32 + (lane & 31)) * LDK + o);
#pragma unroll
      for (int t = 0; t < NTAP; ++t) {
        const int tap = grp + t * NGRP;
        if (tap < 9) {
          const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(
              sB + tap * CIN * LDK + (wn * 32 + (lane & 31)) * LDK + o);
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[t], 0, 0, 0);
        }
      }
    }
  };
  using Set0 = std::integral_constant<int, 0>;
  using Set1 = std::integral_constant<int, 1>;
  if (p0 < p1) fetch(Set0{}, p0);
  if (p0 + KS < p1) fetch(Set1{}, p0 + KS);
  for (int64_t pb = p0; pb < p1; pb += 2 * KS) {
    step(Set0{}, pb);
    if (pb + KS < p1) step(Set1{}, pb + KS);
  }
#pragma unroll
  for (int t = 0; t < NTAP; ++t) {
    const int tap = grp + t * NGRP;
    if (tap < 9) {
      float* out = args.part + ((int64_t)chunk * 9 + tap) * COUT * CIN;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int co = wm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        const int ci = wn * 32 + (lane & 31);
        out[co * CIN + ci] = acc[t][r];
      }
    }
  }
}

// bias gradient partials: part[chunk][co] = sum_{p in chunk} du[p][co].  Thread t reads the
// channel octet t % (cout / 8) of pixels t / (cout / 8), + lanes, ... as 16-byte vectors
// (a block reads whole consecutive pixel rows), then the per-lane sums are added in lane
// order through LDS.
__global__ __launch_bounds__(256) void k_bias_grad_part(const uint16_t* __restrict__ du,
                                                       int64_t npix, int cout, int chunk_pixels,
                                                       float* __restrict__ part) {
  __shared__ float s[256 * 8];
  const int octets = cout / 8, lanes = 256 / octets;
  const int o = threadIdx.x % octets, pl = threadIdx.x / octets;
  const int64_t p0 = (int64_t)blockIdx.x * chunk_pixels;
  const int64_t p1 = min(p0 + (int64_t)chunk_pixels, npix);
  float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t p = p0 + pl; p < p1; p += lanes) {
    const u32x4 w = *reinterpret_cast<const u32x4*>(du + p * cout + o * 8);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc[2 * q] += from_bf16((uint16_t)(w[q] & 0xFFFFu));
      acc[2 * q + 1] += from_bf16((uint16_t)(w[q] >> 16));
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) s[pl * cout + o * 8 + c] = acc[c];
  __syncthreads();
  if (threadIdx.x < cout) {
    float t = 0.0f;
    for (int l = 0; l < lanes; ++l) t += s[l * cout + threadIdx.x];
    part[(int64_t)blockIdx.x * cout + threadIdx.x] = t;
  }
}

// grad[i] = sum over chunks of part[chunk][i] in a fixed order, FP64 accumulation: a
// workgroup takes 64 consecutive entries, its four thread groups the chunks g, g + 4, ...
// (coalesced 256-byte rows), and the four group sums are added in group order.  WGRAD maps the
// partial layout [tap][co][ci] to the parameter layout [co][tap][ci].
template <bool WGRAD>
__global__ __launch_bounds__(256) void k_reduce_parts(const float* __restrict__ part, int64_t n,
                                                      int chunks, int cout, int cin,
                                                      float* __restrict__ grad) {
  __shared__ double sg[4][64];
  const int e = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + e;
  double acc = 0.0;
  if (i < n)
    for (int c = g; c < chunks; c += 4) acc += part[(int64_t)c * n + i];
  sg[g][e] = acc;
  __syncthreads();
  if (g == 0 && i < n) {
    const double t = ((sg[0][e] + sg[1][e]) + sg[2][e]) + sg[3][e];
    if constexpr (WGRAD) {
      const int tap = (int)(i / ((int64_t)cout * cin));
      const int co = (int)((i / cin) % cout), ci = (int)(i % cin);
      grad[((int64_t)co * 9 + tap) * cin + ci] = (float)t;
    } else {
      grad[i] = (float)t;
    }
  }
}

// One wave: lane l adds the l-th of 64 consecutive slices of the partials in order (FP64),
// then lane 0 adds the 64 slice sums in lane order.
__global__ __launch_bounds__(64) void k_sum_loss(const float* __restrict__ part, int n,
                                                double scale, double* __restrict__ out) {
  __shared__ double sl[64];
  const int l = threadIdx.x;
  double s = 0.0;
  for (int i = (int)((int64_t)l * n / 64); i < (int)((int64_t)(l + 1) * n / 64); ++i)
    s += part[i];
  sl[l] = s;
  __syncthreads();
  if (l != 0) return;
  s = 0.0;
  for (int k = 0; k < 64; ++k) s += sl[k];
  *out = s * scale;
}

// Adam (Kingma & Ba, 2015) on the flat FP32 master parameters.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float corr1, float corr2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / corr1, vh = vi / corr2;
  p[i] -= lr * mh / (sqrtf(vh) + eps);
}

// bf16 copies of one layer's weights: wk[co][tap*CIN + ci] and the flipped transpose used
// by the input gradient, wf[ci][(8 - tap)*COUT + co].
__global__ void k_make_bf16_weights(const float* __restrict__ w, int cout, int cin,
                                    uint16_t* __restrict__ wk, uint16_t* __restrict__ wf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 9LL * cout * cin) return;
  const int co = (int)(i / (9LL * cin)), tap = (int)((i / cin) % 9), ci = (int)(i % cin);
  const uint16_t h = to_bf16(w[i]);
  wk[i] = h;
  wf[((int64_t)ci * 9 + (8 - tap)) * cout + co] = h;
}

// ---------------------------------------------------------------------------------------
// host launchers

size_t conv_smem_bytes(int cin, int cout, int W, int rp) {
  return (size_t)cout * (9 * cin + 8) * 2 + (size_t)(rp + 2) * (W + 2) * (cin + 8) * 2;
}

// the dynamic LDS a workgroup may use on gfx950 (160 KB), less room for the static part
constexpr size_t kMaxConvSmem = 159 * 1024;

int conv_rows_per_step(int cin, int cout, int W) {
  return conv_smem_bytes(cin, cout, W, 2) <= kMaxConvSmem ? 2 : 1;
}

template <int CIN, int COUT, int MODE, int RP>
static hipError_t launch_conv_t(const ConvArgs& a, hipStream_t s) {
  const size_t shm = conv_smem_bytes(CIN, COUT, a.W, RP);
  if (shm > kMaxConvSmem) return hipErrorInvalidValue;
  static size_t attr_bytes = 0;
  if (shm > 64 * 1024 && shm > attr_bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_conv<CIN, COUT, MODE, RP>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    attr_bytes = shm;
  }
  dim3 grid((a.H + a.rows - 1) / a.rows, a.batch);
  hipLaunchKernelGGL((k_conv<CIN, COUT, MODE, RP>), grid, dim3(256 * RP), shm, s, a);
  return hipGetLastError();
}

hipError_t launch_conv(int cin, int cout, int mode, const ConvArgs& a, hipStream_t s) {
  const int rp = conv_rows_per_step(cin, cout, a.W);
#define SG_CONV(CI, CO, MD)                                                   \
  if (cin == CI && cout == CO && mode == MD)                                  \
    return rp == 2 ? launch_conv_t<CI, CO, MD, 2>(a, s) : launch_conv_t<CI, CO, MD, 1>(a, s);
  SG_CONV(32, 32, 0) SG_CONV(32, 64, 0) SG_CONV(64, 32, 0) SG_CONV(64, 64, 0)
  SG_CONV(32, 32, 1) SG_CONV(64, 32, 1)
  SG_CONV(32, 32, 2) SG_CONV(32, 64, 2) SG_CONV(64, 32, 2) SG_CONV(64, 64, 2)
#undef SG_CONV
  return hipErrorInvalidValue;
}

hipError_t launch_wgrad(int cin, int cout, const WgradArgs& a, int chunks, hipStream_t s) {
  dim3 grid(chunks);
  const bool halo = a.W % kWgradStep == 0 && a.chunk_pixels % kWgradStep == 0;
#define SG_WG(CI, CO)                                                                        \
  if (cin == CI && cout == CO) {                                                             \
    if (halo)                                                                                \
      hipLaunchKernelGGL((k_conv_wgrad<CI, CO, true>), grid, dim3(kWgradThreads), 0, s, a);  \
    else                                                                                     \
      hipLaunchKernelGGL((k_conv_wgrad<CI, CO, false>), grid, dim3(kWgradThreads), 0, s, a); \
    return hipGetLastError();                                                                \
  }
  SG_WG(32, 32) SG_WG(32, 64) SG_WG(64, 32) SG_WG(64, 64)
#undef SG_WG
  return hipErrorInvalidValue;
}

hipError_t launch_pack_input(const float* x, uint16_t* a, int batch, int c0, int H, int W, int cp,
                             hipStream_t s) {
  const int64_t n = (int64_t)batch * H * W;
  hipLaunchKernelGGL(k_pack_input, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, a,
                     batch, c0, H, W, cp);
  return hipGetLastError();
}

hipError_t launch_bias_grad(const uint16_t* du, int64_t npix, int cout, int chunk_pixels,
                            int chunks, float* part, float* grad, hipStream_t s) {
  hipLaunchKernelGGL(k_bias_grad_part, dim3(chunks), dim3(256), 0, s, du, npix, cout,
                     chunk_pixels, part);
  hipLaunchKernelGGL(k_reduce_parts<false>, dim3((cout + 63) / 64), dim3(256), 0, s, part,
                     (int64_t)cout, chunks, cout, 1, grad);
  return hipGetLastError();
}

hipError_t launch_reduce_wgrad(const float* part, int cout, int cin, int chunks, float* grad,
                               hipStream_t s) {
  const int64_t n = 9LL * cout * cin;
  hipLaunchKernelGGL(k_reduce_parts<true>, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s, part,
                     n, chunks, cout, cin, grad);
  return hipGetLastError();
}

hipError_t launch_sum_loss(const float* part, int n, double scale, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(64), 0, s, part, n, scale, out);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                       float b1, float b2, float eps, float corr1, float corr2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n,
                     lr, b1, b2, eps, corr1, corr2);
  return hipGetLastError();
}

hipError_t launch_make_bf16_weights(const float* w, int cout, int cin, uint16_t* wk,
                                    uint16_t* wf, hipStream_t s) {
  const int64_t n = 9LL * cout * cin;
  hipLaunchKernelGGL(k_make_bf16_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w,
                     cout, cin, wk, wf);
  return hipGetLastError();
}

}  // namespace sg
}  // namespace ensf
