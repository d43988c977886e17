// HIP kernels of the convolutional forecast surrogate (gfx950).
//
// Activations are NHWC bf16 with the channel count padded to CP in {32, 64} (padding is
// zero and stays zero: padded weights and biases are zero).  A 3x3 convolution with
// periodic padding is an implicit GEMM: M = pixels, N = output channels, K = 9 taps x
// input channels.  One workgroup (4 waves) owns one image and a band of output rows; it
// keeps all weights and a ring of three input rows (with a one-pixel periodic halo) in
// LDS, so each new output row costs one new input row from memory.  Wave w computes
// 32-pixel groups w, w+4, ... of the row against all output channels with
// v_mfma_f32_32x32x16_bf16 (FP32 accumulation).
//
// The input-gradient convolution is the same kernel run on the output gradient with the
// taps flipped and the weight matrix transposed.  The weight gradient contracts over
// pixels, which are strided in NHWC, so it stages BF16 tiles channel-major in LDS and uses
// v_mfma_f32_32x32x16_bf16; per-chunk partials are reduced in a fixed order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

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

__device__ __forceinline__ float gelu(float u) {
  return 0.5f * u * (1.0f + erff(u * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float u) {
  const float cdf = 0.5f * (1.0f + erff(u * 0.70710678118654752f));
  const float pdf = 0.3989422804014327f * expf(-0.5f * u * u);
  return cdf + u * pdf;
}

__device__ __forceinline__ int wrap(int v, int n) { return ((v % n) + n) % n; }

// NCHW float32 (c0 channels) -> NHWC bf16 with CP channels (zero padded).
__global__ void k_pack_input(const float* __restrict__ x, uint16_t* __restrict__ a, int batch,
                             int c0, int H, int W, int CP) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t npix = (int64_t)batch * H * W;
  if (p >= npix) return;
  const int64_t b = p / ((int64_t)H * W), yx = p % ((int64_t)H * W);
  uint16_t* dst = a + p * CP;
  for (int c = 0; c < CP; ++c)
    dst[c] = c < c0 ? to_bf16(x[(b * c0 + c) * (int64_t)H * W + yx]) : (uint16_t)0;
}

// ---------------------------------------------------------------------------------------
// implicit-GEMM convolution with fused epilogues

template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) void k_conv(ConvArgs args) {
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  constexpr int LDW = 9 * CIN + 8;        // weight row (one output channel), bf16
  constexpr int LDI = CIN + 8;            // one halo pixel, bf16
  constexpr int TN = COUT / 32;
  const int H = args.H, W = args.W;
  uint16_t* sW = reinterpret_cast<uint16_t*>(smem_raw);
  uint16_t* sIn = sW + COUT * LDW;
  const int64_t row_elems = (int64_t)(W + 2) * LDI;
  __shared__ float red[4];

  const int b = blockIdx.y;
  const int y0 = blockIdx.x * args.rows;
  const int y1 = min(y0 + args.rows, H);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint16_t* in = args.in + (int64_t)b * H * W * CIN;

  // all weights -> LDS, every load of a thread issued before its stores (one memory latency
  // per workgroup instead of one per 16-byte vector)
  {
    constexpr int kWV = COUT * 9 * CIN / 8, kWPer = (kWV + 255) / 256;
    u32x4 wv[kWPer];
#pragma unroll
    for (int k = 0; k < kWPer; ++k) {
      const int v = tid + k * 256;
      if (v < kWV) {
        const int co = v / (9 * CIN / 8), k8 = v % (9 * CIN / 8);
        wv[k] = *reinterpret_cast<const u32x4*>(args.wk + (int64_t)co * 9 * CIN + k8 * 8);
      }
    }
#pragma unroll
    for (int k = 0; k < kWPer; ++k) {
      const int v = tid + k * 256;
      if (v < kWV) {
        const int co = v / (9 * CIN / 8), k8 = v % (9 * CIN / 8);
        *reinterpret_cast<u32x4*>(sW + co * LDW + k8 * 8) = wv[k];
      }
    }
  }
  auto load_row = [&](int yy) {  // unwrapped row index -> ring slot yy mod 3
    const int slot = wrap(yy, 3);
    const uint16_t* src = in + (int64_t)wrap(yy, H) * W * CIN;
    uint16_t* dst = sIn + slot * row_elems;
    for (int v = tid; v < (W + 2) * (CIN / 8); v += 256) {
      const int xh = v / (CIN / 8), c8 = v % (CIN / 8);
      const int xs = wrap(xh - 1, W);
      *reinterpret_cast<u32x4*>(dst + xh * LDI + c8 * 8) =
          *reinterpret_cast<const u32x4*>(src + (int64_t)xs * CIN + c8 * 8);
    }
  };
  // The next input row is fetched into registers before a row's MFMAs and written to its
  // ring slot after them, so its memory latency overlaps the compute (rows of up to
  // kPf * 256 16-byte vectors; longer rows are loaded after the compute instead).
  constexpr int kPf = 8;
  const int row_vecs = (W + 2) * (CIN / 8);
  const bool prefetch = row_vecs <= kPf * 256;
  u32x4 pf[kPf];
  auto fetch_row = [&](int yy) {
    const uint16_t* src = in + (int64_t)wrap(yy, H) * W * CIN;
#pragma unroll
    for (int k = 0; k < kPf; ++k) {
      const int v = tid + k * 256;
      if (v < row_vecs) {
        const int xh = v / (CIN / 8), c8 = v % (CIN / 8);
        pf[k] = *reinterpret_cast<const u32x4*>(src + (int64_t)wrap(xh - 1, W) * CIN + c8 * 8);
      }
    }
  };
  auto commit_row = [&](int yy) {
    uint16_t* dst = sIn + wrap(yy, 3) * row_elems;
#pragma unroll
    for (int k = 0; k < kPf; ++k) {
      const int v = tid + k * 256;
      if (v < row_vecs) {
        const int xh = v / (CIN / 8), c8 = v % (CIN / 8);
        *reinterpret_cast<u32x4*>(dst + xh * LDI + c8 * 8) = pf[k];
      }
    }
  };
  if (prefetch) {
    fetch_row(y0 - 1);
    commit_row(y0 - 1);
    fetch_row(y0);
    commit_row(y0);
    fetch_row(y0 + 1);
    commit_row(y0 + 1);
  } else {
    load_row(y0 - 1);
    load_row(y0);
    load_row(y0 + 1);
  }
  __syncthreads();

  float loss_local = 0.0f;
  for (int y = y0; y < y1; ++y) {
    if (prefetch && y + 1 < y1) fetch_row(y + 2);
    for (int g = wave; g < W / 32; g += 4) {
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
              pre0[tn][r] = args.u_prev[pix * COUT + co];
            } else if (co < args.c0) {
              const int64_t o = (((int64_t)b * args.c0 + co) * H + y) * W + x;
              pre0[tn][r] = args.x_res[o];
              if (args.target) pre1[tn][r] = args.target[o];
            }
          }
        }
      }
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const uint16_t* rowp = sIn + wrap(y + dy, 3) * row_elems +
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
            if (args.u_out) args.u_out[pix * COUT + co] = v;
            args.a_out[pix * COUT + co] = to_bf16(gelu(v));
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
            const float gp = gelu_grad(pre0[tn][r]);
            args.a_out[pix * COUT + co] = to_bf16(v * gp);
          }
        }
      }
    }
    __syncthreads();                      // all reads of row y-1's slot are done
    if (y + 1 < y1) {
      if (prefetch) commit_row(y + 2); else load_row(y + 2);
      __syncthreads();
    }
  }
  if constexpr (MODE == 1) {
    if (args.loss_part) {
      for (int o = 32; o > 0; o >>= 1) loss_local += __shfl_xor(loss_local, o);
      if (lane == 0) red[wave] = loss_local;
      __syncthreads();
      if (tid == 0)
        args.loss_part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] =
            red[0] + red[1] + red[2] + red[3];
    }
  }
}

// ---------------------------------------------------------------------------------------
// weight gradient: part[chunk][tap][co][ci] = sum_{p in chunk} du[p][co] * in[p + tap][ci]
// on v_mfma_f32_32x32x16_bf16 (the operands are the BF16 activations and output gradients;
// FP32 accumulation).  The contraction runs over pixels, which are strided in NHWC, so each
// k-step of KS pixels is staged channel-major in LDS ([channel][pixel], rows padded to
// KS + 8): a thread loads eight channels of two consecutive pixels (two 16-byte loads) and
// writes the eight (pixel, pixel + 1) pairs as 4-byte words; a lane then reads the 8
// consecutive pixels of its channel as one 16-byte fragment.

template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_wgrad(WgradArgs args) {
  constexpr int KS = 64;                  // pixels per k-step
  constexpr int LDK = KS + 8;             // LDS row (one channel), bf16
  __shared__ __attribute__((aligned(16))) uint16_t sA[COUT * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t sB[CIN * LDK];
  constexpr int WM = COUT / 32, WN = CIN / 32;
  const int H = args.H, W = args.W;
  const int chunk = blockIdx.x, tap = blockIdx.y;
  const int dy = tap / 3 - 1, dx = tap % 3 - 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t npix = (int64_t)args.batch * H * W;
  const int64_t p0 = (int64_t)chunk * args.chunk_pixels;
  const int64_t p1 = min(p0 + (int64_t)args.chunk_pixels, npix);
  const bool active = wave < WM * WN;
  const int wm = wave / WN, wn = wave % WN;

  // staging unit of this thread: pixel pair pp, channel octet c8.  A k-step's units are
  // fetched into registers (fetch) one k-step ahead and written to LDS (put) after the
  // previous k-step's MFMAs, so the loads overlap them.
  constexpr int kNA = (KS / 2) * (COUT / 8), kNB = (KS / 2) * (CIN / 8);   // units per step
  constexpr int kUA = (kNA + 255) / 256, kUB = (kNB + 255) / 256;
  struct Units {
    u32x4 a0[kUA], a1[kUA], b0[kUB], b1[kUB];
  } u;
  auto fetch_op = [&](u32x4* w0s, u32x4* w1s, int n, int total, auto src_of, int64_t pb) {
    for (int k = 0; k < n; ++k) {
      const int v = tid + k * 256;
      if (v >= total) break;
      const int pp = v % (KS / 2), c8 = v / (KS / 2);
      u32x4 w0 = {0, 0, 0, 0}, w1 = {0, 0, 0, 0};
      const int64_t p = pb + 2 * pp;
      if (p < p1) w0 = *reinterpret_cast<const u32x4*>(src_of(p) + c8 * 8);
      if (p + 1 < p1) w1 = *reinterpret_cast<const u32x4*>(src_of(p + 1) + c8 * 8);
      w0s[k] = w0;
      w1s[k] = w1;
    }
  };
  auto put_op = [&](uint16_t* dst, const u32x4* w0s, const u32x4* w1s, int n, int total) {
    for (int k = 0; k < n; ++k) {
      const int v = tid + k * 256;
      if (v >= total) break;
      const int pp = v % (KS / 2), c8 = v / (KS / 2);
      uint32_t* d = reinterpret_cast<uint32_t*>(dst + (c8 * 8) * LDK + 2 * pp);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        d[(2 * q) * (LDK / 2)] = (w0s[k][q] & 0xFFFFu) | (w1s[k][q] << 16);
        d[(2 * q + 1) * (LDK / 2)] = (w0s[k][q] >> 16) | (w1s[k][q] & 0xFFFF0000u);
      }
    }
  };
  auto du_row = [&](int64_t p) { return args.du + p * COUT; };
  auto in_row = [&](int64_t p) {
    const int64_t bimg = p / ((int64_t)H * W);
    const int yy = (int)((p / W) % H), xx = (int)(p % W);
    return args.in + ((bimg * H + wrap(yy + dy, H)) * W + wrap(xx + dx, W)) * CIN;
  };

  f32x16_t acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;

  auto fetch = [&](int64_t pb) {
    fetch_op(u.a0, u.a1, kUA, kNA, du_row, pb);
    fetch_op(u.b0, u.b1, kUB, kNB, in_row, pb);
  };
  if (p0 < p1) fetch(p0);
  for (int64_t pb = p0; pb < p1; pb += KS) {
    __syncthreads();
    put_op(sA, u.a0, u.a1, kUA, kNA);
    put_op(sB, u.b0, u.b1, kUB, kNB);
    __syncthreads();
    if (pb + KS < p1) fetch(pb + KS);
    if (active) {
#pragma unroll
      for (int kk = 0; kk < KS; kk += 16) {
        const int o = kk + (lane >> 5) * 8;
        const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(sA + (wm * 32 + (lane & 31)) * LDK + o);
        const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(sB + (wn * 32 + (lane & 31)) * LDK + o);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    }
  }
  if (active) {
    float* out = args.part + ((int64_t)chunk * 9 + tap) * COUT * CIN;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int co = wm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
      const int ci = wn * 32 + (lane & 31);
      out[co * CIN + ci] = acc[r];
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

// grad[i] = sum over chunks of part[chunk][i] (fixed order), FP64 accumulation
__global__ void k_reduce_chunks(const float* __restrict__ part, int64_t n, int chunks,
                                float* __restrict__ grad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * n + i];
  grad[i] = (float)s;
}

// wgrad partial layout [tap][co][ci] -> parameter layout [co][tap][ci]
__global__ void k_reduce_wgrad(const float* __restrict__ part, int cout, int cin, int chunks,
                               float* __restrict__ grad) {
  const int64_t n = 9LL * cout * cin;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int tap = (int)(i / ((int64_t)cout * cin));
  const int co = (int)((i / cin) % cout), ci = (int)(i % cin);
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * n + i];
  grad[((int64_t)co * 9 + tap) * cin + ci] = (float)s;
}

__global__ void k_sum_loss(const float* __restrict__ part, int n, double scale,
                           double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = s * scale;
  }
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

size_t conv_smem_bytes(int cin, int cout, int W) {
  return (size_t)cout * (9 * cin + 8) * 2 + (size_t)3 * (W + 2) * (cin + 8) * 2;
}

template <int CIN, int COUT, int MODE>
static hipError_t launch_conv_t(const ConvArgs& a, hipStream_t s) {
  const size_t shm = conv_smem_bytes(CIN, COUT, a.W);
  static size_t attr_bytes = 0;
  if (shm > 64 * 1024 && shm > attr_bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_conv<CIN, COUT, MODE>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    attr_bytes = shm;
  }
  dim3 grid((a.H + a.rows - 1) / a.rows, a.batch);
  hipLaunchKernelGGL((k_conv<CIN, COUT, MODE>), grid, dim3(256), shm, s, a);
  return hipGetLastError();
}

hipError_t launch_conv(int cin, int cout, int mode, const ConvArgs& a, hipStream_t s) {
#define SG_CONV(CI, CO, MD) \
  if (cin == CI && cout == CO && mode == MD) return launch_conv_t<CI, CO, MD>(a, s);
  SG_CONV(32, 32, 0) SG_CONV(32, 64, 0) SG_CONV(64, 32, 0) SG_CONV(64, 64, 0)
  SG_CONV(32, 32, 1) SG_CONV(64, 32, 1)
  SG_CONV(32, 32, 2) SG_CONV(32, 64, 2) SG_CONV(64, 32, 2) SG_CONV(64, 64, 2)
#undef SG_CONV
  return hipErrorInvalidValue;
}

hipError_t launch_wgrad(int cin, int cout, const WgradArgs& a, int chunks, hipStream_t s) {
  dim3 grid(chunks, 9);
#define SG_WG(CI, CO)                                                                \
  if (cin == CI && cout == CO) {                                                     \
    hipLaunchKernelGGL((k_conv_wgrad<CI, CO>), grid, dim3(256), 0, s, a);            \
    return hipGetLastError();                                                        \
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
  hipLaunchKernelGGL(k_reduce_chunks, dim3((cout + 255) / 256), dim3(256), 0, s, part,
                     (int64_t)cout, chunks, grad);
  return hipGetLastError();
}

hipError_t launch_reduce_wgrad(const float* part, int cout, int cin, int chunks, float* grad,
                               hipStream_t s) {
  const int64_t n = 9LL * cout * cin;
  hipLaunchKernelGGL(k_reduce_wgrad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part,
                     cout, cin, chunks, grad);
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
