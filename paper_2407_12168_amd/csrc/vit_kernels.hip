// HIP kernels of the transformer forecast surrogate (Sec. III-B: a ViT backbone whose cost is
// dominated by its matrix products) for CDNA4 (gfx950).
//
// Every matrix product, forward and backward, is one form: C = alpha A B^T with both operands
// BF16 and contiguous along the contraction (k), on v_mfma_f32_32x32x16_bf16 with FP32
// accumulation, batched over (image, head) for attention.  The operands that a backward
// product needs in the other orientation are written transposed by the kernel that produces
// them (GEMM epilogues, LayerNorm, softmax, patch extraction), so no product reads a strided
// operand.  Everything elementwise (bias, residual add, GELU and its derivative, LayerNorm,
// softmax, the loss) is fused into those producers.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mfma_tile.h"
#include "vit_internal.h"

namespace ensf {
namespace vit {

namespace {

constexpr int kRows = 32;   // rows per workgroup of the row-wise kernels (four waves of eight
                            // rows; eight waves of four in the LayerNorm forward)

__device__ __forceinline__ uint16_t to_bf16(float v) {
  return __builtin_bit_cast(uint16_t, (__bf16)v);
}
__device__ __forceinline__ float from_bf16(uint16_t b) {
  return __builtin_bit_cast(float, (uint32_t)b << 16);
}

__device__ __forceinline__ float gelu_f(float v) {
  return 0.5f * v * (1.0f + erff(v * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad_f(float u) {
  const float cdf = 0.5f * (1.0f + erff(u * 0.70710678118654752f));
  return cdf + u * 0.39894228040143268f * expf(-0.5f * u * u);
}

__device__ __forceinline__ float wave_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Writes a kRows x cols BF16 tile held in LDS (row stride cols + 2, which spreads the column
// reads of the two rows a thread packs over distinct banks) transposed: dst[c * ld + r] for
// r < kRows, two rows per 4-byte store, 16 threads per destination row (64 contiguous bytes).
__device__ __forceinline__ void store_tile_transposed(const uint16_t* tile, int cols,
                                                      uint16_t* dst, int64_t ld) {
  const int lds = cols + 2;
  for (int i = threadIdx.x; i < cols * (kRows / 2); i += blockDim.x) {
    const int c = i / (kRows / 2), pr = i % (kRows / 2);
    const uint32_t w = (uint32_t)tile[(2 * pr) * lds + c] |
                       ((uint32_t)tile[(2 * pr + 1) * lds + c] << 16);
    *reinterpret_cast<uint32_t*>(dst + (int64_t)c * ld + 2 * pr) = w;
  }
}

}  // namespace

// ----------------------------------------------------------------------------------------
// C = alpha A B^T with the fused epilogue of VGemm.

// Four-wave tiles are compiled for three resident waves per SIMD (three workgroups per CU,
// whose LDS stages also fit), eight-wave tiles for four (two workgroups per CU): the register
// budgets that leaves are enough without spills.
// BK is the k-step, ST the LDS stage count (2: ping-pong when both stages fit).
template <int WGM, int WGN, int TM, int TN, int BK, int ST>
__global__ __launch_bounds__(64 * WGM * WGN, WGM * WGN >= 8 ? 4 : (WGM * WGN >= 4 ? 3 : 1))
void k_vgemm(VGemm g) {
  constexpr int NT = 64 * WGM * WGN, BM = WGM * TM * 32, BN = WGN * TN * 32;
  using S = TileSmem<kBF16, BM, BN, BK, false>;
  constexpr bool PP = ST == 2 && 2 * S::kBytes <= kPingPongBytes;
  __shared__ __attribute__((aligned(16))) char smem[PP ? 2 * S::kBytes : S::kBytes];

  const int ntiles = (int)(gridDim.x / g.splits);
  const int lt = xcd_remap(blockIdx.x, gridDim.x);
  const int split = lt / ntiles, tile = lt - split * ntiles;
  const int tn = tile % g.tiles_n, tm = tile / g.tiles_n;
  const int z = blockIdx.y, zb = z / g.nh, zh = z - zb * g.nh;
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int64_t kbeg = g.kchunk ? split * g.kchunk : 0;
  const int64_t kend = g.kchunk ? min(kbeg + g.kchunk, (int64_t)g.K) : (int64_t)g.K;

  f32x16_t acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

  const uint16_t* pa = g.A.p + zb * g.A.sb + zh * g.A.sh;
  const uint16_t* pb = g.B.p + zb * g.B.sb + zh * g.B.sh;
  Bf16KmajLoad<BM, NT, false, BK> la;
  Bf16KmajLoad<BN, NT, false, BK> lb;
  la.init(pa, pa, g.A.ld, m0);
  lb.init(pb, pb, g.B.ld, n0);
  tile_k_loop<kBF16, WGM, WGN, TM, TN, BK, PP, false>(
      smem, kbeg, kend,
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

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  // output bases at the tile's corner: the offsets inside the tile, and the addend's row
  // offsets (token counts times widths), fit 32 bits
  float* f32 = g.f32 ? g.f32 + zb * g.sb_f32 + zh * g.sh_f32 + split * g.part_stride +
                           m0 * g.ld_f32 + n0
                     : nullptr;
  uint16_t* b16 = g.b16 ? g.b16 + zb * g.sb_b16 + zh * g.sh_b16 + m0 * g.ld_b16 + n0 : nullptr;
  uint16_t* b16t = g.b16t ? g.b16t + zb * g.sb_t + zh * g.sh_t + n0 * g.ld_t + m0 : nullptr;
  const float* add = g.add ? g.add + n0 : nullptr;
  const uint16_t* gin = g.gin ? g.gin + m0 * g.ld_gin + n0 : nullptr;
  uint16_t* gd = g.gd ? g.gd + m0 * g.ld_gin + n0 : nullptr;
  const int ldf = (int)g.ld_f32, ldb = (int)g.ld_b16, ldt = (int)g.ld_t;
  const int lda = (int)g.ld_add, ldg = (int)g.ld_gin;
#pragma unroll
  for (int b = 0; b < TN; ++b) {
    const int nl = wn * TN * 32 + b * 32 + (lane & 31);
    const float bias = g.bias ? g.bias[n0 + nl] : 0.0f;
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int gq = 0; gq < 4; ++gq) {
        const int ml = wm * TM * 32 + a * 32 + gq * 8 + (lane >> 5) * 4;
        // addend rows: add_rows is a multiple of 4, so the four rows ml..ml+3 are consecutive
        // rows of the addend too
        const int ar = g.add_rows ? (int)((m0 + ml) % g.add_rows) : (int)(m0 + ml);
        uint16_t h[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int m = ml + j;
          float v = g.alpha * acc[a][b][gq * 4 + j] + bias;
          if (add) v += add[(ar + j) * lda + nl];
          if (f32) f32[m * ldf + nl] = v;
          if (g.act == 1) {
            if (gd) gd[m * ldg + nl] = to_bf16(gelu_grad_f(v));
            v = gelu_f(v);
          } else if (g.act == 2) {
            v *= from_bf16(gin[m * ldg + nl]);
          }
          h[j] = to_bf16(v);
          if (b16) b16[m * ldb + nl] = h[j];
        }
        if (b16t) {
          const uint2 w = make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16),
                                     (uint32_t)h[2] | ((uint32_t)h[3] << 16));
          *reinterpret_cast<uint2*>(b16t + nl * ldt + ml) = w;
        }
        // one register group at a time: keeps the loads and addresses of the other groups
        // from being hoisted (which costs registers, hence occupancy)
        __builtin_amdgcn_sched_barrier(0);
      }
  }
}

// ----------------------------------------------------------------------------------------
// LayerNorm

// Rows are held in registers: lane l owns the V-wide groups (64 j + l) of its row, j < J (V = 4
// loads and stores 16 / 8 bytes at once when D is a multiple of 256, J = D / 256; otherwise
// V = 1 with guards up to D = 2048).

template <int V>
__device__ __forceinline__ void load_v(const float* p, float (&v)[V]) {
  if constexpr (V == 4) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  } else {
#pragma unroll
    for (int c = 0; c < V; ++c) v[c] = p[c];
  }
}
template <int V>
__device__ __forceinline__ void store_v(float* p, const float (&v)[V]) {
  if constexpr (V == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
#pragma unroll
    for (int c = 0; c < V; ++c) p[c] = v[c];
  }
}
template <int V>
__device__ __forceinline__ void store_bf16_v(uint16_t* p, const uint16_t (&h)[V]) {
  if constexpr (V == 4) {
    *reinterpret_cast<uint2*>(p) = make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16),
                                             (uint32_t)h[2] | ((uint32_t)h[3] << 16));
  } else {
#pragma unroll
    for (int c = 0; c < V; ++c) p[c] = h[c];
  }
}

// Eight waves per kRows-row tile, rows strided by eight (two waves per SIMD at one
// workgroup per CU).
constexpr int kLnFwdWaves = 8;

template <int V, int J>
__global__ __launch_bounds__(64 * kLnFwdWaves) void k_ln_fwd(const float* x, int D,
                                                              const float* gam, const float* bet,
                                                              uint16_t* y, uint16_t* yt,
                                                              int64_t ld_t, float* mean,
                                                              float* rstd) {
  extern __shared__ uint16_t tile[];   // kRows x (D + 2)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * kRows;
  // the wave's next row is loaded while the current one is normalised
  float nv[J][V];
  auto fetch = [&](int64_t r) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int d0 = (j * 64 + lane) * V;
      if (d0 < D) load_v<V>(x + r * D + d0, nv[j]);
    }
  };
  fetch(r0 + wave);
  for (int rr = wave; rr < kRows; rr += kLnFwdWaves) {
    const int64_t r = r0 + rr;
    float v[J][V];
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int c = 0; c < V; ++c) v[j][c] = nv[j][c];
    if (rr + kLnFwdWaves < kRows) fetch(r + kLnFwdWaves);
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int d0 = (j * 64 + lane) * V;
      if (d0 < D) {
#pragma unroll
        for (int c = 0; c < V; ++c) s += v[j][c];
      }
    }
    const float mu = wave_sum(s) / (float)D;
    float q = 0.0f;
#pragma unroll
    for (int j = 0; j < J; ++j)
      if ((j * 64 + lane) * V < D)
#pragma unroll
        for (int c = 0; c < V; ++c) q += (v[j][c] - mu) * (v[j][c] - mu);
    const float rs = 1.0f / sqrtf(wave_sum(q) / (float)D + 1e-5f);
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int d0 = (j * 64 + lane) * V;
      if (d0 < D) {
        float g[V], b[V];
        uint16_t h[V];
        load_v<V>(gam + d0, g);
        load_v<V>(bet + d0, b);
#pragma unroll
        for (int c = 0; c < V; ++c) {
          h[c] = to_bf16((v[j][c] - mu) * rs * g[c] + b[c]);
          if (yt) tile[rr * (D + 2) + d0 + c] = h[c];
        }
        store_bf16_v<V>(y + r * D + d0, h);
      }
    }
    if (lane == 0) {
      mean[r] = mu;
      rstd[r] = rs;
    }
  }
  if (!yt) return;
  __syncthreads();
  store_tile_transposed(tile, D, yt + r0, ld_t);
}

// dres += LayerNorm backward of dy; BF16 copies of the updated dres; per-wave partial sums
// of dy * xhat and dy over its 8 rows.
template <int V, int J>
__global__ __launch_bounds__(256) void k_ln_bwd(const float* dy, const float* x,
                                                const float* mean, const float* rstd,
                                                const float* gam, int D, float* dres,
                                                uint16_t* res16, uint16_t* res16t,
                                                int64_t ld_t, float* pg, float* pb) {
  extern __shared__ uint16_t tile[];   // kRows x (D + 2)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * kRows;
  float sg[J][V], sb[J][V];
#pragma unroll
  for (int j = 0; j < J; ++j)
#pragma unroll
    for (int c = 0; c < V; ++c) sg[j][c] = sb[j][c] = 0.0f;
  float gm[J][V];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int d0 = (j * 64 + lane) * V;
    if (d0 < D) load_v<V>(gam + d0, gm[j]);
  }
  // the wave's next row (dy, x, dres, statistics) is loaded while the current one is done
  float ng[J][V], nx[J][V], no[J][V], nmu = 0.0f, nrs = 0.0f;
  auto fetch = [&](int64_t r) {
    nmu = mean[r];
    nrs = rstd[r];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int d0 = (j * 64 + lane) * V;
      if (d0 < D) {
        load_v<V>(dy + r * D + d0, ng[j]);
        load_v<V>(x + r * D + d0, nx[j]);
        load_v<V>(dres + r * D + d0, no[j]);
      }
    }
  };
  fetch(r0 + wave * 8);
  for (int rr = wave * 8; rr < wave * 8 + 8; ++rr) {
    const int64_t r = r0 + rr;
    const float mu = nmu, rs = nrs;
    float g0[J][V], x0[J][V], o0[J][V];
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int c = 0; c < V; ++c) {
        g0[j][c] = ng[j][c];
        x0[j][c] = nx[j][c];
        o0[j][c] = no[j][c];
      }
    if (rr + 1 < wave * 8 + 8) fetch(r + 1);
    float dv[J][V], xh[J][V];
    float s1 = 0.0f, s2 = 0.0f;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int d0 = (j * 64 + lane) * V;
      if (d0 < D) {
#pragma unroll
        for (int c = 0; c < V; ++c) {
          const float g = g0[j][c];
          xh[j][c] = (x0[j][c] - mu) * rs;
          dv[j][c] = g * gm[j][c];
          s1 += dv[j][c];
          s2 += dv[j][c] * xh[j][c];
          sg[j][c] += g * xh[j][c];
          sb[j][c] += g;
        }
      }
    }
    s1 = wave_sum(s1) / (float)D;
    s2 = wave_sum(s2) / (float)D;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int d0 = (j * 64 + lane) * V;
      if (d0 < D) {
        float o[V];
        uint16_t h[V];
#pragma unroll
        for (int c = 0; c < V; ++c) o[c] = o0[j][c];
#pragma unroll
        for (int c = 0; c < V; ++c) {
          o[c] += rs * (dv[j][c] - s1 - xh[j][c] * s2);
          h[c] = to_bf16(o[c]);
          if (res16t) tile[rr * (D + 2) + d0 + c] = h[c];
        }
        store_v<V>(dres + r * D + d0, o);
        if (res16) store_bf16_v<V>(res16 + r * D + d0, h);
      }
    }
  }
  const int64_t prow = (r0 >> 3) + wave;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int d0 = (j * 64 + lane) * V;
    if (d0 < D) {
      store_v<V>(pg + prow * D + d0, sg[j]);
      store_v<V>(pb + prow * D + d0, sb[j]);
    }
  }
  if (!res16t) return;
  __syncthreads();
  store_tile_transposed(tile, D, res16t + r0, ld_t);
}

// ----------------------------------------------------------------------------------------
// reductions

__global__ __launch_bounds__(256) void k_sum_rows(const float* src, int64_t r, int64_t cols,
                                                  float* out, int accumulate) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int64_t i = 0; i < r; ++i) s += src[i * cols + c];
  out[c] = accumulate ? (float)(out[c] + s) : (float)s;
}

// First level of a two-level column sum: group g of G adds rows [g r / G, (g + 1) r / G)
// in order into tmp[g][c] (FP64).
__global__ __launch_bounds__(256) void k_sum_rows_groups(const float* src, int64_t r,
                                                         int64_t cols, double* tmp) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t g = blockIdx.y, G = gridDim.y;
  if (c >= cols) return;
  double s = 0.0;
  for (int64_t i = g * r / G; i < (g + 1) * r / G; ++i) s += src[i * cols + c];
  tmp[g * cols + c] = s;
}

// Second level: 64 columns per workgroup; wave w adds groups [w G / 4, (w + 1) G / 4) in
// order (loads issued together), then the four wave sums are added in wave order.
__global__ __launch_bounds__(256) void k_sum_groups(const double* tmp, int G, int64_t cols,
                                                    float* out, int accumulate) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t c = (int64_t)blockIdx.x * 64 + lane;
  double s = 0.0;
  if (c < cols)
    for (int g = wave * G / 4; g < (wave + 1) * G / 4; ++g) s += tmp[g * cols + c];
  red[wave][lane] = s;
  __syncthreads();
  if (wave != 0 || c >= cols) return;
  s = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
  out[c] = accumulate ? (float)(out[c] + s) : (float)s;
}

// One row per workgroup: thread t adds columns 8 t + 2048 j (16-byte loads, four issued
// together), then the thread sums are added by wave (shuffle tree) and the four wave sums in
// wave order.
__global__ __launch_bounds__(256) void k_rowsum_bf16(const uint16_t* src, int64_t rows,
                                                     int64_t cols, int64_t ld, float* out) {
  __shared__ double red[4];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t row = blockIdx.x;
  double s = 0.0;
  const uint16_t* p = src + row * ld;
  auto add8 = [&](const uint4& w) {
    const uint32_t q[4] = {w.x, w.y, w.z, w.w};
    float a = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      a += from_bf16((uint16_t)(q[k] & 0xFFFFu)) + from_bf16((uint16_t)(q[k] >> 16));
    s += a;
  };
  if ((cols & 7) == 0 && (ld & 7) == 0) {   // 8 values (16 bytes) per thread and load
    int64_t c = (int64_t)t * 8;
    for (; c + 3 * 2048 < cols; c += 4 * 2048) {
      uint4 w[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) w[u] = *reinterpret_cast<const uint4*>(p + c + u * 2048);
#pragma unroll
      for (int u = 0; u < 4; ++u) add8(w[u]);
    }
    for (; c < cols; c += 2048) add8(*reinterpret_cast<const uint4*>(p + c));
  } else {
    for (int64_t c = t; c < cols; c += 256) s += from_bf16(p[c]);
  }
  s = wave_sum_d(s);
  if (lane == 0) red[wave] = s;
  __syncthreads();
  if (t == 0) out[row] = (float)(((red[0] + red[1]) + red[2]) + red[3]);
}

__global__ __launch_bounds__(256) void k_sum_batches(const float* src, int B, int T, int D,
                                                     float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)T * D) return;
  double s = 0.0;
  for (int b = 0; b < B; ++b) s += src[(int64_t)b * T * D + i];
  out[i] = (float)s;
}

// ----------------------------------------------------------------------------------------
// attention rows

// Attention rows of T values: lane l holds the V-wide groups (64 j + l) of a row (V = 4 when T
// is a multiple of 256: 16-byte FP32 loads, 8-byte BF16 loads and stores).
template <int V>
__device__ __forceinline__ void load_bf16_v(const uint16_t* p, float (&v)[V]) {
  if constexpr (V == 4) {
    const uint2 w = *reinterpret_cast<const uint2*>(p);
    v[0] = from_bf16((uint16_t)(w.x & 0xFFFFu));
    v[1] = from_bf16((uint16_t)(w.x >> 16));
    v[2] = from_bf16((uint16_t)(w.y & 0xFFFFu));
    v[3] = from_bf16((uint16_t)(w.y >> 16));
  } else {
#pragma unroll
    for (int c = 0; c < V; ++c) v[c] = from_bf16(p[c]);
  }
}

template <int V>
__global__ __launch_bounds__(256) void k_attn_softmax(const float* S, int T, uint16_t* P,
                                                      uint16_t* Pt) {
  extern __shared__ uint16_t tile[];   // kRows x (T + 2)
  constexpr int kMaxJ = 1024 / (64 * V);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t z = blockIdx.y;
  const int64_t q0 = (int64_t)blockIdx.x * kRows;
  const float* Sz = S + z * T * T;
  for (int rr = wave; rr < kRows; rr += 4) {
    const float* row = Sz + (q0 + rr) * T;
    float v[kMaxJ][V];
    float mx = -INFINITY;
#pragma unroll
    for (int j = 0; j < kMaxJ; ++j) {
      const int c0 = (j * 64 + lane) * V;
      if (c0 < T) {
        load_v<V>(row + c0, v[j]);
#pragma unroll
        for (int c = 0; c < V; ++c) mx = fmaxf(mx, v[j][c]);
      }
    }
    mx = wave_max(mx);
    float sum = 0.0f;
#pragma unroll
    for (int j = 0; j < kMaxJ; ++j)
      if ((j * 64 + lane) * V < T)
#pragma unroll
        for (int c = 0; c < V; ++c) {
          v[j][c] = expf(v[j][c] - mx);
          sum += v[j][c];
        }
    const float inv = 1.0f / wave_sum(sum);
#pragma unroll
    for (int j = 0; j < kMaxJ; ++j) {
      const int c0 = (j * 64 + lane) * V;
      if (c0 < T) {
        uint16_t h[V];
#pragma unroll
        for (int c = 0; c < V; ++c) {
          h[c] = to_bf16(v[j][c] * inv);
          tile[rr * (T + 2) + c0 + c] = h[c];
        }
        store_bf16_v<V>(P + z * T * T + (q0 + rr) * T + c0, h);
      }
    }
  }
  __syncthreads();
  store_tile_transposed(tile, T, Pt + z * T * T + q0, T);
}

template <int V>
__global__ __launch_bounds__(256) void k_attn_ds(const uint16_t* P, const float* dP, int T,
                                                 float scale, uint16_t* dS, uint16_t* dSt) {
  extern __shared__ uint16_t tile[];   // kRows x (T + 2)
  constexpr int kMaxJ = 1024 / (64 * V);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t z = blockIdx.y;
  const int64_t q0 = (int64_t)blockIdx.x * kRows;
  for (int rr = wave; rr < kRows; rr += 4) {
    const int64_t o = z * T * T + (q0 + rr) * T;
    float p[kMaxJ][V], g[kMaxJ][V];
    float dot = 0.0f;
#pragma unroll
    for (int j = 0; j < kMaxJ; ++j) {
      const int c0 = (j * 64 + lane) * V;
      if (c0 < T) {
        load_bf16_v<V>(P + o + c0, p[j]);
        load_v<V>(dP + o + c0, g[j]);
#pragma unroll
        for (int c = 0; c < V; ++c) dot += p[j][c] * g[j][c];
      }
    }
    dot = wave_sum(dot);
#pragma unroll
    for (int j = 0; j < kMaxJ; ++j) {
      const int c0 = (j * 64 + lane) * V;
      if (c0 < T) {
        uint16_t h[V];
#pragma unroll
        for (int c = 0; c < V; ++c) {
          h[c] = to_bf16(scale * p[j][c] * (g[j][c] - dot));
          tile[rr * (T + 2) + c0 + c] = h[c];
        }
        store_bf16_v<V>(dS + o + c0, h);
      }
    }
  }
  __syncthreads();
  store_tile_transposed(tile, T, dSt + z * T * T + q0, T);
}

// ----------------------------------------------------------------------------------------
// patches, head output and loss

struct ImgGeom {
  int B, C, H, W, p;
  __device__ __forceinline__ int tokens() const { return (H / p) * (W / p); }
  __device__ __forceinline__ int pdim() const { return C * p * p; }
  // image element i = ((b C + c) H + y) W + x -> (token row, patch column)
  __device__ __forceinline__ void map(int64_t i, int64_t& tok, int& e) const {
    const int x = (int)(i % W);
    const int y = (int)((i / W) % H);
    const int c = (int)((i / ((int64_t)W * H)) % C);
    const int64_t b = i / ((int64_t)W * H * C);
    tok = b * tokens() + (int64_t)(y / p) * (W / p) + x / p;
    e = c * p * p + (y % p) * p + x % p;
  }
};

__global__ __launch_bounds__(256) void k_patchify(const float* x, ImgGeom G, uint16_t* pt,
                                                  uint16_t* ptt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)G.B * G.C * G.H * G.W;
  if (i >= n) return;
  int64_t tok;
  int e;
  G.map(i, tok, e);
  const uint16_t b = to_bf16(x[i]);
  const int64_t rows = (int64_t)G.B * G.tokens();
  pt[tok * G.pdim() + e] = b;
  ptt[(int64_t)e * rows + tok] = b;
}

__global__ __launch_bounds__(256) void k_head_out(const float* tok, const float* x,
                                                  const float* target, float* y, ImgGeom G,
                                                  uint16_t* dy, uint16_t* dyt, double* lossp) {
  __shared__ double red[4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)G.B * G.C * G.H * G.W;
  double r2 = 0.0;
  if (i < n) {
    int64_t t;
    int e;
    G.map(i, t, e);
    const float v = x[i] + tok[t * G.pdim() + e];
    if (y) y[i] = v;
    if (target) {
      const float r = v - target[i];
      r2 = (double)r * (double)r;
      const uint16_t b = to_bf16(2.0f * r / (float)n);
      const int64_t rows = (int64_t)G.B * G.tokens();
      dy[t * G.pdim() + e] = b;
      dyt[(int64_t)e * rows + t] = b;
    }
  }
  if (!target) return;
  r2 = wave_sum_d(r2);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r2;
  __syncthreads();
  if (threadIdx.x == 0) lossp[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// One wave: lane l adds the l-th of 64 consecutive slices of the partials in order, then lane
// 0 adds the 64 slice sums in lane order.
__global__ __launch_bounds__(64) void k_loss_final(const double* lossp, int n, double numel,
                                                  double* out) {
  __shared__ double part[64];
  const int l = threadIdx.x;
  double s = 0.0;
  for (int i = (int)((int64_t)l * n / 64); i < (int)((int64_t)(l + 1) * n / 64); ++i)
    s += lossp[i];
  part[l] = s;
  __syncthreads();
  if (l != 0) return;
  s = 0.0;
  for (int k = 0; k < 64; ++k) s += part[k];
  *out = s / numel;
}

// ----------------------------------------------------------------------------------------
// parameters

__global__ __launch_bounds__(256) void k_to_bf16(const float* w, int rows, int cols,
                                                 uint16_t* w16, uint16_t* w16t) {
  __shared__ uint16_t t[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int rr = r0 + r, cc = c0 + tx;
    if (rr < rows && cc < cols) {
      const uint16_t b = to_bf16(w[(int64_t)rr * cols + cc]);
      w16[(int64_t)rr * cols + cc] = b;
      t[r][tx] = b;
    }
  }
  __syncthreads();
  for (int c = ty; c < 32; c += 8) {
    const int cc = c0 + c, rr = r0 + tx;
    if (rr < rows && cc < cols) w16t[(int64_t)cc * rows + rr] = t[tx][c];
  }
}

// Adam (bias-corrected) on one parameter.
__device__ __forceinline__ void adam_update(float& w, float g, float& m, float& v,
                                            const AdamArgs& a) {
  m = a.b1 * m + (1.0f - a.b1) * g;
  v = a.b2 * v + (1.0f - a.b2) * g * g;
  w -= a.lr * (m / a.bc1) / (sqrtf(v / a.bc2) + a.eps);
}

// The whole optimizer step in one grouped launch over a segment table.  A matrix segment is
// done in tiles of kAdamTile x kAdamTile parameters: Adam on 16-byte groups of a row, then the
// tile's BF16 copy row-major and, through LDS, transposed.  A plain range is done in chunks of
// kAdamChunk parameters.
__global__ __launch_bounds__(256) void k_adam_bf16(const AdamSeg* segs, int nseg, float* w,
                                                   const float* g, float* m, float* v,
                                                   AdamArgs a) {
  __shared__ uint16_t t[kAdamTile][kAdamTile + 2];
  const int blk = (int)blockIdx.x;
  int lo = 0, hi = nseg - 1;          // the last segment that starts at or before blk
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].blk0 <= blk) lo = mid;
    else hi = mid - 1;
  }
  const AdamSeg sg = segs[lo];
  const int local = blk - sg.blk0;
  if (!sg.w16) {
    const int64_t i0 = sg.off + (int64_t)local * kAdamChunk, end = sg.off + sg.len;
    for (int j = 0; j < kAdamChunk / 256; ++j) {
      const int64_t i = i0 + j * 256 + threadIdx.x;
      if (i < end) {
        float wi = w[i], mi = m[i], vi = v[i];
        adam_update(wi, g[i], mi, vi, a);
        w[i] = wi;
        m[i] = mi;
        v[i] = vi;
      }
    }
    return;
  }
  const int r0 = (local / sg.tiles_c) * kAdamTile, c0 = (local % sg.tiles_c) * kAdamTile;
  const int tc = (threadIdx.x & 15) * 4, tr = threadIdx.x >> 4;   // 16 threads per tile row
  for (int p = 0; p < kAdamTile / 16; ++p) {
    const int rl = p * 16 + tr, r = r0 + rl, c = c0 + tc;
    if (r < sg.rows && c < sg.cols) {   // cols % 4 == 0: the four columns are inside
      const int64_t i = sg.off + (int64_t)r * sg.cols + c;
      float4 W = *reinterpret_cast<const float4*>(w + i);
      float4 M = *reinterpret_cast<const float4*>(m + i);
      float4 V = *reinterpret_cast<const float4*>(v + i);
      const float4 G = *reinterpret_cast<const float4*>(g + i);
      adam_update(W.x, G.x, M.x, V.x, a);
      adam_update(W.y, G.y, M.y, V.y, a);
      adam_update(W.z, G.z, M.z, V.z, a);
      adam_update(W.w, G.w, M.w, V.w, a);
      *reinterpret_cast<float4*>(w + i) = W;
      *reinterpret_cast<float4*>(m + i) = M;
      *reinterpret_cast<float4*>(v + i) = V;
      const uint16_t h[4] = {to_bf16(W.x), to_bf16(W.y), to_bf16(W.z), to_bf16(W.w)};
      *reinterpret_cast<uint2*>(sg.w16 + (int64_t)r * sg.cols + c) =
          make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16));
#pragma unroll
      for (int k = 0; k < 4; ++k) t[rl][tc + k] = h[k];
    }
  }
  __syncthreads();
  // column c of the tile is rows r0.. of w16t's row c: two rows per 4-byte store (rows even)
  for (int q = threadIdx.x; q < kAdamTile * (kAdamTile / 2); q += 256) {
    const int cl = q / (kAdamTile / 2), pr = q % (kAdamTile / 2);
    const int c = c0 + cl, r = r0 + 2 * pr;
    if (c < sg.cols && r < sg.rows)
      *reinterpret_cast<uint32_t*>(sg.w16t + (int64_t)c * sg.rows + r) =
          (uint32_t)t[2 * pr][cl] | ((uint32_t)t[2 * pr + 1][cl] << 16);
  }
}

// ----------------------------------------------------------------------------------------
// host launchers

namespace {
inline unsigned blocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// Compute units of the current device (looked up once per device).
int device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
      n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}
}

hipError_t launch_vgemm(const VGemm& g0, int batch, hipStream_t s) {
  VGemm g = g0;
  if (g.K % 32 != 0 || g.K <= 0) return hipErrorInvalidValue;
  if (g.splits < 1) g.splits = 1;
  if (g.splits > 1 && (g.kchunk % 32 != 0 || g.kchunk * g.splits < g.K || batch != 1))
    return hipErrorInvalidValue;
  auto go = [&](auto kern, int bm, int bn, int bk, int threads) {
    if (g.M % bm || g.N % bn || g.K % bk || (g.splits > 1 && g.kchunk % bk))
      return hipErrorInvalidValue;
    g.tiles_n = g.N / bn;
    hipLaunchKernelGGL(kern, dim3((unsigned)((g.M / bm) * (g.N / bn) * g.splits),
                                  (unsigned)batch),
                       dim3(threads), 0, s, g);
    return hipGetLastError();
  };
  int tile = g.tile;
  if (tile == kTileAuto) {
    const int64_t keff = g.splits > 1 ? g.kchunk : g.K;
    const bool m128 = g.M % 128 == 0 && g.N % 128 == 0, m64 = g.M % 64 == 0 && g.N % 64 == 0;
    if (keff <= 256 && m64) tile = kTile64;
    else if (m128 && keff % 64 == 0) tile = keff >= 4096 ? kTile128pp : kTile128;
    else if (m64) tile = kTile64;
    else tile = kTile32;
    // 256 x 128 for unsplit contractions of 2048 or more where its rounds of resident
    // workgroups (two per CU) are at least as full as those of 128 x 128 (three per CU); on
    // shorter contractions its k-steps of 32 starve it
    if ((tile == kTile128 || tile == kTile128pp) && g.splits == 1 && batch == 1 &&
        g.M % 256 == 0 && g.K >= 2048) {
      const int64_t cus = device_cus();
      auto fill = [&](int64_t tiles, int64_t slots) {
        return (double)tiles / (double)(((tiles + slots - 1) / slots) * slots);
      };
      const int64_t t256 = (int64_t)(g.M / 256) * (g.N / 128), t128 = 2 * t256;
      if (t256 >= 2 * cus && fill(t256, 2 * cus) >= fill(t128, 3 * cus)) tile = kTile256;
    }
  }
  switch (tile) {
    case kTile128: return go(k_vgemm<2, 2, 2, 2, 64, 1>, 128, 128, 64, 256);
    case kTile128pp: return go(k_vgemm<2, 2, 2, 2, 64, 2>, 128, 128, 64, 256);
    case kTile64: return go(k_vgemm<2, 2, 1, 1, 32, 2>, 64, 64, 32, 256);
    case kTile32: return go(k_vgemm<1, 1, 1, 1, 32, 2>, 32, 32, 32, 64);
    case kTile256: return go(k_vgemm<4, 2, 2, 2, 32, 2>, 256, 128, 32, 512);
    default: return hipErrorInvalidValue;
  }
}

hipError_t set_vit_smem_limit(int D, int T) {
  const int ln = kRows * (D + 2) * 2, rows = kRows * (T + 2) * 2;
  hipError_t e = hipSuccess;
  auto set = [&](const void* f, int bytes) {
    if (e == hipSuccess && bytes > 64 * 1024)
      e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  };
  set(reinterpret_cast<const void*>(k_ln_fwd<4, 1>), ln);
  set(reinterpret_cast<const void*>(k_ln_fwd<4, 2>), ln);
  set(reinterpret_cast<const void*>(k_ln_fwd<4, 4>), ln);
  set(reinterpret_cast<const void*>(k_ln_fwd<4, 8>), ln);
  set(reinterpret_cast<const void*>(k_ln_fwd<1, 32>), ln);
  set(reinterpret_cast<const void*>(k_ln_bwd<4, 1>), ln);
  set(reinterpret_cast<const void*>(k_ln_bwd<4, 2>), ln);
  set(reinterpret_cast<const void*>(k_ln_bwd<4, 4>), ln);
  set(reinterpret_cast<const void*>(k_ln_bwd<4, 8>), ln);
  set(reinterpret_cast<const void*>(k_ln_bwd<1, 32>), ln);
  set(reinterpret_cast<const void*>(k_attn_softmax<4>), rows);
  set(reinterpret_cast<const void*>(k_attn_softmax<1>), rows);
  set(reinterpret_cast<const void*>(k_attn_ds<4>), rows);
  set(reinterpret_cast<const void*>(k_attn_ds<1>), rows);
  return e;
}

// LayerNorm kernels: V = 4 with J = D / 256 for the usual widths, else V = 1 up to 2048.
#define VIT_LN_DISPATCH(KERN, ...)                                                             \
  if (D % 256 == 0 && D / 256 == 1) return go(KERN<4, 1>, __VA_ARGS__);                       \
  if (D % 256 == 0 && D / 256 == 2) return go(KERN<4, 2>, __VA_ARGS__);                       \
  if (D % 256 == 0 && D / 256 == 4) return go(KERN<4, 4>, __VA_ARGS__);                       \
  if (D % 256 == 0 && D / 256 == 8) return go(KERN<4, 8>, __VA_ARGS__);                       \
  return go(KERN<1, 32>, __VA_ARGS__);

hipError_t launch_ln_fwd(const float* x, int64_t rows, int D, const float* gamma,
                         const float* beta, uint16_t* y, uint16_t* yt, int64_t ld_t,
                         float* mean, float* rstd, hipStream_t s) {
  if (rows % kRows != 0 || D % 64 != 0 || D > 2048) return hipErrorInvalidValue;
  const size_t shm = yt ? (size_t)kRows * (D + 2) * 2 : 0;
  auto go = [&](auto kern, int) {
    hipLaunchKernelGGL(kern, dim3((unsigned)(rows / kRows)), dim3(64 * kLnFwdWaves), shm, s, x,
                       D, gamma, beta, y, yt, ld_t, mean, rstd);
    return hipGetLastError();
  };
  VIT_LN_DISPATCH(k_ln_fwd, 0)
}

hipError_t launch_ln_bwd(const float* dy, const float* x, const float* mean, const float* rstd,
                         const float* gamma, int64_t rows, int D, float* dres,
                         uint16_t* res16, uint16_t* res16t, int64_t ld_t, float* pg,
                         float* pb, hipStream_t s) {
  if (rows % kRows != 0 || D % 64 != 0 || D > 2048) return hipErrorInvalidValue;
  const size_t shm = res16t ? (size_t)kRows * (D + 2) * 2 : 0;
  auto go = [&](auto kern, int) {
    hipLaunchKernelGGL(kern, dim3((unsigned)(rows / kRows)), dim3(256), shm, s, dy, x, mean,
                       rstd, gamma, D, dres, res16, res16t, ld_t, pg, pb);
    return hipGetLastError();
  };
  VIT_LN_DISPATCH(k_ln_bwd, 0)
}

hipError_t launch_sum_rows(const float* src, int64_t r, int64_t cols, float* out, bool accumulate,
                           hipStream_t s, double* tmp) {
  if (tmp && r >= 64) {
    const int G = kSumGroups;
    hipLaunchKernelGGL(k_sum_rows_groups, dim3(blocks(cols, 256), G), dim3(256), 0, s, src, r,
                       cols, tmp);
    hipLaunchKernelGGL(k_sum_groups, dim3(blocks(cols, 64)), dim3(256), 0, s, tmp, G, cols, out,
                       accumulate ? 1 : 0);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_sum_rows, dim3(blocks(cols, 256)), dim3(256), 0, s, src, r, cols, out,
                     accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_rowsum_bf16(const uint16_t* src, int64_t rows, int64_t cols, int64_t ld,
                              float* out, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rowsum_bf16, dim3((unsigned)rows), dim3(256), 0, s, src, rows, cols, ld,
                     out);
  return hipGetLastError();
}

hipError_t launch_sum_batches(const float* src, int B, int T, int D, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_batches, dim3(blocks((int64_t)T * D, 256)), dim3(256), 0, s, src, B,
                     T, D, out);
  return hipGetLastError();
}

hipError_t launch_attn_softmax(const float* S, int64_t Z, int T, uint16_t* P, uint16_t* Pt,
                               hipStream_t s) {
  if (T % 64 != 0 || T > 1024) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(T / kRows), (unsigned)Z);
  const size_t shm = (size_t)kRows * (T + 2) * 2;
  if (T % 256 == 0)
    hipLaunchKernelGGL(k_attn_softmax<4>, grid, dim3(256), shm, s, S, T, P, Pt);
  else
    hipLaunchKernelGGL(k_attn_softmax<1>, grid, dim3(256), shm, s, S, T, P, Pt);
  return hipGetLastError();
}

hipError_t launch_attn_ds(const uint16_t* P, const float* dP, int64_t Z, int T, float scale,
                          uint16_t* dS, uint16_t* dSt, hipStream_t s) {
  if (T % 64 != 0 || T > 1024) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(T / kRows), (unsigned)Z);
  const size_t shm = (size_t)kRows * (T + 2) * 2;
  if (T % 256 == 0)
    hipLaunchKernelGGL(k_attn_ds<4>, grid, dim3(256), shm, s, P, dP, T, scale, dS, dSt);
  else
    hipLaunchKernelGGL(k_attn_ds<1>, grid, dim3(256), shm, s, P, dP, T, scale, dS, dSt);
  return hipGetLastError();
}

hipError_t launch_patchify(const float* x, int B, int C, int H, int W, int p, uint16_t* pt,
                           uint16_t* ptt, hipStream_t s) {
  const ImgGeom G{B, C, H, W, p};
  const int64_t n = (int64_t)B * C * H * W;
  hipLaunchKernelGGL(k_patchify, dim3(blocks(n, 256)), dim3(256), 0, s, x, G, pt, ptt);
  return hipGetLastError();
}

int loss_blocks(int64_t n) { return (int)((n + 255) / 256); }

hipError_t launch_head_out(const float* tok, const float* x, const float* target, float* y,
                           int B, int C, int H, int W, int p, uint16_t* dy, uint16_t* dyt,
                           double* lossp, hipStream_t s) {
  const ImgGeom G{B, C, H, W, p};
  const int64_t n = (int64_t)B * C * H * W;
  hipLaunchKernelGGL(k_head_out, dim3((unsigned)loss_blocks(n)), dim3(256), 0, s, tok, x, target,
                     y, G, dy, dyt, lossp);
  return hipGetLastError();
}

hipError_t launch_loss_final(const double* lossp, int n, double numel, double* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, lossp, n, numel, out);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float* w, int rows, int cols, uint16_t* w16, uint16_t* w16t,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks(cols, 32), blocks(rows, 32)), dim3(256), 0, s, w,
                     rows, cols, w16, w16t);
  return hipGetLastError();
}

hipError_t launch_adam_bf16(const AdamSeg* segs, int nseg, int nblocks, float* w,
                           const float* g, float* m, float* v, const AdamArgs& a,
                           hipStream_t s) {
  if (nseg <= 0 || nblocks <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_adam_bf16, dim3((unsigned)nblocks), dim3(256), 0, s, segs, nseg, w, g, m,
                     v, a);
  return hipGetLastError();
}

}  // namespace vit
}  // namespace ensf
