// MFMA tile machinery shared by the EnSF kernels and the transformer surrogate's GEMMs
// (CDNA4 / gfx950): LDS tile layouts, the k-loop with LDS ping-pong, operand loaders and
// the XCD-aware tile order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ensf_internal.h"

namespace ensf {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Workgroups are dispatched round-robin over the 8 XCDs of the device; this bijection
// gives each XCD a contiguous range of logical tiles, so tiles that share operands
// (adjacent in the logical order) share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int x = b & 7, local = b >> 3, per = G >> 3, rem = G & 7;
  return x * per + min(x, rem) + local;
}

// ----------------------------------------------------------------------------------------
// MFMA tile machinery.  A workgroup of WGM x WGN waves computes a BM x BN tile with
// BM = WGM*TM*32, BN = WGN*TN*32; each wave owns TM x TN blocks of 32 x 32.
// 32x32 accumulator layout (both MFMA kinds): lane l, register r holds
// row (r/4)*8 + (l/32)*4 + r%4, column l%32.

// LDS tile of the A (BM rows) and B (BN rows) operands of one k-step of BK.  Operands are
// row-major ([row][k], unpadded, 16-byte chunks permuted by chunk_swizzle) so that a lane
// reads consecutive k values of its row as one 16-byte access: 8 values (BF16) or 4 (FP32).
// AK: the FP32 A operand is k-major instead ([k][row], rows padded to BM + 8 floats, which
// puts the k-rows read by the two half-waves in opposite halves of the banks); used where
// the operand's rows are contiguous in global memory (X in W.X).
template <int PREC, int BM, int BN, int BK, bool AK = false>
struct TileSmem {
  static constexpr int LDF_A = BM + 8;                      // k-major FP32 A
  static constexpr int LDH = BK;                            // row-major rows (elements)
  static constexpr int kAFloats = AK ? BK * LDF_A : BM * BK;
  static constexpr int kFp32Bytes = (kAFloats + BN * BK) * 4;
  // BF16 tiles: A hi, then (split form only) A lo, then B hi, B lo; element offsets
  static constexpr int kLo = PREC == kBF16X3 ? 1 : 0;
  static constexpr int kALo = BM * LDH;
  static constexpr int kBHi = (1 + kLo) * BM * LDH;
  static constexpr int kBLo = kBHi + BN * LDH;
  static constexpr int kBf16Bytes = (BM + BN) * LDH * 2 * (1 + kLo);
  static constexpr int kBytes = PREC == kFP32 ? kFp32Bytes : kBf16Bytes;
};

// Position, within row r of a row-major LDS tile whose rows are ROW_BYTES long (at most
// 256), of the row's 16-byte chunk `chunk`.  Chunks are XOR-permuted by the row's position
// among the 256-byte bank spans: a quarter-wave reading one chunk of 16 consecutive rows, and
// lanes writing whole consecutive rows, then touch every bank once.
template <int ROW_BYTES>
__device__ __forceinline__ int chunk_swizzle(int r, int chunk) {
  constexpr int kChunks = ROW_BYTES / 16, kRowsPerSpan = 256 / ROW_BYTES;
  return chunk ^ ((r / kRowsPerSpan) & (kChunks - 1));
}
// element offsets of a chunk: BF16 rows of BK elements (8 per chunk), FP32 rows (4 per chunk)
template <int BK>
__device__ __forceinline__ int bf16_chunk_swizzle(int r, int chunk) {
  return chunk_swizzle<BK * 2>(r, chunk) * 8;
}
template <int BK>
__device__ __forceinline__ int f32_chunk_swizzle(int r, int chunk) {
  return chunk_swizzle<BK * 4>(r, chunk) * 4;
}

template <int PREC, int WGM, int WGN, int TM, int TN, int BK, bool AK = false>
__device__ __forceinline__ void mfma_block_compute(const char* smem, f32x16_t (&acc)[TM][TN]) {
  constexpr int BM = WGM * TM * 32, BN = WGN * TN * 32;
  using S = TileSmem<PREC, BM, BN, BK, AK>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  if constexpr (PREC == kFP32) {
    // Per group of 8 k: lanes 0-31 hold k = kk..kk+3 of their row, lanes 32-63 k = kk+4..kk+7
    // (one 16-byte chunk); MFMA m (2 k values: one per half-wave) takes component m.  A and
    // B use the same assignment, so the 4 MFMAs sum over the 8 k values.
    const float* sA = reinterpret_cast<const float*>(smem);
    const float* sB = sA + S::kAFloats;
    const int half = lane >> 5;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 8) {
      f32x4 a[TM], b[TN];
#pragma unroll
      for (int tm = 0; tm < TM; ++tm) {
        const int r = wm * TM * 32 + tm * 32 + (lane & 31);
        if constexpr (AK) {
          const float* col = sA + (kk + 4 * half) * S::LDF_A + r;
          a[tm] = f32x4{col[0], col[S::LDF_A], col[2 * S::LDF_A], col[3 * S::LDF_A]};
        } else {
          a[tm] = *reinterpret_cast<const f32x4*>(sA + r * BK +
                                                 f32_chunk_swizzle<BK>(r, kk / 4 + half));
        }
      }
#pragma unroll
      for (int tn = 0; tn < TN; ++tn) {
        const int r = wn * TN * 32 + tn * 32 + (lane & 31);
        b[tn] = *reinterpret_cast<const f32x4*>(sB + r * BK +
                                               f32_chunk_swizzle<BK>(r, kk / 4 + half));
      }
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
          for (int tn = 0; tn < TN; ++tn)
            acc[tm][tn] =
                __builtin_amdgcn_mfma_f32_32x32x2f32(a[tm][m], b[tn][m], acc[tm][tn], 0, 0, 0);
    }
  } else {
    const uint16_t* sAh = reinterpret_cast<const uint16_t*>(smem);
    const uint16_t* sAl = sAh + S::kALo;
    const uint16_t* sBh = sAh + S::kBHi;
    const uint16_t* sBl = sAh + S::kBLo;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      bf16x8_t ah[TM], al[TM], bh[TN], bl[TN];
      const int kc = kk / 8 + (lane >> 5);   // 16-byte chunk of the row
#pragma unroll
      for (int tm = 0; tm < TM; ++tm) {
        const int r = wm * TM * 32 + tm * 32 + (lane & 31);
        const int o = r * S::LDH + bf16_chunk_swizzle<BK>(r, kc);
        ah[tm] = *reinterpret_cast<const bf16x8_t*>(sAh + o);
        if constexpr (PREC == kBF16X3) al[tm] = *reinterpret_cast<const bf16x8_t*>(sAl + o);
      }
#pragma unroll
      for (int tn = 0; tn < TN; ++tn) {
        const int r = wn * TN * 32 + tn * 32 + (lane & 31);
        const int o = r * S::LDH + bf16_chunk_swizzle<BK>(r, kc);
        bh[tn] = *reinterpret_cast<const bf16x8_t*>(sBh + o);
        if constexpr (PREC == kBF16X3) bl[tn] = *reinterpret_cast<const bf16x8_t*>(sBl + o);
      }
#pragma unroll
      for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
          acc[tm][tn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[tm], bh[tn], acc[tm][tn], 0, 0, 0);
          if constexpr (PREC == kBF16X3) {
            acc[tm][tn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[tm], bl[tn], acc[tm][tn], 0, 0, 0);
            acc[tm][tn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[tm], bh[tn], acc[tm][tn], 0, 0, 0);
          }
        }
    }
  }
}

// The k loop of a tile.  load(kb) fetches the k-step starting at kb from global memory
// into registers, store(stage) writes those registers into one LDS stage.  With PP (two
// stages fit) the loop ping-pongs between two stages: one barrier per k-step, and the LDS
// store of step k+1 overlaps the other waves' MFMAs on step k while the global loads of
// step k+2 are in flight.  Otherwise one stage is refilled between two barriers.
template <int PREC, int WGM, int WGN, int TM, int TN, int BK, bool PP, bool AK, class Load,
          class Store>
__device__ __forceinline__ void tile_k_loop(char* smem, int64_t kbeg, int64_t kend, Load&& load,
                                            Store&& store, f32x16_t (&acc)[TM][TN]) {
  constexpr int STAGE = TileSmem<PREC, WGM * TM * 32, WGN * TN * 32, BK, AK>::kBytes;
  if (kbeg >= kend) return;
  load(kbeg);
  if constexpr (PP) {
    store(smem);
    if (kbeg + BK < kend) load(kbeg + BK);
    __syncthreads();
    int cur = 0;
    for (int64_t kb = kbeg; kb < kend; kb += BK) {
      mfma_block_compute<PREC, WGM, WGN, TM, TN, BK, AK>(smem + cur * STAGE, acc);
      if (kb + BK < kend) {
        store(smem + (cur ^ 1) * STAGE);
        if (kb + 2 * BK < kend) load(kb + 2 * BK);
      }
      __syncthreads();
      cur ^= 1;
    }
  } else {
    for (int64_t kb = kbeg; kb < kend; kb += BK) {
      __syncthreads();
      store(smem);
      __syncthreads();
      if (kb + BK < kend) load(kb + BK);
      mfma_block_compute<PREC, WGM, WGN, TM, TN, BK, AK>(smem, acc);
    }
  }
}

// With ST = 2 two LDS stages are used when they fit in this budget (leaves room for 1-2
// workgroups); ST = 1 keeps one stage, which halves the LDS per workgroup and can raise the
// number of resident workgroups.  Which is faster depends on the shape (the tuner decides).
constexpr int kPingPongBytes = 96 * 1024;

// Operand loaders.  "Kmaj" sources are row-major with k contiguous (Z, X for the Gram,
// W for W.X); the FP32 W.X operand X is row-major with the output column contiguous.
// init() fixes a thread's base address once; load(k0) issues global (not flat) vector loads
// at base + k0 (flat loads would share the LDS wait counter with the fragment reads), and
// consecutive slots of a thread are a constant row stride apart.

template <typename T>
__device__ __forceinline__ T gload(const T* p) {
  typedef const __attribute__((address_space(1))) T* gptr_t;
  return *(gptr_t)p;
}

template <typename T>
__device__ __forceinline__ void gstore(T* p, const T& v) {
  typedef __attribute__((address_space(1))) T* gptr_t;
  *(gptr_t)p = v;
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// RNE split of two FP32 values into packed bf16 hi and lo pairs (x - hi is exact in FP32).
__device__ __forceinline__ void split_pair(f32x2 x, uint32_t& hi, uint32_t& lo) {
  hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(x, bf16x2_t));
  const f32x2 hf = {__builtin_bit_cast(float, hi << 16), __builtin_bit_cast(float, hi & 0xFFFF0000u)};
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(x - hf, bf16x2_t));
}

// FP32 source, k contiguous, ROWS x BK tile -> registers (f32x4 per slot).
template <int ROWS, int NT, int BK>
struct F32KmajLoad {
  static constexpr int kSlots = ROWS * BK / 4 / NT;
  static constexpr int kRowStep = NT / (BK / 4);
  static_assert(kSlots * NT * 4 == ROWS * BK, "tile must split evenly");
  f32x4 v[kSlots];
  const float* base;
  int64_t step;
  __device__ __forceinline__ void init(const float* src, int64_t ld, int64_t row0) {
    base = src + (row0 + threadIdx.x / (BK / 4)) * ld + (threadIdx.x % (BK / 4)) * 4;
    step = kRowStep * ld;
  }
  __device__ __forceinline__ void load(int64_t k0) {
    const float* p = base + k0;
#pragma unroll
    for (int it = 0; it < kSlots; ++it) v[it] = gload(reinterpret_cast<const f32x4*>(p + it * step));
  }
  // FP32 smem, row-major [row][k] with swizzled 16-byte chunks (the slot is one chunk)
  __device__ __forceinline__ void store_rows(float* s) const {
    const int r = threadIdx.x / (BK / 4), c = threadIdx.x % (BK / 4);
#pragma unroll
    for (int it = 0; it < kSlots; ++it) {
      const int row = r + it * kRowStep;
      *reinterpret_cast<f32x4*>(s + row * BK + f32_chunk_swizzle<BK>(row, c)) = v[it];
    }
  }
  // split to bf16 hi/lo, row-major [row][k]
  template <bool LO>
  __device__ __forceinline__ void store_split(uint16_t* sh, uint16_t* sl, int lds) const {
    const int r = threadIdx.x / (BK / 4), c = threadIdx.x % (BK / 4);
#pragma unroll
    for (int it = 0; it < kSlots; ++it) {
      uint32_t h01, l01, h23, l23;
      split_pair(f32x2{v[it].x, v[it].y}, h01, l01);
      split_pair(f32x2{v[it].z, v[it].w}, h23, l23);
      const int row = r + it * kRowStep;   // c: 8-byte half c % 2 of 16-byte chunk c / 2
      const int o = row * lds + bf16_chunk_swizzle<BK>(row, c >> 1) + (c & 1) * 4;
      *reinterpret_cast<u32x2*>(sh + o) = u32x2{h01, h23};
      if constexpr (LO) *reinterpret_cast<u32x2*>(sl + o) = u32x2{l01, l23};
    }
  }
};

// FP32 source with the tile's columns contiguous: BK rows (k) x COLS -> [k][col] smem.
template <int COLS, int NT, int BK>
struct F32NmajLoad {
  static constexpr int kSlots = COLS * BK / 4 / NT;
  static constexpr int kRowStep = NT / (COLS / 4);
  static_assert(kSlots * NT * 4 == COLS * BK, "tile must split evenly");
  f32x4 v[kSlots];
  const float* base;
  int64_t ld;
  __device__ __forceinline__ void init(const float* src, int64_t ld_, int64_t col0) {
    ld = ld_;
    base = src + (int64_t)(threadIdx.x / (COLS / 4)) * ld + col0 + (threadIdx.x % (COLS / 4)) * 4;
  }
  __device__ __forceinline__ void load(int64_t k0) {
    const float* p = base + k0 * ld;
    const int64_t step = kRowStep * ld;
#pragma unroll
    for (int it = 0; it < kSlots; ++it) v[it] = gload(reinterpret_cast<const f32x4*>(p + it * step));
  }
  __device__ __forceinline__ void store(float* s, int lds) const {
    const int r = threadIdx.x / (COLS / 4), c = threadIdx.x % (COLS / 4);
#pragma unroll
    for (int it = 0; it < kSlots; ++it)
      *reinterpret_cast<f32x4*>(s + (r + it * kRowStep) * lds + c * 4) = v[it];
  }
};

// BF16 source pair (hi, lo), k contiguous, ROWS x BK tile, 16-byte vectors.
template <int ROWS, int NT, bool LO, int BK>
struct Bf16KmajLoad {
  static constexpr int kSlots = (ROWS * BK / 8 + NT - 1) / NT;
  static constexpr int kVec = ROWS * BK / 8;
  static constexpr int kRowStep = NT / (BK / 8);
  u32x4 h[kSlots], l[kSlots];
  const uint16_t* bh;
  const uint16_t* bl;
  int64_t step;
  __device__ __forceinline__ void init(const uint16_t* srch, const uint16_t* srcl, int64_t ld,
                                       int64_t row0) {
    const int64_t off = (row0 + threadIdx.x / (BK / 8)) * ld + (threadIdx.x % (BK / 8)) * 8;
    bh = srch + off;
    bl = srcl + off;
    step = kRowStep * ld;
  }
  __device__ __forceinline__ void load(int64_t k0) {
#pragma unroll
    for (int it = 0; it < kSlots; ++it) {
      if (kVec % NT == 0 || (int)threadIdx.x + it * NT < kVec) {
        h[it] = gload(reinterpret_cast<const u32x4*>(bh + k0 + it * step));
        if constexpr (LO) l[it] = gload(reinterpret_cast<const u32x4*>(bl + k0 + it * step));
      }
    }
  }
  __device__ __forceinline__ void store(uint16_t* sh, uint16_t* sl, int lds) const {
    const int r = threadIdx.x / (BK / 8), c = threadIdx.x % (BK / 8);
#pragma unroll
    for (int it = 0; it < kSlots; ++it) {
      if (kVec % NT == 0 || (int)threadIdx.x + it * NT < kVec) {
        const int row = r + it * kRowStep;
        const int o = row * lds + bf16_chunk_swizzle<BK>(row, c);
        *reinterpret_cast<u32x4*>(sh + o) = h[it];
        if constexpr (LO) *reinterpret_cast<u32x4*>(sl + o) = l[it];
      }
    }
  }
};

}  // namespace ensf
