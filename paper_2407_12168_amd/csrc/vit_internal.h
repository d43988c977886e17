// Internal descriptors and launchers of the transformer surrogate's kernels (vit_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ensf {
namespace vit {

// A BF16 operand with k contiguous: element (row r, k) of batch (zb, zh) at
// p + zb * sb + zh * sh + r * ld + k.
struct VMat {
  const uint16_t* p;
  int64_t ld, sb, sh;
};

// C = alpha * A B^T (M x N, contraction over K) on BF16 MFMA with FP32 accumulation, batch
// z = zb * nh + zh over grid.y, followed by an elementwise epilogue on v = alpha acc:
//   v += bias[n] (if bias), v += add[(m mod add_rows) * ld_add + n] (if add; add_rows 0 = M,
//   otherwise a multiple of 4)
//   f32  (if set) <- v                              (before the activation)
//   act 1: gd[m * ld_gin + n] <- bf16(gelu'(v)) (if gd), then v = gelu(v);
//   act 2: v *= gin[m * ld_gin + n] (a BF16 derivative written by an act 1 product)
//   b16  (if set) <- bf16(v),  b16t (if set) <- bf16(v) at b16t[n * ld_t + m] (transposed)
// add and gin are used only by unbatched products.
struct VGemm {
  VMat A, B;
  int M, N, K, nh, tiles_n;
  float alpha;
  const float* bias;
  const float* add;
  int64_t ld_add;
  int add_rows;
  float* f32;
  int64_t ld_f32, sb_f32, sh_f32;
  uint16_t* b16;
  int64_t ld_b16, sb_b16, sh_b16;
  uint16_t* b16t;
  int64_t ld_t, sb_t, sh_t;
  int act;
  const uint16_t* gin;
  uint16_t* gd;
  int64_t ld_gin;
  // split-K (unbatched products with only the FP32 output): split s of the contraction,
  // [s * kchunk, (s + 1) * kchunk), writes its partial product to f32 + s * part_stride
  int64_t kchunk, part_stride;
  int splits;
  int tile;   // VTile; kTileAuto chooses by shape
};

// Tile shapes (rows x columns of C, k-step, LDS stages), four waves unless noted.  Measured on
// the 64^2 Table II products: 256 x 128 and 256 x 256 tiles were slower than these.
enum VTile : int {
  kTileAuto = 0,
  kTile128 = 1,         // 128 x 128, waves of 64 x 64, k-step 64, one stage
  kTile128pp = 2,       // 128 x 128, k-step 64, two stages
  kTile64 = 3,          // 64 x 64, waves of 32 x 32, k-step 32, two stages
  kTile32 = 4,          // 32 x 32 on one wave, k-step 32
  kTile256 = 5,         // 256 x 128 on eight waves of 64 x 64, k-step 32, two stages
  kNumTiles = 6
};

// M and N must be multiples of the chosen tile, K (and kchunk, when split) of its k-step.
// Automatic choice by the contraction length per workgroup (kchunk when split): up to 256
// (attention, patch embedding) 64 x 64 tiles, whose short k loops need the extra
// workgroups; otherwise 128 x 128 where K is a multiple of 64 (two stages from 4096 on),
// else 64 x 64, else 32 x 32.  An unsplit, unbatched 128 x 128 choice with K >= 2048 becomes
// 256 x 128 when that tile (two resident per CU) fills at least two per CU and its rounds of
// resident workgroups are at least as full as those of 128 x 128 (three per CU).
hipError_t launch_vgemm(const VGemm& g, int batch, hipStream_t s);

// rows x D FP32 -> LayerNorm (population variance, eps 1e-5) -> BF16 rows y (ld D) and,
// if yt, transposed (yt[d * ld_t + row]); mean and 1/std per row.  rows % 32 == 0.
hipError_t launch_ln_fwd(const float* x, int64_t rows, int D, const float* gamma,
                         const float* beta, uint16_t* y, uint16_t* yt, int64_t ld_t,
                         float* mean, float* rstd, hipStream_t s);
// LayerNorm backward for dy (FP32 rows x D, the gradient of the LayerNorm output):
// dres += dx; then, if set, BF16 copies of the updated dres, row-major (res16) and transposed
// (res16t, ld_t); per group of 8 rows the partial sums of dy * xhat and dy (for gamma and
// beta) into pg, pb ([rows / 8] x D).  rows % 32 == 0.
hipError_t launch_ln_bwd(const float* dy, const float* x, const float* mean, const float* rstd,
                         const float* gamma, int64_t rows, int D, float* dres,
                         uint16_t* res16, uint16_t* res16t, int64_t ld_t, float* pg,
                         float* pb, hipStream_t s);
// out[c] (+)= sum over the r rows of src (FP32, r x cols, fixed order, FP64 accumulation).
// With tmp (kSumGroups x cols doubles) and r >= 64 the rows are added in kSumGroups
// consecutive groups first, then the group sums in order.
constexpr int kSumGroups = 64;
hipError_t launch_sum_rows(const float* src, int64_t r, int64_t cols, float* out, bool accumulate,
                           hipStream_t s, double* tmp = nullptr);
// out[i] = sum over the cols entries of row i of a BF16 matrix (ld), FP64 accumulation.
hipError_t launch_rowsum_bf16(const uint16_t* src, int64_t rows, int64_t cols, int64_t ld,
                              float* out, hipStream_t s);
// Attention weights: rows of S (FP32, Z x T x T) -> softmax -> P (BF16) and P^T per batch.
hipError_t launch_attn_softmax(const float* S, int64_t Z, int T, uint16_t* P, uint16_t* Pt,
                               hipStream_t s);
// dS = scale * P o (dP - rowsum(dP o P)) (BF16, and transposed per batch).
hipError_t launch_attn_ds(const uint16_t* P, const float* dP, int64_t Z, int T, float scale,
                          uint16_t* dS, uint16_t* dSt, hipStream_t s);
// x (B x C x H x W FP32) -> patch rows (B*T x Pd BF16) and their transpose (Pd x B*T).
hipError_t launch_patchify(const float* x, int B, int C, int H, int W, int p, uint16_t* pt,
                           uint16_t* ptt, hipStream_t s);
// tok (B*T x Pd FP32, the head's output) -> y = x + unpatchify(tok) (if y); with a target:
// r = y - target, dY = 2 r / numel as BF16 patch rows and their transpose, and per-block
// partial sums of r^2 into lossp (FP64, n_blocks entries, see launch_loss_blocks).
hipError_t launch_head_out(const float* tok, const float* x, const float* target, float* y,
                           int B, int C, int H, int W, int p, uint16_t* dy, uint16_t* dyt,
                           double* lossp, hipStream_t s);
int loss_blocks(int64_t n);
// loss = sum(lossp[0..n)) / numel into *out (device double).
hipError_t launch_loss_final(const double* lossp, int n, double numel, double* out,
                             hipStream_t s);
// out[t * D + d] = sum_b src[(b * T + t) * D + d]
hipError_t launch_sum_batches(const float* src, int B, int T, int D, float* out, hipStream_t s);
// FP32 (rows x cols) -> BF16 copy and BF16 transpose (cols x rows).
hipError_t launch_to_bf16(const float* w, int rows, int cols, uint16_t* w16, uint16_t* w16t,
                          hipStream_t s);
// The optimizer step over the flat FP32 parameters, described by a device table of segments
// in parameter order: a weight matrix (w16 set: rows x cols at off, cols and rows multiples
// of 4, its BF16 copy w16 and transpose w16t rewritten from the updated weights), or a plain
// range (w16 null: len parameters at off).  Segment k covers workgroups [blk0, next blk0):
// ceil(rows / kAdamTile) * tiles_c for a matrix (tiles_c = ceil(cols / kAdamTile)),
// ceil(len / kAdamChunk) for a range.
constexpr int kAdamTile = 64, kAdamChunk = 4096;
struct AdamSeg {
  int64_t off, len;
  int rows, cols, tiles_c, blk0;
  uint16_t* w16;
  uint16_t* w16t;
};
// Adam with bias correction: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// w -= lr (m / bc1) / (sqrt(v / bc2) + eps).
struct AdamArgs {
  float lr, b1, b2, eps, bc1, bc2;
};
hipError_t launch_adam_bf16(const AdamSeg* segs, int nseg, int nblocks, float* w,
                           const float* g, float* m, float* v, const AdamArgs& a,
                           hipStream_t s);
// Raises the dynamic LDS limit of the row-wise kernels where embed D or T tokens need it.
hipError_t set_vit_smem_limit(int D, int T);

}  // namespace vit
}  // namespace ensf
