// Host side of the transformer forecast surrogate: parameter layout, workspace, and the
// sequence of kernels of a forward pass, a backward pass and an Adam step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "../../include/ensf_vit.h"
#include "ensf_internal.h"
#include "vit_internal.h"

using namespace ensf::vit;

namespace {

constexpr int kMaxSplits = 8;

struct Lin {
  int64_t w, b;      // offsets of weight (out x in) and bias (out) in the flat parameters
  int out, in;
  uint16_t* w16;     // BF16 weight (out x in) and its transpose (in x out)
  uint16_t* w16t;
};

struct Layer {
  int64_t ln1_g, ln1_b, ln2_g, ln2_b;
  int qkv, o, fc1, fc2;            // indices into lins
  // saved activations of the forward pass (B*T tokens)
  float* res_mid;                  // residual after attention (T_all x D)
  float* mean1; float* rstd1; float* mean2; float* rstd2;
  uint16_t* a16; uint16_t* a16t;   // LN1 output and transpose
  uint16_t* qkv16; uint16_t* qkv16t;
  uint16_t* P16; uint16_t* Pt16;   // attention weights (B*heads x T x T) and per-batch transpose
  uint16_t* o16; uint16_t* o16t;   // attention output (concatenated heads)
  uint16_t* m16; uint16_t* m16t;   // LN2 output
  uint16_t* gp16;                  // GELU'(fc1 pre-activation), BF16
  uint16_t* g16; uint16_t* g16t;   // GELU output
};

}  // namespace

struct ensf_vit {
  ensf_vit_config cfg{};
  int T = 0, P = 0, D = 0, F = 0, Hh = 0, dh = 0, L = 0, B = 0;
  int cus = 0;                // compute units of the device
  int64_t n_params = 0;
  int64_t pe_pos = 0, lnf_g = 0, lnf_b = 0;
  int pe = 0, head = 0;
  std::vector<Lin> lins;
  std::vector<Layer> layers;
  std::vector<void*> allocs;
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  int64_t adam_step = 0;
  // activations not tied to a layer
  float* res_in = nullptr;    // (L + 1) x T_all x D: input of every layer, then of LNf
  uint16_t *pt = nullptr, *ptt = nullptr;
  float *meanf = nullptr, *rstdf = nullptr;
  uint16_t *f16 = nullptr, *f16t = nullptr;
  float* tok = nullptr;
  // backward scratch
  float* S32 = nullptr;       // scores / dP (B*heads x T x T)
  float* dx32 = nullptr;      // gradient of a LayerNorm output (T_all x D)
  float* dres = nullptr;      // gradient of the residual stream (T_all x D)
  uint16_t *dres16 = nullptr, *dres16t = nullptr;
  uint16_t *datt16 = nullptr, *datt16t = nullptr;
  uint16_t *du16 = nullptr, *du16t = nullptr;
  uint16_t *dqkv16 = nullptr, *dqkv16t = nullptr;
  uint16_t *dS16 = nullptr, *dSt16 = nullptr;
  uint16_t *dy16 = nullptr, *dyt16 = nullptr;
  float *pg = nullptr, *pb = nullptr;
  float* kpart = nullptr;     // split-K partial products of the weight gradients
  size_t kpart_floats = 0;
  double* rtmp = nullptr;     // group sums of the LayerNorm parameter gradients
  double *lossp = nullptr, *loss = nullptr;
  // the optimizer step's segment table (device) and its workgroup count
  AdamSeg* adam_segs = nullptr;
  int n_adam_segs = 0, adam_blocks = 0;
};

namespace {

ensf_status fail(hipError_t e) {
  ensf::record_hip_error(e);
  return e == hipErrorOutOfMemory ? ENSF_ENOMEM : ENSF_EHIP;
}

#define VIT_TRY(expr)                              \
  do {                                             \
    hipError_t _e = (expr);                        \
    if (_e != hipSuccess) return fail(_e);         \
  } while (0)

template <typename Tp>
hipError_t alloc(ensf_vit* v, Tp** p, size_t count) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(Tp));
  if (e == hipSuccess) v->allocs.push_back(q);
  *p = static_cast<Tp*>(q);
  return e;
}

void layout(ensf_vit* v) {
  const int D = v->D, F = v->F, P = v->P, T = v->T;
  int64_t o = 0;
  auto lin = [&](int out, int in) {
    Lin l{};
    l.w = o;
    o += (int64_t)out * in;
    l.b = o;
    o += out;
    l.out = out;
    l.in = in;
    v->lins.push_back(l);
    return (int)v->lins.size() - 1;
  };
  v->pe = lin(D, P);
  v->pe_pos = o;
  o += (int64_t)T * D;
  v->layers.resize(v->L);
  for (Layer& ly : v->layers) {
    ly.ln1_g = o; o += D;
    ly.ln1_b = o; o += D;
    ly.qkv = lin(3 * D, D);
    ly.o = lin(D, D);
    ly.ln2_g = o; o += D;
    ly.ln2_b = o; o += D;
    ly.fc1 = lin(F, D);
    ly.fc2 = lin(D, F);
  }
  v->lnf_g = o; o += D;
  v->lnf_b = o; o += D;
  v->head = lin(P, D);
  v->n_params = o;
}

hipError_t allocate(ensf_vit* v) {
  const int64_t Ta = (int64_t)v->B * v->T, D = v->D, F = v->F, P = v->P;
  const int64_t Z = (int64_t)v->B * v->Hh, TT = (int64_t)v->T * v->T;
  hipError_t e = hipSuccess;
  auto A = [&](auto** p, size_t n) {
    if (e == hipSuccess) e = alloc(v, p, n);
  };
  A(&v->w, v->n_params);
  A(&v->g, v->n_params);
  A(&v->m, v->n_params);
  A(&v->v, v->n_params);
  for (Lin& l : v->lins) {
    A(&l.w16, (size_t)l.out * l.in);
    A(&l.w16t, (size_t)l.out * l.in);
  }
  A(&v->res_in, (size_t)(v->L + 1) * Ta * D);
  A(&v->pt, Ta * P);
  A(&v->ptt, Ta * P);
  for (Layer& ly : v->layers) {
    A(&ly.res_mid, Ta * D);
    A(&ly.mean1, Ta); A(&ly.rstd1, Ta); A(&ly.mean2, Ta); A(&ly.rstd2, Ta);
    A(&ly.a16, Ta * D); A(&ly.a16t, Ta * D);
    A(&ly.qkv16, Ta * 3 * D); A(&ly.qkv16t, Ta * 3 * D);
    A(&ly.P16, Z * TT); A(&ly.Pt16, Z * TT);
    A(&ly.o16, Ta * D); A(&ly.o16t, Ta * D);
    A(&ly.m16, Ta * D); A(&ly.m16t, Ta * D);
    A(&ly.gp16, Ta * F);
    A(&ly.g16, Ta * F); A(&ly.g16t, Ta * F);
  }
  A(&v->meanf, Ta); A(&v->rstdf, Ta);
  A(&v->f16, Ta * D); A(&v->f16t, Ta * D);
  A(&v->tok, Ta * P);
  A(&v->S32, Z * TT);
  A(&v->dx32, Ta * D);
  A(&v->dres, Ta * D);
  A(&v->dres16, Ta * D); A(&v->dres16t, Ta * D);
  A(&v->datt16, Ta * D); A(&v->datt16t, Ta * D);
  A(&v->du16, Ta * F); A(&v->du16t, Ta * F);
  A(&v->dqkv16, Ta * 3 * D); A(&v->dqkv16t, Ta * 3 * D);
  A(&v->dS16, Z * TT); A(&v->dSt16, Z * TT);
  A(&v->dy16, Ta * P); A(&v->dyt16, Ta * P);
  A(&v->pg, Ta / 8 * D); A(&v->pb, Ta / 8 * D);
  size_t maxw = 0;
  for (const Lin& l : v->lins) maxw = std::max(maxw, (size_t)l.out * l.in);
  v->kpart_floats = kMaxSplits * maxw;
  A(&v->kpart, v->kpart_floats);
  A(&v->rtmp, (size_t)kSumGroups * D);
  A(&v->lossp, (size_t)loss_blocks(Ta * P));
  A(&v->loss, 1);
  return e;
}

// The optimizer's segment table: the weight matrices (with their BF16 copies) and the plain
// ranges between them, in parameter order.  Synchronous (at creation).
hipError_t build_adam_table(ensf_vit* v) {
  std::vector<AdamSeg> segs;
  int blk = 0;
  auto plain = [&](int64_t off, int64_t end) {
    if (end <= off) return;
    AdamSeg a{};
    a.off = off;
    a.len = end - off;
    a.blk0 = blk;
    blk += (int)((a.len + kAdamChunk - 1) / kAdamChunk);
    segs.push_back(a);
  };
  int64_t cur = 0;
  for (const Lin& l : v->lins) {
    if (l.w < cur || l.out % 4 != 0 || l.in % 4 != 0) return hipErrorInvalidValue;
    plain(cur, l.w);
    AdamSeg a{};
    a.off = l.w;
    a.rows = l.out;
    a.cols = l.in;
    a.tiles_c = (l.in + kAdamTile - 1) / kAdamTile;
    a.blk0 = blk;
    a.w16 = l.w16;
    a.w16t = l.w16t;
    blk += a.tiles_c * ((l.out + kAdamTile - 1) / kAdamTile);
    segs.push_back(a);
    cur = l.w + (int64_t)l.out * l.in;
  }
  plain(cur, v->n_params);
  hipError_t e = alloc(v, &v->adam_segs, segs.size());
  if (e == hipSuccess)
    e = hipMemcpy(v->adam_segs, segs.data(), segs.size() * sizeof(AdamSeg), hipMemcpyHostToDevice);
  v->n_adam_segs = (int)segs.size();
  v->adam_blocks = blk;
  return e;
}

hipError_t refresh_bf16(ensf_vit* v, hipStream_t s) {
  for (const Lin& l : v->lins) {
    hipError_t e = launch_to_bf16(v->w + l.w, l.out, l.in, l.w16, l.w16t, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

VMat mat(const uint16_t* p, int64_t ld, int64_t sb = 0, int64_t sh = 0) {
  return VMat{p, ld, sb, sh};
}

// C = A B^T for unbatched operands; fields of the epilogue left empty.
VGemm prod(VMat a, VMat b, int M, int N, int K) {
  VGemm g{};
  g.A = a;
  g.B = b;
  g.M = M;
  g.N = N;
  g.K = K;
  g.nh = 1;
  g.alpha = 1.0f;
  return g;
}

// ----- forward pass of `nb` states; the loss pass when target != nullptr
hipError_t run_forward(ensf_vit* v, const float* x, const float* target, float* y, int nb,
                   hipStream_t s) {
  const int D = v->D, F = v->F, P = v->P, T = v->T, Hh = v->Hh, dh = v->dh;
  const int64_t Ta = (int64_t)nb * T, TT = (int64_t)T * T;
  const float* w = v->w;
  hipError_t e = launch_patchify(x, nb, v->cfg.channels, v->cfg.height, v->cfg.width,
                                 v->cfg.patch, v->pt, v->ptt, s);
  if (e != hipSuccess) return e;
  {
    const Lin& l = v->lins[v->pe];
    VGemm g = prod(mat(v->pt, P), mat(l.w16, P), (int)Ta, D, P);
    g.bias = w + l.b;
    g.add = w + v->pe_pos;
    g.ld_add = D;
    g.add_rows = T;
    g.f32 = v->res_in;
    g.ld_f32 = D;
    if ((e = launch_vgemm(g, 1, s)) != hipSuccess) return e;
  }
  for (int li = 0; li < v->L; ++li) {
    Layer& ly = v->layers[li];
    float* rin = v->res_in + (int64_t)li * Ta * D;
    float* rout = v->res_in + (int64_t)(li + 1) * Ta * D;
    if ((e = launch_ln_fwd(rin, Ta, D, w + ly.ln1_g, w + ly.ln1_b, ly.a16, ly.a16t, Ta,
                           ly.mean1, ly.rstd1, s)) != hipSuccess)
      return e;
    {
      const Lin& l = v->lins[ly.qkv];
      VGemm g = prod(mat(ly.a16, D), mat(l.w16, D), (int)Ta, 3 * D, D);
      g.bias = w + l.b;
      g.b16 = ly.qkv16;
      g.ld_b16 = 3 * D;
      g.b16t = ly.qkv16t;
      g.ld_t = Ta;
      if ((e = launch_vgemm(g, 1, s)) != hipSuccess) return e;
    }
    {  // S = q k^T / sqrt(dh), per (state, head)
      VGemm g = prod(mat(ly.qkv16, 3 * D, (int64_t)T * 3 * D, dh),
                     mat(ly.qkv16 + D, 3 * D, (int64_t)T * 3 * D, dh), T, T, dh);
      g.nh = Hh;
      g.alpha = 1.0f / std::sqrt((float)dh);
      g.f32 = v->S32;
      g.ld_f32 = T;
      g.sb_f32 = Hh * TT;
      g.sh_f32 = TT;
      if ((e = launch_vgemm(g, nb * Hh, s)) != hipSuccess) return e;
    }
    if ((e = launch_attn_softmax(v->S32, (int64_t)nb * Hh, T, ly.P16, ly.Pt16, s)) != hipSuccess)
      return e;
    {  // o = P v: the B operand is v^T (rows = features of the head, k = tokens)
      VGemm g = prod(mat(ly.P16, T, Hh * TT, TT),
                     mat(ly.qkv16t + 2 * D * Ta, Ta, T, (int64_t)dh * Ta), T, dh, T);
      g.nh = Hh;
      g.b16 = ly.o16;
      g.ld_b16 = D;
      g.sb_b16 = (int64_t)T * D;
      g.sh_b16 = dh;
      g.b16t = ly.o16t;
      g.ld_t = Ta;
      g.sb_t = T;
      g.sh_t = (int64_t)dh * Ta;
      if ((e = launch_vgemm(g, nb * Hh, s)) != hipSuccess) return e;
    }
    {
      const Lin& l = v->lins[ly.o];
      VGemm g = prod(mat(ly.o16, D), mat(l.w16, D), (int)Ta, D, D);
      g.bias = w + l.b;
      g.add = rin;
      g.ld_add = D;
      g.f32 = ly.res_mid;
      g.ld_f32 = D;
      if ((e = launch_vgemm(g, 1, s)) != hipSuccess) return e;
    }
    if ((e = launch_ln_fwd(ly.res_mid, Ta, D, w + ly.ln2_g, w + ly.ln2_b, ly.m16, ly.m16t, Ta,
                           ly.mean2, ly.rstd2, s)) != hipSuccess)
      return e;
    {
      const Lin& l = v->lins[ly.fc1];
      VGemm g = prod(mat(ly.m16, D), mat(l.w16, D), (int)Ta, F, D);
      g.bias = w + l.b;
      g.act = 1;
      g.gd = ly.gp16;
      g.ld_gin = F;
      g.b16 = ly.g16;
      g.ld_b16 = F;
      g.b16t = ly.g16t;
      g.ld_t = Ta;
      if ((e = launch_vgemm(g, 1, s)) != hipSuccess) return e;
    }
    {
      const Lin& l = v->lins[ly.fc2];
      VGemm g = prod(mat(ly.g16, F), mat(l.w16, F), (int)Ta, D, F);
      g.bias = w + l.b;
      g.add = ly.res_mid;
      g.ld_add = D;
      g.f32 = rout;
      g.ld_f32 = D;
      if ((e = launch_vgemm(g, 1, s)) != hipSuccess) return e;
    }
  }
  const float* rlast = v->res_in + (int64_t)v->L * Ta * D;
  if ((e = launch_ln_fwd(rlast, Ta, D, w + v->lnf_g, w + v->lnf_b, v->f16, v->f16t, Ta, v->meanf,
                         v->rstdf, s)) != hipSuccess)
    return e;
  {
    const Lin& l = v->lins[v->head];
    VGemm g = prod(mat(v->f16, D), mat(l.w16, D), (int)Ta, P, D);
    g.bias = w + l.b;
    g.f32 = v->tok;
    g.ld_f32 = P;
    if ((e = launch_vgemm(g, 1, s)) != hipSuccess) return e;
  }
  e = launch_head_out(v->tok, x, target, y, nb, v->cfg.channels, v->cfg.height, v->cfg.width,
                      v->cfg.patch, v->dy16, v->dyt16, v->lossp, s);
  if (e != hipSuccess || !target) return e;
  const int64_t numel = Ta * P;
  return launch_loss_final(v->lossp, loss_blocks(numel), (double)numel, v->loss, s);
}

// weight gradient dW = dY^T X from the transposed copies (rows x T_all each) and the bias
// gradient from the row sums of dY^T.  The contraction runs over all tokens of the batch
// while the output (out x in) may have few tiles: it is split so that about three
// workgroups per compute unit run (as many as are resident at once, so none waits for a
// compute unit to free up), the partial products summed in split order (FP64) afterwards.
hipError_t weight_grad(ensf_vit* v, const Lin& l, const uint16_t* dyt, const uint16_t* xt,
                       int64_t Ta, hipStream_t s) {
  VGemm g = prod(mat(dyt, Ta), mat(xt, Ta), l.out, l.in, (int)Ta);
  const int tile = (l.out % 128 == 0 && l.in % 128 == 0) ? 128 : (l.out % 64 == 0 && l.in % 64 == 0) ? 64 : 32;
  const int64_t tiles = (int64_t)(l.out / tile) * (l.in / tile);
  int splits = (int)std::min<int64_t>(kMaxSplits, std::max<int64_t>(1, 3 * v->cus / tiles));
  while (splits > 1 && Ta / splits < 256) --splits;
  hipError_t e;
  if (splits > 1) {
    const int64_t q = Ta % 64 == 0 ? 64 : 32;   // the k-step of the larger tiles divides it
    g.kchunk = (Ta / splits + q - 1) / q * q;
    splits = (int)((Ta + g.kchunk - 1) / g.kchunk);
    g.splits = splits;
    g.part_stride = (int64_t)l.out * l.in;
    g.f32 = v->kpart;
    g.ld_f32 = l.in;
    e = launch_vgemm(g, 1, s);
    if (e == hipSuccess)
      e = launch_sum_rows(v->kpart, splits, (int64_t)l.out * l.in, v->g + l.w, false, s);
  } else {
    g.f32 = v->g + l.w;
    g.ld_f32 = l.in;
    e = launch_vgemm(g, 1, s);
  }
  if (e != hipSuccess) return e;
  return launch_rowsum_bf16(dyt, l.out, Ta, Ta, v->g + l.b, s);
}

hipError_t ln_backward(ensf_vit* v, const float* xin, const float* mean, const float* rstd,
                       int64_t g_off, int64_t b_off, int64_t Ta, hipStream_t s) {
  const int D = v->D;
  hipError_t e = launch_ln_bwd(v->dx32, xin, mean, rstd, v->w + g_off, Ta, D, v->dres,
                               v->dres16, v->dres16t, Ta, v->pg, v->pb, s);
  if (e == hipSuccess) e = launch_sum_rows(v->pg, Ta / 8, D, v->g + g_off, false, s, v->rtmp);
  if (e == hipSuccess) e = launch_sum_rows(v->pb, Ta / 8, D, v->g + b_off, false, s, v->rtmp);
  return e;
}

hipError_t run_backward(ensf_vit* v, int nb, hipStream_t s) {
  const int D = v->D, F = v->F, P = v->P, T = v->T, Hh = v->Hh, dh = v->dh;
  const int64_t Ta = (int64_t)nb * T, TT = (int64_t)T * T;
  hipError_t e;
  {  // head: tok = f W_h^T + b_h
    const Lin& l = v->lins[v->head];
    if ((e = weight_grad(v, l, v->dyt16, v->f16t, Ta, s)) != hipSuccess) return e;
    VGemm g = prod(mat(v->dy16, P), mat(l.w16t, P), (int)Ta, D, P);
    g.f32 = v->dx32;
    g.ld_f32 = D;
    if ((e = launch_vgemm(g, 1, s)) != hipSuccess) return e;
  }
  if ((e = hipMemsetAsync(v->dres, 0, (size_t)Ta * D * 4, s)) != hipSuccess) return e;
  if ((e = ln_backward(v, v->res_in + (int64_t)v->L * Ta * D, v->meanf, v->rstdf, v->lnf_g,
                       v->lnf_b, Ta, s)) != hipSuccess)
    return e;
  for (int li = v->L - 1; li >= 0; --li) {
    Layer& ly = v->layers[li];
    const float* rin = v->res_in + (int64_t)li * Ta * D;
    // MLP: h_out = h_mid + gelu(m W_1^T + b_1) W_2^T + b_2; dres holds d h_out
    const Lin& l2 = v->lins[ly.fc2];
    const Lin& l1 = v->lins[ly.fc1];
    if ((e = weight_grad(v, l2, v->dres16t, ly.g16t, Ta, s)) != hipSuccess) return e;
    {
      VGemm g = prod(mat(v->dres16, D), mat(l2.w16t, D), (int)Ta, F, D);
      g.act = 2;
      g.gin = ly.gp16;
      g.ld_gin = F;
      g.b16 = v->du16;
      g.ld_b16 = F;
      g.b16t = v->du16t;
      g.ld_t = Ta;
      if ((e = launch_vgemm(g, 1, s)) != hipSuccess) return e;
    }
    if ((e = weight_grad(v, l1, v->du16t, ly.m16t, Ta, s)) != hipSuccess) return e;
    {
      VGemm g = prod(mat(v->du16, F), mat(l1.w16t, F), (int)Ta, D, F);
      g.f32 = v->dx32;
      g.ld_f32 = D;
      if ((e = launch_vgemm(g, 1, s)) != hipSuccess) return e;
    }
    if ((e = ln_backward(v, ly.res_mid, ly.mean2, ly.rstd2, ly.ln2_g, ly.ln2_b, Ta, s)) !=
        hipSuccess)
      return e;
    // attention: h_mid = h_in + o W_o^T + b_o; dres holds d h_mid
    const Lin& lo = v->lins[ly.o];
    const Lin& lq = v->lins[ly.qkv];
    if ((e = weight_grad(v, lo, v->dres16t, ly.o16t, Ta, s)) != hipSuccess) return e;
    {
      VGemm g = prod(mat(v->dres16, D), mat(lo.w16t, D), (int)Ta, D, D);
      g.b16 = v->datt16;
      g.ld_b16 = D;
      g.b16t = v->datt16t;
      g.ld_t = Ta;
      if ((e = launch_vgemm(g, 1, s)) != hipSuccess) return e;
    }
    {  // dP = dO v^T per (state, head)
      VGemm g = prod(mat(v->datt16, D, (int64_t)T * D, dh),
                     mat(ly.qkv16 + 2 * D, 3 * D, (int64_t)T * 3 * D, dh), T, T, dh);
      g.nh = Hh;
      g.f32 = v->S32;
      g.ld_f32 = T;
      g.sb_f32 = Hh * TT;
      g.sh_f32 = TT;
      if ((e = launch_vgemm(g, nb * Hh, s)) != hipSuccess) return e;
    }
    if ((e = launch_attn_ds(ly.P16, v->S32, (int64_t)nb * Hh, T, 1.0f / std::sqrt((float)dh),
                            v->dS16, v->dSt16, s)) != hipSuccess)
      return e;
    // dq = dS k, dk = dS^T q, dv = P^T dO into the q, k, v column blocks of dqkv
    struct {
      const uint16_t* a;
      const uint16_t* bt;   // transposed operand rows (features x tokens)
      int64_t col;          // column block of dqkv
    } parts[3] = {{v->dS16, ly.qkv16t + (int64_t)D * Ta, 0},
                  {v->dSt16, ly.qkv16t, D},
                  {ly.Pt16, v->datt16t, 2 * D}};
    for (const auto& pp : parts) {
      VGemm g = prod(mat(pp.a, T, Hh * TT, TT), mat(pp.bt, Ta, T, (int64_t)dh * Ta), T, dh, T);
      g.nh = Hh;
      g.b16 = v->dqkv16 + pp.col;
      g.ld_b16 = 3 * D;
      g.sb_b16 = (int64_t)T * 3 * D;
      g.sh_b16 = dh;
      g.b16t = v->dqkv16t + pp.col * Ta;
      g.ld_t = Ta;
      g.sb_t = T;
      g.sh_t = (int64_t)dh * Ta;
      if ((e = launch_vgemm(g, nb * Hh, s)) != hipSuccess) return e;
    }
    if ((e = weight_grad(v, lq, v->dqkv16t, ly.a16t, Ta, s)) != hipSuccess) return e;
    {
      VGemm g = prod(mat(v->dqkv16, 3 * D), mat(lq.w16t, 3 * D), (int)Ta, D, 3 * D);
      g.f32 = v->dx32;
      g.ld_f32 = D;
      if ((e = launch_vgemm(g, 1, s)) != hipSuccess) return e;
    }
    if ((e = ln_backward(v, rin, ly.mean1, ly.rstd1, ly.ln1_g, ly.ln1_b, Ta, s)) != hipSuccess)
      return e;
  }
  // patch embedding: h0 = patches W_pe^T + b_pe + pos
  if ((e = launch_sum_batches(v->dres, nb, T, D, v->g + v->pe_pos, s)) != hipSuccess) return e;
  return weight_grad(v, v->lins[v->pe], v->dres16t, v->ptt, Ta, s);
}

ensf_status grad_impl(ensf_vit* v, const float* x, const float* target, int32_t batch,
                      double* h_loss, hipStream_t s) {
  if (!v || !x || !target || batch < 1 || batch > v->B) return ENSF_EINVAL;
  ensf::clear_stale_hip_error();
  VIT_TRY(hipSetDevice(v->cfg.device));
  VIT_TRY(run_forward(v, x, target, nullptr, batch, s));
  VIT_TRY(run_backward(v, batch, s));
  if (h_loss) {
    VIT_TRY(hipMemcpyAsync(h_loss, v->loss, sizeof(double), hipMemcpyDeviceToHost, s));
    VIT_TRY(hipStreamSynchronize(s));
  }
  return ENSF_OK;
}

}  // namespace

extern "C" {

ensf_status ensf_vit_create(const ensf_vit_config* cfg, ensf_vit** out) {
  if (!cfg || !out) return ENSF_EINVAL;
  *out = nullptr;
  const ensf_vit_config c = *cfg;
  if (c.channels < 1 || c.patch < 1 || c.height < c.patch || c.width < c.patch ||
      c.height % c.patch || c.width % c.patch || c.layers < 1 || c.heads < 1 ||
      c.embed < 64 || c.embed % 64 || c.embed > 2048 || c.embed % c.heads ||
      (c.embed / c.heads) % 32 || c.mlp_hidden < 32 || c.mlp_hidden % 32 || c.max_batch < 1)
    return ENSF_EINVAL;
  const int T = (c.height / c.patch) * (c.width / c.patch);
  const int P = c.channels * c.patch * c.patch;
  if (T % 64 || T > 1024 || P % 32) return ENSF_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return ENSF_EHIP;
  if (c.device < 0 || c.device >= ndev) return ENSF_EINVAL;
  VIT_TRY(hipSetDevice(c.device));
  VIT_TRY(set_vit_smem_limit(c.embed, T));
  int cus = 0;
  VIT_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device));
  ensf_vit* v = new ensf_vit();
  v->cfg = c;
  v->cus = std::max(cus, 1);
  v->T = T;
  v->P = P;
  v->D = c.embed;
  v->F = c.mlp_hidden;
  v->Hh = c.heads;
  v->dh = c.embed / c.heads;
  v->L = c.layers;
  v->B = c.max_batch;
  layout(v);
  hipError_t e = allocate(v);
  if (e == hipSuccess) e = build_adam_table(v);
  if (e == hipSuccess) {
    // N(0, 0.02) weights and positions, zero biases, unit LayerNorm gains, head x 0.1
    std::vector<float> h(v->n_params, 0.0f);
    std::mt19937_64 rng(c.seed);
    std::normal_distribution<float> nd(0.0f, 0.02f);
    for (const Lin& l : v->lins)
      for (int64_t i = 0; i < (int64_t)l.out * l.in; ++i) h[l.w + i] = nd(rng);
    for (int64_t i = 0; i < (int64_t)T * v->D; ++i) h[v->pe_pos + i] = nd(rng);
    const Lin& hd = v->lins[v->head];
    for (int64_t i = 0; i < (int64_t)hd.out * hd.in; ++i) h[hd.w + i] *= 0.1f;
    for (const Layer& ly : v->layers)
      for (int d = 0; d < v->D; ++d) h[ly.ln1_g + d] = h[ly.ln2_g + d] = 1.0f;
    for (int d = 0; d < v->D; ++d) h[v->lnf_g + d] = 1.0f;
    *out = v;
    const ensf_status st = ensf_vit_set_params(v, h.data());
    if (st != ENSF_OK) {
      ensf_vit_destroy(v);
      *out = nullptr;
    }
    return st;
  }
  ensf_vit_destroy(v);
  return fail(e);
}

int64_t ensf_vit_num_params(const ensf_vit* v) { return v ? v->n_params : 0; }

ensf_status ensf_vit_set_params(ensf_vit* v, const float* h_params) {
  if (!v || !h_params) return ENSF_EINVAL;
  ensf::clear_stale_hip_error();
  VIT_TRY(hipSetDevice(v->cfg.device));
  const size_t bytes = (size_t)v->n_params * sizeof(float);
  VIT_TRY(hipMemcpy(v->w, h_params, bytes, hipMemcpyHostToDevice));
  VIT_TRY(hipMemset(v->m, 0, bytes));
  VIT_TRY(hipMemset(v->v, 0, bytes));
  v->adam_step = 0;
  VIT_TRY(refresh_bf16(v, nullptr));
  VIT_TRY(hipDeviceSynchronize());
  return ENSF_OK;
}

ensf_status ensf_vit_get_params(ensf_vit* v, float* h_params) {
  if (!v || !h_params) return ENSF_EINVAL;
  VIT_TRY(hipSetDevice(v->cfg.device));
  VIT_TRY(hipDeviceSynchronize());
  VIT_TRY(hipMemcpy(h_params, v->w, (size_t)v->n_params * sizeof(float), hipMemcpyDeviceToHost));
  return ENSF_OK;
}

ensf_status ensf_vit_forward(ensf_vit* v, const float* d_x, float* d_y, int32_t batch,
                             void* stream) {
  if (!v || !d_x || !d_y || batch < 1) return ENSF_EINVAL;
  const int64_t per = (int64_t)v->cfg.channels * v->cfg.height * v->cfg.width;
  if (d_x < d_y + per * batch && d_y < d_x + per * batch) return ENSF_EINVAL;
  ensf::clear_stale_hip_error();
  VIT_TRY(hipSetDevice(v->cfg.device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int32_t b0 = 0; b0 < batch; b0 += v->B) {
    const int nb = std::min<int32_t>(v->B, batch - b0);
    VIT_TRY(run_forward(v, d_x + per * b0, nullptr, d_y + per * b0, nb, s));
  }
  return ENSF_OK;
}

ensf_status ensf_vit_grad(ensf_vit* v, const float* d_x, const float* d_target, int32_t batch,
                          float* d_grad, double* h_loss, void* stream) {
  if (!d_grad) return ENSF_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const ensf_status st = grad_impl(v, d_x, d_target, batch, nullptr, s);
  if (st != ENSF_OK) return st;
  VIT_TRY(hipMemcpyAsync(d_grad, v->g, (size_t)v->n_params * sizeof(float),
                         hipMemcpyDeviceToDevice, s));
  if (h_loss) {
    VIT_TRY(hipMemcpyAsync(h_loss, v->loss, sizeof(double), hipMemcpyDeviceToHost, s));
    VIT_TRY(hipStreamSynchronize(s));
  }
  return ENSF_OK;
}

ensf_status ensf_vit_train_step(ensf_vit* v, const float* d_x, const float* d_target,
                                int32_t batch, float lr, double* h_loss, void* stream) {
  if (!(lr >= 0.0f)) return ENSF_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const ensf_status st = grad_impl(v, d_x, d_target, batch, nullptr, s);
  if (st != ENSF_OK) return st;
  v->adam_step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = (float)(1.0 - std::pow(0.9, (double)v->adam_step));
  const float bc2 = (float)(1.0 - std::pow(0.999, (double)v->adam_step));
  const AdamArgs a{lr, b1, b2, 1e-8f, bc1, bc2};
  VIT_TRY(launch_adam_bf16(v->adam_segs, v->n_adam_segs, v->adam_blocks, v->w, v->g, v->m, v->v,
                           a, s));
  if (h_loss) {
    VIT_TRY(hipMemcpyAsync(h_loss, v->loss, sizeof(double), hipMemcpyDeviceToHost, s));
    VIT_TRY(hipStreamSynchronize(s));
  }
  return ENSF_OK;
}

ensf_status ensf_vit_destroy(ensf_vit* v) {
  if (!v) return ENSF_OK;
  (void)hipSetDevice(v->cfg.device);
  (void)hipDeviceSynchronize();
  for (void* p : v->allocs) (void)hipFree(p);
  delete v;
  return ENSF_OK;
}

}  // extern "C"
