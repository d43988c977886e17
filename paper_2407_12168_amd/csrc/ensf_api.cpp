// Host side of libensf: argument validation, workspace layout, grouped launches of the
// pseudo-time loop (eager or as one captured hipGraph), status reporting, autotuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/ensf.h"
#include "ensf_internal.h"
#include "ensf_run.h"

namespace ensf {
hipError_t set_softmax_smem_limit(size_t bytes);
}

using namespace ensf;

namespace ensf {
namespace {
thread_local hipError_t g_last_error = hipSuccess;
}
void record_hip_error(hipError_t e) {
  g_last_error = e;
  (void)hipGetLastError();
}
void clear_stale_hip_error() { (void)hipGetLastError(); }
}  // namespace ensf

namespace {

constexpr size_t kAlign = 256;

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct TileChoice {
  int gram = kGram128;
  int wx = kWx128;
  double split_scale = 1.0;  // multiplies the default split-K count
  int gram_bk = 32;          // k-step depth of the Gram main loop (32 or 64)
  int wx_bk = 32;            // k-step depth of the W.X main loop (32 or 64)
  int gram_st = 2;           // LDS stages of the Gram main loop (1, or 2 = ping-pong)
  int wx_st = 2;             // LDS stages of the W.X main loop
  bool same_kernels(const TileChoice& o) const {
    return gram == o.gram && wx == o.wx && gram_bk == o.gram_bk && wx_bk == o.wx_bk &&
           gram_st == o.gram_st && wx_st == o.wx_st;
  }
};

struct GraphKey {
  std::vector<int64_t> sig;   // launch geometry of every captured kernel
  bool operator==(const GraphKey& o) const { return sig == o.sig; }
};

// Table key: precision and log2 buckets of N, M_p and d; for a batch of several problems
// those of the dominant problem (most N M_p d) and the log2 bucket of the batch size.
std::string tune_key(int prec, int64_t n, int64_t mp, int64_t d, int64_t batch = 1) {
  auto bucket = [](int64_t v) {
    int b = 0;
    while ((int64_t(1) << (b + 1)) <= v) ++b;
    return b;
  };
  char buf[96];
  if (batch > 1)
    snprintf(buf, sizeof buf, "gfx950/p%d/b%d/n%d/m%d/d%d", prec, bucket(batch), bucket(n),
             bucket(mp), bucket(d));
  else
    snprintf(buf, sizeof buf, "gfx950/p%d/n%d/m%d/d%d", prec, bucket(n), bucket(mp), bucket(d));
  return buf;
}

size_t dominant_problem(const std::vector<ensf_problem>& probs) {
  size_t dom = 0;
  for (size_t f = 1; f < probs.size(); ++f)
    if ((double)probs[f].n_members * probs[f].n_particles * probs[f].dim >
        (double)probs[dom].n_members * probs[dom].n_particles * probs[dom].dim)
      dom = f;
  return dom;
}

}  // namespace

struct ensf_ctx {
  ensf_options opt{};
  int device = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  // descriptor table + prefix arrays: device copy and pinned host staging
  char* d_tab = nullptr;
  char* h_tab = nullptr;
  size_t tab_bytes = 0;
  hipEvent_t tab_event = nullptr;
  bool tab_event_pending = false;
  // [0] non-finite values, [1] bad obs indices, [2] persistent-loop barrier arrivals,
  // [3] persistent-loop barrier give-ups
  unsigned long long* d_counters = nullptr;
  hipStream_t cap_stream = nullptr;
  hipEvent_t done_event = nullptr;   // recorded at the end of every call, on its stream
  hipStream_t last_stream = nullptr;
  bool has_last_stream = false;
  GraphKey gkey;
  hipGraphExec_t gexec = nullptr;
  std::map<std::string, TileChoice> tune;
  std::string tune_path;
  size_t softmax_smem_set = 0;
  // phase timing (ensf_profile_phases)
  bool profile = false;
  std::vector<hipEvent_t> events;   // pool, 4 per pseudo-step of a profiled call
  std::vector<std::pair<int, int>> pending;  // (first event index, steps) per profiled call
  double phase_ms[3] = {0, 0, 0};
  int64_t phase_count = 0;
  size_t events_used = 0;
};

namespace {

ensf_status hip_fail(hipError_t e) {
  ensf::record_hip_error(e);
  return e == hipErrorOutOfMemory ? ENSF_ENOMEM : ENSF_EHIP;
}

#define HIP_TRY(expr)                               \
  do {                                              \
    hipError_t _e = (expr);                         \
    if (_e != hipSuccess) return hip_fail(_e);      \
  } while (0)

// Problems that use the same kernel variant (Gram shape, W.X shape, k-step depth) form a
// group: one grouped launch per kernel phase and pseudo-step, its problems contiguous in
// the descriptor table.  The softmax does not depend on tile shapes and covers all rows.
// (build_plan currently gives a whole batch one variant, hence one group.)
struct Group {
  TileChoice tiles;
  int first = 0, count = 0;
  std::vector<int32_t> pre_gram, pre_wx;
};

struct Plan {
  std::vector<ProbDev> desc;        // in group order
  std::vector<int> order;           // desc[i] describes problem order[i]
  std::vector<TileChoice> tc;       // per desc entry
  std::vector<int32_t> pre_rows;
  std::vector<Group> groups;
  std::vector<double> wg_target;    // per desc entry
  int kmax = 0;
  int max_ldn = 0;
  size_t ws_needed = 0;
};

ensf_status validate(const ensf_problem& p) {
  if (!p.d_prior || !p.d_post) return ENSF_EINVAL;
  if (p.n_members < 1 || p.n_members > kMaxMembers) return ENSF_EINVAL;
  if (p.n_particles < 1 || p.dim < 1 || p.n_steps < 1) return ENSF_EINVAL;
  if ((int64_t)p.dim * 4 / 4 != p.dim || p.dim > (int64_t(1) << 34)) return ENSF_EINVAL;
  if (p.n_obs < 0 || p.n_obs > INT32_MAX) return ENSF_EINVAL;
  if (p.n_obs > 0) {
    if (!p.d_obs_idx || !p.d_obs_val) return ENSF_EINVAL;
    if (!(p.obs_sigma > 0.0f) || !std::isfinite(p.obs_sigma)) return ENSF_EINVAL;
  }
  const char* a0 = reinterpret_cast<const char*>(p.d_prior);
  const char* a1 = a0 + (size_t)p.n_members * p.dim * sizeof(float);
  const char* b0 = reinterpret_cast<const char*>(p.d_post);
  const char* b1 = b0 + (size_t)p.n_particles * p.dim * sizeof(float);
  if (a0 < b1 && b0 < a1) return ENSF_EINVAL;
  return ENSF_OK;
}

TileChoice heuristic_tiles(int64_t n, int64_t mp) {
  TileChoice c;
  const int64_t mn = std::min(n, mp);
  c.gram = mn >= 768 ? kGram256 : mn >= 128 ? kGram128 : mn >= 48 ? kGram64 : kGram32;
  c.wx = mp >= 768 ? kWx256 : mp >= 128 ? kWx128 : mp >= 48 ? kWx64 : kWx32;
  return c;
}

// Lays out one problem's workspace at offset `off` (bytes) and fills its descriptor.
size_t layout_problem(ProbDev& P, const ensf_problem& p, int prec, const TileChoice& tc,
                      const ensf_options& opt, double wg_target, size_t off, char* base) {
  auto take = [&](size_t bytes) {
    off = round_up(off, kAlign);
    char* ptr = base ? base + off : nullptr;
    off += bytes;
    return ptr;
  };
  P = ProbDev{};
  P.X = p.d_prior;
  P.post = p.d_post;
  P.obs_idx = p.d_obs_idx;
  P.obs_val = p.d_obs_val;
  P.N = p.n_members;
  P.Mp = p.n_particles;
  P.d = p.dim;
  P.n_obs = p.n_obs;
  P.K = p.n_steps;
  P.seed_lo = (uint32_t)(p.seed & 0xFFFFFFFFu);
  P.seed_hi = (uint32_t)(p.seed >> 32);
  P.filter = p.filter_id;
  P.inv_sig2_d = p.n_obs > 0 ? 1.0 / ((double)p.obs_sigma * (double)p.obs_sigma) : 0.0;
  P.obs_op = opt.obs_op;
  P.lik_implicit = opt.lik_step == ENSF_LIK_IMPLICIT ? 1 : 0;
  P.sparse = opt.wx_sparse ? 1 : 0;
  P.eps = opt.eps_alpha;
  P.t_score = 1.0;
  const int bm = gram_bm(tc.gram), bn = gram_bn(tc.gram);
  P.Mp_pad = (int32_t)round_up(P.Mp, std::max({bm, wx_bp(tc.wx), 64}));
  P.N_pad = (int32_t)round_up(P.N, std::max(bn, 64));
  P.ldn = P.N_pad;
  P.ldz = round_up(P.d, std::max(wx_be(tc.wx), 128));

  P.gram_tm = (int32_t)ceil_div(P.Mp, bm);
  P.gram_tn = (int32_t)ceil_div(P.N, bn);
  const int64_t tiles = (int64_t)P.gram_tm * P.gram_tn;
  // split-K: this problem's share of ~1024 workgroups (enough to fill the device), chunks
  // of at least 4 k-steps, and partial sums no larger than a quarter of the operand bytes
  int64_t s = std::max<int64_t>(1, (int64_t)std::ceil(wg_target / (double)tiles));
  s = std::min<int64_t>(s, P.ldz / (4 * kMaxBK));
  s = std::min<int64_t>(s, std::max<int64_t>(1, (P.Mp + P.N) * P.ldz / (4 * (int64_t)P.Mp * P.N)));
  s = std::max<int64_t>(1, (int64_t)std::llround(s * tc.split_scale));
  s = std::min<int64_t>(s, P.ldz / kMaxBK);
  P.kchunk = round_up(ceil_div(P.ldz, s), kMaxBK);
  P.S = (int32_t)ceil_div(P.ldz, P.kchunk);
  P.wx_tp = (int32_t)ceil_div(P.Mp, wx_bp(tc.wx));
  P.wx_te = (int32_t)ceil_div(P.d, wx_be(tc.wx));

  P.Z = reinterpret_cast<float*>(take((size_t)P.Mp_pad * P.ldz * 4));
  if (prec == kFP32) {
    P.Xf = reinterpret_cast<float*>(take((size_t)P.N_pad * P.ldz * 4));
  } else {
    P.Xh = reinterpret_cast<uint16_t*>(take((size_t)P.N_pad * P.ldz * 2));
    P.Xl = reinterpret_cast<uint16_t*>(take((size_t)P.N_pad * P.ldz * 2));
    P.XTh = reinterpret_cast<uint16_t*>(take((size_t)P.ldz * P.ldn * 2));
    P.XTl = reinterpret_cast<uint16_t*>(take((size_t)P.ldz * P.ldn * 2));
  }
  P.xnorm = reinterpret_cast<float*>(take((size_t)P.ldn * 4));
  P.A = reinterpret_cast<float*>(take((size_t)P.ldz * 4));
  P.B = reinterpret_cast<float*>(take((size_t)P.ldz * 4));
  P.part = reinterpret_cast<float*>(take((size_t)P.S * P.Mp_pad * P.ldn * 4));
  if (prec == kFP32) {
    P.W = reinterpret_cast<float*>(take((size_t)P.Mp_pad * P.ldn * 4));
  } else {
    P.Wh = reinterpret_cast<uint16_t*>(take((size_t)P.Mp_pad * P.ldn * 2));
    P.Wl = reinterpret_cast<uint16_t*>(take((size_t)P.Mp_pad * P.ldn * 2));
  }
  P.sp_cnt = reinterpret_cast<int32_t*>(take((size_t)P.Mp_pad * 4));
  P.sp_idx = reinterpret_cast<int32_t*>(take((size_t)P.Mp_pad * kSparseMax * 4));
  P.sp_w = reinterpret_cast<float*>(take((size_t)P.Mp_pad * kSparseMax * 4));
  P.ob_acc = reinterpret_cast<long long*>(take((size_t)(P.ldz + 1) * 8));
  return round_up(off, kAlign);
}

ensf_status ensure_workspace(ensf_ctx* c, size_t bytes) {
  if (bytes <= c->ws_bytes) return ENSF_OK;
  HIP_TRY(hipDeviceSynchronize());
  if (c->ws) HIP_TRY(hipFree(c->ws));
  c->ws = nullptr;
  c->ws_bytes = 0;
  const size_t want = round_up(bytes + bytes / 8, 1 << 20);
  HIP_TRY(hipMalloc(&c->ws, want));
  c->ws_bytes = want;
  return ENSF_OK;
}

ensf_status ensure_table(ensf_ctx* c, size_t bytes) {
  if (bytes <= c->tab_bytes) return ENSF_OK;
  HIP_TRY(hipDeviceSynchronize());
  if (c->d_tab) HIP_TRY(hipFree(c->d_tab));
  if (c->h_tab) HIP_TRY(hipHostFree(c->h_tab));
  c->d_tab = nullptr;
  c->h_tab = nullptr;
  c->tab_bytes = 0;
  const size_t want = round_up(bytes * 2, 4096);
  HIP_TRY(hipMalloc(&c->d_tab, want));
  HIP_TRY(hipHostMalloc(&c->h_tab, want, hipHostMallocDefault));
  c->tab_bytes = want;
  c->tab_event_pending = false;
  if (c->gexec) {
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->gkey = GraphKey{};
  }
  return ENSF_OK;
}

// A batch uses only a table entry measured on a batch (the fastest variant for its largest
// problem alone is not the fastest for the batch), else the heuristic.
TileChoice tiles_for(ensf_ctx* c, int prec, const ensf_problem& p, int64_t batch) {
  auto it = c->tune.find(tune_key(prec, p.n_members, p.n_particles, p.dim, batch));
  if (it != c->tune.end()) return it->second;
  return heuristic_tiles(p.n_members, p.n_particles);
}

ensf_status build_plan(ensf_ctx* c, const std::vector<ensf_problem>& probs, Plan& plan,
                       const TileChoice* force) {
  const int prec = c->opt.precision;
  const int np = (int)probs.size();
  std::vector<TileChoice> tc(np);
  std::vector<int> gid(np);
  plan.groups.clear();
  // One kernel variant for the whole batch (that of the problem with the most work): a
  // single grouped launch per phase keeps every filter's tiles in flight together, which
  // measured faster than one launch per variant.
  const size_t dominant = dominant_problem(probs);
  const TileChoice batch_tiles = force ? *force : tiles_for(c, prec, probs[dominant], np);
  for (int f = 0; f < np; ++f) {
    tc[f] = batch_tiles;
    int g = 0;
    for (; g < (int)plan.groups.size(); ++g) {
      const TileChoice& t = plan.groups[g].tiles;
      if (t.same_kernels(tc[f])) break;
    }
    if (g == (int)plan.groups.size()) {
      plan.groups.emplace_back();
      plan.groups.back().tiles = tc[f];
    }
    gid[f] = g;
  }
  plan.order.clear();
  for (int g = 0; g < (int)plan.groups.size(); ++g) {
    plan.groups[g].first = (int)plan.order.size();
    for (int f = 0; f < np; ++f)
      if (gid[f] == g) plan.order.push_back(f);
    plan.groups[g].count = (int)plan.order.size() - plan.groups[g].first;
    plan.groups[g].pre_gram.assign(plan.groups[g].count + 1, 0);
    plan.groups[g].pre_wx.assign(plan.groups[g].count + 1, 0);
  }
  plan.tc.resize(np);
  plan.desc.resize(np);
  plan.pre_rows.assign(np + 1, 0);
  plan.wg_target.assign(np, 1024.0);
  double total = 0;
  for (const auto& p : probs) total += (double)p.n_members * p.n_particles * p.dim;
  size_t off = 0;
  plan.kmax = 0;
  plan.max_ldn = 0;
  for (int i = 0; i < np; ++i) {
    const int f = plan.order[i];
    const ensf_problem& p = probs[f];
    plan.tc[i] = tc[f];
    // this problem's share of ~1024 workgroups per Gram launch
    plan.wg_target[i] =
        std::max(8.0, 1024.0 * (double)p.n_members * p.n_particles * p.dim / total);
    ProbDev& P = plan.desc[i];
    off = layout_problem(P, p, prec, plan.tc[i], c->opt, plan.wg_target[i], off, nullptr);
    Group& G = plan.groups[gid[f]];
    const int j = i - G.first;
    const int64_t gw = (int64_t)P.gram_tm * P.gram_tn * P.S;
    const int64_t ww = (int64_t)P.wx_tp * P.wx_te;
    if (G.pre_gram[j] + gw > INT32_MAX || G.pre_wx[j] + ww > INT32_MAX ||
        plan.pre_rows[i] + (int64_t)P.Mp > INT32_MAX)
      return ENSF_EINVAL;
    G.pre_gram[j + 1] = G.pre_gram[j] + (int32_t)gw;
    G.pre_wx[j + 1] = G.pre_wx[j] + (int32_t)ww;
    plan.pre_rows[i + 1] = plan.pre_rows[i] + P.Mp;
    plan.kmax = std::max(plan.kmax, P.K);
    plan.max_ldn = std::max(plan.max_ldn, P.ldn);
  }
  plan.ws_needed = off;
  return ENSF_OK;
}

// Second pass: real pointers once the workspace exists.
void bind_plan(ensf_ctx* c, const std::vector<ensf_problem>& probs, Plan& plan) {
  size_t off = 0;
  for (size_t i = 0; i < plan.desc.size(); ++i)
    off = layout_problem(plan.desc[i], probs[plan.order[i]], c->opt.precision, plan.tc[i],
                         c->opt, plan.wg_target[i], off, c->ws);
}

// Schedule of eq. 9 with alpha_t = 1 - t (1 - eps), beta_t^2 = t, damping h = 1 - t
// (eq. 11), evaluated in FP64 and rounded once to FP32.
StepScalars host_step_scalars(double t, double eps, int K) {
  const double alpha = 1.0 - t * (1.0 - eps);
  const double beta2 = t;
  const double b = -(1.0 - eps) / alpha;
  const double sigma2 = 1.0 - 2.0 * b * beta2;
  const double dt = 1.0 / (double)(K > 0 ? K : 1);
  StepScalars s;
  s.alpha = (float)alpha;
  s.inv_beta2 = (float)(1.0 / beta2);
  s.b = (float)b;
  s.sigma2 = (float)sigma2;
  s.h = (float)(1.0 - t);
  s.dt = (float)dt;
  s.cnoise = (float)std::sqrt(sigma2 * dt);
  s.damp = (float)(sigma2 * (1.0 - t) * dt);
  return s;
}

struct Uploaded {
  GroupedLaunch rows;
  std::vector<GroupedLaunch> gram, wx;   // one per group
};

// Lays the descriptor table, prefix arrays and step tables of `plan` out for the device
// address d_tab: writes them into the host buffer h (when not null) and fills u with device
// pointers.  Returns the table's size in bytes.
size_t stage_plan(const Plan& plan, char* h, char* d_tab, Uploaded& u) {
  const int np = (int)plan.desc.size();
  auto al = [](size_t v) { return (size_t)round_up((int64_t)v, 256); };
  size_t off = 0;
  auto put = [&](const void* src, size_t n) {
    if (h) memcpy(h + off, src, n);
    const size_t at = off;
    off += al(n);
    return at;
  };
  // descriptors first (their step-table pointers are filled in below), then prefix arrays,
  // then one step table per problem
  const size_t o_desc = put(plan.desc.data(), sizeof(ProbDev) * np);
  const size_t o_rows = put(plan.pre_rows.data(), sizeof(int32_t) * (np + 1));
  std::vector<std::pair<size_t, size_t>> o_grp;
  for (const Group& G : plan.groups) {
    const size_t a = put(G.pre_gram.data(), sizeof(int32_t) * (G.count + 1));
    const size_t b = put(G.pre_wx.data(), sizeof(int32_t) * (G.count + 1));
    o_grp.emplace_back(a, b);
  }
  std::vector<StepScalars> table;
  for (int f = 0; f < np; ++f) {
    const ProbDev& P = plan.desc[f];
    table.resize(P.K + 1);
    for (int k = 0; k < P.K; ++k)
      table[k] = host_step_scalars(1.0 - (double)k * (1.0 / (double)P.K), P.eps, P.K);
    table[P.K] = host_step_scalars(P.t_score, P.eps, P.K);
    const size_t o = put(table.data(), sizeof(StepScalars) * (P.K + 1));
    if (h)
      reinterpret_cast<ProbDev*>(h + o_desc)[f].steps =
          reinterpret_cast<const StepScalars*>(d_tab + o);
  }
  const ProbDev* d = reinterpret_cast<const ProbDev*>(d_tab + o_desc);
  u.rows = GroupedLaunch{d, reinterpret_cast<const int32_t*>(d_tab + o_rows), np,
                         plan.pre_rows[np]};
  u.gram.clear();
  u.wx.clear();
  for (size_t g = 0; g < plan.groups.size(); ++g) {
    const Group& G = plan.groups[g];
    u.gram.push_back(GroupedLaunch{d + G.first,
                                   reinterpret_cast<const int32_t*>(d_tab + o_grp[g].first),
                                   G.count, G.pre_gram[G.count]});
    u.wx.push_back(GroupedLaunch{d + G.first,
                                 reinterpret_cast<const int32_t*>(d_tab + o_grp[g].second),
                                 G.count, G.pre_wx[G.count]});
  }
  return off;
}

ensf_status upload_plan(ensf_ctx* c, const Plan& plan, hipStream_t s, Uploaded& u) {
  ensf_status st = ensure_table(c, stage_plan(plan, nullptr, nullptr, u));
  if (st != ENSF_OK) return st;
  if (c->tab_event_pending) HIP_TRY(hipEventSynchronize(c->tab_event));
  const size_t bytes = stage_plan(plan, c->h_tab, c->d_tab, u);
  HIP_TRY(hipMemcpyAsync(c->d_tab, c->h_tab, bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipEventRecord(c->tab_event, s));
  c->tab_event_pending = true;
  return ENSF_OK;
}

// Workspace regions that must start at zero (padding, accumulators), cleared by a fill
// kernel rather than hipMemsetAsync so that the enqueued work may be captured in a graph.
ensf_status zero_problem(const ProbDev& P, int prec, hipStream_t s) {
  HIP_TRY(launch_fill_zero(P.Z, (size_t)P.Mp_pad * P.ldz * 4, s));
  if (prec == kFP32) {
    HIP_TRY(launch_fill_zero(P.Xf, (size_t)P.N_pad * P.ldz * 4, s));
    HIP_TRY(launch_fill_zero(P.W, (size_t)P.Mp_pad * P.ldn * 4, s));
  } else {
    HIP_TRY(launch_fill_zero(P.Xh, (size_t)P.N_pad * P.ldz * 2, s));
    HIP_TRY(launch_fill_zero(P.Xl, (size_t)P.N_pad * P.ldz * 2, s));
    HIP_TRY(launch_fill_zero(P.Wh, (size_t)P.Mp_pad * P.ldn * 2, s));
    HIP_TRY(launch_fill_zero(P.Wl, (size_t)P.Mp_pad * P.ldn * 2, s));
  }
  HIP_TRY(launch_fill_zero(P.xnorm, (size_t)P.ldn * 4, s));
  HIP_TRY(launch_fill_zero(P.A, (size_t)P.ldz * 4, s));
  HIP_TRY(launch_fill_zero(P.B, (size_t)P.ldz * 4, s));
  if (P.n_obs > 0) HIP_TRY(launch_fill_zero(P.ob_acc, (size_t)(P.ldz + 1) * 8, s));
  HIP_TRY(launch_fill_zero(P.sp_cnt, (size_t)P.Mp_pad * 4, s));
  return ENSF_OK;
}

ensf_status prep_problem(ensf_ctx* c, const ProbDev& P, bool score_mode, hipStream_t s) {
  const int prec = c->opt.precision;
  ensf_status st = zero_problem(P, prec, s);
  if (st != ENSF_OK) return st;
  HIP_TRY(launch_densify(P, c->d_counters + 1, s));
  HIP_TRY(launch_prep_rows(prec, P, s));
  if (prec != kFP32) HIP_TRY(launch_transpose(P, s));
  if (score_mode)
    HIP_TRY(launch_load_z(P, s));
  else
    HIP_TRY(launch_init_z(P, s));
  return ENSF_OK;
}

ensf_status ensure_softmax_smem(ensf_ctx* c, int max_ldn) {
  const size_t bytes = (size_t)max_ldn * sizeof(double);
  if (bytes > 64 * 1024 && bytes > c->softmax_smem_set) {
    HIP_TRY(set_softmax_smem_limit(bytes));
    c->softmax_smem_set = bytes;
  }
  return ENSF_OK;
}

ensf_status launch_grams(ensf_ctx* c, const Plan& plan, const Uploaded& u, int k, hipStream_t s) {
  for (size_t g = 0; g < plan.groups.size(); ++g)
    HIP_TRY(launch_gram(c->opt.precision, plan.groups[g].tiles.gram, plan.groups[g].tiles.gram_bk,
                        plan.groups[g].tiles.gram_st, u.gram[g], k, s));
  return ENSF_OK;
}

ensf_status launch_wxs(ensf_ctx* c, const Plan& plan, const Uploaded& u, int k, hipStream_t s) {
  for (size_t g = 0; g < plan.groups.size(); ++g)
    HIP_TRY(launch_wx(c->opt.precision, plan.groups[g].tiles.wx, plan.groups[g].tiles.wx_bk,
                      plan.groups[g].tiles.wx_st, false, c->opt.wx_sparse != 0, u.wx[g], k,
                      c->d_counters, s));
  return ENSF_OK;
}

ensf_status enqueue_steps(ensf_ctx* c, const Plan& plan, const Uploaded& u, hipStream_t s) {
  for (int k = 0; k < plan.kmax; ++k) {
    ensf_status st = launch_grams(c, plan, u, k, s);
    if (st != ENSF_OK) return st;
    HIP_TRY(launch_softmax(c->opt.precision, u.rows, k, plan.max_ldn, s));
    st = launch_wxs(c, plan, u, k, s);
    if (st != ENSF_OK) return st;
  }
  return ENSF_OK;
}

ensf_status collect_phase_times(ensf_ctx* c) {
  for (const auto& pr : c->pending) {
    HIP_TRY(hipEventSynchronize(c->events[pr.first + 4 * pr.second - 1]));
    for (int k = 0; k < pr.second; ++k) {
      const int b = pr.first + 4 * k;
      for (int ph = 0; ph < 3; ++ph) {
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, c->events[b + ph], c->events[b + ph + 1]));
        c->phase_ms[ph] += ms;
      }
    }
    c->phase_count += pr.second;
  }
  c->pending.clear();
  c->events_used = 0;
  return ENSF_OK;
}

ensf_status enqueue_steps_profiled(ensf_ctx* c, const Plan& plan, const Uploaded& u,
                                   hipStream_t s) {
  const size_t need = c->events_used + 4 * (size_t)plan.kmax;
  while (c->events.size() < need) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    c->events.push_back(e);
  }
  const size_t first = c->events_used;
  for (int k = 0; k < plan.kmax; ++k) {
    hipEvent_t* ev = &c->events[first + 4 * k];
    HIP_TRY(hipEventRecord(ev[0], s));
    ensf_status st = launch_grams(c, plan, u, k, s);
    if (st != ENSF_OK) return st;
    HIP_TRY(hipEventRecord(ev[1], s));
    HIP_TRY(launch_softmax(c->opt.precision, u.rows, k, plan.max_ldn, s));
    HIP_TRY(hipEventRecord(ev[2], s));
    st = launch_wxs(c, plan, u, k, s);
    if (st != ENSF_OK) return st;
    HIP_TRY(hipEventRecord(ev[3], s));
  }
  c->events_used = need;
  c->pending.emplace_back((int)first, plan.kmax);
  return ENSF_OK;
}

// use_graph 2: the pseudo-time loop as one cooperative launch with grid-wide barriers, when
// the plan's tiles are the persistent kernel's.  It is not the default: on MI355X a grid-wide
// barrier (device-scope release and acquire across the eight XCDs' L2 caches) costs more
// than the launch of a graph node, so the graph is faster even for the smallest problems
// (2x64x64, N = 20: 46 us per pseudo-step against 14 us).
bool use_persistent(const ensf_ctx* c, const Plan& plan) {
  if (c->opt.use_graph != 2) return false;
  if (c->profile || c->opt.wx_sparse || plan.groups.size() != 1) return false;
  const TileChoice& t = plan.groups[0].tiles;
  return persistent_tiles(c->opt.precision, t.gram, t.gram_bk, t.gram_st, t.wx, t.wx_bk,
                          t.wx_st);
}

ensf_status run_steps(ensf_ctx* c, const Plan& plan, const Uploaded& u, hipStream_t s) {
  if (use_persistent(c, plan)) {
    unsigned* bar = reinterpret_cast<unsigned*>(c->d_counters + 2);
    HIP_TRY(launch_fill_zero(bar, sizeof(unsigned long long), s));
    PersistArgs a{u.gram[0], u.rows, u.wx[0], plan.kmax, plan.max_ldn, bar,
                  reinterpret_cast<unsigned*>(c->d_counters + 3), c->d_counters,
                  200000};
    HIP_TRY(launch_persistent(c->opt.precision, a, 1024, s));
    return ENSF_OK;
  }
  if (c->profile) {
    if (c->events_used > 4096) {
      ensf_status st = collect_phase_times(c);
      if (st != ENSF_OK) return st;
    }
    return enqueue_steps_profiled(c, plan, u, s);
  }
  if (!c->opt.use_graph) return enqueue_steps(c, plan, u, s);
  GraphKey key;
  auto addp = [&](const void* p) { key.sig.push_back((int64_t)reinterpret_cast<uintptr_t>(p)); };
  key.sig = {c->opt.precision, plan.kmax, plan.max_ldn, u.rows.np, u.rows.total};
  addp(u.rows.desc);
  addp(u.rows.pre);
  addp(c->d_counters);
  for (size_t g = 0; g < plan.groups.size(); ++g) {
    const TileChoice& t = plan.groups[g].tiles;
    key.sig.insert(key.sig.end(), {t.gram, t.wx, t.gram_bk, t.wx_bk, t.gram_st, t.wx_st,
                                   u.gram[g].np, u.gram[g].total, u.wx[g].total});
    addp(u.gram[g].desc);
    addp(u.gram[g].pre);
    addp(u.wx[g].pre);
  }
  if (!(c->gexec && key == c->gkey)) {
    if (c->gexec) {
      HIP_TRY(hipGraphExecDestroy(c->gexec));
      c->gexec = nullptr;
    }
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    ensf_status st = enqueue_steps(c, plan, u, c->cap_stream);
    hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
    if (st != ENSF_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e);
    e = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      c->gexec = nullptr;
      return hip_fail(e);
    }
    c->gkey = key;
  }
  HIP_TRY(hipGraphLaunch(c->gexec, s));
  return ENSF_OK;
}

// Every call on a context rewrites the context's workspace and descriptor table.  A call on
// a stream other than the previous call's first makes its stream wait for the end of that
// call (done_event), so calls on one context run in call order whatever streams they use.
ensf_status order_after_previous(ensf_ctx* c, hipStream_t s) {
  if (c->has_last_stream && c->last_stream != s)
    HIP_TRY(hipStreamWaitEvent(s, c->done_event, 0));
  return ENSF_OK;
}

ensf_status mark_call_end(ensf_ctx* c, hipStream_t s) {
  HIP_TRY(hipEventRecord(c->done_event, s));
  c->last_stream = s;
  c->has_last_stream = true;
  return ENSF_OK;
}

ensf_status analysis_impl(ensf_ctx* c, const std::vector<ensf_problem>& probs, hipStream_t s,
                          const TileChoice* force) {
  for (const auto& p : probs) {
    ensf_status st = validate(p);
    if (st != ENSF_OK) return st;
  }
  clear_stale_hip_error();
  HIP_TRY(hipSetDevice(c->device));
  ensf_status st = order_after_previous(c, s);
  if (st != ENSF_OK) return st;
  Plan plan;
  st = build_plan(c, probs, plan, force);
  if (st != ENSF_OK) return st;
  st = ensure_workspace(c, plan.ws_needed);
  if (st != ENSF_OK) return st;
  bind_plan(c, probs, plan);
  st = ensure_softmax_smem(c, plan.max_ldn);
  if (st != ENSF_OK) return st;
  Uploaded u;
  st = upload_plan(c, plan, s, u);
  if (st != ENSF_OK) return st;
  for (const ProbDev& P : plan.desc) {
    st = prep_problem(c, P, false, s);
    if (st != ENSF_OK) return st;
  }
  st = run_steps(c, plan, u, s);
  if (st != ENSF_OK) return st;
  for (const ProbDev& P : plan.desc) {
    if (c->opt.spread_relax > 0.0 && P.Mp > 1 && P.N > 1)
      HIP_TRY(launch_relax(P, c->opt.spread_relax, s));
    HIP_TRY(launch_store_post(P, s));
  }
  return mark_call_end(c, s);
}

ensf_status validate_options(const ensf_options& o) {
  if (o.precision < 0 || o.precision > 2 || o.obs_op < 0 || o.obs_op > 1 || o.lik_step < 0 ||
      o.lik_step > 1 || o.wx_sparse < 0 || o.wx_sparse > 1 || o.use_graph < 0 || o.use_graph > 3)
    return ENSF_EINVAL;
  if (!(o.eps_alpha > 0.0 && o.eps_alpha < 1.0)) return ENSF_EINVAL;
  if (!(o.spread_relax >= 0.0 && o.spread_relax <= 1.0)) return ENSF_EINVAL;
  return ENSF_OK;
}

// Layout of run_in_workspace's buffer: the two device counters, the descriptor table, then
// the problem's workspace, each 256-byte aligned.  A context-free plan with the built-in
// tile heuristic (no tune table, no graph).
constexpr size_t kCounterBytes = 256;

struct WsLayout {
  Plan plan;
  Uploaded u;
  size_t table = 0, total = 0;
};

ensf_status plan_in_workspace(ensf_ctx& tmp, const ensf_problem& p, WsLayout& L) {
  const TileChoice tc = heuristic_tiles(p.n_members, p.n_particles);
  ensf_status st = build_plan(&tmp, {p}, L.plan, &tc);
  if (st != ENSF_OK) return st;
  L.table = (size_t)round_up((int64_t)stage_plan(L.plan, nullptr, nullptr, L.u), kAlign);
  L.total = kCounterBytes + L.table + L.plan.ws_needed;
  return ENSF_OK;
}

// ----- tune cache: a flat JSON object {"key": [gram, wx, split_scale], ...}
void load_tune_cache(ensf_ctx* c) {
  if (c->tune_path.empty()) return;
  FILE* fp = fopen(c->tune_path.c_str(), "r");
  if (!fp) return;
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, fp)) > 0) txt.append(buf, n);
  fclose(fp);
  size_t pos = 0;
  while ((pos = txt.find('"', pos)) != std::string::npos) {
    const size_t end = txt.find('"', pos + 1);
    if (end == std::string::npos) break;
    const std::string key = txt.substr(pos + 1, end - pos - 1);
    // [gram, wx, split_scale, gram_bk, wx_bk, gram_st, wx_st]; a 4-entry form gives one
    // k-step depth for both kernels and two stages
    TileChoice tc;
    int bk = 32;
    const int got = sscanf(txt.c_str() + end + 1, " : [ %d , %d , %lf , %d , %d , %d , %d ]",
                           &tc.gram, &tc.wx, &tc.split_scale, &bk, &tc.wx_bk, &tc.gram_st,
                           &tc.wx_st);
    tc.gram_bk = bk;
    if (got == 4) tc.wx_bk = bk;
    auto ok_bk = [](int v) { return v == 32 || v == 64; };
    auto ok_st = [](int v) { return v == 1 || v == 2; };
    if (got >= 3 && tc.gram >= 0 && tc.gram < kNumGram && tc.wx >= 0 && tc.wx < kNumWx &&
        ok_bk(tc.gram_bk) && ok_bk(tc.wx_bk) && ok_st(tc.gram_st) && ok_st(tc.wx_st) &&
        gram_variant_exists(tc.gram, tc.gram_bk))
      c->tune[key] = tc;
    pos = end + 1;
  }
}

void save_tune_cache(ensf_ctx* c) {
  if (c->tune_path.empty()) return;
  FILE* fp = fopen(c->tune_path.c_str(), "w");
  if (!fp) return;
  fprintf(fp, "{\n");
  size_t i = 0;
  for (const auto& kv : c->tune)
    fprintf(fp, "  \"%s\": [%d, %d, %.3f, %d, %d, %d, %d]%s\n", kv.first.c_str(),
            kv.second.gram, kv.second.wx, kv.second.split_scale, kv.second.gram_bk,
            kv.second.wx_bk, kv.second.gram_st, kv.second.wx_st, ++i < c->tune.size() ? "," : "");
  fprintf(fp, "}\n");
  fclose(fp);
}

}  // namespace

namespace ensf {

size_t workspace_bytes(const ensf_options& o, const ensf_problem& p) {
  if (validate_options(o) != ENSF_OK || validate(p) != ENSF_OK) return 0;
  ensf_ctx tmp;
  tmp.opt = o;
  WsLayout L;
  return plan_in_workspace(tmp, p, L) == ENSF_OK ? L.total : 0;
}

ensf_status run_in_workspace(const ensf_options& o, const ensf_problem& p, char* ws,
                             size_t ws_bytes, unsigned long long* counters, hipStream_t s) {
  ensf_status st = validate_options(o);
  if (st == ENSF_OK) st = validate(p);
  if (st != ENSF_OK) return st;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) != 0) return ENSF_EINVAL;
  clear_stale_hip_error();
  ensf_ctx tmp;   // options and views only: owns no device or pinned memory
  tmp.opt = o;
  tmp.device = o.device;
  WsLayout L;
  st = plan_in_workspace(tmp, p, L);
  if (st != ENSF_OK) return st;
  if (L.total > ws_bytes) return ENSF_ESCRATCH;
  char* tab = ws + kCounterBytes;
  tmp.ws = tab + L.table;
  tmp.ws_bytes = L.plan.ws_needed;
  tmp.d_counters = counters ? counters : reinterpret_cast<unsigned long long*>(ws);
  if (!counters) HIP_TRY(launch_fill_zero(ws, kCounterBytes, s));
  const std::vector<ensf_problem> probs{p};
  bind_plan(&tmp, probs, L.plan);
  std::vector<char> host(L.table);
  stage_plan(L.plan, host.data(), tab, L.u);
  HIP_TRY(launch_put_bytes(tab, host.data(), host.size(), s));
  if (L.plan.max_ldn * sizeof(double) > 64 * 1024)
    HIP_TRY(set_softmax_smem_limit((size_t)L.plan.max_ldn * sizeof(double)));
  const ProbDev& P = L.plan.desc[0];
  st = prep_problem(&tmp, P, false, s);
  if (st == ENSF_OK) st = enqueue_steps(&tmp, L.plan, L.u, s);
  if (st != ENSF_OK) return st;
  if (o.spread_relax > 0.0 && P.Mp > 1 && P.N > 1) HIP_TRY(launch_relax(P, o.spread_relax, s));
  HIP_TRY(launch_store_post(P, s));
  return ENSF_OK;
}

}  // namespace ensf

extern "C" {

void ensf_default_options(ensf_options* opt) {
  if (!opt) return;
  opt->precision = ENSF_PREC_FP32;
  opt->obs_op = ENSF_OBS_ARCTAN;
  opt->lik_step = ENSF_LIK_EXPLICIT;
  opt->wx_sparse = 0;
  opt->eps_alpha = 0.05;
  opt->spread_relax = 0.0;
  opt->use_graph = 1;
  opt->device = 0;
  opt->tune_cache = nullptr;
}

ensf_status ensf_create(const ensf_options* opt, ensf_ctx** out) {
  if (!out) return ENSF_EINVAL;
  *out = nullptr;
  ensf_options o;
  ensf_default_options(&o);
  if (opt) o = *opt;
  if (validate_options(o) != ENSF_OK) return ENSF_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return ENSF_EHIP;
  if (o.device < 0 || o.device >= ndev) return ENSF_EINVAL;
  HIP_TRY(hipSetDevice(o.device));
  ensf_ctx* c = new ensf_ctx();
  c->opt = o;
  c->device = o.device;
  const char* tp = o.tune_cache ? o.tune_cache : getenv("ENSF_TUNE_CACHE");
  if (tp) c->tune_path = tp;
  c->opt.tune_cache = nullptr;
  hipError_t e = hipMalloc(&c->d_counters, 4 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMemset(c->d_counters, 0, 4 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->tab_event, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->done_event, hipEventDisableTiming);
  if (e != hipSuccess) {
    ensf_destroy(c);
    return hip_fail(e);
  }
  load_tune_cache(c);
  *out = c;
  return ENSF_OK;
}

ensf_status ensf_analysis(ensf_ctx* ctx, const float* d_prior, int32_t n_members, int64_t dim,
                          float* d_post, int32_t n_particles, const int32_t* d_obs_idx,
                          const float* d_obs_val, int64_t n_obs, float obs_sigma,
                          int32_t n_steps, uint64_t seed, uint32_t filter_id, void* stream) {
  if (!ctx) return ENSF_EINVAL;
  ensf_problem p{d_prior, n_members, dim, d_post, n_particles, d_obs_idx, d_obs_val,
                 n_obs, obs_sigma, n_steps, seed, filter_id};
  return analysis_impl(ctx, {p}, reinterpret_cast<hipStream_t>(stream), nullptr);
}

ensf_status ensf_analysis_batched(ensf_ctx* ctx, const ensf_problem* probs, int32_t n_problems,
                                  void* stream) {
  if (!ctx || !probs || n_problems < 1) return ENSF_EINVAL;
  std::vector<ensf_problem> v(probs, probs + n_problems);
  return analysis_impl(ctx, v, reinterpret_cast<hipStream_t>(stream), nullptr);
}

ensf_status ensf_score(ensf_ctx* ctx, const float* d_prior, int32_t n_members, int64_t dim,
                       const float* d_z, int32_t n_particles, const int32_t* d_obs_idx,
                       const float* d_obs_val, int64_t n_obs, float obs_sigma, double t,
                       float* d_score, float* d_weights, void* stream) {
  if (!ctx || !d_z || !d_score) return ENSF_EINVAL;
  if (!(t > 0.0 && t <= 1.0)) return ENSF_EINVAL;
  ensf_problem p{d_prior, n_members, dim, d_score, n_particles, d_obs_idx, d_obs_val,
                 n_obs, obs_sigma, 1, 0, 0};
  ensf_status st = validate(p);
  if (st != ENSF_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  clear_stale_hip_error();
  HIP_TRY(hipSetDevice(ctx->device));
  st = order_after_previous(ctx, s);
  if (st != ENSF_OK) return st;
  std::vector<ensf_problem> probs{p};
  Plan plan;
  st = build_plan(ctx, probs, plan, nullptr);
  if (st != ENSF_OK) return st;
  st = ensure_workspace(ctx, plan.ws_needed);
  if (st != ENSF_OK) return st;
  bind_plan(ctx, probs, plan);
  ProbDev& P = plan.desc[0];
  P.zin = d_z;
  P.score_out = d_score;
  P.weights_out = d_weights;
  P.post = nullptr;
  P.t_score = t;
  st = ensure_softmax_smem(ctx, plan.max_ldn);
  if (st != ENSF_OK) return st;
  Uploaded u;
  st = upload_plan(ctx, plan, s, u);
  if (st != ENSF_OK) return st;
  st = prep_problem(ctx, P, true, s);
  if (st != ENSF_OK) return st;
  const int prec = ctx->opt.precision;
  const TileChoice& tiles = plan.groups[0].tiles;
  HIP_TRY(launch_gram(prec, tiles.gram, tiles.gram_bk, tiles.gram_st, u.gram[0], -1, s));
  HIP_TRY(launch_softmax(prec, u.rows, -1, plan.max_ldn, s));
  HIP_TRY(launch_wx(prec, tiles.wx, 32, 2, true, false, u.wx[0], -1, ctx->d_counters, s));
  return mark_call_end(ctx, s);
}

ensf_status ensf_rng_normal(uint64_t seed, uint32_t filter_id, uint32_t step, uint32_t particle,
                            int64_t n, float* d_out, uint32_t* d_raw_words, void* stream) {
  if (!d_out || n < 1 || n > (int64_t(1) << 34)) return ENSF_EINVAL;
  clear_stale_hip_error();
  HIP_TRY(launch_rng_normal(seed, filter_id, step, particle, n, d_out, d_raw_words,
                            reinterpret_cast<hipStream_t>(stream)));
  return ENSF_OK;
}

ensf_status ensf_ensemble_stats(const float* d_ens, int32_t n, int64_t dim, float* d_mean,
                                float* d_spread, void* stream) {
  if (!d_ens || !d_mean || !d_spread || n < 2 || dim < 1) return ENSF_EINVAL;
  clear_stale_hip_error();
  HIP_TRY(launch_stats(d_ens, n, dim, d_mean, d_spread, reinterpret_cast<hipStream_t>(stream)));
  return ENSF_OK;
}

ensf_status ensf_sync_status(ensf_ctx* ctx, int64_t* nonfinite_count) {
  if (!ctx) return ENSF_EINVAL;
  HIP_TRY(hipSetDevice(ctx->device));
  if (ctx->has_last_stream) HIP_TRY(hipStreamSynchronize(ctx->last_stream));
  unsigned long long h[4] = {0, 0, 0, 0};
  HIP_TRY(hipMemcpy(h, ctx->d_counters, sizeof h, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(ctx->d_counters, 0, sizeof h));
  if (nonfinite_count) *nonfinite_count = (int64_t)h[0];
  if (h[3]) {   // a grid barrier of the persistent pseudo-time loop gave up waiting
    ensf::record_hip_error(hipErrorLaunchTimeOut);
    return ENSF_EHIP;
  }
  if (h[1]) return ENSF_EINVAL;
  if (h[0]) return ENSF_ENONFINITE;
  return ENSF_OK;
}

ensf_status ensf_autotune(ensf_ctx* ctx, const ensf_problem* prob, void* stream) {
  return ensf_autotune_batched(ctx, prob, 1, stream);
}

ensf_status ensf_autotune_batched(ensf_ctx* ctx, const ensf_problem* probs_in, int32_t n_problems,
                                  void* stream) {
  if (!ctx || !probs_in || n_problems < 1) return ENSF_EINVAL;
  ensf_status st = ENSF_OK;
  for (int32_t f = 0; f < n_problems && st == ENSF_OK; ++f) st = validate(probs_in[f]);
  if (st != ENSF_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  std::vector<ensf_problem> probs(probs_in, probs_in + n_problems);
  for (auto& q : probs) q.n_steps = std::min(q.n_steps, 8);
  const ensf_problem p = probs[dominant_problem(probs)];
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const int use_graph = ctx->opt.use_graph;
  ctx->opt.use_graph = 0;
  // ENSF_TUNE_LOG set: one line per timed candidate on stderr.
  const bool log = getenv("ENSF_TUNE_LOG") != nullptr;
  // Time of one candidate: two timed analyses after a warm-up.
  auto time_of = [&](const TileChoice& tc, float& ms_sum) {
    ms_sum = 0.0f;
    for (int rep = 0; rep < 3 && st == ENSF_OK; ++rep) {
      st = analysis_impl(ctx, probs, s, &tc);  // warm-up on rep 0
      if (st != ENSF_OK || rep == 0) continue;
      if (hipEventRecord(e0, s) != hipSuccess) st = ENSF_EHIP;
      if (st == ENSF_OK) st = analysis_impl(ctx, probs, s, &tc);
      if (st == ENSF_OK && hipEventRecord(e1, s) != hipSuccess) st = ENSF_EHIP;
      if (st == ENSF_OK && hipEventSynchronize(e1) != hipSuccess) st = ENSF_EHIP;
      float ms = 0;
      if (st == ENSF_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = ENSF_EHIP;
      ms_sum += ms;
    }
    if (log && st == ENSF_OK)
      fprintf(stderr, "ensf_autotune: gram %d/%d/%d split %.2f wx %d/%d/%d: %.3f ms\n",
              tc.gram, tc.gram_bk, tc.gram_st, tc.split_scale, tc.wx, tc.wx_bk, tc.wx_st,
              ms_sum / 2);
    if (log) fflush(stderr);
    return st == ENSF_OK;
  };
  // Coordinate search: the Gram side (tile, split-K scale, k-step, stages) with the W.X
  // side fixed, then the W.X side with the Gram side fixed, then the Gram side again.
  TileChoice best = heuristic_tiles(p.n_members, p.n_particles);
  float best_ms = INFINITY;
  const double scales[] = {0.25, 0.5, 1.0, 2.0, 4.0};
  for (int pass = 0; pass < 3 && st == ENSF_OK; ++pass) {
    const TileChoice base = best;
    if (pass != 1) {
      for (int gc = 0; gc < kNumGram && st == ENSF_OK; ++gc)
        for (double sc : scales)
          for (int bk : {32, 64})
            for (int ns : {1, 2}) {
              if (!gram_variant_exists(gc, bk)) continue;
              TileChoice tc = base;
              tc.gram = gc;
              tc.split_scale = sc;
              tc.gram_bk = bk;
              tc.gram_st = ns;
              float ms;
              if (!time_of(tc, ms)) break;
              if (ms < best_ms) {
                best_ms = ms;
                best = tc;
              }
            }
    } else {
      for (int wc = 0; wc < kNumWx && st == ENSF_OK; ++wc)
        for (int bk : {32, 64})
          for (int ns : {1, 2}) {
            TileChoice tc = base;
            tc.wx = wc;
            tc.wx_bk = bk;
            tc.wx_st = ns;
            float ms;
            if (!time_of(tc, ms)) break;
            if (ms < best_ms) {
              best_ms = ms;
              best = tc;
            }
          }
    }
  }
  ctx->opt.use_graph = use_graph;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != ENSF_OK) return st;
  ctx->tune[tune_key(ctx->opt.precision, p.n_members, p.n_particles, p.dim, n_problems)] = best;
  save_tune_cache(ctx);
  return ENSF_OK;
}

ensf_status ensf_profile_phases(ensf_ctx* ctx, int32_t enable) {
  if (!ctx) return ENSF_EINVAL;
  HIP_TRY(hipSetDevice(ctx->device));
  ensf_status st = collect_phase_times(ctx);
  if (st != ENSF_OK) return st;
  ctx->profile = enable != 0;
  for (double& m : ctx->phase_ms) m = 0;
  ctx->phase_count = 0;
  return ENSF_OK;
}

ensf_status ensf_phase_times(ensf_ctx* ctx, double* ms, int64_t* count) {
  if (!ctx || !ms) return ENSF_EINVAL;
  HIP_TRY(hipSetDevice(ctx->device));
  ensf_status st = collect_phase_times(ctx);
  if (st != ENSF_OK) return st;
  for (int i = 0; i < 3; ++i) ms[i] = ctx->phase_ms[i];
  if (count) *count = ctx->phase_count;
  return ENSF_OK;
}

ensf_status ensf_destroy(ensf_ctx* ctx) {
  if (!ctx) return ENSF_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
  if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->d_tab) (void)hipFree(ctx->d_tab);
  if (ctx->h_tab) (void)hipHostFree(ctx->h_tab);
  if (ctx->d_counters) (void)hipFree(ctx->d_counters);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->tab_event) (void)hipEventDestroy(ctx->tab_event);
  if (ctx->done_event) (void)hipEventDestroy(ctx->done_event);
  delete ctx;
  return ENSF_OK;
}

const char* ensf_last_error_string(void) {
  return g_last_error == hipSuccess ? "" : hipGetErrorString(g_last_error);
}

const char* ensf_status_string(ensf_status s) {
  switch (s) {
    case ENSF_OK: return "ok";
    case ENSF_EINVAL: return "invalid argument";
    case ENSF_ENOMEM: return "out of memory";
    case ENSF_EHIP: return "HIP runtime error";
    case ENSF_ENONFINITE: return "non-finite particle values";
    case ENSF_EUNSUPPORTED: return "unsupported";
    case ENSF_ESCRATCH: return "problem exceeds the no-allocation scratch buffer";
  }
  return "unknown status";
}

}  // extern "C"
