// C ABI of libnnef (declared in include/nnef.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/nnef.h"
#include "planner.hpp"

using namespace nnef;

namespace {
thread_local std::string g_last_error;

nnef_status fail(nnef_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

nnef_status hip_fail(int e, const char* what) {
  return fail(NNEF_E_DEVICE, std::string(what) + ": " + hipGetErrorString((hipError_t)e));
}

int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}
}  // namespace

// Error reporting for entry points defined in other translation units.
namespace nnef {
nnef_status report_error(nnef_status st, const std::string& msg) { return fail(st, msg); }
nnef_status report_hip_error(int e, const char* what) { return hip_fail(e, what); }
}  // namespace nnef

struct nnef_plan_s {
  Model m;
  LossSpec ls;
  nnef_options opt;
  std::vector<BlockPlan> blocks;
  std::vector<int64_t> ws_sizes;   // floats per workspace buffer
  std::vector<float*> ws;
  void* ws_base = nullptr;
  std::vector<void*> tables;       // device index tables
  float* partN = nullptr;
  float* partD = nullptr;
  double* loss_part = nullptr;
  double* vloss_part = nullptr;    // validation-entry loss partials (split packs)
  double* loss_tmp = nullptr;
  float* dcol = nullptr;
  float* ypack = nullptr;          // data with missing entries stored as -1
  int64_t n_data = 0;
  int max_wg = 0;
  std::vector<int64_t> numel;
  int64_t numel_total = 0;
  float* learn_buf = nullptr;      // 3 x numel_total: theta_{t-1}, theta_{t-2}, proposal
  double* learn_small = nullptr;   // sigma per factor, then losses
  std::string description;
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
};

extern "C" {

void nnef_default_options(nnef_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->eps = 1e-10;
  o->prec = NNEF_FP32;
  o->deterministic = 1;
}

const char* nnef_last_error(void) { return g_last_error.c_str(); }

static void drop_events(nnef_plan_s* p) {
  for (auto& e : p->events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  p->events.clear();
}

static void free_plan(nnef_plan_s* p) {
  if (!p) return;
  drop_events(p);
  if (p->ws_base) (void)hipFree(p->ws_base);
  for (void* t : p->tables) (void)hipFree(t);
  if (p->partN) (void)hipFree(p->partN);
  if (p->partD) (void)hipFree(p->partD);
  if (p->loss_part) (void)hipFree(p->loss_part);
  if (p->vloss_part) (void)hipFree(p->vloss_part);
  if (p->loss_tmp) (void)hipFree(p->loss_tmp);
  if (p->dcol) (void)hipFree(p->dcol);
  if (p->ypack) (void)hipFree(p->ypack);
  if (p->learn_buf) (void)hipFree(p->learn_buf);
  if (p->learn_small) (void)hipFree(p->learn_small);
  delete p;
}

void nnef_plan_destroy(nnef_plan_t p) { free_plan(p); }

int nnef_plan_num_factors(nnef_plan_t p) { return p ? (int)p->m.ops.size() : 0; }

int64_t nnef_plan_factor_numel(nnef_plan_t p, int l) {
  if (!p || l < 0 || l >= (int)p->numel.size()) return -1;
  return p->numel[l];
}

size_t nnef_plan_describe(nnef_plan_t p, char* buf, size_t n) {
  if (!p) return 0;
  const std::string& s = p->description;
  if (buf && n) {
    const size_t k = std::min(n - 1, s.size());
    std::memcpy(buf, s.data(), k);
    buf[k] = 0;
  }
  return s.size();
}

static nnef_status upload_table(nnef_plan_s* p, const std::vector<uint32_t>& t, uint32_t** out) {
  void* d = nullptr;
  const size_t bytes = std::max<size_t>(4, t.size() * 4);
  if (hipMalloc(&d, bytes) != hipSuccess) return fail(NNEF_E_NOMEM, "hipMalloc of an index table failed");
  p->tables.push_back(d);
  if (!t.empty() && hipMemcpy(d, t.data(), t.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
    return fail(NNEF_E_DEVICE, "copy of an index table failed");
  *out = (uint32_t*)d;
  return NNEF_OK;
}

// Contraction precision as nnef_plan_describe states it (batched plans keep
// an FP32 reconstruction).
static const char* prec_name(int prec, bool batched) {
  switch (prec) {
    case NNEF_BF16: return " contract=bf16";
    case NNEF_FP16: return " contract=fp16";
    case NNEF_BF16_ALL: return batched ? " contract=bf16" : " contract=bf16 recon=bf16";
    default: return batched ? " contract=fp16" : " contract=fp16 recon=fp16";
  }
}

// Plan set-up shared by nnef_plan and the batched plan.  with_pack: allocate
// the buffer that holds the mask-packed data; target_wg: workgroups per pass.
static nnef_status plan_create(const char* model_str, const int64_t* mode_sizes, int n_modes,
                               const int64_t* ranks, int n_ranks, double alpha, double beta,
                               const nnef_options* opt, bool with_pack, int target_wg,
                               nnef_plan_t* out, int batched = 0, bool dry_run = false) {
  // batched: 0 = a single plan (bilinear lowering, else the direct one); 1 = a
  // batched problem whose blocks need no side operands; 2 = a batched problem
  // with side operands and chain-backs (no direct lowering in batched plans)
  if (!model_str || !out) return fail(NNEF_E_ARG, "model_str and out must not be NULL");
  *out = nullptr;
  auto* p = new nnef_plan_s();
  nnef_default_options(&p->opt);
  if (opt) {
    p->opt = *opt;
    if (!(p->opt.eps > 0) || !std::isfinite(p->opt.eps)) {
      free_plan(p);
      return fail(NNEF_E_ARG, "eps must be a positive finite number");
    }
    if (p->opt.prec < NNEF_FP32 || p->opt.prec > NNEF_FP16_ALL) {
      free_plan(p);
      return fail(NNEF_E_ARG, "prec must be one of NNEF_FP32, NNEF_BF16, NNEF_FP16, NNEF_BF16_ALL, NNEF_FP16_ALL");
    }
    if (p->opt.family < NNEF_AB || p->opt.family > NNEF_JS) {
      free_plan(p);
      return fail(NNEF_E_ARG, "family must be one of NNEF_AB, NNEF_NEGBIN, NNEF_BINOMIAL, NNEF_JS");
    }
  }
  std::string err;
  if (parse_model(model_str, p->m, err) != ST_OK) {
    free_plan(p);
    return fail(NNEF_E_PARSE, err);
  }
  Model& m = p->m;
  if (n_modes != (int)m.out.size() || n_ranks != (int)m.latent.size() ||
      (n_modes && !mode_sizes) || (n_ranks && !ranks)) {
    free_plan(p);
    return fail(NNEF_E_SHAPE, "model string has " + std::to_string(m.out.size()) + " modes and " +
                                  std::to_string(m.latent.size()) + " contracted letters");
  }
  int64_t N = 1;
  p->n_data = 0;
  for (int i = 0; i < n_modes; ++i) {
    if (mode_sizes[i] <= 0) {
      free_plan(p);
      return fail(NNEF_E_SHAPE, "mode sizes must be positive");
    }
    m.size[(unsigned char)m.out[i]] = mode_sizes[i];
    N *= mode_sizes[i];
    if (N >= (int64_t(1) << 30)) {
      free_plan(p);
      return fail(NNEF_E_SHAPE, "the data tensor must have fewer than 2^30 entries");
    }
  }
  for (int i = 0; i < n_ranks; ++i) {
    if (ranks[i] <= 0) {
      free_plan(p);
      return fail(NNEF_E_SHAPE, "ranks must be positive");
    }
    m.size[(unsigned char)m.latent[i]] = ranks[i];
  }
  p->n_data = N;
  if ((p->opt.family == NNEF_AB ? make_loss(alpha, beta, p->ls, err)
                                : make_family(p->opt.family, p->opt.family_param, p->ls, err)) != ST_OK) {
    free_plan(p);
    return fail(NNEF_E_LOSS_UNSUPPORTED, err);
  }
  for (auto& t : m.ops) {
    int64_t n = 1;
    for (char c : t) n *= m.size[(unsigned char)c];
    p->numel.push_back(n);
  }
  // ---- lowering of every block
  size_t part_elems = 0;
  for (int l = 0; l < (int)m.ops.size(); ++l) {
    BlockPlan bp;
    Status st = lower_block(m, l, bp, p->ws_sizes, err, batched == 1);
    if (st == ST_UNSUPPORTED && batched == 0) {  // no bilinear split: per-entry latent sums
      std::string err2;
      st = lower_direct(m, l, bp, p->ws_sizes, err2, target_wg);
      if (st != ST_OK) err += "; " + err2;
    }
    if (st != ST_OK) {
      free_plan(p);
      return fail(st == ST_UNSUPPORTED ? NNEF_E_UNSUPPORTED : NNEF_E_SHAPE, err);
    }
    if (!bp.direct && !choose_geometry(m, bp, target_wg)) {
      free_plan(p);
      return fail(NNEF_E_SHAPE, "grid too large");
    }
    part_elems = std::max(part_elems, (size_t)bp.n_chunks * bp.nP * bp.KP);
    p->max_wg = std::max(p->max_wg, bp.n_wg);
    p->blocks.push_back(bp);
  }
  // ---- every buffer the kernels index with 32-bit offsets stays below 2^30 elements
  for (auto v : p->numel)
    if (v >= (int64_t(1) << 30)) {
      free_plan(p);
      return fail(NNEF_E_SHAPE, "a factor has 2^30 or more elements");
    }
  for (auto v : p->ws_sizes)
    if (v >= (int64_t(1) << 30)) {
      free_plan(p);
      return fail(NNEF_E_SHAPE, "an intermediate of the lowering has 2^30 or more elements");
    }
  if (part_elems >= (size_t(1) << 30)) {
    free_plan(p);
    return fail(NNEF_E_SHAPE, "partial sums need 2^30 or more elements");
  }
  if (dry_run) {  // lowering and geometry only: no device memory
    for (const auto& bp : p->blocks) {
      // batched plans contract in FP32 at widths 16 and 64
      const bool lp = !bp.direct && p->opt.prec != NNEF_FP32 && (!batched || bp.KP == 32);
      p->description += describe_block(m, bp) +
                        (lp ? prec_name(p->opt.prec, batched != 0) : " contract=fp32") +
                        "\n";
    }
    *out = p;
    return NNEF_OK;
  }
  // ---- device memory
  size_t ws_total = 0;
  for (auto s : p->ws_sizes) ws_total += (size_t)((s + 63) / 64 * 64);
  if (ws_total) {
    if (hipMalloc(&p->ws_base, ws_total * sizeof(float)) != hipSuccess) {
      free_plan(p);
      return fail(NNEF_E_NOMEM, "workspace allocation failed");
    }
    if (hipMemset(p->ws_base, 0, ws_total * sizeof(float)) != hipSuccess) {
      free_plan(p);
      return fail(NNEF_E_DEVICE, "workspace clear failed");
    }
  }
  size_t off = 0;
  for (auto s : p->ws_sizes) {
    p->ws.push_back((float*)p->ws_base + off);
    off += (size_t)((s + 63) / 64 * 64);
  }
  if (hipMalloc((void**)&p->partN, std::max<size_t>(1, part_elems) * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&p->partD, std::max<size_t>(1, part_elems) * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&p->loss_part, std::max(1, p->max_wg) * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&p->vloss_part, std::max(1, p->max_wg) * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&p->loss_tmp, sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&p->dcol, 64 * sizeof(float)) != hipSuccess ||
      (with_pack && hipMalloc((void**)&p->ypack, (size_t)N * sizeof(float)) != hipSuccess)) {
    free_plan(p);
    return fail(NNEF_E_NOMEM, "partial-sum allocation failed");
  }
  for (auto n : p->numel) p->numel_total += n;
  if ((int)m.ops.size() <= kMaxLearnFactors) {
    if (hipMalloc((void**)&p->learn_buf, (size_t)(3 * p->numel_total) * sizeof(float)) != hipSuccess ||
        hipMalloc((void**)&p->learn_small, (kMaxLearnFactors + 8) * sizeof(double)) != hipSuccess) {
      free_plan(p);
      return fail(NNEF_E_NOMEM, "extrapolation buffer allocation failed");
    }
  }
  for (auto& bp : p->blocks) {
    if (bp.direct) {
      nnef_status st = upload_table(p, offsets_table(m, bp.P), &bp.d_poff);
      if (st == NNEF_OK) st = upload_table(p, offsets_table(m, bp.Q), &bp.d_yq);
      if (st == NNEF_OK) st = upload_table(p, offsets_in(m, bp.P, m.ops[bp.ell]), &bp.d_thp);
      if (st == NNEF_OK) st = upload_table(p, offsets_in(m, bp.kappa, m.ops[bp.ell]), &bp.d_thr);
      for (int o : bp.others) {
        uint32_t *tp = nullptr, *tq = nullptr, *tl = nullptr;
        if (st == NNEF_OK) st = upload_table(p, offsets_in(m, bp.P, m.ops[o]), &tp);
        if (st == NNEF_OK) st = upload_table(p, offsets_in(m, bp.Q, m.ops[o]), &tq);
        if (st == NNEF_OK) st = upload_table(p, offsets_in(m, bp.kappa + bp.S, m.ops[o]), &tl);
        bp.d_opp.push_back(tp);
        bp.d_opq.push_back(tq);
        bp.d_oplat.push_back(tl);
      }
      if (st != NNEF_OK) {
        free_plan(p);
        return st;
      }
      p->description += describe_block(m, bp) + " contract=fp32\n";
      continue;
    }
    nnef_status st = upload_table(p, offsets_table(m, bp.P), &bp.d_poff);
    if (st == NNEF_OK) st = upload_table(p, offsets_table(m, bp.qo), &bp.d_qoyoff);
    if (st == NNEF_OK) {
      auto ib = inner_base_table(m, bp);
      if (!all_zero(ib)) st = upload_table(p, ib, &bp.d_inbase);
    }
    for (size_t i = 0; st == NNEF_OK && i < bp.outers.size(); ++i)
      st = upload_table(p, outer_row_table(m, bp, bp.outers[i]), &bp.d_orow[i]);
    if (st == NNEF_OK && bp.ones_buf >= 0) {
      const float one = 1.0f;
      if (hipMemcpy(p->ws[bp.ones_buf], &one, sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        st = fail(NNEF_E_DEVICE, "workspace init failed");
    }
    if (st != NNEF_OK) {
      free_plan(p);
      return st;
    }
    // batched plans contract in FP32 at widths 16 and 64
    const bool lp = !bp.direct && p->opt.prec != NNEF_FP32 && (!batched || bp.KP == 32);
    p->description += describe_block(m, bp) +
                      (lp ? prec_name(p->opt.prec, batched != 0) : " contract=fp32") + "\n";
  }
  if (hipDeviceSynchronize() != hipSuccess) {
    free_plan(p);
    return fail(NNEF_E_DEVICE, "device synchronisation failed after plan set-up");
  }
  *out = p;
  return NNEF_OK;
}

nnef_status nnef_plan(const char* model_str, const int64_t* mode_sizes, int n_modes,
                      const int64_t* ranks, int n_ranks, double alpha, double beta,
                      const nnef_options* opt, nnef_plan_t* out) {
  return plan_create(model_str, mode_sizes, n_modes, ranks, n_ranks, alpha, beta, opt, true,
                     env_int("NNEF_TARGET_WG", 512), out);
}

size_t nnef_plan_dry(const char* model_str, const int64_t* mode_sizes, int n_modes, const int64_t* ranks,
                     int n_ranks, double alpha, double beta, const nnef_options* opt, nnef_status* status,
                     char* buf, size_t buf_len) {
  nnef_plan_t p = nullptr;
  const nnef_status st = plan_create(model_str, mode_sizes, n_modes, ranks, n_ranks, alpha, beta, opt,
                                     false, env_int("NNEF_TARGET_WG", 512), &p, 0, true);
  if (status) *status = st;
  if (st != NNEF_OK) return 0;
  const size_t n = nnef_plan_describe(p, buf, buf_len);
  free_plan(p);
  return n;
}

// ---------------------------------------------------------------------------
static const float* tensor_ptr(const nnef_plan_s* p, const BlockPlan& bp, const TensorRef& t,
                               const float* const* factors) {
  switch (t.kind) {
    case TK_FACTOR: return factors[t.id];
    case TK_WS: return p->ws[t.id];
    case TK_NL: return p->ws[bp.NL_buf];
    default: return p->ws[bp.DL_buf];
  }
}

static EinsumArgs einsum_args(const nnef_plan_s* p, const BlockPlan& bp, const Step& st,
                              const float* const* factors) {
  const Model& m = p->m;
  EinsumArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n_in = (int)st.in.size();
  a.n_out = (int)st.out.subs.size();
  a.n_sum = (int)st.sum.size();
  a.n_out_total = 1;
  for (int d = 0; d < a.n_out; ++d) {
    const char c = st.out.subs[d];
    a.out_size[d] = m.size[(unsigned char)c];
    a.out_stride[d] = st.out.strides[d];
    a.n_out_total *= a.out_size[d];
  }
  for (int d = 0; d < a.n_sum; ++d) a.sum_size[d] = m.size[(unsigned char)st.sum[d]];
  for (int i = 0; i < a.n_in; ++i) {
    const TensorRef& t = st.in[i];
    a.in[i] = tensor_ptr(p, bp, t, factors);
    for (int d = 0; d < a.n_out; ++d) {
      const size_t pos = t.subs.find(st.out.subs[d]);
      a.in_out_stride[i][d] = pos == std::string::npos ? 0 : t.strides[pos];
    }
    for (int d = 0; d < a.n_sum; ++d) {
      const size_t pos = t.subs.find(st.sum[d]);
      a.in_sum_stride[i][d] = pos == std::string::npos ? 0 : t.strides[pos];
    }
  }
  a.out = const_cast<float*>(tensor_ptr(p, bp, st.out, factors));
  return a;
}

static int run_program(const nnef_plan_s* p, const BlockPlan& bp, const std::vector<Step>& prog,
                       const float* const* factors, hipStream_t s) {
  for (const Step& st : prog) {
    const int e = launch_einsum(einsum_args(p, bp, st, factors), s);
    if (e) return e;
  }
  return 0;
}

// Two contractions that differ only in their operand and output pointers.
static bool same_shape(const EinsumArgs& a, const EinsumArgs& b) {
  bool same = a.n_in == b.n_in && a.n_out == b.n_out && a.n_sum == b.n_sum && a.n_out_total == b.n_out_total;
  for (int d = 0; same && d < a.n_out; ++d) {
    same = a.out_size[d] == b.out_size[d] && a.out_stride[d] == b.out_stride[d];
    for (int j = 0; j < a.n_in; ++j) same = same && a.in_out_stride[j][d] == b.in_out_stride[j][d];
  }
  for (int d = 0; same && d < a.n_sum; ++d) {
    same = a.sum_size[d] == b.sum_size[d];
    for (int j = 0; j < a.n_in; ++j) same = same && a.in_sum_stride[j][d] == b.in_sum_stride[j][d];
  }
  return same;
}

// Two programs evaluated step by step together: the numerator and denominator
// chains of a block, built alike from N_L and D_L, share each launch.
static int run_program_pair(const nnef_plan_s* p, const BlockPlan& bp, const std::vector<Step>& pa,
                            const std::vector<Step>& pb, const float* const* factors, hipStream_t s) {
  if (pa.size() != pb.size()) {
    const int e = run_program(p, bp, pa, factors, s);
    return e ? e : run_program(p, bp, pb, factors, s);
  }
  for (size_t i = 0; i < pa.size(); ++i) {
    EinsumArgs a = einsum_args(p, bp, pa[i], factors);
    EinsumArgs b = einsum_args(p, bp, pb[i], factors);
    const bool same = same_shape(a, b);
    const int e = same ? launch_einsum(a, s, &b) : launch_einsum(a, s);
    if (e) return e;
    if (!same) {
      const int e2 = launch_einsum(b, s);
      if (e2) return e2;
    }
  }
  return 0;
}

static const float* piece_ptr(const nnef_plan_s* p, const Piece& pc, const float* const* factors) {
  return pc.factor >= 0 ? factors[pc.factor] : p->ws[pc.ws];
}

static FusedArgs fused_args(const nnef_plan_s* p, const BlockPlan& bp, const float* Y,
                            bool masked, const float* const* factors) {
  FusedArgs a;
  std::memset(&a, 0, sizeof(a));
  a.Y = Y;
  a.masked = masked ? 1 : 0;
  a.p_off = bp.d_poff;
  a.L = bp.L_direct ? factors[bp.ell] : p->ws[bp.L_buf];
  a.ldL = bp.ldL;
  a.K = bp.K;
  a.nP = (int)bp.nP;
  a.nqo = (int)bp.nqo;
  a.nqi = (int)bp.nqi;
  a.nqis = (int)((bp.nqi + bp.qstep - 1) / bp.qstep);
  a.qi_ystride = (int)bp.qi_ystride;
  a.qo_yoff = bp.d_qoyoff;
  const Piece& in = bp.pieces[bp.inner];
  a.inner = piece_ptr(p, in, factors);
  a.ld_in = in.ld;
  a.in_stride = (int)bp.in_stride;
  a.in_base = bp.d_inbase;
  a.nouter = (int)bp.outers.size();
  for (int i = 0; i < a.nouter; ++i) {
    const Piece& pc = bp.pieces[bp.outers[i]];
    a.outer[i] = piece_ptr(p, pc, factors);
    a.ld_out[i] = pc.ld;
    a.orow[i] = bp.d_orow[i];
  }
  a.n_steps = bp.n_steps;
  a.n_panels = bp.n_panels;
  a.steps_per_wave = bp.steps_per_wave;
  a.n_chunks = bp.n_chunks;
  a.n_wg = bp.n_wg;
  a.xcd_remap = bp.xcd_remap;
  a.wave_rows = bp.wave_rows;
  a.partN = p->partN;
  a.partD = p->partD;
  a.no_d = (p->ls.b_is_one() && !masked && bp.pieces_disjoint) ? 1 : 0;
  a.alpha = (float)p->ls.alpha;
  a.beta = (float)p->ls.beta;
  const double ab = p->ls.alpha * p->ls.beta, apb = p->ls.alpha + p->ls.beta;
  a.ab_inv = ab != 0 ? (float)(1.0 / ab) : 0.f;
  a.apb_inv = apb != 0 ? (float)(1.0 / apb) : 0.f;
  a.lk = p->ls.lk;
  a.fparam = (float)p->ls.fparam;
  a.prec = p->opt.prec;
  a.full = (bp.K == bp.KP && bp.nqi % bp.qstep == 0 && bp.nP % bp.rows == 0 && bp.in_stride == 1 &&
            bp.pieces[bp.inner].ld == bp.KP) ? 1 : 0;
  return a;
}

static DirectArgs direct_args(const nnef_plan_s* p, const BlockPlan& bp, const float* Y, bool masked,
                              const float* const* factors) {
  DirectArgs a;
  std::memset(&a, 0, sizeof(a));
  a.Y = Y;
  a.masked = masked ? 1 : 0;
  a.nP = (int)bp.nP;
  a.nQ = (int)bp.nQ;
  a.yp = bp.d_poff;
  a.yq = bp.d_yq;
  a.theta = factors[bp.ell];
  a.thp = bp.d_thp;
  a.thr = bp.d_thr;
  a.K = bp.K;
  a.KS = bp.KS;
  a.G = bp.G;
  a.n_ops = (int)bp.others.size();
  for (int j = 0; j < a.n_ops; ++j) {
    a.op[j] = factors[bp.others[j]];
    a.opp[j] = bp.d_opp[j];
    a.opq[j] = bp.d_opq[j];
    a.oplat[j] = bp.d_oplat[j];
  }
  a.rows_per_wg = bp.rows_per_wg;
  a.qlanes = bp.qlanes;
  a.q_per_chunk = bp.q_per_chunk;
  a.n_chunks = bp.n_chunks;
  a.n_panels = bp.n_panels;
  a.partN = p->partN;
  a.partD = p->partD;
  a.alpha = (float)p->ls.alpha;
  a.beta = (float)p->ls.beta;
  const double ab = p->ls.alpha * p->ls.beta, apb = p->ls.alpha + p->ls.beta;
  a.ab_inv = ab != 0 ? (float)(1.0 / ab) : 0.f;
  a.apb_inv = apb != 0 ? (float)(1.0 / apb) : 0.f;
  a.lk = p->ls.lk;
  a.fparam = (float)p->ls.fparam;
  return a;
}

static int run_side_prep(const nnef_plan_s* p, const BlockPlan& bp, const float* const* factors,
                         hipStream_t s) {
  int e = run_program(p, bp, bp.L_prog, factors, s);
  if (!e) e = run_program(p, bp, bp.R_prog, factors, s);
  return e;
}

// One sweep of Algorithm 1 over packed data; loss_slot (device, may be null)
// receives the loss at the start of the sweep, vloss_slot (device, may be
// null; needs loss_slot) the loss of the validation entries of a split pack.
static nnef_status run_sweep(nnef_plan_s* p, const float* Yd, bool masked, float* const* factors,
                             double* loss_slot, hipStream_t s, double* vloss_slot = nullptr) {
  const int L = (int)p->m.ops.size();
  const float* const* cf = factors;
  for (int l = 0; l < L; ++l) {
    const BlockPlan& bp = p->blocks[l];
    const bool want_loss = loss_slot && l == 0;
    int e = 0;
    FusedArgs fa;
    std::memset(&fa, 0, sizeof(fa));
    if (!bp.direct) {
      e = run_side_prep(p, bp, cf, s);
      if (e) return hip_fail(e, "side-operand contraction launch");
      fa = fused_args(p, bp, Yd, masked, cf);
      fa.loss_part = want_loss ? p->loss_part : nullptr;
      fa.vloss_part = want_loss && vloss_slot ? p->vloss_part : nullptr;
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (p->timing) {  // recorded by the pass launch itself, at the kernel's start and end
      if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess)
        return fail(NNEF_E_DEVICE, "timing event set-up failed");
      g_pass_events.start = ev0;
      g_pass_events.stop = ev1;
    }
    if (bp.direct) {
      DirectArgs da = direct_args(p, bp, Yd, masked, cf);
      da.loss_part = want_loss ? p->loss_part : nullptr;
      da.vloss_part = want_loss && vloss_slot ? p->vloss_part : nullptr;
      e = launch_direct(da, p->ls.wk, want_loss ? 1 : 0, s);
    } else {
      e = launch_fused(fa, bp.KP, p->ls.wk, bp.vecq, want_loss ? 1 : 0, s);
    }
    g_pass_events = PassEvents();
    if (p->timing) {
      if (e) {
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
      } else {
        p->events.emplace_back(ev0, ev1);
      }
    }
    if (e) return hip_fail(e, "fused pass launch");
    UpdateArgs ua;
    std::memset(&ua, 0, sizeof(ua));
    ua.partN = p->partN;
    ua.partD = p->partD;
    ua.n_chunks = bp.n_chunks;
    ua.nP = (int)bp.nP;
    ua.K = bp.K;
    ua.KP = bp.KP;
    ua.no_d = fa.no_d;
    ua.npieces = (int)bp.pieces.size();
    for (int i = 0; i < ua.npieces; ++i) {
      ua.piece[i] = piece_ptr(p, bp.pieces[i], cf);
      ua.ldpiece[i] = bp.pieces[i].ld;
      ua.nrows[i] = bp.pieces[i].nrows;
    }
    ua.theta = bp.L_direct ? factors[l] : nullptr;
    ua.ldT = bp.ldL;
    ua.NL = bp.L_direct ? nullptr : p->ws[bp.NL_buf];
    ua.DL = bp.L_direct ? nullptr : p->ws[bp.DL_buf];
    ua.upd = p->ls.upd;
    ua.gamma = (float)p->ls.gamma;
    ua.eps = (float)p->opt.eps;
    if (want_loss) {
      ua.loss_part = p->loss_part;
      ua.n_loss_part = bp.n_wg;
      if (vloss_slot) {
        ua.vloss_part = p->vloss_part;
        ua.vloss_out = vloss_slot;
      }
      ua.loss_out = loss_slot;
    }
    e = launch_update(ua, p->dcol, s);
    if (e) return hip_fail(e, "update launch");
    if (!bp.L_direct) {
      e = run_program_pair(p, bp, bp.chainN, bp.chainD, cf, s);
      if (e) return hip_fail(e, "chain-back contraction launch");
      ApplyArgs aa;
      aa.theta = factors[l];
      aa.N = p->ws[bp.Nl_buf];
      aa.D = p->ws[bp.Dl_buf];
      aa.n = p->numel[l];
      aa.upd = p->ls.upd;
      aa.gamma = (float)p->ls.gamma;
      aa.eps = (float)p->opt.eps;
      e = launch_apply(aa, s);
      if (e) return hip_fail(e, "update launch");
    }
  }
  return NNEF_OK;
}

// The loss of the given factors over packed data, into d_loss (device); with
// d_vloss (device) also the loss of the validation entries of a split pack.
static nnef_status run_loss(nnef_plan_s* p, const float* Yd, bool masked, const float* const* factors,
                            double* d_loss, hipStream_t s, double* d_vloss = nullptr) {
  const BlockPlan& bp = p->blocks[0];
  int e = 0;
  if (bp.direct) {
    DirectArgs da = direct_args(p, bp, Yd, masked, factors);
    da.loss_part = p->loss_part;
    da.vloss_part = d_vloss ? p->vloss_part : nullptr;
    e = launch_direct(da, p->ls.wk, 2, s);
  } else {
    e = run_side_prep(p, bp, factors, s);
    if (e) return hip_fail(e, "side-operand contraction launch");
    FusedArgs fa = fused_args(p, bp, Yd, masked, factors);
    fa.loss_part = p->loss_part;
    fa.vloss_part = d_vloss ? p->vloss_part : nullptr;
    e = launch_fused(fa, bp.KP, p->ls.wk, bp.vecq, 2, s);
  }
  if (e) return hip_fail(e, "loss pass launch");
  e = launch_loss_final(p->loss_part, bp.n_wg, d_loss, s);
  if (!e && d_vloss) e = launch_loss_final(p->vloss_part, bp.n_wg, d_vloss, s);
  if (e) return hip_fail(e, "loss reduction launch");
  return NNEF_OK;
}

static nnef_status check_step_args(nnef_plan_s* p, const float* Y, const void* factors, int n_sweeps) {
  if (!p || !Y || !factors) return fail(NNEF_E_ARG, "plan, Y and factors must not be NULL");
  if (n_sweeps < 0) return fail(NNEF_E_ARG, "n_sweeps must be >= 0");
  for (int l = 0; l < (int)p->m.ops.size(); ++l)
    if (!((float* const*)factors)[l]) return fail(NNEF_E_ARG, "factor pointer is NULL");
  return NNEF_OK;
}

nnef_status nnef_step(nnef_plan_t p, const float* Y, const uint8_t* M, float* const* factors,
                      int n_sweeps, double* loss_trace, void* stream) {
  nnef_status st = check_step_args(p, Y, factors, n_sweeps);
  if (st != NNEF_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const float* Yd = Y;
  if (M && n_sweeps > 0) {
    const int e = launch_pack(Y, M, p->ypack, p->n_data, s);
    if (e) return hip_fail(e, "data packing launch");
    Yd = p->ypack;
  }
  for (int sw = 0; sw < n_sweeps; ++sw) {
    st = run_sweep(p, Yd, M != nullptr, factors, loss_trace ? loss_trace + sw : nullptr, s);
    if (st != NNEF_OK) return st;
  }
  return NNEF_OK;
}

nnef_status nnef_plan_set_timing(nnef_plan_t p, int enable) {
  if (!p) return fail(NNEF_E_ARG, "plan must not be NULL");
  p->timing = enable != 0;
  if (!p->timing) drop_events(p);
  return NNEF_OK;
}

nnef_status nnef_plan_timing(nnef_plan_t p, int* n_passes, double* total_ms) {
  if (!p || !n_passes || !total_ms) return fail(NNEF_E_ARG, "NULL argument");
  double tot = 0.0;
  for (auto& e : p->events) {
    if (hipEventSynchronize(e.second) != hipSuccess) return fail(NNEF_E_DEVICE, "event sync failed");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e.first, e.second) != hipSuccess)
      return fail(NNEF_E_DEVICE, "event timing failed");
    tot += ms;
  }
  *n_passes = (int)p->events.size();
  *total_ms = tot;
  drop_events(p);
  return NNEF_OK;
}

nnef_status nnef_loss_device(nnef_plan_t p, const float* Y, const uint8_t* M,
                             const float* const* factors, double* d_loss, void* stream) {
  if (!p || !Y || !factors || !d_loss) return fail(NNEF_E_ARG, "NULL argument");
  for (int l = 0; l < (int)p->m.ops.size(); ++l)
    if (!factors[l]) return fail(NNEF_E_ARG, "factor pointer is NULL");
  hipStream_t s = (hipStream_t)stream;
  const float* Yd = Y;
  if (M) {
    const int e = launch_pack(Y, M, p->ypack, p->n_data, s);
    if (e) return hip_fail(e, "data packing launch");
    Yd = p->ypack;
  }
  return run_loss(p, Yd, M != nullptr, factors, d_loss, s);
}

nnef_status nnef_loss(nnef_plan_t p, const float* Y, const uint8_t* M, const float* const* factors,
                      double* loss_out, void* stream) {
  if (!loss_out) return fail(NNEF_E_ARG, "loss_out must not be NULL");
  nnef_status st = nnef_loss_device(p, Y, M, factors, p ? p->loss_tmp : nullptr, stream);
  if (st != NNEF_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(loss_out, p->loss_tmp, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "loss copy");
  return NNEF_OK;
}

// ---------------------------------------------------------------------------
// Train / validation / heldout splits and the stopping rule
nnef_status nnef_loss_split(nnef_plan_t p, const float* Y, const uint8_t* M, int value,
                            const float* const* factors, double* d_loss, void* stream) {
  if (!p || !Y || !M || !factors || !d_loss) return fail(NNEF_E_ARG, "NULL argument");
  if (value < 0 || value > 255) return fail(NNEF_E_ARG, "value must be a mask byte");
  for (int l = 0; l < (int)p->m.ops.size(); ++l)
    if (!factors[l]) return fail(NNEF_E_ARG, "factor pointer is NULL");
  hipStream_t s = (hipStream_t)stream;
  const int e = launch_pack(Y, M, p->ypack, p->n_data, s, value);
  if (e) return hip_fail(e, "data packing launch");
  return run_loss(p, p->ypack, true, factors, d_loss, s);
}

void nnef_default_fit_options(nnef_fit_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_sweeps = 5000;
  o->patience = 5;
  o->rel_tol = 1e-6;
  o->check_every = 1;
  o->train_value = 1;
  o->val_value = 2;
}

nnef_status nnef_fit(nnef_plan_t p, const float* Y, const uint8_t* M, float* const* factors,
                     const nnef_fit_options* opt_in, nnef_fit_result* res, double* train_trace,
                     double* val_trace, void* stream) {
  nnef_status st = check_step_args(p, Y, factors, 0);
  if (st != NNEF_OK) return st;
  if (!M || !res) return fail(NNEF_E_ARG, "mask and res must not be NULL");
  nnef_fit_options o;
  nnef_default_fit_options(&o);
  if (opt_in) o = *opt_in;
  if (o.max_sweeps < 0 || o.patience < 0 || o.check_every < 1 || !(o.rel_tol >= 0) ||
      o.train_value < 0 || o.train_value > 255 || o.val_value < 0 || o.val_value > 255 ||
      (o.val_value != 0 && o.val_value == o.train_value))
    return fail(NNEF_E_ARG, "invalid fit options");
  hipStream_t s = (hipStream_t)stream;
  const bool use_val = o.val_value != 0;
  const int L = (int)p->m.ops.size();
  // One pack holds both splits: training entries as data, validation entries
  // with the sign bit set.  The losses of state t (training and validation)
  // come from the first fused pass of sweep t + 1, which streams Y anyway; the
  // factors of the last state of each chunk are kept, so that a stop there
  // returns exactly that state.
  const int k = o.check_every;
  double* dl = nullptr;   // [2k] losses of the chunk's states
  float* snap = nullptr;  // the factors of the chunk's last state
  if (hipMalloc((void**)&dl, 2 * (size_t)k * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&snap, (size_t)std::max<int64_t>(1, p->numel_total) * sizeof(float)) != hipSuccess) {
    if (dl) (void)hipFree(dl);
    return fail(NNEF_E_NOMEM, "fit buffers");
  }
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(s);
    (void)hipFree(dl);
    (void)hipFree(snap);
  };
  auto copy_factors = [&](bool to_snap) -> bool {
    int64_t off = 0;
    for (int l = 0; l < L; ++l) {
      float* a = snap + off;
      const hipError_t e = to_snap ? hipMemcpyAsync(a, factors[l], p->numel[l] * sizeof(float),
                                                    hipMemcpyDeviceToDevice, s)
                                   : hipMemcpyAsync(factors[l], a, p->numel[l] * sizeof(float),
                                                    hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return false;
      off += p->numel[l];
    }
    return true;
  };
  int e = launch_pack(Y, M, p->ypack, p->n_data, s, o.train_value, use_val ? o.val_value : 256);
  if (e) {
    cleanup();
    return hip_fail(e, "data packing launch");
  }
  std::vector<double> Lh, Vh, hl(2 * (size_t)k);
  int stop = -1, reason = NNEF_STOP_MAX, returned = 0;
  for (int s0 = 0; stop < 0; s0 += k) {
    const int cnt = std::min(k, o.max_sweeps - s0 + 1);
    // sweep j of the chunk yields the losses of state s0 + j
    for (int j = 0; j < cnt; ++j) {
      if (j == cnt - 1 && !copy_factors(true)) {
        cleanup();
        return fail(NNEF_E_DEVICE, "factor snapshot failed");
      }
      st = run_sweep(p, p->ypack, true, factors, dl + j, s, use_val ? dl + k + j : nullptr);
      if (st != NNEF_OK) {
        cleanup();
        return st;
      }
    }
    if (hipMemcpyAsync(hl.data(), dl, hl.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      cleanup();
      return fail(NNEF_E_DEVICE, "loss read-back failed");
    }
    for (int j = 0; j < cnt && stop < 0; ++j) {
      const int t = s0 + j;
      Lh.push_back(hl[j]);
      Vh.push_back(use_val ? hl[k + j] : 0.0);
      // the paper's rules: validation loss rising `patience` times in a row,
      // relative decrease of the training loss below rel_tol, or the sweep cap
      bool rising = use_val && o.patience > 0 && t >= o.patience;
      for (int q = 0; rising && q < o.patience; ++q) rising = Vh[t - q] > Vh[t - q - 1];
      if (rising) {
        stop = t;
        reason = NNEF_STOP_VALIDATION;
      } else if (t >= 1 && (Lh[t - 1] - Lh[t]) < o.rel_tol * std::fabs(Lh[t - 1])) {
        stop = t;
        reason = NNEF_STOP_TRAIN_TOL;
      } else if (t >= o.max_sweeps) {
        stop = t;
        reason = NNEF_STOP_MAX;
      }
    }
    if (stop >= 0) {  // back to the chunk's last state (the stopping state when check_every = 1)
      if (!copy_factors(false)) {
        cleanup();
        return fail(NNEF_E_DEVICE, "factor restore failed");
      }
      returned = s0 + cnt - 1;
    }
  }
  if (train_trace && hipMemcpyAsync(train_trace, Lh.data(), (size_t)(stop + 1) * sizeof(double),
                                    hipMemcpyHostToDevice, s) != hipSuccess)
    st = fail(NNEF_E_DEVICE, "trace copy failed");
  if (val_trace && use_val &&
      hipMemcpyAsync(val_trace, Vh.data(), (size_t)(stop + 1) * sizeof(double), hipMemcpyHostToDevice, s) !=
          hipSuccess)
    st = fail(NNEF_E_DEVICE, "trace copy failed");
  cleanup();
  res->stop_sweep = stop;
  res->sweeps_run = returned;
  res->reason = reason;
  res->train_loss = Lh[stop];
  res->val_loss = use_val ? Vh[stop] : 0.0;
  return st;
}

// ---------------------------------------------------------------------------
// Learned extrapolation
struct nnef_mlp_s {
  float* params = nullptr;   // FP32 master parameters
  float* m = nullptr;        // Adam moments
  float* v = nullptr;
  float* gpart = nullptr;    // [256, kMlpParams] gradient partials
  double* lpart = nullptr;   // [256]
  int64_t t = 0;             // Adam steps taken
};

static void free_mlp(nnef_mlp_s* q) {
  if (!q) return;
  for (void* b : {(void*)q->params, (void*)q->m, (void*)q->v, (void*)q->gpart, (void*)q->lpart})
    if (b) (void)hipFree(b);
  delete q;
}

int nnef_mlp_num_params(void) { return kMlpParams; }

nnef_status nnef_mlp_create(const float* d_init, nnef_mlp_t* out) {
  if (!d_init || !out) return fail(NNEF_E_ARG, "d_init and out must not be NULL");
  *out = nullptr;
  nnef_mlp_s* q = new nnef_mlp_s();
  const size_t pb = kMlpParams * sizeof(float);
  if (hipMalloc((void**)&q->params, pb) != hipSuccess || hipMalloc((void**)&q->m, pb) != hipSuccess ||
      hipMalloc((void**)&q->v, pb) != hipSuccess ||
      hipMalloc((void**)&q->gpart, 256 * pb) != hipSuccess ||
      hipMalloc((void**)&q->lpart, 256 * sizeof(double)) != hipSuccess) {
    free_mlp(q);
    return fail(NNEF_E_NOMEM, "MLP allocation failed");
  }
  if (hipMemcpy(q->params, d_init, pb, hipMemcpyDeviceToDevice) != hipSuccess ||
      hipMemset(q->m, 0, pb) != hipSuccess || hipMemset(q->v, 0, pb) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    free_mlp(q);
    return fail(NNEF_E_DEVICE, "MLP initialisation failed");
  }
  *out = q;
  return NNEF_OK;
}

void nnef_mlp_destroy(nnef_mlp_t q) { free_mlp(q); }

nnef_status nnef_mlp_params(nnef_mlp_t q, float* d_out, void* stream) {
  if (!q || !d_out) return fail(NNEF_E_ARG, "NULL argument");
  const hipError_t e = hipMemcpyAsync(d_out, q->params, kMlpParams * sizeof(float),
                                      hipMemcpyDeviceToDevice, (hipStream_t)stream);
  return e == hipSuccess ? NNEF_OK : hip_fail(e, "parameter copy");
}

nnef_status nnef_mlp_forward(nnef_mlp_t q, const float* X, int64_t n_rows, float* s_out, void* stream) {
  if (!q || (n_rows > 0 && (!X || !s_out)) || n_rows < 0) return fail(NNEF_E_ARG, "bad argument");
  if (n_rows == 0) return NNEF_OK;
  MlpArgs a;
  std::memset(&a, 0, sizeof(a));
  a.params = q->params;
  a.n_rows = n_rows;
  a.X = X;
  a.s_out = s_out;
  const int e = launch_mlp(a, 0, mlp_grid(n_rows), stream);
  return e ? hip_fail(e, "MLP forward launch") : NNEF_OK;
}

static nnef_status mlp_grad(nnef_mlp_s* q, const float* X, const float* tau, const int32_t* idx,
                            int64_t n_rows, float* grad_out, double* loss_out, double lr, int adam,
                            void* stream) {
  if (!q || !X || !tau || n_rows <= 0) return fail(NNEF_E_ARG, "bad argument");
  if (n_rows >= (int64_t(1) << 31)) return fail(NNEF_E_SHAPE, "too many rows");
  MlpArgs a;
  std::memset(&a, 0, sizeof(a));
  a.params = q->params;
  a.n_rows = n_rows;
  a.X = X;
  a.tau = tau;
  a.idx = idx;
  a.inv_n = (float)(1.0 / (double)n_rows);
  a.gpart = q->gpart;
  a.lpart = q->lpart;
  const int grid = mlp_grid(n_rows);
  int e = launch_mlp(a, 1, grid, stream);
  if (e) return hip_fail(e, "MLP gradient launch");
  const float b1 = 0.9f, b2 = 0.999f;
  float bc1 = 1.f, bc2 = 1.f;
  if (adam) {
    q->t += 1;
    bc1 = (float)(1.0 - std::pow(0.9, (double)q->t));
    bc2 = (float)(1.0 - std::pow(0.999, (double)q->t));
  }
  e = launch_mlp_reduce(q->gpart, q->lpart, grid, a.inv_n, grad_out, loss_out, q->params, q->m, q->v,
                        (float)lr, b1, b2, 1e-8f, bc1, bc2, adam, stream);
  return e ? hip_fail(e, "MLP reduction launch") : NNEF_OK;
}

nnef_status nnef_mlp_gradient(nnef_mlp_t q, const float* X, const float* tau, const int32_t* idx,
                              int64_t n_rows, float* d_grad, double* d_loss, void* stream) {
  if (!d_grad) return fail(NNEF_E_ARG, "d_grad must not be NULL");
  return mlp_grad(q, X, tau, idx, n_rows, d_grad, d_loss, 0.0, 0, stream);
}

nnef_status nnef_mlp_train_step(nnef_mlp_t q, const float* X, const float* tau, const int32_t* idx,
                                int64_t n_rows, double lr, double* d_loss, void* stream) {
  if (!(lr > 0.0) || !std::isfinite(lr)) return fail(NNEF_E_ARG, "lr must be positive and finite");
  return mlp_grad(q, X, tau, idx, n_rows, nullptr, d_loss, lr, 1, stream);
}

// Feature arguments for the plan's factors.
static nnef_status feat_args(nnef_plan_s* p, const float* const* th, const float* const* tm1,
                             const float* const* tm2, FeatArgs& f) {
  const int L = (int)p->m.ops.size();
  if (!p->learn_buf) return fail(NNEF_E_UNSUPPORTED, "learned extrapolation supports at most 8 factors");
  std::memset(&f, 0, sizeof(f));
  f.n_fac = L;
  f.off[0] = 0;
  for (int k = 0; k < L; ++k) {
    f.off[k + 1] = f.off[k] + p->numel[k];
    f.th[k] = th[k];
    f.tm1[k] = tm1[k];
    f.tm2[k] = tm2[k];
    const std::string& sub = p->m.ops[k];
    const int64_t K = sub.empty() ? 1 : p->m.size[(unsigned char)sub.back()];
    f.logK8[k] = (float)(std::log2((double)K) / 8.0);
  }
  f.sigma = p->learn_small;
  f.gamma = (float)(p->ls.upd == UP_EXP ? 1.0 : p->ls.gamma);
  f.eps = (float)p->opt.eps;
  f.log_eps = (float)std::log(p->opt.eps);
  f.inv_abs_log_eps = (float)(1.0 / std::fabs(std::log(p->opt.eps)));
  return NNEF_OK;
}

nnef_status nnef_learned_rows(nnef_plan_t p, const float* const* th_t, const float* const* th_tm1,
                              const float* const* th_tm2, const float* const* th_target, double rel_dec,
                              float* X, float* tau, void* stream) {
  if (!p || !th_t || !th_tm1 || !th_tm2 || !X) return fail(NNEF_E_ARG, "NULL argument");
  if ((th_target == nullptr) != (tau == nullptr))
    return fail(NNEF_E_ARG, "th_target and tau must both be given or both be NULL");
  FeatArgs f;
  nnef_status st = feat_args(p, th_t, th_tm1, th_tm2, f);
  if (st != NNEF_OK) return st;
  f.rel_dec = rel_dec;
  for (int k = 0; k < f.n_fac; ++k) {
    if (!th_t[k] || !th_tm1[k] || !th_tm2[k] || (th_target && !th_target[k]))
      return fail(NNEF_E_ARG, "factor pointer is NULL");
    f.tth[k] = th_target ? th_target[k] : nullptr;
  }
  int e = launch_sigma(f, stream);
  if (!e) e = launch_rows(f, X, tau, stream);
  return e ? hip_fail(e, "feature launch") : NNEF_OK;
}

nnef_status nnef_step_learned(nnef_plan_t p, nnef_mlp_t q, const float* Y, const uint8_t* M,
                              float* const* factors, int n_sweeps, int propose_every,
                              double* loss_trace, int* d_n_accepted, void* stream) {
  nnef_status st = check_step_args(p, Y, factors, n_sweeps);
  if (st != NNEF_OK) return st;
  if (!q) return fail(NNEF_E_ARG, "mlp must not be NULL");
  if (propose_every < 3) return fail(NNEF_E_ARG, "propose_every must be >= 3");
  if (!p->learn_buf) return fail(NNEF_E_UNSUPPORTED, "learned extrapolation supports at most 8 factors");
  hipStream_t s = (hipStream_t)stream;
  const int L = (int)p->m.ops.size();
  const float* Yd = Y;
  if (M && n_sweeps > 0) {
    const int e = launch_pack(Y, M, p->ypack, p->n_data, s);
    if (e) return hip_fail(e, "data packing launch");
    Yd = p->ypack;
  }
  // plan-owned buffers: theta_{t-1}, theta_{t-2}, the proposal
  float* h1[kMaxLearnFactors];
  float* h2[kMaxLearnFactors];
  float* cand[kMaxLearnFactors];
  int64_t o = 0;
  for (int k = 0; k < L; ++k) {
    h1[k] = p->learn_buf + o;
    h2[k] = p->learn_buf + p->numel_total + o;
    cand[k] = p->learn_buf + 2 * p->numel_total + o;
    o += p->numel[k];
  }
  double* loss_prev_slot = p->learn_small + kMaxLearnFactors;  // used when no trace is given
  double* loss_cur = p->learn_small + kMaxLearnFactors + 1;
  double* loss_cand = p->learn_small + kMaxLearnFactors + 2;
  const int P = propose_every;
  for (int sw = 1; sw <= n_sweeps; ++sw) {
    // snapshots: theta_{t-2} before sweep t-1, theta_{t-1} before sweep t (t = proposal sweep)
    if (sw % P == P - 1 || sw % P == 0) {
      FeatArgs c;
      st = feat_args(p, factors, sw % P == 0 ? h1 : h2, factors, c);
      if (st != NNEF_OK) return st;
      const int e = launch_copy_factors(c, s);
      if (e) return hip_fail(e, "snapshot launch");
    }
    double* slot = loss_trace ? loss_trace + (sw - 1) : loss_prev_slot;
    st = run_sweep(p, Yd, M != nullptr, factors, slot, s);
    if (st != NNEF_OK) return st;
    if (sw % P != 0) continue;
    // proposal after sweep t = sw from theta_t (factors), theta_{t-1} (h1), theta_{t-2} (h2)
    st = run_loss(p, Yd, M != nullptr, factors, loss_cur, s);
    if (st != NNEF_OK) return st;
    FeatArgs f;
    st = feat_args(p, factors, h1, h2, f);
    if (st != NNEF_OK) return st;
    f.loss_prev = slot;
    f.loss_cur = loss_cur;
    for (int k = 0; k < L; ++k) {
      f.cand[k] = cand[k];
      f.dst[k] = factors[k];
    }
    int e = launch_sigma(f, s);
    if (e) return hip_fail(e, "feature launch");
    MlpArgs a;
    std::memset(&a, 0, sizeof(a));
    a.params = q->params;
    a.n_rows = p->numel_total;
    a.f = f;
    e = launch_mlp(a, 2, mlp_grid(a.n_rows), s);
    if (e) return hip_fail(e, "proposal launch");
    st = run_loss(p, Yd, M != nullptr, cand, loss_cand, s);
    if (st != NNEF_OK) return st;
    e = launch_accept(f, loss_cand, loss_cur, d_n_accepted, s);
    if (e) return hip_fail(e, "accept launch");
  }
  return NNEF_OK;
}

// ---------------------------------------------------------------------------
// Batched plans: many problems and restarts in persistent launches
struct BatchClass {
  int KP = 0, wk = 0, prec = 0;
  bool vecq = false, full = false;
  int off = 0, n = 0, grid = 0;      // slice of the block's work array
};

struct BatchBlock {
  std::vector<BatchClass> cls[2];     // by mode: 0 = N/D, 1 = N/D + loss (block 0)
  FusedArgs* d_fargs[2] = {nullptr, nullptr};  // [n_runs]
  WorkItem* d_work[2] = {nullptr, nullptr};
  UpdateArgs* d_uargs[2] = {nullptr, nullptr};  // [n_runs]
  int* d_colsum = nullptr;
  int n_colsum = 0;
  WorkItem* d_uwork = nullptr;
  int n_uwork = 0;
  // side operands before the pass and chain-backs after the update, for every
  // run that needs them (each run has its own workspace)
  std::vector<EinsumArgs> side;
  struct Chain {
    EinsumArgs n, d;
    bool pair;
  };
  std::vector<Chain> chain;
  std::vector<ApplyArgs> apply;
};

struct nnef_batch_s {
  std::vector<nnef_plan_s*> sub;      // one plan per problem: lowering and index tables
  std::vector<int> restarts, masked;  // per problem
  std::vector<int> run_prob, run_fac; // per run: problem, offset of its factor pointers
  int n_runs = 0, n_fac_ptrs = 0, L_max = 0;
  std::vector<float*> partN, partD, dcol;
  std::vector<double*> lpart;
  std::vector<float*> run_ws;         // per run: a copy of its problem's workspace (or null)
  double* loss_slots = nullptr;       // [n_runs]
  std::vector<BatchBlock> blocks;
  int target[3] = {128, 128, 128};    // workgroups per run and pass, by width class 16/32/64
  int grid[3] = {0, 0, 0};            // persistent grid per width class (0: one per item)
  std::vector<const void*> bound;     // pointers the device tables were built for
  hipStream_t cap = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  std::string tuning;
};

static int kp_class(int KP) { return KP == 16 ? 0 : KP == 32 ? 1 : 2; }

static void drop_graphs(nnef_batch_s* b) {
  for (int i = 0; i < 2; ++i) {
    if (b->exec[i]) (void)hipGraphExecDestroy(b->exec[i]);
    if (b->graph[i]) (void)hipGraphDestroy(b->graph[i]);
    b->exec[i] = nullptr;
    b->graph[i] = nullptr;
  }
}

static void free_block_tables(BatchBlock& k) {
  for (int m = 0; m < 2; ++m) {
    for (void* q : {(void*)k.d_fargs[m], (void*)k.d_work[m], (void*)k.d_uargs[m]})
      if (q) (void)hipFree(q);
    k.d_fargs[m] = nullptr;
    k.d_work[m] = nullptr;
    k.d_uargs[m] = nullptr;
    k.cls[m].clear();
  }
  for (void* q : {(void*)k.d_colsum, (void*)k.d_uwork})
    if (q) (void)hipFree(q);
  k.d_colsum = nullptr;
  k.d_uwork = nullptr;
  k.side.clear();
  k.chain.clear();
  k.apply.clear();
}

static void free_batch(nnef_batch_s* b) {
  if (!b) return;
  drop_graphs(b);
  for (auto& k : b->blocks) free_block_tables(k);
  for (auto v : {&b->partN, &b->partD, &b->dcol})
    for (float* q : *v)
      if (q) (void)hipFree(q);
  for (double* q : b->lpart)
    if (q) (void)hipFree(q);
  for (float* q : b->run_ws)
    if (q) (void)hipFree(q);
  if (b->loss_slots) (void)hipFree(b->loss_slots);
  for (auto* q : b->sub) free_plan(q);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

void nnef_batch_destroy(nnef_batch_t b) { free_batch(b); }

int nnef_batch_num_runs(nnef_batch_t b) { return b ? b->n_runs : 0; }

// Geometry of every block of every problem for the current per-class targets.
static bool batch_geometry(nnef_batch_s* b) {
  for (auto* q : b->sub)
    for (auto& bp : q->blocks)
      if (!choose_geometry(q->m, bp, b->target[kp_class(bp.KP)])) return false;
  return true;
}

}  // extern "C"

template <class T>
static nnef_status upload(T** d, const std::vector<T>& h) {
  if (*d) (void)hipFree(*d);
  *d = nullptr;
  if (h.empty()) return NNEF_OK;
  if (hipMalloc((void**)d, h.size() * sizeof(T)) != hipSuccess) return fail(NNEF_E_NOMEM, "table allocation failed");
  if (hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return fail(NNEF_E_DEVICE, "table upload failed");
  return NNEF_OK;
}

extern "C" {

// Points a problem's workspace table at one run's copy while that run's
// arguments are built (the lowering refers to buffers by index).
struct WsBinding {
  nnef_plan_s* q;
  std::vector<float*> saved;
  WsBinding(nnef_plan_s* q_, float* base) : q(q_), saved(q_->ws) {
    if (base)
      for (auto& w : q->ws) w = base + (w - (float*)q->ws_base);
  }
  ~WsBinding() { q->ws = saved; }
};

// Device argument and work tables for the given data and factor pointers.
static nnef_status batch_tables(nnef_batch_s* b, const float* const* Y, const uint8_t* const* M,
                                float* const* factors) {
  drop_graphs(b);
  const int R = b->n_runs;
  for (int l = 0; l < b->L_max; ++l) {
    BatchBlock& k = b->blocks[l];
    free_block_tables(k);
    std::vector<UpdateArgs> ua[2];
    ua[0].resize(R);
    ua[1].resize(R);
    std::vector<int> colsum;
    std::vector<WorkItem> uwork;
    for (int mode = 0; mode < (l == 0 ? 2 : 1); ++mode) {
      std::vector<FusedArgs> fa(R);
      std::memset(fa.data(), 0, R * sizeof(FusedArgs));
      // class key -> items, ordered problem, workgroup, restart: the restarts of a
      // problem read the same Y tile at about the same time (shared in the caches)
      std::vector<BatchClass> cls;
      std::vector<std::vector<WorkItem>> items;
      int run0 = 0;
      for (size_t pi = 0; pi < b->sub.size(); ++pi) {
        nnef_plan_s* q = b->sub[pi];
        const int nr = b->restarts[pi];
        if (l < (int)q->blocks.size()) {
          const BlockPlan& bp = q->blocks[l];
          const bool msk = M && M[pi];
          const float* Yd = msk ? q->ypack : Y[pi];
          int ci = -1;
          for (int r = 0; r < nr; ++r) {
            const int run = run0 + r;
            float* const* fr = factors + b->run_fac[run];
            WsBinding bind(q, b->run_ws[run]);
            FusedArgs a = fused_args(q, bp, Yd, msk, fr);
            // batched passes: widths 16 and 64 contract in FP32, the reconstruction stays FP32
            a.prec = bp.KP != 32 ? 0 : a.prec > 2 ? a.prec - 2 : a.prec;
            a.partN = b->partN[run];
            a.partD = b->partD[run];
            a.loss_part = mode ? b->lpart[run] : nullptr;
            a.xcd_remap = 0;
            fa[run] = a;
            if (r == 0) {
              BatchClass c;
              c.KP = bp.KP;
              c.wk = q->ls.wk;
              c.prec = a.prec;
              c.vecq = bp.vecq;
              c.full = a.full != 0;
              for (size_t j = 0; j < cls.size(); ++j)
                if (cls[j].KP == c.KP && cls[j].wk == c.wk && cls[j].prec == c.prec &&
                    cls[j].vecq == c.vecq && cls[j].full == c.full)
                  ci = (int)j;
              if (ci < 0) {
                ci = (int)cls.size();
                cls.push_back(c);
                items.emplace_back();
              }
            }
            if (mode == 0) {
              UpdateArgs u;
              std::memset(&u, 0, sizeof(u));
              u.partN = b->partN[run];
              u.partD = b->partD[run];
              u.n_chunks = bp.n_chunks;
              u.nP = (int)bp.nP;
              u.K = bp.K;
              u.KP = bp.KP;
              u.no_d = a.no_d;
              u.npieces = (int)bp.pieces.size();
              for (int i = 0; i < u.npieces; ++i) {
                u.piece[i] = piece_ptr(q, bp.pieces[i], fr);
                u.ldpiece[i] = bp.pieces[i].ld;
                u.nrows[i] = bp.pieces[i].nrows;
              }
              u.theta = bp.L_direct ? fr[l] : nullptr;
              u.ldT = bp.ldL;
              u.NL = bp.L_direct ? nullptr : q->ws[bp.NL_buf];
              u.DL = bp.L_direct ? nullptr : q->ws[bp.DL_buf];
              u.upd = q->ls.upd;
              u.gamma = (float)q->ls.gamma;
              u.eps = (float)q->opt.eps;
              u.dcol = b->dcol[run];
              ua[0][run] = u;
              u.loss_part = b->lpart[run];
              u.n_loss_part = bp.n_wg;
              u.loss_out = b->loss_slots + run;
              ua[1][run] = u;
              if (a.no_d) colsum.push_back(run);
              const int nb = (int)((bp.nP * bp.K + 63) / 64);
              for (int j = 0; j < nb; ++j) uwork.push_back(WorkItem{run, j});
              for (const Step& stp : bp.L_prog) k.side.push_back(einsum_args(q, bp, stp, fr));
              for (const Step& stp : bp.R_prog) k.side.push_back(einsum_args(q, bp, stp, fr));
              if (!bp.L_direct) {
                std::vector<EinsumArgs> cn, cd;
                for (const Step& stp : bp.chainN) cn.push_back(einsum_args(q, bp, stp, fr));
                for (const Step& stp : bp.chainD) cd.push_back(einsum_args(q, bp, stp, fr));
                bool pair = cn.size() == cd.size();
                for (size_t i = 0; pair && i < cn.size(); ++i) pair = same_shape(cn[i], cd[i]);
                if (pair) {
                  for (size_t i = 0; i < cn.size(); ++i) k.chain.push_back(BatchBlock::Chain{cn[i], cd[i], true});
                } else {  // the two chains one after the other
                  for (const EinsumArgs& e : cn) k.chain.push_back(BatchBlock::Chain{e, e, false});
                  for (const EinsumArgs& e : cd) k.chain.push_back(BatchBlock::Chain{e, e, false});
                }
                ApplyArgs aa;
                aa.theta = fr[l];
                aa.N = q->ws[bp.Nl_buf];
                aa.D = q->ws[bp.Dl_buf];
                aa.n = q->numel[l];
                aa.upd = q->ls.upd;
                aa.gamma = (float)q->ls.gamma;
                aa.eps = (float)q->opt.eps;
                k.apply.push_back(aa);
              }
            }
          }
          for (int w = 0; w < bp.n_wg; ++w)
            for (int r = 0; r < nr; ++r) items[ci].push_back(WorkItem{run0 + r, w});
        }
        run0 += nr;
      }
      std::vector<WorkItem> all;
      for (size_t j = 0; j < cls.size(); ++j) {
        cls[j].off = (int)all.size();
        cls[j].n = (int)items[j].size();
        const int g = b->grid[kp_class(cls[j].KP)];
        cls[j].grid = g > 0 ? std::min(g, cls[j].n) : cls[j].n;
        all.insert(all.end(), items[j].begin(), items[j].end());
      }
      k.cls[mode] = cls;
      nnef_status st = upload(&k.d_fargs[mode], fa);
      if (st == NNEF_OK) st = upload(&k.d_work[mode], all);
      if (st != NNEF_OK) return st;
    }
    nnef_status st = upload(&k.d_uargs[0], ua[0]);
    if (st == NNEF_OK && l == 0) st = upload(&k.d_uargs[1], ua[1]);
    if (st == NNEF_OK) st = upload(&k.d_colsum, colsum);
    if (st == NNEF_OK) st = upload(&k.d_uwork, uwork);
    if (st != NNEF_OK) return st;
    k.n_colsum = (int)colsum.size();
    k.n_uwork = (int)uwork.size();
  }
  b->bound.clear();
  for (size_t pi = 0; pi < b->sub.size(); ++pi) {
    b->bound.push_back(Y[pi]);
    b->bound.push_back(M ? (const void*)M[pi] : nullptr);
  }
  for (int i = 0; i < b->n_fac_ptrs; ++i) b->bound.push_back(factors[i]);
  return NNEF_OK;
}

// One sweep over every run (the launch sequence that is captured in a graph).
static nnef_status batch_sweep(nnef_batch_s* b, bool with_loss, hipStream_t s) {
  for (int l = 0; l < b->L_max; ++l) {
    BatchBlock& k = b->blocks[l];
    const int mode = (with_loss && l == 0) ? 1 : 0;
    for (const EinsumArgs& e : k.side) {
      const int ec = launch_einsum(e, s);
      if (ec) return hip_fail(ec, "side-operand contraction launch");
    }
    for (const BatchClass& c : k.cls[mode]) {
      BatchedLaunch L;
      L.args = k.d_fargs[mode];
      L.work = k.d_work[mode] + c.off;
      L.n_work = c.n;
      L.grid = c.grid;
      L.KP = c.KP;
      L.wk = c.wk;
      L.mode = mode;
      L.prec = c.prec;
      L.vecq = c.vecq;
      L.full = c.full;
      const int e = launch_fused_batched(L, s);
      if (e) return hip_fail(e, "batched fused pass launch");
    }
    const int ugrid = std::min(k.n_uwork, 4096);
    const int e = launch_update_batched(k.d_uargs[mode], k.d_colsum, k.n_colsum, k.d_uwork, k.n_uwork,
                                        ugrid, s);
    if (e) return hip_fail(e, "batched update launch");
    for (const BatchBlock::Chain& c : k.chain) {
      const int ec = c.pair ? launch_einsum(c.n, s, &c.d) : launch_einsum(c.n, s);
      if (ec) return hip_fail(ec, "chain-back contraction launch");
    }
    for (const ApplyArgs& a : k.apply) {
      const int ec = launch_apply(a, s);
      if (ec) return hip_fail(ec, "update launch");
    }
  }
  return NNEF_OK;
}

nnef_status nnef_batch_plan(const nnef_problem* probs, int n_problems, const nnef_options* opt,
                            nnef_batch_t* out) {
  if (!probs || n_problems <= 0 || !out) return fail(NNEF_E_ARG, "problems, n_problems and out must be valid");
  *out = nullptr;
  auto* b = new nnef_batch_s();
  for (int pi = 0; pi < n_problems; ++pi) {
    const nnef_problem& d = probs[pi];
    if (d.n_restarts < 1) {
      free_batch(b);
      return fail(NNEF_E_ARG, "n_restarts must be >= 1");
    }
    nnef_plan_t q = nullptr;
    // CP-like strings keep the lowering without side operands; others (Tucker,
    // tensor train, custom strings) take side operands and chain-backs
    nnef_status st = plan_create(d.model_str, d.mode_sizes, d.n_modes, d.ranks, d.n_ranks, d.alpha,
                                 d.beta, opt, d.masked != 0, 128, &q, 1);
    if (st == NNEF_E_UNSUPPORTED)
      st = plan_create(d.model_str, d.mode_sizes, d.n_modes, d.ranks, d.n_ranks, d.alpha, d.beta, opt,
                       d.masked != 0, 128, &q, 2);
    if (st != NNEF_OK) {
      free_batch(b);
      return fail(st, "problem " + std::to_string(pi) + ": " + g_last_error);
    }
    b->sub.push_back(q);
    b->restarts.push_back(d.n_restarts);
    b->masked.push_back(d.masked != 0);
    const int L = (int)q->m.ops.size();
    b->L_max = std::max(b->L_max, L);
    for (int r = 0; r < d.n_restarts; ++r) {
      b->run_prob.push_back(pi);
      b->run_fac.push_back(b->n_fac_ptrs);
      b->n_fac_ptrs += L;
      ++b->n_runs;
    }
  }
  // partial buffers per run, sized for the largest tiling the autotuner tries
  const int cand[3] = {32, 128, 512};
  size_t run0 = 0;
  for (size_t pi = 0; pi < b->sub.size(); ++pi) {
    nnef_plan_s* q = b->sub[pi];
    size_t part = 1;
    int wg = 1;
    for (int t : cand)
      for (BlockPlan bp : q->blocks) {
        if (!choose_geometry(q->m, bp, t)) {
          free_batch(b);
          return fail(NNEF_E_SHAPE, "grid too large");
        }
        part = std::max(part, (size_t)bp.n_chunks * bp.nP * bp.KP);
        wg = std::max(wg, bp.n_wg);
      }
    if (part >= (size_t(1) << 30)) {
      free_batch(b);
      return fail(NNEF_E_SHAPE, "partial sums need 2^30 or more elements");
    }
    size_t ws_total = 0;  // the problem's workspace, copied per run (with its initial contents)
    for (auto v : q->ws_sizes) ws_total += (size_t)((v + 63) / 64 * 64);
    for (int r = 0; r < b->restarts[pi]; ++r) {
      float *pn = nullptr, *pd = nullptr, *dc = nullptr, *ws = nullptr;
      double* lp = nullptr;
      const bool ok = hipMalloc((void**)&pn, part * sizeof(float)) == hipSuccess &&
                      hipMalloc((void**)&pd, part * sizeof(float)) == hipSuccess &&
                      hipMalloc((void**)&dc, 64 * sizeof(float)) == hipSuccess &&
                      hipMalloc((void**)&lp, wg * sizeof(double)) == hipSuccess &&
                      (ws_total == 0 ||
                       (hipMalloc((void**)&ws, ws_total * sizeof(float)) == hipSuccess &&
                        hipMemcpy(ws, q->ws_base, ws_total * sizeof(float), hipMemcpyDeviceToDevice) == hipSuccess));
      b->partN.push_back(pn);
      b->partD.push_back(pd);
      b->dcol.push_back(dc);
      b->lpart.push_back(lp);
      b->run_ws.push_back(ws);
      if (!ok) {
        free_batch(b);
        return fail(NNEF_E_NOMEM, "per-run buffer allocation failed");
      }
    }
    run0 += b->restarts[pi];
  }
  if (hipMalloc((void**)&b->loss_slots, b->n_runs * sizeof(double)) != hipSuccess ||
      hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    free_batch(b);
    return fail(NNEF_E_DEVICE, "batch set-up failed");
  }
  b->blocks.resize(b->L_max);
  if (!batch_geometry(b)) {
    free_batch(b);
    return fail(NNEF_E_SHAPE, "grid too large");
  }
  *out = b;
  return NNEF_OK;
}

static bool same_binding(const nnef_batch_s* b, const float* const* Y, const uint8_t* const* M,
                         float* const* factors) {
  if (b->bound.size() != 2 * b->sub.size() + (size_t)b->n_fac_ptrs) return false;
  size_t i = 0;
  for (size_t pi = 0; pi < b->sub.size(); ++pi) {
    if (b->bound[i++] != Y[pi]) return false;
    if (b->bound[i++] != (M ? (const void*)M[pi] : nullptr)) return false;
  }
  for (int f = 0; f < b->n_fac_ptrs; ++f)
    if (b->bound[i++] != factors[f]) return false;
  return true;
}

static nnef_status batch_check(nnef_batch_s* b, const float* const* Y, const uint8_t* const* M,
                               float* const* factors) {
  if (!b || !Y || !factors) return fail(NNEF_E_ARG, "batch, Y and factors must not be NULL");
  for (size_t pi = 0; pi < b->sub.size(); ++pi) {
    if (!Y[pi]) return fail(NNEF_E_ARG, "Y pointer is NULL");
    if (M && M[pi] && !b->masked[pi])
      return fail(NNEF_E_ARG, "problem " + std::to_string(pi) + " was planned without a mask");
  }
  for (int f = 0; f < b->n_fac_ptrs; ++f)
    if (!factors[f]) return fail(NNEF_E_ARG, "factor pointer is NULL");
  return NNEF_OK;
}

static nnef_status batch_pack(nnef_batch_s* b, const float* const* Y, const uint8_t* const* M,
                              hipStream_t s) {
  if (!M) return NNEF_OK;
  for (size_t pi = 0; pi < b->sub.size(); ++pi)
    if (M[pi]) {
      const int e = launch_pack(Y[pi], M[pi], b->sub[pi]->ypack, b->sub[pi]->n_data, s);
      if (e) return hip_fail(e, "data packing launch");
    }
  return NNEF_OK;
}

nnef_status nnef_batch_step(nnef_batch_t b, const float* const* Y, const uint8_t* const* M,
                            float* const* factors, int n_sweeps, double* loss_trace, void* stream) {
  nnef_status st = batch_check(b, Y, M, factors);
  if (st != NNEF_OK) return st;
  if (n_sweeps < 0) return fail(NNEF_E_ARG, "n_sweeps must be >= 0");
  if (n_sweeps == 0) return NNEF_OK;
  hipStream_t s = (hipStream_t)stream;
  if (!same_binding(b, Y, M, factors)) {
    st = batch_tables(b, Y, M, factors);
    if (st != NNEF_OK) return st;
  }
  st = batch_pack(b, Y, M, s);
  if (st != NNEF_OK) return st;
  const int gi = loss_trace ? 1 : 0;
  if (!b->exec[gi]) {
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return fail(NNEF_E_DEVICE, "graph capture could not start");
    st = batch_sweep(b, gi == 1, b->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (st != NNEF_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess || !g) return hip_fail(e, "graph capture");
    b->graph[gi] = g;
    if (hipGraphInstantiate(&b->exec[gi], g, nullptr, nullptr, 0) != hipSuccess) {
      b->exec[gi] = nullptr;
      return fail(NNEF_E_DEVICE, "graph instantiation failed");
    }
  }
  for (int sw = 0; sw < n_sweeps; ++sw) {
    const hipError_t e = hipGraphLaunch(b->exec[gi], s);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    if (loss_trace) {
      const int ec = launch_copy_f64(loss_trace + (size_t)sw * b->n_runs, b->loss_slots, b->n_runs, s);
      if (ec) return hip_fail(ec, "loss copy launch");
    }
  }
  return NNEF_OK;
}

nnef_status nnef_batch_autotune(nnef_batch_t b, const float* const* Y, const uint8_t* const* M,
                                float* const* factors, void* stream) {
  nnef_status st = batch_check(b, Y, M, factors);
  if (st != NNEF_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  st = batch_pack(b, Y, M, s);
  if (st != NNEF_OK) return st;
  struct Cand {
    int target, grid;
  };
  const Cand cands[] = {{32, 0}, {128, 0}, {512, 0}, {32, 1024}, {128, 1024}, {512, 1024},
                        {128, 2048}, {512, 2048}};
  double best[3] = {1e300, 1e300, 1e300};
  Cand pick[3] = {{128, 0}, {128, 0}, {128, 0}};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(NNEF_E_DEVICE, "event creation failed");
  for (const Cand& c : cands) {
    for (int i = 0; i < 3; ++i) {
      b->target[i] = c.target;
      b->grid[i] = c.grid;
    }
    if (!batch_geometry(b)) continue;
    st = batch_tables(b, Y, M, factors);
    if (st != NNEF_OK) break;
    double t[3] = {0, 0, 0};
    for (int rep = 0; rep < 2; ++rep) {
      double tr[3] = {0, 0, 0};
      for (int l = 0; l < b->L_max; ++l)
        for (const BatchClass& k : b->blocks[l].cls[0]) {
          BatchedLaunch L;
          L.args = b->blocks[l].d_fargs[0];
          L.work = b->blocks[l].d_work[0] + k.off;
          L.n_work = k.n;
          L.grid = k.grid;
          L.KP = k.KP;
          L.wk = k.wk;
          L.mode = 0;
          L.prec = k.prec;
          L.vecq = k.vecq;
          L.full = k.full;
          float ms = 0.f;
          if (hipEventRecord(e0, s) != hipSuccess || launch_fused_batched(L, s) ||
              hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return fail(NNEF_E_DEVICE, "autotune timing failed");
          }
          tr[kp_class(k.KP)] += ms;
        }
      for (int i = 0; i < 3; ++i) t[i] = rep == 0 ? tr[i] : std::min(t[i], tr[i]);
    }
    for (int i = 0; i < 3; ++i)
      if (t[i] < best[i]) {
        best[i] = t[i];
        pick[i] = c;
      }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != NNEF_OK) return st;
  b->tuning.clear();
  const char* names[3] = {"16", "32", "64"};
  for (int i = 0; i < 3; ++i) {
    b->target[i] = pick[i].target;
    b->grid[i] = pick[i].grid;
    if (best[i] > 0 && best[i] < 1e300)
      b->tuning += std::string("width ") + names[i] + ": " + std::to_string(pick[i].target) +
                   " workgroups per run, grid " +
                   (pick[i].grid ? std::to_string(pick[i].grid) : std::string("all items")) + ", " +
                   std::to_string(best[i]) + " ms per sweep of fused passes\n";
  }
  if (!batch_geometry(b)) return fail(NNEF_E_SHAPE, "grid too large");
  st = batch_tables(b, Y, M, factors);
  if (st != NNEF_OK) return st;
  return hipStreamSynchronize(s) == hipSuccess ? NNEF_OK : fail(NNEF_E_DEVICE, "sync failed");
}

size_t nnef_batch_describe(nnef_batch_t b, char* buf, size_t n) {
  if (!b) return 0;
  std::string d = std::to_string(b->sub.size()) + " problems, " + std::to_string(b->n_runs) + " runs\n";
  for (size_t pi = 0; pi < b->sub.size(); ++pi)
    d += "problem " + std::to_string(pi) + " x" + std::to_string(b->restarts[pi]) + ":\n" +
         b->sub[pi]->description;
  d += b->tuning;
  if (buf && n) {
    const size_t k = std::min(n - 1, d.size());
    std::memcpy(buf, d.data(), k);
    buf[k] = 0;
  }
  return d.size();
}

}  // extern "C"
