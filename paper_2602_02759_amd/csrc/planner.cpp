// Host planner of libnnef: parse the model string, choose the loss case, and
// lower every block update of Algorithm 1 to the fused pass.
//
// Lowering of block l.  Split the observed modes into P (containing the modes
// of operand l) and Q, with every operand's observed modes entirely on one
// side; operands without observed modes go to either side.  With kappa the
// contracted letters used on both sides,
//   yhat[p, q] = sum_kappa L[p, kappa] R[q, kappa]                      (eq. 2.1)
// where L (R) contracts the P-side (Q-side) operands over their other
// letters.  The numerator of eq. 3.6 for operand l factors through L:
//   N_L[p, kappa] = sum_q a(y, yhat)[p, q] R[q, kappa],
//   N_l = einsum(P-side operands except l, N_L -> subscripts of l),
// the last step ("chain-back") being the P-side part of einstr_l.  When l is
// the only P-side operand and is laid out as [P modes, kappa], N_l = N_L.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <sstream>
#include <stdexcept>

#include "planner.hpp"

namespace nnef {

static bool is_letter(char c) { return (c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z'); }

// The other decomposable likelihoods of App. B: negative binomial (phi),
// binomial odds (n trials; n = 1 is Bernoulli): a = y/yh, g = lambda;
// Jensen-Shannon: a = log((y + yh)/(2 yh)), b = 1, g = log.
Status make_family(int family, double param, LossSpec& ls, std::string& err) {
  ls.alpha = 1.0;
  ls.beta = 0.0;
  ls.wk = WK_FAM;
  ls.gamma = 1.0;
  ls.fparam = param;
  if (family == 1 || family == 2) {
    if (!(param > 0.0) || !std::isfinite(param)) {
      err = family == 1 ? "the negative binomial dispersion phi must be positive and finite"
                        : "the number of binomial trials n must be positive and finite";
      return ST_LOSS;
    }
    ls.upd = UP_ONE;
    ls.lk = family == 1 ? LK_NB : LK_BIN;
    return ST_OK;
  }
  if (family == 3) {
    ls.upd = UP_EXP;
    ls.lk = LK_JS;
    return ST_OK;
  }
  err = "unknown likelihood family";
  return ST_LOSS;
}

// ---------------------------------------------------------------------------
// Model strings (Sec. 2, eq. 2.2)
// ---------------------------------------------------------------------------
Status parse_model(const std::string& s_in, Model& m, std::string& err) {
  std::string s;
  for (char c : s_in)
    if (c != ' ') s.push_back(c);
  const size_t arrow = s.find("->");
  if (arrow == std::string::npos || s.find("->", arrow + 2) != std::string::npos) {
    err = "model string needs exactly one '->'";
    return ST_PARSE;
  }
  std::string lhs = s.substr(0, arrow);
  m.out = s.substr(arrow + 2);
  m.ops.clear();
  std::string cur;
  for (size_t i = 0; i <= lhs.size(); ++i) {
    if (i == lhs.size() || lhs[i] == ',') {
      if (cur.empty()) {
        err = "empty operand in model string";
        return ST_PARSE;
      }
      m.ops.push_back(cur);
      cur.clear();
    } else {
      cur.push_back(lhs[i]);
    }
  }
  std::vector<std::string> all = m.ops;
  all.push_back(m.out);
  for (const auto& t : all) {
    std::set<char> seen;
    for (char c : t) {
      if (!is_letter(c)) {
        err = std::string("bad subscript character '") + c + "'";
        return ST_PARSE;
      }
      if (!seen.insert(c).second) {
        err = "letter '" + std::string(1, c) + "' repeated in '" + t + "'";
        return ST_PARSE;
      }
    }
  }
  for (char c : m.out) {
    bool used = false;
    for (const auto& t : m.ops) used |= t.find(c) != std::string::npos;
    if (!used) {
      err = "output letter '" + std::string(1, c) + "' appears in no operand";
      return ST_PARSE;
    }
  }
  m.latent.clear();
  for (const auto& t : m.ops)
    for (char c : t)
      if (m.out.find(c) == std::string::npos && m.latent.find(c) == std::string::npos)
        m.latent.push_back(c);
  return ST_OK;
}

// ---------------------------------------------------------------------------
// (alpha, beta) -> weights, update exponent, loss case (App. B)
// ---------------------------------------------------------------------------
Status make_loss(double al, double be, LossSpec& ls, std::string& err) {
  if (!std::isfinite(al) || !std::isfinite(be)) {
    err = "alpha and beta must be finite";
    return ST_LOSS;
  }
  ls.alpha = al;
  ls.beta = be;
  if (al == 0.0) {
    if (be != 1.0) {
      err = "alpha = 0 with beta != 1 has no multiplicative update (App. B)";
      return ST_LOSS;
    }
    ls.wk = WK_RKL;
    ls.upd = UP_EXP;
    ls.gamma = 1.0;
    ls.lk = LK_ALPHA0;
    return ST_OK;
  }
  // g(lambda) of App. B with rho = (1 - beta)/alpha; g^{-1}(r) = r^gamma
  const double rho = (1.0 - be) / al;
  if (rho > 1.0) ls.gamma = 1.0 / (1.0 - be);
  else if (rho < 0.0) ls.gamma = 1.0 / (al + be - 1.0);
  else ls.gamma = 1.0 / al;
  ls.upd = ls.gamma == 1.0 ? UP_ONE : ls.gamma == 2.0 ? UP_SQR : ls.gamma == 0.5 ? UP_SQRT : UP_POW;
  if (al == 1.0 && be == 0.0) ls.wk = WK_KL;
  else if (al == 1.0 && be == 1.0) ls.wk = WK_EUC;
  else if (al == 0.5 && be == 1.0) ls.wk = WK_SQRT;
  else if (al == 1.0 && be == -1.0) ls.wk = WK_IS;
  else ls.wk = WK_GEN;
  // loss case, in the order of the definition
  if (al == 1.0 && be == 0.0) ls.lk = LK_KL;
  else if (al == 1.0 && be == 1.0) ls.lk = LK_EUC;
  else if (al == 1.0 && be == -1.0) ls.lk = LK_IS;
  else if (al == 0.5 && be == 1.0) ls.lk = LK_SQRT;
  else if (be != 0.0 && al + be != 0.0) ls.lk = LK_GENERIC;
  else if (be == 0.0) ls.lk = LK_BETA0;
  else ls.lk = LK_AMB;
  return ST_OK;
}

// ---------------------------------------------------------------------------
// Pairwise contraction programs
// ---------------------------------------------------------------------------
int64_t TensorRef::size_of(const Model& m) const {
  int64_t n = 1;
  for (char c : subs) n *= m.size[(unsigned char)c];
  return n;
}

std::vector<int64_t> row_major_strides(const Model& m, const std::string& subs, int64_t inner) {
  std::vector<int64_t> st(subs.size());
  int64_t s = inner;
  for (int i = (int)subs.size() - 1; i >= 0; --i) {
    st[i] = s;
    s *= m.size[(unsigned char)subs[i]];
  }
  return st;
}

// Contract `in` into `out` (whose subs and strides are fixed), greedily
// contracting the pair with the smallest intermediate first.  New
// intermediates are workspace buffers appended to `ws_sizes`.
std::vector<Step> plan_contraction(const Model& m, std::vector<TensorRef> in, const TensorRef& out,
                                   std::vector<int64_t>& ws_sizes, int64_t& macs) {
  std::vector<Step> steps;
  auto letters_of = [](const std::vector<TensorRef>& v, int skip1, int skip2) {
    std::set<char> s;
    for (int i = 0; i < (int)v.size(); ++i)
      if (i != skip1 && i != skip2)
        for (char c : v[i].subs) s.insert(c);
    return s;
  };
  while (in.size() > 2) {
    int bi = -1, bj = -1;
    int64_t best = -1;
    std::string best_subs;
    for (int i = 0; i < (int)in.size(); ++i)
      for (int j = i + 1; j < (int)in.size(); ++j) {
        std::set<char> keep = letters_of(in, i, j);
        for (char c : out.subs) keep.insert(c);
        std::string subs;
        std::set<char> u;
        for (char c : in[i].subs + in[j].subs)
          if (keep.count(c) && u.insert(c).second) subs.push_back(c);
        int64_t n = 1;
        for (char c : subs) n *= m.size[(unsigned char)c];
        if (best < 0 || n < best) {
          best = n;
          bi = i;
          bj = j;
          best_subs = subs;
        }
      }
    // letters of the intermediate: those summed later first, then the final
    // output's letters in its order, so that the intermediate's fastest index
    // is the output's fastest one and the next step reads it coalesced
    std::stable_sort(best_subs.begin(), best_subs.end(), [&](char x, char y) {
      const size_t px = out.subs.find(x), py = out.subs.find(y);
      const long kx = px == std::string::npos ? -1 : (long)px, ky = py == std::string::npos ? -1 : (long)py;
      return kx < ky;
    });
    TensorRef tmp;
    tmp.kind = TK_WS;
    tmp.id = (int)ws_sizes.size();
    tmp.subs = best_subs;
    tmp.strides = row_major_strides(m, best_subs, 1);
    ws_sizes.push_back(best);
    Step st;
    st.in = {in[bi], in[bj]};
    st.out = tmp;
    steps.push_back(st);
    in.erase(in.begin() + bj);
    in.erase(in.begin() + bi);
    in.push_back(tmp);
  }
  Step st;
  st.in = in;
  st.out = out;
  steps.push_back(st);
  for (auto& s : steps) {
    std::set<char> all;
    for (auto& t : s.in)
      for (char c : t.subs) all.insert(c);
    s.sum.clear();
    for (char c : all)
      if (s.out.subs.find(c) == std::string::npos) s.sum.push_back(c);
    int64_t n = s.out.size_of(m);
    for (char c : s.sum) n *= m.size[(unsigned char)c];
    macs += n;
  }
  return steps;
}

// ---------------------------------------------------------------------------
// Block lowering
// ---------------------------------------------------------------------------
static std::string letters_in_order(const std::string& order, const std::set<char>& s) {
  std::string r;
  for (char c : order)
    if (s.count(c)) r.push_back(c);
  return r;
}

static int pad_kappa(int64_t K) { return K <= 16 ? 16 : K <= 32 ? 32 : K <= 64 ? 64 : -1; }

Status lower_block(const Model& m, int ell, BlockPlan& bp, std::vector<int64_t>& ws_sizes,
                   std::string& err, bool direct_only) {
  const int L = (int)m.ops.size();
  const int M = (int)m.out.size();
  auto obs_of = [&](int o) {
    std::string r;
    for (char c : m.ops[o])
      if (m.out.find(c) != std::string::npos) r.push_back(c);
    return r;
  };
  double best_cost = -1;
  BlockPlan best;
  std::vector<int64_t> best_ws;
  const std::string obs_l = obs_of(ell);
  for (int pmask = 1; pmask < (1 << M); ++pmask) {
    std::set<char> P;
    for (int i = 0; i < M; ++i)
      if (pmask >> i & 1) P.insert(m.out[i]);
    bool ok = true;
    for (char c : obs_l) ok &= P.count(c) > 0;
    if (!ok) continue;
    // side of each operand: 0 = P, 1 = Q, -1 = free
    std::vector<int> side(L, -1);
    std::vector<int> free_ops;
    for (int o = 0; o < L && ok; ++o) {
      std::string ob = obs_of(o);
      if (ob.empty()) {
        if (o == ell) side[o] = 0;
        else free_ops.push_back(o);
        continue;
      }
      int inP = 0;
      for (char c : ob) inP += P.count(c) ? 1 : 0;
      if (inP == (int)ob.size()) side[o] = 0;
      else if (inP == 0) side[o] = 1;
      else ok = false;
    }
    if (!ok) continue;
    const bool q_empty = (int)P.size() == M;
    for (int fmask = 0; fmask < (1 << free_ops.size()); ++fmask) {
      std::vector<int> sd = side;
      for (size_t f = 0; f < free_ops.size(); ++f) sd[free_ops[f]] = q_empty ? 0 : (fmask >> f & 1);
      if (q_empty && fmask) break;
      std::set<char> latP, latQ;
      for (int o = 0; o < L; ++o)
        for (char c : m.ops[o])
          if (m.out.find(c) == std::string::npos) (sd[o] == 0 ? latP : latQ).insert(c);
      std::set<char> kap;
      for (char c : latP)
        if (latQ.count(c)) kap.insert(c);
      // kappa order: operand l's order if it holds them all, else first appearance
      std::string kappa = letters_in_order(m.ops[ell], kap);
      if (kappa.size() != kap.size()) kappa = letters_in_order(m.latent, kap);
      int64_t K = 1;
      for (char c : kappa) K *= m.size[(unsigned char)c];
      const int KP = pad_kappa(K);
      if (KP < 0) continue;

      BlockPlan bp2;
      std::vector<int64_t> ws2 = ws_sizes;
      bp2.ell = ell;
      bp2.P = letters_in_order(m.out, P);
      std::set<char> Qs;
      for (char c : m.out)
        if (!P.count(c)) Qs.insert(c);
      bp2.Q = letters_in_order(m.out, Qs);
      bp2.kappa = kappa;
      bp2.K = (int)K;
      bp2.KP = KP;
      bp2.nP = 1;
      for (char c : bp2.P) bp2.nP *= m.size[(unsigned char)c];
      bp2.nQ = 1;
      for (char c : bp2.Q) bp2.nQ *= m.size[(unsigned char)c];
      bp2.side = sd;
      int64_t macs = 0;
      double mat_elems = 0;
      // ---- row side L
      std::vector<TensorRef> pops, qops;
      for (int o = 0; o < L; ++o) {
        TensorRef t;
        t.kind = TK_FACTOR;
        t.id = o;
        t.subs = m.ops[o];
        t.strides = row_major_strides(m, t.subs, 1);
        (sd[o] == 0 ? pops : qops).push_back(t);
      }
      bp2.L_direct = pops.size() == 1 && m.ops[ell] == bp2.P + kappa;
      // every observed letter on the row side: L would be the reconstruction
      // itself, materialised, unless operand l is it (the direct lowering
      // takes such blocks instead)
      if (q_empty && !bp2.L_direct) continue;
      if (bp2.L_direct) {
        bp2.ldL = (int)K;
      } else {
        TensorRef out;
        out.kind = TK_WS;
        out.id = (int)ws2.size();
        out.subs = bp2.P + kappa;
        ws2.push_back(bp2.nP * KP);
        out.strides = row_major_strides(m, bp2.P, KP);
        auto ks = row_major_strides(m, kappa, 1);
        out.strides.insert(out.strides.end(), ks.begin(), ks.end());
        bp2.L_buf = out.id;
        bp2.ldL = KP;
        bp2.L_prog = plan_contraction(m, pops, out, ws2, macs);
        mat_elems += (double)bp2.nP * (KP + 2.0 * K);  // L, and N_L, D_L for the chain-back
        // chain-back: N_l = einsum(P-side operands except l, N_L -> ops[l])
        std::vector<TensorRef> cin;
        for (auto& t : pops)
          if (t.id != ell) cin.push_back(t);
        TensorRef nl;
        nl.kind = TK_NL;
        nl.id = 0;
        nl.subs = bp2.P + kappa;
        nl.strides = row_major_strides(m, nl.subs, 1);
        cin.push_back(nl);
        TensorRef no;
        no.kind = TK_WS;
        no.id = (int)ws2.size();
        no.subs = m.ops[ell];
        no.strides = row_major_strides(m, no.subs, 1);
        ws2.push_back(no.size_of(m));
        bp2.Nl_buf = no.id;
        int64_t cb = 0;
        bp2.chainN = plan_contraction(m, cin, no, ws2, cb);
        for (auto& t : cin)
          if (t.kind == TK_NL) t.kind = TK_DL;
        no.id = (int)ws2.size();
        ws2.push_back(no.size_of(m));
        bp2.Dl_buf = no.id;
        bp2.chainD = plan_contraction(m, cin, no, ws2, cb);
        macs += cb;
        bp2.NL_buf = (int)ws2.size();
        ws2.push_back(bp2.nP * K);
        bp2.DL_buf = (int)ws2.size();
        ws2.push_back(bp2.nP * K);
      }
      // ---- column side R: a product of pieces.  Column-side operands that
      // share an observed letter, or a latent letter outside kappa, belong to
      // one piece (operands with no observed letter join the first piece).  A
      // piece of one operand laid out as [its observed letters, kappa] is that
      // factor itself; any other piece is contracted before the pass into a
      // buffer [its observed letters in Y order, kappa] (when that piece spans
      // every column letter, this is the whole column side materialised).
      bp2.pieces.clear();
      std::vector<std::vector<int>> groups;  // indices into qops
      if (!q_empty && !qops.empty()) {
        const int nq = (int)qops.size();
        std::vector<int> root(nq);
        for (int i = 0; i < nq; ++i) root[i] = i;
        auto find = [&](int i) {
          while (root[i] != i) i = root[i] = root[root[i]];
          return i;
        };
        for (int i = 0; i < nq; ++i)
          for (int j = i + 1; j < nq; ++j)
            for (char c : qops[i].subs)
              if (qops[j].subs.find(c) != std::string::npos && !kap.count(c)) root[find(j)] = find(i);
        std::vector<int> order;  // group roots, first appearance
        for (int i = 0; i < nq; ++i)
          if (std::find(order.begin(), order.end(), find(i)) == order.end()) order.push_back(find(i));
        for (int g : order) {
          std::vector<int> mem;
          for (int i = 0; i < nq; ++i)
            if (find(i) == g) mem.push_back(i);
          groups.push_back(mem);
        }
        auto has_obs = [&](const std::vector<int>& mem) {
          for (int i : mem)
            for (char c : qops[i].subs)
              if (m.out.find(c) != std::string::npos) return true;
          return false;
        };
        int first = -1;
        for (int g = 0; g < (int)groups.size() && first < 0; ++g)
          if (has_obs(groups[g])) first = g;
        for (int g = (int)groups.size() - 1; g >= 0 && first >= 0; --g)
          if (!has_obs(groups[g])) {
            groups[first].insert(groups[first].end(), groups[g].begin(), groups[g].end());
            groups.erase(groups.begin() + g);
            if (g < first) --first;
          }
      }
      if (q_empty) {
        Piece pc;
        pc.factor = -1;
        pc.ld = KP;
        pc.nrows = bp2.nQ;
        pc.ws = (int)ws2.size();  // a single row [1, 0, ...]
        ws2.push_back(KP);
        bp2.ones_buf = pc.ws;
        bp2.pieces.push_back(pc);
      } else {
        if (groups.empty() || (int)groups.size() > kMaxPieces) continue;
        for (auto& mem : groups) {
          std::set<char> obs_set;
          std::vector<TensorRef> gops;
          for (int i : mem) {
            gops.push_back(qops[i]);
            for (char c : qops[i].subs)
              if (m.out.find(c) != std::string::npos) obs_set.insert(c);
          }
          Piece pc;
          pc.nrows = 1;
          for (char c : obs_set) pc.nrows *= m.size[(unsigned char)c];
          std::string ob0;
          for (char c : gops[0].subs)
            if (m.out.find(c) != std::string::npos) ob0.push_back(c);
          if (gops.size() == 1 && gops[0].subs == ob0 + kappa) {
            pc.factor = gops[0].id;
            pc.ld = (int)K;
            pc.obs = ob0;
          } else {
            const bool whole = obs_set.size() == bp2.Q.size();
            pc.factor = -1;
            pc.obs = letters_in_order(m.out, obs_set);
            pc.ld = whole ? KP : (int)K;
            TensorRef out;
            out.kind = TK_WS;
            out.id = (int)ws2.size();
            out.subs = pc.obs + kappa;
            ws2.push_back(pc.nrows * pc.ld);
            out.strides = row_major_strides(m, pc.obs, pc.ld);
            auto ks = row_major_strides(m, kappa, 1);
            out.strides.insert(out.strides.end(), ks.begin(), ks.end());
            pc.ws = out.id;
            auto steps = plan_contraction(m, gops, out, ws2, macs);
            bp2.R_prog.insert(bp2.R_prog.end(), steps.begin(), steps.end());
            mat_elems += (double)pc.nrows * pc.ld;
          }
          bp2.pieces.push_back(pc);
        }
      }
      {
        std::set<char> seen;
        bp2.pieces_disjoint = true;
        for (auto& pc : bp2.pieces)
          for (char c : pc.obs) bp2.pieces_disjoint &= seen.insert(c).second;
      }
      // ---- column decomposition q = (qo, qi)
      bp2.qi = q_empty ? 0 : bp2.Q.back();
      bp2.qo = q_empty ? std::string() : bp2.Q.substr(0, bp2.Q.size() - 1);
      bp2.nqi = q_empty ? 1 : m.size[(unsigned char)bp2.qi];
      bp2.nqo = bp2.nQ / bp2.nqi;
      bp2.qi_ystride = 0;
      if (!q_empty) {
        int64_t st = 1;
        for (int i = (int)m.out.size() - 1; i >= 0 && m.out[i] != bp2.qi; --i) st *= m.size[(unsigned char)m.out[i]];
        bp2.qi_ystride = st;
      }
      bp2.outers.clear();
      bp2.inner = 0;
      bp2.in_stride = q_empty ? 0 : 1;
      if (!q_empty) {
        for (int i = 0; i < (int)bp2.pieces.size(); ++i) {
          const Piece& pc = bp2.pieces[i];
          const size_t pos = pc.obs.find(bp2.qi);
          if (pos == std::string::npos) {
            bp2.outers.push_back(i);
          } else {
            bp2.inner = i;
            int64_t st = 1;
            for (size_t j = pos + 1; j < pc.obs.size(); ++j) st *= m.size[(unsigned char)pc.obs[j]];
            bp2.in_stride = st;
          }
        }
      }
      // ---- cost: fused MFMA work on padded tiles, plus the generic contractions
      // tile of the fused pass: 64 rows x 16 columns (width 16, 16x16 MFMA), 32 x 32 (widths 32
      // and 64, 32x32 MFMA)
      const int rows = KP == 16 ? 64 : 32;
      const int qstep = KP == 16 ? 16 : 32;
      const double Neff = std::ceil((double)bp2.nP / rows) * rows * (double)bp2.nqo *
                          std::ceil((double)bp2.nqi / qstep) * qstep;
      // a materialised float is written once and read back once: about 8 bytes
      // of HBM traffic, priced at ~12 MFMA flops per byte (the fused pass's
      // sustained flop rate over the sustained HBM rate of the side kernels)
      const double cost = Neff * 6.0 * KP + 16.0 * macs + 96.0 * mat_elems;
      if (direct_only && (!bp2.L_direct || q_empty || !bp2.R_prog.empty())) continue;
      if (best_cost < 0 || cost < best_cost) {
        best_cost = cost;
        best = bp2;
        best_ws = ws2;
      }
    }
  }
  if (best_cost < 0) {
    err = "block " + std::to_string(ell) + " ('" + m.ops[ell] +
          (direct_only ? "') has no lowering without side operands with a contraction width <= 64"
                       : "') has no lowering with a contraction width <= 64");
    return ST_UNSUPPORTED;
  }
  bp = best;
  ws_sizes = best_ws;
  return ST_OK;
}

std::vector<uint32_t> offsets_in(const Model& m, const std::string& letters, const std::string& subs) {
  const std::vector<int64_t> st = row_major_strides(m, subs, 1);
  std::vector<int64_t> sz, str;
  for (char c : letters) {
    sz.push_back(m.size[(unsigned char)c]);
    const size_t pos = subs.find(c);
    str.push_back(pos == std::string::npos ? 0 : st[pos]);
  }
  int64_t n = 1;
  for (auto v : sz) n *= v;
  std::vector<uint32_t> t((size_t)n);
  std::vector<int64_t> idx(sz.size(), 0);
  int64_t off = 0;
  for (int64_t i = 0; i < n; ++i) {
    t[(size_t)i] = (uint32_t)off;
    for (int d = (int)sz.size() - 1; d >= 0; --d) {
      ++idx[d];
      off += str[d];
      if (idx[d] < sz[d]) break;
      off -= sz[d] * str[d];
      idx[d] = 0;
    }
  }
  return t;
}

Status lower_direct(const Model& m, int ell, BlockPlan& bp, std::vector<int64_t>& ws_sizes,
                    std::string& err, int target_wg) {
  const int L = (int)m.ops.size();
  const std::string tag = "block " + std::to_string(ell) + " ('" + m.ops[ell] + "')";
  if (L - 1 > kMaxDirectOps) {
    err = tag + ": the direct lowering takes at most " + std::to_string(kMaxDirectOps + 1) + " operands";
    return ST_UNSUPPORTED;
  }
  BlockPlan b;
  std::vector<int64_t> ws = ws_sizes;
  b.ell = ell;
  b.direct = true;
  std::set<char> Ps;
  std::string R;
  for (char c : m.ops[ell]) {
    if (m.out.find(c) != std::string::npos) Ps.insert(c);
    else R.push_back(c);
  }
  b.P = letters_in_order(m.out, Ps);
  std::set<char> Qs;
  for (char c : m.out)
    if (!Ps.count(c)) Qs.insert(c);
  b.Q = letters_in_order(m.out, Qs);
  for (char c : m.latent)
    if (R.find(c) == std::string::npos) b.S.push_back(c);
  b.kappa = R;
  int64_t K = 1, KS = 1;
  for (char c : R) K *= m.size[(unsigned char)c];
  for (char c : b.S) KS *= m.size[(unsigned char)c];
  if (K > kDirectMaxK || (int64_t)(L - 1) * K * KS > kDirectMaxLat) {
    err = tag + ": the direct lowering takes at most " + std::to_string(kDirectMaxK) +
          " latent combinations in the block's operand and " + std::to_string(kDirectMaxLat) +
          " (other operands x latent combinations) in all; this block has " + std::to_string(K) + " and " +
          std::to_string((int64_t)(L - 1) * K * KS);
    return ST_UNSUPPORTED;
  }
  b.K = (int)K;
  b.KP = (int)K;
  b.KS = (int)KS;
  b.nP = 1;
  for (char c : b.P) b.nP *= m.size[(unsigned char)c];
  b.nQ = 1;
  for (char c : b.Q) b.nQ *= m.size[(unsigned char)c];
  for (int o = 0; o < L; ++o)
    if (o != ell) b.others.push_back(o);
  b.ldL = (int)K;
  b.L_direct = m.ops[ell] == b.P + R;
  if (!b.L_direct) {  // N_L, D_L as [P][R], then permuted to operand l's layout
    TensorRef nl;
    nl.kind = TK_NL;
    nl.subs = b.P + R;
    nl.strides = row_major_strides(m, nl.subs, 1);
    TensorRef no;
    no.kind = TK_WS;
    no.id = (int)ws.size();
    no.subs = m.ops[ell];
    no.strides = row_major_strides(m, no.subs, 1);
    ws.push_back(no.size_of(m));
    b.Nl_buf = no.id;
    int64_t cb = 0;
    b.chainN = plan_contraction(m, {nl}, no, ws, cb);
    nl.kind = TK_DL;
    no.id = (int)ws.size();
    ws.push_back(no.size_of(m));
    b.Dl_buf = no.id;
    b.chainD = plan_contraction(m, {nl}, no, ws, cb);
    b.NL_buf = (int)ws.size();
    ws.push_back(b.nP * K);
    b.DL_buf = (int)ws.size();
    ws.push_back(b.nP * K);
  }
  // geometry: G threads per entry (each at most kDirectKPT latent combinations),
  // 256 / G entry groups per workgroup split into rows x column lanes
  int G = 1;
  while (G * kDirectKPT < K) G *= 2;
  b.G = G;
  const int eg = 256 / G;
  int ql = 1;  // column lanes per row: about eight entries per thread when the row is long enough
  while (ql * 2 <= eg && ql * 2 <= std::max<int64_t>(1, b.nQ / 8)) ql *= 2;
  b.qlanes = ql;
  b.rows_per_wg = eg / ql;
  const int64_t panels = (b.nP + b.rows_per_wg - 1) / b.rows_per_wg;
  int64_t chunks = std::max<int64_t>(1, (target_wg + panels - 1) / panels);
  chunks = std::min<int64_t>(chunks, (b.nQ + ql - 1) / ql);
  const int64_t qpc = (b.nQ + chunks - 1) / chunks;
  chunks = (b.nQ + qpc - 1) / qpc;
  if (panels * chunks >= (int64_t(1) << 31) || b.nP >= (int64_t(1) << 31) || b.nQ >= (int64_t(1) << 31)) {
    err = tag + ": grid too large";
    return ST_SHAPE;
  }
  b.n_panels = (int)panels;
  b.q_per_chunk = (int)qpc;
  b.n_chunks = (int)chunks;
  b.n_wg = (int)(panels * chunks);
  bp = b;
  ws_sizes = ws;
  return ST_OK;
}

// Element offsets in Y (row-major over the output letters) of every
// multi-index over `letters` (enumerated row-major, last letter fastest).
std::vector<uint32_t> offsets_table(const Model& m, const std::string& letters) {
  std::vector<int64_t> ystride(m.out.size());
  int64_t s = 1;
  for (int i = (int)m.out.size() - 1; i >= 0; --i) {
    ystride[i] = s;
    s *= m.size[(unsigned char)m.out[i]];
  }
  std::vector<int64_t> sz, st;
  for (char c : letters) {
    sz.push_back(m.size[(unsigned char)c]);
    st.push_back(ystride[m.out.find(c)]);
  }
  int64_t n = 1;
  for (auto v : sz) n *= v;
  std::vector<uint32_t> t((size_t)n);
  std::vector<int64_t> idx(sz.size(), 0);
  int64_t off = 0;
  for (int64_t i = 0; i < n; ++i) {
    t[(size_t)i] = (uint32_t)off;
    for (int d = (int)sz.size() - 1; d >= 0; --d) {
      ++idx[d];
      off += st[d];
      if (idx[d] < sz[d]) break;
      off -= sz[d] * st[d];
      idx[d] = 0;
    }
  }
  return t;
}

// Row of every column multi-index q (over Q letters) in a piece whose
// observed letters are `obs` (in the piece's own order).
std::vector<uint32_t> piece_rows_table(const Model& m, const std::string& Q, const std::string& obs) {
  std::vector<int64_t> rstride(obs.size());
  int64_t s = 1;
  for (int i = (int)obs.size() - 1; i >= 0; --i) {
    rstride[i] = s;
    s *= m.size[(unsigned char)obs[i]];
  }
  std::vector<int64_t> sz, st;
  for (char c : Q) {
    sz.push_back(m.size[(unsigned char)c]);
    const size_t pos = obs.find(c);
    st.push_back(pos == std::string::npos ? 0 : rstride[pos]);
  }
  int64_t n = 1;
  for (auto v : sz) n *= v;
  std::vector<uint32_t> t((size_t)n);
  std::vector<int64_t> idx(sz.size(), 0);
  int64_t off = 0;
  for (int64_t i = 0; i < n; ++i) {
    t[(size_t)i] = (uint32_t)off;
    for (int d = (int)sz.size() - 1; d >= 0; --d) {
      ++idx[d];
      off += st[d];
      if (idx[d] < sz[d]) break;
      off -= sz[d] * st[d];
      idx[d] = 0;
    }
  }
  return t;
}


bool choose_geometry(const Model& m, BlockPlan& bp, int target_wg) {
  (void)m;
  bp.qstep = bp.KP == 16 ? 16 : 32;
  const int64_t nqis = (bp.nqi + bp.qstep - 1) / bp.qstep;
  bp.n_steps = bp.nqo * nqis;
  // many rows and few column steps: give each wave its own rows, so that a
  // wave runs all steps of its chunk instead of a quarter of them
  bp.wave_rows = (bp.KP != 16 && bp.n_steps <= 64 && bp.nP >= 4096) ? 1 : 0;
  bp.rows = bp.KP == 16 ? 64 : (bp.wave_rows ? 128 : 32);
  const int rows = bp.rows;
  bp.n_panels = (int)((bp.nP + rows - 1) / rows);
  const int split = bp.wave_rows ? 1 : 4;  // waves sharing a chunk's steps
  int64_t chunks = std::max<int64_t>(1, (target_wg + bp.n_panels - 1) / bp.n_panels);
  chunks = std::min<int64_t>(chunks, std::max<int64_t>(1, (bp.n_steps + split - 1) / split));
  const int64_t spw = (bp.n_steps + split * chunks - 1) / (split * chunks);
  if (spw >= (int64_t(1) << 31)) return false;
  bp.steps_per_wave = (int)spw;
  bp.n_chunks = (int)((bp.n_steps + split * spw - 1) / (split * spw));
  const int64_t nwg = (int64_t)bp.n_panels * bp.n_chunks;
  if (nwg >= (int64_t(1) << 31)) return false;
  bp.n_wg = (int)nwg;
  bp.xcd_remap = (bp.n_wg % 8 == 0 && bp.n_wg >= 64) ? 1 : 0;
  bp.vecq = bp.qi_ystride == 1 && bp.nqi % 4 == 0;
  return true;
}

std::vector<uint32_t> inner_base_table(const Model& m, const BlockPlan& bp) {
  const Piece& pc = bp.pieces[bp.inner];
  if (pc.obs.empty()) {  // the single row of an empty column side
    std::vector<uint32_t> t((size_t)bp.nqo);
    for (int64_t i = 0; i < bp.nqo; ++i) t[(size_t)i] = (uint32_t)(i * bp.nqi);
    return t;
  }
  return piece_rows_table(m, bp.qo, pc.obs);
}

std::vector<uint32_t> outer_row_table(const Model& m, const BlockPlan& bp, int piece) {
  return piece_rows_table(m, bp.qo, bp.pieces[piece].obs);
}

bool all_zero(const std::vector<uint32_t>& t) {
  for (auto v : t)
    if (v) return false;
  return true;
}

std::string describe_block(const Model& m, const BlockPlan& bp) {
  std::ostringstream o;
  if (bp.direct) {
    o << "block " << bp.ell << " '" << m.ops[bp.ell] << "': direct P={" << bp.P << "} Q={" << bp.Q
      << "} R={" << bp.kappa << "} S={" << bp.S << "} K=" << bp.K << " KS=" << bp.KS << " nP=" << bp.nP
      << " nQ=" << bp.nQ << " threads/entry=" << bp.G << " rows/wg=" << bp.rows_per_wg
      << (bp.L_direct ? "" : " permute-back") << " grid=" << bp.n_wg << " chunks=" << bp.n_chunks;
    return o.str();
  }
  o << "block " << bp.ell << " '" << m.ops[bp.ell] << "': P={" << bp.P << "} Q={" << bp.Q
    << "} kappa={" << bp.kappa << "} K=" << bp.K << " KP=" << bp.KP << " nP=" << bp.nP
    << " nQ=" << bp.nQ << " L=" << (bp.L_direct ? "direct" : "materialised") << " R=";
  if (bp.pieces.size() == 1 && bp.pieces[0].factor < 0) o << "materialised";
  else {
    o << "product(";
    for (size_t i = 0; i < bp.pieces.size(); ++i) {
      const Piece& pc = bp.pieces[i];
      o << (i ? "," : "") << (pc.factor >= 0 ? m.ops[pc.factor] : "[" + pc.obs + bp.kappa + "]");
    }
    o << ")";
  }
  o << (bp.L_direct ? "" : " chain-back") << " qo={" << bp.qo << "} qi=" << (bp.qi ? bp.qi : '-')
    << (bp.vecq ? " vecq" : "") << " grid=" << bp.n_wg << " chunks=" << bp.n_chunks
    << " steps/wave=" << bp.steps_per_wave << (bp.wave_rows ? " wave-rows" : "");
  return o.str();
}

}  // namespace nnef
