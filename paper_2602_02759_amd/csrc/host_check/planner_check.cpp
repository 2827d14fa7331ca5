// Host-only exercise of the planner (parsing, loss cases, block lowering,
// tile geometry and the index tables) for a sanitizer build: compiled with
// g++ -fsanitize=address,undefined together with planner.cpp, it walks valid
// and malformed model strings, random CP/Tucker/tensor-train/many-body sizes
// and the direct lowering, and checks the tables' invariants.  Any
// out-of-bounds access or undefined behaviour aborts the program; an invariant
// that does not hold makes it exit with status 1.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "../planner.hpp"

using namespace nnef;

static int g_fail = 0;
#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++g_fail;                                                       \
    }                                                                 \
  } while (0)

static void plan_model(const std::string& s, const std::vector<int64_t>& sizes,
                       const std::vector<int64_t>& ranks) {
  Model m;
  std::string err;
  if (parse_model(s, m, err) != ST_OK) return;
  if (sizes.size() != m.out.size() || ranks.size() != m.latent.size()) return;
  for (size_t i = 0; i < sizes.size(); ++i) m.size[(unsigned char)m.out[i]] = sizes[i];
  for (size_t i = 0; i < ranks.size(); ++i) m.size[(unsigned char)m.latent[i]] = ranks[i];
  int64_t N = 1;
  for (auto v : sizes) N *= v;
  std::vector<int64_t> ws;
  for (int l = 0; l < (int)m.ops.size(); ++l) {
    BlockPlan bp;
    Status st = lower_block(m, l, bp, ws, err);
    if (st == ST_UNSUPPORTED) st = lower_direct(m, l, bp, ws, err, 512);
    if (st != ST_OK) continue;
    if (bp.direct) {
      CHECK(bp.nP * bp.nQ == N);
      auto yp = offsets_table(m, bp.P), yq = offsets_table(m, bp.Q);
      CHECK((int64_t)yp.size() == bp.nP && (int64_t)yq.size() == bp.nQ);
      for (auto v : yp) CHECK((int64_t)v < N);
      for (auto v : yq) CHECK((int64_t)v < N);
      auto thr = offsets_in(m, bp.kappa, m.ops[l]);
      CHECK((int64_t)thr.size() == bp.K);
      for (int o : bp.others) {
        auto lat = offsets_in(m, bp.kappa + bp.S, m.ops[o]);
        CHECK((int64_t)lat.size() == (int64_t)bp.K * bp.KS);
      }
      CHECK(bp.n_wg == bp.n_panels * bp.n_chunks && bp.rows_per_wg * bp.qlanes * bp.G == 256);
      (void)describe_block(m, bp);
      continue;
    }
    if (!choose_geometry(m, bp, 512)) continue;
    CHECK(bp.nP * bp.nQ == N);
    CHECK(!bp.Q.empty() || bp.L_direct);  // never the reconstruction materialised
    auto poff = offsets_table(m, bp.P), qoy = offsets_table(m, bp.qo);
    CHECK((int64_t)poff.size() == bp.nP && (int64_t)qoy.size() == bp.nqo);
    for (auto v : poff) CHECK((int64_t)v < N);
    for (auto v : qoy) CHECK((int64_t)v < N);
    auto ib = inner_base_table(m, bp);
    const Piece& in = bp.pieces[bp.inner];
    for (auto v : ib) CHECK((int64_t)v + (bp.nqi - 1) * bp.in_stride < in.nrows);
    for (int i : bp.outers) {
      auto t = outer_row_table(m, bp, i);
      for (auto v : t) CHECK((int64_t)v < bp.pieces[i].nrows);
    }
    CHECK(bp.n_chunks * (bp.wave_rows ? 1 : 4) * (int64_t)bp.steps_per_wave >= bp.n_steps);
    (void)describe_block(m, bp);
  }
}

int main() {
  const char* bad[] = {"ir,jr", "ir,jr->ij->k", "ir,jr->iz", "iir,jr->ij", "ir,jr->iij", "i1,jr->ij",
                       "ir,,jr->ij", "", "->", ",->i", "ir,jr->", "  ir , jr -> ij "};
  for (const char* s : bad) {
    Model m;
    std::string err;
    (void)parse_model(s, m, err);
  }
  LossSpec ls;
  std::string err;
  const double ab[][2] = {{1, 0}, {1, 1}, {0.5, 1}, {1, -1}, {0.7, 0.3}, {0, 1}, {0, 0.5}, {2, -1}, {1.5, -1.5},
                          {-1, 2}, {1e300, 1}, {0, 0}};
  for (auto& x : ab) (void)make_loss(x[0], x[1], ls, err);
  for (int f = 0; f < 5; ++f) (void)make_family(f, f == 2 ? 3.0 : -1.0, ls, err);

  std::mt19937_64 rng(7);
  auto U = [&](int lo, int hi) { return (int64_t)(lo + (int)(rng() % (uint64_t)(hi - lo + 1))); };
  for (int it = 0; it < 60; ++it) {
    plan_model("ir,jr,kr->ijk", {U(1, 300), U(1, 300), U(1, 300)}, {U(1, 100)});
    plan_model("ia,jb,kc,abc->ijk", {U(1, 90), U(1, 90), U(1, 40)}, {U(1, 40), U(1, 40), U(1, 20)});
    plan_model("ia,jab,kbc,lc->ijkl", {U(1, 40), U(1, 40), U(1, 30), U(1, 30)}, {U(1, 20), U(1, 20), U(1, 20)});
    plan_model("ij,jk,ik->ijk", {U(1, 60), U(1, 60), U(1, 60)}, {});
    plan_model("rij,jk,ik->ijk", {U(1, 30), U(1, 30), U(1, 30)}, {U(1, 6)});
    plan_model("wr,dr,hr,irk,jrk->wdhij", {U(1, 9), U(1, 7), U(1, 9), U(1, 20), U(1, 20)}, {U(1, 12), U(1, 8)});
    plan_model("ir,jr,ak,kr,tr->ijat", {U(1, 40), U(1, 40), U(1, 12), U(1, 20)}, {U(1, 70), U(1, 9)});
    plan_model("ij,i->ij", {U(1, 50), U(1, 50)}, {});
    plan_model("ia,jb,kc,ar,br,cr->ijk", {U(1, 50), U(1, 50), U(1, 30)}, {U(1, 20), U(1, 20), U(1, 10), U(1, 40)});
  }
  std::printf("planner host check: %d failed checks\n", g_fail);
  return g_fail ? 1 : 0;
}
