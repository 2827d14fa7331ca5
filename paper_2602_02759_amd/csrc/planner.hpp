// Host-side plan structures of libnnef.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "nnef_internal.hpp"

namespace nnef {

enum Status { ST_OK = 0, ST_PARSE = 1, ST_SHAPE = 2, ST_LOSS = 3, ST_ARG = 4, ST_DEVICE = 5,
              ST_NOMEM = 6, ST_UNSUPPORTED = 7 };

struct Model {
  std::vector<std::string> ops;  // operand subscripts
  std::string out;               // observed letters, in Y's axis order
  std::string latent;            // contracted letters, first-appearance order
  int64_t size[128] = {0};       // size of every letter
};

// Operand of a contraction program.
enum TensorKind { TK_FACTOR = 0, TK_WS = 1, TK_NL = 2, TK_DL = 3 };
struct TensorRef {
  int kind = TK_FACTOR;
  int id = 0;                      // factor index or workspace buffer index
  std::string subs;
  std::vector<int64_t> strides;    // element stride of every letter of subs
  int64_t size_of(const Model& m) const;
};
struct Step {
  std::vector<TensorRef> in;
  TensorRef out;
  std::string sum;                 // letters summed over
};

// One factor of the column-side product, or one materialised buffer.
struct Piece {
  int factor = -1;                 // factor index, or -1 for workspace buffer `ws`
  int ws = -1;
  int ld = 0;                      // row stride (elements)
  int64_t nrows = 0;
  std::string obs;                 // observed letters, in the factor's order
  int idx_buf = -1;                // device table slot of the row index (or -1: identity)
};

struct BlockPlan {
  int ell = 0;
  std::string P, Q, kappa;
  int K = 1, KP = 16;
  int64_t nP = 1, nQ = 1;
  std::vector<int> side;           // 0 = row side, 1 = column side, per operand
  bool L_direct = false;
  int ldL = 0;
  int L_buf = -1;                  // workspace buffer of a materialised L
  std::vector<Step> L_prog;        // builds L (row side) from the current factors
  std::vector<Step> R_prog;        // builds a materialised R
  std::vector<Piece> pieces;
  bool pieces_disjoint = true;     // no observed letter in two pieces (closed-form D valid)
  int ones_buf = -1;               // R = [1] when every mode is on the row side
  std::vector<Step> chainN, chainD;
  int NL_buf = -1, DL_buf = -1;    // [nP][K] reduced N_L, D_L
  int Nl_buf = -1, Dl_buf = -1;    // N_l, D_l shaped like operand l
  // column multi-index q = (qo, qi): qi is the last column-side letter
  std::string qo;
  char qi = 0;
  int64_t nqo = 1, nqi = 1;
  int64_t qi_ystride = 0;          // Y stride of qi
  int inner = 0;                   // piece holding qi (or the materialised buffer)
  std::vector<int> outers;         // pieces indexed by qo only
  int64_t in_stride = 1;           // row stride of qi inside the inner piece
  // launch geometry and device tables (filled by the ABI layer)
  int qstep = 16;                  // columns per step of the fused pass
  int rows = 64;                   // rows per wave (panel height)
  bool vecq = false;
  int n_panels = 0, steps_per_wave = 0, n_chunks = 0, n_wg = 0;
  int64_t n_steps = 0;
  int xcd_remap = 0;
  int wave_rows = 0;  // width 32: waves take separate row panels over the same steps
  uint32_t* d_poff = nullptr;
  uint32_t* d_qoyoff = nullptr;
  uint32_t* d_inbase = nullptr;    // nullptr: all zero
  uint32_t* d_orow[2] = {nullptr, nullptr};
  // direct lowering (strings with no bilinear split of contraction width <= 64):
  // per entry, the latent sums in registers; rows p over P = the observed letters
  // of operand l (Y order), r over R = its latent letters (its order), s over S =
  // the latent letters it does not hold; K = |R| (kappa = R), KS = |S|
  bool direct = false;
  std::string S;
  int KS = 1;
  int G = 1;                       // threads per entry
  int rows_per_wg = 1, qlanes = 1, q_per_chunk = 1;
  std::vector<int> others;         // operands other than l, in order
  uint32_t* d_yq = nullptr;        // [nQ] Y offset of column q
  uint32_t* d_thp = nullptr;       // [nP] offset of row p in operand l
  uint32_t* d_thr = nullptr;       // [K] offset of latent combination r in operand l
  std::vector<uint32_t*> d_opp, d_opq, d_oplat;
};

Status parse_model(const std::string& s, Model& m, std::string& err);
Status make_loss(double alpha, double beta, LossSpec& ls, std::string& err);
Status make_family(int family, double param, LossSpec& ls, std::string& err);
Status lower_block(const Model& m, int ell, BlockPlan& bp, std::vector<int64_t>& ws_sizes,
                   std::string& err, bool direct_only = false);
std::vector<Step> plan_contraction(const Model& m, std::vector<TensorRef> in, const TensorRef& out,
                                   std::vector<int64_t>& ws_sizes, int64_t& macs);
std::vector<int64_t> row_major_strides(const Model& m, const std::string& subs, int64_t inner);
std::vector<uint32_t> offsets_table(const Model& m, const std::string& letters);
std::vector<uint32_t> piece_rows_table(const Model& m, const std::string& Q, const std::string& obs);
// Tables of the column decomposition (host side, uploaded by the ABI layer).
std::vector<uint32_t> inner_base_table(const Model& m, const BlockPlan& bp);
std::vector<uint32_t> outer_row_table(const Model& m, const BlockPlan& bp, int piece);
bool all_zero(const std::vector<uint32_t>& t);
bool choose_geometry(const Model& m, BlockPlan& bp, int target_wg);
// Direct lowering of block l (see BlockPlan::direct); ST_UNSUPPORTED with a
// message when the string is beyond its limits.
Status lower_direct(const Model& m, int ell, BlockPlan& bp, std::vector<int64_t>& ws_sizes,
                    std::string& err, int target_wg);
// Element offsets into a tensor with subscripts `subs` (row-major) of every
// multi-index over `letters` (row-major, last letter fastest); letters the
// tensor does not hold contribute nothing.
std::vector<uint32_t> offsets_in(const Model& m, const std::string& letters, const std::string& subs);
std::string describe_block(const Model& m, const BlockPlan& bp);

}  // namespace nnef
