// Internal declarations shared by the planner (host C++) and the kernels (HIP).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace nnef {

// Events (hipEvent_t) that the next fused or direct pass launch records at the
// start and the end of the kernel itself (hipExtLaunchKernel), for per-pass
// durations without the cost of separate event records; both null: an
// ordinary launch.  Set by the host around one launch when timing is on.
struct PassEvents {
  void* start = nullptr;
  void* stop = nullptr;
};
extern thread_local PassEvents g_pass_events;

constexpr int kMaxPieces = 3;     // factors multiplied together to form one side row
constexpr int kMaxEinsumIn = 4;   // inputs of one einsum step
constexpr int kMaxEinsumLetters = 10;
constexpr int kMaxDirectOps = 7;   // operands besides l on the direct lowering
constexpr int kDirectKPT = 16;     // latent combinations of operand l per thread
constexpr int kDirectMaxK = 256;   // latent combinations of operand l (16 threads x 16)
constexpr int kDirectMaxLat = 6144;  // table entries (n_ops x K x KS) staged in LDS

// Weight functions a, b (App. B), specialised by (alpha, beta).
enum WeightKind : int {
  WK_KL = 0,    // (1, 0):   a = y/yh,              b = 1
  WK_EUC = 1,   // (1, 1):   a = y,                 b = yh
  WK_SQRT = 2,  // (.5, 1):  a = sqrt(y),           b = sqrt(yh)
  WK_IS = 3,    // (1, -1):  a = y/yh^2,            b = 1/yh
  WK_GEN = 4,   // alpha!=0: a = y^al yh^(be-1),    b = yh^(al+be-1)
  WK_RKL = 5,   // (0, 1):   a = log(y/yh),         b = 1
  WK_FAM = 6,   // other families (LossKind selects): negative binomial,
                // binomial odds, Jensen-Shannon
  WK_COUNT = 7
};

// g^{-1} of App. B: r^gamma with the exponent specialised, or exp(r).
enum UpdateKind : int { UP_ONE = 0, UP_SQR = 1, UP_SQRT = 2, UP_POW = 3, UP_EXP = 4 };

// Case of the (alpha, beta)-divergence definition (App. B), plus closed forms.
enum LossKind : int {
  LK_GENERIC = 0, LK_BETA0 = 1, LK_AMB = 2, LK_ALPHA0 = 3, LK_ZERO = 4,
  LK_KL = 5, LK_EUC = 6, LK_IS = 7, LK_SQRT = 8,
  LK_NB = 9, LK_BIN = 10, LK_JS = 11  // with WK_FAM
};

struct LossSpec {
  double alpha = 1, beta = 0, gamma = 1;
  double fparam = 0;           // negative binomial phi, binomial n
  int wk = WK_KL, upd = UP_ONE, lk = LK_KL;
  bool b_is_one() const { return wk == WK_KL || wk == WK_RKL || (wk == WK_FAM && lk == LK_JS); }
};

// ---------------------------------------------------------------------------
// Kernel argument blocks (plain data, passed by value).
// ---------------------------------------------------------------------------
// Fused pass: for a split of the observed modes into P (rows) and Q (columns),
//   yhat[p,q] = sum_k L[p,k] R[q,k]
//   Wa = m * a(y, yhat), Wb = m * b(y, yhat)
//   N[p,k] = sum_q Wa[p,q] R[q,k],  D[p,k] = sum_q Wb[p,q] R[q,k]
// A column q is a pair (qo, qi): qi runs over the last column-side mode and qo
// over the others, q = qo * nqi + qi.  One step covers 16 consecutive qi at one
// qo, so every per-qo quantity is uniform across a wave.  The column side is
//   R[q,k] = inner[(in_base[qo] + qi * in_stride) * ld_in + k]
//            * prod_m outer_m[orow_m[qo] * ld_out_m + k],
// either a product of factors (CP-like models) or one materialised buffer.
// One workgroup = 4 waves on one panel of rows, each over its own run of
// steps; it writes one partial N, D of shape [nP][KP] at slot `chunk`.
struct FusedArgs {
  const float* Y;              // data; with `masked`, a missing entry holds -1
  int masked;                  // 0: every entry observed
  const uint32_t* p_off;       // [nP] Y offset of row p
  const float* L;              // L[p*ldL + k], k < K
  int ldL;
  int K;                       // true contraction width (<= KP)
  int nP;
  int nqo, nqi, nqis;          // nqis = ceil(nqi / 16)
  int qi_ystride;              // Y stride of the qi mode
  const uint32_t* qo_yoff;     // [nqo] Y offset of qo
  const float* inner;
  int ld_in, in_stride;
  const uint32_t* in_base;     // [nqo] or nullptr (= 0)
  int nouter;
  const float* outer[2];
  int ld_out[2];
  const uint32_t* orow[2];     // [nqo]
  int64_t n_steps;             // nqo * nqis
  int n_panels;
  int steps_per_wave;
  int n_chunks;                // partial slots
  int n_wg;                    // grid size
  int xcd_remap;               // 1: consecutive work items share an XCD
  int wave_rows;               // width 32: each wave its own 32 rows, all waves the same steps
  float* partN;                // [n_chunks][nP][KP]
  float* partD;                // [n_chunks][nP][KP] (unused when no_d)
  double* loss_part;           // [n_wg] (loss passes)
  double* vloss_part;          // [n_wg] or null: also the loss of the validation entries (split pack)
  int no_d;                    // D is a closed form (b = 1, no mask): skip it
  float alpha, beta;           // for WK_GEN and the generic loss
  float ab_inv, apb_inv;       // 1/(alpha*beta), 1/(alpha+beta)
  int lk;                      // LossKind (generic weights and WK_FAM)
  float fparam;                // WK_FAM: negative binomial phi, binomial n
  int full;                    // no ragged edges: K = KP, nqi % 16 = 0, nP % rows = 0
  int prec;                    // contraction inputs: 0 FP32, 1 BF16, 2 FP16 (width 32)
};

// Direct pass (strings with no bilinear split): for every observed entry
// (p, q) and latent combination r of operand l,
//   c[r] = sum_s prod_j op_j[opp_j[p] + opq_j[q] + oplat_j[r * KS + s]]
//   yhat = sum_r theta[thp[p] + thr[r]] c[r]
//   N[p, r] += Wa c[r],  D[p, r] += Wb c[r]
// G threads share an entry (each a strided subset of r, combined with a
// butterfly); a workgroup of 256 threads covers rows_per_wg rows x qlanes
// entry groups per row over one chunk of columns and writes one partial
// [nP][K] at slot `chunk` (the fused pass's partial layout with KP = K).
struct DirectArgs {
  const float* Y;              // data; with `masked`, a missing entry holds -1
  int masked;
  int nP, nQ;
  const uint32_t* yp;          // [nP] Y offset of row p
  const uint32_t* yq;          // [nQ] Y offset of column q
  const float* theta;          // operand l
  const uint32_t* thp;         // [nP]
  const uint32_t* thr;         // [K]
  int K, KS, G;
  int n_ops;
  const float* op[kMaxDirectOps];
  const uint32_t* opp[kMaxDirectOps];    // [nP]
  const uint32_t* opq[kMaxDirectOps];    // [nQ]
  const uint32_t* oplat[kMaxDirectOps];  // [K * KS]
  int rows_per_wg, qlanes, q_per_chunk, n_chunks, n_panels;
  float* partN;                // [n_chunks][nP][K]
  float* partD;
  double* loss_part;           // [grid]
  double* vloss_part;          // [grid] or null (validation entries of a split pack)
  float alpha, beta, ab_inv, apb_inv;
  int lk;
  float fparam;
};
int launch_direct(const DirectArgs& a, int wk, int mode, void* stream);

// Reduce the partials of a fused pass and apply the update (or store N_L/D_L).
struct UpdateArgs {
  const float* partN; const float* partD;
  int n_chunks, nP, K, KP;
  int no_d;
  // closed-form D (no_d): D[p,k] = prod_m colsum(piece_m)[k] (column-side pieces)
  int npieces;
  const float* piece[kMaxPieces];
  int ldpiece[kMaxPieces];
  int64_t nrows[kMaxPieces];
  // direct update target (theta = L itself) or N_L/D_L output
  float* theta; int ldT;       // theta[p*ldT + k]
  float* NL; float* DL;        // [nP][K] when chaining back (theta == nullptr)
  int upd; float gamma; float eps;
  // loss finalisation (first block of a sweep); vloss: validation entries of a split pack
  const double* loss_part; int n_loss_part; double* loss_out;
  const double* vloss_part; double* vloss_out;
  float* dcol;                 // [K] closed-form D scratch (no_d)
};

// Generic n-ary contraction out[o] = sum_c prod_i in_i[...] over explicit strides.
struct EinsumArgs {
  int n_in;
  const float* in[kMaxEinsumIn];
  int n_out;                                   // number of output letters
  int n_sum;                                   // number of summed letters
  int64_t out_size[kMaxEinsumLetters];
  int64_t out_stride[kMaxEinsumLetters];       // output strides (elements)
  int64_t sum_size[kMaxEinsumLetters];
  int64_t in_out_stride[kMaxEinsumIn][kMaxEinsumLetters];
  int64_t in_sum_stride[kMaxEinsumIn][kMaxEinsumLetters];
  int64_t n_out_total;
  float* out;
};

// Elementwise update from full-size N, D (after a chain-back).
struct ApplyArgs {
  float* theta; const float* N; const float* D; int64_t n;
  int upd; float gamma; float eps;
};

// Launchers (kernels.hip).  Return 0 or a hipError_t value.
// mode: 0 = N, D only; 1 = N, D and the loss; 2 = the loss only
int launch_fused(const FusedArgs& a, int KP, int wk, bool vecq, int mode, void* stream);

// Persistent launch over many problems ("runs"): work item = (run, workgroup
// index within that run's grid); args[run] holds the run's FusedArgs.
struct WorkItem {
  int run, blk;
};
struct BatchedLaunch {
  const FusedArgs* args;   // device
  const WorkItem* work;    // device
  int n_work, grid;
  int KP, wk, mode, prec;  // mode 0: N/D, 1: N/D + loss
  bool vecq, full;
};
int launch_fused_batched(const BatchedLaunch& L, void* stream);
int launch_update(const UpdateArgs& a, float* dcol, void* stream);  // dcol: [K] scratch for a closed-form D
// Many runs: colsum over runs[0..n_colsum) (one workgroup each, those with
// no_d), then the update over the work items (run, 64-output block).
int launch_update_batched(const UpdateArgs* args, const int* colsum_runs, int n_colsum,
                          const WorkItem* work, int n_work, int grid, void* stream);
// second (may be null): a contraction of the same shape and strides, other
// pointers; both are evaluated (in one launch where the form allows)
int launch_einsum(const EinsumArgs& a, void* stream, const EinsumArgs* second = nullptr);
int launch_apply(const ApplyArgs& a, void* stream);
int launch_loss_final(const double* part, int n, double* out, void* stream);
int launch_zero(float* p, int64_t n, void* stream);
int launch_copy_f64(double* dst, const double* src, int n, void* stream);
// Packed data: Yp[i] = Y[i] where mask[i] == value (observed; data are
// nonnegative, so the sign bit is clear), -Y[i] with the sign bit set (-0 for
// a zero) where mask[i] == vvalue (a validation entry of a split), -inf
// elsewhere.  vvalue outside 0..255: no validation entries.
int launch_pack(const float* Y, const uint8_t* M, float* Yp, int64_t n, void* stream, int value = 1,
                int vvalue = 256);

// ---- learned extrapolation (a small MLP over per-element trajectory features)
constexpr int kMlpIn = 8, kMlpWidth = 128;
constexpr int kMlpOffW1 = 0, kMlpOffB1 = kMlpIn * kMlpWidth, kMlpOffW2 = kMlpOffB1 + kMlpWidth,
              kMlpOffB2 = kMlpOffW2 + kMlpWidth * kMlpWidth, kMlpOffW3 = kMlpOffB2 + kMlpWidth,
              kMlpOffB3 = kMlpOffW3 + kMlpWidth, kMlpParams = kMlpOffB3 + 1;
constexpr int kMaxLearnFactors = 8;

// Per-element features of the factors' recent iterates (theta_t, theta_{t-1},
// theta_{t-2}); the factors are concatenated in operand order.
struct FeatArgs {
  int n_fac;
  int64_t off[kMaxLearnFactors + 1];
  const float* th[kMaxLearnFactors];
  const float* tm1[kMaxLearnFactors];
  const float* tm2[kMaxLearnFactors];
  const float* tth[kMaxLearnFactors];   // theta_{t+h} (training targets) or null
  float* cand[kMaxLearnFactors];        // proposal output
  float* dst[kMaxLearnFactors];         // accept: factors to overwrite
  float logK8[kMaxLearnFactors];        // log2(contraction width) / 8
  const double* sigma;                  // [n_fac]
  const double* loss_prev;              // loss at t-1 (device) or null: use rel_dec
  const double* loss_cur;               // loss at t (device)
  double rel_dec;
  float gamma, eps, log_eps, inv_abs_log_eps;
};

struct MlpArgs {
  const float* params;   // FP32 master parameters [kMlpParams]
  int64_t n_rows;
  const float* X;        // rows [n_rows or max idx + 1, 8]
  const float* tau;      // training targets
  const int32_t* idx;    // optional row indices into X / tau
  float* s_out;          // forward: step multipliers
  float inv_n;           // 1 / n_rows (mean loss)
  float* gpart;          // gradient partials [grid, kMlpParams]
  double* lpart;         // loss partials [grid]
  FeatArgs f;            // proposal mode
};

int mlp_grid(int64_t n_rows);
int launch_mlp(const MlpArgs& a, int mode, int grid, void* stream);  // 0 forward, 1 gradient, 2 proposal
int launch_mlp_reduce(const float* gpart, const double* lpart, int grid, float inv_n, float* grad_out,
                      double* loss_out, float* params, float* m, float* v, float lr, float b1, float b2,
                      float eps, float bc1, float bc2, int adam, void* stream);
int launch_sigma(const FeatArgs& f, void* stream);
int launch_rows(const FeatArgs& f, float* X, float* tau, void* stream);
int launch_accept(const FeatArgs& f, const double* loss_cand, const double* loss_cur, int* n_acc,
                  void* stream);
int launch_copy_factors(const FeatArgs& f, void* stream);  // tm1[k] <- th[k]

}  // namespace nnef
