/*
 * nnef.h - C ABI of libnnef: multiplicative-update (MU) sweeps for nonnegative
 * einsum factorizations on AMD Instinct MI355X (gfx950).
 *
 * The method is NNEinFact (Hood and Schein, "Near-Universal Multiplicative
 * Updates for Nonnegative Einsum Factorization"):
 *   - a model is an einsum string  i_1 r_1, ..., i_L r_L -> i_1 ... i_M
 *     (Sec. 2, eqs. 2.1-2.3): letters on the right are the observed modes of
 *     the data tensor Y, letters only on the left are contracted;
 *   - one sweep is the inner loop of Algorithm 1 (Sec. 3): for l = 1..L,
 *     rebuild Yhat, form the numerator and denominator einsums einstr_l with
 *     a(Y, Yhat) and b(Y, Yhat), and set
 *     Theta^(l) <- max(eps, Theta^(l) * g^{-1}(N_l / D_l))  (eq. 3.4);
 *   - the loss is the (alpha, beta)-divergence of App. B, in the paper's
 *     convention: KL = (1, 0), squared Euclidean = (1, 1), Itakura-Saito =
 *     (1, -1);
 *   - missing data are a binary mask (Sec. 6, "Experimental design"); the
 *     weights a, b are multiplied by the mask, so missing entries of Y are
 *     never read into arithmetic and may hold any bit pattern (NaN included).
 *
 * Memory and streams
 *   All tensor arguments are DEVICE pointers owned by the caller; the library
 *   never frees or reallocates them.  Layouts are dense row-major:
 *     Y, mask : axes in the order of the output letters of the model string;
 *     factor l: axes in the order of operand l's subscripts.
 *   Y is float32; mask is uint8 with 1 = observed, any other value = not used (NULL = fully
 *   observed).  Factors are float32 and are updated in place.
 *   `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Entry points only enqueue work on that stream, except where a comment
 *   says the call synchronises.  Calls that share a plan must not overlap:
 *   a plan owns one workspace.
 *
 * Errors
 *   Every entry point returns an nnef_status and never aborts.  A non-OK
 *   status leaves a message for nnef_last_error() (thread-local).  A status
 *   returned after work was enqueued (NNEF_E_DEVICE) means the stream's
 *   contents are undefined.
 */
#ifndef NNEF_H
#define NNEF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nnef_plan_s* nnef_plan_t;

typedef enum {
  NNEF_OK = 0,
  NNEF_E_PARSE = 1,            /* malformed model string                        */
  NNEF_E_SHAPE = 2,            /* sizes <= 0, count mismatch, tensor too large  */
  NNEF_E_LOSS_UNSUPPORTED = 3, /* alpha = 0 with beta != 1, or non-finite       */
  NNEF_E_ARG = 4,              /* NULL pointer, bad option, bad sweep count     */
  NNEF_E_DEVICE = 5,           /* a HIP call failed                             */
  NNEF_E_NOMEM = 6,            /* device workspace allocation failed            */
  NNEF_E_UNSUPPORTED = 7       /* a model the planner cannot lower              */
} nnef_status;

/* Input precision of the numerator and denominator contractions (the einsums
 * with a(Y,Yhat) and b(Y,Yhat) of Algorithm 1) on MFMA, with FP32
 * accumulation.  It applies to every block of the bilinear lowering (widths
 * up to 64; in batched plans to width 32 only); blocks on the direct lowering
 * (see nnef_plan), the reconstruction Yhat, the weights, the ratio N/D, the
 * power and the update, and the loss terms are float32; loss sums are
 * float64.  nnef_plan_describe reports the precision chosen for every block. */
/* NNEF_BF16_ALL / NNEF_FP16_ALL also round the inputs of the reconstruction
 * Yhat to BF16 / FP16 (FP32 accumulation) in the passes that compute no loss;
 * the passes that do (the first block of a sweep when a loss trace is
 * requested, nnef_loss, the accept test) keep an FP32 reconstruction, so every
 * reported loss has FP32 terms. */
typedef enum { NNEF_FP32 = 0, NNEF_BF16 = 1, NNEF_FP16 = 2, NNEF_BF16_ALL = 3, NNEF_FP16_ALL = 4 } nnef_prec;

/* Likelihood family.  NNEF_AB: the (alpha, beta)-divergence (App. B), with
 * the alpha, beta passed to nnef_plan.  The other decomposable likelihoods of
 * App. B ignore alpha and beta:
 *   NNEF_NEGBIN   negative binomial with dispersion phi = family_param > 0:
 *                 a = y/yhat, b = (phi + y)/(phi + yhat), update exponent 1;
 *                 loss (phi + y) log(phi + yhat) - y log yhat.
 *   NNEF_BINOMIAL binomial odds with n = family_param > 0 trials (n = 1:
 *                 Bernoulli), yhat the odds: a = y/yhat, b = n/(1 + yhat),
 *                 exponent 1; loss n log(1 + yhat) - y log yhat.
 *   NNEF_JS       Jensen-Shannon: a = log((y + yhat)/(2 yhat)), b = 1,
 *                 exponential update; loss (y log y + yhat log yhat)/2
 *                 - m log m, m = (y + yhat)/2.                               */
typedef enum { NNEF_AB = 0, NNEF_NEGBIN = 1, NNEF_BINOMIAL = 2, NNEF_JS = 3 } nnef_family;

typedef struct {
  double eps;          /* floor of eq. 3.1; default 1e-10                        */
  int    prec;         /* nnef_prec; default NNEF_FP32                           */
  int    deterministic;/* 1 (default): fixed-order reductions, bitwise repeatable */
  int    family;       /* nnef_family; default NNEF_AB                           */
  int    reserved[5];  /* must be zero                                           */
  double family_param; /* phi (NNEF_NEGBIN) or n (NNEF_BINOMIAL)                 */
} nnef_options;

/* Fill *opt with the defaults. */
void nnef_default_options(nnef_options* opt);

/*
 * nnef_plan - parse and lower a model string; allocate the plan's workspace.
 * Every block update is lowered one of two ways; neither stores the
 * reconstruction (one value per data entry) in device memory:
 *   bilinear  the observed modes split into rows P (holding operand l's
 *             modes) and columns Q with Yhat[p,q] = sum_k L[p,k] R[q,k] over a
 *             contraction width of at most 64, computed tile by tile on MFMA;
 *   direct    when no such split exists (the many-body models of Sec. 2, such
 *             as "ij,jk,ik->ijk", or CP-like ranks above 64): each data
 *             entry's reconstruction is summed over its latent combinations in
 *             registers (FP32 vector arithmetic).  Limits: at most 8 operands,
 *             at most 256 latent combinations in operand l, and at most 6144
 *             (other operands x all latent combinations).
 * nnef_plan_describe names the lowering of every block.
 *   model_str : e.g. "ir,jr,kr->ijk" or "ia,jab,kbc,lc->ijkl" (eq. 2.2).
 *   mode_sizes: n_modes sizes, in the order of the output letters.
 *   ranks     : n_ranks sizes of the contracted letters, in order of their
 *               first appearance on the left-hand side.
 *   alpha,beta: the (alpha, beta)-divergence of App. B.
 *   opt       : NULL for defaults.
 *   out       : receives the plan; free it with nnef_plan_destroy.
 * Rejects (status, nothing allocated):
 *   NNEF_E_PARSE  missing or repeated "->", a non-letter, an empty operand,
 *                 a letter repeated inside one operand or in the output, an
 *                 output letter used by no operand;
 *   NNEF_E_SHAPE  n_modes / n_ranks not matching the string, a size <= 0,
 *                 2^30 or more data entries;
 *   NNEF_E_LOSS_UNSUPPORTED  alpha = 0 with beta != 1 (App. B gives no
 *                 decomposition), non-finite alpha or beta;
 *   NNEF_E_UNSUPPORTED  a block with no bilinear split of width <= 64 that
 *                 is also beyond the limits of the direct lowering (the
 *                 message names the block and the limit).
 * Synchronises the device once (workspace set-up).
 */
nnef_status nnef_plan(const char* model_str, const int64_t* mode_sizes, int n_modes,
                      const int64_t* ranks, int n_ranks, double alpha, double beta,
                      const nnef_options* opt, nnef_plan_t* out);

void nnef_plan_destroy(nnef_plan_t plan);

/*
 * nnef_plan_dry - the planning of nnef_plan without any device work: parses,
 * validates and lowers the model and chooses the tiling, then writes the text
 * nnef_plan_describe would give (at most buf_len - 1 characters) and returns
 * its full length.  *status receives what nnef_plan would return (0 length
 * on error).  Needs no GPU.
 */
size_t nnef_plan_dry(const char* model_str, const int64_t* mode_sizes, int n_modes,
                     const int64_t* ranks, int n_ranks, double alpha, double beta,
                     const nnef_options* opt, nnef_status* status, char* buf, size_t buf_len);

/* Number of factors L, and the number of elements of factor l (0-based). */
int     nnef_plan_num_factors(nnef_plan_t plan);
int64_t nnef_plan_factor_numel(nnef_plan_t plan, int l);

/*
 * Human-readable description of the lowering chosen for every block
 * (split of the observed modes, contraction width, side operands, chain-back).
 * Returns the number of characters the full text needs (excluding the
 * terminator) and copies at most buf_len - 1 of them.
 */
size_t nnef_plan_describe(nnef_plan_t plan, char* buf, size_t buf_len);

/*
 * nnef_step - run n_sweeps sweeps of Algorithm 1 (Sec. 3) in place.
 *   factors   : host array of L device pointers (float32, layouts above).
 *   loss_trace: NULL, or a device array of n_sweeps doubles; entry s receives
 *               the masked loss sum_{observed} D(y, yhat) of the state at the
 *               START of sweep s (computed during that sweep's first block).
 * Enqueue only; no host synchronisation.  n_sweeps = 0 is a no-op.
 */
nnef_status nnef_step(nnef_plan_t plan, const float* Y, const uint8_t* mask,
                      float* const* factors, int n_sweeps, double* loss_trace,
                      void* stream);

/*
 * nnef_loss - masked loss sum_{observed} D_{alpha,beta}(y, yhat) (eq. 3.1,
 * App. B) of the given factors, reduced in float64.  Writes *loss_out (host).
 * Synchronises `stream`.
 */
nnef_status nnef_loss(nnef_plan_t plan, const float* Y, const uint8_t* mask,
                      const float* const* factors, double* loss_out, void* stream);

/* As nnef_loss, but writes the double to device memory and does not sync. */
nnef_status nnef_loss_device(nnef_plan_t plan, const float* Y, const uint8_t* mask,
                             const float* const* factors, double* d_loss_out,
                             void* stream);

/*
 * Kernel timing for measurement tools.  While enabled, nnef_step launches
 * every fused pass (the pass over Y of each block update) with a hipEvent
 * pair that the launch itself records at the kernel's start and end
 * (hipExtLaunchKernel), so the durations are those of the kernels.
 * nnef_plan_timing synchronises on those events and returns the number of
 * timed passes and their total duration in milliseconds, then forgets them.
 * Disabled by default.
 */
nnef_status nnef_plan_set_timing(nnef_plan_t plan, int enable);
nnef_status nnef_plan_timing(nnef_plan_t plan, int* n_passes, double* total_ms);

/* ------------------------------------------------------------------------
 * Learned extrapolation of the iterates.
 *
 * The paper has no learned component; this is the library's own addition on
 * top of Algorithm 1.  A small network (8 -> 128 -> 128 -> 1, ReLU, softplus
 * output s >= 0) reads eight features of every factor element's recent
 * multiplicative-update iterates theta_t, theta_{t-1}, theta_{t-2}:
 *   d1 = log(theta_t / theta_{t-1}), d2 = log(theta_{t-1} / theta_{t-2}),
 *   sigma = root mean square of d1 over the element's factor,
 *   x = [d1/sigma, d2/sigma, log10(sigma)/8, (log theta_t - log eps)/|log eps|,
 *        log10(max(rel_dec, 1e-30))/8, gamma, log2(K)/8, 1]
 * (rel_dec = (loss_{t-1} - loss_t)/loss_t; gamma = the update exponent, 1 for
 * the exponential update; K = the factor's last-axis size), and proposes
 * theta' = max(eps, theta_t exp(s d1)), positive by construction.
 *
 * Parameters are float32 in one flat vector of nnef_mlp_num_params() values:
 * W1 [8][128] (input-major), b1 [128], W2 [128][128] (W2[i][j] joins unit i
 * of layer 1 to unit j of layer 2), b2 [128], w3 [128], b3 [1].  The 128 x 128
 * layer runs on BF16 MFMA with float32 accumulation (forward and backward);
 * everything else is float32.
 * ------------------------------------------------------------------------ */
typedef struct nnef_mlp_s* nnef_mlp_t;

int nnef_mlp_num_params(void);

/* Create a network from initial parameters (device, float32, layout above;
 * copied, the caller keeps ownership).  Adam moments start at zero.  Syncs
 * the device. */
nnef_status nnef_mlp_create(const float* d_init_params, nnef_mlp_t* out);
void nnef_mlp_destroy(nnef_mlp_t mlp);

/* Copy the current float32 parameters to d_out (device). */
nnef_status nnef_mlp_params(nnef_mlp_t mlp, float* d_out, void* stream);

/* s[r] = softplus(network(X[r])) for n_rows rows X [n_rows][8] (device). */
nnef_status nnef_mlp_forward(nnef_mlp_t mlp, const float* X, int64_t n_rows, float* s_out,
                             void* stream);

/*
 * Training loss over n_rows rows: mean over rows of (s X[r][0] - tau[r])^2,
 * where rows are X[idx[r]], tau[idx[r]] (idx: device int32, or NULL for
 * r = 0..n_rows-1).  nnef_mlp_gradient writes the gradient (float32, the
 * parameter layout) to d_grad and the loss to *d_loss (device, may be NULL);
 * nnef_mlp_train_step instead applies one Adam step (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected; Kingma and Ba 2015) with learning rate lr.  The
 * gradient is summed over workgroups in a fixed order (deterministic).
 */
nnef_status nnef_mlp_gradient(nnef_mlp_t mlp, const float* X, const float* tau, const int32_t* idx,
                              int64_t n_rows, float* d_grad, double* d_loss, void* stream);
nnef_status nnef_mlp_train_step(nnef_mlp_t mlp, const float* X, const float* tau,
                                const int32_t* idx, int64_t n_rows, double lr, double* d_loss,
                                void* stream);

/*
 * nnef_mlp_gradient with no device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same rows, kernels and fixed-order sums
 * as nnef_mlp_gradient, so the same gradient (float32, parameter layout) in
 * d_grad and mean loss in *d_loss (device, may be NULL); the parameters are
 * read from d_params (kMlpParams = nnef_mlp_num_params() float32 values,
 * device, caller-owned) instead of an MLP handle.
 *
 * The per-workgroup partials live in one static device array of 18.2 MB
 * (256 partial slots; the library never launches more workgroups for this
 * call), held on every GPU the library runs on until the process ends.
 * Nothing in it needs clearing (every call writes each slot it reads).
 * Calls that overlap on one GPU (two streams, two threads) share the array
 * and race: serialise them.  Enqueue only; no host synchronisation.
 * Errors: NNEF_E_ARG for NULL pointers or n_rows <= 0, NNEF_E_SHAPE for
 * n_rows >= 2^31, NNEF_E_DEVICE if the array's address cannot be obtained.
 */
nnef_status nnef_mlp_gradient_noalloc(const float* d_params, const float* X, const float* tau,
                                      const int32_t* idx, int64_t n_rows, float* d_grad,
                                      double* d_loss, void* stream);

/*
 * Training rows from a multiplicative-update trajectory of `plan`'s model:
 * for every factor element (factors concatenated in operand order), the eight
 * features above into X [numel_total][8], and, when th_target (theta_{t+h})
 * is given, the target tau = clip(log(theta_{t+h}/theta_t)/sigma, -64, 64).
 * All arrays are host arrays of L device pointers / device buffers.
 * Returns NNEF_E_UNSUPPORTED for models with more than 8 factors.
 */
nnef_status nnef_learned_rows(nnef_plan_t plan, const float* const* th_t,
                              const float* const* th_tm1, const float* const* th_tm2,
                              const float* const* th_target, double rel_dec, float* X, float* tau,
                              void* stream);

/*
 * nnef_step - with proposals: n_sweeps sweeps of Algorithm 1; after every
 * sweep t that is a multiple of propose_every (>= 3) the network proposes
 * theta' from theta_t, theta_{t-1}, theta_{t-2}; the proposal replaces the
 * factors only if its loss (float32 terms, float64 sum, computed on the GPU)
 * is strictly lower than the loss of theta_t.  Otherwise the iterate is kept,
 * so the loss never increases.  loss_trace as in nnef_step (device, may be
 * NULL); *d_n_accepted (device int, may be NULL) is incremented per accepted
 * proposal.  Enqueue only.  Uses plan-owned buffers: calls on one plan must not
 * overlap.
 */
nnef_status nnef_step_learned(nnef_plan_t plan, nnef_mlp_t mlp, const float* Y,
                              const uint8_t* mask, float* const* factors, int n_sweeps,
                              int propose_every, double* loss_trace, int* d_n_accepted,
                              void* stream);

/* ------------------------------------------------------------------------
 * Batched plans: many independent problems, each with several restarts (sets
 * of factors sharing the problem's data), swept together.  Every block update
 * of every run goes into one persistent launch per kernel class (contraction
 * width, loss, layout), with the restarts of a problem interleaved so that they
 * read each data tile at about the same time; one sweep over all runs is
 * captured in a hipGraph and replayed.  Tile sizes per width class are chosen
 * by nnef_batch_autotune.  CP-like strings (such as "ir,jr,kr,lr->ijkl") take
 * the lowering without side operands; strings whose blocks need side operands
 * or chain-back contractions (Tucker eq. 2.4, tensor train eq. 2.6, custom
 * strings) run those contractions per run, in the captured sequence around the
 * batched passes, each run with its own copy of its problem's workspace.
 * Strings with no bilinear split (the direct lowering) return
 * NNEF_E_UNSUPPORTED.
 * ------------------------------------------------------------------------ */
typedef struct nnef_batch_s* nnef_batch_t;

typedef struct {
  const char* model_str;      /* as for nnef_plan */
  const int64_t* mode_sizes;
  int n_modes;
  const int64_t* ranks;
  int n_ranks;
  double alpha, beta;
  int n_restarts;             /* >= 1 factor sets sharing this problem's data */
  int masked;                 /* 1 if a mask will be passed for this problem */
} nnef_problem;

/* Plan n_problems problems (options as for nnef_plan, shared).  Runs are
 * numbered problem-major, restart-minor.  Allocates per-run partial buffers
 * and, for problems with side operands, a per-run workspace. */
nnef_status nnef_batch_plan(const nnef_problem* problems, int n_problems, const nnef_options* opt,
                            nnef_batch_t* out);
void nnef_batch_destroy(nnef_batch_t batch);
int nnef_batch_num_runs(nnef_batch_t batch);

/*
 * n_sweeps sweeps of Algorithm 1 for every run.
 *   Y        : host array of n_problems device pointers (float32 data).
 *   mask     : NULL, or host array of n_problems device pointers (uint8, NULL
 *              entries for fully observed problems).
 *   factors  : host array of device pointers, the L factor pointers of run 0,
 *              then of run 1, ... (layouts as for nnef_step), updated in place.
 *   loss_trace: NULL or device [n_sweeps][n_runs] doubles: the loss of every
 *              run at the start of each sweep.
 * The first call for a given set of pointers builds device argument tables and
 * captures the sweep in a graph (the call synchronises then); later calls with
 * the same pointers only replay it.  Enqueue only otherwise.
 */
nnef_status nnef_batch_step(nnef_batch_t batch, const float* const* Y, const uint8_t* const* mask,
                            float* const* factors, int n_sweeps, double* loss_trace, void* stream);

/*
 * Autotuner: times the fused passes of every block for each candidate tiling
 * (workgroups per run and pass, persistent grid size) on the given data, and
 * keeps the fastest per contraction-width class.  Factors are not modified.
 * Synchronises `stream`.
 */
nnef_status nnef_batch_autotune(nnef_batch_t batch, const float* const* Y, const uint8_t* const* mask,
                                float* const* factors, void* stream);

/* Lowering of every problem and the tiling chosen (as nnef_plan_describe). */
size_t nnef_batch_describe(nnef_batch_t batch, char* buf, size_t buf_len);

/* ------------------------------------------------------------------------
 * Splits and early stopping (Sec. 6, "Experimental design"; App. B,
 * "Stopping criterion").  A split mask holds one byte per entry: entries
 * equal to train_value (default 1) are fitted, val_value (default 2) marks
 * the validation set, any other value (0 missing, 3 heldout, ...) is unused.
 * The mask passed to nnef_step and nnef_loss follows the same rule: only
 * entries equal to 1 are observed.
 * ------------------------------------------------------------------------ */

/* Loss over the entries whose mask byte equals `value` (e.g. 2 validation,
 * 3 heldout), written to *d_loss (device); uses the plan's packing buffer. */
nnef_status nnef_loss_split(nnef_plan_t plan, const float* Y, const uint8_t* mask, int value,
                            const float* const* factors, double* d_loss, void* stream);

typedef enum { NNEF_STOP_MAX = 0, NNEF_STOP_TRAIN_TOL = 1, NNEF_STOP_VALIDATION = 2 } nnef_stop_reason;

typedef struct {
  int    max_sweeps;   /* sweep cap; default 5000                                        */
  int    patience;     /* stop when the validation loss rose this many sweeps in a row;
                          default 5, 0 disables                                          */
  double rel_tol;      /* stop when (L_{t-1} - L_t) / L_{t-1} < rel_tol for the training
                          loss; default 1e-6                                             */
  int    check_every;  /* losses are read back every check_every sweeps; 1 (default)
                          stops exactly at the first state that meets a rule, larger
                          values run up to check_every - 1 sweeps past it             */
  int    train_value;  /* mask byte of training entries; default 1                       */
  int    val_value;    /* mask byte of validation entries; default 2, 0 = none           */
} nnef_fit_options;

typedef struct {
  int    stop_sweep;   /* t of the state theta_t that met a rule (0 = the input state)  */
  int    sweeps_run;   /* sweeps applied to the factors (>= stop_sweep)                  */
  int    reason;       /* nnef_stop_reason; checked in the order validation, training, cap */
  double train_loss;   /* losses of theta_{stop_sweep}                                   */
  double val_loss;
} nnef_fit_result;

void nnef_default_fit_options(nnef_fit_options* opt);

/*
 * Fit with the paper's stopping rules: for t = 0, 1, ... the training and
 * validation losses of theta_t are taken (float32 terms, float64 sums), the
 * rules are checked, and otherwise one sweep is run on the training entries.
 * train_trace / val_trace (device, may be NULL) receive the losses of
 * theta_0 .. theta_{stop_sweep}; they need room for max_sweeps + 1 doubles.
 * One packed copy of the data (the plan's packing buffer) holds both splits,
 * and the two losses of theta_t come from the first fused pass of sweep t + 1
 * (no separate loss passes); the factors of the last state of every chunk of
 * check_every states are kept on the device, so a stop there returns exactly
 * that state.  Allocates those small buffers for the call and synchronises the
 * stream once per chunk.
 */
nnef_status nnef_fit(nnef_plan_t plan, const float* Y, const uint8_t* mask, float* const* factors,
                     const nnef_fit_options* opt, nnef_fit_result* res, double* train_trace,
                     double* val_trace, void* stream);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char* nnef_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NNEF_H */
