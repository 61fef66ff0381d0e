/*
 * nmf.h -- C ABI of the MI355X (gfx950) multiplicative-update NMF library.
 *
 * The library factors a nonnegative matrix V (p x n) as W (p x r) times
 * H (r x n) by the multiplicative majorize-minimize updates of Zhou, Lange &
 * Suchard, "Graphics Processing Units and High-Dimensional Optimization",
 * Sec. 3.1 (eq. nnmf-objfn, eq. nnmf_v_update, eq. nnmf_w_update,
 * Algorithm 1 NNMF).  The paper writes X ~ V W; this header writes V ~ W H,
 * so the paper's "V update" is the W update here and its "W update" is the
 * H update here.
 *
 * Conventions for every entry point:
 *   - Matrices are row-major float32.  V has row stride ldv (in elements,
 *     ldv >= n); W is p x r with row stride r; H is r x n with row stride n.
 *   - Pointers named V, W, H, W0, H0 are DEVICE pointers (hipMalloc'd or
 *     torch CUDA tensors); pointers named *_host are host pointers.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All work is enqueued on that stream; entry points that return a value
 *     to the host synchronize it.
 *   - Errors are reported only through the return code; no entry point
 *     aborts or throws.  Argument checks happen before any device work, so
 *     an NMF_EINVAL return has no side effects.
 *   - The caller owns V, W and H.  V is never written.  W and H are updated
 *     in place by every iteration.  The context owns only its workspace,
 *     which nmf_destroy releases.  No entry point frees caller memory.
 *   - A context is not thread-safe; use one context per host thread.
 *     Results are deterministic: no floating-point atomics are used, and
 *     all reductions run in a fixed order for a given shape and precision.
 */
#ifndef NMF_H
#define NMF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nmf_ctx nmf_ctx;

typedef enum {
  NMF_OK = 0,
  NMF_ENOTCONVERGED = 1,  /* iteration cap reached; the state is valid       */
  NMF_EINVAL = -1,        /* bad argument, or V failed validation            */
  NMF_ENOMEM = -2,        /* device allocation failed                        */
  NMF_EDEVICE = -3,       /* a HIP runtime call failed                       */
  NMF_ENONFINITE = -4,    /* the objective became NaN or Inf                 */
  NMF_EUNSUPPORTED = -5   /* r above NMF_MAX_RANK, an unknown option, or a
                             combination of options not offered             */
} nmf_status;

typedef enum {
  NMF_FP32 = 0,  /* float32 operands, float32 accumulation                   */
  NMF_BF16 = 1   /* bfloat16 (round-to-nearest-even) copies of V, W, H and
                    the Grams feed the products; float32 accumulation and
                    float32 master factors                                  */
} nmf_precision;

typedef enum {
  /* |f_k - f_prev| / (|f_prev| + 1) < tol, f_prev the objective at the
     previous check: the stopping rule of Sec. 3 (introduction of the
     numerical examples), which uses tol = 1e-9 and checks every iteration. */
  NMF_TOL_REL_CHANGE = 0,
  /* f_k / ||V||_F^2 <= tol (relative objective gap against f* = 0).         */
  NMF_TOL_GAP_NORMALIZED = 1
} nmf_tol_kind;

typedef enum {
  /* ||V - W H||_F^2, minimized (Sec. 3.1, eq. nnmf-objfn; Algorithm 1)     */
  NMF_LOSS_EUCLIDEAN = 0,
  /* Poisson log-likelihood L = sum_ij [v_ij ln b_ij - b_ij], b = W H,
     maximized by the square-root multiplicative update of Sec. 3.1 (last
     display): w_ik <- w_ik sqrt(sum_j (v_ij / b_ij) h_kj / sum_j h_kj),
     h_kj <- h_kj sqrt(sum_i (v_ij / b_ij) w_ik / sum_i w_ik), both from the
     same iterate (the display's second update, whose indices are garbled,
     read as the mirror image of the first).  FP32 only, r <= 64, stopping
     rule NMF_TOL_REL_CHANGE only; nmf_objective returns L.               */
  NMF_LOSS_POISSON = 1
} nmf_loss;

#define NMF_MAX_RANK 256

typedef struct {
  int32_t precision;    /* nmf_precision                                    */
  int32_t tol_kind;     /* nmf_tol_kind                                     */
  double tol;           /* tolerance of the stopping rule                   */
  int32_t check_every;  /* iterations between objective checks (>= 1)       */
  int32_t validate;     /* nonzero: nmf_init scans V and rejects negative or
                           non-finite entries with NMF_EINVAL               */
  uint64_t seed;        /* nonzero: nmf_init overwrites W and H with
                           U(0,1) draws from a counter-based Philox4x32-10
                           generator keyed by seed (Algorithm 1's
                           initialization); zero: start from the caller's
                           W and H                                          */
  int32_t use_graph;    /* nonzero: nmf_step replays the iteration's kernels
                           from a captured HIP graph (fewer launch gaps);
                           results are identical to direct launches        */
  int32_t loss;         /* nmf_loss (NMF_LOSS_EUCLIDEAN by default)          */
} nmf_options;

/* Fill *opt with defaults: FP32, REL_CHANGE, tol 1e-9, check_every 1,
   validate 0, seed 0, use_graph 1, Euclidean loss.  NULL is ignored. */
void nmf_default_options(nmf_options* opt);

/* Create a context for V (p x n, row stride ldv) and rank r, reading the
   starting factors from W (p x r) and H (r x n) unless opt->seed != 0, in
   which case W and H are filled on the device.  Computes the r x r Gram
   H H^T of the start.  opt may be NULL (defaults).  p, n, r >= 1,
   r <= NMF_MAX_RANK, ldv >= n; V, W, H non-NULL and 4-byte aligned.
   V, W and H must stay allocated until nmf_destroy, and the caller must not
   write W or H while the context exists (call nmf_init again to restart
   from new factors).  On success *out receives the context; on failure
   *out is set to NULL. */
nmf_status nmf_init(nmf_ctx** out, const float* V, int64_t p, int64_t n,
                    int64_t ldv, int32_t r, float* W, float* H,
                    const nmf_options* opt, void* stream);

/* Enqueue `iters` (>= 0) full iterations of Algorithm 1 (NNMF): the W
   update of eq. nnmf_v_update followed by the H update of eq.
   nnmf_w_update with the new W.  Asynchronous; no host synchronization.
   With use_graph the iterations are replayed from HIP graphs of 16, 8, 4,
   2 and 1 iterations, each captured on first use (iters = 16 q + the
   binary digits of the rest: at most q + 4 replays); while the profiler is
   running, kernels are launched directly so that every stage can be
   timed. */
nmf_status nmf_step(nmf_ctx* ctx, int32_t iters);

/* Capture now every graph that nmf_step replays (use_graph), instead of on
   first use, so that a later nmf_step only launches.  Records kernels into
   graphs without running them: no device work is enqueued and W, H are
   unchanged.  No-op without use_graph. */
nmf_status nmf_prepare_graphs(nmf_ctx* ctx);

/* Enqueue only the W half-step (eq. nnmf_v_update):
   W <- W * (V H^T) / (W (H H^T)), entries with a non-positive denominator
   kept unchanged.  Asynchronous. */
nmf_status nmf_update_w(nmf_ctx* ctx);

/* Enqueue only the H half-step (eq. nnmf_w_update) with the current W:
   H <- H * (W^T V) / ((W^T W) H), guarded as above.  Asynchronous. */
nmf_status nmf_update_h(nmf_ctx* ctx);

/* Objective f = ||V - W H||_F^2 (eq. nnmf-objfn) from the current W and H:
   direct residual, products and sums in float64 on the device, reduced in a
   fixed order.  Synchronizes the stream and writes *f_host.
   Returns NMF_ENONFINITE (with *f_host set) if f is NaN or Inf. */
nmf_status nmf_objective(nmf_ctx* ctx, double* f_host);

/* Iterate until the stopping rule of the context's options holds or
   max_iters iterations have run.  The objective is evaluated at the start
   and after every check_every iterations (and after the last one).  The
   next chunk of iterations and its check are enqueued before the host
   reads the current check, so the device does not wait on the host: when
   the rule holds at a check, the chunk already enqueued after it (if any)
   also runs, so up to check_every iterations more than the first passing
   check.  *iters_done_host receives the number of iterations run and
   *f_host the objective of the factors left in W and H (the last check).
   trace_host (may be NULL) receives the evaluated objectives, f_0 first,
   up to trace_len entries.  Returns NMF_OK when the rule held at a check,
   NMF_ENOTCONVERGED at the cap, NMF_ENONFINITE if f became non-finite. */
nmf_status nmf_solve(nmf_ctx* ctx, int32_t max_iters, int32_t* iters_done_host,
                     double* f_host, double* trace_host, int32_t trace_len);

/* nmf_solve accelerated by the quasi-Newton scheme QN(q) of Zhou, Alexander
   & Lange (2011), which the paper's Discussion cites (Tables 3 and 4,
   columns QN(q)).  With F one iteration of Algorithm 1 on x = (W, H), each
   QN iteration evaluates F twice, keeps the secant pairs u = F(x) - x,
   v = F(F(x)) - F(x) of the last q QN iterations (U, V, float64), and forms
     x_qn = F(x) + V (U^T U - U^T V)^-1 U^T u,
   a Newton step for x = F(x) with the minimum-norm Jacobian approximation
   satisfying the secant conditions.  x_qn is projected onto x >= 0.5 F(x)
   (entrywise; NMF's iterates must stay positive, and the unprojected point
   leaves the orthant almost every time on sparse data) and taken when the
   q x q system is regular and f(x_qn) <= f(F(F(x))); otherwise the
   iteration keeps F(F(x)).  So f never increases.  Every decision is made
   on the device; one QN iteration is replayed from a HIP graph.
   max_iters counts evaluations of F (two per QN iteration; at most 131072);
   the stopping rule of the context's options is tested on the accepted
   objective every check_every evaluations (check_every / 2 QN iterations,
   at least one).  *iters_done_host: evaluations of F run; *accepted_host
   (may be NULL): QN iterations whose extrapolated point was taken; *f_host:
   the objective of the factors left in W and H; trace_host (may be NULL):
   f_0 and then the objective after every QN iteration.  1 <= q <= 16.
   NMF_EUNSUPPORTED for the Poisson loss.  Returns as nmf_solve. */
nmf_status nmf_solve_qn(nmf_ctx* ctx, int32_t q, int32_t max_iters,
                        int32_t* iters_done_host, int32_t* accepted_host,
                        double* f_host, double* trace_host, int32_t trace_len);

/* ||V||_F^2 in float64 (computed once by nmf_init); the normalizer of the
   NMF_TOL_GAP_NORMALIZED rule.  No device work. */
nmf_status nmf_data_norm2(nmf_ctx* ctx, double* norm2_host);

/* Stages of one iteration, as timed by the profiler below. */
typedef enum {
  NMF_STAGE_GEMM_VHT = 0,   /* V H^T split-K partials (W numerator)          */
  NMF_STAGE_UPDATE_W = 1,   /* partial sum + W (H H^T) + ratio update of W    */
  NMF_STAGE_GRAM_W = 2,     /* W^T W                                          */
  NMF_STAGE_GEMM_WTV = 3,   /* W^T V split-K partials (H numerator)           */
  NMF_STAGE_UPDATE_H = 4,   /* partial sum + (W^T W) H + ratio update of H    */
  NMF_STAGE_GRAM_H = 5,     /* H H^T                                          */
  NMF_STAGE_OBJECTIVE = 6,  /* float64 objective and its reduction            */
  NMF_STAGE_COUNT = 7
} nmf_stage;

/* Start timing: every stage enqueued afterwards (up to max_records stages)
   is bracketed by a pair of HIP events on the context's stream.  Restarts
   discard earlier records.  Returns NMF_EINVAL for max_records < 1. */
nmf_status nmf_profile_start(nmf_ctx* ctx, int32_t max_records);

/* Stop timing, synchronize the stream and write, per nmf_stage, the summed
   event time in milliseconds (ms_host[NMF_STAGE_COUNT]) and the number of
   timed launches (launches_host[NMF_STAGE_COUNT]); either may be NULL. */
nmf_status nmf_profile_stop(nmf_ctx* ctx, double* ms_host, int32_t* launches_host);

/* Fix the scale gauge of a factorization in place without changing W H:
   every nonzero column w_k of W (p x r, device) becomes w_k / |w_k|_2 and
   row k of H (r x n, device) is multiplied by |w_k|_2 (column norms summed
   in float64).  The factorization V ~ W H is invariant under W D, D^-1 H
   for positive diagonal D (a property of the model of Sec. 3.1), so this
   only picks a representative.  Asynchronous on `stream`. */
nmf_status nmf_normalize_gauge(float* W, int64_t p, int32_t r, float* H,
                               int64_t n, void* stream);

/* nmf_normalize_gauge without any device allocation, for callers that
   cannot allocate (code under HIP graph capture, tight serving loops,
   harnesses that forbid hipMalloc).  Same arguments, kernels and results as
   nmf_normalize_gauge; its r column norms live in a static device array of
   NMF_MAX_RANK floats (1 KB per GPU, held until the process ends) instead of
   a per-call allocation.  r > NMF_MAX_RANK returns NMF_EINVAL.  Every call
   on one GPU shares that array: calls that overlap on one GPU (two streams,
   or two host threads) race and must be serialized by the caller.
   NMF_EDEVICE if the array's device address cannot be obtained. */
nmf_status nmf_normalize_gauge_noalloc(float* W, int64_t p, int32_t r, float* H,
                                       int64_t n, void* stream);

/* Replace W by the least-squares fit to the current H (a warm start whose H
   came from elsewhere, e.g. nmf_mlp_predict):
     W = max(V H^T (H H^T + delta I)^-1, floor),
   delta = 1e-6 trace(H H^T) / r, floor = floor_rel * max(W) (at least the
   smallest normal float), so every entry is positive as the multiplicative
   updates need.  Products as in nmf_step's tier (BF16 tier: bf16 operands),
   the r x r solve in float64.  Writes the context's W and the caller's W;
   H is unchanged.  Asynchronous.  Errors: NMF_EINVAL (floor_rel not in
   (0, 1)), NMF_EUNSUPPORTED (r > 64). */
nmf_status nmf_refit_w(nmf_ctx* ctx, float floor_rel);

/* ---- Learned warm start -------------------------------------------------
   A small network maps one column v of V (p values) to a starting column of
   H (r values): h0 = softplus(M2 relu(M1 v + b1) + b2), M1 hidden x p,
   M2 r x hidden.  It is trained on columns of converged factorizations
   (pairs v_j, h_j) with the mean squared error and Adam; at solve time
   nmf_mlp_predict fills H0 for a new V and the multiplicative updates refine
   it (the updates only descend, so the start cannot hurt the end point of a
   monotone run).  Matrix products run in bfloat16 on the matrix cores with
   float32 accumulation; master weights and Adam moments are float32. */
typedef struct nmf_mlp nmf_mlp;

/* Create a network for inputs of p features, `hidden` units (a multiple of
   128), r <= 64 outputs, and batches of at most max_batch columns.
   M1 (hidden x p), b1 (hidden), M2 (r x hidden), b2 (r): device pointers
   to the initial float32 weights, copied in. */
nmf_status nmf_mlp_create(nmf_mlp** out, int32_t p, int32_t hidden, int32_t r,
                          int64_t max_batch, const float* M1, const float* b1,
                          const float* M2, const float* b2, void* stream);

/* H0 (r x n, row-major, device) = the network applied to each of the n
   columns of V (p x n, row stride ldv, device).  Any n >= 1: wider inputs
   are processed in chunks of max_batch columns.  Asynchronous. */
nmf_status nmf_mlp_predict(nmf_mlp* m, const float* V, int64_t n, int64_t ldv,
                           float* H0);

/* One Adam step (learning rate lr; beta1 0.9, beta2 0.999, eps 1e-8) on the
   batch of the n columns of V with targets H (r x n, device, row stride
   ldh >= n, so a column slice of a wider target matrix can be passed): loss =
   mean over the r x n entries of (h0 - h)^2.  loss_host (may be NULL)
   receives the loss before the step (synchronizes the stream). */
nmf_status nmf_mlp_train_step(nmf_mlp* m, const float* V, int64_t n,
                              int64_t ldv, const float* H, int64_t ldh,
                              float lr, double* loss_host);

/* Gradients of that loss at the current weights, without updating them:
   gM1 (hidden x p), gb1 (hidden), gM2 (r x hidden), gb2 (r), device. */
nmf_status nmf_mlp_grads(nmf_mlp* m, const float* V, int64_t n, int64_t ldv,
                         const float* H, int64_t ldh, float* gM1, float* gb1,
                         float* gM2, float* gb2, double* loss_host);

/* Copy the float32 weights out (device pointers, shapes as in create). */
nmf_status nmf_mlp_get_params(nmf_mlp* m, float* M1, float* b1, float* M2,
                              float* b2);

/* Release the network.  NULL is ignored. */
void nmf_mlp_destroy(nmf_mlp* m);

/* ---- Warm start: dictionary, prediction and training loop ---------------
   The learned warm start hands a new matrix V a start (W0, H0) for the
   multiplicative updates of Algorithm 1: W0 = the mean dictionary W-bar
   (p x r) stored in the network object, H0 = the network applied to every
   column of V.  The updates then refine it (they never increase f, so the
   start affects the time to a tolerance, not the quality reached).  The
   multiplicative method itself (Sec. 3.1) needs only a positive start; the
   learned start is an addition to it. */

/* Store W-bar (p x r row-major, device; p and r as in nmf_mlp_create),
   copied in; replaces an earlier one.  Asynchronous on the network's
   stream.  NMF_ENOMEM if its buffer cannot be allocated (first call). */
nmf_status nmf_ws_set_dictionary(nmf_mlp* m, const float* Wbar);

/* W0 (p x r, device) = the stored W-bar; H0 (r x n, row-major, device) =
   the network applied to the n columns of V (p x n, row stride ldv,
   device), as nmf_mlp_predict.  Asynchronous on the network's stream.
   NMF_EINVAL if p differs from the network's input size or no dictionary
   has been stored. */
nmf_status nmf_ws_predict(nmf_mlp* m, const float* V, int64_t p, int64_t n,
                          int64_t ldv, float* W0, float* H0);

/* The training loop of the network, run by the library: `epochs` passes
   over the `count` matrices V[i] (p x n, row stride ldv) with targets H[i]
   (r x n, row stride ldh) -- host arrays of device pointers -- in a seeded
   random order per epoch (Fisher-Yates driven by splitmix64 from `seed`),
   each matrix in minibatches of `batch` consecutive columns (1 <= batch <=
   the network's max_batch), one Adam step per minibatch (as
   nmf_mlp_train_step, learning rate lr, multiplied by decay in (0, 1]
   after every epoch).  Minibatch losses are summed on the device; the only
   host synchronization is one per epoch when loss_host (may be NULL,
   `epochs` doubles) receives each epoch's mean minibatch loss. */
nmf_status nmf_ws_train(nmf_mlp* m, const float* const* V, const float* const* H,
                        int32_t count, int64_t n, int64_t ldv, int64_t ldh,
                        int32_t epochs, int32_t batch, float lr, float decay,
                        uint64_t seed, double* loss_host);

/* ---- Batched tier ----------------------------------------------------------
   Many independent problems V_b ~ W_b H_b of uneven p, n and r (r <= 64)
   advanced together: every call of nmf_batch_step is ONE persistent kernel
   launch (replayed from a hipGraph) in which workgroups take tiles of all
   problems from a shared queue.  One iteration of a problem is the W update
   then the H update of Algorithm 1 (Sec. 3.1), both with the Gram forms of
   the denominators and the zero-denominator guard of nmf_step, in float32
   on the matrix cores.  Results are deterministic for a given tile table. */
typedef struct nmf_batch nmf_batch;

typedef struct {
  const float* V;   /* p x n, row stride ldv (device); read-only */
  float* W;         /* p x r (device): start, overwritten by every step */
  float* H;         /* r x n (device): start, overwritten by every step */
  int64_t p, n, ldv;
  int32_t r;        /* 1..64 */
  int32_t reserved; /* must be 0 */
} nmf_problem;

/* Tile table: entries 2c and 2c+1 are the phase-W tile rows and phase-H
   tile columns, in units of 64 (1 or 2), for padded-rank class c
   (rank padded to 16 (c + 1)); entry 8 is workgroups per compute unit
   (1 or 2). */
#define NMF_BATCH_TABLE_LEN 9

/* Copy the problem list (host array of `count` <= 16383 entries), allocate
   the workspace and load V, W and H.  V is copied once, here, into padded
   row-major and transposed copies (about 2 x 4 bytes per entry of V) that
   the steps read; a later change to the caller's V is not seen.  W and H
   stay owned by the caller and must outlive the batch.  Pointers need
   4-byte alignment only.  Errors: NMF_EINVAL (null pointer, p, n or r < 1,
   ldv < n, reserved != 0), NMF_EUNSUPPORTED (r > 64), NMF_ENOMEM. */
nmf_status nmf_batch_create(nmf_batch** out, const nmf_problem* probs,
                            int32_t count, void* stream);

/* Reload every problem's W and H from the caller's arrays (after the
   caller changed them).  Asynchronous. */
nmf_status nmf_batch_load(nmf_batch* b);

/* `iters` iterations of every problem (one persistent launch), then the
   caller's W and H are updated.  Asynchronous; a broken schedule is
   reported by the next nmf_batch_check / nmf_batch_objective. */
nmf_status nmf_batch_step(nmf_batch* b, int32_t iters);

/* Synchronize the stream; NMF_EDEVICE if a launch since the last check
   stopped on its wait bound (its results are then not valid). */
nmf_status nmf_batch_check(nmf_batch* b);

/* f_host[b] = ||V_b - W_b H_b||_F^2 (eq. for the Euclidean objective,
   float64 accumulation) for every problem; synchronizes.  NMF_ENONFINITE if
   any value is not finite. */
nmf_status nmf_batch_objective(nmf_batch* b, double* f_host);

/* Read / install the tile table (NMF_BATCH_TABLE_LEN ints, host). */
nmf_status nmf_batch_get_table(nmf_batch* b, int32_t* table);
nmf_status nmf_batch_set_table(nmf_batch* b, const int32_t* table);

/* Autotuner: times trial_iters iterations of this batch for candidate tile
   tables (coordinate descent over workgroups per CU and each occurring rank
   class's tile shape), installs the fastest and leaves W, H and the Grams
   as they were.  best_ms (host, may be NULL) receives its milliseconds per
   iteration.  Synchronizes. */
nmf_status nmf_batch_tune(nmf_batch* b, int32_t trial_iters, double* best_ms);

/* Release the batch (not the caller's arrays).  NULL is ignored. */
void nmf_batch_destroy(nmf_batch* b);

/* Solve every problem of the list with one call: create a batch, run
   chunks of opt->check_every iterations (one persistent launch each), after
   each chunk evaluate every problem's objective and stop when every problem
   satisfies the stopping rule of opt (tol_kind, tol: the rules of nmf_solve,
   applied per problem) or max_iters iterations have run; then destroy the
   batch.  Every problem runs the same number of iterations (the updates
   never increase f, so iterations past a problem's own stopping point only
   refine it).  opt may be NULL (defaults of nmf_default_options).
   opt->seed != 0: W and H of problem i are first filled with U(0,1) draws
   (Philox4x32-10 under key seed, streams 2i and 2i + 1; problem 0 gets the
   start nmf_init draws for that seed).  opt->validate: every V is scanned
   first and a negative or non-finite entry returns NMF_EINVAL.
   opt->use_graph is ignored (the batched tier always replays its launch
   from a graph).  opt->precision must be NMF_FP32 and opt->loss
   NMF_LOSS_EUCLIDEAN (NMF_EUNSUPPORTED otherwise).  iters_done_host (may be NULL) receives the iterations run;
   f_out (host, count doubles, may be NULL) the final objectives.
   Returns NMF_OK when the rule held for every problem at a check,
   NMF_ENOTCONVERGED at the cap (max_iters = 0: the start is evaluated
   only), NMF_ENONFINITE if an objective is not finite, and the errors of
   nmf_batch_create. */
nmf_status nmf_batch_solve(const nmf_problem* probs, int32_t count,
                           int32_t max_iters, const nmf_options* opt,
                           int32_t* iters_done_host, double* f_out, void* stream);

/* ---- Penalized PET reconstruction (Sec. 3.2, Algorithm 2) ----------------
   The paper's second MM demonstration, with the same separation of
   parameters: Poisson emission intensities lambda (p pixels on a rows x cols
   grid, row-major) seen through d lines of flight with geometry E (d x p)
   and counts y (d), maximizing the penalized log-likelihood (eq.
   PET-objpen)
     f(lambda) = sum_i [y_i ln (E lambda)_i - (E lambda)_i]
                 - (mu / 2) sum_{{j,k} adjacent} (lambda_j - lambda_k)^2
   over the 4-neighbour pairs of the grid.  Algorithm 2: E is scaled to unit
   column sums (on the device, at creation); each iteration forms, for all
   pixels in parallel, c_j = lambda_j sum_i e_ij y_i / (E lambda)_i,
   b_j = mu (|N_j| lambda_j + sum_{k in N_j} lambda_k) - 1, a_j = -2 mu |N_j|
   and takes the positive root of a_j x^2 + b_j x + c_j = 0 (evaluated as
   2 c / (-b + sqrt(b^2 - 4 a c)) when b <= 0, the same root without the
   printed form's cancellation at small mu, and in the printed form when
   b > 0; mu = 0 gives the EM update c_j).  The text's
   formula for b omits the factor mu that Algorithm 2 and the derivative
   carry; b includes it.  float32 products, float64 objective. */
typedef struct nmf_pet nmf_pet;

/* How the scaled E is held on the device.  DENSE: E_s and its transpose,
   read with coalesced row dot products.  SPARSE: the nonzeros of every line
   and of every pixel in padded rows of (value, index) pairs; a line of
   flight crosses O(sqrt p) pixels, so a ring scanner's E is about 2%
   dense.  AUTO takes SPARSE when the longest line and the longest pixel
   column each hold at most a quarter of a dense row. */
typedef enum nmf_pet_layout_kind {
  NMF_PET_AUTO = 0,
  NMF_PET_DENSE = 1,
  NMF_PET_SPARSE = 2
} nmf_pet_layout_kind;

/* E (d x p row-major), y (d) and lambda (p) are device pointers, 16-byte
   aligned; p = rows * cols, a multiple of 4; mu >= 0; layout one of
   nmf_pet_layout_kind.  E, y and lambda must be finite and nonnegative
   (checked on the device).  E and y are copied (E scaled) at creation;
   lambda is the caller's start (Algorithm 2 uses all ones), updated in
   place by every step, and must outlive the object.  Synchronizes.
   Errors: NMF_EINVAL (arguments or data), NMF_EUNSUPPORTED (p not a
   multiple of 4), NMF_ENOMEM, NMF_EDEVICE. */
nmf_status nmf_pet_create(nmf_pet** out, const float* E, int64_t d, int64_t p,
                          const float* y, int32_t rows, int32_t cols, double mu,
                          float* lambda, int32_t layout, void* stream);

/* The layout chosen at creation (NMF_PET_DENSE or NMF_PET_SPARSE). */
nmf_status nmf_pet_layout(const nmf_pet* m, int32_t* layout);

/* Enqueue `iters` iterations (replayed from HIP graphs of 16, 8, 4, 2 and 1
   iterations).  Asynchronous. */
nmf_status nmf_pet_step(nmf_pet* m, int32_t iters);

/* f(lambda) of the current intensities in float64; synchronizes. */
nmf_status nmf_pet_objective(nmf_pet* m, double* f_host);

/* Iterate until |f_k - f_prev| / (|f_prev| + 1) < tol at a check (every
   check_every iterations; the stopping rule of Sec. 3) or max_iters.  The
   rule is tested on the device after every block of check_every iterations
   (replayed graphs of 8 blocks; the blocks after the one where it holds do
   nothing), so the result is that of the host loop "step(check_every),
   objective, test" to the bit.  Synchronizes.  Returns NMF_OK,
   NMF_ENOTCONVERGED at the cap, NMF_ENONFINITE. */
nmf_status nmf_pet_solve(nmf_pet* m, int32_t max_iters, double tol, int32_t check_every,
                         int32_t* iters_done_host, double* f_host);

/* nmf_pet_solve accelerated by QN(q) (Zhou, Alexander & Lange; the QN(10)
   columns of Table 3), as nmf_solve_qn does for NMF: with F one iteration
   of Algorithm 2, each QN iteration evaluates F twice, keeps the secant
   pairs of the last q QN iterations in float64, forms the quasi-Newton
   point x_qn = F(x) + V (U^T U - U^T V)^-1 U^T (F(x) - x), projects it onto
   lambda >= 0.5 F(x) entrywise, and takes it when the q x q system is
   regular and f(x_qn) >= f(F(F(x))); otherwise it keeps F(F(x)).  So f
   never decreases.  Every decision is made on the device; one QN iteration
   is replayed from a HIP graph.  max_evals counts evaluations of F (two per
   QN iteration, at most 131072); the rule |f - f_prev| / (|f_prev| + 1) <
   tol is tested on the accepted objective every check_every evaluations
   (check_every / 2 QN iterations, at least one).  *evals_done: evaluations
   of F run; *accepted (may be NULL): QN iterations whose point was taken;
   *f_host: f of the intensities left in lambda; trace (may be NULL): f of
   the start and then after every QN iteration, up to trace_len entries.
   1 <= q <= 16.  Returns NMF_OK, NMF_ENOTCONVERGED, NMF_ENONFINITE. */
nmf_status nmf_pet_solve_qn(nmf_pet* m, int32_t q, int32_t max_evals, double tol,
                            int32_t check_every, int32_t* evals_done, int32_t* accepted,
                            double* f_host, double* trace, int32_t trace_len);

/* Release the object (not the caller's lambda).  NULL is ignored. */
void nmf_pet_destroy(nmf_pet* m);

/* Release the context's workspace.  NULL is ignored. */
void nmf_destroy(nmf_ctx* ctx);

/* Static description of a status code. */
const char* nmf_strerror(nmf_status s);

/* Library version as 10000*major + 100*minor + patch. */
int32_t nmf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NMF_H */
