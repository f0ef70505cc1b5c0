/*
 * scs.h - Sketched Preconditioned SVRG for ridge regression on AMD MI355X (gfx950).
 *
 * Gonen, Orabona, Shalev-Shwartz, "Solving Ridge Regression using Sketched
 * Preconditioned SVRG", arXiv:1602.02350.
 *
 * Problem (Sec. 1, Eq. (ridge)):  minimize  L(w) = (1/n) sum_i 1/2 (w^T x_i - y_i)^2 + (lambda/2)||w||^2.
 *
 * Conventions for every entry point:
 *   - Matrices are ROW-MAJOR with an explicit leading dimension (elements between
 *     consecutive rows, >= the row length). X is n x d: one instance per row
 *     (the paper stores instances as columns; formulas are transposed).
 *   - Unless stated otherwise, array arguments are DEVICE pointers on the
 *     context's device. Inputs are borrowed: never freed, never modified.
 *     Outputs are caller-allocated. Scratch memory is owned by the context,
 *     allocated on first use, reused, and released by scs_destroy.
 *   - Work is enqueued on the context's stream. Entry points that return host
 *     values (reports, status) synchronize that stream before returning;
 *     the others are asynchronous with respect to the host.
 *   - Return value: SCS_OK (0); a negative code for caller or device errors
 *     (nothing useful was written); a positive code for a numerical outcome
 *     with a valid best-so-far output. No C++ exception crosses this boundary.
 *     scs_last_error() gives a human-readable message for the last failure.
 *   - Floating point: inputs FP32; the full-gradient pass and the inner loop
 *     compute in FP32 with FP64 cross-workgroup reductions; the small dense
 *     sketch algebra (Gram, Cholesky, eigendecomposition) is FP64.
 */
#ifndef SCS_H
#define SCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------------- */
#define SCS_OK 0
#define SCS_EINVAL (-1)       /* bad argument: lambda <= 0, k < 0, k > d, n < k + p, null pointer, bad stride */
#define SCS_ENONFINITE (-2)   /* NaN or Inf met in X or y (found by the first full-gradient pass) */
#define SCS_ENOMEM (-3)       /* device allocation failed */
#define SCS_EDEVICE (-4)      /* HIP runtime error (message in scs_last_error) */
#define SCS_NOT_CONVERGED 1   /* epoch cap reached before the stop rule held; output = last snapshot */
#define SCS_DIVERGED 2        /* objective became non-finite or grew 10x over its start even after 6 step halvings;
                                 output = last good snapshot */
#define SCS_SKETCH_RANK_DEFICIENT 3 /* range-finder block lost rank (e.g. X = 0); solved without preconditioning */

/* Precision of the sketch GEMMs and of the preconditioned rows used by the inner loop. */
/* wave_rows value of the look-ahead inner loop: each step's next dot products are formed while the step's
   cross-workgroup exchange is in flight, as P - eta G g with P = R_{t+1}(delta_t - eta mu) and the Gram block
   G = R_{t+1} R_t^T of the workgroup's columns (Alg. 1's update expanded one step; FP32 rows use a three-term
   BF16 product for G, about 2^-16 relative error per entry; BF16 rows are exact). Same results as the
   direct loop up to rounding. */
#define SCS_LOOKAHEAD 8

#define SCS_PREC_FP32 0       /* FP32 MFMA for Rayleigh-Ritz and the apply, FP32 rows (range finder: see sketch_fp32) */
#define SCS_PREC_MIXED 1      /* BF16 MFMA GEMMs (FP32 accumulation), BF16 rows in the inner loop */

/* Stop rules for scs_svrg_solve (checked at the start of every epoch's full-gradient pass). */
#define SCS_STOP_EPOCHS 0     /* run exactly max_epochs epochs (Alg. 1's parameter S) */
#define SCS_STOP_CERTIFICATE 1/* stop when ||grad||^2 (lam~_1 + lambda)/(2 lambda) <= eps (||grad||^2/(2 lambda) for k = 0),
                                 an upper bound on L - L* */
#define SCS_STOP_GAP 2        /* stop when L(w) - f_star <= eps (f_star supplied by the caller) */

typedef struct scs_ctx scs_ctx;

/* Options. Fill with scs_opts_default() and change what you need. */
typedef struct scs_opts {
  int oversample;         /* p: range-finder width is k + p (default 5) */
  int batch;              /* b: i.i.d. draws per inner step, 1..256 (default 64) */
  int64_t steps;          /* m: inner steps per epoch; 0 = ceil(epoch_factor n / b), or ceil(2 n / b) */
  double step_scale;      /* c: step eta = c / beta_hat with beta_hat = (1/(n+d)) sum_i beta_i (default 1) */
  int max_epochs;         /* S: epoch cap (default 30) */
  int stop_rule;          /* SCS_STOP_* (default SCS_STOP_CERTIFICATE) */
  double f_star;          /* optimum value for SCS_STOP_GAP */
  int average;            /* 1: snapshot = average of the m inner iterates (Alg. 1); 0: last iterate */
  int precision;          /* SCS_PREC_* (default SCS_PREC_FP32) */
  int workgroups;         /* inner-loop workgroups per problem; 0 = chosen from d; -1 = autotuned: timed on the
                             problem's own rows on first use per (d, b, precision), cached in the context
                             (single solves). Batched and path solves take a positive value as given (at
                             least one per 512 columns of the widest problem, at most 16) and otherwise use
                             one per 256 columns */
  uint64_t seed;          /* seed of the Gaussian test matrix and of the index stream */
  const float* omega;     /* optional device (k+p) x d row-major Gaussian test matrix (transposed Omega); NULL = drawn from seed */
  const int32_t* indices; /* optional device index stream, max_epochs x m x b entries in [0, n+d); NULL = drawn from seed */
  float* trace_w;         /* optional device max_epochs x d: w = P^{-1/2} w~ of the snapshot entering each epoch
                             (rows of epochs after the stop rule held are left untouched) */
  double* epoch_ms;       /* optional HOST array of max_epochs: milliseconds from the call's start to each epoch's
                             end; -1 for epochs never enqueued because the stop rule had held. Asking for it
                             records an event after every epoch, a few microseconds each */
  int timing;             /* 1: time every inner-loop launch with HIP events (report.ms_inner); 2: also every
                             full-gradient pass (report.ms_grad). Each event adds a few microseconds between kernels */
  double epoch_factor;    /* with steps = 0 and epoch_factor > 0: m = ceil(epoch_factor n / b) per problem (default 0) */
  int implicit_apply;     /* scs_svrg_solve_path only: 1 = never form the preconditioned rows; the inner loop uses
                             x_i and z_i = U~^T x_i, O(d + k) per row (FP32 rows; needs d <= 2048, k <= 128) */
  int uniform_sampling;   /* 1: draw the n + d components uniformly, q_i = 1/(n+d) (the uniform sampling of
                             Johnson and Zhang, Sec. 4.2) instead of q_i proportional to beta_i (Xiao and Zhang,
                             the default 0); eta = c / beta_hat either way, so c is tuned per sampling rule */
  int wave_rows;          /* inner-loop layout (single solves): how each workgroup's 8 waves split the minibatch's
                             rows, 1, 2 or 4 wave-rows of 8 / wave_rows waves (64 rows each at most; slices of at
                             most 512, 128 or 64 columns); SCS_LOOKAHEAD = the look-ahead loop (b <= 64, slices of
                             at most 64 columns, see below); 0 = chosen from b and the slice width, or autotuned
                             together with the workgroups when workgroups = -1 */
  /* Warm starts and checkpoints (single solves). A solve stopped after S1 epochs with wt_out set, then
     resumed with w0 = that snapshot, w0_preconditioned = 1 and epoch_offset = S1 (same X, y, lambda, k,
     seed and options), reproduces the uninterrupted solve bit for bit (the sketch and every epoch's
     index stream are functions of the seed and the epoch number). */
  const float* w0;        /* optional device d: start point (default 0). In the original space (w), mapped to
                             the solver's variable by w~ = P^{1/2} w, unless w0_preconditioned = 1 */
  int w0_preconditioned;  /* 1: w0 is the solver's own variable w~ (for example a snapshot written to wt_out) */
  int epoch_offset;       /* epoch s of this call draws the index stream of epoch s + epoch_offset */
  float* wt_out;          /* optional device d: the final snapshot w~ (the checkpoint to resume from) */
  int sketch_fp32;        /* 1: in FP32 precision the range finder's GEMMs (X Omega, X^T (X Omega) and the further
                             Krylov blocks) use FP32 MFMA; 0 (default): BF16 MFMA with FP32 accumulation in every
                             precision (the range only fixes the subspace; Rayleigh-Ritz, X Q and Z = X U~, follows
                             `precision`, and the fixed point is set by the exact FP32 gradient) */
  int krylov_blocks;      /* q: the sketch's Krylov space [C Omega, C^2 Omega, ..., C^q Omega] (Block Lanczos, Alg. 2;
                             C = X^T X / n); 0 or 1 = the one-block range finder Y = X^T (X Omega). Each block
                             after the first costs two more passes over X; q (k + p) <= min(d, n, 136) */
  int no_graph;           /* batched and path solves: 1 = the host enqueues every epoch's kernels; 0 (default) = the
                             epochs replay a captured hipGraph of 8 epochs whose kernels read the epoch number from
                             the device (the same kernels in the same order: results are bit-identical). timing > 0
                             uses the enqueued mode (its events sit between kernels) */
  int warm_start;         /* scs_svrg_solve_path only: 1 = solve the lambdas one after another in the order given
                             (largest first is the usual continuation order), each lambda's ny solves starting
                             from the previous lambda's solutions (a regularization path with warm starts,
                             Sec. 2.2); 0 = all solves together from 0 */
} scs_opts;

typedef struct scs_report {
  int status;             /* same as the return value */
  int epochs;             /* epochs completed */
  int k_used;             /* sketch rank actually used (k, or 0 after SCS_SKETCH_RANK_DEFICIENT) */
  int64_t steps;          /* m used */
  double eta;             /* step used */
  double beta_hat;        /* average smoothness of the n+d components */
  double objective;       /* L(w) at the returned w, from the last full-gradient pass */
  double grad_norm;       /* ||grad L~(w~)|| at the returned snapshot */
  double certificate;     /* ||grad||^2 (lam~_1 + lambda)/(2 lambda); ||grad||^2/(2 lambda) for k = 0 */
  double lam_top;         /* lam~_1 (largest sketched eigenvalue; 0 if k = 0) */
  double ms_sketch, ms_apply, ms_solve; /* stage times */
  double ms_grad, ms_inner; /* summed durations of the full-gradient passes (opts.timing >= 2) and inner-loop launches
                               (opts.timing >= 1); batched and path solves: the shared inner-loop launches of all
                               problems (every report holds the same figure), no ms_grad */
  int n_grad, n_inner;      /* number of launches summed in ms_grad and ms_inner */
  int backoffs;             /* rejected snapshots: each restored the previous one and halved the step */
  int workgroups;           /* inner-loop workgroups used per problem */
  int wave_rows;            /* inner-loop layout used (single solves): 1, 2, 4 wave-rows or SCS_LOOKAHEAD */
} scs_report;

void scs_opts_default(scs_opts* opts);
const char* scs_status_string(int status);
const char* scs_last_error(void);

/* Create a context on HIP device `device`, enqueueing on `hip_stream` (a hipStream_t; NULL = the null stream). */
int scs_create(scs_ctx** out, int device, void* hip_stream);
int scs_destroy(scs_ctx* ctx);

/*
 * Randomized sketch (Alg. 2 with one Krylov block, Sec. 4.3): Y = X^T (X Omega),
 * Q = orth(Y) by CholeskyQR2 in FP64, B = (X Q)^T (X Q) / n, B = V Theta V^T by a
 * symmetric tridiagonal eigensolver in FP64 (Householder reduction, multisection for
 * the eigenvalues, inverse iteration for the vectors), lam~ = Theta_{1..k}
 * (descending, clamped >= 0), U~ = Q V_{:,1..k}.
 * The lam~ estimate the eigenvalues of C = X^T X / n (Eq. (covSpec)), i.e. the
 * squared singular values of n^{-1/2} X.
 *   X: n x d (ld ldx); k in [1, d]; q (k + p) <= min(d, n, 136) with q = opts->krylov_blocks (>= 1).
 * With q > 1 the range is the Krylov space of Block Lanczos (Alg. 2) started from C Omega: each further
 * block is C times the previous orthonormal block, projected twice against the earlier blocks and
 * orthonormalized by CholeskyQR2; Rayleigh-Ritz then runs on all q (k + p) columns.
 *   U_out: d x k row-major FP32 (ld k); U64_out (nullable): d x k FP64; lam_out: k FP64.
 * Returns SCS_SKETCH_RANK_DEFICIENT if the Gram matrix of Y is not positive definite.
 */
int scs_sketch_build(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, int k,
                     const scs_opts* opts, float* U_out, double* U64_out, double* lam_out);

/*
 * Preconditioner of Eq. (condSketch), P^{-1/2} = sum_i u_i u_i^T/sqrt(lam_i+lambda) + (I - U U^T)/sqrt(lam_k+lambda),
 * applied to every row (Alg. 3, x~_i = P^{-1/2} x_i) and to the regularizer rows b_j = P^{-1/2} e_j (Sec. 5.1):
 *   Xt_out  (n x d, ld ldt): x~_i = x_i / s + U~ (D (U~^T x_i)),  s = sqrt(lam_k + lambda), D_j = 1/sqrt(lam_j + lambda) - 1/s
 *   reg_out (d x d, ld ldt): sqrt(n lambda) b_j  (so that the n+d components are 1/2 (n+d)/n (a_i^T w - t_i)^2)
 *   beta_out (n + d, nullable): ||x~_i||^2 then ||sqrt(n lambda) b_j||^2 (proportional to the smoothness beta_i of Alg. 3)
 * xt_bf16 = 1 stores Xt_out and reg_out as BF16 (round to nearest even); 0 stores FP32.
 * U is d x k FP32 (ld k), lam k FP64 (descending). k = 0 gives P = I. ldt >= d.
 */
int scs_precondition_apply(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx,
                           const float* U, const double* lam, int k, double lambda,
                           int xt_bf16, void* Xt_out, void* reg_out, int64_t ldt, float* beta_out);

/*
 * Full gradient of the preconditioned objective at w~ (Alg. 1, the snapshot gradient; Sec. 5.1):
 *   grad L~(w~) = P^{-1/2} [ X^T (X w - y)/n + lambda w ],  w = P^{-1/2} w~,
 * which equals X~^T (X~ w~ - y)/n + lambda P^{-1} w~ (the n+d-component form) and is
 * evaluated with X itself so that its fixed point is exactly that of L.
 *   wt: d FP32 (device); grad_out: d FP32 (device); obj_out (nullable, HOST): L(w) = L~(w~).
 */
int scs_full_gradient(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, const float* y,
                      const float* U, const double* lam, int k, double lambda,
                      const float* wt, float* grad_out, double* obj_out);

/*
 * One SVRG epoch (Alg. 1, inner loop) on the n+d rows a_i = x~_i (i < n), sqrt(n lambda) b_{i-n} (i >= n):
 *   for t = 1..m: draws i_1..i_b = idx[(t-1) b ..]; v = (1/b) sum_j (a_ij^T (w_{t-1} - w~)) a_ij / (n q_ij) + mu;
 *                 w_t = w_{t-1} - eta v
 *   w~ <- (1/m) sum_t w_t  (average = 1)  or  w_m  (average = 0).
 * q_i are the sampling probabilities of the quantized weights of `beta` (see scs_sample_indices).
 * Xt: n x d rows, reg: d x d rows, both with leading dimension ldt (a multiple of 4), FP32 or BF16 as
 * xt_bf16; beta: n + d, idx: m x b int32 in [0, n+d) (device); 1 <= b <= 256.
 * wt is updated in place; mu = grad L~(w~) (device FP32). workgroups = 0 chooses from d and b;
 * wave_rows as scs_opts.wave_rows (0 = chosen from b and the slice width; SCS_LOOKAHEAD for the look-ahead loop).
 */
int scs_svrg_epoch(scs_ctx* ctx, int64_t n, int64_t d, const void* Xt, const void* reg, int64_t ldt, int xt_bf16,
                   const float* beta, const float* mu, const int32_t* idx, int64_t m, int b,
                   double eta, int average, int workgroups, int wave_rows, float* wt);

/*
 * Importance sampling of Alg. 1 (q_i = beta_i / sum_j beta_j): the beta are quantized to
 * integer weights W_i = max(1, rint(beta_i 2^B / max beta)) (0 for beta_i = 0), B = 62 - ceil(log2 N),
 * and draw g of `epoch` is the first i whose cumulative weight exceeds floor(r_g T / 2^64),
 * r_g a 64-bit Philox4x32-10 output (Salmon et al. 2011), T = sum W. Bit-exact and reproducible.
 *   beta: N FP32 (device); out: count int32 (device).
 */
int scs_sample_indices(scs_ctx* ctx, const float* beta, int64_t N, uint64_t seed, int epoch,
                       int64_t count, int32_t* out);

/* N(0,1) values from Philox4x32-10 + Box-Muller in FP64, rounded to FP32 (device `out`, count entries). */
int scs_gaussian(scs_ctx* ctx, uint64_t seed, int64_t count, float* out);

/*
 * Sketched Preconditioned SVRG (Alg. 3): sketch (k >= 1), precondition, SVRG epochs with
 * minibatches of b, then w = P^{-1/2} w~ (Eq. (condRidge)). k = 0 runs plain SVRG (P = I).
 *   X: n x d (ld ldx), y: n (device FP32). w_out: d FP32 (device). report: HOST, nullable.
 * eps is the target of the stop rule (see SCS_STOP_*).
 */
int scs_svrg_solve(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, const float* y,
                   double lambda, int k, double eps, const scs_opts* opts, float* w_out,
                   scs_report* report);

/*
 * The FP64 instantiation (Alg. 3 with X, y, the sketch, the preconditioned rows, the iterate and every
 * sum in FP64), for problems whose columns fit one workgroup: d <= 4096, n + d < 2^31, one Krylov
 * block with k + p <= min(d, n, 136).
 * Sketch (Alg. 2, q = 1): Y = X^T (X Omega), Q = CholeskyQR2(Y), B = (X Q)^T (X Q) / n = V Theta V^T,
 * lam~ = Theta_{1..k} (descending, clamped >= 0), U~ = Q V_{:,1..k}, all products FP64. Omega^T is
 * opts->omega (FP32, (k + p) x d) widened to FP64, or drawn from opts->seed as in scs_sketch_build.
 *   X: n x d FP64 (ld ldx, device); U_out: d x k FP64 (ld k, device); lam_out: k FP64 (device).
 * Returns SCS_SKETCH_RANK_DEFICIENT if the Gram matrix of Y is not positive definite.
 */
int scs_sketch_build_f64(scs_ctx* ctx, const double* X, int64_t n, int64_t d, int64_t ldx, int k,
                         const scs_opts* opts, double* U_out, double* lam_out);

/*
 * Sketched Preconditioned SVRG in FP64: scs_svrg_solve's method and options (batch b <= 256, steps /
 * epoch_factor, step_scale, max_epochs, stop rules, f_star, seed, omega, indices, epoch_offset,
 * average, uniform_sampling, epoch_ms), with the rows x~_i = x_i/s + U~ D U~^T x_i and the
 * regularizer rows sqrt(n lambda) P^{-1/2} e_j formed in FP64, the index draws of scs_sample_indices
 * (weights quantized from FP64 beta_i, 1/(n q_i) kept in FP64), the full gradient, the stop rules and
 * the inner loop in FP64 (one persistent workgroup per epoch). w0, trace_w and wt_out are FP32-only
 * (SCS_EINVAL here); workgroups, wave_rows, precision and sketch_fp32 are ignored; timing >= 1 times
 * the inner loops (ms_inner, n_inner) and nothing more.
 *   X: n x d FP64 (ld ldx), y: n FP64 (device). w_out: d FP64 (device). report: HOST, nullable
 *   (workgroups = 1; ms_grad is not measured).
 * Status codes as scs_svrg_solve.
 */
int scs_svrg_solve_f64(scs_ctx* ctx, const double* X, int64_t n, int64_t d, int64_t ldx, const double* y,
                       double lambda, int k, double eps, const scs_opts* opts, double* w_out,
                       scs_report* report);

/*
 * The bias-complexity rule (Sec. 2.2): the regularization at which each method's runtime is O~(ndk),
 *   lambda_precond = (k lam_k + sum_{i>k} lam_i) / (n k)   (Eq. (decay), preconditioned SVRG)
 *   lambda_plain   = (sum_i lam_i) / (n k)                 (Eq. (decaySVRG), plain SVRG),
 * lam_i the eigenvalues of C = X^T X / n. The k largest come from the sketch (as scs_sketch_build, with
 * opts), the tail sum is tr(C) minus their sum, and tr(C) = ||X||_F^2 / n (FP64 sum of FP32 row norms).
 * Sketched values are Rayleigh-Ritz values, at most the true ones, so the tail and lambda_precond err
 * on the large side. Outputs are HOST doubles; the call waits for its stream.
 *   k in [1, d], q (k + p) <= min(d, n, 136). Returns SCS_SKETCH_RANK_DEFICIENT (values still written) if the
 *   sketch lost rank.
 */
int scs_regularization_for_budget(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, int k,
                                  const scs_opts* opts, double* lambda_precond, double* lambda_plain);

/*
 * Autotuner of the solver's free parameters on the caller's problem: the minibatch b (32, 64, 128),
 * the step scale c (eta = c / beta_hat, Alg. 1; 1 .. 512), the epoch length m = epoch_factor n / b
 * (epoch_factor 1/64 .. 2; the paper takes m proportional to n, Sec. 6) and the inner loop's launch
 * shape (workgroups and wave-rows, timed per b). Each candidate is a full scs_svrg_solve to the stop
 * rule of `base` (certificate or gap; eps as given), scored by its wall time; the scan over c for a
 * (b, m) stops at the first divergence or step halving, and once the time has risen twice in a row.
 * The four fastest candidates are then solved three more times, each with another sampler stream,
 * and the lowest median of the four wall times wins.
 * Candidates draw Omega and the index stream from seeds derived from base->seed, never from it.
 *   base (nullable): the options to start from; tuned (HOST): receives them with batch, step_scale,
 *   epoch_factor (steps = 0), workgroups and wave_rows set, seed/timing/epoch_ms from base.
 *   best_ms (HOST, nullable): the winner's median wall time in milliseconds.
 * Returns SCS_NOT_CONVERGED if no candidate met the stop rule within base->max_epochs.
 */
int scs_autotune(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, const float* y, double lambda,
                 int k, double eps, const scs_opts* base, scs_opts* tuned, double* best_ms);

/*
 * Many independent ridge problems (uneven n, d, lambda, k) solved together: every problem's
 * sketch, preconditioning and SVRG epochs run as in scs_svrg_solve, with the epochs of all
 * problems advancing together inside shared launches (one persistent inner-loop launch per
 * epoch for all problems). Stop rule and options as in scs_svrg_solve (omega, indices and trace_w
 * must be NULL; opts.f_star is ignored: the gap rule takes f_star, a HOST array of nprob optima,
 * NULL otherwise). Arrays of pointers and sizes are HOST arrays of length nprob; the pointed-to
 * data are device arrays. reports: HOST array of nprob, nullable. The sketch and preconditioner
 * time of all problems is reported as ms_sketch (ms_apply = 0).
 */
int scs_svrg_solve_batched(scs_ctx* ctx, int nprob, const float* const* X, const int64_t* n,
                           const int64_t* d, const int64_t* ldx, const float* const* y,
                           const double* lambda, const int* k, double eps, const double* f_star,
                           const scs_opts* opts, float* const* w_out, scs_report* reports);

/*
 * Regularization path with one shared sketch: one X, ny right-hand sides and nl values of lambda,
 * nl * ny solves. The sketch of X (Alg. 2; it does not involve lambda) is built once; every lambda
 * gets its own preconditioner from the same U~ and lam~ (Eq. (condSketch) with that lambda) and its
 * own preconditioned rows, sampling weights and step size; the ny solves of one lambda share them.
 * All solves advance together: each epoch's full gradients are two FP32 MFMA GEMMs over X
 * (R = X W^T - Y, G = X^T R, FP64 sums of the row-chunk partials), and one batched launch runs every
 * inner loop.
 *   X: n x d (ld ldx), Y: ny x n row-major (right-hand side r is row r), both device FP32.
 *   lambdas: HOST array of nl. W_out: device (nl * ny) x d row-major; solve (j, r) is row j * ny + r.
 *   reports: HOST array of nl * ny, nullable (same order). f_star: HOST array of nl * ny optima for
 *   the gap rule (same order), NULL otherwise. omega, indices and trace_w must be NULL. Workspace
 *   grows with nl (one set of preconditioned rows per lambda).
 */
int scs_svrg_solve_path(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, const float* Y,
                        int ny, const double* lambdas, int nl, int k, double eps, const double* f_star,
                        const scs_opts* opts, float* W_out, scs_report* reports);

/*
 * For callers that cannot allocate device memory (code under HIP stream capture, tight serving
 * loops, harnesses that forbid hipMalloc): scs_full_gradient with the same arguments and results,
 * running the same kernels, but with every scratch buffer taken from one fixed device array of
 * SCS_NOALLOC_SCRATCH_BYTES that the library holds on each device until the process ends. The call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 *   The scratch it needs is 256-aligned pieces of: 4 k d (U~^T) + 4 d + 8 d + 128 d + 4 d bytes and,
 *   with G = min(512, ceil(n / 8)) workgroups, 4 G d + 8 G bytes, plus the solver state. A problem
 *   needing more returns SCS_EINVAL without launching anything (d = 2048, k = 128 needs about 5.6 MB).
 *   obj_out (HOST, nullable): when given, the call copies the objective back, waits for the stream and
 *   reports SCS_ENONFINITE like scs_full_gradient; when NULL it only enqueues work (nothing waits, nothing
 *   is copied to the host), so it may be recorded into a graph.
 * Every call on one device shares that device's array and leaves its contents behind (the solver
 * state is cleared by a kernel at the start of each call). Calls that overlap in time on one device,
 * from different streams or threads, race on the array and give undefined results.
 */
#define SCS_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
int scs_full_gradient_noalloc(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, const float* y,
                              const float* U, const double* lam, int k, double lambda,
                              const float* wt, float* grad_out, double* obj_out);

#ifdef __cplusplus
}
#endif
#endif /* SCS_H */
