/*
 * pr.h -- C ABI of libpr: certified lower bounds for branch-and-bound nodes of
 * cardinality-constrained GLMs on one AMD Instinct MI355X (gfx950).
 *
 * Method: arXiv 2603.01306.  Each node relaxation is the perspective
 * relaxation (Section 2.3, eq. perspective_relaxation over the domain D) in
 * composite form Phi(beta) = F(X beta) + 2 lambda2 g_N(beta) (Section 2.4),
 * solved by FISTA with the duality-gap restart (Section 3.3 and "Restart in
 * practice"); every iterate's induced dual vector zeta = -grad F(X beta)
 * (Section 3.2) gives the weak-duality lower bound Psi(zeta) =
 * -F*(-zeta) - G*(X^T zeta) (eq. fenchel_dual), evaluated in FP64.
 *
 * Losses (the paper does not spell them out; this library's reading):
 *   PR_LSQ      F(u) = ||u - y||^2
 *   PR_LOGISTIC F(u) = sum_i log(1 + exp(-y_i u_i)),  y_i in {-1, +1}
 *
 * Conventions for every entry point:
 *   - Pointers documented "device" are caller-owned device memory that must
 *     stay valid for the duration of the call; pointers documented "host" are
 *     caller-owned host memory.  Nothing is retained after a call returns
 *     except what lives inside a pr_ctx (its workspace and cached ||X||^2).
 *   - X is column-major n x p with leading dimension n (column j at X + j*n).
 *     Vectors of length n or p are contiguous FP64.
 *   - Calls on one pr_ctx must not overlap (one context per stream).  All
 *     calls are synchronous with respect to the host: results are complete
 *     when they return.  Work is ordered on the context's stream.
 *   - Return value: PR_OK (0) or a negative error code (pr_strerror).  On
 *     error no output is written unless stated.
 */
#ifndef PR_H
#define PR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes (negative) */
#define PR_OK 0
#define PR_EINVAL (-1)   /* bad size, parameter, dtype or index */
#define PR_EOVERLAP (-2) /* J0 and J1 share an index */
#define PR_EDEVICE (-3)  /* a HIP runtime call failed */
#define PR_ENOMEM (-4)   /* device or host allocation failed */

/* per-node status codes (positive, in pr_result.status) */
#define PR_CONVERGED 1    /* (UB - LB) / |UB| <= rel_gap_tol */
#define PR_MAXITER 2      /* iteration limit; lower_bound is still valid */
#define PR_INFEASIBLE 3   /* |J1| > k: empty domain, lower_bound = +inf */
#define PR_CUTOFF_PRUNE 4 /* lower_bound >= cutoff (Section 5.3, rule 2) */
#define PR_CUTOFF_BRANCH 5 /* primal <= cutoff (Section 5.3, rule 1) */

/* node-status codes of a coordinate (pr_prox, pr_regularizer) */
#define PR_FREE 0  /* j in J_f: z_j in [0, 1] */
#define PR_ZERO 1  /* j in J_0: z_j = 0 */
#define PR_ONE 2   /* j in J_1: z_j = 1 */

typedef enum { PR_LSQ = 0, PR_LOGISTIC = 1 } pr_loss;
typedef enum { PR_F64 = 0, PR_F32 = 1, PR_BF16 = 2 } pr_dtype;

/* Problem data shared by every node of a tree (Section 2.3, problem (1)). */
typedef struct {
  const void *X;  /* device, column-major n x p, element type xdtype */
  int32_t xdtype; /* pr_dtype; PR_F64/PR_F32 need n % 2 / n % 4 == 0 for
                     vector loads, PR_BF16 needs n % 8 == 0 */
  int32_t loss;   /* pr_loss */
  const double *y; /* device, n; for PR_LOGISTIC every y_i is -1 or +1 */
  int64_t n, p;    /* n >= 1, p >= 1 */
} pr_problem;

/* One branch-and-bound node: cardinality k, ridge weight lambda2, box M and
 * the fixed-zero / fixed-one index sets J0, J1 (domain D, Section 2.3). */
typedef struct {
  int32_t k;       /* >= 1 */
  int32_t pad0;
  double lambda2;  /* > 0 */
  double M;        /* > 0; +INFINITY allowed (no box) */
  const int32_t *J0; /* host, n0 indices in [0, p), may be NULL when n0 = 0 */
  int64_t n0;
  const int32_t *J1; /* host, n1 indices in [0, p) */
  int64_t n1;
} pr_node;

/* Iteration variants (pr_opts.method), as compared in the paper's
 * convergence study (Section 5.2): FISTA with the duality-gap restart of
 * Section 3.3 (the method; default), FISTA without restarts, FISTA restarted
 * whenever Phi increases (function-value restart), proximal gradient, and
 * AC-FGM (the accelerated composite method of Li and Lan with its first-step
 * line search, Section 3.3's rate table) with and without the duality-gap
 * restart.  All evaluate the same bounds and stopping test.
 *
 * AC-FGM as implemented (this library's reading; the paper cites the method
 * without restating it): z_t = prox_{eta_t G}(y_{t-1} - eta_t grad f(x_{t-1})),
 * y_t = (1 - b) y_{t-1} + b z_t, x_t = (z_t + tau_t x_{t-1}) / (1 + tau_t),
 * tau_1 = 0, tau_t = t / 2; with Lhat_t = ||grad f(x_t) - grad f(x_{t-1})|| /
 * ||x_t - x_{t-1}||: eta_1 = 1 / L1, eta_2 = min((1 - b) eta_1, 1 / (4 Lhat_1)),
 * eta_t = min((tau_{t-1} + 1) / tau_t eta_{t-1}, tau_{t-1} / (4 Lhat_{t-1}));
 * the first step is retried with L1 <- c L1 while Lhat_1 > L1 (L1 starts at
 * L0).  x_t is the primal iterate of the certificate.  A gap restart starts a
 * new epoch at x_t (y = x_t, t = 1) keeping L1.  One X^T pass per
 * evaluation (the gradient point is the certificate's point) for both
 * losses, and a product over the support of z_t.  Every evaluated point,
 * rejected trials included, counts in pr_result.iters. */
#define PR_FISTA_GAP 0
#define PR_FISTA 1
#define PR_FISTA_FV 2
#define PR_PGD 3
#define PR_ACFGM_GAP 4
#define PR_ACFGM 5
/* FISTA with backtracking (the "FISTA with line search" the paper runs with
 * its restart, Section 5; the monotone rule of Beck, First-Order Methods in
 * Optimization, Section 10.7), with (PR_FISTA_BT_GAP) or without the
 * duality-gap restart.  The step constant starts at L0 (opts->L0; 0 = L / 16)
 * and is multiplied by c (opts->acfgm_c) while the trial x = prox(y -
 * grad f(y) / L) breaks the quadratic model f(x) <= f(y) + <grad f(y), x - y>
 * + (L / 2) ||x - y||^2; it never exceeds the fixed-step constant L
 * (opts->L, default as above), at which a trial is accepted.  Momentum, the
 * bounds, the stopping test and the restart act at accepted iterates; a
 * restart runs the method afresh from its iterate, the line search from L0.
 * A rejected trial is not evaluated: it costs one product over its support
 * (the X^T pass takes the same decision from the same sums and exits at
 * once) and the redone step; pr_result.iters counts accepted iterates,
 * .trials the rejected ones, .L is the last step constant.  p <= 16384 (pr_solve returns
 * PR_EINVAL beyond); pr_solve_batch runs it per node on the batched path. */
#define PR_FISTA_BT_GAP 6
#define PR_FISTA_BT 7

typedef struct {
  double rel_gap_tol; /* stop when (UB - LB) / |UB| <= tol; default 1e-6 */
  double eta;         /* restart factor (> 1); default e^3 */
  double cutoff;      /* incumbent value for dynamic termination; NaN = off */
  double L;           /* step 1/L; 0 = 1.01 * loss curvature * ||X||^2 estimate */
  int32_t max_iter;   /* default 100000 */
  int32_t check_every; /* iterations per captured graph launch (rounded up to even); default 32.
                        * pr_solve runs the iterations it predicts to be a solve's last ones
                        * as launches of an 8-iteration graph; the iterates do not depend on
                        * either length */
  int32_t method;      /* iteration variant, PR_FISTA_GAP (default) .. PR_FISTA_BT */
  int32_t pad0;
  double *trace;       /* pr_solve / pr_lasso_solve only, optional device array of
                          2 * (max_iter + 1) doubles: (Phi, Psi) of iterates 0, 1, ..., iters */
  double acfgm_b;      /* AC-FGM averaging weight b in (0, 1 - sqrt(6)/3]; default 0.1 */
  double acfgm_c;      /* line-search factor c > 1 (AC-FGM's first step, FISTA with backtracking); default 2 */
  double L0;           /* initial curvature estimate of the line search; 0 = the default
                          (AC-FGM L / 64, FISTA with backtracking L / 16) */
} pr_opts;

typedef struct {
  double lower_bound; /* best Psi(zeta^t) seen: a valid bound on the node */
  double primal;      /* best Phi(beta^t) seen */
  double rel_gap;     /* (primal - lower_bound) / |primal| */
  double L;           /* step constant used */
  int32_t iters;      /* proximal-gradient steps taken */
  int32_t restarts;   /* duality-gap restarts */
  int32_t status;     /* PR_CONVERGED ... PR_CUTOFF_BRANCH */
  int32_t trials;     /* trials rejected by a line search (AC-FGM's first step, FISTA with
                         backtracking); else 0 */
} pr_result;

typedef struct pr_ctx pr_ctx;

/* Fill opts with the defaults listed in pr_opts. */
void pr_opts_default(pr_opts *opts);

/* Create a context for problem `prob` on HIP stream `stream` (a hipStream_t;
 * NULL = the default stream) of the current device.  Estimates ||X||_2^2 by
 * the Lanczos recurrence on X^T X (used for the step 1/L, Section 5.2 FISTA)
 * and allocates a workspace for up to max_batch nodes (>= 1).  X and y are
 * not copied: they must outlive the context and must not change.  PR_EINVAL
 * for n < 1, p < 1, p >= 2^29 or max_batch < 1. */
int pr_ctx_create(pr_ctx **out, const pr_problem *prob, int32_t max_batch, void *stream);
int pr_ctx_destroy(pr_ctx *ctx);
/* Test switches of a context (a bit set; 0 = normal operation).
 * PR_DEBUG_GRAM_RECHECK: in Gram mode, treat every pr_solve decision as not
 * confirmed by the recomputation over X, so the matrix-vector re-solve runs
 * (lets tests reach that path).  PR_EINVAL for unknown bits. */
#define PR_DEBUG_GRAM_RECHECK 1
/* PR_DEBUG_FORCE_BATCH: pr_solve_batch on a context with the batched path
 * always iterates the nodes together to the end, also where its cost estimate
 * would run a small round, or the last nodes of a round, one at a time. */
#define PR_DEBUG_FORCE_BATCH 2
int pr_ctx_set_debug(pr_ctx *ctx, int32_t flags);
/* Cached estimate of ||X||_2^2 (largest eigenvalue of X^T X). */
int pr_ctx_norm2(pr_ctx *ctx, double *norm2_out);

/* Least squares from the Gram matrix.  Precomputes G = X^T X (p x p, FP64
 * MFMA over the stored X, kept in device memory: 8 p^2 bytes), b = X^T y and
 * y^T y, and from then on runs every pr_solve of the context as
 *   h = b - G_S x_S  (a column-list product over the support of x)
 * in place of the two matrix-vector products X x and X^T r: F(X x) =
 * y^T y - x^T (b + h) and -F*(-zeta) = 2 (y^T y - b^T x) - F for zeta =
 * 2 (y - X x), the same iteration in exact arithmetic.  At the end of each
 * solve the reported bounds are recomputed over the stored X (pr_dual_bound)
 * and a decision they do not confirm is redone on the matrix-vector path
 * from the best iterate (that run's bounds and zeta are then returned; iters
 * and restarts count both runs).
 * On a context with the batched path, pr_solve_batch then runs one product
 * U = G X_it per iteration (FP64 MFMA over the m current iterates; its
 * reduction split is autotuned here) in place of its two products with X, and
 * h = b - U; every stopped node is still recertified over the stored X.
 * Requires least squares, p a multiple of 128 and at most 16384, n a multiple
 * of 32; PR_EINVAL otherwise, PR_ENOMEM if G does not fit. */
int pr_ctx_enable_gram(pr_ctx *ctx);

/* Solve one node relaxation (Sections 3.3 and 4): FISTA steps
 * x = prox_{(2 lambda2 / L) g_N}(y - grad/L) with the Algorithm 2 prox,
 * Phi with the Algorithm 1 value of g_N, Psi with the closed-form conjugate
 * (Lemma function_g_conjugate_in_BnB), restart when the gap falls by eta.
 *   beta0    device p or NULL (start at 0); any point is allowed, a point off
 *            dom g_N only makes the first primal value +inf (warm start).
 *   beta_out device p or NULL: the iterate attaining `primal`.
 *   zeta_out device n or NULL: the dual vector attaining lower_bound.
 *   out      host. */
int pr_solve(pr_ctx *ctx, const pr_node *node, const pr_opts *opts, const double *beta0,
             double *beta_out, double *zeta_out, pr_result *out);

/* ---- The duality-gap restart beyond perspective relaxations: LASSO ------
 * (Section 5.2.)  Least squares F(u) = ||u - y||^2 on the context's X and y
 * with G = lam ||beta||_1 (PR_L1_REG) or G = the indicator of the l1-ball
 * ||beta||_1 <= lam (PR_L1_BALL), solved by FISTA with step 1/L and the
 * duality-gap restart of Section 3.3 (opts->method PR_FISTA_GAP, default) or
 * without it (PR_FISTA).  Dual points from zeta = -grad F(X beta) =
 * 2 (y - X beta): for PR_L1_REG zeta is scaled by s = min(1, lam /
 * ||X^T zeta||_inf) into dom G* (G* = indicator of ||w||_inf <= lam) and
 * Psi = s zeta^T y - s^2 ||zeta||^2 / 4; for PR_L1_BALL G*(w) = lam ||w||_inf
 * and Psi = zeta^T y - ||zeta||^2 / 4 - lam ||X^T zeta||_inf.  Prox: soft
 * thresholding at lam / L; Euclidean projection onto the l1-ball.
 *   beta0 device p or NULL; beta_out device p or NULL (iterate attaining
 *   primal); zeta_out device n or NULL (the scaled dual point attaining
 *   lower_bound); out host.  PR_EINVAL for a logistic context, kind outside
 *   the two forms, lam <= 0, or another method. */
#define PR_L1_REG 0
#define PR_L1_BALL 1
typedef struct {
  int32_t kind;  /* PR_L1_REG or PR_L1_BALL */
  int32_t pad0;
  double lam;    /* penalty weight, or the ball's radius */
} pr_lasso;

int pr_lasso_solve(pr_ctx *ctx, const pr_lasso *lasso, const pr_opts *opts, const double *beta0, double *beta_out,
                   double *zeta_out, pr_result *out);

/* prox_{rho g_N}(v) by the extended Moreau decomposition (eq. prox:gN) and
 * Algorithm 2, for the node given by `status` (device int8 p, PR_FREE /
 * PR_ZERO / PR_ONE) and cardinality k (kbar = k - |J1| clipped to |J_f|).
 *   v, out device p (may alias), rho > 0, M > 0 (or +inf).
 *   stream: hipStream_t or NULL.  Returns PR_EINVAL if |J1| > k. */
int pr_prox(void *stream, const double *v, int64_t p, double rho, int32_t k, double M,
            const int8_t *status, double *out);

/* prox_{rho g_N}(v) exactly as pr_prox (same kernel arithmetic, bit-identical
 * output), for callers that cannot allocate: code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Nothing is allocated, on
 * the device or the host: the workspace is a fixed device array of the
 * library, one copy per GPU, held until the process ends (8 bytes per
 * coordinate of PR_PROX_NOALLOC_MAX_P plus 256 bytes, 8 MiB).  |J1| and |J_f|
 * are counted on the device from `status`, so the host never reads it.
 *   Arguments as pr_prox; additionally p <= PR_PROX_NOALLOC_MAX_P.
 *   Returns PR_EINVAL for a bad argument, p > PR_PROX_NOALLOC_MAX_P, a status
 *   code outside {PR_FREE, PR_ZERO, PR_ONE} or |J1| > k (then `out` is not
 *   written), PR_EDEVICE for a HIP error.  Synchronises `stream`.
 * Every call on one GPU uses that GPU's single workspace: calls that overlap
 * in time on the same GPU (other streams or host threads) race and must be
 * serialised by the caller. */
#define PR_PROX_NOALLOC_MAX_P 1048576
int pr_prox_noalloc(void *stream, const double *v, int64_t p, double rho, int32_t k, double M,
                    const int8_t *status, double *out);

/* g_N(beta) by Algorithm 1 (+inf off dom g_N, tested with relative slack
 * 1e-9) and g_N*(alpha) by Lemma function_g_conjugate_in_BnB, each skipped
 * when its input pointer is NULL.  beta, alpha, status device p; outputs host. */
int pr_regularizer(void *stream, const double *beta, const double *alpha, int64_t p, int32_t k,
                   double M, const int8_t *status, double *g_out, double *gstar_out);

/* FP64 Fenchel dual bound Psi(zeta) = -F*(-zeta) - 2 lambda2 g_N*(X^T zeta /
 * (2 lambda2)) of eq. fenchel_dual for `node`, accumulated in FP64 over the
 * stored X values.  If zeta is NULL it is induced from beta as
 * zeta = -grad F(X beta) (Section 3.2).  If beta is non-NULL and primal_out
 * non-NULL, Phi(beta) is returned as well.
 *   zeta device n or NULL, beta device p or NULL (not both NULL),
 *   lb_out, primal_out host. */
int pr_dual_bound(pr_ctx *ctx, const pr_node *node, const double *zeta, const double *beta,
                  double *lb_out, double *primal_out);

/* Dense products with the context's X, FP64 accumulation (test and
 * measurement entry points; the solver uses the same kernels).
 *   pr_gemv:    u = X b,   b device p, u device n
 *   pr_gemv_t:  h = X^T r, r device n, h device p
 *   pr_gemv_t2: h1 = X^T r1 and h2 = X^T r2 in one pass over X (the
 *               transposed product of a logistic iteration, Section 3.2:
 *               X^T zeta at the iterate and X^T grad F at the momentum
 *               point); r1, r2 device n, h1, h2 device p, all distinct.
 * Return PR_EINVAL for NULL arguments. */
int pr_gemv(pr_ctx *ctx, const double *b, double *u);
int pr_gemv_t(pr_ctx *ctx, const double *r, double *h);
int pr_gemv_t2(pr_ctx *ctx, const double *r1, const double *r2, double *h1, double *h2);

/* Solve m nodes that share X (m <= max_batch), each as pr_solve would:
 * same bounds, stopping test, iteration variant and dynamic termination
 * (cutoff).  On a context with the batched path (created with max_batch > 1,
 * n and p multiples of 128, p <= 16384; either loss, X in any pr_dtype) the
 * nodes iterate together on FP64 MFMA products: the forward product of the
 * m iterates with X and one transposed product X^T R per iteration (least
 * squares: the residual rows; logistic: two rows per node, zeta at the
 * iterate and the loss gradient at the momentum point).  Every stopped
 * node's Phi and Psi are then recomputed over the stored X, and a node whose
 * decision (converged / prune / branch) is not confirmed continues alone on
 * the pr_solve path.  Other contexts run pr_solve node by node, and so does a
 * round whose measured per-iteration cost is lower one node at a time (the
 * batch's GEMMs at m active rows, timed at context creation, against m
 * single-node iterations: a 64-row MFMA tile costs as much for one node as
 * for 64); by the same measure, once the nodes still iterating are that few,
 * they leave the batch and finish on the single-node path from their current
 * iterates (their iters / restarts / trials count both parts).  Every
 * iteration variant but AC-FGM (which runs node by node) runs batched, the
 * backtracking line search per node.  Traces (opts->trace) are not recorded.
 *   B0 device m x p (row i = warm start of node i) or NULL; B_out device
 *   m x p (row i receives node i's iterate) or NULL; out host m. */
int pr_solve_batch(pr_ctx *ctx, const pr_node *nodes, int32_t m, const pr_opts *opts,
                   const double *B0, double *B_out, pr_result *out);

/* Time the prox of g_N (as pr_prox) and the value g_N at its output (as
 * pr_regularizer) with HIP events on `stream`: one untimed launch, then `reps`
 * back-to-back launches of each; *ms_prox, *ms_g = elapsed / reps.  out
 * (device, p) receives prox_{rho g_N}(v).  The workspace is allocated before
 * and freed after the timed launches.  Arguments and errors as pr_prox. */
int pr_time_prox(void *stream, const double *v, int64_t p, double rho, int32_t k, double M, const int8_t *status,
                 double *out, int32_t reps, double *ms_prox, double *ms_g);

/* Time `reps` back-to-back launches of the X^T r kernel (the solver's
 * dominant kernel, same launch configuration) with HIP events on the
 * context stream; *ms_avg = elapsed / reps.  r device n, h device p.  On a
 * logistic context the kernel is timed in the two-right-hand-side form the
 * logistic solve runs ([X^T r, X^T r'] in one pass over X, r' a copy of r in
 * the context's workspace); h receives X^T r. */
int pr_time_gemv_t(pr_ctx *ctx, const double *r, double *h, int32_t reps, double *ms_avg);

/* Time `reps` back-to-back dense forward products u = X b (the column-list
 * product over all p columns and its summing kernel, as pr_gemv runs them)
 * with HIP events on the context stream; *ms_avg = elapsed / reps.
 * b device p, u device n.  PR_EINVAL for NULL arguments or reps < 1. */
int pr_time_gemv(pr_ctx *ctx, const double *b, double *u, int32_t reps, double *ms_avg);

/* The streaming-read rate that the HBM-bound kernels are measured against:
 * time `reps` back-to-back launches of a plain read of `bytes` bytes of the
 * device buffer `buf` (16-byte non-temporal loads, `blocks` workgroups of 256
 * threads striding over the buffer, `unroll` = 1 or 4 loads per lane in
 * flight) with HIP events on `stream`, after one untimed launch; *ms_avg =
 * elapsed / reps.  The buffer is only read (its contents are not changed) and
 * stays owned by the caller.  PR_EINVAL for a NULL or unaligned (16 B) buffer,
 * bytes not a positive multiple of 16, blocks outside [1, 2^20], another
 * unroll, reps < 1 or NULL ms_avg; PR_EDEVICE for a failed launch or event. */
int pr_time_read(const void *buf, int64_t bytes, int32_t blocks, int32_t unroll, int32_t reps, void *stream,
                 double *ms_avg);

/* Splits chosen by the context's batched-GEMM autotuner (run at context
 * creation): for i = 0 .. len-1, the number of reduction splits of the forward
 * and of the transpose GEMM when i+1 tiles of 64 rows are active (host arrays
 * of len entries).  PR_EINVAL if the context has no batched path. */
int pr_batch_tuning(pr_ctx *ctx, int32_t len, int32_t *ksf_out, int32_t *kst_out);

/* Time `reps` back-to-back launches of each of the two GEMMs of one
 * pr_solve_batch iteration for a batch of m nodes (forward U = Xit X^T, then
 * transpose H = R X) with all m rows active, in the launch configuration the
 * solve uses (split count, persistent grid, tile counter reset before each
 * launch), with HIP events on the context stream; *ms_fwd, *ms_t = elapsed /
 * reps.  The operands are the context's batch buffers (contents irrelevant to
 * timing).  PR_EINVAL unless the context was created with max_batch >= m. */
int pr_time_batch_gemm(pr_ctx *ctx, int32_t m, int32_t reps, double *ms_fwd, double *ms_t);

/* Batched Gram mode (pr_solve_batch after pr_ctx_enable_gram on a context
 * with the batched path): each iteration's one product U = G X_it (FP64 MFMA,
 * X_it the m current iterates) replaces the two products with X.  Time `reps`
 * back-to-back launches of that product for m active rows in the solve's
 * configuration (autotuned split, persistent grid), HIP events on the context
 * stream; *ms = elapsed / reps.  PR_EINVAL unless Gram mode is on, the
 * context has the batched path and max_batch >= m. */
int pr_time_gram_gemm(pr_ctx *ctx, int32_t m, int32_t reps, double *ms);

/* Support-union compaction of the batched product with the iterates (G X_it
 * in Gram mode, X_it X^T otherwise): after the first graph launch of
 * pr_solve_batch, the union U of the iterates' supports is taken; while its
 * size padded to the GEMM's reduction granule (*kp) is at most 3/4 of p, each
 * product runs over the kp columns of U only (G[:, U] X_it[U, :], X_it[:, U]
 * X[:, U]^T), plus the (few) nonzeros outside U added column by column, so
 * the result is the full product up to summation order.  Reports |U| (*ku), *kp
 * and the number of nonzeros outside U summed over the nodes' last iterates
 * (*nout) of the last pr_solve_batch on this context, all 0 when it ran
 * without the compaction.  ku, kp, nout: host. */
int pr_batch_union_size(pr_ctx *ctx, int64_t *ku, int64_t *kp, int64_t *nout);

/* FP64 MFMA product used by pr_solve_batch for both of its matrix products
 * (test and measurement entry point): C[z][r][c] = sum over k in split z of
 * A[c][k] * B[r][k].  A is Mc x K, row-major BF16 bit patterns (uint16,
 * converted exactly), leading dimension lda (multiple of 8); B is Nr x K,
 * row-major FP64, leading dimension ldb (even); FP64 accumulation, output C
 * FP64, KS x Nr x Mc (one plane per split of the reduction dimension into KS
 * equal parts).  Requires Mc a multiple of 128, Nr of 64, K of 32*KS; A and
 * B 16-byte aligned.  A, B, C device; the launch is enqueued on `stream`
 * (hipStream_t or NULL) and not waited for.  PR_EINVAL on a violated
 * requirement (nothing is launched). */
int pr_gemm(void *stream, const uint16_t *A, int64_t lda, const double *B, int64_t ldb, double *C, int64_t Mc,
            int64_t Nr, int64_t K, int32_t KS);

/* ---- Branch and bound -------------------------------------------------
 * Best-first branch and bound for problem (1), least-squares or logistic
 * loss, built on pr_solve_batch (one node at a time where the context has no
 * batched path): every node bound is the certified FP64 bound of its
 * perspective relaxation, solved with dynamic termination against the
 * incumbent (Section 5.3).  Branching on the free coordinate with the largest
 * |beta_j| of the node's relaxation solution (children: fixed to one, fixed to
 * zero), children warm-started from the parent's solution.  Incumbents on the
 * support S = J1 + the kbar largest free |beta_j| of each relaxation solution:
 * pr_solve on the leaf node J1 = S, J0 = the rest, to a 1e-9 relative gap
 * (there the relaxation is problem (1) restricted to S, the box-constrained
 * fit on S), each support once; a node with nothing left to branch on is
 * such a leaf and is offered as an incumbent before it is fathomed. */
#define PR_BNB_OPTIMAL 1     /* (UB - LB) / |UB| <= rel_gap_tol */
#define PR_BNB_NODE_LIMIT 2
#define PR_BNB_TIME_LIMIT 3

typedef struct {
  double rel_gap_tol;   /* stop when (UB - LB) / |UB| <= this; default 1e-4 */
  double time_limit_s;  /* wall-clock limit; default +inf */
  int32_t max_nodes;    /* node relaxations solved at most; default 100000 */
  int32_t batch;        /* nodes per pr_solve_batch call; 0 = the context's max_batch */
  pr_opts node_opts;    /* options of every node relaxation (cutoff and trace are set by pr_bnb) */
} pr_bnb_opts;

typedef struct {
  double lower_bound;   /* certified: min over open nodes (= upper_bound when the tree is closed) */
  double upper_bound;   /* objective of the incumbent (a feasible k-sparse point) */
  double rel_gap;
  double seconds;       /* wall clock of the call */
  double relaxation_seconds; /* of which inside pr_solve_batch */
  int64_t nodes_solved, nodes_pruned, nodes_open;
  int32_t max_depth, status; /* PR_BNB_OPTIMAL / PR_BNB_NODE_LIMIT / PR_BNB_TIME_LIMIT */
} pr_bnb_result;

void pr_bnb_opts_default(pr_bnb_opts *opts);

/* Run branch and bound from `root` (its J0 / J1 are kept in every node).
 * beta_best: device p or NULL, receives the incumbent.  out: host.  PR_EINVAL
 * for bad options; node errors as pr_solve. */
int pr_bnb(pr_ctx *ctx, const pr_node *root, const pr_bnb_opts *opts, double *beta_best, pr_bnb_result *out);

/* ---- Learned warm start for child nodes --------------------------------
 * Not part of the paper's method (which warm-starts a child from its
 * parent's solution).  A per-coordinate network proposes how each coordinate
 * of a child's solution differs from the parent's; pr_mlp_warm_start keeps the
 * proposal only if its FP64 duality gap on the child is below the parent
 * solution's, so no bound ever depends on the network.
 *
 * Network 8 -> 64 -> 64 -> 1 with ReLU.  Parameters: one flat FP32 device
 * vector of PR_MLP_NPARAM values, W1 (64 x 8) | b1 (64) | W2 (64 x 64) |
 * b2 (64) | w3 (64) | b3, weights row-major (out = w3 . relu(W2 relu(W1 f +
 * b1) + b2) + b3).  The kernels round weights and hidden activations to BF16
 * for the MFMA products and accumulate in FP32.
 *
 * Features (one row of PR_MLP_NFEAT BF16 values per coordinate j of a child
 * node, from the parent solution beta): beta_j; w_j / max_i |w_i| with
 * w = X^T zeta, zeta = -grad F(X beta) (0 if w = 0); #{i : |beta_i| >
 * |beta_j|} / p; the child's status of j (-1 fixed to zero, 0 free, +1 fixed
 * to one); lambda2; |J1| / k; |J0| / k; kbar / k. */
#define PR_MLP_NFEAT 8
#define PR_MLP_NPARAM 4801

/* Feature rows of m child nodes (host array nodes[m]) from their parents'
 * solutions Bparent (device, m x p FP64, row i = parent of node i).  F
 * (device, m x p x 8 BF16 bit patterns, 16-byte aligned) receives the rows,
 * node-major.  If Bchild (device, m x p) is given, T (device, m x p FP32)
 * receives the training targets Bchild - Bparent.  Synchronises the context
 * stream.  PR_EINVAL / PR_EOVERLAP as pr_solve for a malformed node. */
int pr_mlp_features(pr_ctx *ctx, const pr_node *nodes, int32_t m, const double *Bparent, const double *Bchild,
                    uint16_t *F, float *T);

/* out[r] = network output for feature row r, r < rows (device buffers, F
 * 16-byte aligned).  Enqueued on `stream`, not waited for. */
int pr_mlp_forward(void *stream, const float *params, const uint16_t *F, int64_t rows, float *out);

/* Number of floats of device workspace pr_mlp_grad needs for `rows` rows. */
int64_t pr_mlp_workspace(int64_t rows);

/* Gradient of the mean squared error (1/rows) sum_r (out_r - T_r)^2 with
 * respect to the parameters: grad (device, PR_MLP_NPARAM + 1 floats) receives
 * the gradient and, in its last entry, the loss.  work: device workspace of
 * pr_mlp_workspace(rows) floats.  The sum over rows is in a fixed order (the
 * result is deterministic).  Enqueued on `stream`, not waited for. */
int pr_mlp_grad(void *stream, const float *params, const uint16_t *F, const float *T, int64_t rows, float *work,
                float *grad);

/* One Adam step (step counts from 1, bias-corrected) on the FP32 master
 * parameters, with first / second moment vectors m1, m2 (device,
 * PR_MLP_NPARAM floats each, zero before step 1).  Enqueued on `stream`. */
int pr_mlp_adam(void *stream, float *params, const float *grad, float *m1, float *m2, int32_t step, double lr,
                double beta1, double beta2, double eps);

/* Starting points for m child nodes, judged by the FP64 duality gap
 * Phi(x) - Psi(zeta(x)) on the child (+inf outside the domain): B0 row i
 * (device, m x p FP64) receives whichever of these has the smallest gap:
 *   0  the parent solution beta_parent (row i of Bparent),
 *   1  prox_{rho g_N}(beta_parent), rho = 2 lambda2 / L (the solver's default
 *      step): the judged start without the network,
 *   2  prox_{rho g_N}(beta_parent + network output) (only with params).
 * choice (host, m, optional) receives that index; gaps (host, 3m, optional)
 * the three gaps per node in that order (+inf for a candidate not built or an
 * infeasible node, which keeps its parent).  On a context with the batched
 * path and m <= max_batch all children are evaluated together (gaps from the
 * batch's FP64 products over the stored X); otherwise one at a time.
 * Synchronises the context stream. */
int pr_mlp_warm_start(pr_ctx *ctx, const pr_node *nodes, int32_t m, const float *params, const double *Bparent,
                      double *B0, int32_t *choice, double *gaps);

const char *pr_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* PR_H */
