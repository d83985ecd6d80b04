// Internal declarations shared by the kernel and host translation units of
// libpr.  Not part of the public ABI (include/pr.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/pr.h"

namespace pr {

constexpr int kNodeThreads = 512;    // threads of a per-node workgroup
constexpr int kGemvThreads = 256;    // 4 waves of the X^T r kernel
constexpr int kSpChunksMax = 16;     // column chunks of the column-list product at most
constexpr int kSpChunksFill = 64;    // ... and at most this many to give every compute unit a workgroup
constexpr int kCUs = 256;            // compute units of the target (MI355X)
constexpr int kSpThreads = 256;      // column-list GEMV workgroup

enum : int32_t { kFree = 0, kZero = 1, kOne = 2 };
enum : int32_t { kLsq = 0, kLogistic = 1 };
// Support lists of the register-resident node routines mark J1 and J0
// entries with these bits of the coordinate index (p < 2^29); readers mask
// them off.
constexpr int32_t kJ1Flag = 1 << 30;
constexpr int32_t kJ0Flag = 1 << 29;
constexpr int32_t kIdxMask = kJ0Flag - 1;
enum : int32_t { kF64 = 0, kF32 = 1, kBF16 = 2 };
enum : int32_t { kConverged = 1, kMaxIter = 2, kInfeasible = 3, kCutoffPrune = 4, kCutoffBranch = 5 };

// Per-node constants, device resident (written by the host before a solve).
// iteration variants (pr_opts.method)
enum { kFistaGap = 0, kFista = 1, kFistaFv = 2, kPgd = 3, kAcfgmGap = 4, kAcfgm = 5, kFistaBtGap = 6, kFistaBt = 7 };
// FISTA with backtracking (with or without the gap restart)
__host__ __device__ inline bool is_bt(int method) { return method == kFistaBtGap || method == kFistaBt; }

struct NodeParams {
  const int8_t *st;   // status, p entries
  // the same status packed 2 bits per entry for the register-resident step:
  // word q * kNodeThreads + t holds entries j = t + (16 q + i) * kNodeThreads,
  // i = 0 .. 15, in bits 2i, 2i + 1 (3 = beyond p)
  const uint32_t *stp;
  int64_t p, pbar;
  int32_t kbar, loss;
  double lambda2, M, eta, tol, cutoff;  // cutoff NaN = off
  int32_t max_iter, method;             // method: kFistaGap .. kFistaBt
  double *trace;                        // optional: (Phi, Psi) of iterates 0 .. max_iter
  // backtracking (kFistaBt*): initial step constant (and after each restart),
  // cap (a Lipschitz constant of grad f: a trial at Lmax is accepted), growth
  double L0, Lmax, ls_c;
  // least squares from the Gram matrix (NULL: from the matrix-vector products):
  // b = X^T y, yy = y^T y; h = b - G x arrives in place of X^T r
  const double *gram_b;
  double gram_yy;
};

// Per-node iteration state, device resident.
struct NodeState {
  double L;        // step constant
  double t;        // FISTA momentum parameter
  double gap_ref;  // gap at the start of the current restart epoch
  double lb, ub;   // best dual / primal values
  double phi, psi; // values at the current iterate
  double rel_gap;
  double gval;     // g_N at the current iterate (Algorithm 1)
  double tau;      // last pooled-block threshold of the prox (warm start)
  double mom;      // momentum coefficient used by the last step
  int32_t iter, restarts, done, status;
  int32_t parity;  // which of the two x buffers holds the current iterate
  int32_t nsupp;   // support size of the current iterate
  int32_t improved; // lb improved at the current iterate
  int32_t indom;   // current iterate lies in dom g_N
  int32_t tau_iters; // evaluations used by the last threshold search
  int32_t bt;      // backtracking method (the loss epilogue keeps the momentum point's X y)
  int32_t bt_acc;  // backtracking: the last evaluated point was accepted (or is the start point)
  int32_t trials;  // backtracking: rejected trials
  double tk;       // kbar-th largest free |w| of the dual at the last iterate (<= 0: none)
  double tkw;      // relative half-width of the selection window around tk
  double dxy;      // backtracking: ||x_trial - y||^2 of the pending trial
  double bt_A;     // backtracking, least squares: (x_trial - y)^T h(y), h(y) = -grad f(y) / 2
};

// Node-local vectors.
struct NodeBufs {
  double *x0, *x1;     // iterate buffers (current / previous by parity)
  double *xbest;       // iterate attaining the best primal value
  double *hprev;       // least squares: X^T r at the previous iterate
  double *vbuf;        // prox input
  double *abuf;        // magnitudes scratch (negative = not free)
  int32_t *sidx;       // support list of the current iterate
  double *sval;
  double *xlb;         // Gram mode: iterate whose dual vector attains the best Psi
  double *ybt, *gbt;   // backtracking: momentum point y of the pending trial and grad f(y)
};

// Shared per-problem vectors of a single-node solve.
struct ProbBufs {
  double *r;      // least squares residual y - X x; logistic: zeta
  double *gm;     // logistic: grad F at the momentum point
  double *ucur, *uprev; // logistic: X x at the current / previous iterate
  double *zbest;  // dual vector attaining lb
  double *h1, *h2;      // X^T (first / second right-hand side)
  double *part;   // column-list GEMV partial sums [nch][n]
  double *rbsum;  // per finalize-block loss sums [nfin][2]
  double *uy;     // logistic backtracking: X y of the pending trial's momentum point
  double *dsum;   // logistic backtracking: per finalize-block Bregman remainder [nfin]
  int32_t rb, nch, rows, nfin;
};

// Batched solve buffers (m nodes, node i's vectors at offset i * p).
struct BatchBufs {
  int32_t m, Nr, nfb;     // nodes, GEMM rows (m padded to 64), residual row blocks
  int32_t NrT, rs;        // rows of the planes the step reads (rs per node: logistic 2, else 1), padded to 64
  int32_t loss;
  const int32_t *ksp;     // device: number of X^T R partial planes written this iteration
  double *x0, *x1, *xbest, *hprev;
  int32_t *sidx;
  double *sval;
  const double *CT;   // [*ksp][NrT][p] partial products X^T r (logistic: rows 2q = X^T zeta, 2q+1 = the
                      // gradient at the momentum point; Gram mode: G x)
  const double *fsum; // [m][nfb][2] partial sums of F(X x) and -F*(-zeta)
  double *Bx;         // [Nr][p] current iterates (rows of the forward GEMM)
  int32_t *active;    // number of nodes not yet done
  double gap_factor;  // stop when Phi - Psi <= gap_factor * tol * |Phi| (margin for the host re-check)
  int64_t p;
  const uint32_t *stp;  // packed status of the nodes (NodeParams::stp layout), stpw words per node
  int64_t stpw;
  const double *gb;     // Gram mode: b = X^T y (NULL: products over X); gyy = y^T y
  double gyy;
  double *ybt, *gbt;    // backtracking: per node the momentum point of the pending trial and grad f there [m][p]
  const double *dsum;   // logistic backtracking: per (node, residual block) Bregman remainder [m][nfb]
};

// AC-FGM state of a single-node solve (pr_variants.hip), device resident.
struct AcState {
  double L1;         // first-step curvature estimate (line search)
  double gap_ref;    // gap at the start of the current epoch
  double eta_cur, tau_cur;  // step size and tau that produced the point being evaluated
  double eta_prev, tau_prev, lhat_prev;  // of the last accepted step
  int32_t step;      // epoch step index t of the point being evaluated (0: the start point)
  int32_t rejected;  // first-step trials rejected by the line search
};
// AC-FGM vectors: base (accepted) point x_b, its gradient g_b and prox centre
// y_b; the evaluated point x_c with its y_c and z; the support list of x_c
// (scratch of the Algorithm 1 evaluation); X z and X x_c (n).
struct AcBufs {
  double *xb, *gb, *yb, *xc, *yc, *z;
  int32_t *sidx2;
  double *sval2;
  double *uz, *ucur;
};
// LASSO state beside NodeState: the scale s of the last dual point, of the best one.
struct LassoState {
  double zscale, zscale_best;
};

struct Problem {
  const void *X;
  int32_t xdt, loss;
  const double *y;
  int64_t n, p;
};

// ---- host helpers (pr_api.hip) ----
// Validate a node and build its status vector; *infeasible when |J1| > k.
int build_status(const pr_node *node, int64_t p, std::vector<int8_t> &st, int64_t &n1, int64_t &pbar,
                 int32_t &kbar, bool &infeasible);
const Problem &ctx_problem(const pr_ctx *c);
hipStream_t ctx_stream(const pr_ctx *c);
int32_t ctx_max_batch(const pr_ctx *c);

// ---- kernel launchers ----
// With `node` (and S, the node's support list sidx / sval of length *nlist),
// one extra workgroup evaluates g_N and the dom test of the listed iterate
// into S->gval / S->indom beside the product.  With `node` and dsum
// (backtracking), a trial the model test rejects (bt_accept over the loss
// epilogue's remainder sums) skips the product: its step is redone from the
// saved momentum point without it.
hipError_t launch_gemv_t(const Problem &P, const double *r1, const double *r2, double *h1, double *h2,
                         const int32_t *done, hipStream_t s, const NodeParams *node = nullptr,
                         NodeState *S = nullptr, const int32_t *sidx = nullptr, const double *sval = nullptr,
                         const int32_t *nlist = nullptr, const double *dsum = nullptr, int32_t nfin = 0);
// u_partials / finalize: generic column-list GEMV u = sum_t X[:, idx[t]] * val[t]
// followed by the per-row-block epilogue selected by `mode`.
enum SpMode : int32_t { kSpPlain = 0, kSpLsq = 1, kSpLogistic = 2, kSpGram = 3 };
hipError_t launch_read_stream(const void *buf, int64_t n16, int blocks, int unroll, hipStream_t s);
hipError_t launch_spfwd(const Problem &P, const ProbBufs &B, const int32_t *idx, const double *val,
                        const int32_t *nlist, int32_t mode, const NodeState *S, double *u_out,
                        hipStream_t s);
int spfwd_final_blocks(int64_t n);
int node_ept(int64_t p);  // entries per thread of the register-resident node kernels (0: strided)
hipError_t launch_node_init(const NodeParams *prm, NodeState *S, NodeBufs nb, const double *beta0,
                            double L, int64_t p, hipStream_t s);
// Per-context constants of the single-node step, fixed when the iteration
// graph is captured: p, the packed status (NodeParams::stp), Gram mode's b
// (NULL: matrix-vector mode) and which x buffer holds x^k in this unit (every
// graph launch runs an even number of units and starts at parity 0).
struct StepArgs {
  int64_t p;
  const uint32_t *stp;
  const double *gb;
  int32_t parity;
  int32_t bt;  // the backtracking variant of the step (pr_opts.method PR_FISTA_BT*)
};
hipError_t launch_node_step(const NodeParams *prm, NodeState *S, NodeBufs nb, const ProbBufs &B,
                            int64_t p, hipStream_t s, const StepArgs *a = nullptr);
hipError_t launch_batch_init(const NodeParams *prm, NodeState *S, BatchBufs bb, const double *B0, double L,
                             int64_t p, hipStream_t s);
hipError_t launch_batch_step(const NodeParams *prm, NodeState *S, BatchBufs bb, int64_t p, hipStream_t s);
// row-major copy out (n x p) of the column-major X of dtype xdt
hipError_t launch_transpose(int xdt, const void *in, void *out, int64_t n, int64_t p, hipStream_t s);
int batch_resid_blocks(int64_t n);
// loss side of the batch (least squares: R rows r; logistic: R rows 2q = zeta,
// 2q+1 = gradient at the momentum point while iterating, u kept in Uprev)
hipError_t launch_batch_resid(const double *U, const int32_t *ksp, int64_t n, int m, int Nr, const double *y,
                              double *R, double *fsum, const NodeState *S, int32_t loss, double *Uprev,
                              hipStream_t s, double *Ucur = nullptr, double *Uy = nullptr, double *dsum = nullptr);
hipError_t launch_gemm_f64(const uint16_t *A, int64_t lda, const double *B, int64_t ldb, double *C, int64_t Mc,
                           int64_t Nr, int64_t K, int KS, const int32_t *active, const int32_t *rowmap,
                           const int32_t *nrow, const int32_t *ksp, int ks_max, int32_t *counter, hipStream_t s);
// Same product with operand types adt, bdt in {kBF16, kF32, kF64}: supported
// pairs (BF16, FP64), (FP32, FP64), (BF16, BF16), (FP32, FP32), (FP64, FP64).
hipError_t launch_gemm_any(int adt, const void *A, int64_t lda, int bdt, const void *B, int64_t ldb, double *C,
                           int64_t Mc, int64_t Nr, int64_t K, int KS, const int32_t *active, const int32_t *rowmap,
                           const int32_t *nrow, const int32_t *ksp, int ks_max, int32_t *counter, hipStream_t s);
hipError_t launch_batch_rowmap(const NodeState *S, int m, int32_t *rowmap, int32_t *sp, int32_t *counters,
                               const int32_t *ftab, int ksf, int kst, int trow, int64_t kred, int64_t kfull, int rs,
                               int32_t *rowmap2, hipStream_t s);
hipError_t launch_union_mask(const double *Bx, int m, int64_t p, int32_t *mask, hipStream_t s);
hipError_t launch_gather_cols(const double *G, int64_t p, const int32_t *ulist, int64_t ku, int64_t kp, double *GU,
                              hipStream_t s);
hipError_t launch_union_compact(const double *Bx, int64_t p, const int32_t *rowmap, const int32_t *nrow, int Nr,
                                const int32_t *ulist, int64_t ku, int64_t kp, const int32_t *olist, int64_t no,
                                double *BxU, int32_t *ocnt, int32_t *oidx, double *oval, const int32_t *active,
                                hipStream_t s);
hipError_t launch_union_fix(const double *G, int64_t p, const int32_t *rowmap, const int32_t *nrow, int Nr,
                            const int32_t *ocnt, const int32_t *oidx, const double *oval, double *C,
                            const int32_t *active, hipStream_t s);
hipError_t launch_gather_cols_x(int xdt, const void *A, int64_t rows, int64_t p, const int32_t *ulist, int64_t ku,
                                int64_t kp, void *AU, hipStream_t s);
hipError_t launch_union_fix_x(int xdt, const void *X, int64_t n, int64_t p, const int32_t *rowmap, const int32_t *nrow,
                              int Nr, const int32_t *ocnt, const int32_t *oidx, const double *oval, double *C,
                              const int32_t *active, hipStream_t s);
hipError_t launch_batch_zeta(const double *R, int64_t n, int node, double *zeta, hipStream_t s);
// W[q][j] = scale * sum_z C[z][rs q][j] for q < m (C: [KS][Nr][p] split planes, rs rows per node)
hipError_t launch_sum_planes(const double *C, int KS, int Nr, int rs, int64_t p, int m, double scale, double *W,
                             hipStream_t s);
// prox of g_N for m nodes (params prm[q], rho_q = 2 lambda2_q invL), rows of V -> Xo; abuf m x p scratch
hipError_t launch_prox_batch(const NodeParams *prm, const double *V, double *Xo, double *abuf, int64_t p, int m,
                             double invL, hipStream_t s);
// batched-GEMM autotuner: split factors per count of active 64-row tiles,
// one table per product (forward, X^T R, Gram)
constexpr int kTuneMax = 64;            // table entries (row-tile counts 1 .. 63)
constexpr int kTuneTables = 3;
constexpr int kTuneReps = 2;            // timed launches per candidate
constexpr double kTunePlaneBW = 5.0e12; // B/s assumed for reading the split partial planes

// learned warm start
constexpr int kMlpPartStride = 4804;  // floats per block partial: 4801 gradient entries, loss, pad
struct FeatScalars {
  double lambda2;
  int32_t k, n0, n1, kbar;
};
int mlp_grid(int64_t rows, int *cpb);
hipError_t launch_mlp_forward(const float *P, const uint16_t *F, int64_t rows, float *out, hipStream_t s);
hipError_t launch_mlp_grad(const float *P, const uint16_t *F, const float *T, int64_t rows, float *part,
                           float *grad, hipStream_t s);
hipError_t launch_mlp_adam(float *P, const float *g, float *m1, float *m2, float lr, float beta1, float beta2,
                           float eps, float c1, float c2, hipStream_t s);
hipError_t launch_features(const double *beta, const double *w, const int8_t *st, int64_t p, double *nzv,
                           double *fs, FeatScalars sc, const double *beta_child, uint16_t *F, float *T,
                           hipStream_t s);
hipError_t launch_mlp_propose(const double *beta, const float *out, int64_t p, double *vhat, hipStream_t s);
hipError_t launch_zbest_final(const NodeState *S, const ProbBufs &B, int32_t loss, int64_t n,
                              hipStream_t s);
hipError_t launch_prox(const double *v, double *out, int64_t p, double rho, int32_t kbar, double M,
                       const int8_t *st, double *abuf, double *vtmp, hipStream_t s);
// prox with kbar counted on the device from st; *flag: 0 ok, 1 bad status
// code, 2 |J1| > k (out untouched unless 0).  abuf: p doubles of scratch.
hipError_t launch_prox_counted(const double *v, double *out, int64_t p, double rho, int32_t k, double M,
                               const int8_t *st, double *abuf, int32_t *flag, hipStream_t s);
hipError_t launch_regularizer(const double *beta, const double *alpha, int64_t p, int32_t kbar,
                              double M, const int8_t *st, double *abuf, double *out2,
                              hipStream_t s);
hipError_t launch_loss_terms(int32_t loss, const double *u, const double *y, int64_t n,
                             double *zeta_out, double *sums_out, hipStream_t s);
hipError_t launch_zeta_terms(int32_t loss, const double *zeta, const double *y, int64_t n,
                             double *sums_out, hipStream_t s);
hipError_t launch_sumsq(const double *v, int64_t n, double *out, hipStream_t s);
hipError_t launch_scale_copy(const double *src, double *dst, double a, int64_t n, hipStream_t s);
hipError_t launch_cert_batch(const NodeParams *prm, const double *Xit, const double *H, int KS, int Nr, int rs,
                             const double *fsum, int nfb, int64_t p, double *abuf, int32_t *sidx, double *sval,
                             double *out, int m, hipStream_t s);
hipError_t launch_lanczos(double *w, double *v, double *vprev, const double *alpha, const double *beta_prev,
                          double *beta_out, int64_t p, hipStream_t s);
hipError_t launch_iota(int32_t *idx, int64_t n, hipStream_t s);
// iteration variants (pr_variants.hip)
hipError_t launch_ac_init(const NodeParams *prm, NodeState *S, AcState *A, const AcBufs &ab, const NodeBufs &nb,
                          const double *beta0, double L0, hipStream_t s);
hipError_t launch_ac_resid(const Problem &P, const ProbBufs &B, const double *uz, double *ucur, const NodeState *S,
                           const AcState *A, hipStream_t s);
hipError_t launch_ac_step(const NodeParams *prm, NodeState *S, AcState *A, const AcBufs &ab, const NodeBufs &nb,
                          const ProbBufs &B, double b, double c, int32_t restart_gap, hipStream_t s);
hipError_t launch_lasso_init(NodeState *S, LassoState *LX, const NodeBufs &nb, const double *beta0, int64_t p,
                             int32_t kind, double lam, double L, hipStream_t s);
hipError_t launch_lasso_step(const NodeParams *prm, NodeState *S, LassoState *LX, const NodeBufs &nb,
                             const ProbBufs &B, int32_t kind, double lam, hipStream_t s);

}  // namespace pr
