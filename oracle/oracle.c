/*
 * oracle.c -- plain, slow FP64 reference for the perspective-relaxation hot path
 * of "GPU-friendly and Linearly Convergent First-order Methods for Certifying
 * Optimal k-sparse GLMs" (arXiv 2603.01306).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP path.
 *
 * Everything is IEEE double, round-to-nearest, evaluated in the order the
 * paper states it.  Library primitives used as single steps: qsort (the sorts
 * of Algorithms 1 and 2), libm (exp, log1p, sqrt).  Matrix-vector products
 * are the textbook loops for a column-major matrix, parallelised with OpenMP
 * over independent outputs only (each output is summed in index order by one
 * thread, so results do not depend on the thread count).
 *
 * Notation follows the paper: node status s_j in {free (J_f), fixed zero
 * (J_0), fixed one (J_1)}, pbar = |J_f|, kbar = k - |J_1| (clipped to pbar),
 * F(u) = f(u, y), G = 2*lambda2*g_N, Phi(beta) = F(X beta) + G(beta),
 * Psi(zeta) = -F*(-zeta) - G*(X^T zeta).
 *
 * Readings where the paper is silent (loss scaling, M convention, rounding,
 * relative-gap denominator, restart operands) are listed in the design notes;
 * each function below names the passage it follows.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_FREE 0
#define ORC_ZERO 1 /* J_0: z_j fixed to 0 */
#define ORC_ONE 2  /* J_1: z_j fixed to 1 */

#define ORC_LSQ 0
#define ORC_LOGISTIC 1

#define ORC_F64 0
#define ORC_F32 1
#define ORC_BF16 2

#define ORC_CONVERGED 1
#define ORC_MAXITER 2
#define ORC_INFEASIBLE 3
#define ORC_CUTOFF_PRUNE 4
#define ORC_CUTOFF_BRANCH 5

/* ---------------------------------------------------------------- helpers */

/* Stored matrix entry, exactly upcast to double. */
static double xat(const void *X, int xdt, int64_t idx) {
  if (xdt == ORC_F64) return ((const double *)X)[idx];
  if (xdt == ORC_F32) return (double)((const float *)X)[idx];
  /* bf16: the 16 stored bits are the top half of an IEEE float */
  uint32_t bits = ((uint32_t)((const uint16_t *)X)[idx]) << 16;
  float f;
  memcpy(&f, &bits, sizeof f);
  return (double)f;
}

static int cmp_desc(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x < y) - (x > y);
}

/* Huber function H_M of eq. (huber_loss_in_bnb), Section 4.1. */
double orc_huber(double a, double M) {
  double x = fabs(a);
  if (x <= M) return 0.5 * x * x;
  return M * x - 0.5 * M * M;
}

/* prox_{c H_M}(u) = argmin_a 0.5 (a-u)^2 + c H_M(a), c >= 0 (used by
 * Algorithm 2).  Quadratic branch while |u| <= M(1+c), else a shifted copy. */
double orc_prox_huber(double u, double c, double M) {
  double x = fabs(u), r;
  if (x <= M * (1.0 + c)) r = x / (1.0 + c);
  else r = x - c * M;
  return u < 0 ? -r : r;
}

/* Partition sizes of a node (Section 2.3, domain D): returns -1 when
 * |J_1| > k (empty domain, the node is infeasible). */
int orc_node_dims(const int8_t *st, int64_t p, int32_t k, int64_t *pbar, int64_t *kbar) {
  int64_t n1 = 0, nf = 0;
  for (int64_t j = 0; j < p; j++) {
    if (st[j] == ORC_ONE) n1++;
    else if (st[j] == ORC_FREE) nf++;
  }
  if (n1 > (int64_t)k) return -1;
  int64_t kb = (int64_t)k - n1;
  if (kb > nf) kb = nf;
  *pbar = nf;
  *kbar = kb;
  return 0;
}

/* --------------------------------------------------- regulariser g_N, g_N* */

/* g_N(beta) for beta in dom g_N, from Theorem compute_g_value (Section 4.2):
 * g_N(beta) = 1/2 sum_{J_1} beta_j^2 + 1/2 min sum_{j <= kbar} omega_j^2 over
 * non-increasing omega >= 0 supported on the first kbar positions that
 * majorise the sorted free magnitudes q_1 >= q_2 >= ... (q = |beta_{J_f}|).
 * The minimiser fills the kbar slots to a common water level s where it can:
 * omega_j = max(q_j, s), j <= kbar, with s the root of
 *     phi(s) = sum_{j <= kbar} max(q_j, s) - theta = 0,   theta = sum_j q_j,
 * (equal total, as majorisation requires; the partial-sum conditions hold
 * because omega dominates q term by term on the first kbar positions and the
 * tail of q is below s).  phi is non-decreasing and piecewise linear with
 * breakpoints at the q_j; phi(q_j) = sum_{i < j} q_i + (kbar - j + 1) q_j -
 * theta is non-increasing in j and phi(q_kbar) = phi(0) <= 0, so the number
 * of entries above the level is m = #{j <= kbar : phi(q_j) > 0} and on that
 * piece s = (theta - sum_{j <= m} q_j) / (kbar - m).  A full sort (a library
 * primitive) orders q. */
double orc_g(const double *beta, const int8_t *st, int64_t p, int32_t k) {
  int64_t pbar, kbar;
  if (orc_node_dims(st, p, k, &pbar, &kbar) < 0) return INFINITY;
  double s1 = 0.0, theta = 0.0;
  double *q = (double *)malloc(sizeof(double) * (size_t)(pbar > 0 ? pbar : 1));
  int64_t nq = 0;
  for (int64_t j = 0; j < p; j++) {
    if (st[j] == ORC_ONE) s1 += beta[j] * beta[j];
    else if (st[j] == ORC_FREE) q[nq++] = fabs(beta[j]);
  }
  qsort(q, (size_t)nq, sizeof(double), cmp_desc);
  /* theta summed in sorted order, the order of the partial sums below: adding
     non-negative terms never decreases a rounded sum, so phi(q_kbar) <= 0
     holds in floating point too and m < kbar */
  for (int64_t j = 0; j < nq; j++) theta += q[j];
  double free_part = 0.0;
  if (kbar > 0 && theta > 0.0) {
    /* m = number of leading entries kept above the water level */
    int64_t m = 0;
    double head = 0.0; /* sum of the first j - 1 sorted magnitudes */
    for (int64_t j = 0; j < kbar; j++) {
      const double phi_j = head + (double)(kbar - j) * q[j] - theta;
      if (phi_j > 0.0) m = j + 1;
      head += q[j];
    }
    double kept = 0.0, kept_sq = 0.0;
    for (int64_t j = 0; j < m; j++) {
      kept += q[j];
      kept_sq += q[j] * q[j];
    }
    const double level = (theta - kept) / (double)(kbar - m);
    free_part = kept_sq + (double)(kbar - m) * level * level;
  }
  free(q);
  return 0.5 * s1 + 0.5 * free_part;
}

/* Membership test for dom g_N (Section 2.3, domain D; Lemma
 * g_is_proper_closed_and_convex): beta_J0 = 0, |beta_j| <= M, and the free
 * part fits in M times the kbar-sparse simplex, i.e. sum_{J_f} |beta_j| <=
 * M kbar (with kbar = 0 forcing beta_Jf = 0).  rtol absorbs round-off of the
 * point being tested. */
int orc_in_dom(const double *beta, const int8_t *st, int64_t p, int32_t k, double M, double rtol) {
  int64_t pbar, kbar;
  if (orc_node_dims(st, p, k, &pbar, &kbar) < 0) return 0;
  double amax = 0.0, l1 = 0.0;
  for (int64_t j = 0; j < p; j++) amax = fmax(amax, fabs(beta[j]));
  double zt = rtol * fmax(1.0, amax);
  for (int64_t j = 0; j < p; j++) {
    double b = fabs(beta[j]);
    if (st[j] == ORC_ZERO) {
      if (b > zt) return 0;
      continue;
    }
    if (isfinite(M) && b > M * (1.0 + rtol)) return 0;
    if (st[j] == ORC_FREE) l1 += b;
  }
  if (kbar == 0) return l1 <= zt;
  if (isfinite(M) && l1 > M * (double)kbar * (1.0 + rtol)) return 0;
  return 1;
}

/* Closed-form conjugate of Lemma function_g_conjugate_in_BnB:
 * g_N*(alpha) = sum_{J_1} H_M(alpha_j) + TopSum_{kbar}(H_M(alpha_{J_f})).
 * J_0 coordinates do not enter.  An empty domain gives -infinity. */
double orc_gstar(const double *alpha, const int8_t *st, int64_t p, int32_t k, double M) {
  int64_t pbar, kbar;
  if (orc_node_dims(st, p, k, &pbar, &kbar) < 0) return -INFINITY;
  double s = 0.0;
  double *h = (double *)malloc(sizeof(double) * (size_t)(pbar > 0 ? pbar : 1));
  int64_t m = 0;
  for (int64_t j = 0; j < p; j++) {
    if (st[j] == ORC_ONE) s += orc_huber(alpha[j], M);
    else if (st[j] == ORC_FREE) h[m++] = orc_huber(alpha[j], M);
  }
  qsort(h, (size_t)m, sizeof(double), cmp_desc);
  for (int64_t j = 0; j < kbar; j++) s += h[j];
  free(h);
  return s;
}

typedef struct {
  int64_t lo, hi; /* positions in sorted order, inclusive */
  double sum_rho, sum_xi, value;
} orc_block;

typedef struct {
  double key;
  int64_t idx;
} orc_keyidx;

static int cmp_keyidx_desc(const void *a, const void *b) {
  const orc_keyidx *x = (const orc_keyidx *)a, *y = (const orc_keyidx *)b;
  if (x->key > y->key) return -1;
  if (x->key < y->key) return 1;
  return (x->idx > y->idx) - (x->idx < y->idx);
}

/* Algorithm 2 (Section 4.2, Theorem evaluate_prox_g_algorithm_correctness):
 * prox_{rho g_N*}(b).  The free part is sorted by magnitude with permutation
 * pi, every sorted position gets weight rho (first kbar positions) or 0, each
 * position is first sent through prox_{rho_j H_M}, and adjacent blocks whose
 * values increase are pooled (pool-adjacent-violators) with block value
 * prox_{rhobar H_M}(xibar), rhobar and xibar being block means.  The pooling
 * here is the usual left-to-right stack; the pooled solution of this
 * isotonic problem is unique, so any merge order yields it.  The sort and
 * the pooling act on magnitudes and the signs of b are restored at the end.
 * J_0 coordinates are returned unchanged, J_1 ones through prox_{rho H_M}. */
void orc_prox_gstar(const double *b, const int8_t *st, int64_t p, double rho, int32_t k, double M,
                    double *out) {
  int64_t pbar, kbar;
  if (orc_node_dims(st, p, k, &pbar, &kbar) < 0) {
    for (int64_t j = 0; j < p; j++) out[j] = NAN;
    return;
  }
  orc_keyidx *srt = (orc_keyidx *)malloc(sizeof(orc_keyidx) * (size_t)(pbar > 0 ? pbar : 1));
  int64_t m = 0;
  for (int64_t j = 0; j < p; j++) {
    if (st[j] == ORC_ZERO) out[j] = b[j];
    else if (st[j] == ORC_ONE) out[j] = orc_prox_huber(b[j], rho, M);
    else {
      srt[m].key = fabs(b[j]);
      srt[m].idx = j;
      m++;
    }
  }
  qsort(srt, (size_t)m, sizeof(orc_keyidx), cmp_keyidx_desc);
  orc_block *stk = (orc_block *)malloc(sizeof(orc_block) * (size_t)(m > 0 ? m : 1));
  int64_t top = -1;
  for (int64_t j = 0; j < m; j++) {
    double rj = (j < kbar) ? rho : 0.0;
    top++;
    stk[top].lo = j;
    stk[top].hi = j;
    stk[top].sum_rho = rj;
    stk[top].sum_xi = srt[j].key;
    stk[top].value = orc_prox_huber(srt[j].key, rj, M);
    while (top >= 1 && stk[top - 1].value < stk[top].value) {
      orc_block *a = &stk[top - 1], *c = &stk[top];
      a->hi = c->hi;
      a->sum_rho += c->sum_rho;
      a->sum_xi += c->sum_xi;
      double len = (double)(a->hi - a->lo + 1);
      a->value = orc_prox_huber(a->sum_xi / len, a->sum_rho / len, M);
      top--;
    }
  }
  for (int64_t t = 0; t <= top; t++) {
    for (int64_t j = stk[t].lo; j <= stk[t].hi; j++) {
      int64_t i = srt[j].idx;
      double s = (b[i] > 0) ? 1.0 : ((b[i] < 0) ? -1.0 : 0.0);
      out[i] = s * stk[t].value;
    }
  }
  free(stk);
  free(srt);
}

/* Extended Moreau decomposition, eq. (prox:gN):
 * prox_{rho g_N}(v) = v - rho prox_{rho^{-1} g_N*}(v / rho). */
void orc_prox_g(const double *v, const int8_t *st, int64_t p, double rho, int32_t k, double M,
                double *out) {
  double *w = (double *)malloc(sizeof(double) * (size_t)(p > 0 ? p : 1));
  double *a = (double *)malloc(sizeof(double) * (size_t)(p > 0 ? p : 1));
  for (int64_t j = 0; j < p; j++) w[j] = v[j] / rho;
  orc_prox_gstar(w, st, p, 1.0 / rho, k, M, a);
  for (int64_t j = 0; j < p; j++) out[j] = v[j] - rho * a[j];
  free(a);
  free(w);
}

/* ---------------------------------------------------------------- losses */

static double softplus(double z) { return fmax(z, 0.0) + log1p(exp(-fabs(z))); }

/* F(u) = f(u, y): least squares ||u - y||^2 (problem (1) carries no 1/2
 * or 1/n), logistic sum_i log(1 + exp(-y_i u_i)) with y_i in {-1, +1}. */
double orc_loss(int loss, const double *u, const double *y, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; i++) {
    if (loss == ORC_LSQ) s += (u[i] - y[i]) * (u[i] - y[i]);
    else s += softplus(-y[i] * u[i]);
  }
  return s;
}

/* gradient of F at u */
void orc_loss_grad(int loss, const double *u, const double *y, int64_t n, double *g) {
  for (int64_t i = 0; i < n; i++) {
    if (loss == ORC_LSQ) g[i] = 2.0 * (u[i] - y[i]);
    else g[i] = -y[i] / (1.0 + exp(y[i] * u[i]));
  }
}

/* -F*(-zeta), the loss part of the Fenchel dual (eq. fenchel_dual):
 * least squares zeta^T y - ||zeta||^2 / 4; logistic sum of binary entropies of
 * a_i = y_i zeta_i (-infinity if some a_i leaves [0, 1]), with 0 ln 0 = 0. */
double orc_neg_conj(int loss, const double *zeta, const double *y, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; i++) {
    if (loss == ORC_LSQ) {
      s += zeta[i] * y[i] - 0.25 * zeta[i] * zeta[i];
    } else {
      double a = y[i] * zeta[i];
      if (a < 0.0 || a > 1.0) return -INFINITY;
      if (a > 0.0) s -= a * log(a);
      if (a < 1.0) s -= (1.0 - a) * log1p(-a);
    }
  }
  return s;
}

/* ------------------------------------------------------- matrix products */

/* u = X b for column-major X (n x p, leading dimension n). */
void orc_matvec(const void *X, int xdt, int64_t n, int64_t p, const double *b, double *u) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    double s = 0.0;
    for (int64_t j = 0; j < p; j++) s += xat(X, xdt, i + j * n) * b[j];
    u[i] = s;
  }
}

/* h = X^T r */
void orc_rmatvec(const void *X, int xdt, int64_t n, int64_t p, const double *r, double *h) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < p; j++) {
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += xat(X, xdt, i + j * n) * r[i];
    h[j] = s;
  }
}

/* Largest eigenvalue of X^T X by the power method with Rayleigh quotient
 * ||X v||^2 / ||v||^2 (a lower estimate), started from the all-ones vector. */
double orc_power_norm2(const void *X, int xdt, int64_t n, int64_t p, int64_t max_iter, double tol) {
  double *v = (double *)malloc(sizeof(double) * (size_t)p);
  double *u = (double *)malloc(sizeof(double) * (size_t)n);
  /* start: entries of random sign and magnitude (xorshift64*, fixed seed), so
     that no eigenvector of X^T X is orthogonal to it except by accident; a
     constant start misses the top eigenvector of designs such as [A, -A] */
  uint64_t sx = 0x2545F4914F6CDD1Dull;
  double n0 = 0.0;
  for (int64_t j = 0; j < p; j++) {
    sx ^= sx >> 12;
    sx ^= sx << 25;
    sx ^= sx >> 27;
    const uint64_t r = sx * 0x2545F4914F6CDD1Dull;
    const double mag = 1.0 + (double)(r >> 11) / 9007199254740992.0; /* [1, 2) */
    v[j] = (r & 1u) ? -mag : mag;
    n0 += mag * mag;
  }
  for (int64_t j = 0; j < p; j++) v[j] /= sqrt(n0);
  double lam = 0.0;
  for (int64_t it = 0; it < max_iter; it++) {
    orc_matvec(X, xdt, n, p, v, u);
    double nu = 0.0;
    for (int64_t i = 0; i < n; i++) nu += u[i] * u[i];
    orc_rmatvec(X, xdt, n, p, u, v);
    double nv = 0.0;
    for (int64_t j = 0; j < p; j++) nv += v[j] * v[j];
    nv = sqrt(nv);
    if (nv == 0.0) {
      lam = nu;
      break;
    }
    for (int64_t j = 0; j < p; j++) v[j] /= nv;
    int stop = (it > 0 && fabs(nu - lam) <= tol * nu);
    lam = nu;
    if (stop) break;
  }
  free(u);
  free(v);
  return lam;
}

/* ---------------------------------------------------- primal and dual */

/* Phi(beta) = F(X beta) + 2 lambda2 g_N(beta), +infinity off dom g_N
 * (eq. composite reformulation, Section 2.4). */
double orc_primal(const void *X, int xdt, const double *y, int64_t n, int64_t p, int loss,
                  double lambda2, double M, int32_t k, const int8_t *st, const double *beta) {
  if (!orc_in_dom(beta, st, p, k, M, 1e-9)) return INFINITY;
  double *u = (double *)malloc(sizeof(double) * (size_t)n);
  orc_matvec(X, xdt, n, p, beta, u);
  double F = orc_loss(loss, u, y, n);
  free(u);
  return F + 2.0 * lambda2 * orc_g(beta, st, p, k);
}

/* Psi(zeta) = -F*(-zeta) - G*(X^T zeta), G*(w) = 2 lambda2 g_N*(w / (2 lambda2))
 * (eq. fenchel_dual; the scaling is the conjugate of G = 2 lambda2 g_N).
 * Weak duality makes this a valid lower bound for every zeta. */
double orc_dual(const void *X, int xdt, const double *y, int64_t n, int64_t p, int loss,
                double lambda2, double M, int32_t k, const int8_t *st, const double *zeta) {
  double *w = (double *)malloc(sizeof(double) * (size_t)p);
  orc_rmatvec(X, xdt, n, p, zeta, w);
  for (int64_t j = 0; j < p; j++) w[j] /= (2.0 * lambda2);
  double v = orc_neg_conj(loss, zeta, y, n) - 2.0 * lambda2 * orc_gstar(w, st, p, k, M);
  free(w);
  return v;
}

enum { ORC_FISTA_GAP = 0, ORC_FISTA = 1, ORC_FISTA_FV = 2, ORC_PGD = 3 };

/* ------------------------------------------------------------ solver */

/* FISTA (fixed step 1/L, Beck-Teboulle momentum) with the duality-gap
 * restart of Section 3.3 / "Restart in practice": at every iterate x^t the
 * induced dual zeta^t = -grad F(X x^t) (Section 3.2) gives Psi(zeta^t); the
 * method restarts (t <- 1, y <- x) as soon as Phi(x^t) - Psi(zeta^t) <=
 * (Phi - Psi at the epoch start) / eta, and stops when the best-so-far bounds
 * satisfy (UB - LB) / |UB| <= tol.  Dynamic termination against an incumbent
 * value (Section 5.3): Psi >= cutoff prunes, Phi <= cutoff branches.
 *
 * method selects the iteration compared in Section 5.2's convergence study:
 *   ORC_FISTA_GAP   FISTA with the duality-gap restart (the method above)
 *   ORC_FISTA       FISTA without restarts
 *   ORC_FISTA_FV    FISTA restarted whenever Phi increases (function-value
 *                   restart of O'Donoghue and Candes): t <- 1, y <- x
 *   ORC_PGD         proximal gradient, x <- prox(x - grad / L) (no momentum)
 * Every variant evaluates the same bounds and stopping test.
 *
 * res[0..7] = {LB, UB, rel_gap, L, iters, restarts, status, 0}.
 * trace (optional, length trace_cap) receives Phi - Psi at iterates 0, 1, ...
 * and phi_trace (optional, same length) Phi at those iterates.
 * restart_at (optional, length restart_cap) receives the iterate indices t at
 * which a restart was taken (the next step starts from x^t with t <- 1).
 * zeta_out receives the dual vector that attains LB.
 */
int orc_solve(const void *X, int xdt, const double *y, int64_t n, int64_t p, int loss, double lambda2,
              double M, int32_t k, const int8_t *st, double L, double tol, double eta, int64_t max_iter,
              double cutoff, const double *beta0, double *beta_out, double *zeta_out, double *res,
              double *trace, int64_t trace_cap, int method, double *phi_trace, int64_t *restart_at,
              int64_t restart_cap) {
  int64_t pbar, kbar;
  for (int i = 0; i < 8; i++) res[i] = 0.0;
  if (orc_node_dims(st, p, k, &pbar, &kbar) < 0) {
    res[0] = INFINITY;
    res[1] = INFINITY;
    res[6] = ORC_INFEASIBLE;
    for (int64_t j = 0; j < p; j++) beta_out[j] = 0.0;
    return ORC_INFEASIBLE;
  }
  if (L <= 0.0) {
    double s = orc_power_norm2(X, xdt, n, p, 2000, 1e-12);
    L = (loss == ORC_LSQ) ? 2.0 * s : 0.25 * s;
  }
  double *x = (double *)calloc((size_t)p, sizeof(double));
  double *xn = (double *)malloc(sizeof(double) * (size_t)p);
  double *yv = (double *)malloc(sizeof(double) * (size_t)p);
  double *gp = (double *)malloc(sizeof(double) * (size_t)p);
  double *u = (double *)malloc(sizeof(double) * (size_t)n);
  double *gn = (double *)malloc(sizeof(double) * (size_t)n);
  double *zeta = (double *)malloc(sizeof(double) * (size_t)n);
  if (beta0)
    for (int64_t j = 0; j < p; j++) x[j] = beta0[j];
  memcpy(yv, x, sizeof(double) * (size_t)p);
  double t = 1.0;

  /* evaluation of (Phi, Psi) at x */
#define ORC_EVAL(PHI, PSI)                                                     \
  do {                                                                         \
    orc_matvec(X, xdt, n, p, x, u);                                            \
    orc_loss_grad(loss, u, y, n, gn);                                          \
    for (int64_t i_ = 0; i_ < n; i_++) zeta[i_] = -gn[i_];                     \
    PSI = orc_dual(X, xdt, y, n, p, loss, lambda2, M, k, st, zeta);            \
    PHI = orc_in_dom(x, st, p, k, M, 1e-9)                                     \
              ? orc_loss(loss, u, y, n) + 2.0 * lambda2 * orc_g(x, st, p, k)   \
              : INFINITY;                                                      \
  } while (0)

  double Phi, Psi;
  ORC_EVAL(Phi, Psi);
  double LB = Psi, UB = Phi, gap_ref = Phi - Psi;
  memcpy(zeta_out, zeta, sizeof(double) * (size_t)n);
  if (trace && trace_cap > 0) trace[0] = Phi - Psi;
  if (phi_trace && trace_cap > 0) phi_trace[0] = Phi;
  double Phi_prev = Phi;
  int64_t it = 0, restarts = 0;
  int status = ORC_MAXITER;
  double rel = (UB - LB) / fmax(fabs(UB), 1e-300);
  if (rel <= tol) status = ORC_CONVERGED;
  else if (!isnan(cutoff) && LB >= cutoff) status = ORC_CUTOFF_PRUNE;
  else if (!isnan(cutoff) && UB <= cutoff) status = ORC_CUTOFF_BRANCH;
  while (status == ORC_MAXITER && it < max_iter) {
    it++;
    /* gradient of F(X .) at the momentum point */
    orc_matvec(X, xdt, n, p, yv, u);
    orc_loss_grad(loss, u, y, n, gn);
    orc_rmatvec(X, xdt, n, p, gn, gp);
    for (int64_t j = 0; j < p; j++) gp[j] = yv[j] - gp[j] / L;
    orc_prox_g(gp, st, p, 2.0 * lambda2 / L, k, M, xn);
    double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
    double mom = (method == ORC_PGD) ? 0.0 : (t - 1.0) / tn;
    for (int64_t j = 0; j < p; j++) {
      yv[j] = xn[j] + mom * (xn[j] - x[j]);
      x[j] = xn[j];
    }
    t = tn;
    ORC_EVAL(Phi, Psi);
    if (Psi > LB) {
      LB = Psi;
      memcpy(zeta_out, zeta, sizeof(double) * (size_t)n);
    }
    if (Phi < UB) UB = Phi;
    double gap = Phi - Psi;
    if (trace && it < trace_cap) trace[it] = gap;
    if (phi_trace && it < trace_cap) phi_trace[it] = Phi;
    rel = (UB - LB) / fmax(fabs(UB), 1e-300);
    if (rel <= tol) {
      status = ORC_CONVERGED;
      break;
    }
    if (!isnan(cutoff) && LB >= cutoff) {
      status = ORC_CUTOFF_PRUNE;
      break;
    }
    if (!isnan(cutoff) && UB <= cutoff) {
      status = ORC_CUTOFF_BRANCH;
      break;
    }
    int restart = 0;
    if (method == ORC_FISTA_GAP && gap <= gap_ref / eta) {
      gap_ref = gap;
      restart = 1;
    } else if (method == ORC_FISTA_FV && Phi > Phi_prev) {
      restart = 1;
    }
    if (restart) {
      memcpy(yv, x, sizeof(double) * (size_t)p);
      t = 1.0;
      if (restart_at && restarts < restart_cap) restart_at[restarts] = it;
      restarts++;
    }
    Phi_prev = Phi;
  }
#undef ORC_EVAL
  memcpy(beta_out, x, sizeof(double) * (size_t)p);
  res[0] = LB;
  res[1] = UB;
  res[2] = (UB - LB) / fmax(fabs(UB), 1e-300);
  res[3] = L;
  res[4] = (double)it;
  res[5] = (double)restarts;
  res[6] = (double)status;
  free(x);
  free(xn);
  free(yv);
  free(gp);
  free(u);
  free(gn);
  free(zeta);
  return status;
}

/* Euclidean distance of two m-vectors. */
static double orc_dist(const double *a, const double *b, int64_t m) {
  double s = 0.0;
  for (int64_t j = 0; j < m; j++) s += (a[j] - b[j]) * (a[j] - b[j]);
  return sqrt(s);
}

/* ------------------------------------------- FISTA with backtracking */

/* Bregman remainder of F between two points u (at x) and w (at y) in the
 * image of X: F(u) - F(w) - <grad F(w), u - w>, summed row by row.  For the
 * smooth part f(beta) = F(X beta) this is f(x) - f(y) - <grad f(y), x - y>,
 * the quantity bounded by the quadratic model of a step 1/L.  Least squares:
 * (u_i - w_i)^2 exactly.  Logistic: with a = -y_i w_i and d = -y_i (u_i -
 * w_i), log(1 + exp(a + d)) - log(1 + exp(a)) - sigma(a) d, the first
 * difference taken as log1p(sigma(a) expm1(d)) so that it carries no
 * cancellation of the two softplus values. */
static double orc_bregman(int loss, const double *u, const double *w, const double *y, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; i++) {
    if (loss == ORC_LSQ) {
      s += (u[i] - w[i]) * (u[i] - w[i]);
    } else {
      const double a = -y[i] * w[i], d = -y[i] * (u[i] - w[i]);
      const double sg = 1.0 / (1.0 + exp(-a));
      s += log1p(sg * expm1(d)) - sg * d;
    }
  }
  return s;
}

/* FISTA with backtracking (Beck, "First-Order Methods in Optimization",
 * 2017, Section 10.7, the monotone backtracking rule), the "FISTA with line
 * search" of Section 5 that the paper runs with its duality-gap restart.
 * From the momentum point y with gradient grad f(y), the step constant L
 * starts from the previous one and is multiplied by c until the trial
 * x = prox_{(2 lambda2 / L) g_N}(y - grad f(y) / L) satisfies the
 * quadratic-model condition
 *     f(x) <= f(y) + <grad f(y), x - y> + (L / 2) ||x - y||^2,
 * tested in the Bregman form above; L never exceeds Lmax (a Lipschitz
 * constant of grad f, where the condition holds by itself: a trial at Lmax is
 * accepted).  The accepted trial is the next iterate; momentum, the bounds,
 * the stopping test and the dynamic termination are those of orc_solve at
 * the accepted iterates; rejected trials are not evaluated.  With restart_gap
 * the duality-gap restart runs the method afresh from the restart iterate:
 * t <- 1, y <- x and the line search starts again from L0.  restart_gap = 0
 * runs plain FISTA with backtracking.
 *
 * res[0..7] = {LB, UB, rel_gap, final L, iterations (accepted), restarts,
 * status, rejected trials}.  Traces (length trace_cap, optional) per accepted
 * iterate: Phi - Psi, Phi, and the L of the step that produced it (L0 at the
 * start point). */
int orc_solve_bt(const void *X, int xdt, const double *y, int64_t n, int64_t p, int loss, double lambda2,
                 double M, int32_t k, const int8_t *st, double L0, double c, double Lmax, int restart_gap,
                 double tol, double eta, int64_t max_iter, double cutoff, const double *beta0, double *beta_out,
                 double *zeta_out, double *res, double *trace, double *phi_trace, double *L_trace,
                 int64_t trace_cap) {
  int64_t pbar, kbar;
  for (int i = 0; i < 8; i++) res[i] = 0.0;
  if (orc_node_dims(st, p, k, &pbar, &kbar) < 0) {
    res[0] = INFINITY;
    res[1] = INFINITY;
    res[6] = ORC_INFEASIBLE;
    for (int64_t j = 0; j < p; j++) beta_out[j] = 0.0;
    return ORC_INFEASIBLE;
  }
  if (!(L0 > 0.0) || !(c > 1.0) || !(Lmax >= L0)) return -1;
  double *x = (double *)calloc((size_t)p, sizeof(double));
  double *xn = (double *)malloc(sizeof(double) * (size_t)p);
  double *yv = (double *)malloc(sizeof(double) * (size_t)p);
  double *gp = (double *)malloc(sizeof(double) * (size_t)p);
  double *vv = (double *)malloc(sizeof(double) * (size_t)p);
  double *uy = (double *)malloc(sizeof(double) * (size_t)n);
  double *ux = (double *)malloc(sizeof(double) * (size_t)n);
  double *gn = (double *)malloc(sizeof(double) * (size_t)n);
  double *zeta = (double *)malloc(sizeof(double) * (size_t)n);
  if (beta0)
    for (int64_t j = 0; j < p; j++) x[j] = beta0[j];
  memcpy(yv, x, sizeof(double) * (size_t)p);
  double t = 1.0, L = L0;

  /* (Phi, Psi) at the iterate x from u = X x */
#define ORC_EVAL_BT(PHI, PSI)                                                  \
  do {                                                                         \
    orc_loss_grad(loss, ux, y, n, gn);                                         \
    for (int64_t i_ = 0; i_ < n; i_++) zeta[i_] = -gn[i_];                     \
    PSI = orc_dual(X, xdt, y, n, p, loss, lambda2, M, k, st, zeta);            \
    PHI = orc_in_dom(x, st, p, k, M, 1e-9)                                     \
              ? orc_loss(loss, ux, y, n) + 2.0 * lambda2 * orc_g(x, st, p, k)  \
              : INFINITY;                                                      \
  } while (0)

  double Phi, Psi;
  orc_matvec(X, xdt, n, p, x, ux);
  ORC_EVAL_BT(Phi, Psi);
  double LB = Psi, UB = Phi, gap_ref = Phi - Psi;
  memcpy(zeta_out, zeta, sizeof(double) * (size_t)n);
  if (trace_cap > 0) {
    if (trace) trace[0] = Phi - Psi;
    if (phi_trace) phi_trace[0] = Phi;
    if (L_trace) L_trace[0] = L;
  }
  int64_t it = 0, restarts = 0, rejected = 0;
  int status = ORC_MAXITER;
  double rel = (UB - LB) / fmax(fabs(UB), 1e-300);
  if (rel <= tol) status = ORC_CONVERGED;
  else if (!isnan(cutoff) && LB >= cutoff) status = ORC_CUTOFF_PRUNE;
  else if (!isnan(cutoff) && UB <= cutoff) status = ORC_CUTOFF_BRANCH;
  while (status == ORC_MAXITER && it < max_iter) {
    it++;
    /* gradient of f at the momentum point */
    orc_matvec(X, xdt, n, p, yv, uy);
    orc_loss_grad(loss, uy, y, n, gn);
    orc_rmatvec(X, xdt, n, p, gn, gp);
    for (;;) {
      for (int64_t j = 0; j < p; j++) vv[j] = yv[j] - gp[j] / L;
      orc_prox_g(vv, st, p, 2.0 * lambda2 / L, k, M, xn);
      orc_matvec(X, xdt, n, p, xn, ux);
      if (L >= Lmax) break;
      const double dxy = orc_dist(xn, yv, p);
      if (orc_bregman(loss, ux, uy, y, n) <= 0.5 * L * dxy * dxy) break;
      L = fmin(c * L, Lmax);
      rejected++;
    }
    double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
    double mom = (t - 1.0) / tn;
    for (int64_t j = 0; j < p; j++) {
      yv[j] = xn[j] + mom * (xn[j] - x[j]);
      x[j] = xn[j];
    }
    t = tn;
    ORC_EVAL_BT(Phi, Psi);
    if (Psi > LB) {
      LB = Psi;
      memcpy(zeta_out, zeta, sizeof(double) * (size_t)n);
    }
    if (Phi < UB) UB = Phi;
    double gap = Phi - Psi;
    if (it < trace_cap) {
      if (trace) trace[it] = gap;
      if (phi_trace) phi_trace[it] = Phi;
      if (L_trace) L_trace[it] = L;
    }
    rel = (UB - LB) / fmax(fabs(UB), 1e-300);
    if (rel <= tol) {
      status = ORC_CONVERGED;
      break;
    }
    if (!isnan(cutoff) && LB >= cutoff) {
      status = ORC_CUTOFF_PRUNE;
      break;
    }
    if (!isnan(cutoff) && UB <= cutoff) {
      status = ORC_CUTOFF_BRANCH;
      break;
    }
    if (restart_gap && gap <= gap_ref / eta) {
      gap_ref = gap;
      memcpy(yv, x, sizeof(double) * (size_t)p);
      t = 1.0;
      L = L0;
      restarts++;
    }
  }
#undef ORC_EVAL_BT
  memcpy(beta_out, x, sizeof(double) * (size_t)p);
  res[0] = LB;
  res[1] = UB;
  res[2] = (UB - LB) / fmax(fabs(UB), 1e-300);
  res[3] = L;
  res[4] = (double)it;
  res[5] = (double)restarts;
  res[6] = (double)status;
  res[7] = (double)rejected;
  free(x);
  free(xn);
  free(yv);
  free(gp);
  free(vv);
  free(uy);
  free(ux);
  free(gn);
  free(zeta);
  return status;
}

/* ------------------------------------------------------------ AC-FGM */

/* Gradient of f(beta) = F(X beta) at x (p-vector g), the induced dual vector
 * zeta = -grad F(X x) (n-vector), F(X x) and Psi(zeta).  u: n scratch. */
static void orc_eval_point(const void *X, int xdt, const double *y, int64_t n, int64_t p, int loss,
                           double lambda2, double M, int32_t k, const int8_t *st, const double *x, double *u,
                           double *zeta, double *g, double *Fx, double *Psi) {
  orc_matvec(X, xdt, n, p, x, u);
  orc_loss_grad(loss, u, y, n, zeta); /* zeta <- grad F(u) */
  orc_rmatvec(X, xdt, n, p, zeta, g); /* g = X^T grad F(X x) */
  for (int64_t i = 0; i < n; i++) zeta[i] = -zeta[i];
  *Fx = orc_loss(loss, u, y, n);
  *Psi = orc_dual(X, xdt, y, n, p, loss, lambda2, M, k, st, zeta);
}

/* AC-FGM (accelerated composite fast gradient method of Li and Lan, "A simple
 * uniformly optimal method without line search for convex optimization",
 * 2023), the parameter-free method of Section 3.3's rate table and the
 * Section 5.2 convergence study, applied to Phi = f + G with f(beta) =
 * F(X beta), G = 2 lambda2 g_N.  Three sequences: the prox step
 *     z_t = prox_{eta_t G}(y_{t-1} - eta_t grad f(x_{t-1})),
 * the averaged prox centre y_t = (1 - b) y_{t-1} + b z_t (b = the averaging
 * weight, in (0, 1 - sqrt(6)/3]) and the iterate x_t = (z_t + tau_t x_{t-1}) /
 * (1 + tau_t) with tau_1 = 0, tau_t = t / 2.  Step sizes from the local
 * curvature estimates Lhat_t = ||grad f(x_t) - grad f(x_{t-1})|| /
 * ||x_t - x_{t-1}||: eta_2 = min((1 - b) eta_1, 1 / (4 Lhat_1)), eta_t =
 * min((tau_{t-1} + 1) / tau_t eta_{t-1}, tau_{t-1} / (4 Lhat_{t-1})) for
 * t >= 3.  The first step is a backtracking line search from an initial
 * underestimate L0 of the curvature: eta_1 = 1 / L1, and while Lhat_1 > L1
 * the trial is rejected and L1 <- c L1 (c > 1).  The iterate x_t is the
 * primal point of the certificate: zeta_t = -grad F(X x_t) (Section 3.2).
 * The readings (step rules, first-step test, what a restart keeps) are listed
 * in the design notes.
 *
 * With restart_gap the duality-gap restart of Section 3.3 applies: when the
 * gap at an accepted iterate falls to 1/eta of the gap at the epoch start,
 * the method restarts from that iterate (x_0 = y_0 = x_t, t = 1) keeping the
 * accepted first-step constant L1.  Every evaluated point (rejected trials
 * included) enters the best-so-far bounds and the stopping test.
 *
 * res[0..7] = {LB, UB, rel_gap, final L1, evaluations, restarts, status,
 * rejected trials}.  Traces (length trace_cap, optional) per evaluation:
 * gap, Phi, Lhat (against the point the step left from) and the epoch step
 * index t (negative for a rejected trial). */
int orc_solve_acfgm(const void *X, int xdt, const double *y, int64_t n, int64_t p, int loss, double lambda2,
                    double M, int32_t k, const int8_t *st, double L0, double c, double b, int restart_gap,
                    double tol, double eta, int64_t max_iter, const double *beta0, double *beta_out,
                    double *zeta_out, double *res, double *trace, double *phi_trace, double *lhat_trace,
                    double *step_trace, int64_t trace_cap) {
  int64_t pbar, kbar;
  for (int i = 0; i < 8; i++) res[i] = 0.0;
  if (orc_node_dims(st, p, k, &pbar, &kbar) < 0) {
    res[0] = INFINITY;
    res[1] = INFINITY;
    res[6] = ORC_INFEASIBLE;
    for (int64_t j = 0; j < p; j++) beta_out[j] = 0.0;
    return ORC_INFEASIBLE;
  }
  const size_t P8 = sizeof(double) * (size_t)p, N8 = sizeof(double) * (size_t)n;
  double *x = (double *)calloc((size_t)p, sizeof(double)); /* x_{t-1} before a step, x_t after */
  double *g = (double *)malloc(P8);                         /* grad f at x */
  double *xo = (double *)malloc(P8), *go = (double *)malloc(P8); /* the point the step left from */
  double *yv = (double *)malloc(P8), *z = (double *)malloc(P8), *v = (double *)malloc(P8);
  double *xn = (double *)malloc(P8), *gn = (double *)malloc(P8), *yn = (double *)malloc(P8);
  double *xbest = (double *)malloc(P8);
  double *u = (double *)malloc(N8), *zeta = (double *)malloc(N8);
  if (beta0)
    for (int64_t j = 0; j < p; j++) x[j] = beta0[j];
  double Fx, Psi;
  orc_eval_point(X, xdt, y, n, p, loss, lambda2, M, k, st, x, u, zeta, g, &Fx, &Psi);
  double Phi = orc_in_dom(x, st, p, k, M, 1e-9) ? Fx + 2.0 * lambda2 * orc_g(x, st, p, k) : INFINITY;
  double LB = Psi, UB = Phi, gap_ref = Phi - Psi;
  memcpy(zeta_out, zeta, N8);
  memcpy(xbest, x, P8);
  if (trace && trace_cap > 0) trace[0] = Phi - Psi;
  if (phi_trace && trace_cap > 0) phi_trace[0] = Phi;
  if (lhat_trace && trace_cap > 0) lhat_trace[0] = NAN;
  if (step_trace && trace_cap > 0) step_trace[0] = 0.0;
  memcpy(yv, x, P8);
  double L1 = L0, eta_prev = 0.0, tau_prev = 0.0, lhat_prev = 0.0;
  int64_t t = 1, it = 0, restarts = 0, rejected = 0;
  int status = ORC_MAXITER;
  double rel = (UB - LB) / fmax(fabs(UB), 1e-300);
  if (rel <= tol) status = ORC_CONVERGED;
  while (status == ORC_MAXITER && it < max_iter) {
    it++;
    double eta_t, tau_t;
    if (t == 1) {
      eta_t = 1.0 / L1;
      tau_t = 0.0;
    } else {
      tau_t = 0.5 * (double)t;
      const double cap = (lhat_prev > 0.0) ? tau_prev / (4.0 * lhat_prev) : INFINITY;
      if (t == 2) eta_t = fmin((1.0 - b) * eta_prev, (lhat_prev > 0.0) ? 1.0 / (4.0 * lhat_prev) : INFINITY);
      else eta_t = fmin((tau_prev + 1.0) / tau_t * eta_prev, cap);
    }
    /* z_t = prox_{eta_t G}(y_{t-1} - eta_t grad f(x_{t-1})), G = 2 lambda2 g_N */
    for (int64_t j = 0; j < p; j++) v[j] = yv[j] - eta_t * g[j];
    orc_prox_g(v, st, p, 2.0 * lambda2 * eta_t, k, M, z);
    for (int64_t j = 0; j < p; j++) {
      yn[j] = (1.0 - b) * yv[j] + b * z[j];
      xn[j] = (z[j] + tau_t * x[j]) / (1.0 + tau_t);
    }
    double Fn, Psin;
    orc_eval_point(X, xdt, y, n, p, loss, lambda2, M, k, st, xn, u, zeta, gn, &Fn, &Psin);
    const double Phin = orc_in_dom(xn, st, p, k, M, 1e-9) ? Fn + 2.0 * lambda2 * orc_g(xn, st, p, k) : INFINITY;
    const double dx = orc_dist(xn, x, p);
    const double lhat = dx > 0.0 ? orc_dist(gn, g, p) / dx : 0.0;
    if (Psin > LB) {
      LB = Psin;
      memcpy(zeta_out, zeta, N8);
    }
    if (Phin < UB) {
      UB = Phin;
      memcpy(xbest, xn, P8);
    }
    const int reject = (t == 1 && lhat > L1);
    if (it < trace_cap) {
      if (trace) trace[it] = Phin - Psin;
      if (phi_trace) phi_trace[it] = Phin;
      if (lhat_trace) lhat_trace[it] = lhat;
      if (step_trace) step_trace[it] = reject ? -(double)t : (double)t;
    }
    rel = (UB - LB) / fmax(fabs(UB), 1e-300);
    if (rel <= tol) {
      status = ORC_CONVERGED;
      break;
    }
    if (reject) { /* line search of the first step: a larger curvature estimate */
      L1 *= c;
      rejected++;
      continue;
    }
    memcpy(xo, x, P8);
    memcpy(go, g, P8);
    memcpy(x, xn, P8);
    memcpy(g, gn, P8);
    memcpy(yv, yn, P8);
    eta_prev = eta_t;
    tau_prev = tau_t;
    lhat_prev = lhat;
    t++;
    if (restart_gap && Phin - Psin <= gap_ref / eta) {
      gap_ref = Phin - Psin;
      memcpy(yv, x, P8);
      t = 1;
      restarts++;
    }
  }
  memcpy(beta_out, xbest, P8);
  res[0] = LB;
  res[1] = UB;
  res[2] = (UB - LB) / fmax(fabs(UB), 1e-300);
  res[3] = L1;
  res[4] = (double)it;
  res[5] = (double)restarts;
  res[6] = (double)status;
  res[7] = (double)rejected;
  free(x); free(g); free(xo); free(go); free(yv); free(z); free(v); free(xn); free(gn); free(yn); free(xbest);
  free(u); free(zeta);
  return status;
}

/* ------------------------------------------------------------ LASSO */

/* The duality-gap restart applied beyond the perspective relaxation
 * (Section 5.2): least squares F(u) = ||u - y||^2 with
 *   kind 0 (l1-regularised): G(beta) = lam ||beta||_1,
 *   kind 1 (l1-ball):        G(beta) = indicator of ||beta||_1 <= lam.
 * Conjugates: kind 0, G*(w) = indicator of ||w||_inf <= lam; kind 1,
 * G*(w) = lam ||w||_inf.  Prox of t G: kind 0, soft thresholding at t lam;
 * kind 1, Euclidean projection onto the l1-ball (sort-based: the threshold
 * theta solves sum_j max(|v_j| - theta, 0) = lam). */
double orc_lasso_G(int kind, const double *beta, int64_t p, double lam) {
  double l1 = 0.0;
  for (int64_t j = 0; j < p; j++) l1 += fabs(beta[j]);
  if (kind == 0) return lam * l1;
  return (l1 <= lam * (1.0 + 1e-9)) ? 0.0 : INFINITY;
}

double orc_lasso_Gstar(int kind, const double *w, int64_t p, double lam) {
  double mx = 0.0;
  for (int64_t j = 0; j < p; j++) mx = fmax(mx, fabs(w[j]));
  if (kind == 0) return (mx <= lam) ? 0.0 : INFINITY;
  return lam * mx;
}

void orc_lasso_prox(int kind, const double *v, int64_t p, double t, double lam, double *out) {
  if (kind == 0) {
    const double th = t * lam;
    for (int64_t j = 0; j < p; j++) {
      const double a = fabs(v[j]) - th;
      out[j] = a > 0.0 ? copysign(a, v[j]) : 0.0;
    }
    return;
  }
  double l1 = 0.0;
  for (int64_t j = 0; j < p; j++) l1 += fabs(v[j]);
  if (l1 <= lam) {
    memcpy(out, v, sizeof(double) * (size_t)p);
    return;
  }
  double *a = (double *)malloc(sizeof(double) * (size_t)p);
  for (int64_t j = 0; j < p; j++) a[j] = fabs(v[j]);
  qsort(a, (size_t)p, sizeof(double), cmp_desc);
  /* theta = (sum of the m largest - lam) / m for the largest m with
     a_(m) > (sum of the m largest - lam) / m */
  double cum = 0.0, theta = 0.0;
  for (int64_t m = 1; m <= p; m++) {
    cum += a[m - 1];
    const double th = (cum - lam) / (double)m;
    if (a[m - 1] > th) theta = th;
  }
  free(a);
  for (int64_t j = 0; j < p; j++) {
    const double r = fabs(v[j]) - theta;
    out[j] = r > 0.0 ? copysign(r, v[j]) : 0.0;
  }
}

/* Psi at a dual-feasible point built from zeta = -grad F(X beta) = 2 (y - X beta):
 * kind 0 scales it into dom G*, s = min(1, lam / ||X^T zeta||_inf), Psi =
 * -F*(-s zeta); kind 1 uses zeta itself, Psi = -F*(-zeta) - lam ||X^T zeta||_inf.
 * *scale_out (optional) receives s (1 for kind 1). */
double orc_lasso_dual(const void *X, int xdt, const double *y, int64_t n, int64_t p, int kind, double lam,
                      const double *zeta, double *scale_out) {
  double *w = (double *)malloc(sizeof(double) * (size_t)p);
  orc_rmatvec(X, xdt, n, p, zeta, w);
  double mx = 0.0;
  for (int64_t j = 0; j < p; j++) mx = fmax(mx, fabs(w[j]));
  free(w);
  double zy = 0.0, zz = 0.0;
  for (int64_t i = 0; i < n; i++) {
    zy += zeta[i] * y[i];
    zz += zeta[i] * zeta[i];
  }
  if (kind == 0) {
    const double s = (mx > lam) ? lam / mx : 1.0;
    if (scale_out) *scale_out = s;
    return s * zy - 0.25 * s * s * zz;
  }
  if (scale_out) *scale_out = 1.0;
  return zy - 0.25 * zz - lam * mx;
}

/* FISTA (fixed step 1/L) with the duality-gap restart on the LASSO problem of
 * `kind`; the same loop as orc_solve with G and its prox replaced.
 * res[0..7] = {LB, UB, rel_gap, L, iters, restarts, status, 0}; trace and
 * phi_trace as orc_solve (method: ORC_FISTA_GAP or ORC_FISTA). */
int orc_lasso_solve(const void *X, int xdt, const double *y, int64_t n, int64_t p, int kind, double lam, double L,
                    double tol, double eta, int64_t max_iter, int method, const double *beta0, double *beta_out,
                    double *zeta_out, double *res, double *trace, double *phi_trace, int64_t trace_cap) {
  for (int i = 0; i < 8; i++) res[i] = 0.0;
  if (L <= 0.0) L = 2.0 * orc_power_norm2(X, xdt, n, p, 2000, 1e-12);
  const size_t P8 = sizeof(double) * (size_t)p, N8 = sizeof(double) * (size_t)n;
  double *x = (double *)calloc((size_t)p, sizeof(double));
  double *xn = (double *)malloc(P8), *yv = (double *)malloc(P8), *gp = (double *)malloc(P8);
  double *u = (double *)malloc(N8), *gn = (double *)malloc(N8), *zeta = (double *)malloc(N8);
  double *xbest = (double *)malloc(P8);
  if (beta0)
    for (int64_t j = 0; j < p; j++) x[j] = beta0[j];
  memcpy(yv, x, P8);
  memcpy(xbest, x, P8);
  double t = 1.0, s = 1.0;
#define ORC_LEVAL(PHI, PSI)                                                      \
  do {                                                                           \
    orc_matvec(X, xdt, n, p, x, u);                                              \
    for (int64_t i_ = 0; i_ < n; i_++) zeta[i_] = 2.0 * (y[i_] - u[i_]);         \
    PSI = orc_lasso_dual(X, xdt, y, n, p, kind, lam, zeta, &s);                  \
    PHI = orc_loss(ORC_LSQ, u, y, n) + orc_lasso_G(kind, x, p, lam);             \
  } while (0)
  double Phi, Psi;
  ORC_LEVAL(Phi, Psi);
  double LB = Psi, UB = Phi, gap_ref = Phi - Psi;
  for (int64_t i = 0; i < n; i++) zeta_out[i] = s * zeta[i];
  if (trace && trace_cap > 0) trace[0] = Phi - Psi;
  if (phi_trace && trace_cap > 0) phi_trace[0] = Phi;
  int64_t it = 0, restarts = 0;
  int status = ORC_MAXITER;
  double rel = (UB - LB) / fmax(fabs(UB), 1e-300);
  if (rel <= tol) status = ORC_CONVERGED;
  while (status == ORC_MAXITER && it < max_iter) {
    it++;
    orc_matvec(X, xdt, n, p, yv, u);
    orc_loss_grad(ORC_LSQ, u, y, n, gn);
    orc_rmatvec(X, xdt, n, p, gn, gp);
    for (int64_t j = 0; j < p; j++) gp[j] = yv[j] - gp[j] / L;
    orc_lasso_prox(kind, gp, p, 1.0 / L, lam, xn);
    const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
    const double mom = (t - 1.0) / tn;
    for (int64_t j = 0; j < p; j++) {
      yv[j] = xn[j] + mom * (xn[j] - x[j]);
      x[j] = xn[j];
    }
    t = tn;
    ORC_LEVAL(Phi, Psi);
    if (Psi > LB) {
      LB = Psi;
      for (int64_t i = 0; i < n; i++) zeta_out[i] = s * zeta[i];
    }
    if (Phi < UB) {
      UB = Phi;
      memcpy(xbest, x, P8);
    }
    const double gap = Phi - Psi;
    if (trace && it < trace_cap) trace[it] = gap;
    if (phi_trace && it < trace_cap) phi_trace[it] = Phi;
    rel = (UB - LB) / fmax(fabs(UB), 1e-300);
    if (rel <= tol) {
      status = ORC_CONVERGED;
      break;
    }
    if (method == ORC_FISTA_GAP && gap <= gap_ref / eta) {
      gap_ref = gap;
      memcpy(yv, x, P8);
      t = 1.0;
      restarts++;
    }
  }
#undef ORC_LEVAL
  memcpy(beta_out, xbest, P8);
  res[0] = LB;
  res[1] = UB;
  res[2] = (UB - LB) / fmax(fabs(UB), 1e-300);
  res[3] = L;
  res[4] = (double)it;
  res[5] = (double)restarts;
  res[6] = (double)status;
  free(x); free(xn); free(yv); free(gp); free(u); free(gn); free(zeta); free(xbest);
  return status;
}

/* Number of OpenMP threads the matrix products use. */
int orc_num_threads(void) {
  int nt = 1;
#pragma omp parallel
  {
#pragma omp single
    {
#ifdef _OPENMP
      extern int omp_get_num_threads(void);
      nt = omp_get_num_threads();
#endif
    }
  }
  return nt;
}
