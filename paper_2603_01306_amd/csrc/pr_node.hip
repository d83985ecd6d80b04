// Per-node kernels of libpr on gfx950: one 512-thread workgroup per node.
//
//   k_node_step  dual value at the current iterate (closed-form conjugate of
//                Lemma function_g_conjugate_in_BnB with an exact radix top-kbar
//                selection), gap / restart / termination (Section 3.3), FISTA
//                momentum, the prox of Algorithm 2 + Moreau in pooled-threshold
//                form, Algorithm 1 value of the new iterate, support list.
//   k_node_init  start point: support, Algorithm 1 value, dom test.
//   k_prox, k_regularizer, k_loss_terms, ...: entry points of the C ABI.
//
// Two variants: register-resident (p <= 16384, coordinates j = tid + e*512
// held in registers across all passes) and a global-memory one for larger p.
#include "pr_device.h"

#include "pr_regularizer.h"

namespace pr {
namespace {
using namespace dev;

// ------------------------------------------------------------ node kernels

__global__ __launch_bounds__(NT) void k_node_init(const NodeParams *__restrict__ prm, NodeState *S,
                                                  NodeBufs nb, const double *__restrict__ beta0,
                                                  double L) {
  __shared__ double red[NW * 4];
  __shared__ int scan[NW];
  const int64_t p = prm->p;
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
    const double b = beta0 ? beta0[j] : 0.0;
    nb.x0[j] = b;
    nb.xbest[j] = b;
    nb.x1[j] = 0.0;
    nb.hprev[j] = 0.0;
  }
  __syncthreads();
  IterStats is = finish_iterate(nb.x0, prm->st, p, prm->kbar, prm->M, nb.abuf, nb.sidx, nb.sval, red,
                                scan);
  if (threadIdx.x == 0) {
    NodeState s{};
    s.L = L;
    s.t = 1.0;
    s.gap_ref = INFINITY;
    s.lb = -INFINITY;
    s.ub = INFINITY;
    s.phi = INFINITY;
    s.psi = -INFINITY;
    s.rel_gap = INFINITY;
    s.gval = is.gval;
    s.tau = -1.0;
    s.mom = 0.0;
    s.iter = 0;
    s.restarts = 0;
    s.done = 0;
    s.status = kMaxIter;
    s.parity = 0;
    s.nsupp = is.nsupp;
    s.improved = 0;
    s.indom = is.indom;
    s.tau_iters = 0;
    *S = s;
  }
}

// One iteration for one node: evaluate (Phi, Psi) at the current iterate
// x^k from the products of this pass, update bounds, decide termination and
// restart, then take the FISTA step to x^{k+1}.
//   least squares: h1 = X^T r_k, r_k = y - X x^k, zeta_k = 2 r_k,
//                  X^T zeta_k / (2 lambda2) = h1 / lambda2, and the gradient at
//                  the momentum point y^{k+1} = (1+m) x^k - m x^{k-1} is
//                  -2((1+m) h_k - m h_{k-1}) by linearity.
//   logistic:      h1 = X^T zeta_k, h2 = X^T grad F(X y^{k+1}) for the
//                  non-restart momentum; on restart the gradient at x^k is -h1.
__global__ __launch_bounds__(NT) void k_node_step(const NodeParams *__restrict__ prm, NodeState *S,
                                                  NodeBufs nb, ProbBufs B) {
  __shared__ double red[NW * 4];
  __shared__ int scan[NW];
  __shared__ SelLds sel;
  __shared__ double bcd[4];
  __shared__ int bci[4];
  if (S->done) return;
  const int tid = threadIdx.x;
  const int64_t p = prm->p;
  const int kbar = prm->kbar, loss = prm->loss;
  const double lam2 = prm->lambda2, M = prm->M;
  const int8_t *__restrict__ st = prm->st;
  const int parity = S->parity;
  const double L = S->L;

  // loss-side terms of this iterate, summed over row blocks in fixed order
  double Fk = 0.0, negconj = 0.0;
  for (int i = 0; i < B.nfin; i++) {
    Fk += B.rbsum[2 * i];
    negconj += B.rbsum[2 * i + 1];
  }
  // dual: w = X^T zeta / (2 lambda2)
  const double wscale = (loss == kLsq) ? 1.0 / lam2 : 0.5 / lam2;
  double sj1[1] = {0.0};
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
    const double w = B.h1[j] * wscale;
    const int s = st[j];
    if (s == kOne) sj1[0] += huber(w, M);
    nb.abuf[j] = (s == kFree) ? fabs(w) : -1.0;
  }
  block_sum<NT, 1>(sj1, red);
  __syncthreads();
  const double topsum = topsum_huber(nb.abuf, p, kbar, M, sel, red);
  const double psi = negconj - 2.0 * lam2 * (sj1[0] + topsum);
  const double phi = S->indom ? Fk + 2.0 * lam2 * S->gval : INFINITY;

  if (tid == 0) {
    const int it = S->iter;
    if (prm->trace && it <= prm->max_iter) {
      prm->trace[2 * it] = phi;
      prm->trace[2 * it + 1] = psi;
    }
    const double gap = phi - psi;
    double lb = S->lb, ub = S->ub;
    int improved = 0;
    if (psi > lb) {
      lb = psi;
      improved = 1;
    }
    int ub_improved = 0;
    if (phi < ub) {
      ub = phi;
      ub_improved = 1;
    }
    const double rel = (ub - lb) / fmax(fabs(ub), 1e-300);
    int done = 0, status = kMaxIter;
    if (rel <= prm->tol) {
      done = 1;
      status = kConverged;
    } else if (!isnan(prm->cutoff) && lb >= prm->cutoff) {
      done = 1;
      status = kCutoffPrune;
    } else if (!isnan(prm->cutoff) && ub <= prm->cutoff) {
      done = 1;
      status = kCutoffBranch;
    } else if (it >= prm->max_iter) {
      done = 1;
      status = kMaxIter;
    }
    double m = 0.0, t = S->t, gap_ref = S->gap_ref;
    int restart = 0, restarts = S->restarts;
    if (!done) {
      restart = decide_restart(prm, it, gap, phi, S->phi, gap_ref, restarts);
      if (restart) {
        m = 0.0;
        t = 1.0;
      } else {
        const double tn = fista_next_t(t);
        m = (t - 1.0) / tn;
        t = tn;
      }
    }
    S->phi = phi;
    S->psi = psi;
    S->lb = lb;
    S->ub = ub;
    S->rel_gap = rel;
    S->improved = improved;
    S->status = status;
    S->t = t;
    S->gap_ref = gap_ref;
    S->restarts = restarts;
    S->mom = m;
    if (done) S->done = 1;
    bcd[0] = m;
    bci[0] = done;
    bci[1] = restart;
    bci[2] = ub_improved;
  }
  __syncthreads();
  double *__restrict__ xc = parity ? nb.x1 : nb.x0;
  double *__restrict__ xn = parity ? nb.x0 : nb.x1;  // holds x^{k-1}, receives x^{k+1}
  if (bci[2]) {
#pragma unroll 8
    for (int64_t j = threadIdx.x; j < p; j += NT) nb.xbest[j] = xc[j];
  }
  if (bci[0]) return;
  const double m = bcd[0];
  const int restart = bci[1];

  // gradient step at the momentum point
  const double invL = 1.0 / L;
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
    const double xk = xc[j], xq = xn[j];
    const double yj = xk + m * (xk - xq);
    double gj;
    if (loss == kLsq) {
      const double h = B.h1[j], hp = nb.hprev[j];
      gj = -2.0 * ((1.0 + m) * h - m * hp);
      nb.hprev[j] = h;
    } else {
      gj = restart ? -B.h1[j] : B.h2[j];
    }
    const double v = yj - gj * invL;
    nb.vbuf[j] = v;
    nb.abuf[j] = (st[j] == kFree) ? fabs(v) : -1.0;
  }
  __syncthreads();
  const double rho = 2.0 * lam2 * invL;
  int evals = 0;
  const double tau = solve_tau(nb.abuf, p, kbar, rho, M, S->tau, red, &evals);
  const double inv1p = 1.0 / (1.0 + rho);
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
    const double v = nb.vbuf[j];
    const int s = st[j];
    double x = 0.0;
    if (s != kZero) {
      const double av = fabs(v);
      double r = fmin(av * inv1p, M);
      if (s == kFree) r = fmin(r, fmax(av - tau, 0.0));
      x = (r == 0.0) ? 0.0 : copysign(r, v);
    }
    xn[j] = x;
  }
  __syncthreads();
  IterStats is = finish_iterate(xn, st, p, kbar, M, nb.abuf, nb.sidx, nb.sval, red, scan);
  if (tid == 0) {
    S->gval = is.gval;
    S->indom = is.indom;
    S->nsupp = is.nsupp;
    S->tau = tau;
    S->tau_iters = evals;
    S->parity = parity ^ 1;
    S->iter = S->iter + 1;
  }
}

__global__ void k_zbest_final(const NodeState *S, const double *__restrict__ r, double *zbest,
                              double scale, int64_t n) {
  if (!S->improved) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    zbest[i] = scale * r[i];
}

// Standalone prox_{rho g_N}(v) (Algorithm 2 + Moreau in pooled-threshold form).
__global__ __launch_bounds__(NT) void k_prox(const double *v, double *out, int64_t p, double rho,
                                             int kbar, double M, const int8_t *__restrict__ st,
                                             double *abuf) {
  __shared__ double red[NW * 4];
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) abuf[j] = (st[j] == kFree) ? fabs(v[j]) : -1.0;
  __syncthreads();
  int evals;
  const double tau = solve_tau(abuf, p, kbar, rho, M, -1.0, red, &evals);
  const double inv1p = 1.0 / (1.0 + rho);
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
    const double vj = v[j];
    const int s = st[j];
    double x = 0.0;
    if (s != kZero) {
      const double av = fabs(vj);
      double r = fmin(av * inv1p, M);
      if (s == kFree) r = fmin(r, fmax(av - tau, 0.0));
      x = (r == 0.0) ? 0.0 : copysign(r, vj);
    }
    out[j] = x;
  }
}

// prox_{rho_q g_N}(v_q) for m nodes at once, one workgroup per node (the
// body of k_prox): node q's parameters prm[q] (status, kbar, lambda2, M),
// rho_q = 2 lambda2_q / L, rows q of V / Xo / abuf (p entries each).
__global__ __launch_bounds__(NT) void k_prox_batch(const NodeParams *__restrict__ prm, const double *V, double *Xo,
                                                   double *abuf_all, int64_t p, double invL) {
  __shared__ double red[NW * 4];
  const int q = blockIdx.x;
  const NodeParams P = prm[q];
  const double *v = V + (int64_t)q * p;
  double *out = Xo + (int64_t)q * p;
  double *abuf = abuf_all + (int64_t)q * p;
  const int8_t *__restrict__ st = P.st;
  const double rho = 2.0 * P.lambda2 * invL, M = P.M;
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) abuf[j] = (st[j] == kFree) ? fabs(v[j]) : -1.0;
  __syncthreads();
  int evals;
  const double tau = solve_tau(abuf, p, P.kbar, rho, M, -1.0, red, &evals);
  const double inv1p = 1.0 / (1.0 + rho);
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
    const double vj = v[j];
    const int s = st[j];
    double x = 0.0;
    if (s != kZero) {
      const double av = fabs(vj);
      double r = fmin(av * inv1p, M);
      if (s == kFree) r = fmin(r, fmax(av - tau, 0.0));
      x = (r == 0.0) ? 0.0 : copysign(r, vj);
    }
    out[j] = x;
  }
}

// The same prox with the node dimensions counted on the device, for callers
// that pass no host-side status: |J1| and |J_f| are reduced from st, kbar =
// min(k - |J1|, |J_f|).  *flag receives 0, or 1 for a status code outside
// {free, J0, J1}, or 2 for |J1| > k; out is not written when *flag != 0.
// abuf and the flag are caller-provided scratch (nothing needs clearing:
// every entry read is written first).  Its output equals k_prox's bit for bit.
__global__ __launch_bounds__(NT) void k_prox_counted(const double *v, double *out, int64_t p, double rho,
                                                     int k, double M, const int8_t *__restrict__ st,
                                                     double *abuf, int32_t *flag) {
  __shared__ double red[NW * 4];
  double cnt[3] = {0.0, 0.0, 0.0};  // |J1|, |J_f|, invalid codes
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
    const int s = st[j];
    cnt[0] += (s == kOne) ? 1.0 : 0.0;
    cnt[1] += (s == kFree) ? 1.0 : 0.0;
    cnt[2] += (s != kFree && s != kZero && s != kOne) ? 1.0 : 0.0;
    abuf[j] = (s == kFree) ? fabs(v[j]) : -1.0;
  }
  block_sum<NT, 3>(cnt, red);
  const int32_t err = cnt[2] > 0.0 ? 1 : (cnt[0] > (double)k ? 2 : 0);
  if (threadIdx.x == 0) *flag = err;
  if (err) return;  // uniform across the workgroup
  const double kb = fmin((double)k - cnt[0], cnt[1]);
  const int kbar = (int)kb;
  __syncthreads();
  int evals;
  const double tau = solve_tau(abuf, p, kbar, rho, M, -1.0, red, &evals);
  const double inv1p = 1.0 / (1.0 + rho);
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
    const double vj = v[j];
    const int s = st[j];
    double x = 0.0;
    if (s != kZero) {
      const double av = fabs(vj);
      double r = fmin(av * inv1p, M);
      if (s == kFree) r = fmin(r, fmax(av - tau, 0.0));
      x = (r == 0.0) ? 0.0 : copysign(r, vj);
    }
    out[j] = x;
  }
}

// g_N(beta) (Algorithm 1, +inf off dom) into out2[0]; g_N*(alpha) into out2[1].
__global__ __launch_bounds__(NT) void k_regularizer(const double *beta, const double *alpha, int64_t p,
                                                    int kbar, double M, const int8_t *__restrict__ st,
                                                    double *abuf, int32_t *sidx, double *sval,
                                                    double *out2) {
  __shared__ double red[NW * 4];
  __shared__ int scan[NW];
  __shared__ SelLds sel;
  if (beta) {
    IterStats is = finish_iterate(beta, st, p, kbar, M, abuf, sidx, sval, red, scan);
    if (threadIdx.x == 0) out2[0] = is.indom ? is.gval : INFINITY;
    __syncthreads();
  }
  if (alpha) {
    double s1[1] = {0.0};
#pragma unroll 8
    for (int64_t j = threadIdx.x; j < p; j += NT) {
      const int s = st[j];
      if (s == kOne) s1[0] += huber(alpha[j], M);
      abuf[j] = (s == kFree) ? fabs(alpha[j]) : -1.0;
    }
    block_sum<NT, 1>(s1, red);
    __syncthreads();
    const double ts = topsum_huber(abuf, p, kbar, M, sel, red);
    if (threadIdx.x == 0) out2[1] = s1[0] + ts;
  }
}

// Certified values of m batched nodes at their stopping iterates x (rows of
// X_it), all over the stored X: workgroup q takes F(Xx) and -F*(-zeta)
// (least squares zeta = 2 (y - X x), logistic zeta = -grad F(X x)) from the
// per-block sums of its loss row in block order, w = X^T zeta / (2 lambda2)
// from the split planes of the transposed product (row rs q) in plane order,
// and evaluates g_N(x) (Algorithm 1 with the domain
// test) and g_N*(w) (sum of H_M over J1 + TopSum of H_M over the free
// coordinates, eq. of g*): out[q] = {Psi(zeta), Phi(x)} (Phi = +inf off dom).
__global__ __launch_bounds__(NT) void k_cert_batch(const NodeParams *__restrict__ prm, const double *__restrict__ Xit,
                                                   const double *__restrict__ H, int KS, int Nr, int rs,
                                                   const double *__restrict__ fsum, int nfb, int64_t p,
                                                   double *__restrict__ abuf, int32_t *__restrict__ sidx,
                                                   double *__restrict__ sval, double *__restrict__ out) {
  __shared__ double red[NW * 4];
  __shared__ int scan[NW];
  __shared__ SelLds sel;
  const int q = blockIdx.x;
  const NodeParams P = prm[q];
  const double *x = Xit + (int64_t)q * p;
  double *a = abuf + (int64_t)q * p;
  double F = 0.0, Fs = 0.0;  // every thread sums the same values in the same order
  for (int b = 0; b < nfb; b++) {
    F += fsum[2 * ((int64_t)q * nfb + b)];
    Fs += fsum[2 * ((int64_t)q * nfb + b) + 1];
  }
  const IterStats is = finish_iterate(x, P.st, p, P.kbar, P.M, a, sidx + (int64_t)q * p, sval + (int64_t)q * p,
                                      red, scan);
  __syncthreads();
  const int64_t plane = (int64_t)Nr * p;
  // w = X^T zeta / (2 lambda2): least squares zeta = 2 r and the planes hold X^T r
  const double inv = (P.loss == kLsq ? 1.0 : 0.5) / P.lambda2;
  double s1[1] = {0.0};
  for (int64_t j = threadIdx.x; j < p; j += NT) {
    double h = 0.0;
    for (int z = 0; z < KS; z++) h += H[(int64_t)z * plane + (int64_t)rs * q * p + j];
    const double wj = h * inv;
    const int sj = P.st[j];
    if (sj == kOne) s1[0] += huber(wj, P.M);
    a[j] = (sj == kFree) ? fabs(wj) : -1.0;
  }
  block_sum<NT, 1>(s1, red);
  __syncthreads();
  const double gs = s1[0] + topsum_huber(a, p, P.kbar, P.M, sel, red);
  if (threadIdx.x == 0) {
    out[2 * q] = Fs - 2.0 * P.lambda2 * gs;
    out[2 * q + 1] = is.indom ? F + 2.0 * P.lambda2 * is.gval : INFINITY;
  }
}

// F(u), zeta = -grad F(u) and -F*(-zeta) for an arbitrary u (dual bound of a
// given beta).  sums_out = {F(u), -F*(-zeta)}.
__global__ __launch_bounds__(NT) void k_loss_terms(int32_t loss, const double *u, const double *y,
                                                   int64_t n, double *zeta, double *sums_out) {
  __shared__ double red[NW * 4];
  double v[2] = {0.0, 0.0};
  for (int64_t i = threadIdx.x; i < n; i += NT) {
    const double yi = y[i], ui = u[i];
    if (loss == kLsq) {
      const double r = yi - ui;
      zeta[i] = 2.0 * r;
      v[0] += r * r;
      v[1] += 2.0 * r * yi - r * r;
    } else {
      const double z = yi * ui;
      const double a = 1.0 / (1.0 + exp(z));
      zeta[i] = yi * a;
      v[0] += softplus(-z);
      v[1] += a * softplus(z) + (1.0 - a) * softplus(-z);
    }
  }
  block_sum<NT, 2>(v, red);
  if (threadIdx.x == 0) {
    sums_out[0] = v[0];
    sums_out[1] = v[1];
  }
}

// -F*(-zeta) of a given zeta into sums_out[1] (-inf if a logistic a_i = y_i
// zeta_i leaves [0, 1]).
__global__ __launch_bounds__(NT) void k_zeta_terms(int32_t loss, const double *zeta, const double *y,
                                                   int64_t n, double *sums_out) {
  __shared__ double red[NW * 4];
  double v[2] = {0.0, 0.0};  // value, number of entries out of the domain
  for (int64_t i = threadIdx.x; i < n; i += NT) {
    const double zi = zeta[i], yi = y[i];
    if (loss == kLsq) {
      v[0] += zi * yi - 0.25 * zi * zi;
    } else {
      const double a = yi * zi;
      if (a < 0.0 || a > 1.0) {
        v[1] += 1.0;
      } else {
        if (a > 0.0) v[0] -= a * log(a);
        if (a < 1.0) v[0] -= (1.0 - a) * log1p(-a);
      }
    }
  }
  block_sum<NT, 2>(v, red);
  if (threadIdx.x == 0) sums_out[1] = (v[1] > 0.0) ? -INFINITY : v[0];
}

__global__ __launch_bounds__(NT) void k_sumsq(const double *v, int64_t n, double *out) {
  __shared__ double red[NW * 4];
  double s[1] = {0.0};
#pragma unroll 8
  for (int64_t i = threadIdx.x; i < n; i += NT) s[0] += v[i] * v[i];
  block_sum<NT, 1>(s, red);
  if (threadIdx.x == 0) *out = s[0];
}

__global__ void k_scale_copy(const double *src, double *dst, double a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = a * src[i];
}

// One step of the Lanczos recurrence on A = X^T X.  On entry w = A v_j;
// w <- w - alpha_j v_j - beta_{j-1} v_{j-1}, beta_j = ||w||, then
// v_{j-1} <- v_j and v_j <- w / beta_j (zero when beta_j = 0).  alpha_j and
// beta_{j-1} come from device memory (no beta_{j-1} at j = 0); beta_j is
// written to beta_out.  Every thread owns the same indices in both passes.
__global__ __launch_bounds__(NT) void k_lanczos(double *w, double *v, double *vprev, const double *alpha,
                                                const double *beta_prev, double *beta_out, int64_t p) {
  __shared__ double red[NW * 4];
  const double a = *alpha;
  const double b = beta_prev ? *beta_prev : 0.0;
  double s[1] = {0.0};
#pragma unroll 8
  for (int64_t i = threadIdx.x; i < p; i += NT) {
    double t = w[i] - a * v[i];
    if (beta_prev) t -= b * vprev[i];
    w[i] = t;
    s[0] += t * t;
  }
  block_sum<NT, 1>(s, red);
  const double nb = sqrt(s[0]);
  if (threadIdx.x == 0) *beta_out = nb;
  const double inv = nb > 0.0 ? 1.0 / nb : 0.0;
#pragma unroll 8
  for (int64_t i = threadIdx.x; i < p; i += NT) {
    vprev[i] = v[i];
    v[i] = w[i] * inv;
  }
}

__global__ void k_iota(int32_t *idx, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    idx[i] = (int32_t)i;
}


// ------------------------------------------------------------ register-resident node routines
//
// For p <= 16384 every thread keeps EPT = ceil(p / 512) coordinates
// j = tid + e * 512 (coalesced) in one register array, with the node status
// packed 2 bits per coordinate (3 = beyond p).  The passes of the selection,
// the threshold search and Algorithm 1 read their entries through a functor
// aval(e) (>= 0: a free entry; < 0: ignored), so only one FP64 array is live.

template <int EPT>
struct PackedStatus {
  uint32_t w[(EPT + 15) / 16];
  __device__ __forceinline__ int operator()(int e) const { return (int)((w[e >> 4] >> (2 * (e & 15))) & 3u); }
  __device__ __forceinline__ void load(const int8_t *__restrict__ st, int64_t p) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < (EPT + 15) / 16; q++) w[q] = 0u;
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const int64_t j = tid + (int64_t)e * NT;
      const uint32_t c = (j < p) ? (uint32_t)st[j] : 3u;
      w[e >> 4] |= c << (2 * (e & 15));
    }
  }
};

template <int EPT, class F>
__device__ double select_kth_f(F aval, int k, SelLds &sm) {
  const int tid = threadIdx.x;
  unsigned long long prefix = 0ull;
  int above = 0, shift = 52, width = 11;
  for (;;) {
    for (int b = tid; b < 2048; b += NT) sm.hist[b] = 0u;
    __syncthreads();
    const unsigned long long mask = (1ull << width) - 1ull;
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const double x = aval(e);
      if (x >= 0.0) {
        const unsigned long long key = (unsigned long long)__double_as_longlong(x);
        if ((key >> (shift + width)) == prefix) atomicAdd(&sm.hist[(key >> shift) & mask], 1u);
      }
    }
    __syncthreads();
    hist_locate(sm, above, k);
    const int B = sm.bin, cnt = sm.cnt;
    above = sm.above;
    prefix = (prefix << width) | (unsigned long long)B;
    if (shift == 0) {
      __syncthreads();
      return __longlong_as_double((long long)prefix);
    }
    if (cnt <= 64) {
      if (tid == 0) sm.ngat = 0;
      __syncthreads();
#pragma unroll
      for (int e = 0; e < EPT; e++) {
        const double x = aval(e);
        if (x >= 0.0) {
          const unsigned long long key = (unsigned long long)__double_as_longlong(x);
          if ((key >> shift) == prefix) {
            const int pos = atomicAdd(&sm.ngat, 1);
            if (pos < 64) sm.gat[pos] = x;
          }
        }
      }
      __syncthreads();
      if (tid < 64) {
        double v = (tid < cnt) ? sm.gat[tid] : -1.0;
        v = wave_sort_desc(v);
        if (tid == k - above - 1) sm.result = v;
      }
      __syncthreads();
      const double r = sm.result;
      __syncthreads();
      return r;
    }
    const int nw = shift < 11 ? shift : 11;
    shift -= nw;
    width = nw;
  }
}

template <int EPT, class F>
__device__ double alg1_f(F aval, int kbar, double theta, double *red) {
  if (kbar <= 0 || !(theta > 0.0)) return 0.0;
  const double K = (double)kbar;
  double s = theta / K;
  double prevK = 0.0;
  for (int it = 0; it <= kbar + 1; it++) {
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const double x = aval(e);
      if (x >= 0.0) {
        if (x > s) {
          v[0] += 1.0;
          v[2] += x * x;
        } else {
          v[1] += x;
        }
      }
    }
    block_sum<NT, 3>(v, red);
    if (v[0] == prevK || v[0] >= K) return 0.5 * (v[2] + (K - v[0]) * s * s);
    prevK = v[0];
    s = fmin(s, v[1] / (K - v[0]));
  }
  return NAN;
}

struct NodeLds {
  double red[NW * 4];
  int scan[NW];
  int cnt_ew[256];   // EPT * NW <= 256
  SelLds sel;
  double bcd[4];
  int bci[4];
};

// Support list (ascending j), Algorithm 1 value and dom test of the iterate x
// held in registers.
template <int EPT>
__device__ IterStats finish_r(const double (&x)[EPT], const PackedStatus<EPT> &sv, int kbar, double M,
                              int32_t *__restrict__ sidx, double *__restrict__ sval, NodeLds &L) {
  const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
  double v[2] = {0.0, 0.0};  // theta, sum_{J1} x^2
  double amax = 0.0, j0max = 0.0, boxmax = 0.0;
#pragma unroll
  for (int e = 0; e < EPT; e++) {
    const int s = sv(e);
    const double xj = x[e];
    const double ax = fabs(xj);
    if (s != 3) {
      amax = fmax(amax, ax);
      if (s == kZero) j0max = fmax(j0max, ax);
      else boxmax = fmax(boxmax, ax);
      if (s == kFree) v[0] += ax;
      else if (s == kOne) v[1] += xj * xj;
    }
    const unsigned long long m = __ballot(s != 3 && xj != 0.0);
    if (lane == 0) L.cnt_ew[e * NW + w] = __popcll(m);
  }
  __syncthreads();
  const int c = (tid < EPT * NW) ? L.cnt_ew[tid] : 0;
  int tot;
  const int off = block_excl_scan<NT>(c, L.scan, &tot);
  __syncthreads();
  if (tid < EPT * NW) L.cnt_ew[tid] = off;
  __syncthreads();
  const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
  for (int e = 0; e < EPT; e++) {
    const bool nz = sv(e) != 3 && x[e] != 0.0;
    const unsigned long long m = __ballot(nz);
    if (nz) {
      const int pos = L.cnt_ew[e * NW + w] + __popcll(m & below);
      sidx[pos] = (int32_t)(tid + e * NT) | (sv(e) == kOne ? kJ1Flag : (sv(e) == kZero ? kJ0Flag : 0));
      sval[pos] = x[e];
    }
  }
  block_sum<NT, 2>(v, L.red);
  const double gA = block_max<NT>(amax, L.red);
  const double g0 = block_max<NT>(j0max, L.red);
  const double gB = block_max<NT>(boxmax, L.red);
  const double zt = 1e-9 * fmax(1.0, gA);
  int ok = (g0 <= zt);
  if (isfinite(M) && gB > M * (1.0 + 1e-9)) ok = 0;
  if (kbar == 0) {
    if (v[0] > zt) ok = 0;
  } else if (isfinite(M) && v[0] > M * (double)kbar * (1.0 + 1e-9)) {
    ok = 0;
  }
  auto aval = [&](int e) { return sv(e) == kFree ? fabs(x[e]) : -1.0; };
  const double gv = 0.5 * v[1] + alg1_f<EPT>(aval, kbar, v[0], L.red);
  return IterStats{gv, ok, tot};
}

template <int EPT>
__global__ __launch_bounds__(NT) void k_node_init_r(const NodeParams *__restrict__ prm, NodeState *S,
                                                    NodeBufs nb, const double *__restrict__ beta0, double L) {
  __shared__ NodeLds lds;
  const int tid = threadIdx.x;
  const int64_t p = prm->p;
  PackedStatus<EPT> sv;
  sv.load(prm->st, p);
  double x[EPT];
#pragma unroll
  for (int e = 0; e < EPT; e++) {
    const int64_t j = tid + (int64_t)e * NT;
    x[e] = 0.0;
    if (j < p) {
      const double b = beta0 ? beta0[j] : 0.0;
      x[e] = b;
      nb.x0[j] = b;
      nb.xbest[j] = b;
      nb.x1[j] = 0.0;
      nb.hprev[j] = 0.0;
    }
  }
  IterStats is = finish_r<EPT>(x, sv, prm->kbar, prm->M, nb.sidx, nb.sval, lds);
  if (tid == 0) {
    NodeState s{};
    s.L = L;
    s.t = 1.0;
    s.gap_ref = INFINITY;
    s.lb = -INFINITY;
    s.ub = INFINITY;
    s.phi = INFINITY;
    s.psi = -INFINITY;
    s.rel_gap = INFINITY;
    s.gval = is.gval;
    s.tau = -1.0;
    s.tk = -1.0;
    s.tkw = 0.25;
    s.status = kMaxIter;
    s.nsupp = is.nsupp;
    s.indom = is.indom;
    s.bt = is_bt(prm->method) ? 1 : 0;
    *S = s;
  }
}

// ---- single-node step, latency-ordered
//
// One workgroup owns the node.  Every global load of the step is issued in
// the prologue (status as packed 2-bit words, X^T r, the two last iterates,
// the previous gradient), the reductions take one barrier each (two
// alternating LDS slots), and the dual's top-kbar selection first tries a
// window around the previous iteration's kbar-th value: when the window
// brackets the new kbar-th value and holds at most kWinCap entries, one wave
// sorts them and no radix pass is needed.

// Workgroup sums (and maxima) with one barrier: reduction i writes slot i % 2
// before its barrier and reads it after.  A thread writes for reduction i + 1
// only after it has read reduction i's slot, and slot i % 2 is written again
// by reduction i + 2 only after every thread has passed barrier i + 1, so no
// second barrier is needed.  Every thread must run the same sequence.
struct Red2 {
  double *buf;  // 2 * NW * 8 doubles of LDS
  int ph;
  template <int KS, int KM>
  __device__ __forceinline__ void run(double *s, double *m) {
    constexpr int K = KS + KM;
    static_assert(K >= 1 && K <= 8, "at most 8 values per reduction");
#pragma unroll
    for (int k = 0; k < KS; k++) s[k] = wave_sum(s[k]);
#pragma unroll
    for (int k = 0; k < KM; k++) m[k] = wave_max(m[k]);
    double *r = buf + ph * (NW * 8);
    if (lane_id() == 0) {
#pragma unroll
      for (int k = 0; k < KS; k++) r[wave_id() * K + k] = s[k];
#pragma unroll
      for (int k = 0; k < KM; k++) r[wave_id() * K + KS + k] = m[k];
    }
    lds_barrier();
#pragma unroll
    for (int k = 0; k < KS; k++) {
      double acc = 0.0;
      for (int w = 0; w < NW; w++) acc += r[w * K + k];
      s[k] = acc;
    }
#pragma unroll
    for (int k = 0; k < KM; k++) {
      double acc = r[KS + k];
      for (int w = 1; w < NW; w++) acc = fmax(acc, r[w * K + KS + k]);
      m[k] = acc;
    }
    ph ^= 1;
  }
  template <int KS>
  __device__ __forceinline__ void sum(double (&s)[KS]) {
    run<KS, 0>(s, nullptr);
  }
  template <int KS, int KM>
  __device__ __forceinline__ void summax(double (&s)[KS], double (&m)[KM]) {
    run<KS, KM>(s, m);
  }
};

constexpr int kWinCap = 64;  // window entries one wave sorts

template <int EPT>
struct StepLds {
  double red[2 * NW * 8];
  SelLds sel;
  int cnt[EPT * NW];       // support entries per (e, wave) group
  int ofs[NW][EPT * NW];   // each wave's copy of their exclusive prefix
  double xsum[NW * 2];     // per-wave partials summed beside the support list's count exchange
  double bcd[4];
  int bci[4];
};

template <int EPT>
__device__ __forceinline__ void load_packed_status(PackedStatus<EPT> &sv, const uint32_t *__restrict__ stp) {
#pragma unroll
  for (int q = 0; q < (EPT + 15) / 16; q++) sv.w[q] = stp[q * NT + threadIdx.x];
}

// The prox threshold tau of the pooled-threshold form (same search as
// solve_tau above) over the register-resident magnitudes aval(e), warm-started
// from the previous iteration's tau, one-barrier reductions.
template <int EPT, class F>
__device__ __forceinline__ double solve_tau_2(F aval, int kbar, double rho, double M, double warm, Red2 &R, int *evals) {
  double st[2] = {0.0, 0.0};
  double mx[1] = {0.0};
#pragma unroll
  for (int e = 0; e < EPT; e++) {
    const double x = aval(e);
    if (x > 0.0) {
      st[0] += 1.0;
      st[1] += x;
      mx[0] = fmax(mx[0], x);
    }
  }
  R.summax(st, mx);
  const double amax = mx[0];
  *evals = 0;
  if (kbar <= 0) return INFINITY;
  const double K = (double)kbar;
  if (st[0] <= K) return 0.0;
  const bool finM = isfinite(M);
  auto Dof = [&](double t) { return finM ? fmin(t / rho, M) : t / rho; };
  auto froot = [&](double h, double nb, double sB) -> double {
    if (nb <= 0.0) return NAN;
    if (finM) {
      const double Sf = h + (sB - nb * rho * M) / M;
      if (Sf >= K) return (sB - M * (K - h)) / nb;
    }
    return rho * sB / (K - h + rho * nb);
  };
  double lo = 0.0, hi = amax;
  double tau = (warm > lo && warm < hi) ? warm : froot(0.0, st[0], st[1]);
  if (!(tau > lo && tau < hi)) tau = 0.5 * (lo + hi);
  bool from_root = false;
  double ph = -1.0, pb = -1.0;
  int nsteps = 0;
  double wref = hi - lo;
  for (int it = 0; it < 200; it++) {
    const double D = Dof(tau);
    double v[3] = {0.0, 0.0, 0.0};
    const double top = tau + D;
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const double x = aval(e);
      if (x > tau) {
        v[1] += 1.0;
        if (x > top) v[0] += 1.0;
        else v[2] += x;
      }
    }
    R.sum(v);
    *evals = it + 1;
    if (from_root && v[0] == ph && v[1] == pb) return tau;
    const double S = v[0] + (v[2] - (v[1] - v[0]) * tau) / D;
    if (S > K) lo = tau;
    else if (S < K) hi = tau;
    else return tau;
    double c = froot(v[0], v[1] - v[0], v[2]);
    if (c == tau) return tau;
    if (nsteps >= 2 && hi - lo > 0.5 * wref) {
      nsteps = 0;
      wref = hi - lo;
      c = NAN;
    }
    if (c > lo && c < hi) {
      from_root = true;
      nsteps++;
    } else {
      c = 0.5 * (lo + hi);
      from_root = false;
      nsteps = 0;
      wref = hi - lo;
    }
    ph = v[0];
    pb = v[1];
    if (!(c > lo && c < hi)) return c;
    tau = c;
  }
  return tau;
}

template <int EPT, class F>
__device__ __forceinline__ double alg1_2(F aval, int kbar, double theta, Red2 &R) {
  if (kbar <= 0 || !(theta > 0.0)) return 0.0;
  const double K = (double)kbar;
  double s = theta / K;
  double prevK = 0.0;
  for (int it = 0; it <= kbar + 1; it++) {
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const double x = aval(e);
      if (x >= 0.0) {
        if (x > s) {
          v[0] += 1.0;
          v[2] += x * x;
        } else {
          v[1] += x;
        }
      }
    }
    R.sum(v);
    if (v[0] == prevK || v[0] >= K) return 0.5 * (v[2] + (K - v[0]) * s * s);
    prevK = v[0];
    s = fmin(s, v[1] / (K - v[0]));
  }
  return NAN;
}

// Support list of the iterate x held in registers (ascending j, every nonzero;
// J1 / J0 entries flagged with kJ1Flag / kJ0Flag).  Groups (e, wave) come in
// j order o = e * NW + w; after one barrier every wave scans all group counts
// itself.  Returns the list length.
template <int EPT>
__device__ __forceinline__ int support_list_2(const double (&x)[EPT], const PackedStatus<EPT> &sv,
                                              int32_t *__restrict__ sidx, double *__restrict__ sval,
                                              StepLds<EPT> &L, double *xs = nullptr) {
  constexpr int NO = EPT * NW;
  constexpr int C = (NO + 63) / 64;
  const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
#pragma unroll
  for (int e = 0; e < EPT; e++) {
    const unsigned long long mk = __ballot(sv(e) != 3 && x[e] != 0.0);
    if (lane == 0) L.cnt[e * NW + w] = __popcll(mk);
  }
  // optional: two per-thread partials summed over the block through the same
  // barrier (per-wave sums in wave order, the same value in every thread)
  if (xs) {
#pragma unroll
    for (int k = 0; k < 2; k++) {
      const double v = wave_sum(xs[k]);
      if (lane == 0) L.xsum[w * 2 + k] = v;
    }
  }
  lds_barrier();
  if (xs) {
#pragma unroll
    for (int k = 0; k < 2; k++) {
      double acc = 0.0;
      for (int q = 0; q < NW; q++) acc += L.xsum[q * 2 + k];
      xs[k] = acc;
    }
  }
  int c[C];
  int loc = 0;
#pragma unroll
  for (int q = 0; q < C; q++) {
    const int o = lane * C + q;
    c[q] = (o < NO) ? L.cnt[o] : 0;
    loc += c[q];
  }
  int incl = loc;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  const int tot = __shfl(incl, 63, 64);
  int run = incl - loc;
#pragma unroll
  for (int q = 0; q < C; q++) {
    const int o = lane * C + q;
    if (o < NO) L.ofs[w][o] = run;
    run += c[q];
  }
  __asm__ volatile("" ::: "memory");  // this wave's LDS writes stay ahead of its reads
  const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
  for (int e = 0; e < EPT; e++) {
    const bool nz = sv(e) != 3 && x[e] != 0.0;
    const unsigned long long mk = __ballot(nz);
    if (nz) {
      const uint32_t pos = (uint32_t)(L.ofs[w][e * NW + w] + __popcll(mk & below));
      sidx[pos] = (int32_t)(tid + e * NT) | (sv(e) == kOne ? kJ1Flag : (sv(e) == kZero ? kJ0Flag : 0));
      sval[pos] = x[e];
    }
  }
  return tot;
}

// Support list, Algorithm 1 value and dom test of the iterate x held in
// registers.
template <int EPT>
__device__ __forceinline__ IterStats finish_2(const double (&x)[EPT], const PackedStatus<EPT> &sv, int kbar, double M,
                              int32_t *__restrict__ sidx, double *__restrict__ sval, StepLds<EPT> &L, Red2 &R) {
  double sm[2] = {0.0, 0.0};       // theta, sum_{J1} x^2
  double mx[3] = {0.0, 0.0, 0.0};  // max |x|, over J0, over the box coordinates
#pragma unroll
  for (int e = 0; e < EPT; e++) {
    const int s = sv(e);
    const double xj = x[e];
    const double ax = fabs(xj);
    if (s != 3) {
      mx[0] = fmax(mx[0], ax);
      if (s == kZero) mx[1] = fmax(mx[1], ax);
      else mx[2] = fmax(mx[2], ax);
      if (s == kFree) sm[0] += ax;
      else if (s == kOne) sm[1] += xj * xj;
    }
  }
  const int tot = support_list_2<EPT>(x, sv, sidx, sval, L);
  R.summax(sm, mx);
  const double gA = mx[0], g0 = mx[1], gB = mx[2];
  const double zt = 1e-9 * fmax(1.0, gA);
  int ok = (g0 <= zt);
  if (isfinite(M) && gB > M * (1.0 + 1e-9)) ok = 0;
  if (kbar == 0) {
    if (sm[0] > zt) ok = 0;
  } else if (isfinite(M) && sm[0] > M * (double)kbar * (1.0 + 1e-9)) {
    ok = 0;
  }
  auto aval = [&](int e) { return sv(e) == kFree ? fabs(x[e]) : -1.0; };
  const double gv = 0.5 * sm[1] + alg1_2<EPT>(aval, kbar, sm[0], R);
  return IterStats{gv, ok, tot};
}

template <int EPT, bool BT>
__global__ __launch_bounds__(NT) void k_node_step_r(const NodeParams *__restrict__ prm, NodeState *S,
                                                    NodeBufs nb, ProbBufs B, StepArgs A) {
  __shared__ StepLds<EPT> lds;
  // with 32 entries per thread the radix selection reads the magnitudes from
  // LDS (the register-resident passes would not stay in registers)
  constexpr bool kSelLds = EPT > 16;
  __shared__ double wl[kSelLds ? EPT * NT : 1];
  const int tid = threadIdx.x;
  const int64_t p = A.p;
  const double *__restrict__ gb = A.gb;
  const int parity = A.parity;
  // scalar state and parameters: independent loads, issued together with the
  // vector loads below; the done test waits for them only after those
  const int done0 = S->done, indom0 = S->indom, it0 = S->iter;
  const double L = S->L, gval0 = S->gval, tau0 = S->tau, tkp = S->tk, dlt = S->tkw, dxy0 = S->dxy;
  const double btA = S->bt_A;
  const int kbar = prm->kbar, loss = prm->loss;
  const double lam2 = prm->lambda2, M = prm->M;
  // backtracking (a compile-time variant, so the fixed-step kernel carries none
  // of its registers)
  constexpr bool bt = BT;
  // x^k (backtracking: a rejected trial is overwritten by the last accepted
  // iterate through xcw, so xc carries no restrict qualifier)
  const double *xc = parity ? nb.x1 : nb.x0;
  double *xcw = parity ? nb.x1 : nb.x0;
  double *__restrict__ xn = parity ? nb.x0 : nb.x1;  // holds x^{k-1}, receives x^{k+1}
  // the loads of the step: X^T r (Gram mode: b - G x), x^k and b first; the
  // operands of the gradient step (x^{k-1}, previous gradient) are issued
  // once b has been consumed and arrive during the dual evaluation (with 16
  // or more entries per thread they are loaded at the gradient step instead,
  // which keeps the selection passes out of scratch memory; with 32 entries
  // x^k is not held either: the gradient step loads its operands in halves)
  constexpr bool kPre = EPT <= 8;
  constexpr bool kHoldXk = EPT <= 16;
  constexpr int EK = kHoldXk ? EPT : 1;
  PackedStatus<EPT> sv;
  load_packed_status<EPT>(sv, A.stp);
  double x[EPT], xk[EK], xq[EK], g2[EK];
  double r1[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if constexpr (kHoldXk) {
    double bv[EPT];
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const uint32_t j = (uint32_t)(tid + e * NT);
      const bool in = j < (uint32_t)p;
      x[e] = in ? B.h1[j] : 0.0;
      xk[e] = in ? xc[j] : 0.0;
      bv[e] = (in && gb) ? gb[j] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      r1[1] += xk[e] * (bv[e] + x[e]);
      r1[2] += bv[e] * xk[e];
    }
  } else {
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const uint32_t j = (uint32_t)(tid + e * NT);
      x[e] = j < (uint32_t)p ? B.h1[j] : 0.0;
    }
    if (gb) {
#pragma unroll
      for (int e = 0; e < EPT; e++) {
        const uint32_t j = (uint32_t)(tid + e * NT);
        if (j < (uint32_t)p) {
          const double xv = xc[j], bj = gb[j];
          r1[1] += xv * (bj + x[e]);
          r1[2] += bj * xv;
        }
      }
    }
  }
  // loss sums of the finalize blocks: lane-parallel loads, fixed-order wave sums
  double Fk = 0.0, negconj = 0.0;
  if (!gb) {
    for (int i = lane_id(); i < B.nfin; i += 64) {
      Fk += B.rbsum[2 * i];
      negconj += B.rbsum[2 * i + 1];
    }
  }
  if (done0) return;
  const double *__restrict__ gp = (loss == kLsq) ? nb.hprev : B.h2;
  if (kPre) {
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const uint32_t j = (uint32_t)(tid + e * NT);
      const bool in = j < (uint32_t)p;
      xq[e] = in ? xn[j] : 0.0;
      g2[e] = in ? gp[j] : 0.0;
    }
  }
  Red2 R;
  R.buf = lds.red;
  R.ph = 0;
  if (tid == 0) lds.sel.ngat = 0;
  if (!gb) {
    Fk = wave_sum(Fk);
    negconj = wave_sum(negconj);
  }
  // The proximal step from v (in x[]) with step constant Ls, shared by the
  // accepted and the rejected branch: x[] <- prox_{(2 lambda2 / Ls) g_N}(v)
  // by the pooled threshold, written to xn (after a rejected trial the last
  // accepted iterate moves from xn to the current buffer first, so that the
  // parity of the next evaluation finds the new trial current and x^k
  // previous); backtracking keeps ||x - y||^2 and (least squares) the part
  // (x - y)^T h(y) of the model test of the new trial (h(y) = -grad f(y) / 2),
  // with y and grad f(y) in xq[] and g2[] where x^k is held in registers.
  auto prox_finish = [&](double Ls, bool rejected) {
    const double rho = 2.0 * lam2 / Ls;
    int evals = 0;
    auto vabs = [&](int e) { return sv(e) == kFree ? fabs(x[e]) : -1.0; };
    const double tau = solve_tau_2<EPT>(vabs, kbar, rho, M, tau0, R, &evals);
    const double inv1p = 1.0 / (1.0 + rho);
    double dxy[2] = {0.0, 0.0};
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const int s = sv(e);
      double xv = 0.0;
      if (s != 3) {
        if (s != kZero) {
          const double av = fabs(x[e]);
          double r = fmin(av * inv1p, M);
          if (s == kFree) r = fmin(r, fmax(av - tau, 0.0));
          xv = (r == 0.0) ? 0.0 : copysign(r, x[e]);
        }
        const uint32_t j = (uint32_t)(tid + e * NT);
        if (rejected) xcw[j] = xn[j];
        xn[j] = xv;
        if (bt) {
          // y from registers (x^k held) or from the LDS copy the gradient
          // step left (32 entries per thread); grad f(y) only for Gram's A
          double yv;
          if constexpr (kHoldXk) yv = xq[e];
          else yv = wl[j];
          const double dy = xv - yv;
          dxy[0] += dy * dy;
          if (A.gb) {
            double gv;
            if constexpr (kHoldXk) gv = g2[e];
            else gv = nb.gbt[j];
            dxy[1] -= 0.5 * dy * gv;
          }
        }
      }
      x[e] = xv;
    }
    if (A.gb) {
      // Gram mode: no X^T r product follows, so the step evaluates g_N of the
      // new iterate and its dom test itself
      if (bt) R.sum(dxy);
      IterStats is = finish_2<EPT>(x, sv, kbar, M, nb.sidx, nb.sval, lds, R);
      if (tid == 0) {
        S->gval = is.gval;
        S->indom = is.indom;
        S->nsupp = is.nsupp;
      }
    } else {
      // the extra workgroup of the next X^T r product evaluates them from this
      // support list (S->gval / S->indom before the next step reads them);
      // backtracking's sums ride on the list's count exchange
      const int nsupp = support_list_2<EPT>(x, sv, nb.sidx, nb.sval, lds, bt ? dxy : nullptr);
      if (tid == 0) S->nsupp = nsupp;
    }
    if (tid == 0) {
      S->tau = tau;
      S->tau_iters = evals;
      S->parity = parity ^ 1;
      if (!rejected) S->iter = S->iter + 1;
      if (bt) {
        S->L = Ls;
        S->dxy = dxy[0];
        S->bt_A = dxy[1];
        S->bt_acc = rejected ? 0 : 1;
        if (rejected) {
          S->trials = S->trials + 1;
          S->improved = 0;
        }
      }
    }
  };
  // Backtracking: every point after the start is a trial of the step from the
  // momentum point y; it is accepted when f(x) - f(y) - <grad f(y), x - y> <=
  // (L / 2) ||x - y||^2 (or L has reached Lmax), else the step is redone
  // from the saved y and grad f(y) with c L, and the trial is not evaluated.
  // The test needs f(x) - f(y) - <grad f(y), x - y>: from the loss
  // epilogue's row-wise remainder (least squares ||X x - X y||^2; the X^T pass
  // before this step took the same decision and skipped a rejected trial), in
  // Gram mode ||X (x - y)||^2 = (x - y)^T (h(y) - h(x)) = A - (x - y)^T h(x),
  // A kept by the step that made x and the second term summed with the dual's
  // first reduction below (h = b - G .).
  const bool trial = bt && it0 > 0;
  const bool trial_ls = trial && gb != nullptr;
  double dlog = 0.0;
  if (trial && !gb) dlog = bt_remainder(B.dsum, B.nfin);
  // dual value at x^k: w = X^T zeta / (2 lambda2); the top-kbar window of
  // free |w| around the previous kbar-th value
  const double wscale = (loss == kLsq) ? 1.0 / lam2 : 0.5 / lam2;
  const bool wv = tkp > 0.0 && kbar > 0;
  const double wa = wv ? tkp * (1.0 - dlt) : INFINITY, wb = wv ? tkp * (1.0 + dlt) : INFINITY;
  // r1: sum_{J1} H_M(w_j); Gram: x^T (b + h), b^T x; #{w > wb}, #{w >= wa}, sum_{w > wb} H_M(w);
  // backtracking least squares: (x - y)^T h(x)
  double r1x[1] = {0.0};
#pragma unroll
  for (int e = 0; e < EPT; e++) {
    const int s = sv(e);
    if (s == 3) continue;
    const double w = x[e] * wscale;
    if (s == kOne) r1[0] += huber(w, M);
    if (s == kFree) {
      const double aw = fabs(w);
      if (aw > wb) {
        r1[3] += 1.0;
        r1[5] += huber(aw, M);
      }
      if (aw >= wa) r1[4] += 1.0;
    }
    if (trial_ls) {
      const uint32_t j = (uint32_t)(tid + e * NT);
      double xe;
      if constexpr (kHoldXk) xe = xk[e];
      else xe = xc[j];
      r1x[0] += (xe - nb.ybt[j]) * x[e];
    }
  }
  if (trial_ls) {
    double r7[7] = {r1[0], r1[1], r1[2], r1[3], r1[4], r1[5], r1x[0]};
    R.sum(r7);
#pragma unroll
    for (int q = 0; q < 6; q++) r1[q] = r7[q];
    r1x[0] = r7[6];
  } else {
    R.sum(r1);
  }
  // Backtracking: every point after the start is a trial of the step from the
  // momentum point y; it is accepted when f(x) - f(y) - <grad f(y), x - y> <=
  // (L / 2) ||x - y||^2 (or L has reached Lmax), else the step is redone
  // from the saved y and grad f(y) with c L, and the trial is not evaluated.
  // a rejected trial skips the evaluation; both branches end in one prox step
  bool rejected = false;
  double Lstep = L;
  if (trial) {
    const double dv = trial_ls ? btA - r1x[0] : dlog;
    if (!bt_accept(dv, L, dxy0, prm->Lmax)) {
      const double Ls = fmin(prm->ls_c * L, prm->Lmax);
      const double invLs = 1.0 / Ls;
#pragma unroll
      for (int e = 0; e < EPT; e++) {
        const uint32_t j = (uint32_t)(tid + e * NT);
        const bool in = sv(e) != 3;
        const double yj = in ? nb.ybt[j] : 0.0, gj = in ? nb.gbt[j] : 0.0;
        if constexpr (kHoldXk) {
          xq[e] = yj;
          g2[e] = gj;
        } else {
          wl[j] = yj;
        }
        x[e] = in ? yj - gj * invLs : 0.0;
      }
      Lstep = Ls;
      rejected = true;
    }
  }
  if (!rejected) {
    if (gb) {
      // F(X x) = y^T y - x^T (b + h) and -F*(-zeta) = 2 (y^T y - b^T x) - F, as
      // h = b - G x: both from the Gram quantities, no pass over X
      const double yy = prm->gram_yy;
      Fk = yy - r1[1];
      negconj = 2.0 * (yy - r1[2]) - Fk;
    }
    auto wabs = [&](int e) { return sv(e) == kFree ? fabs(x[e] * wscale) : -1.0; };
    const double cgt = r1[3], cge = r1[4];
    const bool fast = wv && cgt < (double)kbar && (double)kbar <= cge && cge - cgt <= (double)kWinCap;
    double topsum = 0.0, tkn = -1.0;
    if (kbar > 0 && fast) {
#pragma unroll
      for (int e = 0; e < EPT; e++) {
        const double aw = wabs(e);
        if (aw >= wa && aw <= wb) lds.sel.gat[atomicAdd(&lds.sel.ngat, 1)] = aw;
      }
      lds_barrier();
      if (wave_id() == 0) {
        const int lane = lane_id();
        const int cw = (int)(cge - cgt);
        const int mm = kbar - (int)cgt;  // 1 <= mm <= cw
        double v = (lane < cw) ? lds.sel.gat[lane] : -1.0;
        v = wave_sort_desc(v);
        tkn = __shfl(v, mm - 1, 64);
        topsum = r1[5] + wave_sum(lane < mm ? huber(v, M) : 0.0);
      }
    } else if (kbar > 0) {
      if constexpr (kSelLds) {
#pragma unroll
        for (int e = 0; e < EPT; e++) wl[tid + e * NT] = wabs(e);
        __syncthreads();
        tkn = select_kth(wl, (int64_t)EPT * NT, kbar, lds.sel);
      } else {
        tkn = select_kth_f<EPT>(wabs, kbar, lds.sel);
      }
      const double Ht = huber(tkn, M);
      double v1[1] = {0.0};
#pragma unroll
      for (int e = 0; e < EPT; e++) {
        const double aw = wabs(e);
        if (aw >= 0.0) v1[0] += fmax(huber(aw, M) - Ht, 0.0);
      }
      R.sum(v1);
      topsum = (double)kbar * Ht + v1[0];
    }
    if (tid == 0) {
      const double psi = negconj - 2.0 * lam2 * (r1[0] + topsum);
      const double phi = indom0 ? Fk + 2.0 * lam2 * gval0 : INFINITY;
      const int it = S->iter;
      if (prm->trace && it <= prm->max_iter) {
        prm->trace[2 * it] = phi;
        prm->trace[2 * it + 1] = psi;
      }
      const double gap = phi - psi;
      double lb = S->lb, ub = S->ub;
      int improved = 0, ub_improved = 0;
      if (psi > lb) {
        lb = psi;
        improved = 1;
      }
      if (phi < ub) {
        ub = phi;
        ub_improved = 1;
      }
      const double rel = (ub - lb) / fmax(fabs(ub), 1e-300);
      int done = 0, status = kMaxIter;
      if (rel <= prm->tol) {
        done = 1;
        status = kConverged;
      } else if (!isnan(prm->cutoff) && lb >= prm->cutoff) {
        done = 1;
        status = kCutoffPrune;
      } else if (!isnan(prm->cutoff) && ub <= prm->cutoff) {
        done = 1;
        status = kCutoffBranch;
      } else if (it >= prm->max_iter) {
        done = 1;
        status = kMaxIter;
      }
      double m = 0.0, t = S->t, gap_ref = S->gap_ref;
      int restart = 0, restarts = S->restarts;
      if (!done) {
        restart = decide_restart(prm, it, gap, phi, S->phi, gap_ref, restarts);
        if (restart) {
          m = 0.0;
          t = 1.0;
        } else {
          const double tn = fista_next_t(t);
          m = (t - 1.0) / tn;
          t = tn;
        }
      }
      // next window: twice the relative move of the kbar-th value, narrowed when
      // the window held the value but had too many entries
      double tw = 0.25;
      if (wv && tkn > 0.0) tw = fmin(0.25, fmax(1e-12, 2.0 * fabs(tkn - tkp) / tkn));
      if (wv && !fast && cgt < (double)kbar && (double)kbar <= cge) tw = fmin(tw, 0.25 * dlt);
      S->phi = phi;
      S->psi = psi;
      S->lb = lb;
      S->ub = ub;
      S->rel_gap = rel;
      S->improved = improved;
      S->status = status;
      S->t = t;
      S->gap_ref = gap_ref;
      S->restarts = restarts;
      S->mom = m;
      S->tk = tkn;
      S->tkw = tw;
      if (done) S->done = 1;
      lds.bcd[0] = m;
      lds.bci[0] = done;
      lds.bci[1] = restart;
      lds.bci[2] = ub_improved;
      lds.bci[3] = improved;
    }
    lds_barrier();
    const bool done = lds.bci[0] != 0;
    const double m = lds.bcd[0];
    const int restart = lds.bci[1];
    // backtracking: a restart runs the method afresh, the line search from L0
    const double Lnew = (bt && restart) ? prm->L0 : L;
    const double invL = 1.0 / Lnew;
    // gradient step at the momentum point on entries [e0, e1); x[] then holds v
    // (backtracking: y and grad f(y) are stored for a redo and, where x^k is
    // held in registers, left in xq[] / g2[] for the model-test terms)
    auto grad = [&](int e, double xke, double &xqe, double &g2e) {
      const double h = x[e];
      const double yj = xke + m * (xke - xqe);
      double gj;
      if (loss == kLsq) gj = -2.0 * ((1.0 + m) * h - m * g2e);
      else gj = restart ? -h : g2e;
      x[e] = sv(e) != 3 ? yj - gj * invL : 0.0;
      if (loss == kLsq && sv(e) != 3) nb.hprev[(uint32_t)(tid + e * NT)] = h;
      if (bt && sv(e) != 3) {
        const uint32_t j = (uint32_t)(tid + e * NT);
        nb.ybt[j] = yj;
        nb.gbt[j] = gj;
      }
      if (bt) {
        xqe = yj;
        g2e = gj;
        if constexpr (!kHoldXk) wl[(uint32_t)(tid + e * NT)] = yj;  // the selection's LDS array is free by now
      }
    };
    if constexpr (kHoldXk) {
      if (lds.bci[2]) {
#pragma unroll
        for (int e = 0; e < EPT; e++)
          if (sv(e) != 3) nb.xbest[(uint32_t)(tid + e * NT)] = xk[e];
      }
      if (gb && lds.bci[3]) {
#pragma unroll
        for (int e = 0; e < EPT; e++)
          if (sv(e) != 3) nb.xlb[(uint32_t)(tid + e * NT)] = xk[e];
      }
      if (done) return;
      if (!kPre) {
#pragma unroll
        for (int e = 0; e < EPT; e++) {
          const uint32_t j = (uint32_t)(tid + e * NT);
          const bool in = j < (uint32_t)p;
          xq[e] = in ? xn[j] : 0.0;
          g2[e] = in ? gp[j] : 0.0;
        }
      }
#pragma unroll
      for (int e = 0; e < EPT; e++) grad(e, xk[e], xq[e], g2[e]);
    } else {
      constexpr int HE = EPT / 2;
#pragma unroll
      for (int hh = 0; hh < 2; hh++) {
        double xkh[HE], xqh[HE], g2h[HE];
#pragma unroll
        for (int i = 0; i < HE; i++) {
          const uint32_t j = (uint32_t)(tid + (hh * HE + i) * NT);
          const bool in = j < (uint32_t)p;
          xkh[i] = in ? xc[j] : 0.0;
          xqh[i] = (in && !done) ? xn[j] : 0.0;
          g2h[i] = (in && !done) ? gp[j] : 0.0;
        }
        if (lds.bci[2]) {
#pragma unroll
          for (int i = 0; i < HE; i++)
            if (sv(hh * HE + i) != 3) nb.xbest[(uint32_t)(tid + (hh * HE + i) * NT)] = xkh[i];
        }
        if (gb && lds.bci[3]) {
#pragma unroll
          for (int i = 0; i < HE; i++)
            if (sv(hh * HE + i) != 3) nb.xlb[(uint32_t)(tid + (hh * HE + i) * NT)] = xkh[i];
        }
        if (!done) {
#pragma unroll
          for (int i = 0; i < HE; i++) grad(hh * HE + i, xkh[i], xqh[i], g2h[i]);
        }
      }
      if (done) return;
    }
    Lstep = Lnew;
  }
  prox_finish(Lstep, rejected);
}


// ------------------------------------------------------------ batched node kernels
//
// One workgroup per node (grid = m).  The products come from the FP64 MFMA
// GEMMs of the batch, summed over the reduction splits: least squares
// h = X^T r (r = y - X x, zeta = 2 r); logistic h = X^T zeta (zeta =
// -grad F(X x)) and X^T grad F at the momentum point, the two right-hand
// sides of one GEMM.  Phi(x), Psi(zeta), the gap, restart and termination
// then follow the single-node step exactly.  The host recomputes Phi and Psi
// of every stopped node over the stored X (k_cert_batch).

template <int EPT>
__global__ __launch_bounds__(NT) void k_batch_init(const NodeParams *__restrict__ prmA, NodeState *SA, BatchBufs bb,
                                                   const double *__restrict__ B0, double L) {
  __shared__ NodeLds lds;
  const int node = blockIdx.x;
  const NodeParams *prm = prmA + node;
  NodeState *S = SA + node;
  const int tid = threadIdx.x;
  const int64_t p = prm->p;
  const int64_t off = (int64_t)node * p;
  PackedStatus<EPT> sv;
  sv.load(prm->st, p);
  double x[EPT];
#pragma unroll
  for (int e = 0; e < EPT; e++) {
    const int64_t j = tid + (int64_t)e * NT;
    x[e] = 0.0;
    if (j < p) {
      const double b = B0 ? B0[off + j] : 0.0;
      x[e] = b;
      bb.x0[off + j] = b;
      bb.xbest[off + j] = b;
      bb.x1[off + j] = 0.0;
      bb.hprev[off + j] = 0.0;
      bb.Bx[off + j] = b;
    }
  }
  IterStats is = finish_r<EPT>(x, sv, prm->kbar, prm->M, bb.sidx + off, bb.sval + off, lds);
  if (tid == 0) {
    NodeState s{};
    s.L = L;
    s.t = 1.0;
    s.gap_ref = INFINITY;
    s.lb = -INFINITY;
    s.ub = INFINITY;
    s.phi = INFINITY;
    s.psi = -INFINITY;
    s.rel_gap = INFINITY;
    s.gval = is.gval;
    s.tau = -1.0;
    s.tk = -1.0;
    s.tkw = 0.25;
    s.status = kMaxIter;
    s.nsupp = is.nsupp;
    s.indom = is.indom;
    s.bt = is_bt(prm->method) ? 1 : 0;
    *S = s;
  }
}

// GRAM: the batch runs in Gram mode (bb.gb set); a compile-time variant, so
// that the other batches carry none of its loads in registers.
template <int EPT, bool GRAM>
__global__ __launch_bounds__(NT) void k_batch_step(const NodeParams *__restrict__ prmA, NodeState *SA, BatchBufs bb) {
  __shared__ StepLds<EPT> lds;
  // with 32 entries per thread (the single-node step's form): x^k is read
  // again where it is used and the gradient step runs in two halves, and the
  // radix selection reads the dual magnitudes from LDS, so that the step stays
  // out of scratch memory
  constexpr bool kHoldXk = EPT <= 16;
  constexpr int EK = kHoldXk ? EPT : 1;
  constexpr bool kSelLds = EPT > 16;
  __shared__ double wl[kSelLds ? EPT * NT : 1];
  const int node = blockIdx.x;
  const NodeParams *prm = prmA + node;
  NodeState *S = SA + node;
  const int tid = threadIdx.x;
  const int64_t p = bb.p;
  const int64_t off = (int64_t)node * p;
  const double *__restrict__ gb = GRAM ? bb.gb : nullptr;
  // scalar state: independent loads, issued with the vector loads below
  const int done0 = S->done, parity = S->parity, indom0 = S->indom, it0 = S->iter;
  const double L = S->L, gval0 = S->gval, tau0 = S->tau, tkp = S->tk, dlt = S->tkw, dxy0 = S->dxy;
  const int kbar = prm->kbar;
  const double lam2 = prm->lambda2, M = prm->M;
  const bool bt = is_bt(prm->method);
  // x^k; backtracking writes a redone trial over a rejected one (xcw, same
  // buffer, so xc carries no restrict qualifier) and keeps the parity
  const double *xc = (parity ? bb.x1 : bb.x0) + off;
  double *xcw = (parity ? bb.x1 : bb.x0) + off;
  double *__restrict__ xn = (parity ? bb.x0 : bb.x1) + off;
  PackedStatus<EPT> sv;
  load_packed_status<EPT>(sv, bb.stp + (int64_t)node * bb.stpw);
  // h = X^T r from the GEMM split partials (Gram mode: G x, turned into
  // h = b - G x below); x^k
  const int64_t stride = (int64_t)bb.NrT * p;
  const int KS = *bb.ksp;
  const bool lsq = bb.loss == kLsq;
  const double *__restrict__ Hn = bb.CT + (int64_t)bb.rs * off;
  double h[EPT], xk[EK];
#pragma unroll
  for (int e = 0; e < EPT; e++) {
    const uint32_t j = (uint32_t)(tid + e * NT);
    const bool in = j < (uint32_t)p;
    h[e] = in ? Hn[j] : 0.0;
    if constexpr (kHoldXk) xk[e] = in ? xc[j] : 0.0;
  }
  auto xkv = [&](int e) -> double {
    if constexpr (kHoldXk) {
      return xk[e];
    } else {
      const uint32_t j = (uint32_t)(tid + e * NT);
      return j < (uint32_t)p ? xc[j] : 0.0;
    }
  };
  for (int z = 1; z < KS; z++) {
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const uint32_t j = (uint32_t)(tid + e * NT);
      if (j < (uint32_t)p) h[e] += Hn[z * stride + j];
    }
  }
  // loss sums of the residual blocks: lane-parallel loads, fixed-order wave sums
  double Fk = 0.0, negconj = 0.0;
  if (!gb) {
    for (int i = lane_id(); i < bb.nfb; i += 64) {
      Fk += bb.fsum[2 * ((int64_t)node * bb.nfb + i)];
      negconj += bb.fsum[2 * ((int64_t)node * bb.nfb + i) + 1];
    }
  }
  if (done0) return;
  Red2 R;
  R.buf = lds.red;
  R.ph = 0;
  if (tid == 0) lds.sel.ngat = 0;
  if (!gb) {
    Fk = wave_sum(Fk);
    negconj = wave_sum(negconj);
  }
  // The proximal step from v (in h[]) with step constant Ls, shared by the
  // accepted and the rejected branch (the single-node step's form): the new
  // point goes to the next buffer (accepted) or over the rejected trial, and to
  // the node's row of the forward GEMM's operand; backtracking keeps
  // ||x - y||^2 for the test of the new trial.
  double *__restrict__ ybt = bb.ybt + off;
  auto prox_finish = [&](double Ls, bool rejected) {
    const double rho = 2.0 * lam2 / Ls;
    int evals = 0;
    auto vabs = [&](int e) { return sv(e) == kFree ? fabs(h[e]) : -1.0; };
    const double tau = solve_tau_2<EPT>(vabs, kbar, rho, M, tau0, R, &evals);
    const double inv1p = 1.0 / (1.0 + rho);
    double *dst = rejected ? xcw : xn;
    double dxy[1] = {0.0};
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const int s = sv(e);
      double xv = 0.0;
      if (s != 3) {
        if (s != kZero) {
          const double av = fabs(h[e]);
          double r = fmin(av * inv1p, M);
          if (s == kFree) r = fmin(r, fmax(av - tau, 0.0));
          xv = (r == 0.0) ? 0.0 : copysign(r, h[e]);
        }
        const uint32_t j = (uint32_t)(tid + e * NT);
        dst[j] = xv;
        bb.Bx[off + j] = xv;
        if (bt) {
          const double dy = xv - ybt[j];
          dxy[0] += dy * dy;
        }
      }
      h[e] = xv;
    }
    if (bt) R.sum(dxy);
    IterStats is = finish_2<EPT>(h, sv, kbar, M, bb.sidx + off, bb.sval + off, lds, R);
    if (tid == 0) {
      S->gval = is.gval;
      S->indom = is.indom;
      S->nsupp = is.nsupp;
      S->tau = tau;
      S->tau_iters = evals;
      if (!rejected) {
        S->parity = parity ^ 1;
        S->iter = S->iter + 1;
      }
      if (bt) {
        S->L = Ls;
        S->dxy = dxy[0];
        S->bt_acc = rejected ? 0 : 1;
        if (rejected) S->trials = S->trials + 1;
      }
    }
  };
  // Backtracking: every point after the start is a trial of the step from the
  // momentum point y, accepted when f(x) - f(y) - <grad f(y), x - y> <=
  // (L / 2) ||x - y||^2 (or L has reached Lmax); else the step is redone from
  // the saved y and grad f(y) with c L and the trial is not evaluated.
  if (bt && it0 > 0) {
    const double *__restrict__ gbt = bb.gbt + off;
    double dv = 0.0;
    if (lsq) {
      // ||X (x - y)||^2 = (x - y)^T (h(y) - h(x)), h(y) = -grad f(y) / 2
      // (Gram mode: h = b - G x from the planes of G x)
      double d1[1] = {0.0};
#pragma unroll
      for (int e = 0; e < EPT; e++) {
        if (sv(e) == 3) continue;
        const uint32_t j = (uint32_t)(tid + e * NT);
        const double hx = gb ? gb[j] - h[e] : h[e];
        d1[0] += (xkv(e) - ybt[j]) * (-0.5 * gbt[j] - hx);
      }
      R.sum(d1);
      dv = d1[0];
    } else {
      // logistic: the residual kernel summed the remainder row by row per block
      for (int i = lane_id(); i < bb.nfb; i += 64) dv += bb.dsum[(int64_t)node * bb.nfb + i];
      dv = wave_sum(dv);
    }
    if (!(L >= prm->Lmax || dv <= 0.5 * L * dxy0)) {
      const double Ls = fmin(prm->ls_c * L, prm->Lmax);
      const double invLs = 1.0 / Ls;
#pragma unroll
      for (int e = 0; e < EPT; e++) {
        const uint32_t j = (uint32_t)(tid + e * NT);
        h[e] = sv(e) != 3 ? ybt[j] - gbt[j] * invLs : 0.0;
      }
      prox_finish(Ls, true);
      return;
    }
  }
  // dual at x^k: w = X^T zeta / (2 lambda2) (least squares h / lambda2, logistic
  // h / (2 lambda2)); the top-kbar window of free |w| around the previous
  // kbar-th value (as in the single-node step)
  const double wscale = (lsq ? 1.0 : 0.5) / lam2;
  const bool wv = tkp > 0.0 && kbar > 0;
  const double wa = wv ? tkp * (1.0 - dlt) : INFINITY, wb = wv ? tkp * (1.0 + dlt) : INFINITY;
  // r1: sum_{J1} H_M(w_j); Gram: x^T (b + h), b^T x; #{w > wb}, #{w >= wa}, sum_{w > wb} H_M(w)
  double r1[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < EPT; e++) {
    const int s = sv(e);
    if (s == 3) continue;
    if (gb) {
      const double bj = gb[tid + (int64_t)e * NT];
      h[e] = bj - h[e];
      const double xe = xkv(e);
      r1[1] += xe * (bj + h[e]);
      r1[2] += bj * xe;
    }
    const double w = h[e] * wscale;
    if (s == kOne) r1[0] += huber(w, M);
    if (s == kFree) {
      const double aw = fabs(w);
      if (aw > wb) {
        r1[3] += 1.0;
        r1[5] += huber(aw, M);
      }
      if (aw >= wa) r1[4] += 1.0;
    }
  }
  R.sum(r1);
  if (gb) {
    // F(X x) = y^T y - x^T (b + h), -F*(-zeta) = 2 (y^T y - b^T x) - F
    Fk = bb.gyy - r1[1];
    negconj = 2.0 * (bb.gyy - r1[2]) - Fk;
  }
  auto wabs = [&](int e) { return sv(e) == kFree ? fabs(h[e] * wscale) : -1.0; };
  const double cgt = r1[3], cge = r1[4];
  const bool fast = wv && cgt < (double)kbar && (double)kbar <= cge && cge - cgt <= (double)kWinCap;
  double topsum = 0.0, tkn = -1.0;
  if (kbar > 0 && fast) {
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const double aw = wabs(e);
      if (aw >= wa && aw <= wb) lds.sel.gat[atomicAdd(&lds.sel.ngat, 1)] = aw;
    }
    lds_barrier();
    if (wave_id() == 0) {
      const int lane = lane_id();
      const int cw = (int)(cge - cgt);
      const int mm = kbar - (int)cgt;  // 1 <= mm <= cw
      double v = (lane < cw) ? lds.sel.gat[lane] : -1.0;
      v = wave_sort_desc(v);
      tkn = __shfl(v, mm - 1, 64);
      topsum = r1[5] + wave_sum(lane < mm ? huber(v, M) : 0.0);
    }
  } else if (kbar > 0) {
    if constexpr (kSelLds) {
#pragma unroll
      for (int e = 0; e < EPT; e++) wl[tid + e * NT] = wabs(e);
      __syncthreads();
      tkn = select_kth(wl, (int64_t)EPT * NT, kbar, lds.sel);
    } else {
      tkn = select_kth_f<EPT>(wabs, kbar, lds.sel);
    }
    const double Ht = huber(tkn, M);
    double v1[1] = {0.0};
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const double aw = wabs(e);
      if (aw >= 0.0) v1[0] += fmax(huber(aw, M) - Ht, 0.0);
    }
    R.sum(v1);
    topsum = (double)kbar * Ht + v1[0];
  }
  if (tid == 0) {
    // Psi(zeta) and Phi(x) from the FP64 products of this pass
    const double psi = negconj - 2.0 * lam2 * (r1[0] + topsum);
    const double phi = indom0 ? Fk + 2.0 * lam2 * gval0 : INFINITY;
    const double gap = phi - psi;
    const int it = S->iter;
    if (prm->trace && it <= prm->max_iter) {
      prm->trace[2 * it] = phi;
      prm->trace[2 * it + 1] = psi;
    }
    double lb = S->lb, ub = S->ub;
    if (psi > lb) lb = psi;
    if (phi < ub) ub = phi;
    // the stopping test uses the current pair (x, zeta(x)): it is the pair the
    // host re-certifies, so no per-node snapshot of zeta is kept
    const double rel = gap / fmax(fabs(phi), 1e-300);
    int done = 0, status = kMaxIter;
    if (rel <= bb.gap_factor * prm->tol) {
      done = 1;
      status = kConverged;
    } else if (!isnan(prm->cutoff) && psi >= prm->cutoff) {
      done = 1;
      status = kCutoffPrune;
    } else if (!isnan(prm->cutoff) && phi <= prm->cutoff) {
      done = 1;
      status = kCutoffBranch;
    } else if (it >= prm->max_iter) {
      done = 1;
      status = kMaxIter;
    }
    double m = 0.0, t = S->t, gap_ref = S->gap_ref;
    int restart = 0, restarts = S->restarts;
    if (!done) {
      restart = decide_restart(prm, it, gap, phi, S->phi, gap_ref, restarts);
      if (restart) {
        m = 0.0;
        t = 1.0;
      } else {
        const double tn = fista_next_t(t);
        m = (t - 1.0) / tn;
        t = tn;
      }
    }
    double tw = 0.25;
    if (wv && tkn > 0.0) tw = fmin(0.25, fmax(1e-12, 2.0 * fabs(tkn - tkp) / tkn));
    if (wv && !fast && cgt < (double)kbar && (double)kbar <= cge) tw = fmin(tw, 0.25 * dlt);
    S->phi = phi;
    S->psi = psi;
    S->lb = lb;
    S->ub = ub;
    S->rel_gap = rel;
    S->status = status;
    S->t = t;
    S->gap_ref = gap_ref;
    S->restarts = restarts;
    S->mom = m;
    S->tk = tkn;
    S->tkw = tw;
    if (done) {
      S->done = 1;
      atomicSub(bb.active, 1);
    }
    lds.bcd[0] = m;
    lds.bci[0] = done;
    lds.bci[1] = restart;
  }
  lds_barrier();
  const bool done = lds.bci[0] != 0;
  if (done) {
    // the certified point is the iterate whose gap passed the test
#pragma unroll
    for (int e = 0; e < EPT; e++)
      if (sv(e) != 3) bb.xbest[off + tid + (int64_t)e * NT] = xkv(e);
    return;
  }
  // gradient at the momentum point y = x^k + m (x^k - x^{k-1}):
  //   least squares -2 ((1 + m) h_k - m h_{k-1}) by linearity (hq = h_{k-1});
  //   logistic the second plane row of the node (hq), or -h at a restart (y = x^k)
  double *__restrict__ hp = bb.hprev + off;
  const double *__restrict__ H2 = Hn + p;
  const double m = lds.bcd[0];
  const bool restart = lds.bci[1] != 0;
  // backtracking: a restart runs the method afresh, the line search from L0
  const double Lnew = (bt && restart) ? prm->L0 : L;
  const double invL = 1.0 / Lnew;
  // entries [E0, E0 + HE): x^{k-1} and the previous gradient term loaded, then
  // the step; h[] then holds v (least squares: h_k stored as the next h_{k-1})
  constexpr int HE = kHoldXk ? EPT : EPT / 2;
  auto grad_part = [&](auto e0c) {
    constexpr int E0 = decltype(e0c)::value;
    double xkh[HE], xq[HE], hq[HE];
#pragma unroll
    for (int i = 0; i < HE; i++) {
      const uint32_t j = (uint32_t)(tid + (E0 + i) * NT);
      const bool in = j < (uint32_t)p;
      xkh[i] = xkv(E0 + i);
      xq[i] = in ? xn[j] : 0.0;
      hq[i] = in ? (lsq ? hp[j] : H2[j]) : 0.0;
    }
    if (!lsq) {
      for (int z = 1; z < KS; z++) {
#pragma unroll
        for (int i = 0; i < HE; i++) {
          const uint32_t j = (uint32_t)(tid + (E0 + i) * NT);
          if (j < (uint32_t)p) hq[i] += H2[z * stride + j];
        }
      }
    }
#pragma unroll
    for (int i = 0; i < HE; i++) {
      const int e = E0 + i;
      const uint32_t j = (uint32_t)(tid + e * NT);
      const double yj = xkh[i] + m * (xkh[i] - xq[i]);
      const double gj = lsq ? -2.0 * ((1.0 + m) * h[e] - m * hq[i]) : (restart ? -h[e] : hq[i]);
      if (lsq && sv(e) != 3) hp[j] = h[e];
      h[e] = sv(e) != 3 ? yj - gj * invL : 0.0;
      if (bt && sv(e) != 3) {
        ybt[j] = yj;
        bb.gbt[off + j] = gj;
      }
    }
  };
  grad_part(std::integral_constant<int, 0>{});
  if constexpr (!kHoldXk) grad_part(std::integral_constant<int, HE>{});
  prox_finish(Lnew, false);
}

}  // namespace

int node_ept(int64_t p) {
  for (int e = 1; e <= 32; e *= 2)
    if (p <= (int64_t)e * NT) return e;
  return 0;
}

hipError_t launch_node_init(const NodeParams *prm, NodeState *S, NodeBufs nb, const double *beta0,
                            double L, int64_t p, hipStream_t s) {
  switch (node_ept(p)) {
    case 1: k_node_init_r<1><<<1, NT, 0, s>>>(prm, S, nb, beta0, L); break;
    case 2: k_node_init_r<2><<<1, NT, 0, s>>>(prm, S, nb, beta0, L); break;
    case 4: k_node_init_r<4><<<1, NT, 0, s>>>(prm, S, nb, beta0, L); break;
    case 8: k_node_init_r<8><<<1, NT, 0, s>>>(prm, S, nb, beta0, L); break;
    case 16: k_node_init_r<16><<<1, NT, 0, s>>>(prm, S, nb, beta0, L); break;
    case 32: k_node_init_r<32><<<1, NT, 0, s>>>(prm, S, nb, beta0, L); break;
    default: k_node_init<<<1, NT, 0, s>>>(prm, S, nb, beta0, L); break;
  }
  return hipGetLastError();
}

hipError_t launch_node_step(const NodeParams *prm, NodeState *S, NodeBufs nb, const ProbBufs &B,
                            int64_t p, hipStream_t s, const StepArgs *a) {
  const int ept = node_ept(p);
  if (ept != 0 && !a) return hipErrorInvalidValue;
  switch (ept) {
#define PR_STEP_CASE(E)                                                          \
  case E:                                                                        \
    if (a->bt) k_node_step_r<E, true><<<1, NT, 0, s>>>(prm, S, nb, B, *a);       \
    else k_node_step_r<E, false><<<1, NT, 0, s>>>(prm, S, nb, B, *a);            \
    break;
    PR_STEP_CASE(1)
    PR_STEP_CASE(2)
    PR_STEP_CASE(4)
    PR_STEP_CASE(8)
    PR_STEP_CASE(16)
    PR_STEP_CASE(32)
#undef PR_STEP_CASE
    default: k_node_step<<<1, NT, 0, s>>>(prm, S, nb, B); break;
  }
  return hipGetLastError();
}

hipError_t launch_batch_init(const NodeParams *prm, NodeState *S, BatchBufs bb, const double *B0, double L,
                             int64_t p, hipStream_t s) {
  const unsigned g = (unsigned)bb.m;
  switch (node_ept(p)) {
    case 1: k_batch_init<1><<<g, NT, 0, s>>>(prm, S, bb, B0, L); break;
    case 2: k_batch_init<2><<<g, NT, 0, s>>>(prm, S, bb, B0, L); break;
    case 4: k_batch_init<4><<<g, NT, 0, s>>>(prm, S, bb, B0, L); break;
    case 8: k_batch_init<8><<<g, NT, 0, s>>>(prm, S, bb, B0, L); break;
    case 16: k_batch_init<16><<<g, NT, 0, s>>>(prm, S, bb, B0, L); break;
    case 32: k_batch_init<32><<<g, NT, 0, s>>>(prm, S, bb, B0, L); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_step(const NodeParams *prm, NodeState *S, BatchBufs bb, int64_t p, hipStream_t s) {
  const unsigned g = (unsigned)bb.m;
#define PR_BSTEP_CASE(E)                                                   \
  case E:                                                                  \
    if (bb.gb) k_batch_step<E, true><<<g, NT, 0, s>>>(prm, S, bb);         \
    else k_batch_step<E, false><<<g, NT, 0, s>>>(prm, S, bb);              \
    break;
  switch (node_ept(p)) {
    PR_BSTEP_CASE(1)
    PR_BSTEP_CASE(2)
    PR_BSTEP_CASE(4)
    PR_BSTEP_CASE(8)
    PR_BSTEP_CASE(16)
    PR_BSTEP_CASE(32)
    default: return hipErrorInvalidValue;
  }
#undef PR_BSTEP_CASE
  return hipGetLastError();
}

hipError_t launch_zbest_final(const NodeState *S, const ProbBufs &B, int32_t loss, int64_t n,
                              hipStream_t s) {
  k_zbest_final<<<256, 256, 0, s>>>(S, B.r, B.zbest, loss == kLsq ? 2.0 : 1.0, n);
  return hipGetLastError();
}

hipError_t launch_prox(const double *v, double *out, int64_t p, double rho, int32_t kbar, double M,
                       const int8_t *st, double *abuf, double *, hipStream_t s) {
  k_prox<<<1, NT, 0, s>>>(v, out, p, rho, kbar, M, st, abuf);
  return hipGetLastError();
}

hipError_t launch_prox_batch(const NodeParams *prm, const double *V, double *Xo, double *abuf, int64_t p, int m,
                             double invL, hipStream_t s) {
  k_prox_batch<<<(unsigned)m, NT, 0, s>>>(prm, V, Xo, abuf, p, invL);
  return hipGetLastError();
}

hipError_t launch_prox_counted(const double *v, double *out, int64_t p, double rho, int32_t k, double M,
                               const int8_t *st, double *abuf, int32_t *flag, hipStream_t s) {
  k_prox_counted<<<1, NT, 0, s>>>(v, out, p, rho, k, M, st, abuf, flag);
  return hipGetLastError();
}

hipError_t launch_regularizer(const double *beta, const double *alpha, int64_t p, int32_t kbar,
                              double M, const int8_t *st, double *abuf, double *out2,
                              hipStream_t s) {
  // the support list written by finish_iterate is scratch here: reuse abuf's
  // tail is not possible, so the caller's workspace provides 2p extra entries
  int32_t *sidx = reinterpret_cast<int32_t *>(abuf + p);
  double *sval = abuf + 2 * p;
  k_regularizer<<<1, NT, 0, s>>>(beta, alpha, p, kbar, M, st, abuf, sidx, sval, out2);
  return hipGetLastError();
}

hipError_t launch_loss_terms(int32_t loss, const double *u, const double *y, int64_t n,
                             double *zeta_out, double *sums_out, hipStream_t s) {
  k_loss_terms<<<1, NT, 0, s>>>(loss, u, y, n, zeta_out, sums_out);
  return hipGetLastError();
}

hipError_t launch_zeta_terms(int32_t loss, const double *zeta, const double *y, int64_t n,
                             double *sums_out, hipStream_t s) {
  k_zeta_terms<<<1, NT, 0, s>>>(loss, zeta, y, n, sums_out);
  return hipGetLastError();
}

hipError_t launch_sumsq(const double *v, int64_t n, double *out, hipStream_t s) {
  k_sumsq<<<1, NT, 0, s>>>(v, n, out);
  return hipGetLastError();
}

hipError_t launch_scale_copy(const double *src, double *dst, double a, int64_t n, hipStream_t s) {
  k_scale_copy<<<256, 256, 0, s>>>(src, dst, a, n);
  return hipGetLastError();
}

hipError_t launch_cert_batch(const NodeParams *prm, const double *Xit, const double *H, int KS, int Nr, int rs,
                             const double *fsum, int nfb, int64_t p, double *abuf, int32_t *sidx, double *sval,
                             double *out, int m, hipStream_t s) {
  k_cert_batch<<<(unsigned)m, NT, 0, s>>>(prm, Xit, H, KS, Nr, rs, fsum, nfb, p, abuf, sidx, sval, out);
  return hipGetLastError();
}

hipError_t launch_lanczos(double *w, double *v, double *vprev, const double *alpha, const double *beta_prev,
                          double *beta_out, int64_t p, hipStream_t s) {
  k_lanczos<<<1, NT, 0, s>>>(w, v, vprev, alpha, beta_prev, beta_out, p);
  return hipGetLastError();
}

hipError_t launch_iota(int32_t *idx, int64_t n, hipStream_t s) {
  k_iota<<<256, 256, 0, s>>>(idx, n);
  return hipGetLastError();
}

}  // namespace pr
