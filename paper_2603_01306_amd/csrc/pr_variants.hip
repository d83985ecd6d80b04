// Iteration variants beyond the FISTA path of pr_node.hip, on gfx950: one
// 512-thread workgroup per step, vectors in global memory (strided passes),
// around the same column-list product (pr_spfwd.hip) and X^T pass
// (pr_gemv.hip).
//
//   AC-FGM on the perspective relaxation (Section 3.3's rate table, Section
//   5.2's convergence study; Li and Lan's accelerated composite method):
//     k_ac_init   start point x_0: support list, Algorithm 1 value, dom test
//     k_ac_resid  X x_t = (X z_t + tau_t X x_{t-1}) / (1 + tau_t) by
//                 linearity from the product over z_t's support, then the loss
//                 epilogue (least squares r = y - X x, logistic zeta) and the
//                 per-block loss sums
//     k_ac_step   (Phi, Psi) at x_t, bounds, stopping test, the local
//                 curvature estimate Lhat_t, the first-step line search, the
//                 duality-gap restart, the step sizes, and the next point:
//                 z = prox_{eta G}(y - eta grad f(x)), y <- (1 - b) y + b z,
//                 x <- (z + tau x) / (1 + tau)
//   LASSO with the duality-gap restart (Section 5.2, the restart applied
//   beyond perspective relaxations), least squares, FISTA:
//     k_lasso_init, k_lasso_step  (Phi, Psi) with G = lam ||.||_1 (dual point
//                 zeta scaled into dom G*) or G = indicator of the l1-ball of
//                 radius lam (G* = lam ||.||_inf), restart, momentum, and the
//                 prox: soft thresholding or the l1-ball projection (threshold
//                 by the finite active-set fixed point of Michelot).
#include "pr_regularizer.h"

namespace pr {
namespace {
using namespace dev;

constexpr int kRows = 2;          // rows per thread of k_ac_resid (the spfwd finalize layout)
constexpr int kResidThreads = 128;  // the spfwd finalize's block (B.nfin blocks cover n)

__device__ __forceinline__ int compact_list(const double *__restrict__ x, int64_t p, int32_t *__restrict__ sidx,
                                            double *__restrict__ sval, int *scan) {
  int cnt = 0;
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) cnt += (x[j] != 0.0);
  int tot;
  int off = block_excl_scan<NT>(cnt, scan, &tot);
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
    const double v = x[j];
    if (v != 0.0) {
      sidx[off] = (int32_t)j;
      sval[off] = v;
      off++;
    }
  }
  return tot;
}

// ------------------------------------------------------------------ AC-FGM

__global__ __launch_bounds__(NT) void k_ac_init(const NodeParams *__restrict__ prm, NodeState *S, AcState *A,
                                                AcBufs ab, NodeBufs nb, const double *__restrict__ beta0,
                                                double L0) {
  __shared__ double red[NW * 4];
  __shared__ int scan[NW];
  const int64_t p = prm->p;
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
    const double b = beta0 ? beta0[j] : 0.0;
    ab.xc[j] = b;
    ab.yc[j] = b;
    ab.z[j] = b;
    ab.xb[j] = b;
    ab.gb[j] = 0.0;
    ab.yb[j] = b;
    nb.xbest[j] = b;
  }
  __syncthreads();
  // the forward product of the first unit runs over the list of z = x_0
  IterStats is = finish_iterate(ab.xc, prm->st, p, prm->kbar, prm->M, nb.abuf, nb.sidx, nb.sval, red, scan);
  if (threadIdx.x == 0) {
    NodeState s{};
    s.L = L0;
    s.t = 1.0;
    s.gap_ref = INFINITY;
    s.lb = -INFINITY;
    s.ub = INFINITY;
    s.phi = INFINITY;
    s.psi = -INFINITY;
    s.rel_gap = INFINITY;
    s.gval = is.gval;
    s.tau = -1.0;
    s.status = kMaxIter;
    s.nsupp = is.nsupp;
    s.indom = is.indom;
    *S = s;
    AcState a{};
    a.L1 = L0;
    a.gap_ref = INFINITY;
    a.tau_cur = 0.0;
    a.eta_cur = 0.0;
    a.step = 0;
    *A = a;
  }
}

__global__ __launch_bounds__(kResidThreads) void k_ac_resid(int64_t n, const double *__restrict__ y, int32_t loss,
                                                            ProbBufs B, const double *__restrict__ uz,
                                                            double *__restrict__ ucur, const NodeState *S,
                                                            const AcState *A) {
  __shared__ double red[(kResidThreads / 64) * 4];
  if (S->done) return;
  const double tau = A->tau_cur;
  const double inv = 1.0 / (1.0 + tau);
  const int improved = S->improved;
  const int fb = blockIdx.x;
  const int64_t row0 = ((int64_t)fb * kResidThreads + threadIdx.x) * kRows;
  double sums[2] = {0.0, 0.0};
#pragma unroll
  for (int e = 0; e < kRows; e++) {
    const int64_t i = row0 + e;
    if (i >= n) break;
    const double u = (tau > 0.0) ? (uz[i] + tau * ucur[i]) * inv : uz[i];
    ucur[i] = u;
    const double yi = y[i];
    if (loss == kLsq) {
      if (improved) B.zbest[i] = 2.0 * B.r[i];
      const double ri = yi - u;
      B.r[i] = ri;
      sums[0] += ri * ri;
      sums[1] += 2.0 * ri * yi - ri * ri;
    } else {
      if (improved) B.zbest[i] = B.r[i];
      const double z = yi * u;
      const double a = 1.0 / (1.0 + exp(z));
      B.r[i] = yi * a;
      sums[0] += softplus(-z);
      sums[1] += a * softplus(z) + (1.0 - a) * softplus(-z);
    }
  }
  block_sum<kResidThreads, 2>(sums, red);
  if (threadIdx.x == 0) {
    B.rbsum[2 * fb] = sums[0];
    B.rbsum[2 * fb + 1] = sums[1];
  }
}

// Step size and tau for epoch step t (t >= 1) from the accepted history.
__device__ __forceinline__ void ac_step_size(const AcState &a, int t, double b, double &eta, double &tau) {
  if (t == 1) {
    eta = 1.0 / a.L1;
    tau = 0.0;
    return;
  }
  tau = 0.5 * (double)t;
  const double lp = a.lhat_prev;
  if (t == 2) {
    eta = fmin((1.0 - b) * a.eta_prev, lp > 0.0 ? 1.0 / (4.0 * lp) : INFINITY);
  } else {
    eta = fmin((a.tau_prev + 1.0) / tau * a.eta_prev, lp > 0.0 ? a.tau_prev / (4.0 * lp) : INFINITY);
  }
}

__global__ __launch_bounds__(NT) void k_ac_step(const NodeParams *__restrict__ prm, NodeState *S, AcState *A,
                                                AcBufs ab, NodeBufs nb, ProbBufs B, double b, double c,
                                                int32_t restart_gap) {
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
  const int step = A->step;

  double Fk = 0.0, negconj = 0.0;
  for (int i = 0; i < B.nfin; i++) {
    Fk += B.rbsum[2 * i];
    negconj += B.rbsum[2 * i + 1];
  }
  // dual w = X^T zeta / (2 lambda2); gradient of f at x_t is gscale * h1
  const double wscale = (loss == kLsq) ? 1.0 / lam2 : 0.5 / lam2;
  const double gscale = (loss == kLsq) ? -2.0 : -1.0;
  double acc[3] = {0.0, 0.0, 0.0};  // sum_{J1} H_M(w), ||g_t - g_b||^2, ||x_t - x_b||^2
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
    const double h = B.h1[j];
    const double w = h * wscale;
    const int s = st[j];
    if (s == kOne) acc[0] += huber(w, M);
    nb.abuf[j] = (s == kFree) ? fabs(w) : -1.0;
    const double dg = gscale * h - ab.gb[j], dx = ab.xc[j] - ab.xb[j];
    acc[1] += dg * dg;
    acc[2] += dx * dx;
  }
  block_sum<NT, 3>(acc, red);
  __syncthreads();
  const double topsum = topsum_huber(nb.abuf, p, kbar, M, sel, red);
  const double psi = negconj - 2.0 * lam2 * (acc[0] + topsum);
  const double phi = S->indom ? Fk + 2.0 * lam2 * S->gval : INFINITY;

  if (tid == 0) {
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
    }
    AcState a = *A;
    int accept = 0, restart = 0, next = 1;
    double eta = 0.0, tau = 0.0;
    if (!done) {
      const double lhat = acc[2] > 0.0 ? sqrt(acc[1]) / sqrt(acc[2]) : 0.0;
      if (step == 0) {  // the start point becomes the first epoch's base
        accept = 1;
        a.gap_ref = gap;
        next = 1;
      } else if (step == 1 && lhat > a.L1) {  // line search of the first step
        a.L1 *= c;
        a.rejected++;
        next = 1;
      } else {
        accept = 1;
        a.eta_prev = a.eta_cur;
        a.tau_prev = a.tau_cur;
        a.lhat_prev = lhat;
        next = step + 1;
        if (restart_gap && gap <= a.gap_ref / prm->eta) {
          a.gap_ref = gap;
          restart = 1;
          next = 1;
          S->restarts = S->restarts + 1;
        }
      }
      ac_step_size(a, next, b, eta, tau);
      a.eta_cur = eta;
      a.tau_cur = tau;
      a.step = next;
    }
    *A = a;
    S->phi = phi;
    S->psi = psi;
    S->lb = lb;
    S->ub = ub;
    S->rel_gap = rel;
    S->improved = improved;
    S->status = status;
    S->L = a.L1;
    if (done) S->done = 1;
    bcd[0] = eta;
    bcd[1] = tau;
    bci[0] = done;
    bci[1] = accept;
    bci[2] = restart;
    bci[3] = ub_improved;
  }
  __syncthreads();
  if (bci[3]) {
#pragma unroll 8
    for (int64_t j = threadIdx.x; j < p; j += NT) nb.xbest[j] = ab.xc[j];
  }
  if (bci[0]) return;
  const double eta = bcd[0], tau = bcd[1];
  const int accept = bci[1], restart = bci[2];
  // accepted point becomes the base (x_b, g_b, y_b); a restart also resets y;
  // then v = y_b - eta g_b (each thread touches only its own coordinates)
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
    double xb, gb, yb;
    if (accept) {
      xb = ab.xc[j];
      gb = gscale * B.h1[j];
      yb = restart ? xb : ab.yc[j];
      ab.xb[j] = xb;
      ab.gb[j] = gb;
      ab.yb[j] = yb;
    } else {
      xb = ab.xb[j];
      gb = ab.gb[j];
      yb = ab.yb[j];
    }
    const double v = yb - eta * gb;
    nb.vbuf[j] = v;
    nb.abuf[j] = (st[j] == kFree) ? fabs(v) : -1.0;
  }
  __syncthreads();
  const double rho = 2.0 * lam2 * eta;
  int evals = 0;
  const double thr = solve_tau(nb.abuf, p, kbar, rho, M, -1.0, red, &evals);
  const double inv1p = 1.0 / (1.0 + rho);
  const double itau = 1.0 / (1.0 + tau);
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
    const double v = nb.vbuf[j];
    const int s = st[j];
    double zj = 0.0;
    if (s != kZero) {
      const double av = fabs(v);
      double r = fmin(av * inv1p, M);
      if (s == kFree) r = fmin(r, fmax(av - thr, 0.0));
      zj = (r == 0.0) ? 0.0 : copysign(r, v);
    }
    ab.z[j] = zj;
    ab.yc[j] = (1.0 - b) * ab.yb[j] + b * zj;
    ab.xc[j] = (tau > 0.0) ? (zj + tau * ab.xb[j]) * itau : zj;
  }
  __syncthreads();
  IterStats is = finish_iterate(ab.xc, st, p, kbar, M, nb.abuf, ab.sidx2, ab.sval2, red, scan);
  const int ns = compact_list(ab.z, p, nb.sidx, nb.sval, scan);
  if (tid == 0) {
    S->gval = is.gval;
    S->indom = is.indom;
    S->nsupp = ns;
    S->iter = S->iter + 1;
  }
}

// ------------------------------------------------------------------ LASSO

__device__ __forceinline__ double lasso_G(int kind, double lam, double l1) {
  return kind == 0 ? lam * l1 : 0.0;
}

__global__ __launch_bounds__(NT) void k_lasso_init(NodeState *S, LassoState *LX, NodeBufs nb,
                                                   const double *__restrict__ beta0, int64_t p, int32_t kind,
                                                   double lam, double L) {
  __shared__ double red[NW * 4];
  __shared__ int scan[NW];
  double l1[1] = {0.0};
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
    const double b = beta0 ? beta0[j] : 0.0;
    nb.x0[j] = b;
    nb.xbest[j] = b;
    nb.x1[j] = 0.0;
    nb.hprev[j] = 0.0;
    l1[0] += fabs(b);
  }
  block_sum<NT, 1>(l1, red);
  __syncthreads();
  const int ns = compact_list(nb.x0, p, nb.sidx, nb.sval, scan);
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
    s.gval = lasso_G(kind, lam, l1[0]);
    s.status = kMaxIter;
    s.nsupp = ns;
    s.indom = (kind == 0) || (l1[0] <= lam * (1.0 + 1e-9));
    *S = s;
    LassoState lx{};
    lx.zscale = 1.0;
    lx.zscale_best = 1.0;
    *LX = lx;
  }
}

__global__ __launch_bounds__(NT) void k_lasso_step(const NodeParams *__restrict__ prm, NodeState *S, LassoState *LX,
                                                   NodeBufs nb, ProbBufs B, int32_t kind, double lam) {
  __shared__ double red[NW * 4];
  __shared__ int scan[NW];
  __shared__ double bcd[2];
  __shared__ int bci[4];
  if (S->done) return;
  const int tid = threadIdx.x;
  const int64_t p = prm->p;
  const int parity = S->parity;
  const double L = S->L;
  double F = 0.0, negconj = 0.0;  // ||r||^2 and 2 r^T y - ||r||^2 of r = y - X x^k
  for (int i = 0; i < B.nfin; i++) {
    F += B.rbsum[2 * i];
    negconj += B.rbsum[2 * i + 1];
  }
  // ||X^T zeta||_inf with zeta = 2 r, X^T r = h1
  double hm = 0.0;
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) hm = fmax(hm, fabs(B.h1[j]));
  const double wmax = 2.0 * block_max<NT>(hm, red);
  double psi, sc = 1.0;
  if (kind == 0) {
    // scale zeta into dom G* = {||w||_inf <= lam}: Psi(s zeta) = s zeta^T y - s^2 ||zeta||^2 / 4
    sc = (wmax > lam) ? lam / wmax : 1.0;
    psi = sc * (negconj + F) - sc * sc * F;
  } else {
    psi = negconj - lam * wmax;
  }
  const double phi = S->indom ? F + S->gval : INFINITY;

  if (tid == 0) {
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
      LX->zscale_best = sc;
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
    } else if (it >= prm->max_iter) {
      done = 1;
    }
    double m = 0.0, t = S->t, gap_ref = S->gap_ref;
    int restarts = S->restarts;
    if (!done) {
      if (decide_restart(prm, it, gap, phi, S->phi, gap_ref, restarts)) {
        t = 1.0;
      } else {
        const double tn = fista_next_t(t);
        m = (t - 1.0) / tn;
        t = tn;
      }
    }
    LX->zscale = sc;
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
    bci[1] = ub_improved;
  }
  __syncthreads();
  double *__restrict__ xc = parity ? nb.x1 : nb.x0;
  double *__restrict__ xn = parity ? nb.x0 : nb.x1;  // holds x^{k-1}, receives x^{k+1}
  if (bci[1]) {
#pragma unroll 8
    for (int64_t j = threadIdx.x; j < p; j += NT) nb.xbest[j] = xc[j];
  }
  if (bci[0]) return;
  const double m = bcd[0];
  const double invL = 1.0 / L;
  // gradient of F(X .) at the momentum point: -2 ((1+m) h_k - m h_{k-1})
  double l1v[1] = {0.0};
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
    const double xk = xc[j], xq = xn[j];
    const double yj = xk + m * (xk - xq);
    const double h = B.h1[j], hp = nb.hprev[j];
    nb.hprev[j] = h;
    const double v = yj + 2.0 * ((1.0 + m) * h - m * hp) * invL;
    nb.vbuf[j] = v;
    l1v[0] += fabs(v);
  }
  double thr;
  if (kind == 0) {
    thr = lam * invL;
  } else {
    // projection onto {||x||_1 <= lam}: threshold theta with sum max(|v| - theta, 0) = lam,
    // by the fixed point theta <- (sum_{|v| > theta} |v| - lam) / #{|v| > theta}
    // from theta = 0 (the active set shrinks monotonically; exact once it repeats)
    block_sum<NT, 1>(l1v, red);
    thr = 0.0;
    if (l1v[0] > lam) {
      double prev = -1.0;
      for (int k = 0; k <= p; k++) {
        double cs[2] = {0.0, 0.0};
#pragma unroll 8
        for (int64_t j = threadIdx.x; j < p; j += NT) {
          const double a = fabs(nb.vbuf[j]);
          if (a > thr) {
            cs[0] += 1.0;
            cs[1] += a;
          }
        }
        block_sum<NT, 2>(cs, red);
        if (cs[0] == prev) break;
        prev = cs[0];
        thr = (cs[1] - lam) / cs[0];
      }
    }
  }
  double l1[1] = {0.0};
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
    const double v = nb.vbuf[j];
    const double a = fabs(v) - thr;
    const double x = a > 0.0 ? copysign(a, v) : 0.0;
    xn[j] = x;
    l1[0] += fabs(x);
  }
  block_sum<NT, 1>(l1, red);
  __syncthreads();
  const int ns = compact_list(xn, p, nb.sidx, nb.sval, scan);
  if (tid == 0) {
    S->gval = lasso_G(kind, lam, l1[0]);
    S->indom = (kind == 0) || (l1[0] <= lam * (1.0 + 1e-9));
    S->nsupp = ns;
    S->parity = parity ^ 1;
    S->iter = S->iter + 1;
  }
}

}  // namespace

hipError_t launch_ac_init(const NodeParams *prm, NodeState *S, AcState *A, const AcBufs &ab, const NodeBufs &nb,
                          const double *beta0, double L0, hipStream_t s) {
  k_ac_init<<<1, NT, 0, s>>>(prm, S, A, ab, nb, beta0, L0);
  return hipGetLastError();
}

hipError_t launch_ac_resid(const Problem &P, const ProbBufs &B, const double *uz, double *ucur, const NodeState *S,
                           const AcState *A, hipStream_t s) {
  const int blocks = (int)((P.n + kResidThreads * kRows - 1) / (kResidThreads * kRows));
  if (blocks != B.nfin) return hipErrorInvalidValue;  // rbsum holds B.nfin block sums
  k_ac_resid<<<blocks, kResidThreads, 0, s>>>(P.n, P.y, P.loss, B, uz, ucur, S, A);
  return hipGetLastError();
}

hipError_t launch_ac_step(const NodeParams *prm, NodeState *S, AcState *A, const AcBufs &ab, const NodeBufs &nb,
                          const ProbBufs &B, double b, double c, int32_t restart_gap, hipStream_t s) {
  k_ac_step<<<1, NT, 0, s>>>(prm, S, A, ab, nb, B, b, c, restart_gap);
  return hipGetLastError();
}

hipError_t launch_lasso_init(NodeState *S, LassoState *LX, const NodeBufs &nb, const double *beta0, int64_t p,
                             int32_t kind, double lam, double L, hipStream_t s) {
  k_lasso_init<<<1, NT, 0, s>>>(S, LX, nb, beta0, p, kind, lam, L);
  return hipGetLastError();
}

hipError_t launch_lasso_step(const NodeParams *prm, NodeState *S, LassoState *LX, const NodeBufs &nb,
                             const ProbBufs &B, int32_t kind, double lam, hipStream_t s) {
  k_lasso_step<<<1, NT, 0, s>>>(prm, S, LX, nb, B, kind, lam);
  return hipGetLastError();
}

}  // namespace pr
