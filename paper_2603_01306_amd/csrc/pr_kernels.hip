// HIP kernels of libpr for gfx950 (MI355X, wave64).
//
// Matrix products (HBM bound):
//   k_gemv_t   h = X^T r (1 or 2 right-hand sides), FP32/BF16/FP64 X loaded
//              16 bytes per lane with non-temporal loads, FP64 accumulation,
//              one wave per 4 adjacent columns, deterministic in-wave
//              transpose-reduction.  Bytes per launch: n*p*sizeof(X) plus the
//              right-hand sides (read from L2).
//   k_spfwd    u = sum_t X[:, idx[t]] val[t] over a column list (the support
//              of the iterate, or all columns), split over row blocks x column
//              chunks; the last workgroup of a row block sums the chunk
//              partials in fixed order and runs the loss epilogue (residual /
//              induced dual vector, F and -F*(-zeta) partial sums).
// Per-node work (one 1024-thread workgroup per node):
//   k_node_step  dual value (closed-form conjugate, exact top-kbar selection),
//                gap / restart / termination, FISTA momentum, the prox of
//                Algorithm 2 in its pooled-threshold form, Algorithm 1 value of
//                the new iterate, support compaction.
#include <math.h>

#include "pr_internal.h"

namespace pr {
namespace {

constexpr int NT = kNodeThreads;
constexpr int NW = NT / 64;

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum of K values over a workgroup of NTH threads.  Every thread adds the
// per-wave totals in wave order, so all threads get the same, run-to-run
// reproducible result.  `red` needs NTH/64*K doubles of LDS.
template <int NTH, int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double *red) {
  constexpr int NWV = NTH / 64;
#pragma unroll
  for (int k = 0; k < K; k++) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane_id() == 0) {
#pragma unroll
    for (int k = 0; k < K; k++) red[wave_id() * K + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; k++) {
    double s = 0.0;
    for (int w = 0; w < NWV; w++) s += red[w * K + k];
    v[k] = s;
  }
}

template <int NTH>
__device__ __forceinline__ double block_max(double v, double *red) {
  constexpr int NWV = NTH / 64;
  v = wave_max(v);
  __syncthreads();
  if (lane_id() == 0) red[wave_id()] = v;
  __syncthreads();
  double s = red[0];
  for (int w = 1; w < NWV; w++) s = fmax(s, red[w]);
  return s;
}

// Exclusive prefix sum of an int over the workgroup (thread order).
template <int NTH>
__device__ __forceinline__ int block_excl_scan(int v, int *lds, int *total) {
  constexpr int NWV = NTH / 64;
  const int lane = lane_id(), w = wave_id();
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == 63) lds[w] = x;
  __syncthreads();
  int off = 0, tot = 0;
  for (int i = 0; i < NWV; i++) {
    int t = lds[i];
    if (i < w) off += t;
    tot += t;
  }
  *total = tot;
  return off + x - v;
}

// Descending bitonic sort of one double per lane of a wave.
__device__ __forceinline__ double wave_sort_desc(double v) {
  const int lane = lane_id();
#pragma unroll
  for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      double o = __shfl_xor(v, stride, 64);
      bool desc = (lane & size) == 0;
      bool lower = (lane & stride) == 0;
      bool take_max = (lower == desc);
      v = take_max ? (v > o ? v : o) : (v < o ? v : o);
    }
  }
  return v;
}

__device__ __forceinline__ double huber(double a, double M) {
  double x = fabs(a);
  return (x <= M) ? 0.5 * x * x : M * x - 0.5 * M * M;
}

__device__ __forceinline__ double softplus(double z) { return fmax(z, 0.0) + log1p(exp(-fabs(z))); }

__device__ __forceinline__ double fista_next_t(double t) { return 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t)); }

// ------------------------------------------------------------ selection

struct SelLds {
  unsigned int hist[2048];
  double gat[64];
  int scan[NW];
  int bin, above, cnt, ngat;
  double result;
};

// Exact k-th largest (1-based) of the entries a[j] >= 0, j in [0, p)
// (negative entries are ignored).  Radix selection on the IEEE bit pattern
// (monotone for non-negative doubles), 11 bits per level, and once the bin
// that holds the k-th value has at most 64 members they are gathered and
// sorted by one wave.  Requires 1 <= k <= #{a[j] >= 0}.
__device__ double select_kth(const double *__restrict__ a, int64_t p, int k, SelLds &sm) {
  const int tid = threadIdx.x;
  const int64_t E = (p + NT - 1) / NT;
  const int64_t j0 = (int64_t)tid * E, j1 = (j0 + E < p) ? j0 + E : p;
  unsigned long long prefix = 0ull;
  int above = 0, shift = 52, width = 11;
  for (;;) {
    for (int b = tid; b < 2048; b += NT) sm.hist[b] = 0u;
    __syncthreads();
    const unsigned long long mask = (1ull << width) - 1ull;
    for (int64_t j = j0; j < j1; j++) {
      double x = a[j];
      if (x >= 0.0) {
        unsigned long long key = (unsigned long long)__double_as_longlong(x);
        if ((key >> (shift + width)) == prefix) atomicAdd(&sm.hist[(key >> shift) & mask], 1u);
      }
    }
    __syncthreads();
    const int b0 = 2047 - 2 * tid, b1 = 2046 - 2 * tid;
    const int c0 = (int)sm.hist[b0], c1 = (int)sm.hist[b1];
    int tot;
    const int ex = block_excl_scan<NT>(c0 + c1, sm.scan, &tot);
    const int a0 = above + ex;
    if (a0 < k && k <= a0 + c0) {
      sm.bin = b0;
      sm.above = a0;
      sm.cnt = c0;
    }
    if (a0 + c0 < k && k <= a0 + c0 + c1) {
      sm.bin = b1;
      sm.above = a0 + c0;
      sm.cnt = c1;
    }
    __syncthreads();
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
      for (int64_t j = j0; j < j1; j++) {
        double x = a[j];
        if (x >= 0.0) {
          unsigned long long key = (unsigned long long)__double_as_longlong(x);
          if ((key >> shift) == prefix) {
            int pos = atomicAdd(&sm.ngat, 1);
            sm.gat[pos] = x;
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
      double r = sm.result;
      __syncthreads();
      return r;
    }
    const int nw = shift < 11 ? shift : 11;
    shift -= nw;
    width = nw;
  }
}

// TopSum_kbar of H_M over the entries a[j] >= 0: kbar H(t) + sum max(H(a_j) - H(t), 0)
// with t the exact kbar-th largest entry (Lemma function_g_conjugate_in_BnB).
__device__ double topsum_huber(const double *__restrict__ a, int64_t p, int kbar, double M, SelLds &sm,
                               double *red) {
  if (kbar <= 0) return 0.0;
  const double t = select_kth(a, p, kbar, sm);
  const double Ht = huber(t, M);
  const int64_t E = (p + NT - 1) / NT;
  const int64_t j0 = (int64_t)threadIdx.x * E, j1 = (j0 + E < p) ? j0 + E : p;
  double v[1] = {0.0};
  for (int64_t j = j0; j < j1; j++) {
    double x = a[j];
    if (x >= 0.0) v[0] += fmax(huber(x, M) - Ht, 0.0);
  }
  block_sum<NT, 1>(v, red);
  return (double)kbar * Ht + v[0];
}

// ------------------------------------------------------------ prox threshold

// Pooled-threshold form of Algorithm 2 + Moreau (eq. prox:gN).  With
// a_j = |v_j| on J_f, sorted magnitudes u = a / rho and weight 1/rho on the
// first kbar sorted positions, pool-adjacent-violators leaves exactly one
// pooled block straddling position kbar; writing tau = rho * (block value),
// the prox is
//     x_j = sgn(v_j) min( max(a_j - tau, 0), a_j / (1 + rho), M )
// (head positions keep the ridge/box map, pooled ones are shifted by tau,
// the tail is zero) and tau is the root of
//     S(tau) = sum_j clamp((a_j - tau) / D(tau), 0, 1) = kbar,
//     D(tau) = min(tau / rho, M),
// which is the block equation  c = prox_{rhobar H_M}(xibar)  written as a
// sum over all coordinates.  S is continuous and non-increasing; between
// breakpoints (a_j = tau, a_j = tau + D(tau), tau = rho M) the head count h,
// block count nb and block sum sB are fixed and the root has a closed form.
// The search iterates that closed form from the sets at the current point
// (an active-set Newton step), keeps a bracket, bisects when a step leaves
// it, and stops when the sets at a closed-form point equal the sets it was
// computed from, at which point the root is exact.
struct TauEval {
  double h, b, sB;
};

__device__ __forceinline__ TauEval tau_eval(const double *__restrict__ a, int64_t j0, int64_t j1,
                                            double tau, double D, double *red) {
  double v[3] = {0.0, 0.0, 0.0};
  const double hi = tau + D;
  for (int64_t j = j0; j < j1; j++) {
    double x = a[j];
    if (x > tau) {
      v[1] += 1.0;
      if (x > hi) v[0] += 1.0;
      else v[2] += x;
    }
  }
  block_sum<NT, 3>(v, red);
  return TauEval{v[0], v[1], v[2]};
}

__device__ double solve_tau(const double *__restrict__ a, int64_t p, int kbar, double rho, double M,
                            double warm, double *red, int *evals) {
  const int64_t E = (p + NT - 1) / NT;
  const int64_t j0 = (int64_t)threadIdx.x * E, j1 = (j0 + E < p) ? j0 + E : p;
  double st[2] = {0.0, 0.0};
  double mx = 0.0;
  for (int64_t j = j0; j < j1; j++) {
    double x = a[j];
    if (x > 0.0) {
      st[0] += 1.0;
      st[1] += x;
      mx = fmax(mx, x);
    }
  }
  block_sum<NT, 2>(st, red);
  const double amax = block_max<NT>(mx, red);
  *evals = 0;
  if (kbar <= 0) return INFINITY;
  const double K = (double)kbar;
  if (st[0] <= K) return 0.0;
  const bool finM = isfinite(M);
  auto Dof = [&](double t) { return finM ? fmin(t / rho, M) : t / rho; };
  auto froot = [&](double h, double nb, double sB) -> double {
    if (nb <= 0.0) return NAN;
    if (finM) {
      double Sf = h + (sB - nb * rho * M) / M;
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
    TauEval e = tau_eval(a, j0, j1, tau, D, red);
    *evals = it + 1;
    if (from_root && e.h == ph && e.b == pb) return tau;  // sets reproduced: exact root
    const double S = e.h + (e.sB - (e.b - e.h) * tau) / D;
    if (S > K) lo = tau;
    else if (S < K) hi = tau;
    else return tau;
    double c = froot(e.h, e.b - e.h, e.sB);
    if (c == tau) return tau;
    // safeguard: closed-form steps must stay strictly inside the bracket and
    // halve it at least every two steps, otherwise bisect
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
    ph = e.h;
    pb = e.b;
    if (!(c > lo && c < hi)) return c;  // bracket exhausted at double resolution
    tau = c;
  }
  return tau;
}

// Algorithm 1 on the free magnitudes q_j = a[j] >= 0 with theta = sum q.
// The loop of Algorithm 1 keeps the leading sorted values q_(j) while
// q_(j) > thetabar_j and fills the remaining kbar - |kept| slots of omega
// with thetabar = (theta - sum kept) / (kbar - |kept|).  The kept set is
// {q > thetabar}, so it is found without sorting by the fixed-point
// iteration s <- (sum_{q <= s} q) / (kbar - #{q > s}) from s = theta / kbar,
// whose kept sets grow monotonically to Algorithm 1's (at most kbar steps).
// Returns 0.5 * sum omega^2.
__device__ double alg1_free(const double *__restrict__ a, int64_t p, int kbar, double theta,
                            double *red) {
  if (kbar <= 0 || !(theta > 0.0)) return 0.0;
  const int64_t E = (p + NT - 1) / NT;
  const int64_t j0 = (int64_t)threadIdx.x * E, j1 = (j0 + E < p) ? j0 + E : p;
  const double K = (double)kbar;
  double s = theta / K;
  double prevK = 0.0;
  for (int it = 0; it <= kbar + 1; it++) {
    double v[3] = {0.0, 0.0, 0.0};  // #{q > s}, sum_{q <= s} q, sum_{q > s} q^2
    for (int64_t j = j0; j < j1; j++) {
      double x = a[j];
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
    // never let rounding move the threshold up: the kept set only grows
    s = fmin(s, v[1] / (K - v[0]));
  }
  return NAN;
}

// Support compaction, Algorithm 1 value, and dom g_N test (relative slack
// 1e-9, as the oracle) for the iterate x.  Writes |x_j| (free) or -1 into
// abuf, and the support list in ascending index order.
struct IterStats {
  double gval;
  int indom, nsupp;
};

__device__ IterStats finish_iterate(const double *__restrict__ x, const int8_t *__restrict__ st,
                                    int64_t p, int kbar, double M, double *__restrict__ abuf,
                                    int32_t *__restrict__ sidx, double *__restrict__ sval,
                                    double *red, int *scan) {
  const int64_t E = (p + NT - 1) / NT;
  const int64_t j0 = (int64_t)threadIdx.x * E, j1 = (j0 + E < p) ? j0 + E : p;
  double v[2] = {0.0, 0.0};  // theta, sum_{J1} x^2
  double amax = 0.0, j0max = 0.0, boxmax = 0.0;
  int cnt = 0;
  for (int64_t j = j0; j < j1; j++) {
    const double xj = x[j];
    const int s = st[j];
    const double ax = fabs(xj);
    amax = fmax(amax, ax);
    if (s == kZero) j0max = fmax(j0max, ax);
    else boxmax = fmax(boxmax, ax);
    if (s == kFree) v[0] += ax;
    else if (s == kOne) v[1] += xj * xj;
    abuf[j] = (s == kFree) ? ax : -1.0;
    cnt += (xj != 0.0);
  }
  int tot;
  int off = block_excl_scan<NT>(cnt, scan, &tot);
  for (int64_t j = j0; j < j1; j++) {
    const double xj = x[j];
    if (xj != 0.0) {
      sidx[off] = (int32_t)j;
      sval[off] = xj;
      off++;
    }
  }
  block_sum<NT, 2>(v, red);
  const double gA = block_max<NT>(amax, red);
  const double g0 = block_max<NT>(j0max, red);
  const double gB = block_max<NT>(boxmax, red);
  __syncthreads();  // abuf written above is read by every thread below
  const double zt = 1e-9 * fmax(1.0, gA);
  int ok = (g0 <= zt);
  if (isfinite(M) && gB > M * (1.0 + 1e-9)) ok = 0;
  if (kbar == 0) {
    if (v[0] > zt) ok = 0;
  } else if (isfinite(M) && v[0] > M * (double)kbar * (1.0 + 1e-9)) {
    ok = 0;
  }
  const double gv = 0.5 * v[1] + alg1_free(abuf, p, kbar, v[0], red);
  return IterStats{gv, ok, tot};
}

// ------------------------------------------------------------ node kernels

__global__ __launch_bounds__(NT) void k_node_init(const NodeParams *__restrict__ prm, NodeState *S,
                                                  NodeBufs nb, const double *__restrict__ beta0,
                                                  double L) {
  __shared__ double red[NW * 4];
  __shared__ int scan[NW];
  const int64_t p = prm->p;
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
  const int64_t E = (p + NT - 1) / NT;
  const int64_t j0 = (int64_t)tid * E, j1 = (j0 + E < p) ? j0 + E : p;
  const int parity = S->parity;
  const double L = S->L;

  // loss-side terms of this iterate, summed over row blocks in fixed order
  double Fk = 0.0, negconj = 0.0;
  for (int i = 0; i < B.rb; i++) {
    Fk += B.rbsum[2 * i];
    negconj += B.rbsum[2 * i + 1];
  }
  // dual: w = X^T zeta / (2 lambda2)
  const double wscale = (loss == kLsq) ? 1.0 / lam2 : 0.5 / lam2;
  double sj1[1] = {0.0};
  for (int64_t j = j0; j < j1; j++) {
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
      if (it == 0) {
        restart = 1;
        gap_ref = gap;
      } else if (gap <= gap_ref / prm->eta) {
        restart = 1;
        gap_ref = gap;
        restarts++;
      }
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
  if (bci[2])
    for (int64_t j = j0; j < j1; j++) nb.xbest[j] = xc[j];
  if (bci[0]) return;
  const double m = bcd[0];
  const int restart = bci[1];

  // gradient step at the momentum point
  const double invL = 1.0 / L;
  for (int64_t j = j0; j < j1; j++) {
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
  for (int64_t j = j0; j < j1; j++) {
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
  const int64_t E = (p + NT - 1) / NT;
  const int64_t j0 = (int64_t)threadIdx.x * E, j1 = (j0 + E < p) ? j0 + E : p;
  for (int64_t j = j0; j < j1; j++) abuf[j] = (st[j] == kFree) ? fabs(v[j]) : -1.0;
  __syncthreads();
  int evals;
  const double tau = solve_tau(abuf, p, kbar, rho, M, -1.0, red, &evals);
  const double inv1p = 1.0 / (1.0 + rho);
  for (int64_t j = j0; j < j1; j++) {
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
  const int64_t E = (p + NT - 1) / NT;
  const int64_t j0 = (int64_t)threadIdx.x * E, j1 = (j0 + E < p) ? j0 + E : p;
  if (beta) {
    IterStats is = finish_iterate(beta, st, p, kbar, M, abuf, sidx, sval, red, scan);
    if (threadIdx.x == 0) out2[0] = is.indom ? is.gval : INFINITY;
    __syncthreads();
  }
  if (alpha) {
    double s1[1] = {0.0};
    for (int64_t j = j0; j < j1; j++) {
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
  for (int64_t i = threadIdx.x; i < n; i += NT) s[0] += v[i] * v[i];
  block_sum<NT, 1>(s, red);
  if (threadIdx.x == 0) *out = s[0];
}

__global__ void k_scale_copy(const double *src, double *dst, double a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = a * src[i];
}

__global__ void k_iota(int32_t *idx, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    idx[i] = (int32_t)i;
}

// ------------------------------------------------------------ X^T r

template <typename T>
struct XLoad;

template <>
struct XLoad<float> {
  static constexpr int VEC = 4;
  __device__ __forceinline__ static void load(const float *p, double (&d)[4]) {
    f4_t v = __builtin_nontemporal_load(reinterpret_cast<const f4_t *>(p));
    d[0] = (double)v.x;
    d[1] = (double)v.y;
    d[2] = (double)v.z;
    d[3] = (double)v.w;
  }
};

template <>
struct XLoad<double> {
  static constexpr int VEC = 2;
  __device__ __forceinline__ static void load(const double *p, double (&d)[2]) {
    d2_t v = __builtin_nontemporal_load(reinterpret_cast<const d2_t *>(p));
    d[0] = v.x;
    d[1] = v.y;
  }
};

// bf16 stored as uint16_t bit patterns
template <>
struct XLoad<uint16_t> {
  static constexpr int VEC = 8;
  __device__ __forceinline__ static void load(const uint16_t *p, double (&d)[8]) {
    u4_t v = __builtin_nontemporal_load(reinterpret_cast<const u4_t *>(p));
    const unsigned int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; q++) {
      d[2 * q] = (double)__uint_as_float(w[q] << 16);
      d[2 * q + 1] = (double)__uint_as_float(w[q] & 0xffff0000u);
    }
  }
};

template <int VEC>
__device__ __forceinline__ void load_rhs(const double *__restrict__ r, int64_t i, double (&d)[VEC]) {
#pragma unroll
  for (int q = 0; q < VEC; q += 2) {
    d2_t v = *reinterpret_cast<const d2_t *>(r + i + q);
    d[q] = v.x;
    d[q + 1] = v.y;
  }
}

// Deterministic transpose-reduction of 4 per-lane partial sums (one per
// column) over the 64 lanes: afterwards lane 16*c holds the total of column c.
__device__ __forceinline__ double reduce4(double (&v)[4]) {
  const int lane = lane_id();
  const bool b5 = (lane & 32) != 0, b4 = (lane & 16) != 0;
  double s0 = b5 ? v[0] : v[2], s1 = b5 ? v[1] : v[3];
  double k0 = b5 ? v[2] : v[0], k1 = b5 ? v[3] : v[1];
  k0 += __shfl_xor(s0, 32, 64);
  k1 += __shfl_xor(s1, 32, 64);
  double s = b4 ? k0 : k1;
  double k = b4 ? k1 : k0;
  k += __shfl_xor(s, 16, 64);
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) k += __shfl_xor(k, o, 64);
  return k;
}

template <typename T, int NRHS>
__global__ __launch_bounds__(kGemvThreads) void k_gemv_t(const T *__restrict__ X, int64_t n, int64_t p,
                                                         const double *__restrict__ r1,
                                                         const double *__restrict__ r2,
                                                         double *__restrict__ h1,
                                                         double *__restrict__ h2,
                                                         const int32_t *__restrict__ done) {
  if (done && *done) return;
  constexpr int VEC = XLoad<T>::VEC;
  constexpr int U = 2;  // row steps in flight
  const int lane = lane_id();
  const int64_t col0 = ((int64_t)blockIdx.x * (kGemvThreads / 64) + wave_id()) * kColsPerWave;
  if (col0 >= p) return;
  const T *c[4];
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int64_t cj = (col0 + q < p) ? col0 + q : p - 1;
    c[q] = X + cj * n;
  }
  double acc[NRHS][4];
#pragma unroll
  for (int h = 0; h < NRHS; h++)
#pragma unroll
    for (int q = 0; q < 4; q++) acc[h][q] = 0.0;
  const int64_t step = 64 * VEC;
  int64_t i = (int64_t)lane * VEC;
  for (; i + (U - 1) * step + VEC <= n; i += U * step) {
    double xv[U][4][VEC];
    double rv[U][NRHS][VEC];
#pragma unroll
    for (int u = 0; u < U; u++) {
#pragma unroll
      for (int q = 0; q < 4; q++) XLoad<T>::load(c[q] + i + u * step, xv[u][q]);
      load_rhs<VEC>(r1, i + u * step, rv[u][0]);
      if (NRHS > 1) load_rhs<VEC>(r2, i + u * step, rv[u][NRHS - 1]);
    }
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
      for (int h = 0; h < NRHS; h++)
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
          for (int e = 0; e < VEC; e++) acc[h][q] = fma(xv[u][q][e], rv[u][h][e], acc[h][q]);
  }
  for (; i + VEC <= n; i += step) {
    double xv[4][VEC];
    double rv[NRHS][VEC];
#pragma unroll
    for (int q = 0; q < 4; q++) XLoad<T>::load(c[q] + i, xv[q]);
    load_rhs<VEC>(r1, i, rv[0]);
    if (NRHS > 1) load_rhs<VEC>(r2, i, rv[NRHS - 1]);
#pragma unroll
    for (int h = 0; h < NRHS; h++)
#pragma unroll
      for (int q = 0; q < 4; q++)
#pragma unroll
        for (int e = 0; e < VEC; e++) acc[h][q] = fma(xv[q][e], rv[h][e], acc[h][q]);
  }
  const int64_t col = col0 + (lane >> 4);
  const bool writer = (lane & 15) == 0 && col < p;
  {
    double t = reduce4(acc[0]);
    if (writer) h1[col] = t;
  }
  if (NRHS > 1) {
    double t = reduce4(acc[NRHS - 1]);
    if (writer) h2[col] = t;
  }
}

// ------------------------------------------------------------ column-list GEMV

template <typename T>
__global__ __launch_bounds__(kSpThreads) void k_spfwd(const T *__restrict__ X, int64_t n,
                                                      const double *__restrict__ y, ProbBufs B,
                                                      const int32_t *__restrict__ idx,
                                                      const double *__restrict__ val,
                                                      const int32_t *__restrict__ nlist, int32_t mode,
                                                      const NodeState *S, double *u_out) {
  constexpr int VEC = XLoad<T>::VEC;
  __shared__ double red[(kSpThreads / 64) * 4];
  __shared__ int last;
  if (S && S->done) return;
  const int rb = blockIdx.x, ch = blockIdx.y;
  const int ns = *nlist;
  const int cs = (ns + B.nch - 1) / B.nch;
  const int t0 = ch * cs;
  const int t1 = (t0 + cs < ns) ? t0 + cs : ns;
  const int64_t row0 = (int64_t)rb * B.rows + (int64_t)threadIdx.x * VEC;
  const bool active = row0 < n;
  double acc[VEC];
#pragma unroll
  for (int e = 0; e < VEC; e++) acc[e] = 0.0;
  if (active) {
    int t = t0;
    for (; t + 4 <= t1; t += 4) {
      double xv[4][VEC];
      double w[4];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        XLoad<T>::load(X + (int64_t)idx[t + q] * n + row0, xv[q]);
        w[q] = val[t + q];
      }
#pragma unroll
      for (int q = 0; q < 4; q++)
#pragma unroll
        for (int e = 0; e < VEC; e++) acc[e] = fma(xv[q][e], w[q], acc[e]);
    }
    for (; t < t1; t++) {
      double xv[VEC];
      XLoad<T>::load(X + (int64_t)idx[t] * n + row0, xv);
      const double w = val[t];
#pragma unroll
      for (int e = 0; e < VEC; e++) acc[e] = fma(xv[e], w, acc[e]);
    }
    double *part = B.part + (int64_t)ch * n + row0;
#pragma unroll
    for (int e = 0; e < VEC; e++) __hip_atomic_store(part + e, acc[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int prev = atomicAdd(&B.counter[rb], 1u);
    last = (prev == (unsigned int)(B.nch - 1));
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x == 0) B.counter[rb] = 0u;
  double u[VEC];
#pragma unroll
  for (int e = 0; e < VEC; e++) u[e] = 0.0;
  if (active) {
    for (int c = 0; c < B.nch; c++) {
      const double *part = B.part + (int64_t)c * n + row0;
#pragma unroll
      for (int e = 0; e < VEC; e++) u[e] += __hip_atomic_load(part + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  double sums[2] = {0.0, 0.0};
  if (mode == kSpPlain) {
    if (active)
#pragma unroll
      for (int e = 0; e < VEC; e++) u_out[row0 + e] = u[e];
    return;
  }
  const int improved = S->improved;
  if (mode == kSpLsq) {
    if (active) {
#pragma unroll
      for (int e = 0; e < VEC; e++) {
        const int64_t i = row0 + e;
        if (improved) B.zbest[i] = 2.0 * B.r[i];
        const double yi = y[i];
        const double ri = yi - u[e];
        B.r[i] = ri;
        sums[0] += ri * ri;
        sums[1] += 2.0 * ri * yi - ri * ri;
      }
    }
  } else {
    const double t = S->t;
    const double mt = (t - 1.0) / fista_next_t(t);
    if (active) {
#pragma unroll
      for (int e = 0; e < VEC; e++) {
        const int64_t i = row0 + e;
        const double uo = B.ucur[i];
        B.uprev[i] = uo;
        B.ucur[i] = u[e];
        if (improved) B.zbest[i] = B.r[i];
        const double yi = y[i];
        const double z = yi * u[e];
        const double a = 1.0 / (1.0 + exp(z));
        B.r[i] = yi * a;
        sums[0] += softplus(-z);
        sums[1] += a * softplus(z) + (1.0 - a) * softplus(-z);
        const double sm = (1.0 + mt) * u[e] - mt * uo;
        B.gm[i] = -yi / (1.0 + exp(yi * sm));
      }
    }
  }
  block_sum<kSpThreads, 2>(sums, red);
  if (threadIdx.x == 0) {
    B.rbsum[2 * rb] = sums[0];
    B.rbsum[2 * rb + 1] = sums[1];
  }
}

}  // namespace

// ------------------------------------------------------------ launchers

hipError_t launch_gemv_t(const Problem &P, const double *r1, const double *r2, double *h1, double *h2,
                         const int32_t *done, hipStream_t s) {
  const int cols_per_block = (kGemvThreads / 64) * kColsPerWave;
  dim3 grid((unsigned)((P.p + cols_per_block - 1) / cols_per_block));
  dim3 block(kGemvThreads);
  const bool two = (r2 != nullptr);
  switch (P.xdt) {
    case kF32:
      if (two) k_gemv_t<float, 2><<<grid, block, 0, s>>>((const float *)P.X, P.n, P.p, r1, r2, h1, h2, done);
      else k_gemv_t<float, 1><<<grid, block, 0, s>>>((const float *)P.X, P.n, P.p, r1, r2, h1, h2, done);
      break;
    case kF64:
      if (two) k_gemv_t<double, 2><<<grid, block, 0, s>>>((const double *)P.X, P.n, P.p, r1, r2, h1, h2, done);
      else k_gemv_t<double, 1><<<grid, block, 0, s>>>((const double *)P.X, P.n, P.p, r1, r2, h1, h2, done);
      break;
    default:
      if (two) k_gemv_t<uint16_t, 2><<<grid, block, 0, s>>>((const uint16_t *)P.X, P.n, P.p, r1, r2, h1, h2, done);
      else k_gemv_t<uint16_t, 1><<<grid, block, 0, s>>>((const uint16_t *)P.X, P.n, P.p, r1, r2, h1, h2, done);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_spfwd(const Problem &P, const ProbBufs &B, const int32_t *idx, const double *val,
                        const int32_t *nlist, int32_t mode, const NodeState *S, double *u_out,
                        hipStream_t s) {
  dim3 grid((unsigned)B.rb, (unsigned)B.nch);
  dim3 block(kSpThreads);
  switch (P.xdt) {
    case kF32:
      k_spfwd<float><<<grid, block, 0, s>>>((const float *)P.X, P.n, P.y, B, idx, val, nlist, mode, S, u_out);
      break;
    case kF64:
      k_spfwd<double><<<grid, block, 0, s>>>((const double *)P.X, P.n, P.y, B, idx, val, nlist, mode, S, u_out);
      break;
    default:
      k_spfwd<uint16_t><<<grid, block, 0, s>>>((const uint16_t *)P.X, P.n, P.y, B, idx, val, nlist, mode, S, u_out);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_node_init(const NodeParams *prm, NodeState *S, NodeBufs nb, const double *beta0,
                            double L, hipStream_t s) {
  k_node_init<<<1, NT, 0, s>>>(prm, S, nb, beta0, L);
  return hipGetLastError();
}

hipError_t launch_node_step(const NodeParams *prm, NodeState *S, NodeBufs nb, const ProbBufs &B,
                            hipStream_t s) {
  k_node_step<<<1, NT, 0, s>>>(prm, S, nb, B);
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

hipError_t launch_iota(int32_t *idx, int64_t n, hipStream_t s) {
  k_iota<<<256, 256, 0, s>>>(idx, n);
  return hipGetLastError();
}

}  // namespace pr
