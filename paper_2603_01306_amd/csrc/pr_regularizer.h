// Device routines of the regulariser g_N shared by the per-node kernels
// (pr_node.hip) and the iteration-variant kernels (pr_variants.hip): exact
// top-k selection, TopSum of the Huber function (g_N*), the pooled-threshold
// prox of Algorithm 2 + Moreau, Algorithm 1's value and the support list of
// an iterate.  One 512-thread workgroup; vectors in global memory.
#pragma once
#include "pr_device.h"

namespace pr {
namespace {
using namespace dev;

// ------------------------------------------------------------ selection

struct SelLds {
  unsigned int hist[2048];
  double gat[64];
  int scan[NW];
  int bin, above, cnt, ngat;
  double result;
};

// Locate, in a 2048-bin histogram scanned from the top bin down, the bin that
// holds the k-th largest entry given `above` entries in higher bins.  Each
// thread owns 2048 / NT consecutive bins (descending).
__device__ __forceinline__ void hist_locate(SelLds &sm, int above, int k) {
  constexpr int BPT = 2048 / NT;
  const int tid = threadIdx.x;
  int c[BPT];
  int loc = 0;
#pragma unroll
  for (int q = 0; q < BPT; q++) {
    c[q] = (int)sm.hist[2047 - BPT * tid - q];
    loc += c[q];
  }
  int tot;
  int acc = above + block_excl_scan<NT>(loc, sm.scan, &tot);
#pragma unroll
  for (int q = 0; q < BPT; q++) {
    if (acc < k && k <= acc + c[q]) {
      sm.bin = 2047 - BPT * tid - q;
      sm.above = acc;
      sm.cnt = c[q];
    }
    acc += c[q];
  }
  __syncthreads();
}

// Exact k-th largest (1-based) of the entries a[j] >= 0, j in [0, p)
// (negative entries are ignored).  Radix selection on the IEEE bit pattern
// (monotone for non-negative doubles), 11 bits per level, and once the bin
// that holds the k-th value has at most 64 members they are gathered and
// sorted by one wave.  Requires 1 <= k <= #{a[j] >= 0}.
__device__ double select_kth(const double *__restrict__ a, int64_t p, int k, SelLds &sm) {
  const int tid = threadIdx.x;
  unsigned long long prefix = 0ull;
  int above = 0, shift = 52, width = 11;
  for (;;) {
    for (int b = tid; b < 2048; b += NT) sm.hist[b] = 0u;
    __syncthreads();
    const unsigned long long mask = (1ull << width) - 1ull;
#pragma unroll 8
    for (int64_t j = threadIdx.x; j < p; j += NT) {
      double x = a[j];
      if (x >= 0.0) {
        unsigned long long key = (unsigned long long)__double_as_longlong(x);
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
#pragma unroll 8
      for (int64_t j = threadIdx.x; j < p; j += NT) {
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
  double v[1] = {0.0};
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
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

__device__ __forceinline__ TauEval tau_eval(const double *__restrict__ a, int64_t p, double tau, double D,
                                            double *red) {
  double v[3] = {0.0, 0.0, 0.0};
  const double hi = tau + D;
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
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
  double st[2] = {0.0, 0.0};
  double mx = 0.0;
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
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
    TauEval e = tau_eval(a, p, tau, D, red);
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
  const double K = (double)kbar;
  double s = theta / K;
  double prevK = 0.0;
  for (int it = 0; it <= kbar + 1; it++) {
    double v[3] = {0.0, 0.0, 0.0};  // #{q > s}, sum_{q <= s} q, sum_{q > s} q^2
#pragma unroll 8
    for (int64_t j = threadIdx.x; j < p; j += NT) {
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
// abuf, and the support list in a fixed order: thread t owns j = t, t + 512,
// ... (coalesced passes) and its entries follow those of threads 0 .. t-1.
struct IterStats {
  double gval;
  int indom, nsupp;
};

__device__ IterStats finish_iterate(const double *__restrict__ x, const int8_t *__restrict__ st,
                                    int64_t p, int kbar, double M, double *__restrict__ abuf,
                                    int32_t *__restrict__ sidx, double *__restrict__ sval,
                                    double *red, int *scan) {
  double v[2] = {0.0, 0.0};  // theta, sum_{J1} x^2
  double amax = 0.0, j0max = 0.0, boxmax = 0.0;
  int cnt = 0;
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
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
#pragma unroll 8
  for (int64_t j = threadIdx.x; j < p; j += NT) {
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

}  // namespace
}  // namespace pr
