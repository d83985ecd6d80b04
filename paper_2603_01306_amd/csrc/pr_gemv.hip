// X^T r on gfx950: h = X^T r (one or two right-hand sides) for column-major X
// stored FP32 / BF16 / FP64, accumulated in FP64.
//
// One wave per C adjacent columns streams the full column length: each lane
// loads 16 bytes of every column per step with non-temporal loads (X is read
// once per launch and should not displace the L2-resident right-hand side),
// one row step per lane in flight (a measured sweep over 1, 2, 4 steps on
// MI355X favoured 1), then a deterministic in-wave transpose reduction leaves
// column c's total in lane (64 / C) c.  With one right-hand side the stream
// runs best with as many waves as are resident at once (about 5 per SIMD):
// 4096 waves give 6.9 TB/s, 2048 5.9, and 8192 (1.6 rounds) 5.5-5.7, so C
// is the smallest of 2, 4, 8 that keeps p / C at or below 5120 (2 up to
// p = 10240; C = 2 beat 1, 4 and 8 on the 16384 x 8192 design).  With two,
// every wave re-reads both right-hand sides from L2 for its columns, and at
// small C that L2 traffic (at C = 2 twice the bytes of X) competes with X
// (logistic 32768 x 16384: 585 / 537 / 504 / 498 us per iteration at C = 2 /
// 4 / 8 / 16; 16 needs 254 VGPRs), while at large C small designs leave the
// grid short of waves (16384 x 8192: 5.6 TB/s at C = 8, 6.0 at C = 4): C is
// the smallest of 2, 4, 8 that keeps p / C at or below 2048 waves.  With
// all loads of a step issued together (below), C = 4 / 4096 waves and two
// row steps in flight stayed slower than C = 8, one step (345 / 325 vs 313
// us), and staging both right-hand sides in LDS per workgroup (one barrier
// per 1024-row tile) cost 380-440 us.
// Algorithmic bytes per launch: n*p*sizeof(X) + 8n per right-hand side + 8p
// per output.
#include "pr_device.h"

namespace pr {
namespace {
using namespace dev;

constexpr int kGemvWavesMax = 5120;  // waves of one resident round of the one-RHS kernel
constexpr int kGemvWaves2 = 2048;    // waves the two-RHS kernel aims for
// columns per wave, the smallest of 2, 4, 8 that keeps the grid within
// kGemvWavesMax waves (one right-hand side) or kGemvWaves2 (two)
inline int gemv_cols(int nrhs, int64_t p) {
  const int64_t wmax = nrhs == 1 ? kGemvWavesMax : kGemvWaves2;
  int c = 2;
  while (c < 8 && p > (int64_t)c * wmax) c *= 2;
  return c;
}

// Deterministic transpose reduction of C per-lane partial sums (one per
// column) over the 64 lanes: at each exchange over lane bit s (32, 16, ...)
// the lanes with that bit set keep the upper half of their columns and add
// their partner's, the others the lower half; once one column is left the
// plain butterfly finishes.  Column c's total ends in lane (64 / C) c.
template <int C>
__device__ __forceinline__ double reduce_cols(double (&v)[C]) {
  const int lane = lane_id();
  double cur[C];
#pragma unroll
  for (int i = 0; i < C; i++) cur[i] = v[i];
  int s = 32;
#pragma unroll
  for (int w = C; w > 1; w >>= 1, s >>= 1) {
    const bool hi = (lane & s) != 0;
#pragma unroll
    for (int i = 0; i < w / 2; i++) {
      const double send = hi ? cur[i] : cur[i + w / 2];
      const double keep = hi ? cur[i + w / 2] : cur[i];
      cur[i] = keep + __shfl_xor(send, s, 64);
    }
  }
#pragma unroll
  for (; s > 0; s >>= 1) cur[0] += __shfl_xor(cur[0], s, 64);
  return cur[0];
}

// g_N and the dom test of a node's iterate whose nonzeros (and only those)
// are listed in idx / val (ns entries, J1 and J0 entries flagged with
// kJ1Flag / kJ0Flag), for the node with parameters P, by one workgroup of NTH
// threads: theta = sum of the free |x_j|, the J1 sum of squares and the
// largest |x_j| off and on J0 in one block reduction (the dom test of the
// node step), then Algorithm 1 over the free magnitudes as the fixed point
// s <- (sum of the values <= s) / (kbar - #{q > s}) from s = theta / kbar,
// one block reduction per round (zeros of the free set change none of these
// sums).  Each pass loads eight entries per thread before using them.
// Writes S->gval and S->indom.  Runs as one extra workgroup of the X^T r
// product, which follows the column-list product of the same iterate and
// outlasts this evaluation.
template <int NTH>
__device__ void list_values(const NodeParams *__restrict__ P, const int32_t *__restrict__ idx,
                            const double *__restrict__ val, int ns, NodeState *S) {
  constexpr int NWS = NTH / 64;
  constexpr int U = 8;
  __shared__ double red[NWS * 4];
  const int kbar = P->kbar;
  const double M = P->M;
  double v[4] = {0.0, 0.0, 0.0, 0.0};  // theta, sum_{J1} x^2, max |x| off J0, max |x| on J0
  for (int t0 = threadIdx.x; t0 < ns; t0 += U * NTH) {
    int32_t it[U];
    double xv[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int t = t0 + u * NTH;
      it[u] = t < ns ? idx[t] : 0;
      xv[u] = t < ns ? val[t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const double ax = fabs(xv[u]);
      if (it[u] & kJ0Flag) {
        v[3] = fmax(v[3], ax);
      } else {
        if (it[u] & kJ1Flag) v[1] += xv[u] * xv[u];
        else v[0] += ax;
        v[2] = fmax(v[2], ax);
      }
    }
  }
  v[0] = wave_sum(v[0]);
  v[1] = wave_sum(v[1]);
  v[2] = wave_max(v[2]);
  v[3] = wave_max(v[3]);
  if (lane_id() == 0) {
#pragma unroll
    for (int k = 0; k < 4; k++) red[wave_id() * 4 + k] = v[k];
  }
  __syncthreads();
  double theta = 0.0, sq = 0.0, gB = 0.0, g0 = 0.0;
  for (int w = 0; w < NWS; w++) {
    theta += red[w * 4];
    sq += red[w * 4 + 1];
    gB = fmax(gB, red[w * 4 + 2]);
    g0 = fmax(g0, red[w * 4 + 3]);
  }
  const double zt = 1e-9 * fmax(1.0, fmax(gB, g0));
  int ok = (g0 <= zt);
  if (isfinite(M) && gB > M * (1.0 + 1e-9)) ok = 0;
  if (kbar == 0) {
    if (theta > zt) ok = 0;
  } else if (isfinite(M) && theta > M * (double)kbar * (1.0 + 1e-9)) {
    ok = 0;
  }
  double a1 = 0.0;
  if (kbar > 0 && theta > 0.0) {
    const double K = (double)kbar;
    double sv = theta / K, prevK = 0.0;
    a1 = NAN;
    for (int round = 0; round <= kbar + 1; round++) {
      double r[3] = {0.0, 0.0, 0.0};  // #{q > s}, sum of q <= s, sum of q^2 over q > s
      for (int t0 = threadIdx.x; t0 < ns; t0 += U * NTH) {
        int32_t it[U];
        double xv[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
          const int t = t0 + u * NTH;
          it[u] = t < ns ? idx[t] : kJ0Flag;  // past the list: skipped below
          xv[u] = t < ns ? val[t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
          if (it[u] & (kJ1Flag | kJ0Flag)) continue;
          const double q = fabs(xv[u]);
          if (q > sv) {
            r[0] += 1.0;
            r[2] += q * q;
          } else {
            r[1] += q;
          }
        }
      }
      block_sum<NTH, 3>(r, red);
      if (r[0] == prevK || r[0] >= K) {
        a1 = 0.5 * (r[2] + (K - r[0]) * sv * sv);
        break;
      }
      prevK = r[0];
      sv = fmin(sv, r[1] / (K - r[0]));
    }
  }
  if (threadIdx.x == 0) {
    S->gval = 0.5 * sq + a1;
    S->indom = ok;
  }
}


template <typename T, int NRHS, int C>
__global__ __launch_bounds__(kGemvThreads) void k_gemv_t(const T *__restrict__ X, int64_t n, int64_t p,
                                                         const double *__restrict__ r1,
                                                         const double *__restrict__ r2,
                                                         double *__restrict__ h1,
                                                         double *__restrict__ h2,
                                                         const int32_t *__restrict__ done,
                                                         const NodeParams *__restrict__ node, NodeState *S,
                                                         const int32_t *__restrict__ sidx,
                                                         const double *__restrict__ sval,
                                                         const int32_t *__restrict__ nlist,
                                                         const double *__restrict__ dsum, int nfin) {
  if (done && *done) return;
  // backtracking: a rejected trial needs no product (every wave takes the
  // node step's decision from the same sums)
  if (dsum && S->bt && S->iter > 0 && !bt_accept(bt_remainder(dsum, nfin), S->L, S->dxy, node->Lmax)) return;
  // with `node` the first workgroup (dispatched first) evaluates g_N of the
  // listed iterate; the product's workgroups follow it
  int bx = (int)blockIdx.x;
  if (node) {
    if (bx == 0) {
      list_values<kGemvThreads>(node, sidx, sval, *nlist, S);
      return;
    }
    bx--;
  }
  constexpr int VEC = XLoad<T>::VEC;
#ifndef PR_GEMVT_STEPS
#define PR_GEMVT_STEPS 1
#endif
  constexpr int U = PR_GEMVT_STEPS;  // row steps in flight
  const int lane = lane_id();
  const int64_t col0 = ((int64_t)bx * (kGemvThreads / 64) + wave_id()) * C;
  if (col0 >= p) return;
  const T *c[C];
#pragma unroll
  for (int q = 0; q < C; q++) {
    const int64_t cj = (col0 + q < p) ? col0 + q : p - 1;
    c[q] = X + cj * n;
  }
  double acc[NRHS][C];
#pragma unroll
  for (int h = 0; h < NRHS; h++)
#pragma unroll
    for (int q = 0; q < C; q++) acc[h][q] = 0.0;
  const int64_t step = 64 * VEC;
  int64_t i = (int64_t)lane * VEC;
  // With two right-hand sides every load of a step is issued before its first
  // use: the scheduling barrier keeps the compiler from sinking the
  // right-hand-side loads below the widening of the first X vector, which
  // made a step three dependent memory round trips (logistic 32768 x 16384:
  // 338 -> 312 us).  With one right-hand side the compiler's own order (X,
  // then the right-hand side once the first column has arrived) measured
  // faster: 316 vs 340 us on a 32768 x 16384 FP32 design, 89.8 vs 94.0 on
  // 16000 x 16000 BF16, equal on 16384 x 8192.
  for (; i + (U - 1) * step + VEC <= n; i += U * step) {
    typename XLoad<T>::raw_t xr[U][C];
    double rv[U][NRHS][VEC];
#pragma unroll
    for (int u = 0; u < U; u++) {
#pragma unroll
      for (int q = 0; q < C; q++) xr[u][q] = XLoad<T>::raw(c[q] + i + u * step);
      load_rhs<VEC>(r1, i + u * step, rv[u][0]);
      if (NRHS > 1) load_rhs<VEC>(r2, i + u * step, rv[u][NRHS - 1]);
    }
    if constexpr (NRHS > 1) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
      for (int q = 0; q < C; q++) {
        double xv[VEC];
        XLoad<T>::cvt(xr[u][q], xv);
#pragma unroll
        for (int h = 0; h < NRHS; h++)
#pragma unroll
          for (int e = 0; e < VEC; e++) acc[h][q] = fma(xv[e], rv[u][h][e], acc[h][q]);
      }
  }
  for (; i + VEC <= n; i += step) {
    typename XLoad<T>::raw_t xr[C];
    double rv[NRHS][VEC];
#pragma unroll
    for (int q = 0; q < C; q++) xr[q] = XLoad<T>::raw(c[q] + i);
    load_rhs<VEC>(r1, i, rv[0]);
    if (NRHS > 1) load_rhs<VEC>(r2, i, rv[NRHS - 1]);
    if constexpr (NRHS > 1) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < C; q++) {
      double xv[VEC];
      XLoad<T>::cvt(xr[q], xv);
#pragma unroll
      for (int h = 0; h < NRHS; h++)
#pragma unroll
        for (int e = 0; e < VEC; e++) acc[h][q] = fma(xv[e], rv[h][e], acc[h][q]);
    }
  }
  constexpr int LPC = 64 / C;  // lanes per column after the reduction
  const int64_t col = col0 + lane / LPC;
  const bool writer = (lane % LPC) == 0 && col < p;
  {
    double t = reduce_cols(acc[0]);
    if (writer) h1[col] = t;
  }
  if (NRHS > 1) {
    double t = reduce_cols(acc[NRHS - 1]);
    if (writer) h2[col] = t;
  }
}

}  // namespace

hipError_t launch_gemv_t(const Problem &P, const double *r1, const double *r2, double *h1, double *h2,
                         const int32_t *done, hipStream_t s, const NodeParams *node, NodeState *S,
                         const int32_t *sidx, const double *sval, const int32_t *nlist, const double *dsum,
                         int32_t nfin) {
  if (node && (!S || !sidx || !sval || !nlist)) return hipErrorInvalidValue;
  if (dsum && !node) return hipErrorInvalidValue;
  const bool two = (r2 != nullptr);
  const int cols = gemv_cols(two ? 2 : 1, P.p);
  const int cols_per_block = (kGemvThreads / 64) * cols;
  dim3 grid((unsigned)((P.p + cols_per_block - 1) / cols_per_block) + (node ? 1u : 0u));
  dim3 block(kGemvThreads);
#define PR_GEMVT(T, R, C)                                                                                \
  k_gemv_t<T, R, C><<<grid, block, 0, s>>>((const T *)P.X, P.n, P.p, r1, r2, h1, h2, done, node, S, sidx, sval, \
                                           nlist, dsum, nfin)
#define PR_GEMVT1(T, R)                \
  switch (cols) {                      \
    case 2: PR_GEMVT(T, R, 2); break;  \
    case 4: PR_GEMVT(T, R, 4); break;  \
    default: PR_GEMVT(T, R, 8); break; \
  }
  switch (P.xdt) {
    case kF32:
      if (two) PR_GEMVT1(float, 2)
      else PR_GEMVT1(float, 1)
      break;
    case kF64:
      if (two) PR_GEMVT1(double, 2)
      else PR_GEMVT1(double, 1)
      break;
    default:
      if (two) PR_GEMVT1(uint16_t, 2)
      else PR_GEMVT1(uint16_t, 1)
      break;
  }
#undef PR_GEMVT1
#undef PR_GEMVT
  return hipGetLastError();
}

}  // namespace pr
