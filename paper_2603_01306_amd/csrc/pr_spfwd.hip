// Column-list GEMV on gfx950: u = sum_t X[:, idx[t]] val[t] over the support
// of the iterate (or all columns), FP64 accumulation, followed by the loss
// epilogue of the solver.  Two kernels:
//
// k_spfwd_part  grid = row blocks x column chunks.  The list entries of a
//               chunk are wave-uniform, so column bases live in scalar
//               registers and every lane keeps 16 independent 16-byte
//               non-temporal loads in flight (2 to 8 rows per lane),
//               converted to FP64 at the FMA; the chunk's last columns form
//               one masked round of 16.  Writes its partial sums to
//               part[chunk][n].
// k_spfwd_final grid over rows: sums the chunk partials in chunk order (so the
//               result does not depend on scheduling) and runs the epilogue:
//   least squares: r = y - u, F = ||r||^2, -F*(-zeta) = 2 r^T y - ||r||^2;
//   logistic:      zeta = y sigma(-y u), F, binary entropies, and the gradient
//                  at the momentum point (1+m)u - m u_prev;
//   Gram (least squares with X^T X held in memory): the "matrix" is G = X^T X
//                  and y holds b = X^T y, so the kernel writes h = b - G x.
// Bytes per launch pair: |list| * n * sizeof(X) + 16 * nch * n (partials)
// + the epilogue vectors.
#include "pr_device.h"

namespace pr {
namespace {
using namespace dev;

constexpr int kSpInFlight = 16;   // columns in flight per lane
constexpr int kFinThreads = 128;  // 2 waves: twice the workgroups of 256, more CUs on the partial planes
constexpr int kFinRows = 2;       // rows per thread in the finalize kernel

// 16 raw bytes of X and their FP64 value e (exact upcast)
template <typename T>
struct XRaw;
template <>
struct XRaw<float> {
  static constexpr int VEC = 4;
  __device__ __forceinline__ static double at(const u4_t &r, int e) { return (double)__uint_as_float(r[e]); }
};
template <>
struct XRaw<double> {
  static constexpr int VEC = 2;
  __device__ __forceinline__ static double at(const u4_t &r, int e) {
    return __hiloint2double((int)r[2 * e + 1], (int)r[2 * e]);
  }
};
template <>
struct XRaw<uint16_t> {
  static constexpr int VEC = 8;
  __device__ __forceinline__ static double at(const u4_t &r, int e) {
    const unsigned int w = r[e >> 1];
    return (double)__uint_as_float((e & 1) ? (w & 0xffff0000u) : (w << 16));
  }
};

// The chunk's last, partial round of kSpInFlight column loads (16 bytes per
// lane each) for list entries t .. t1 - 1: the slots at or past t1 re-read
// the chunk's last column, which sp_use_r then weights by zero.
template <typename T>
__device__ __forceinline__ void sp_issue_tail(u4_t (&raw)[kSpInFlight], const T *__restrict__ X, int64_t n,
                                              int64_t row0, const int32_t *__restrict__ idx, int t, int t1) {
#pragma unroll
  for (int c = 0; c < kSpInFlight; c++) {
    const int tc = (t + c < t1) ? t + c : t1 - 1;
    const T *col = X + (int64_t)(idx[tc] & kIdxMask) * n;   // wave-uniform column base
    raw[c] = __builtin_nontemporal_load(reinterpret_cast<const u4_t *>(col + row0));
  }
}

template <typename T, bool FULL>
__device__ __forceinline__ void sp_use_r(const u4_t (&raw)[kSpInFlight], double (&acc)[XRaw<T>::VEC],
                                         const double *__restrict__ val, int t, int t1) {
#pragma unroll
  for (int c = 0; c < kSpInFlight; c++) {
    const double w = FULL ? val[t + c] : ((t + c < t1) ? val[t + c < t1 ? t + c : t1 - 1] : 0.0);
#pragma unroll
    for (int e = 0; e < XRaw<T>::VEC; e++) acc[e] = fma(XRaw<T>::at(raw[c], e), w, acc[e]);
  }
}

template <typename T>
__global__ __launch_bounds__(kSpThreads) void k_spfwd_part(const T *__restrict__ X, int64_t n, ProbBufs B,
                                                           const int32_t *__restrict__ idx,
                                                           const double *__restrict__ val,
                                                           const int32_t *__restrict__ nlist,
                                                           const NodeState *S) {
  constexpr int VEC = XRaw<T>::VEC;
  if (S && S->done) return;
  const int rb = blockIdx.x, ch = blockIdx.y;
  const int ns = *nlist;
  const int cs = (ns + B.nch - 1) / B.nch;
  const int t0 = ch * cs;
  const int t1 = (t0 + cs < ns) ? t0 + cs : ns;
  const int64_t row0 = (int64_t)rb * B.rows + (int64_t)threadIdx.x * VEC;
  if (row0 >= n) return;
  double acc[VEC];
#pragma unroll
  for (int e = 0; e < VEC; e++) acc[e] = 0.0;
  // full rounds of kSpInFlight columns, then the chunk's remaining columns as
  // one masked round (all its loads in flight together)
  int t = t0;
  if (t + kSpInFlight <= t1) {
    // the next round's column indices are loaded while this round's columns
    // stream, so a round does not start with a wait on its own indices
    // (root solves 0.7-0.9% faster; issuing the next round's column loads
    // ahead of this round's arithmetic from two load buffers gained nothing)
    int32_t ci[kSpInFlight];
#pragma unroll
    for (int c = 0; c < kSpInFlight; c++) ci[c] = idx[t + c];
    for (;;) {
      u4_t raw[kSpInFlight];
#pragma unroll
      for (int c = 0; c < kSpInFlight; c++)
        raw[c] = __builtin_nontemporal_load(
            reinterpret_cast<const u4_t *>(X + (int64_t)(ci[c] & kIdxMask) * n + row0));
      const int tn = t + kSpInFlight;
      const bool more = tn + kSpInFlight <= t1;
      if (more) {
#pragma unroll
        for (int c = 0; c < kSpInFlight; c++) ci[c] = idx[tn + c];
      }
      sp_use_r<T, true>(raw, acc, val, t, t1);
      t = tn;
      if (!more) break;
    }
  }
  if (t < t1) {
    u4_t raw[kSpInFlight];
    sp_issue_tail<T>(raw, X, n, row0, idx, t, t1);
    sp_use_r<T, false>(raw, acc, val, t, t1);
  }
  double *part = B.part + (int64_t)ch * n + row0;
#pragma unroll
  for (int e = 0; e < VEC; e += 2) *reinterpret_cast<d2_t *>(part + e) = d2_t{acc[e], acc[e + 1]};
}

__global__ __launch_bounds__(kFinThreads) void k_spfwd_final(int64_t n, const double *__restrict__ y, ProbBufs B,
                                                             int32_t mode, const NodeState *S, double *u_out) {
  constexpr int VEC = kFinRows;
  __shared__ double red[(kFinThreads / 64) * 4];
  if (S && S->done) return;
  const int fb = blockIdx.x;
  const int64_t row0 = ((int64_t)fb * kFinThreads + threadIdx.x) * VEC;
  const bool active = row0 < n;
  double u[VEC];
#pragma unroll
  for (int e = 0; e < VEC; e++) u[e] = 0.0;
  if (active) {
    const int nch = B.nch;
    int c = 0;
    for (; c + 8 <= nch; c += 8) {
      d2_t pv[8];
#pragma unroll
      for (int q = 0; q < 8; q++) pv[q] = *reinterpret_cast<const d2_t *>(B.part + (int64_t)(c + q) * n + row0);
#pragma unroll
      for (int q = 0; q < 8; q++) {
        u[0] += pv[q].x;
        u[1] += pv[q].y;
      }
    }
    for (; c < nch; c++) {
      const d2_t pv = *reinterpret_cast<const d2_t *>(B.part + (int64_t)c * n + row0);
      u[0] += pv.x;
      u[1] += pv.y;
    }
  }
  double sums[3] = {0.0, 0.0, 0.0};
  if (mode == kSpPlain) {
    if (active)
#pragma unroll
      for (int e = 0; e < VEC; e++) u_out[row0 + e] = u[e];
    return;
  }
  if (mode == kSpGram) {
    // the product is G x over the Gram matrix and y holds b = X^T y: h = b - G x
    if (active)
#pragma unroll
      for (int e = 0; e < VEC; e++) B.h1[row0 + e] = y[row0 + e] - u[e];
    return;
  }
  const int improved = S->improved;
  if (mode == kSpLsq) {
    // backtracking: X y of the pending trial as in the logistic branch below,
    // and its model-test remainder ||X x - X y||^2 row by row
    const int bt = S->bt, acc = S->bt_acc;
    const double mp = S->mom;
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
        if (bt) {
          const double uo = B.ucur[i];
          double uyv;
          if (acc) {
            uyv = (1.0 + mp) * uo - mp * B.uprev[i];
            B.uy[i] = uyv;
            B.uprev[i] = uo;
          } else {
            uyv = B.uy[i];
          }
          B.ucur[i] = u[e];
          const double du = u[e] - uyv;
          sums[2] += du * du;
        }
      }
    }
  } else {
    const double t = S->t;
    const double mt = (t - 1.0) / fista_next_t(t);
    // backtracking: uprev holds X x of the last accepted iterate; when the
    // previous evaluation was accepted it moves there and the momentum point
    // y of the pending trial, X y = (1 + m) X x_k - m X x_{k-1} (m the step's
    // momentum, 0 after a restart), is kept in uy until the trial is decided
    const int bt = S->bt, acc = S->bt_acc;
    const double mp = S->mom;
    if (active) {
#pragma unroll
      for (int e = 0; e < VEC; e++) {
        const int64_t i = row0 + e;
        const double uo = B.ucur[i];
        double up = uo;
        if (bt) {
          up = B.uprev[i];
          if (acc) {
            const double uyv = (1.0 + mp) * uo - mp * up;
            B.uy[i] = uyv;
            up = uo;
            B.uprev[i] = up;
          }
        } else {
          B.uprev[i] = uo;
        }
        B.ucur[i] = u[e];
        if (improved) B.zbest[i] = B.r[i];
        const double yi = y[i];
        const double z = yi * u[e];
        const double a = 1.0 / (1.0 + exp(z));
        B.r[i] = yi * a;
        sums[0] += softplus(-z);
        sums[1] += a * softplus(z) + (1.0 - a) * softplus(-z);
        if (bt) {
          // F(X x) - F(X y) - <grad F(X y), X x - X y> of this row, with
          // a = -y_i (X y)_i and d = -y_i (X x - X y)_i: log1p(s expm1(d)) - s d,
          // s = 1 / (1 + exp(-a))
          const double uyv = B.uy[i];
          const double aa = -yi * uyv, dd = -yi * (u[e] - uyv);
          const double sg = 1.0 / (1.0 + exp(-aa));
          sums[2] += log1p(sg * expm1(dd)) - sg * dd;
        }
        const double sm = (1.0 + mt) * u[e] - mt * up;
        B.gm[i] = -yi / (1.0 + exp(yi * sm));
      }
    }
  }
  block_sum<kFinThreads, 3>(sums, red);
  if (threadIdx.x == 0) {
    B.rbsum[2 * fb] = sums[0];
    B.rbsum[2 * fb + 1] = sums[1];
    if (B.dsum) B.dsum[fb] = sums[2];
  }
}

}  // namespace

hipError_t launch_spfwd(const Problem &P, const ProbBufs &B, const int32_t *idx, const double *val,
                        const int32_t *nlist, int32_t mode, const NodeState *S, double *u_out,
                        hipStream_t s) {
  dim3 grid((unsigned)B.rb, (unsigned)B.nch);
  dim3 block(kSpThreads);
  switch (P.xdt) {
    case kF32:
      k_spfwd_part<float><<<grid, block, 0, s>>>((const float *)P.X, P.n, B, idx, val, nlist, S);
      break;
    case kF64:
      k_spfwd_part<double><<<grid, block, 0, s>>>((const double *)P.X, P.n, B, idx, val, nlist, S);
      break;
    default:
      k_spfwd_part<uint16_t><<<grid, block, 0, s>>>((const uint16_t *)P.X, P.n, B, idx, val, nlist, S);
      break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_spfwd_final<<<(unsigned)B.nfin, kFinThreads, 0, s>>>(P.n, P.y, B, mode, S, u_out);
  return hipGetLastError();
}

int spfwd_final_blocks(int64_t n) { return (int)((n + kFinThreads * kFinRows - 1) / (kFinThreads * kFinRows)); }

}  // namespace pr
