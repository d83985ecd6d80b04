// X^T r on gfx950: h = X^T r (one or two right-hand sides) for column-major X
// stored FP32 / BF16 / FP64, accumulated in FP64.
//
// One wave per C adjacent columns streams the full column length: each lane
// loads 16 bytes of every column per step with non-temporal loads (X is read
// once per launch and should not displace the L2-resident right-hand side),
// one row step per lane in flight (a measured sweep over 1, 2, 4 steps on
// MI355X favoured 1), then a deterministic in-wave transpose reduction leaves
// column c's total in lane (64 / C) c.  With one right-hand side, C = 2 (a
// sweep over 1, 2, 4, 8 columns per wave): twice the waves of C = 4, which the
// HBM stream needs to stay full.  With two, C = 8: every wave re-reads both
// right-hand sides from L2 for its columns, and at small C that L2 traffic
// (at C = 2 twice the bytes of X) becomes the limit (logistic 32768 x 16384:
// 585 / 537 / 504 / 498 us per iteration at C = 2 / 4 / 8 / 16; 16 needs 254
// VGPRs).  Algorithmic bytes per launch: n*p*sizeof(X) + 8n per right-hand
// side + 8p per output.
#include "pr_device.h"

namespace pr {
namespace {
using namespace dev;

constexpr int gemv_cols(int nrhs) { return nrhs == 1 ? 2 : 8; }

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

template <typename T, int NRHS>
__global__ __launch_bounds__(kGemvThreads) void k_gemv_t(const T *__restrict__ X, int64_t n, int64_t p,
                                                         const double *__restrict__ r1,
                                                         const double *__restrict__ r2,
                                                         double *__restrict__ h1,
                                                         double *__restrict__ h2,
                                                         const int32_t *__restrict__ done) {
  if (done && *done) return;
  constexpr int VEC = XLoad<T>::VEC;
#ifndef PR_GEMVT_STEPS
#define PR_GEMVT_STEPS 1
#endif
  constexpr int U = PR_GEMVT_STEPS;  // row steps in flight
  const int lane = lane_id();
  constexpr int C = gemv_cols(NRHS);
  const int64_t col0 = ((int64_t)blockIdx.x * (kGemvThreads / 64) + wave_id()) * C;
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
  for (; i + (U - 1) * step + VEC <= n; i += U * step) {
    double xv[U][C][VEC];
    double rv[U][NRHS][VEC];
#pragma unroll
    for (int u = 0; u < U; u++) {
#pragma unroll
      for (int q = 0; q < C; q++) XLoad<T>::load(c[q] + i + u * step, xv[u][q]);
      load_rhs<VEC>(r1, i + u * step, rv[u][0]);
      if (NRHS > 1) load_rhs<VEC>(r2, i + u * step, rv[u][NRHS - 1]);
    }
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
      for (int h = 0; h < NRHS; h++)
#pragma unroll
        for (int q = 0; q < C; q++)
#pragma unroll
          for (int e = 0; e < VEC; e++) acc[h][q] = fma(xv[u][q][e], rv[u][h][e], acc[h][q]);
  }
  for (; i + VEC <= n; i += step) {
    double xv[C][VEC];
    double rv[NRHS][VEC];
#pragma unroll
    for (int q = 0; q < C; q++) XLoad<T>::load(c[q] + i, xv[q]);
    load_rhs<VEC>(r1, i, rv[0]);
    if (NRHS > 1) load_rhs<VEC>(r2, i, rv[NRHS - 1]);
#pragma unroll
    for (int h = 0; h < NRHS; h++)
#pragma unroll
      for (int q = 0; q < C; q++)
#pragma unroll
        for (int e = 0; e < VEC; e++) acc[h][q] = fma(xv[q][e], rv[h][e], acc[h][q]);
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
                         const int32_t *done, hipStream_t s) {
  const bool two = (r2 != nullptr);
  const int cols_per_block = (kGemvThreads / 64) * gemv_cols(two ? 2 : 1);
  dim3 grid((unsigned)((P.p + cols_per_block - 1) / cols_per_block));
  dim3 block(kGemvThreads);
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

}  // namespace pr
