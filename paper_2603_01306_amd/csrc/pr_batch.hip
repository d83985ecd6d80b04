// Batched node relaxations sharing X (BF16) on gfx950 MFMA.
//
// m nodes iterate together.  Both products of an iteration are GEMMs whose
// operands are contiguous along the reduction dimension:
//   forward   U (m x n) = Xit (m x p) . X_row^T   (X_row: row-major copy of X)
//   transpose H (m x p) = R (m x n) . X_col^T
// on FP64 MFMA (v_mfma_f64_16x16x4f64, BF16 X upcast exactly, FP64 iterates
// and residuals), so every node follows the single-node iteration with exact
// Phi and Psi.  FP32-accumulated BF16 products (even with the iterate split
// into BF16 hi + lo parts and FP64 flushes every 512 indices) leave an error of
// about eps_32 * sqrt(K) * |x||r| in every output; g_N* is not differentiable
// on the tied coordinates of the pooled block, so that error enters the duality
// gap at first order and the gap stalls near 1e-5, above the 1e-6 tolerance.
//
// Tile order is XCD-aware: consecutive block indices go round-robin over the 8
// XCDs, so block b is given the (c tile, split) group (b / 8 / NT) * 8 + b % 8
// and r tile (b / 8) % NT: the NT blocks sharing an A tile run on one XCD and
// read it from HBM once per XCD L2.
#include <type_traits>

#include "pr_device.h"

namespace pr {
namespace {
using namespace dev;

typedef double d2v_t __attribute__((ext_vector_type(2)));
typedef double d4v_t __attribute__((ext_vector_type(4)));
constexpr int kPipe = 2;       // reduction steps of operands held per wave in k_gemm_f64
constexpr int kGemmGrid = 512;   // persistent grid of k_gemm_f64: two workgroups per CU
typedef unsigned short us8_t __attribute__((ext_vector_type(8)));
typedef float f4v_t __attribute__((ext_vector_type(4)));

// Eight consecutive operand elements of one lane (one reduction step of a
// lane quarter), loaded with 16-byte loads and read back as FP64: BF16 bit
// patterns and FP32 values convert exactly.
template <typename T>
struct Lane8;
template <>
struct Lane8<uint16_t> {
  us8_t v;
  __device__ __forceinline__ void load(const uint16_t *p) { v = *reinterpret_cast<const us8_t *>(p); }
  __device__ __forceinline__ double get(int s) const { return (double)__uint_as_float(((unsigned int)v[s]) << 16); }
};
template <>
struct Lane8<float> {
  f4v_t v[2];
  __device__ __forceinline__ void load(const float *p) {
    v[0] = *reinterpret_cast<const f4v_t *>(p);
    v[1] = *reinterpret_cast<const f4v_t *>(p + 4);
  }
  __device__ __forceinline__ double get(int s) const { return (double)v[s >> 2][s & 3]; }
};
template <>
struct Lane8<double> {
  d2v_t v[4];
  __device__ __forceinline__ void load(const double *p) {
#pragma unroll
    for (int i = 0; i < 4; i++) v[i] = *reinterpret_cast<const d2v_t *>(p + 2 * i);
  }
  __device__ __forceinline__ double get(int s) const { return v[s >> 1][s & 1]; }
};

// C[z][r][c] = sum_{k in split z} A[c][k] * B[r][k] on FP64 MFMA, operands
// BF16 / FP32 / FP64 (converted exactly).  Block = 4 waves, block tile 128 (c)
// x 64 (r), wave tile 64 x 32 = 4 x 2 MFMA tiles of 16 x 16.  The reduction
// runs in steps of 32: the lanes of quarter q own the 8 consecutive indices
// 8q .. 8q+7 of a step (16-byte loads; a wave reads whole cache lines of each
// row over consecutive steps); MFMA s of the step combines index 8q + s of
// every quarter.  Operands are loaded PIPE - 1 steps ahead of the MFMAs.
template <typename TA, typename TB, int PIPE>
__device__ __forceinline__ void gemm_tile(const TA *__restrict__ A, int64_t lda, const TB *__restrict__ B,
                                          int64_t ldb, double *__restrict__ C, int64_t Mc, int64_t Nr, int64_t Kc,
                                          int mt, int z, int nt, int nr, const int32_t *__restrict__ rowmap) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = lane >> 4, rr = lane & 15;
  const int64_t c0 = (int64_t)mt * 128 + (w & 1) * 64;
  const int64_t r0 = (int64_t)nt * 64 + (w >> 1) * 32;
  const int64_t k0 = (int64_t)z * Kc + 8 * q;
  // B row of each of the lane's two r positions, and the C row it is stored
  // to (-1: past the compacted rows, read a valid row and store nothing)
  int64_t brow[2], orow[2];
#pragma unroll
  for (int u = 0; u < 2; u++) {
    const int64_t l = r0 + 16 * u + rr;
    if (rowmap) {
      orow[u] = l < nr ? rowmap[l] : -1;
      brow[u] = l < nr ? orow[u] : rowmap[0];
    } else {
      orow[u] = brow[u] = l;
    }
  }
  const TA *pa[4];
  const TB *pb[2];
#pragma unroll
  for (int t = 0; t < 4; t++) pa[t] = A + (c0 + 16 * t + rr) * lda + k0;
#pragma unroll
  for (int u = 0; u < 2; u++) pb[u] = B + brow[u] * ldb + k0;
  d4v_t acc[4][2];
#pragma unroll
  for (int t = 0; t < 4; t++)
#pragma unroll
    for (int u = 0; u < 2; u++) acc[t][u] = d4v_t{0.0, 0.0, 0.0, 0.0};
  const int64_t nsteps = Kc / 32;
  Lane8<TA> ar[PIPE][4];
  Lane8<TB> br[PIPE][2];
  auto load = [&](int64_t st, Lane8<TA>(&a)[4], Lane8<TB>(&bb)[2]) {
    const int64_t kk = st * 32;
#pragma unroll
    for (int t = 0; t < 4; t++) a[t].load(pa[t] + kk);
#pragma unroll
    for (int u = 0; u < 2; u++) bb[u].load(pb[u] + kk);
  };
  auto step = [&](const Lane8<TA>(&a)[4], const Lane8<TB>(&bb)[2]) {
#pragma unroll
    for (int s8 = 0; s8 < 8; s8++) {
      double av[4], bv[2];
#pragma unroll
      for (int t = 0; t < 4; t++) av[t] = a[t].get(s8);
#pragma unroll
      for (int u = 0; u < 2; u++) bv[u] = bb[u].get(s8);
#pragma unroll
      for (int t = 0; t < 4; t++)
#pragma unroll
        for (int u = 0; u < 2; u++) acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], bv[u], acc[t][u], 0, 0, 0);
    }
  };
#pragma unroll
  for (int d = 0; d < PIPE - 1; d++)
    if (d < nsteps) load(d, ar[d], br[d]);
  for (int64_t s0 = 0; s0 < nsteps; s0 += PIPE) {
#pragma unroll
    for (int d = 0; d < PIPE; d++) {
      const int64_t sp = s0 + d + PIPE - 1;
      if (PIPE > 1 && sp < nsteps) load(sp, ar[(d + PIPE - 1) % PIPE], br[(d + PIPE - 1) % PIPE]);
      if (s0 + d < nsteps) {
        if (PIPE == 1) load(s0 + d, ar[0], br[0]);
        step(ar[d], br[d]);
      }
    }
  }
  // MFMA output: register v of lane l is (c = 4v + l/16, r = l%16)
  double *Cz = C + (int64_t)z * Nr * Mc;
#pragma unroll
  for (int u = 0; u < 2; u++) {
    if (orow[u] < 0) continue;
#pragma unroll
    for (int t = 0; t < 4; t++)
#pragma unroll
      for (int v = 0; v < 4; v++) Cz[orow[u] * Mc + c0 + 16 * t + 4 * v + q] = acc[t][u][v];
  }
}

// The same block tile for FP64 A and B, staged through LDS.  With 8-byte
// operands the direct loads above fetch each A row twice and each B row twice
// per block (two waves share every row), which the per-CU load bandwidth
// cannot feed; here the block loads its 128 x 16 A and 64 x 16 B slices of a
// reduction step once (coalesced 16-byte loads, 8 threads per 128-byte row)
// into one of two LDS buffers while the MFMAs consume the other.  Rows are
// padded to 18 doubles against bank conflicts.  Lane quarter q owns reduction
// indices 4q .. 4q+3 of a step; MFMA j combines index 4q + j of every quarter.
constexpr int kLdsRow = 18;
constexpr int kLdsStage = (128 + 64) * kLdsRow;  // doubles per buffer

__device__ __forceinline__ void gemm_tile_f64_lds(const double *__restrict__ A, int64_t lda,
                                                  const double *__restrict__ B, int64_t ldb, double *__restrict__ C,
                                                  int64_t Mc, int64_t Nr, int64_t Kc, int mt, int z, int nt, int nr,
                                                  const int32_t *__restrict__ rowmap, double *lds) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int q = lane >> 4, rr = lane & 15;
  // cooperative loads: A chunk id = tid + 256 i (i < 4), B chunk id = tid + 256 i (i < 2);
  // row = id / 8, 16-byte part = id % 8
  const int part = tid & 7;
  const double *ga[4];
  const double *gbp[2];
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const int row = (tid >> 3) + 32 * i;
    ga[i] = A + ((int64_t)mt * 128 + row) * lda + (int64_t)z * Kc + 2 * part;
  }
#pragma unroll
  for (int i = 0; i < 2; i++) {
    const int row = (tid >> 3) + 32 * i;
    const int l = nt * 64 + row;
    const int64_t br = rowmap ? (l < nr ? rowmap[l] : rowmap[0]) : l;
    gbp[i] = B + br * ldb + (int64_t)z * Kc + 2 * part;
  }
  // C rows of the lane's two r positions (-1: past the compacted rows)
  const int64_t c0 = (int64_t)mt * 128 + (w & 1) * 64;
  const int lr0 = nt * 64 + (w >> 1) * 32;
  int64_t orow[2];
#pragma unroll
  for (int u = 0; u < 2; u++) {
    const int l = lr0 + 16 * u + rr;
    orow[u] = rowmap ? (l < nr ? rowmap[l] : -1) : l;
  }
  d4v_t acc[4][2];
#pragma unroll
  for (int t = 0; t < 4; t++)
#pragma unroll
    for (int u = 0; u < 2; u++) acc[t][u] = d4v_t{0.0, 0.0, 0.0, 0.0};
  const int64_t nsteps = Kc / 16;
  d2v_t ra[4], rb[2];
  auto gload = [&](int64_t st) {
#pragma unroll
    for (int i = 0; i < 4; i++) ra[i] = *reinterpret_cast<const d2v_t *>(ga[i] + st * 16);
#pragma unroll
    for (int i = 0; i < 2; i++) rb[i] = *reinterpret_cast<const d2v_t *>(gbp[i] + st * 16);
  };
  auto lstore = [&](double *buf) {
#pragma unroll
    for (int i = 0; i < 4; i++) *reinterpret_cast<d2v_t *>(buf + ((tid >> 3) + 32 * i) * kLdsRow + 2 * part) = ra[i];
#pragma unroll
    for (int i = 0; i < 2; i++)
      *reinterpret_cast<d2v_t *>(buf + (128 + (tid >> 3) + 32 * i) * kLdsRow + 2 * part) = rb[i];
  };
  gload(0);
  lstore(lds);
  __syncthreads();
  const int arow = (w & 1) * 64 + rr, brow = 128 + (w >> 1) * 32 + rr;
  for (int64_t st = 0; st < nsteps; st++) {
    double *cur = lds + (st & 1) * kLdsStage;
    if (st + 1 < nsteps) gload(st + 1);
    d4v_t fa[4], fb[2];
#pragma unroll
    for (int t = 0; t < 4; t++) fa[t] = *reinterpret_cast<const d4v_t *>(cur + (arow + 16 * t) * kLdsRow + 4 * q);
#pragma unroll
    for (int u = 0; u < 2; u++) fb[u] = *reinterpret_cast<const d4v_t *>(cur + (brow + 16 * u) * kLdsRow + 4 * q);
#pragma unroll
    for (int j = 0; j < 4; j++)
#pragma unroll
      for (int t = 0; t < 4; t++)
#pragma unroll
        for (int u = 0; u < 2; u++)
          acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[t][j], fb[u][j], acc[t][u], 0, 0, 0);
    if (st + 1 < nsteps) lstore(lds + ((st + 1) & 1) * kLdsStage);
    __syncthreads();
  }
  double *Cz = C + (int64_t)z * Nr * Mc;
#pragma unroll
  for (int u = 0; u < 2; u++) {
    if (orow[u] < 0) continue;
#pragma unroll
    for (int t = 0; t < 4; t++)
#pragma unroll
      for (int v = 0; v < 4; v++) Cz[orow[u] * Mc + c0 + 16 * t + 4 * v + q] = acc[t][u][v];
  }
}

// W[q][j] = scale * sum over the KS split planes of C[z][rs q][j] (row rs q,
// q < m, of a batched product written as [KS][Nr][p] partial planes; rs rows
// per node), planes summed in order.
__global__ void k_sum_planes(const double *__restrict__ C, int KS, int Nr, int rs, int64_t p, int m, double scale,
                             double *__restrict__ W) {
  const int64_t total = (int64_t)m * p;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = t / p, j = t - q * p;
    double acc = 0.0;
    for (int z = 0; z < KS; z++) acc += C[((int64_t)z * Nr + rs * q) * p + j];
    W[t] = scale * acc;
  }
}

// Persistent launch: the grid (at most two workgroups per CU) walks the tile
// list.  Row compaction: with rowmap != NULL only the first *nrow rows are
// computed, local row l reading B row rowmap[l] and writing C row rowmap[l],
// so rows of finished nodes cost nothing.  The split count may come from the
// device (ksp != NULL).  Tile order is XCD-aware: consecutive workgroups go
// round-robin over the 8 XCDs, item i goes to workgroup i mod grid (a
// multiple of 8), and item i is (c tile, split) group (i / 8 / nta) * 8 + i % 8,
// r tile (i / 8) % nta: the r tiles sharing an A tile run on one XCD and read
// it from HBM once per XCD L2.
template <typename TA, typename TB, int PIPE>
__global__ __launch_bounds__(256, 2) void k_gemm_f64(const TA *__restrict__ A, int64_t lda, const TB *__restrict__ B,
                                                     int64_t ldb, double *__restrict__ C, int64_t Mc, int64_t Nr,
                                                     int64_t K, int MT, int NT, int KS,
                                                     const int32_t *__restrict__ active,
                                                     const int32_t *__restrict__ rowmap,
                                                     const int32_t *__restrict__ nrow,
                                                     const int32_t *__restrict__ ksp, int32_t *__restrict__ counter) {
  if (active && *active == 0) return;
  if (ksp) KS = *ksp;
  const int nr = rowmap ? *nrow : (int)Nr;
  const int nta = rowmap ? (nr + 63) / 64 : NT;
  const int groups = MT * KS;
  const int nitems = ((groups + 7) / 8) * 8 * nta;
  const int64_t Kc = K / KS;
  __shared__ int next;
  constexpr bool kLds = std::is_same<TA, double>::value && std::is_same<TB, double>::value;
  __shared__ double stage[kLds ? 2 * kLdsStage : 1];
  // items in order: the workgroup's own first item, then (with a counter)
  // whichever item is next when it finishes
  int item = blockIdx.x;
  while (item < nitems) {
    const int x = item & 7, qq = item >> 3;
    const int g = qq / nta, nt = qq - g * nta;
    const int G = g * 8 + x;
    if (G < groups) {
      if constexpr (std::is_same<TA, double>::value && std::is_same<TB, double>::value)
        gemm_tile_f64_lds(A, lda, B, ldb, C, Mc, Nr, Kc, G % MT, G / MT, nt, nr, rowmap, stage);
      else
        gemm_tile<TA, TB, PIPE>(A, lda, B, ldb, C, Mc, Nr, Kc, G % MT, G / MT, nt, nr, rowmap);
    }
    if (counter) {
      __syncthreads();
      if (threadIdx.x == 0) next = (int)gridDim.x + atomicAdd(counter, 1);
      __syncthreads();
      item = next;
    } else {
      item += gridDim.x;
    }
  }
}

// Compacted row list of the batch: rowmap[0..nrow) = the slots of the nodes
// that are still iterating, in increasing order, and the reduction split of
// each GEMM for this iteration: the base split times the factor the autotuner
// chose for this many active 64-row tiles (ftab[0][nta] for the forward
// product, ftab[trow][nta] for the product whose planes the node step reads:
// trow = 1 for X^T R, 2 for the Gram product G X_it).
// sp = {nrow, forward split, second split, split of the product compacted to
// kred of its kfull reduction indices}, sp[8] = rows of the second product:
// with rs = 2 (logistic: zeta and the gradient at the momentum point per
// node) rowmap2 lists rows 2 i and 2 i + 1 of every listed node i, and the
// second product's split is looked up for its own row-tile count; the two
// tile counters of the GEMMs are reset.  One block of 256 threads.
__global__ __launch_bounds__(256) void k_batch_rowmap(const NodeState *__restrict__ S, int m,
                                                      int32_t *__restrict__ rowmap, int32_t *__restrict__ sp,
                                                      int32_t *__restrict__ counters, const int32_t *__restrict__ ftab,
                                                      int ksf, int kst, int trow, int64_t kred, int64_t kfull,
                                                      int rs, int32_t *__restrict__ rowmap2) {
  __shared__ int base;
  __shared__ int wsum[4];
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i0 = 0; i0 < m; i0 += 256) {
    const int i = i0 + (int)threadIdx.x;
    const bool act = i < m && !S[i].done;
    const unsigned long long bal = __ballot(act);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[w] = __popcll(bal);
    __syncthreads();
    int off = base;
    for (int v = 0; v < w; v++) off += wsum[v];
    if (act) {
      rowmap[off + before] = i;
      if (rs == 2) {
        rowmap2[2 * (off + before)] = 2 * i;
        rowmap2[2 * (off + before) + 1] = 2 * i + 1;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) base += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int nta = (base + 63) / 64;
    if (nta >= kTuneMax) nta = kTuneMax - 1;
    int nta2 = (rs * base + 63) / 64;
    if (nta2 >= kTuneMax) nta2 = kTuneMax - 1;
    sp[0] = base;
    sp[1] = ksf * ftab[nta];
    sp[2] = kst * ftab[trow * kTuneMax + nta2];
    sp[8] = rs * base;
    // split of the compacted product over kred < kfull reduction indices: the
    // tuned split scaled by kred / kfull, rounded down to a power of two (>= 1)
    const int base = trow == 2 ? sp[2] : sp[1];  // the Gram product, else the forward product
    int ks3 = 1;
    while (2 * ks3 <= (int)(((int64_t)base * kred) / kfull)) ks3 *= 2;
    sp[3] = ks3;
    counters[0] = 0;
    counters[1] = 0;
  }
}

// Row-major copy of a column-major matrix (n x p): out[i][j] = in[j][i].
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const T *__restrict__ in, T *__restrict__ out, int64_t n,
                                                   int64_t p) {
  __shared__ T tile[64][65];
  const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int jj = ty; jj < 64; jj += 4) {
    const int64_t i = i0 + tx, j = j0 + jj;
    tile[jj][tx] = (i < n && j < p) ? in[j * n + i] : (T)0;
  }
  __syncthreads();
  for (int ii = ty; ii < 64; ii += 4) {
    const int64_t i = i0 + ii, j = j0 + tx;
    if (i < n && j < p) out[i * p + j] = tile[tx][ii];
  }
}


// Loss side of the batch from the forward product's split planes, u_i =
// sum_z U[z][node][i] in plane order (FP64), per (node, row block) sums of
// F(u) and -F*(-zeta).  grid = (ceil(n / 512), m); 2 rows per thread.
//   least squares: r = y - u into row node of R ([Nr][n]); sums of r^2 and
//                  2 r^T y - r^T r (zeta = 2 r).
//   logistic:      zeta = y / (1 + exp(y u)) (= -grad F(u)) into row 2 node of
//                  R ([2 Nr][n]); while iterating (S != NULL) also the
//                  gradient of F at the momentum point (1 + m) u - m u_prev,
//                  m the node's non-restart FISTA coefficient, into row
//                  2 node + 1, and u into Uprev for the next iteration; sums
//                  of sum_i log(1 + exp(-y_i u_i)) and the binary entropies
//                  of a_i = 1 / (1 + exp(y_i u_i)).
//                  Backtracking nodes keep X x of the last evaluation (Ucur),
//                  of the last accepted iterate (Uprev) and of the pending
//                  trial's momentum point (Uy, formed when the last evaluation
//                  was accepted), and sum the row-wise Bregman remainder of F
//                  between u and X y per block into dsum.
__global__ __launch_bounds__(256) void k_batch_resid(const double *__restrict__ U, const int32_t *__restrict__ ksp,
                                                     int64_t n, int Nr, const double *__restrict__ y,
                                                     double *__restrict__ R, double *__restrict__ fsum,
                                                     const NodeState *S, int32_t loss, double *__restrict__ Uprev,
                                                     double *__restrict__ Ucur, double *__restrict__ Uy,
                                                     double *__restrict__ dsum) {
  __shared__ double red[4 * 4];
  const int node = blockIdx.y;
  if (S && S[node].done) return;  // S == NULL: every row (certification)
  const int KSF = *ksp;
  const int64_t i0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 2;
  const int64_t plane = (int64_t)Nr * n;
  double s[3] = {0.0, 0.0, 0.0};
  if (i0 < n) {
    double u[2];
#pragma unroll
    for (int e = 0; e < 2; e++) {
      const int64_t i = i0 + e;
      u[e] = 0.0;
      for (int z = 0; z < KSF; z++) u[e] += U[(int64_t)z * plane + (int64_t)node * n + i];
    }
    if (loss == kLsq) {
#pragma unroll
      for (int e = 0; e < 2; e++) {
        const int64_t i = i0 + e;
        const double ri = y[i] - u[e];
        R[(int64_t)node * n + i] = ri;
        s[0] += ri * ri;
        s[1] += 2.0 * ri * y[i] - ri * ri;
      }
    } else {
      double mt = 0.0, mp = 0.0;
      int bt = 0, acc = 0;
      if (S) {
        const double t = S[node].t;
        mt = (t - 1.0) / fista_next_t(t);
        bt = S[node].bt;
        acc = S[node].bt_acc;
        mp = S[node].mom;
      }
      double *zr = R + (int64_t)(2 * node) * n, *gr = zr + n;
      double *up = Uprev + (int64_t)node * n;
#pragma unroll
      for (int e = 0; e < 2; e++) {
        const int64_t i = i0 + e;
        const double yi = y[i];
        const double z = yi * u[e];
        const double a = 1.0 / (1.0 + exp(z));
        zr[i] = yi * a;
        s[0] += softplus(-z);
        s[1] += a * softplus(z) + (1.0 - a) * softplus(-z);
        if (S && bt) {
          const int64_t ni = (int64_t)node * n + i;
          const double uc = Ucur[ni];
          double ua = up[i], uyv;
          if (acc) {
            uyv = (1.0 + mp) * uc - mp * ua;
            Uy[ni] = uyv;
            ua = uc;
            up[i] = ua;
          } else {
            uyv = Uy[ni];
          }
          Ucur[ni] = u[e];
          const double aa = -yi * uyv, dd = -yi * (u[e] - uyv);
          const double sg = 1.0 / (1.0 + exp(-aa));
          s[2] += log1p(sg * expm1(dd)) - sg * dd;
          const double sm = (1.0 + mt) * u[e] - mt * ua;
          gr[i] = -yi / (1.0 + exp(yi * sm));
        } else if (S) {
          const double uo = up[i];
          up[i] = u[e];
          const double sm = (1.0 + mt) * u[e] - mt * uo;
          gr[i] = -yi / (1.0 + exp(yi * sm));
        }
      }
    }
  }
  block_sum<256, 3>(s, red);
  if (threadIdx.x == 0) {
    fsum[2 * ((int64_t)node * gridDim.x + blockIdx.x)] = s[0];
    fsum[2 * ((int64_t)node * gridDim.x + blockIdx.x) + 1] = s[1];
    if (dsum) dsum[(int64_t)node * gridDim.x + blockIdx.x] = s[2];
  }
}

// zeta = 2 r of one node from its last residual row (certification input).
__global__ void k_batch_zeta(const double *__restrict__ R, int64_t n, int node, double *__restrict__ zeta) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    zeta[i] = 2.0 * R[(int64_t)node * n + i];
}


// ---- Support-union compaction of the batch's product with the iterates -------
// The iterates of a batch are sparse and their supports overlap, so after the
// first iterations the union U of the supports covers only part of the p
// coordinates.  Then G X_it = G[:, U] X_it[U, :] (Gram mode) and X_it X^T =
// X_it[:, U] X[:, U]^T (products over X), each plus the few nonzeros outside
// U, and the GEMM runs over |U| (padded) reduction indices instead of p.

// mask[j] = 1 where some row of Bx (m rows of length p) is nonzero; mask is
// cleared beforehand.  Every writer stores the same value.
__global__ __launch_bounds__(256) void k_union_mask(const double *__restrict__ Bx, int64_t p,
                                                    int32_t *__restrict__ mask) {
  const double *row = Bx + (int64_t)blockIdx.x * p;
  for (int64_t j = threadIdx.x; j < p; j += 256)
    if (row[j] != 0.0) mask[j] = 1;
}

// AU[c][q] = A[c][ulist[q]] for q < ku, 0 for ku <= q < kp, for the rows c
// of a row-major A with p columns (G, or the row-major copy of X).
template <typename T>
__global__ __launch_bounds__(256) void k_gather_cols(const T *__restrict__ A, int64_t p,
                                                     const int32_t *__restrict__ ulist, int64_t ku, int64_t kp,
                                                     T *__restrict__ AU) {
  const int64_t c = blockIdx.x;
  const T *row = A + c * p;
  T *out = AU + c * kp;
  for (int64_t q = threadIdx.x; q < kp; q += 256) out[q] = q < ku ? row[ulist[q]] : (T)0;
}

// For the first *nrow compacted rows (node = rowmap[r]): BxU[node][q] =
// Bx[node][ulist[q]] (0 past ku), and the nonzeros of the node's row outside
// the union (olist, no entries) listed in oidx / oval[node][...] with their
// count in ocnt[node].
__global__ __launch_bounds__(256) void k_union_compact(const double *__restrict__ Bx, int64_t p,
                                                       const int32_t *__restrict__ rowmap,
                                                       const int32_t *__restrict__ nrow,
                                                       const int32_t *__restrict__ ulist, int64_t ku, int64_t kp,
                                                       const int32_t *__restrict__ olist, int64_t no,
                                                       double *__restrict__ BxU, int32_t *__restrict__ ocnt,
                                                       int32_t *__restrict__ oidx, double *__restrict__ oval,
                                                       const int32_t *__restrict__ active) {
  if (active && *active == 0) return;
  if ((int)blockIdx.x >= *nrow) return;
  __shared__ int cnt;
  const int64_t node = rowmap[blockIdx.x];
  const double *row = Bx + node * p;
  double *out = BxU + node * kp;
  for (int64_t q = threadIdx.x; q < kp; q += 256) out[q] = q < ku ? row[ulist[q]] : 0.0;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int64_t t = threadIdx.x; t < no; t += 256) {
    const int32_t j = olist[t];
    const double v = row[j];
    if (v != 0.0) {
      const int slot = atomicAdd(&cnt, 1);  // LDS counter
      oidx[node * p + slot] = j;
      oval[node * p + slot] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) ocnt[node] = cnt;
}

// Plane 0 of the product, row node = rowmap[r]: C[node][c] += sum over the
// node's nonzeros x_j outside the union of column j of the matrix (length L:
// column j of the symmetric G, or of the column-major X; BF16 upcast
// exactly), read contiguously.  grid = (rows, L / kFixSpan): a workgroup
// covers kFixSpan output entries, thread i the 8 consecutive entries
// c0 + 8 i .. c0 + 8 i + 7 (one or four 16-byte loads per column), four
// columns in flight.  Nothing to do for most rows.  L is a multiple of 8.
constexpr int kFixSpan = 2048;
template <typename T>
struct Fix8;
template <>
struct Fix8<double> {
  d2v_t v[4];
  __device__ __forceinline__ void load(const double *p) {
#pragma unroll
    for (int i = 0; i < 4; i++) v[i] = *reinterpret_cast<const d2v_t *>(p + 2 * i);
  }
  __device__ __forceinline__ double get(int e) const { return v[e >> 1][e & 1]; }
};
template <>
struct Fix8<float> {
  f4v_t v[2];
  __device__ __forceinline__ void load(const float *p) {
    v[0] = *reinterpret_cast<const f4v_t *>(p);
    v[1] = *reinterpret_cast<const f4v_t *>(p + 4);
  }
  __device__ __forceinline__ double get(int e) const { return (double)v[e >> 2][e & 3]; }
};
template <>
struct Fix8<uint16_t> {
  us8_t v;
  __device__ __forceinline__ void load(const uint16_t *p) { v = *reinterpret_cast<const us8_t *>(p); }
  __device__ __forceinline__ double get(int e) const { return (double)__uint_as_float(((unsigned int)v[e]) << 16); }
};
template <typename T>
__global__ __launch_bounds__(256) void k_union_fix(const T *__restrict__ Mat, int64_t L, int64_t p,
                                                   const int32_t *__restrict__ rowmap,
                                                   const int32_t *__restrict__ nrow,
                                                   const int32_t *__restrict__ ocnt,
                                                   const int32_t *__restrict__ oidx, const double *__restrict__ oval,
                                                   double *__restrict__ C, const int32_t *__restrict__ active) {
  if (active && *active == 0) return;
  if ((int)blockIdx.x >= *nrow) return;
  const int64_t node = rowmap[blockIdx.x];
  const int cnt = ocnt[node];
  if (cnt == 0) return;
  const int64_t c = (int64_t)blockIdx.y * kFixSpan + 8 * (int64_t)threadIdx.x;
  if (c >= L) return;
  const int32_t *ix = oidx + node * p;
  const double *vx = oval + node * p;
  double acc[8];
#pragma unroll
  for (int e = 0; e < 8; e++) acc[e] = 0.0;
  int t = 0;
  for (; t + 4 <= cnt; t += 4) {
    Fix8<T> g[4];
#pragma unroll
    for (int u = 0; u < 4; u++) g[u].load(Mat + (int64_t)ix[t + u] * L + c);
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const double v = vx[t + u];
#pragma unroll
      for (int e = 0; e < 8; e++) acc[e] = fma(g[u].get(e), v, acc[e]);
    }
  }
  for (; t < cnt; t++) {
    Fix8<T> g;
    g.load(Mat + (int64_t)ix[t] * L + c);
    const double v = vx[t];
#pragma unroll
    for (int e = 0; e < 8; e++) acc[e] = fma(g.get(e), v, acc[e]);
  }
  double *crow = C + node * L + c;
#pragma unroll
  for (int e = 0; e < 8; e++) crow[e] += acc[e];
}

}  // namespace

template <typename TA, typename TB, int PIPE>
hipError_t launch_gemm_t(const TA *A, int64_t lda, const TB *B, int64_t ldb, double *C, int64_t Mc, int64_t Nr,
                         int64_t K, int KS, const int32_t *active, const int32_t *rowmap, const int32_t *nrow,
                         const int32_t *ksp, int ks_max, int32_t *counter, hipStream_t s) {
  const int MT = (int)(Mc / 128), NT = (int)(Nr / 64);
  const int groups = MT * (ksp ? ks_max : KS);
  const int items = (groups + 7) / 8 * 8 * NT;
  const int grid = items < kGemmGrid ? (items + 7) / 8 * 8 : kGemmGrid;
  k_gemm_f64<TA, TB, PIPE><<<(unsigned)grid, 256, 0, s>>>(A, lda, B, ldb, C, Mc, Nr, K, MT, NT, KS, active, rowmap,
                                                          nrow, ksp, counter);
  return hipGetLastError();
}

hipError_t launch_gemm_f64(const uint16_t *A, int64_t lda, const double *B, int64_t ldb, double *C, int64_t Mc,
                           int64_t Nr, int64_t K, int KS, const int32_t *active, const int32_t *rowmap,
                           const int32_t *nrow, const int32_t *ksp, int ks_max, int32_t *counter, hipStream_t s) {
  return launch_gemm_t<uint16_t, double, kPipe>(A, lda, B, ldb, C, Mc, Nr, K, KS, active, rowmap, nrow, ksp, ks_max,
                                                counter, s);
}

hipError_t launch_gemm_any(int adt, const void *A, int64_t lda, int bdt, const void *B, int64_t ldb, double *C,
                           int64_t Mc, int64_t Nr, int64_t K, int KS, const int32_t *active, const int32_t *rowmap,
                           const int32_t *nrow, const int32_t *ksp, int ks_max, int32_t *counter, hipStream_t s) {
#define PR_GEMM_CASE(A_T, B_T, PIPE_)                                                                              \
  return launch_gemm_t<A_T, B_T, PIPE_>((const A_T *)A, lda, (const B_T *)B, ldb, C, Mc, Nr, K, KS, active, rowmap, \
                                        nrow, ksp, ks_max, counter, s)
  if (adt == kBF16 && bdt == kF64) PR_GEMM_CASE(uint16_t, double, kPipe);
  if (adt == kF32 && bdt == kF64) PR_GEMM_CASE(float, double, kPipe);
  if (adt == kBF16 && bdt == kBF16) PR_GEMM_CASE(uint16_t, uint16_t, kPipe);
  if (adt == kF32 && bdt == kF32) PR_GEMM_CASE(float, float, kPipe);
  if (adt == kF64 && bdt == kF64) PR_GEMM_CASE(double, double, 1);  // two stages would spill
#undef PR_GEMM_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_batch_rowmap(const NodeState *S, int m, int32_t *rowmap, int32_t *sp, int32_t *counters,
                               const int32_t *ftab, int ksf, int kst, int trow, int64_t kred, int64_t kfull, int rs,
                               int32_t *rowmap2, hipStream_t s) {
  if (rs != 1 && rs != 2) return hipErrorInvalidValue;
  k_batch_rowmap<<<1, 256, 0, s>>>(S, m, rowmap, sp, counters, ftab, ksf, kst, trow, kred, kfull, rs, rowmap2);
  return hipGetLastError();
}

hipError_t launch_transpose(int xdt, const void *in, void *out, int64_t n, int64_t p, hipStream_t s) {
  dim3 grid((unsigned)((n + 63) / 64), (unsigned)((p + 63) / 64));
  switch (xdt) {
    case kF64: k_transpose<double><<<grid, 256, 0, s>>>((const double *)in, (double *)out, n, p); break;
    case kF32: k_transpose<float><<<grid, 256, 0, s>>>((const float *)in, (float *)out, n, p); break;
    case kBF16: k_transpose<uint16_t><<<grid, 256, 0, s>>>((const uint16_t *)in, (uint16_t *)out, n, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_union_mask(const double *Bx, int m, int64_t p, int32_t *mask, hipStream_t s) {
  k_union_mask<<<(unsigned)m, 256, 0, s>>>(Bx, p, mask);
  return hipGetLastError();
}

hipError_t launch_gather_cols(const double *G, int64_t p, const int32_t *ulist, int64_t ku, int64_t kp, double *GU,
                              hipStream_t s) {
  k_gather_cols<double><<<(unsigned)p, 256, 0, s>>>(G, p, ulist, ku, kp, GU);
  return hipGetLastError();
}

hipError_t launch_gather_cols_x(int xdt, const void *A, int64_t rows, int64_t p, const int32_t *ulist, int64_t ku,
                                int64_t kp, void *AU, hipStream_t s) {
  switch (xdt) {
    case kF64: k_gather_cols<double><<<(unsigned)rows, 256, 0, s>>>((const double *)A, p, ulist, ku, kp, (double *)AU);
      break;
    case kF32: k_gather_cols<float><<<(unsigned)rows, 256, 0, s>>>((const float *)A, p, ulist, ku, kp, (float *)AU);
      break;
    case kBF16:
      k_gather_cols<uint16_t><<<(unsigned)rows, 256, 0, s>>>((const uint16_t *)A, p, ulist, ku, kp, (uint16_t *)AU);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_union_compact(const double *Bx, int64_t p, const int32_t *rowmap, const int32_t *nrow, int Nr,
                                const int32_t *ulist, int64_t ku, int64_t kp, const int32_t *olist, int64_t no,
                                double *BxU, int32_t *ocnt, int32_t *oidx, double *oval, const int32_t *active,
                                hipStream_t s) {
  k_union_compact<<<(unsigned)Nr, 256, 0, s>>>(Bx, p, rowmap, nrow, ulist, ku, kp, olist, no, BxU, ocnt, oidx, oval,
                                               active);
  return hipGetLastError();
}

hipError_t launch_union_fix(const double *G, int64_t p, const int32_t *rowmap, const int32_t *nrow, int Nr,
                            const int32_t *ocnt, const int32_t *oidx, const double *oval, double *C,
                            const int32_t *active, hipStream_t s) {
  dim3 grid((unsigned)Nr, (unsigned)((p + kFixSpan - 1) / kFixSpan));
  k_union_fix<double><<<grid, 256, 0, s>>>(G, p, p, rowmap, nrow, ocnt, oidx, oval, C, active);
  return hipGetLastError();
}

hipError_t launch_union_fix_x(int xdt, const void *X, int64_t n, int64_t p, const int32_t *rowmap, const int32_t *nrow,
                              int Nr, const int32_t *ocnt, const int32_t *oidx, const double *oval, double *C,
                              const int32_t *active, hipStream_t s) {
  dim3 grid((unsigned)Nr, (unsigned)((n + kFixSpan - 1) / kFixSpan));
  switch (xdt) {
    case kF64:
      k_union_fix<double><<<grid, 256, 0, s>>>((const double *)X, n, p, rowmap, nrow, ocnt, oidx, oval, C, active);
      break;
    case kF32:
      k_union_fix<float><<<grid, 256, 0, s>>>((const float *)X, n, p, rowmap, nrow, ocnt, oidx, oval, C, active);
      break;
    case kBF16:
      k_union_fix<uint16_t><<<grid, 256, 0, s>>>((const uint16_t *)X, n, p, rowmap, nrow, ocnt, oidx, oval, C, active);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int batch_resid_blocks(int64_t n) { return (int)((n + 511) / 512); }

hipError_t launch_batch_resid(const double *U, const int32_t *ksp, int64_t n, int m, int Nr, const double *y,
                              double *R, double *fsum, const NodeState *S, int32_t loss, double *Uprev,
                              hipStream_t s, double *Ucur, double *Uy, double *dsum) {
  if (loss != kLsq && (loss != kLogistic || (S && !Uprev))) return hipErrorInvalidValue;
  dim3 grid((unsigned)batch_resid_blocks(n), (unsigned)m);
  k_batch_resid<<<grid, 256, 0, s>>>(U, ksp, n, Nr, y, R, fsum, S, loss, Uprev, Ucur, Uy, dsum);
  return hipGetLastError();
}

hipError_t launch_sum_planes(const double *C, int KS, int Nr, int rs, int64_t p, int m, double scale, double *W,
                             hipStream_t s) {
  const int64_t total = (int64_t)m * p;
  const int64_t blocks = (total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096;
  k_sum_planes<<<(unsigned)blocks, 256, 0, s>>>(C, KS, Nr, rs, p, m, scale, W);
  return hipGetLastError();
}

hipError_t launch_batch_zeta(const double *R, int64_t n, int node, double *zeta, hipStream_t s) {
  k_batch_zeta<<<64, 256, 0, s>>>(R, n, node, zeta);
  return hipGetLastError();
}

}  // namespace pr
