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
#include "pr_device.h"

namespace pr {
namespace {
using namespace dev;

typedef double d2v_t __attribute__((ext_vector_type(2)));
typedef double d4v_t __attribute__((ext_vector_type(4)));
typedef unsigned short us4_t __attribute__((ext_vector_type(4)));

// C[z][r][c] = sum_{k in split z} A[c][k] * B[r][k], A BF16 (upcast exactly),
// B FP64, FP64 MFMA.  Block = 4 waves, block tile 128 (c) x 64 (r), wave tile
// 64 x 32 = 4 x 2 MFMA tiles of 16 x 16.  Within a reduction step of 16 the
// lanes of quarter q take the 4 consecutive indices 4q..4q+3 (one 8-byte A load,
// one 32-byte B load per tile) and MFMA s combines index 4q+s of every quarter.
//
// Row compaction: with rowmap != NULL only the first *nrow rows are computed,
// local row l reading B row rowmap[l] and writing C row rowmap[l]; r tiles
// past *nrow exit at once.  Rows of finished nodes thus cost nothing.
// The split count may also come from the device (ksp != NULL): the grid is
// sized for the largest count and the groups past MT * (*ksp) exit.
__global__ __launch_bounds__(256) void k_gemm_f64(const uint16_t *__restrict__ A, int64_t lda,
                                                  const double *__restrict__ B, int64_t ldb, double *__restrict__ C,
                                                  int64_t Mc, int64_t Nr, int64_t K, int MT, int NT, int KS,
                                                  const int32_t *__restrict__ active,
                                                  const int32_t *__restrict__ rowmap,
                                                  const int32_t *__restrict__ nrow,
                                                  const int32_t *__restrict__ ksp) {
  if (active && *active == 0) return;
  if (ksp) KS = *ksp;
  const int64_t Kc = K / KS;
  const int b = blockIdx.x;
  const int x = b & 7, qq = b >> 3;
  const int g = qq / NT, nt = qq - g * NT;
  const int G = g * 8 + x;
  if (G >= MT * KS) return;
  const int mt = G % MT, z = G / MT;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = lane >> 4, rr = lane & 15;
  const int64_t c0 = (int64_t)mt * 128 + (w & 1) * 64;
  const int64_t r0 = (int64_t)nt * 64 + (w >> 1) * 32;
  const int64_t k0 = (int64_t)z * Kc + 4 * q;
  // B row of each of the lane's two r positions, and the C row it is stored
  // to (-1: past the compacted rows, read a valid row and store nothing)
  int64_t brow[2], orow[2];
  if (rowmap) {
    const int nr = *nrow;
    if ((int64_t)nt * 64 >= nr) return;  // so nr >= 1 below
#pragma unroll
    for (int u = 0; u < 2; u++) {
      const int64_t l = r0 + 16 * u + rr;
      orow[u] = l < nr ? rowmap[l] : -1;
      brow[u] = l < nr ? orow[u] : rowmap[0];
    }
  } else {
#pragma unroll
    for (int u = 0; u < 2; u++) orow[u] = brow[u] = r0 + 16 * u + rr;
  }
  const uint16_t *pa[4];
  const double *pb[2];
#pragma unroll
  for (int t = 0; t < 4; t++) pa[t] = A + (c0 + 16 * t + rr) * lda + k0;
#pragma unroll
  for (int u = 0; u < 2; u++) pb[u] = B + brow[u] * ldb + k0;
  d4v_t acc[4][2];
#pragma unroll
  for (int t = 0; t < 4; t++)
#pragma unroll
    for (int u = 0; u < 2; u++) acc[t][u] = d4v_t{0.0, 0.0, 0.0, 0.0};
  for (int64_t kk = 0; kk < Kc; kk += 16) {
    us4_t ar[4];
    d2v_t br[2][2];
#pragma unroll
    for (int t = 0; t < 4; t++) ar[t] = *reinterpret_cast<const us4_t *>(pa[t] + kk);
#pragma unroll
    for (int u = 0; u < 2; u++) {
      br[u][0] = *reinterpret_cast<const d2v_t *>(pb[u] + kk);
      br[u][1] = *reinterpret_cast<const d2v_t *>(pb[u] + kk + 2);
    }
#pragma unroll
    for (int s4 = 0; s4 < 4; s4++) {
      double av[4], bv[2];
#pragma unroll
      for (int t = 0; t < 4; t++) av[t] = (double)__uint_as_float(((unsigned int)ar[t][s4]) << 16);
#pragma unroll
      for (int u = 0; u < 2; u++) bv[u] = br[u][s4 >> 1][s4 & 1];
#pragma unroll
      for (int t = 0; t < 4; t++)
#pragma unroll
        for (int u = 0; u < 2; u++) acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], bv[u], acc[t][u], 0, 0, 0);
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

// Compacted row list of the batch: rowmap[0..nrow) = the slots of the nodes
// that are still iterating, in increasing order, and the reduction split of
// each GEMM for this iteration: the base split times the largest power of two
// f <= min(fmax, NT / ceil(nrow / 64)), so the number of busy workgroups stays
// near that of the full batch.  sp = {nrow, forward split, transpose split}.
// One block of 256 threads.
__global__ __launch_bounds__(256) void k_batch_rowmap(const NodeState *__restrict__ S, int m,
                                                      int32_t *__restrict__ rowmap, int32_t *__restrict__ sp,
                                                      int NT, int ksf, int fmaxf, int kst, int fmaxt) {
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
    if (act) rowmap[off + before] = i;
    __syncthreads();
    if (threadIdx.x == 0) base += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int nta = (base + 63) / 64;
    const int room = nta > 0 ? NT / nta : 1;
    int ff = 1, ft = 1;
    while (2 * ff <= fmaxf && 2 * ff <= room) ff *= 2;
    while (2 * ft <= fmaxt && 2 * ft <= room) ft *= 2;
    sp[0] = base;
    sp[1] = ksf * ff;
    sp[2] = kst * ft;
  }
}

// Row-major copy of a column-major BF16 matrix (n x p): out[i][j] = in[j][i].
__global__ __launch_bounds__(256) void k_transpose_bf16(const uint16_t *__restrict__ in, uint16_t *__restrict__ out,
                                                        int64_t n, int64_t p) {
  __shared__ uint16_t tile[64][65];
  const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int jj = ty; jj < 64; jj += 4) {
    const int64_t i = i0 + tx, j = j0 + jj;
    tile[jj][tx] = (i < n && j < p) ? in[j * n + i] : (uint16_t)0;
  }
  __syncthreads();
  for (int ii = ty; ii < 64; ii += 4) {
    const int64_t i = i0 + ii, j = j0 + tx;
    if (i < n && j < p) out[i * p + j] = tile[tx][ii];
  }
}


// Residuals of the batch: u_i = sum_z U[z][i] (FP64), r_i = y - u_i into row i
// of R ([Nr][n], FP64), and per (node, row block) sums of r^2 and
// 2 r^T y - r^T r.  grid = (ceil(n / 512), m); 2 rows per thread.
__global__ __launch_bounds__(256) void k_batch_resid(const double *__restrict__ U, const int32_t *__restrict__ ksp,
                                                     int64_t n, int Nr, const double *__restrict__ y,
                                                     double *__restrict__ R, double *__restrict__ fsum,
                                                     const NodeState *S) {
  __shared__ double red[4 * 4];
  const int node = blockIdx.y;
  if (S[node].done) return;
  const int KSF = *ksp;
  const int64_t i0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 2;
  const int64_t plane = (int64_t)Nr * n;
  double s[2] = {0.0, 0.0};
  if (i0 < n) {
#pragma unroll
    for (int e = 0; e < 2; e++) {
      const int64_t i = i0 + e;
      double u = 0.0;
      for (int z = 0; z < KSF; z++) u += U[(int64_t)z * plane + (int64_t)node * n + i];
      const double ri = y[i] - u;
      R[(int64_t)node * n + i] = ri;
      s[0] += ri * ri;
      s[1] += 2.0 * ri * y[i] - ri * ri;
    }
  }
  block_sum<256, 2>(s, red);
  if (threadIdx.x == 0) {
    fsum[2 * ((int64_t)node * gridDim.x + blockIdx.x)] = s[0];
    fsum[2 * ((int64_t)node * gridDim.x + blockIdx.x) + 1] = s[1];
  }
}

// zeta = 2 r of one node from its last residual row (certification input).
__global__ void k_batch_zeta(const double *__restrict__ R, int64_t n, int node, double *__restrict__ zeta) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    zeta[i] = 2.0 * R[(int64_t)node * n + i];
}

}  // namespace

hipError_t launch_gemm_f64(const uint16_t *A, int64_t lda, const double *B, int64_t ldb, double *C, int64_t Mc,
                           int64_t Nr, int64_t K, int KS, const int32_t *active, const int32_t *rowmap,
                           const int32_t *nrow, const int32_t *ksp, int ks_max, hipStream_t s) {
  const int MT = (int)(Mc / 128), NT = (int)(Nr / 64);
  const int groups = MT * (ksp ? ks_max : KS);
  const int gpad = (groups + 7) / 8 * 8;
  k_gemm_f64<<<(unsigned)(gpad * NT), 256, 0, s>>>(A, lda, B, ldb, C, Mc, Nr, K, MT, NT, KS, active, rowmap, nrow,
                                                    ksp);
  return hipGetLastError();
}

hipError_t launch_batch_rowmap(const NodeState *S, int m, int32_t *rowmap, int32_t *sp, int ksf, int fmaxf, int kst,
                               int fmaxt, hipStream_t s) {
  const int NT = (m + 63) / 64;
  k_batch_rowmap<<<1, 256, 0, s>>>(S, m, rowmap, sp, NT, ksf, fmaxf, kst, fmaxt);
  return hipGetLastError();
}

hipError_t launch_transpose_bf16(const uint16_t *in, uint16_t *out, int64_t n, int64_t p, hipStream_t s) {
  dim3 grid((unsigned)((n + 63) / 64), (unsigned)((p + 63) / 64));
  k_transpose_bf16<<<grid, 256, 0, s>>>(in, out, n, p);
  return hipGetLastError();
}

int batch_resid_blocks(int64_t n) { return (int)((n + 511) / 512); }

hipError_t launch_batch_resid(const double *U, const int32_t *ksp, int64_t n, int m, int Nr, const double *y,
                              double *R, double *fsum, const NodeState *S, hipStream_t s) {
  dim3 grid((unsigned)batch_resid_blocks(n), (unsigned)m);
  k_batch_resid<<<grid, 256, 0, s>>>(U, ksp, n, Nr, y, R, fsum, S);
  return hipGetLastError();
}

hipError_t launch_batch_zeta(const double *R, int64_t n, int node, double *zeta, hipStream_t s) {
  k_batch_zeta<<<64, 256, 0, s>>>(R, n, node, zeta);
  return hipGetLastError();
}

}  // namespace pr
