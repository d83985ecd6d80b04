// Learned warm start for child nodes: per-coordinate features, and the MLP
// 8 -> 64 -> 64 -> 1 (ReLU) on gfx950 BF16 MFMA (v_mfma_f32_32x32x16_bf16)
// with FP32 master parameters.  Not part of the paper's method: its output is
// only a candidate starting point that the FP64 duality gap accepts or rejects.
//
// Layout.  A wave takes 32 rows (coordinates) at a time and keeps every layer
// transposed, units x rows: Z1^T = W1 F^T, Z2^T = W2 A1^T, so the weights are
// the A operands (loaded once per wave) and the activations stay in the MFMA
// C layout, where register v of lane l holds unit 8(v/4) + 4(l/32) + v%4 of row
// l%32.  Turning a C tile into the B operand of the next product (lane l needs
// 8 consecutive units of row l%32) takes one exchange of 4 values between
// lanes l and l^32 per 16-unit step.  The weight gradients are products over
// rows (dW2 = dZ2^T A1, dW1 = dZ1^T F); their operands are transposed through
// LDS tiles of 64 units x 32 rows.  The bias gradient of layer 1 rides on a
// column of ones next to the 8 features in the dW1 product.
#include "pr_device.h"
#include "pr_internal.h"

namespace pr {
namespace {

constexpr int kH = 64, kNF = 8;
constexpr int OW1 = 0, OB1 = 512, OW2 = 576, OB2 = 4672, OW3 = 4736, OB3 = 4800;
constexpr int kNP = 4801;
constexpr int kWaves = 4;

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

// FP32 -> BF16, round to nearest even (one v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ unsigned short f2bf(float f) { return __builtin_bit_cast(unsigned short, (__bf16)f); }
__device__ __forceinline__ bf16x8_t as_bf(u16x8_t u) { return __builtin_bit_cast(bf16x8_t, u); }
__device__ __forceinline__ f32x16_t mma(bf16x8_t a, bf16x8_t b, f32x16_t c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
// unit (tile row) held in C register v by the lanes of half hh
__device__ __forceinline__ int crow(int v, int hh) { return 8 * (v >> 2) + 4 * hh + (v & 3); }

// B operand of the next product from a C-layout tile: units 16*S .. 16*S+15
// of the tile as the reduction index, the lane's row as the column.  Lane
// l < 32 holds units 16S + 0..3 (registers 8S + i) and 16S + 8..11 (8S + 4 + i)
// and needs 16S + 0..7; lane l + 32 holds 16S + 4..7 and 16S + 12..15 and
// needs 16S + 8..15.  One v_permlane32_swap per register pair exchanges the
// upper half of the first register with the lower half of the second.
template <int S>
__device__ __forceinline__ bf16x8_t b_from_c(const f32x16_t &c) {
  bf16x8_t r;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(c[8 * S + i]),
                                                     __float_as_uint(c[8 * S + 4 + i]), false, false);
    r[i] = (__bf16)__uint_as_float(sw[0]);
    r[4 + i] = (__bf16)__uint_as_float(sw[1]);
  }
  return r;
}

__device__ __forceinline__ bf16x8_t lds8(const unsigned short *p) {
  return as_bf(*reinterpret_cast<const u16x8_t *>(p));
}

// Forward (TRAIN = false: out[row] = network output) or forward + backward
// (TRAIN = true: block partial sums of the gradient of
// inv_n * sum_rows (out - T)^2 and of sum_rows (out - T)^2 into part[block]).
// Block = 4 waves; block b takes row chunks (b * cpb + it) * 4 + wave.
template <bool TRAIN>
__global__ __launch_bounds__(256) void k_mlp(const float *__restrict__ P, const uint16_t *__restrict__ F,
                                             const float *__restrict__ T, int64_t rows, int cpb, float inv_n,
                                             float *__restrict__ out, float *__restrict__ part) {
  __shared__ float sp[kNP];
  __shared__ __align__(16) unsigned short t_dz2[TRAIN ? kWaves : 1][kH * 32];
  __shared__ __align__(16) unsigned short t_a1[TRAIN ? kWaves : 1][kH * 32];
  __shared__ __align__(16) unsigned short t_dz1[TRAIN ? kWaves : 1][kH * 32];
  __shared__ __align__(16) unsigned short t_f[TRAIN ? kWaves : 1][16 * 32];
  for (int i = threadIdx.x; i < kNP; i += blockDim.x) sp[i] = P[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, hh = lane >> 5, lr = lane & 31;

  bf16x8_t aw1[2], aw2[2][4], aw2t[2][4];
#pragma unroll
  for (int u = 0; u < 2; u++) {
    u16x8_t t;
#pragma unroll
    for (int e = 0; e < 8; e++) t[e] = hh ? (unsigned short)0 : f2bf(sp[OW1 + (32 * u + lr) * kNF + e]);
    aw1[u] = as_bf(t);
  }
#pragma unroll
  for (int o = 0; o < 2; o++)
#pragma unroll
    for (int s = 0; s < 4; s++) {
      u16x8_t t, tt;
#pragma unroll
      for (int e = 0; e < 8; e++) {
        t[e] = f2bf(sp[OW2 + (32 * o + lr) * kH + 16 * s + 8 * hh + e]);
        tt[e] = f2bf(sp[OW2 + (16 * s + 8 * hh + e) * kH + 32 * o + lr]);
      }
      aw2[o][s] = as_bf(t);
      aw2t[o][s] = as_bf(tt);  // A operand of W2^T (tile o of its rows = input units)
    }
  const float b3 = sp[OB3];
  const f32x16_t zero = {};

  f32x16_t gW2[2][2] = {{zero, zero}, {zero, zero}}, gW1[2] = {zero, zero};
  float gb2[2][16], gw3[2][16], gb3 = 0.f, lsum = 0.f;
#pragma unroll
  for (int o = 0; o < 2; o++)
#pragma unroll
    for (int v = 0; v < 16; v++) gb2[o][v] = gw3[o][v] = 0.f;

  if (TRAIN && hh == 0) {
    // rows 8..15 of the transposed feature tile: a row of ones (bias of layer 1), zeros
#pragma unroll
    for (int e = 8; e < 16; e++) t_f[w][e * 32 + lr] = (e == 8) ? (unsigned short)0x3f80 : (unsigned short)0;
  }

  for (int it = 0; it < cpb; it++) {
    const int64_t row = (((int64_t)blockIdx.x * cpb + it) * kWaves + w) * 32 + lr;
    const bool valid = row < rows;
    u16x8_t fu = {0, 0, 0, 0, 0, 0, 0, 0};
    if (valid && hh == 0) fu = *reinterpret_cast<const u16x8_t *>(F + row * kNF);
    const bf16x8_t fb = as_bf(fu);
    f32x16_t a1[2];
#pragma unroll
    for (int u = 0; u < 2; u++) {
      a1[u] = mma(aw1[u], fb, zero);
#pragma unroll
      for (int v = 0; v < 16; v++) a1[u][v] = fmaxf(a1[u][v] + sp[OB1 + 32 * u + crow(v, hh)], 0.f);
    }
    f32x16_t a2[2] = {zero, zero};
    {
      const bf16x8_t b0 = b_from_c<0>(a1[0]), b1 = b_from_c<1>(a1[0]);
      const bf16x8_t b2 = b_from_c<0>(a1[1]), b3v = b_from_c<1>(a1[1]);
#pragma unroll
      for (int o = 0; o < 2; o++) {
        a2[o] = mma(aw2[o][0], b0, a2[o]);
        a2[o] = mma(aw2[o][1], b1, a2[o]);
        a2[o] = mma(aw2[o][2], b2, a2[o]);
        a2[o] = mma(aw2[o][3], b3v, a2[o]);
      }
    }
    float po = 0.f;
#pragma unroll
    for (int o = 0; o < 2; o++)
#pragma unroll
      for (int v = 0; v < 16; v++) {
        const int u = 32 * o + crow(v, hh);
        a2[o][v] = fmaxf(a2[o][v] + sp[OB2 + u], 0.f);
        po += sp[OW3 + u] * a2[o][v];
      }
    const float orow = po + __shfl_xor(po, 32) + b3;
    if (!TRAIN) {
      if (valid && hh == 0) out[row] = orow;
      continue;
    }
    const float d = valid ? orow - T[row] : 0.f;
    if (hh == 0) {
      lsum += d * d;
    }
    const float dout = 2.f * d * inv_n;
    if (hh == 0) gb3 += dout;
    f32x16_t dz2[2];
#pragma unroll
    for (int o = 0; o < 2; o++)
#pragma unroll
      for (int v = 0; v < 16; v++) {
        const int u = 32 * o + crow(v, hh);
        gw3[o][v] += a2[o][v] * dout;
        const float g = a2[o][v] > 0.f ? sp[OW3 + u] * dout : 0.f;
        dz2[o][v] = g;
        gb2[o][v] += g;
      }
    // dA1^T = W2^T dZ2^T, then the ReLU mask of layer 1
    f32x16_t dz1[2] = {zero, zero};
    {
      const bf16x8_t b0 = b_from_c<0>(dz2[0]), b1 = b_from_c<1>(dz2[0]);
      const bf16x8_t b2 = b_from_c<0>(dz2[1]), b3v = b_from_c<1>(dz2[1]);
#pragma unroll
      for (int i = 0; i < 2; i++) {
        dz1[i] = mma(aw2t[i][0], b0, dz1[i]);
        dz1[i] = mma(aw2t[i][1], b1, dz1[i]);
        dz1[i] = mma(aw2t[i][2], b2, dz1[i]);
        dz1[i] = mma(aw2t[i][3], b3v, dz1[i]);
      }
    }
    // transposed tiles for the products over rows
#pragma unroll
    for (int o = 0; o < 2; o++)
#pragma unroll
      for (int v = 0; v < 16; v++) {
        const int u = 32 * o + crow(v, hh);
        t_dz2[w][u * 32 + lr] = f2bf(dz2[o][v]);
        t_a1[w][u * 32 + lr] = f2bf(a1[o][v]);
        t_dz1[w][u * 32 + lr] = f2bf(a1[o][v] > 0.f ? dz1[o][v] : 0.f);
      }
    if (hh == 0) {
#pragma unroll
      for (int e = 0; e < 8; e++) t_f[w][e * 32 + lr] = fu[e];
    }
    __syncthreads();
#pragma unroll
    for (int s2 = 0; s2 < 2; s2++) {
      const int kofs = 16 * s2 + 8 * hh;
      bf16x8_t ad[2], ba[2], a1t[2];
#pragma unroll
      for (int q = 0; q < 2; q++) {
        ad[q] = lds8(&t_dz2[w][(32 * q + lr) * 32 + kofs]);
        ba[q] = lds8(&t_a1[w][(32 * q + lr) * 32 + kofs]);
        a1t[q] = lds8(&t_dz1[w][(32 * q + lr) * 32 + kofs]);
      }
      u16x8_t zf = {0, 0, 0, 0, 0, 0, 0, 0};
      const bf16x8_t bf = lr < 16 ? lds8(&t_f[w][lr * 32 + kofs]) : as_bf(zf);
#pragma unroll
      for (int o = 0; o < 2; o++)
#pragma unroll
        for (int i = 0; i < 2; i++) gW2[o][i] = mma(ad[o], ba[i], gW2[o][i]);
#pragma unroll
      for (int i = 0; i < 2; i++) gW1[i] = mma(a1t[i], bf, gW1[i]);
    }
    __syncthreads();
  }
  if (!TRAIN) return;

  // block reduction, wave by wave in a fixed order, into LDS (reusing sp)
  __syncthreads();
  for (int i = threadIdx.x; i < kNP; i += blockDim.x) sp[i] = 0.f;
  __syncthreads();
  float lsw = lsum, gb3w = gb3;
#pragma unroll
  for (int o = 0; o < 2; o++)
#pragma unroll
    for (int v = 0; v < 16; v++) {
      float x = gb2[o][v], y = gw3[o][v];
#pragma unroll
      for (int m = 1; m < 32; m <<= 1) {
        x += __shfl_xor(x, m);
        y += __shfl_xor(y, m);
      }
      gb2[o][v] = x;
      gw3[o][v] = y;
    }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    lsw += __shfl_xor(lsw, m);
    gb3w += __shfl_xor(gb3w, m);
  }
  __shared__ float lred[kWaves];
  for (int cur = 0; cur < kWaves; cur++) {
    if (w == cur) {
#pragma unroll
      for (int o = 0; o < 2; o++)
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
          for (int v = 0; v < 16; v++) sp[OW2 + (32 * o + crow(v, hh)) * kH + 32 * i + lr] += gW2[o][i][v];
      if (lr < kNF) {
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
          for (int v = 0; v < 16; v++) sp[OW1 + (32 * i + crow(v, hh)) * kNF + lr] += gW1[i][v];
      } else if (lr == kNF) {
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
          for (int v = 0; v < 16; v++) sp[OB1 + 32 * i + crow(v, hh)] += gW1[i][v];
      }
      if (lr == 0) {
#pragma unroll
        for (int o = 0; o < 2; o++)
#pragma unroll
          for (int v = 0; v < 16; v++) {
            sp[OB2 + 32 * o + crow(v, hh)] += gb2[o][v];
            sp[OW3 + 32 * o + crow(v, hh)] += gw3[o][v];
          }
      }
      if (lane == 0) {
        sp[OB3] += gb3w;
        lred[w] = lsw;
      }
    }
    __syncthreads();
  }
  float *dst = part + (int64_t)blockIdx.x * kMlpPartStride;
  for (int i = threadIdx.x; i < kNP; i += blockDim.x) dst[i] = sp[i];
  if (threadIdx.x == 0) dst[kNP] = ((lred[0] + lred[1]) + lred[2]) + lred[3];
}

// grad[i] = sum over blocks of part[b][i]; grad[kNP] = loss.  A workgroup
// owns 64 consecutive entries (one per lane) and its kRedWaves waves split
// the blocks into contiguous ranges: each wave adds its range in block order
// with the loads of 16 blocks issued together, then lane i of the first wave
// adds the wave totals in wave order, so the sum is fixed and reproducible.
// (One thread per entry walking all blocks left 76 waves on the chip, each
// waiting on nblk / 16 dependent memory round trips.)
constexpr int kRedWaves = 16;
__global__ __launch_bounds__(64 * kRedWaves) void k_mlp_reduce(const float *__restrict__ part, int nblk, float inv_n,
                                                               float *__restrict__ grad) {
  __shared__ float red[kRedWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const int b0 = (int)((int64_t)nblk * w / kRedWaves), b1 = (int)((int64_t)nblk * (w + 1) / kRedWaves);
  constexpr int kBatch = 16;
  float s = 0.f;
  if (i <= kNP) {
    int b = b0;
    for (; b + kBatch <= b1; b += kBatch) {
      float v[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; u++) v[u] = part[(int64_t)(b + u) * kMlpPartStride + i];
#pragma unroll
      for (int u = 0; u < kBatch; u++) s += v[u];
    }
    for (; b < b1; b++) s += part[(int64_t)b * kMlpPartStride + i];
  }
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && i <= kNP) {
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < kRedWaves; k++) t += red[k][lane];
    grad[i] = i == kNP ? t * inv_n : t;
  }
}

__global__ __launch_bounds__(256) void k_mlp_adam(float *__restrict__ P, const float *__restrict__ g,
                                                  float *__restrict__ m1, float *__restrict__ m2, float lr,
                                                  float beta1, float beta2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kNP) return;
  const float gi = g[i];
  const float m = beta1 * m1[i] + (1.f - beta1) * gi;
  const float v = beta2 * m2[i] + (1.f - beta2) * gi * gi;
  m1[i] = m;
  m2[i] = v;
  P[i] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

// Feature prologue of one node: max |w| and the nonzero magnitudes of beta,
// compacted in index order into nzv[0 .. nnz).  fs = {max |w|, nnz}.  One
// block of NT threads.
__global__ __launch_bounds__(dev::NT) void k_feat_prep(const double *__restrict__ beta, const double *__restrict__ w,
                                                       int64_t p, double *__restrict__ nzv, double *__restrict__ fs) {
  using namespace dev;
  __shared__ double red[NW];
  __shared__ int cnt[NW];
  __shared__ int64_t base;
  if (threadIdx.x == 0) base = 0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double hm = 0.0;
  for (int64_t j0 = 0; j0 < p; j0 += NT) {
    const int64_t j = j0 + threadIdx.x;
    double a = 0.0;
    if (j < p) {
      hm = fmax(hm, fabs(w[j]));
      a = fabs(beta[j]);
    }
    const bool nz = a != 0.0;
    const unsigned long long bal = __ballot(nz);
    if (lane == 0) cnt[wv] = __popcll(bal);
    __syncthreads();
    int64_t off = base;
    for (int v = 0; v < wv; v++) off += cnt[v];
    if (nz) nzv[off + __popcll(bal & ((1ull << lane) - 1ull))] = a;
    __syncthreads();
    if (threadIdx.x == 0)
      for (int v = 0; v < NW; v++) base += cnt[v];
    __syncthreads();
  }
  hm = block_max<NT>(hm, red);
  if (threadIdx.x == 0) {
    fs[0] = hm;
    fs[1] = (double)base;
  }
}

__global__ __launch_bounds__(256) void k_feat_rows(const double *__restrict__ beta, const double *__restrict__ w,
                                                   const int8_t *__restrict__ st, int64_t p,
                                                   const double *__restrict__ nzv, const double *__restrict__ fs,
                                                   FeatScalars sc, const double *__restrict__ beta_child,
                                                   uint16_t *__restrict__ F, float *__restrict__ T) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= p) return;
  const double hm = fs[0];
  const int64_t nnz = (int64_t)fs[1];
  const double b = beta[j], a = fabs(b);
  int64_t rank = nnz;
  if (a != 0.0) {
    rank = 0;
    for (int64_t i = 0; i < nnz; i++) rank += nzv[i] > a;
  }
  const int s = st[j];
  double f[kNF];
  f[0] = b;
  f[1] = hm > 0.0 ? w[j] / hm : 0.0;
  f[2] = (double)rank / (double)p;
  f[3] = s == kZero ? -1.0 : (s == kOne ? 1.0 : 0.0);
  f[4] = sc.lambda2;
  f[5] = (double)sc.n1 / sc.k;
  f[6] = (double)sc.n0 / sc.k;
  f[7] = (double)sc.kbar / sc.k;
  u16x8_t u;
#pragma unroll
  for (int e = 0; e < kNF; e++) u[e] = f2bf((float)f[e]);
  *reinterpret_cast<u16x8_t *>(F + j * kNF) = u;
  if (T && beta_child) T[j] = (float)(beta_child[j] - b);
}

// vhat = beta + out (the network's proposal before the prox step)
__global__ void k_mlp_propose(const double *__restrict__ beta, const float *__restrict__ out, int64_t p,
                              double *__restrict__ vhat) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < p; j += (int64_t)gridDim.x * blockDim.x)
    vhat[j] = beta[j] + (double)out[j];
}

}  // namespace

int mlp_grid(int64_t rows, int *cpb) {
  const int64_t per = 32 * kWaves;
  int64_t c = (rows + per * 512 - 1) / (per * 512);
  if (c < 1) c = 1;
  *cpb = (int)c;
  return (int)((rows + per * c - 1) / (per * c));
}

hipError_t launch_mlp_forward(const float *P, const uint16_t *F, int64_t rows, float *out, hipStream_t s) {
  int cpb;
  const int blocks = mlp_grid(rows, &cpb);
  k_mlp<false><<<blocks, 256, 0, s>>>(P, F, nullptr, rows, cpb, 0.f, out, nullptr);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *P, const uint16_t *F, const float *T, int64_t rows, float *part,
                           float *grad, hipStream_t s) {
  int cpb;
  const int blocks = mlp_grid(rows, &cpb);
  const float inv_n = 1.0f / (float)rows;
  k_mlp<true><<<blocks, 256, 0, s>>>(P, F, T, rows, cpb, inv_n, nullptr, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_mlp_reduce<<<(kNP + 1 + 63) / 64, 64 * kRedWaves, 0, s>>>(part, blocks, inv_n, grad);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float *P, const float *g, float *m1, float *m2, float lr, float beta1, float beta2,
                           float eps, float c1, float c2, hipStream_t s) {
  k_mlp_adam<<<(kNP + 255) / 256, 256, 0, s>>>(P, g, m1, m2, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_features(const double *beta, const double *w, const int8_t *st, int64_t p, double *nzv,
                           double *fs, FeatScalars sc, const double *beta_child, uint16_t *F, float *T,
                           hipStream_t s) {
  k_feat_prep<<<1, dev::NT, 0, s>>>(beta, w, p, nzv, fs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_feat_rows<<<(unsigned)((p + 255) / 256), 256, 0, s>>>(beta, w, st, p, nzv, fs, sc, beta_child, F, T);
  return hipGetLastError();
}

hipError_t launch_mlp_propose(const double *beta, const float *out, int64_t p, double *vhat, hipStream_t s) {
  k_mlp_propose<<<(unsigned)((p + 255) / 256 < 1024 ? (p + 255) / 256 : 1024), 256, 0, s>>>(beta, out, p, vhat);
  return hipGetLastError();
}

}  // namespace pr
