// Device helpers shared by the kernel translation units of libpr (gfx950,
// wave64): deterministic workgroup reductions and scans, 16-byte vector loads
// of the stored X (FP64 / FP32 / BF16, exact upcast to FP64), and the scalar
// maps of the method (Huber function, softplus, FISTA momentum sequence).
#pragma once
#include <math.h>

#include "pr_internal.h"

namespace pr {
namespace dev {

constexpr int NT = kNodeThreads;
constexpr int NW = NT / 64;

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// Workgroup barrier for LDS traffic only: waits for this wave's LDS
// operations and meets the other waves, but leaves its global stores in
// flight (a full __syncthreads also waits for every outstanding global
// access).  Only for code whose threads do not read each other's global
// writes within the kernel.
__device__ __forceinline__ void lds_barrier() { __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// One DPP move of a double (two 32-bit halves); lanes outside row_mask, or
// reading outside their row, receive `idb` (the identity's bit pattern).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double v, long long idb) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)(idb & 0xffffffffll), (int)(b & 0xffffffffll), CTRL, ROWMASK, 0xf,
                                             false);
  const int hi = __builtin_amdgcn_update_dpp((int)(idb >> 32), (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave reductions on the VALU cross-lane (DPP) network: pairs and quads by
// quad permutations, 8 and 16 lanes by the half-row and row mirrors, then row
// broadcasts of lane 15 and lane 31 leave the total in lane 63, which every
// lane reads.  The order of the additions is fixed, so the result is
// reproducible.
template <class OP>
__device__ __forceinline__ double wave_reduce(double v, long long idb, OP op) {
  v = op(v, dpp_f64<0xb1, 0xf>(v, idb));   // quad_perm [1,0,3,2]
  v = op(v, dpp_f64<0x4e, 0xf>(v, idb));   // quad_perm [2,3,0,1]
  v = op(v, dpp_f64<0x141, 0xf>(v, idb));  // row_half_mirror
  v = op(v, dpp_f64<0x140, 0xf>(v, idb));  // row_mirror
  v = op(v, dpp_f64<0x142, 0xa>(v, idb));  // row_bcast:15 into rows 1 and 3
  v = op(v, dpp_f64<0x143, 0xc>(v, idb));  // row_bcast:31 into rows 2 and 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_sum(double v) {
  return wave_reduce(v, 0ll, [](double a, double b) { return a + b; });
}

__device__ __forceinline__ double wave_max(double v) {
  return wave_reduce(v, (long long)0xfff0000000000000ull, [](double a, double b) { return fmax(a, b); });
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

// Backtracking model test of a trial, shared by the X^T pass (which skips a
// rejected trial) and the node step, so that both take the same decision: the
// remainder f(x) - f(y) - <grad f(y), x - y> summed over the loss epilogue's
// blocks by one wave in a fixed order, against (L / 2) ||x - y||^2; a trial
// at the cap Lmax is accepted.
__device__ __forceinline__ double bt_remainder(const double *dsum, int nfin) {
  double v = 0.0;
  for (int i = lane_id(); i < nfin; i += 64) v += dsum[i];
  return wave_sum(v);
}
__device__ __forceinline__ bool bt_accept(double D, double L, double dxy, double Lmax) {
  return L >= Lmax || D <= 0.5 * L * dxy;
}

// Restart decision after the evaluation of iterate `it` (gap = Phi - Psi at
// it, phi_prev = Phi at it - 1): the first iterate always starts an epoch;
// then the duality-gap restart of Section 3.3 (gap fell by the factor eta
// since the epoch start), the function-value restart (Phi increased), no
// restart (plain FISTA), or a restart every step (proximal gradient: zero
// momentum; not counted as a restart).
__device__ __forceinline__ int decide_restart(const NodeParams *prm, int it, double gap, double phi, double phi_prev,
                                              double &gap_ref, int &restarts) {
  if (it == 0) {
    gap_ref = gap;
    return 1;
  }
  switch (prm->method) {
    case kFistaGap:
    case kFistaBtGap:
      if (gap <= gap_ref / prm->eta) {
        gap_ref = gap;
        restarts++;
        return 1;
      }
      return 0;
    case kFistaFv:
      if (phi > phi_prev) {
        restarts++;
        return 1;
      }
      return 0;
    case kPgd:
      return 1;
    default:
      return 0;
  }
}

// One 16-byte non-temporal load of the stored X (raw), its exact widening to
// FP64 (cvt), or both (load).  Kernels that must have every load of a step in
// flight before any arithmetic issue the raw loads first.
template <typename T>
struct XLoad;

template <>
struct XLoad<float> {
  static constexpr int VEC = 4;
  typedef f4_t raw_t;
  __device__ __forceinline__ static raw_t raw(const float *p) {
    return __builtin_nontemporal_load(reinterpret_cast<const f4_t *>(p));
  }
  __device__ __forceinline__ static void cvt(const raw_t &v, double (&d)[4]) {
    d[0] = (double)v.x;
    d[1] = (double)v.y;
    d[2] = (double)v.z;
    d[3] = (double)v.w;
  }
  __device__ __forceinline__ static void load(const float *p, double (&d)[4]) { cvt(raw(p), d); }
};

template <>
struct XLoad<double> {
  static constexpr int VEC = 2;
  typedef d2_t raw_t;
  __device__ __forceinline__ static raw_t raw(const double *p) {
    return __builtin_nontemporal_load(reinterpret_cast<const d2_t *>(p));
  }
  __device__ __forceinline__ static void cvt(const raw_t &v, double (&d)[2]) {
    d[0] = v.x;
    d[1] = v.y;
  }
  __device__ __forceinline__ static void load(const double *p, double (&d)[2]) { cvt(raw(p), d); }
};

// bf16 stored as uint16_t bit patterns
template <>
struct XLoad<uint16_t> {
  static constexpr int VEC = 8;
  typedef u4_t raw_t;
  __device__ __forceinline__ static raw_t raw(const uint16_t *p) {
    return __builtin_nontemporal_load(reinterpret_cast<const u4_t *>(p));
  }
  __device__ __forceinline__ static void cvt(const raw_t &v, double (&d)[8]) {
    const unsigned int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; q++) {
      d[2 * q] = (double)__uint_as_float(w[q] << 16);
      d[2 * q + 1] = (double)__uint_as_float(w[q] & 0xffff0000u);
    }
  }
  __device__ __forceinline__ static void load(const uint16_t *p, double (&d)[8]) { cvt(raw(p), d); }
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


}  // namespace dev
}  // namespace pr
