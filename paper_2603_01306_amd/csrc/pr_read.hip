// Plain streaming read of a device buffer on gfx950: 16-byte non-temporal
// loads, U per lane in flight, grid-stride over the buffer.  It measures the
// read rate that the HBM-bound kernels (the X^T pass, the column-list
// product) are compared with, next to the data-sheet peak.  The sum only
// decides a store to pr::g_read_sink (external linkage, so the compiler keeps
// the store and with it the loads) that never happens for finite data below
// 1.5e38 in sum.
#include "pr_device.h"

namespace pr {

__device__ float g_read_sink;

namespace {
using dev::f4_t;

template <int U>
__global__ __launch_bounds__(256) void k_read_stream(const f4_t *__restrict__ x, int64_t n16) {
  f4_t acc = {0.f, 0.f, 0.f, 0.f};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (U - 1) * stride < n16; i += U * stride) {
    f4_t v[U];
#pragma unroll
    for (int u = 0; u < U; u++) v[u] = __builtin_nontemporal_load(x + i + u * stride);
#pragma unroll
    for (int u = 0; u < U; u++) acc += v[u];
  }
  for (; i < n16; i += stride) acc += __builtin_nontemporal_load(x + i);
  if (acc.x + acc.y + acc.z + acc.w == 1.5e38f) g_read_sink = 1.f;
}

}  // namespace

hipError_t launch_read_stream(const void *buf, int64_t n16, int blocks, int unroll, hipStream_t s) {
  if (unroll == 4)
    k_read_stream<4><<<blocks, 256, 0, s>>>((const f4_t *)buf, n16);
  else
    k_read_stream<1><<<blocks, 256, 0, s>>>((const f4_t *)buf, n16);
  return hipGetLastError();
}

}  // namespace pr
