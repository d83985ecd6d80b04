// pr_prox_noalloc: the prox of g_N without any allocation, for callers that
// cannot allocate device memory (code under stream capture, tight serving
// loops, harnesses that forbid hipMalloc).  Its workspace is a file-scope
// device array; every GPU the library runs on holds its own copy until the
// process ends, and every call on that GPU shares it.
#include <math.h>

#include <mutex>

#include "../../include/pr.h"
#include "pr_internal.h"

using namespace pr;

namespace {

constexpr int64_t kMaxP = PR_PROX_NOALLOC_MAX_P;
constexpr int kMaxDevices = 64;

// kMaxP doubles of |v| magnitudes, then one 256-byte slot holding the error
// flag the kernel writes on every call (so nothing has to start at zero).
static __device__ __align__(256) double scratch[kMaxP + 32];

std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};  // device address of `scratch` on each device

// The device address of this device's copy of `scratch`, looked up once per
// device with that device current.  In host code the array's name is only a
// host-side stand-in, so kernels and copies always get this address.
int scratch_of_current_device(double **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PR_EDEVICE;
  if (dev < 0 || dev >= kMaxDevices) return PR_EDEVICE;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PR_EDEVICE;
    g_ptr[dev] = static_cast<double *>(ptr);
  }
  *out = g_ptr[dev];
  return PR_OK;
}

}  // namespace

extern "C" {

int pr_prox_noalloc(void *stream, const double *v, int64_t p, double rho, int32_t k, double M,
                    const int8_t *status, double *out) {
  if (!v || !out || !status || p < 1 || !(rho > 0.0) || !isfinite(rho) || !(M > 0.0) || k < 1) return PR_EINVAL;
  if (p > kMaxP) return PR_EINVAL;
  double *ws = nullptr;
  const int rc = scratch_of_current_device(&ws);
  if (rc != PR_OK) return rc;
  int32_t *flag = reinterpret_cast<int32_t *>(ws + kMaxP);
  hipStream_t s = (hipStream_t)stream;
  int32_t hflag = -1;
  hipError_t e = launch_prox_counted(v, out, p, rho, k, M, status, ws, flag, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flag, sizeof(hflag), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return PR_EDEVICE;
  return hflag == 0 ? PR_OK : PR_EINVAL;
}

}  // extern "C"
