// The allocation-free variant of lc_dot: the block partial sums and the result live in a
// file-scope device array instead of a context's scratch, so the call needs no context and
// never allocates.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/lidkrylov.h"
#include "lk_internal.h"

namespace {

// k_dot writes at most kDotMaxParts partial sums (its grid is capped there); the fixed-order
// final sum goes to the element after them.
constexpr int kDotMaxParts = 4096;
constexpr int kMaxDevices = 64;
__device__ __align__(256) double scratch[kDotMaxParts + 32];

std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// This device's copy of `scratch` (its address taken once per device, with it current).
hipError_t scratch_ptr(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = (double*)p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

extern "C" int lc_dot_noalloc(const double* a, const double* b, size_t n, double* out, void* hip_stream) {
  if (!a || !b || !out || (uintptr_t)a % 8 || (uintptr_t)b % 8) return LC_EINVAL;
  if (n < 1 || n > LC_NOALLOC_MAX_N) return LC_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  double* s = nullptr;
  if (scratch_ptr(&s) != hipSuccess) return LC_EHIP;
  int nparts = 0;
  if (lk::launch_dot_partials(a, b, n, s, &nparts, st) != hipSuccess) return LC_EHIP;
  if (nparts > kDotMaxParts) return LC_EINVAL;  // cannot happen: the partial grid is capped
  if (lk::launch_sum(s, nparts, s + kDotMaxParts, st) != hipSuccess) return LC_EHIP;
  if (hipMemcpyAsync(out, s + kDotMaxParts, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess) return LC_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return LC_EHIP;
  return LC_OK;
}
