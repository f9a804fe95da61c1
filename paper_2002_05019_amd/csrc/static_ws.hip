// Allocation-free binding: the workspace is a static device array of the
// library, for callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dd.h"

namespace dd {
dd_status bind_static(dd_ctx c, void *dev, int64_t bytes, int device);
dd_status set_error(dd_status s, const char *msg);
}  // namespace dd

namespace {
// One copy per GPU, held until the process ends.  In host code `scratch`
// names a host-side stand-in: its device address comes from
// hipGetSymbolAddress, once per device (scratch_ptr).
static __device__ __align__(256) unsigned char scratch[DD_STATIC_WORKSPACE_BYTES];

constexpr int MAX_DEV = 64;
std::mutex g_mu;
void *g_ptr[MAX_DEV] = {};
}  // namespace

extern "C" dd_status dd_bind_static_workspace(dd_ctx ctx) {
  if (!ctx) return dd::set_error(DD_ERR_ARG, "null context");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEV)
    return dd::set_error(DD_ERR_DEVICE, "no current HIP device");
  void *p = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
      void *q = nullptr;
      const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !q) return dd::set_error(DD_ERR_DEVICE, "hipGetSymbolAddress of the static workspace failed");
      g_ptr[dev] = q;
    }
    p = g_ptr[dev];
  }
  return dd::bind_static(ctx, p, (int64_t)DD_STATIC_WORKSPACE_BYTES, dev);
}
