// colloc_eval_noalloc: the pattern-value call for callers that cannot allocate device memory
// (code under graph capture, tight serving loops, harnesses that forbid allocation).  The
// per-element partial sums that colloc_eval keeps in the caller's workspace live here in a
// file-scope device array instead, one copy per GPU, addressed through the pointer that
// hipGetSymbolAddress returns on that GPU (the array's name is not a device address on the host).
#include <mutex>

#include "../../include/colloc.h"
#include "kernels.h"

namespace cl {

static __device__ __align__(256) double scratch[COLLOC_NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};
}  // namespace

// Device address of this GPU's scratch array, looked up once per device with that device
// current.  Returns 0, or COLLOC_EHIP when the device or the symbol cannot be resolved.
int static_scratch(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return COLLOC_EHIP;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return COLLOC_EHIP;
    g_ptr[dev] = (double*)p;
  }
  *out = g_ptr[dev];
  return COLLOC_OK;
}

}  // namespace cl
