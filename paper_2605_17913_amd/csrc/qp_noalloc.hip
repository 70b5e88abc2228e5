// Allocation-free variant of qp_solve: the factor workspace of QPs whose
// bordered factor does not fit LDS comes from a fixed device array of this
// file instead of the context's growable workspace, so the call makes no
// allocation (for callers that cannot allocate: code under graph capture,
// tight serving loops, harnesses that forbid it).
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "../../include/qpx.h"
#include "qp_internal.h"

namespace {

// The workspace array.  Each GPU the library runs on holds its own copy
// until the process ends.  In host code this name is only a stand-in for
// the symbol: the device address comes from hipGetSymbolAddress, per device.
constexpr size_t kScratchBytes = (size_t)QPX_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) float scratch[kScratchBytes / sizeof(float)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
float *g_ptr[kMaxDevices] = {};

}  // namespace

namespace qpk {

// Resolve this device's copy of the array (the device must be current).
// Called by qp_create once per device; later calls return the stored value.
int noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return QPX_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return QPX_OK;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return QPX_ERR_HIP;
  g_ptr[device] = static_cast<float *>(p);
  return QPX_OK;
}

float *noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

}  // namespace qpk
