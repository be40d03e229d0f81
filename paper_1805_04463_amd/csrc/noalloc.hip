// Allocation-free variant of the interval-abundance call: its scratch memory (the
// counters' work-queue counters) lives in a file-scope device array instead of a
// caller workspace, for callers that cannot allocate device memory.
//
// Each GPU the library runs on holds its own copy of `scratch` (kScratchBytes) until the
// process ends.  The array's name is a host-side stand-in in host code: its device address
// is looked up once per device with hipGetSymbolAddress, with that device current, and
// only that address is handed to kernels.  Every call on a device shares the array and
// the counters restart at zero in each call (a fill kernel on the call's stream), so
// calls on one device that overlap in time (several streams, several host threads
// without ordering) race on it.
#include <mutex>

#include "common.h"

namespace cs {

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mutex;
void* g_scratch[kMaxDevices] = {};

}  // namespace

cs_status scratch_for_current_device(void** out) {
  int dev = -1;
  CS_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return CS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    CS_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return CS_ERR_HIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return CS_OK;
}

}  // namespace cs
