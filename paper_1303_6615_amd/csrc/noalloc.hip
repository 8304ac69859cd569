// Device scratch of the fine-batch entry point that allocates nothing
// (aparareal_fine_batch_noalloc): one file-scope array per device, which each
// device holds until the process ends.  Host code never uses the array's name
// as an address (in host code it is a host-side stand-in); it asks for this
// device's address once, with the device current, and keeps it per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "noalloc.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[ap::kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

}  // namespace

namespace ap {

hipError_t noalloc_scratch(int device, void** ptr) {
  if (device < 0 || device >= kMaxDevices || !ptr) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // the address is looked up with its device current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_addr[device] = p;
  }
  *ptr = g_addr[device];
  return hipSuccess;
}

}  // namespace ap
