// Fixed device scratch of steps_forces_noalloc: a file-scope device array,
// one copy per GPU, held from module load until the process ends, so that
// the entry point that uses it never allocates device memory.
//
// In host code `scratch` names a host-side stand-in, not a device address:
// every host use goes through the address hipGetSymbolAddress returns for
// the current device, looked up once per device and kept here.

#include <hip/hip_runtime.h>

#include <mutex>

#include "steps_internal.h"

namespace steps {
namespace {

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 256;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};  // per device ordinal: this device's copy

}  // namespace

hipError_t noalloc_scratch(int device, void **out) {
  *out = nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (g_addr[device]) {
    *out = g_addr[device];
    return hipSuccess;
  }
  int prev = -1;
  hipError_t e = hipGetDevice(&prev);
  if (e != hipSuccess) return e;
  if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void *p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (prev != device) (void)hipSetDevice(prev);
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_addr[device] = p;
  *out = p;
  return hipSuccess;
}

}  // namespace steps
