// Device scratch of octgrav_forces_noalloc: one file-scope array per GPU, so
// that the entry point needs no allocation.  The array's host-side name is
// only a stand-in; its device address is looked up once per device with
// hipGetSymbolAddress (that device current) and kept here.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "octgrav_internal.h"

namespace octgrav {

namespace {

constexpr size_t kNoallocScratchBytes = size_t(128) << 20;  // 128 MiB per GPU

__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

size_t noalloc_scratch_bytes() { return kNoallocScratchBytes; }

int noalloc_scratch(void** ptr, std::string& err) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    err = "no usable current HIP device";
    return -1;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t rc = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (rc != hipSuccess || !p) {
      (void)hipGetLastError();
      err = std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(rc);
      return -1;
    }
    g_ptr[dev] = p;
  }
  *ptr = g_ptr[dev];
  return 0;
}

}  // namespace octgrav
