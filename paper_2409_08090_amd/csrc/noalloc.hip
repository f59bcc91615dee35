// noalloc.hip -- the device scratch of the allocation-free periodogram
// (mils_periodogram_noalloc): a file-scope device array, one per GPU, whose
// address each GPU gets once, with that GPU current.  Host code uses only the
// address returned here, never the array's own name (which on the host is a
// stand-in symbol, not device memory).
#include <hip/hip_runtime.h>

#include <mutex>

#include "api_internal.h"

namespace mils {

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

void* noalloc_scratch(int device, hipError_t* err) {
  static std::mutex mu;
  static void* ptr[kNoAllocDevices] = {};
  std::lock_guard<std::mutex> lk(mu);
  if (device < 0 || device >= kNoAllocDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  if (!ptr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipSetDevice(device);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) {
      *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
      return nullptr;
    }
    ptr[device] = p;
  }
  *err = hipSuccess;
  return ptr[device];
}

}  // namespace mils
