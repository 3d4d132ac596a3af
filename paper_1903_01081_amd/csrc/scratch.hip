// The static exchange space of emt_step_noalloc (include/emt.h): the split
// components' partial voltages, give-up flag and XCD record, held in one
// file-scope device array instead of the context's allocations, for callers
// that cannot allocate while they step. Each device that runs the library
// holds its own copy until the process ends. Host code never uses the
// array's name as an address: its device address is looked up once per
// device (static_scratch_ptr) and only that address reaches kernels and
// fills.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "launch.h"

namespace emt {

__device__ __align__(256) static unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch_ptr(int device, void **ptr) {
  static std::mutex mu;
  static std::vector<void *> ptrs;
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0) return hipErrorInvalidDevice;
  if ((size_t)device >= ptrs.size()) ptrs.resize((size_t)device + 1, nullptr);
  if (!ptrs[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    // the host-side stand-in is not a device address: never hand it out
    if (p == nullptr || p == static_cast<void *>(scratch)) return hipErrorInvalidSymbol;
    ptrs[device] = p;
  }
  *ptr = ptrs[device];
  return hipSuccess;
}

}  // namespace emt
