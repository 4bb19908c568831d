// Device memory of the allocation-free entry point bg_me2_noalloc: one
// file-scope array, of which every GPU the library runs on holds its own
// copy until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: its device address is looked up once per
// device (noalloc_scratch_address, called at context creation with the
// device current) and only that address is ever passed to kernels.
#include <hip/hip_runtime.h>

#include "bg_kernels.h"

namespace bg {
namespace {

__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

}  // namespace

int noalloc_scratch_address(void** out) {
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return -1;
  *out = p;
  return 0;
}

}  // namespace bg
