// Small device utilities of the C-ABI layer: word fills that can be recorded
// into a graph (no memset nodes) and the input check of BG_FLAG_VALIDATE.
#include "bg_kernels.h"

namespace bg {
namespace {

__global__ void __launch_bounds__(64) fill_u32_kernel(unsigned* __restrict__ p, int n, unsigned v) {
  for (int i = threadIdx.x; i < n; i += 64) p[i] = v;
}

// bad[0] |= 1 if some hel entry is not +1/-1 or some col entry is not 0, 1, 2.
__global__ void __launch_bounds__(256) validate_kernel(int64_t nh, const int8_t* __restrict__ hel,
                                                      int64_t nc, const int8_t* __restrict__ col,
                                                      unsigned* __restrict__ bad) {
  const int64_t total = nh > nc ? nh : nc;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool b = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    if (i < nh) {
      const int x = hel[i];
      b |= x != 1 && x != -1;
    }
    if (i < nc) {
      const int x = col[i];
      b |= x < 0 || x > 2;
    }
  }
  if (__ballot(b) != 0ull && (threadIdx.x & 63) == 0) atomicOr(bad, 1u);
}

}  // namespace

int fill_u32(unsigned* p, int n, unsigned v, hipStream_t stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, stream, p, n, v);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int validate_inputs(int64_t nh, const int8_t* hel, int64_t nc, const int8_t* col, unsigned* bad,
                    hipStream_t stream) {
  const int64_t total = nh > nc ? nh : nc;
  if (total <= 0) return 0;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(validate_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, nh, hel, nc,
                     col, bad);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace bg
