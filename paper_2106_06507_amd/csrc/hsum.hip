// Helicity-summed colour-ordered |M|^2 (Section 2.2, eq. color_summed_analytic,
// summed over all 2^n helicity configurations) for few events in FP64, n <= 6.
// The fused kernel evaluates the configurations of a 32-event tile in turn on
// one wave, which leaves most of the GPU idle when there are only a few dozen
// tiles.  Here block (x, y) evaluates configuration y of tile x with the same
// device routines (recursion into LDS, then the colour sum per plane), writes
// its two planes' sums to part, and a second kernel adds them per event in
// configuration order and forms the result exactly as the fused kernel does:
// the same operations in the same order, so the same bits.
#include "fused_impl.h"

namespace bg {
namespace hsumk {

using fusedk::Cobg;
using fusedk::kTileEvents;

// part[(2 hc + h) E + e]: plane h of the colour sum of configuration hc
template <int N>
__global__ void __launch_bounds__(64) part_kernel(int64_t E, const double* __restrict__ mom,
                                                 const double* __restrict__ Cb,
                                                 double* __restrict__ part) {
  extern __shared__ __align__(16) unsigned char bg_hsum_lds[];
  constexpr int K = Cobg<N>::K;
  double* amp_lds =
      reinterpret_cast<double*>(bg_hsum_lds + pairk::Lds<N>::template bytes<double, false>());
  const int lane = threadIdx.x, pair = lane >> 1, h = lane & 1;
  const int64_t first = (int64_t)blockIdx.x * kTileEvents;
  const int count = (int)(E - first < kTileEvents ? E - first : kTileEvents);
  const bool live = pair < count;
  const int64_t e = first + (live ? pair : count - 1);
  const int hc = (int)blockIdx.y;
  double est[2] = {0.0, 0.0};
  pairk::cobg_pair_body<N, double, true, false, false, false>(
      bg_hsum_lds, E, mom, nullptr, hc, e, true, nullptr, 0, 0, amp_lds, est);
  const double q = fusedk::lower_quadform<K>(Cb, amp_lds + (size_t)h * K * kTileEvents + pair,
                                             kTileEvents);
  if (live) part[((int64_t)hc * 2 + h) * E + e] = q;
}

// me2[e]: each plane summed over the configurations in order, scaled by the
// squared couplings, then the two planes added (the fused kernel's order)
__global__ void __launch_bounds__(256) reduce_kernel(int n, int64_t E,
                                                    const double* __restrict__ part,
                                                    double* __restrict__ me2) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= E) return;
  double scale = 1.0;
  for (int i = 0; i < n - 2; ++i) scale *= kGsOverSqrt2;
  double q0 = 0.0, q1 = 0.0;
  for (int hc = 0; hc < (1 << n); ++hc) {
    q0 += part[((int64_t)hc * 2 + 0) * E + e];
    q1 += part[((int64_t)hc * 2 + 1) * E + e];
  }
  const double s2 = scale * scale;
  const double a = q0 * s2, b = q1 * s2;
  me2[e] = a + b;
}

template <int N>
int launch(int64_t E, const double* mom, const double* Cb, double* part, double* me2,
           hipStream_t stream) {
  const unsigned tiles = (unsigned)((E + kTileEvents - 1) / kTileEvents);
  hipLaunchKernelGGL((part_kernel<N>), dim3(tiles, 1u << N), dim3(64),
                     (Cobg<N>::template lds_bytes<double>()), stream, E, mom, Cb, part);
  hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, stream, N, E,
                     part, me2);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace hsumk

int cobg_hsum_split(int n, int64_t E, const double* mom, const double* Cb, double* part,
                    double* me2, hipStream_t stream) {
  if (E <= 0) return 0;
  switch (n) {
    case 4: return hsumk::launch<4>(E, mom, Cb, part, me2, stream);
    case 5: return hsumk::launch<5>(E, mom, Cb, part, me2, stream);
    case 6: return hsumk::launch<6>(E, mom, Cb, part, me2, stream);
    default: return -2;
  }
}

}  // namespace bg
