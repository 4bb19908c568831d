// Launchers of the lane-pair colour-ordered recursion (templates in
// cobg_pair_impl.h).
#include "cobg_pair_impl.h"

namespace bg {
namespace pairk {

template <int N, typename T>
int launch(int64_t E, int64_t e0, int64_t count, const double* mom, const int8_t* hel, int hconf,
           double* amp, hipStream_t stream) {
  const int64_t grid = (count + Lds<N>::kPairs - 1) / Lds<N>::kPairs;
  hipLaunchKernelGGL((cobg_pair_kernel<N, T>), dim3((unsigned)grid), dim3(64),
                     Lds<N>::template bytes<T>(), stream, E, e0, count, mom, hel, hconf, amp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace pairk

int cobg_amplitudes(int n, bool fp32, int64_t E, const double* mom, const int8_t* hel, int hconf,
                    double* amp, hipStream_t stream) {
  return cobg_amplitudes_range(n, fp32, E, 0, E, mom, hel, hconf, amp, stream);
}

int cobg_amplitudes_range(int n, bool fp32, int64_t E, int64_t e0, int64_t count,
                          const double* mom, const int8_t* hel, int hconf, double* amp,
                          hipStream_t stream) {
  if (count <= 0) return 0;
  switch (n) {
#define BG_CASE(NN)                                                                             \
  case NN:                                                                                      \
    return fp32 ? pairk::launch<NN, float>(E, e0, count, mom, hel, hconf, amp, stream)         \
                : pairk::launch<NN, double>(E, e0, count, mom, hel, hconf, amp, stream);
    BG_CASE(4)
    BG_CASE(5)
    BG_CASE(6)
    BG_CASE(7)
    BG_CASE(8)
#undef BG_CASE
    default:
      return -2;
  }
}

}  // namespace bg
