// Launchers of the lane-pair colour-ordered recursion (templates in
// cobg_pair_impl.h).
#include "cobg_pair_impl.h"

namespace bg {
namespace pairk {

template <int N, typename T>
int launch(int64_t E, const double* mom, const int8_t* hel, int hconf, double* amp,
           hipStream_t stream) {
  const int64_t grid = (E + Lds<N>::kPairs - 1) / Lds<N>::kPairs;
  hipLaunchKernelGGL((cobg_pair_kernel<N, T>), dim3((unsigned)grid), dim3(64),
                     Lds<N>::template bytes<T>(), stream, E, mom, hel, hconf, amp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace pairk

int cobg_amplitudes(int n, bool fp32, int64_t E, const double* mom, const int8_t* hel, int hconf,
                    double* amp, hipStream_t stream) {
  if (E <= 0) return 0;
  switch (n) {
    case 4: return fp32 ? pairk::launch<4, float>(E, mom, hel, hconf, amp, stream)
                        : pairk::launch<4, double>(E, mom, hel, hconf, amp, stream);
    case 5: return fp32 ? pairk::launch<5, float>(E, mom, hel, hconf, amp, stream)
                        : pairk::launch<5, double>(E, mom, hel, hconf, amp, stream);
    case 6: return fp32 ? pairk::launch<6, float>(E, mom, hel, hconf, amp, stream)
                        : pairk::launch<6, double>(E, mom, hel, hconf, amp, stream);
    case 7: return fp32 ? pairk::launch<7, float>(E, mom, hel, hconf, amp, stream)
                        : pairk::launch<7, double>(E, mom, hel, hconf, amp, stream);
    default: return -2;
  }
}

}  // namespace bg
