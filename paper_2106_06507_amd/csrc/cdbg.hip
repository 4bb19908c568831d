// Launchers of the colour-dressed recursion (templates in cdbg_impl.h).
#include "cdbg_impl.h"

namespace bg {
namespace cdbgk {

// Valid-flow classification and compaction.  Invalid events get me2 = 0.
// One atomic per 1024-thread block (the waves' counts are combined in LDS):
// a single counter hit once per wave serialises ~10^4 atomics per 2^20
// events in L2.
constexpr int kClassifyThreads = 1024;

__global__ void __launch_bounds__(kClassifyThreads) cdbg_classify_kernel(
    int n, int64_t E, const int8_t* __restrict__ col, double* __restrict__ me2,
    unsigned* __restrict__ list, unsigned* __restrict__ count) {
  __shared__ unsigned wave_count[kClassifyThreads / 64];
  __shared__ unsigned block_base;
  const int64_t e = (int64_t)blockIdx.x * kClassifyThreads + threadIdx.x;
  bool valid = false;
  if (e < E) {
    valid = flow_valid(n, E, col, e);
    if (!valid) me2[e] = 0.0;
  }
  const unsigned long long bal = __ballot(valid);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) wave_count[w] = (unsigned)__popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned tot = 0u;
    for (int v = 0; v < kClassifyThreads / 64; ++v) tot += wave_count[v];
    block_base = tot ? atomicAdd(count, tot) : 0u;
  }
  __syncthreads();
  if (valid) {
    unsigned base = block_base;
    for (int v = 0; v < w; ++v) base += wave_count[v];
    const unsigned long long below = lane ? (bal & ((~0ull) >> (64 - lane))) : 0ull;
    list[base + __popcll(below)] = (unsigned)e;
  }
}

__global__ void zero_u32_kernel(unsigned* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// Lanes per event of the standalone kernel, measured on MI355X for 2^20
// sampled flows with the packed colour entries (ms, 64 / 128 / 256 lanes):
// n = 7 FP64 0.93 / 1.89 / -, FP32 0.72 / 0.98 / -; n = 8 FP64 2.60 / 2.64 /
// -, FP32 1.17 / 1.41 / -; n = 9 FP64 - / 7.85 / 6.89, FP32 - / 3.26 / 3.60.
// Fewer lanes per event keep more events in flight and idle fewer lanes on
// the levels with few targets, until the per-event LDS (n = 9 FP64: 64 KB)
// caps the events per CU.
template <int N, typename T>
struct EventLanes {
  static constexpr int value = N <= 8 ? 64 : (sizeof(T) == 4 ? 128 : 256);
};

template <int N, typename T, bool EST = false>
int launch_events(int64_t E, const double* mom, const int8_t* hel, const int8_t* col,
                  const unsigned* list, const unsigned* count, unsigned* work, double* me2,
                  int grid, DressedCheck chk, hipStream_t stream) {
  constexpr int NL = EventLanes<N, T>::value;
  hipLaunchKernelGGL((cdbg_event_kernel<N, T, NL, EST>), dim3(grid), dim3(NL),
                     (Lay<N, T, EST>::bytes()), stream, E, mom, hel, col, list, count, work, me2,
                     chk);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N, typename T, bool EST = false>
int event_occupancy() {
  constexpr int NL = EventLanes<N, T>::value;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cdbg_event_kernel<N, T, NL, EST>, NL,
                                                   Lay<N, T, EST>::bytes()) != hipSuccess)
    return -1;
  return nb;
}

// The valid events (FP32 with the check when chk is given, else T), then
// the FP64 re-evaluation of the listed ones.
template <int N>
int run_events(bool fp32, int64_t E, const double* mom, const int8_t* hel, const int8_t* col,
               unsigned* ws, double* me2, int grid, const CheckArgs* chk, int fix_grid,
               hipStream_t stream) {
  const unsigned* list = ws + 4;
  if (!fp32)
    return launch_events<N, double>(E, mom, hel, col, list, ws, ws + 1, me2, grid, DressedCheck{},
                                    stream);
  if (!chk)
    return launch_events<N, float>(E, mom, hel, col, list, ws, ws + 1, me2, grid, DressedCheck{},
                                   stream);
  unsigned* flist = ws + 4 + E;
  int r = launch_events<N, float, true>(E, mom, hel, col, list, ws, ws + 1, me2, grid,
                                        DressedCheck{chk->tau, ws + 2, flist}, stream);
  if (r) return r;
  return launch_events<N, double>(E, mom, hel, col, flist, ws + 2, ws + 3, me2, fix_grid,
                                  DressedCheck{}, stream);
}

}  // namespace cdbgk

size_t cdbg_lds_bytes(int n, bool fp32) {
  switch (n) {
    case 4: return fp32 ? cdbgk::Lay<4, float>::bytes() : cdbgk::Lay<4, double>::bytes();
    case 5: return fp32 ? cdbgk::Lay<5, float>::bytes() : cdbgk::Lay<5, double>::bytes();
    case 6: return fp32 ? cdbgk::Lay<6, float>::bytes() : cdbgk::Lay<6, double>::bytes();
    case 7: return fp32 ? cdbgk::Lay<7, float>::bytes() : cdbgk::Lay<7, double>::bytes();
    case 8: return fp32 ? cdbgk::Lay<8, float>::bytes() : cdbgk::Lay<8, double>::bytes();
    case 9: return fp32 ? cdbgk::Lay<9, float>::bytes() : cdbgk::Lay<9, double>::bytes();
    default: return 0;
  }
}

int cdbg_blocks_per_cu(int n, bool fp32, bool chk) {
  switch (n) {
#define BG_CASE(NN)                                                                     \
  case NN:                                                                              \
    return !fp32 ? cdbgk::event_occupancy<NN, double>()                                 \
                 : (chk ? cdbgk::event_occupancy<NN, float, true>()                     \
                        : cdbgk::event_occupancy<NN, float>());
    BG_CASE(4)
    BG_CASE(5)
    BG_CASE(6)
    BG_CASE(7)
    BG_CASE(8)
    BG_CASE(9)
#undef BG_CASE
    default: return -2;
  }
}

// ws: unsigned [4 + 2 E]: valid-event count and work counter, listed-event
// count and work counter, the valid-event list, the listed-event list.
// Stream-ordered; the counts stay on the device.
int cdbg_me2(int n, bool fp32, int64_t E, const double* mom, const int8_t* hel, const int8_t* col,
             unsigned* ws, double* me2, int grid, const CheckArgs* chk, int fix_grid,
             hipStream_t stream) {
  if (E <= 0) return 0;
  unsigned* list = ws + 4;
  hipLaunchKernelGGL(cdbgk::zero_u32_kernel, dim3(1), dim3(64), 0, stream, ws, 4);
  hipLaunchKernelGGL(cdbgk::cdbg_classify_kernel,
                     dim3((unsigned)((E + cdbgk::kClassifyThreads - 1) / cdbgk::kClassifyThreads)),
                     dim3(cdbgk::kClassifyThreads), 0, stream, n, E, col, me2, list, ws);
  if (hipGetLastError() != hipSuccess) return -1;
  switch (n) {
    case 4: return cdbgk::run_events<4>(fp32, E, mom, hel, col, ws, me2, grid, chk, fix_grid, stream);
    case 5: return cdbgk::run_events<5>(fp32, E, mom, hel, col, ws, me2, grid, chk, fix_grid, stream);
    case 6: return cdbgk::run_events<6>(fp32, E, mom, hel, col, ws, me2, grid, chk, fix_grid, stream);
    case 7: return cdbgk::run_events<7>(fp32, E, mom, hel, col, ws, me2, grid, chk, fix_grid, stream);
    case 8: return cdbgk::run_events<8>(fp32, E, mom, hel, col, ws, me2, grid, chk, fix_grid, stream);
    case 9: return cdbgk::run_events<9>(fp32, E, mom, hel, col, ws, me2, grid, chk, fix_grid, stream);
    default: return -2;
  }
}

}  // namespace bg
