// Fused colour-ordered kernel (recursion and colour sum in one pass), the
// leading-colour kernels, and the host side of the persistent
// mixed-multiplicity batch (kernel template: batch_impl.h).  Tile routines:
// fused_impl.h.
#include "batch_impl.h"

namespace bg {
// the batch kernel instances live in batch_kinds_*.hip
#define BG_EXTERN_KINDS(KK)                                                                   \
  extern template int batch_occupancy_kinds<KK>(bool, int, int, size_t);                      \
  extern template void batch_launch_kinds<KK>(bool, int, int, const BatchSegTable&,            \
                                              const BatchTile*, unsigned, unsigned,            \
                                              const unsigned*, unsigned*, double*, int64_t,    \
                                              int, size_t, hipStream_t);
BG_EXTERN_KINDS(kBatchKindsAll)
BG_EXTERN_KINDS(kBatchKindsCobg)
BG_EXTERN_KINDS(kBatchKindsCdbg)
#undef BG_EXTERN_KINDS
}  // namespace bg

namespace bg {
namespace fusedk {

// n <= 6: one 32-event tile per block, amplitudes in LDS; the hardware
// dispatcher balances the blocks.  CHK: FP32 pass that lists ill-conditioned
// events (TileCheck).
template <int N, typename T, bool HSUM, bool CHK = false>
__global__ void __launch_bounds__(64) cobg_fused_kernel(int64_t E, const double* __restrict__ mom,
                                                       const int8_t* __restrict__ hel,
                                                       const double* __restrict__ Cb,
                                                       double* __restrict__ me2, TileCheck chk) {
  extern __shared__ __align__(16) unsigned char bg_fused_lds[];
  const int64_t first = (int64_t)blockIdx.x * kTileEvents;
  const int64_t left = E - first;
  cobg_tile<N, T, HSUM, false, CHK>(bg_fused_lds, E, mom, hel, Cb, nullptr, me2, first,
                                    (int)(left < kTileEvents ? left : kTileEvents), chk);
}

// n = 7: persistent blocks, each with its own scratch slice, take tiles from
// an atomic queue (reset by zero_counter_kernel before the launch).
template <typename T, bool HSUM, bool CHK = false>
__global__ void __launch_bounds__(64, sizeof(T) == 4 ? 2 : 1) cobg_fused_queue_kernel(int64_t E,
                                                             const double* __restrict__ mom,
                                                             const int8_t* __restrict__ hel,
                                                             const double* __restrict__ Cb,
                                                             double* __restrict__ scratch,
                                                             unsigned* __restrict__ counter,
                                                             double* __restrict__ me2,
                                                             TileCheck chk) {
  extern __shared__ __align__(16) unsigned char bg_fused_lds[];
  double* blk = scratch + (size_t)blockIdx.x * Cobg<7>::kScratch;
  const unsigned tiles = (unsigned)((E + kTileEvents - 1) / kTileEvents);
  for (;;) {
    unsigned t = 0;
    if (threadIdx.x == 0) t = atomicAdd(counter, 1u);
    t = (unsigned)__builtin_amdgcn_readfirstlane((int)__shfl(t, 0));
    if (t >= tiles) break;
    const int64_t first = (int64_t)t * kTileEvents;
    const int64_t left = E - first;
    cobg_tile<7, T, HSUM, false, CHK>(bg_fused_lds, E, mom, hel, Cb, blk, me2, first,
                                      (int)(left < kTileEvents ? left : kTileEvents), chk);
  }
}

// FP64 re-evaluation of the events listed by a CHK pass: persistent blocks
// stride over 32-event tiles of the list; the list length is read on the
// device, so the launch needs no host synchronisation.  scratch: one slice
// of Cobg<N>::kScratch doubles per block (n = 7).
template <int N, bool HSUM>
__global__ void __launch_bounds__(64) cobg_fix_kernel(int64_t E, const double* __restrict__ mom,
                                                     const int8_t* __restrict__ hel,
                                                     const double* __restrict__ Cb,
                                                     double* __restrict__ scratch,
                                                     const unsigned* __restrict__ count,
                                                     const unsigned* __restrict__ list,
                                                     double* __restrict__ me2) {
  extern __shared__ __align__(16) unsigned char bg_fused_lds[];
  double* blk = Cobg<N>::kScratch ? scratch + (size_t)blockIdx.x * Cobg<N>::kScratch : nullptr;
  const unsigned cnt = *count;
  for (unsigned first = blockIdx.x * kTileEvents; first < cnt; first += gridDim.x * kTileEvents) {
    const unsigned left = cnt - first;
    cobg_tile<N, double, HSUM, false, false, true>(
        bg_fused_lds, E, mom, hel, Cb, blk, me2, first,
        (int)(left < (unsigned)kTileEvents ? left : (unsigned)kTileEvents), TileCheck{}, list);
  }
}

// Leading colour, one 32-event tile per block (CHK: FP32 pass that lists
// ill-conditioned events, see lc_tile).
template <int N, typename T, bool CHK = false>
__global__ void __launch_bounds__(64) lc_kernel(int64_t E, const double* __restrict__ mom,
                                               const int8_t* __restrict__ hel,
                                               double* __restrict__ me2, TileCheck chk) {
  extern __shared__ __align__(16) unsigned char bg_lc_lds[];
  const int64_t first = (int64_t)blockIdx.x * kTileEvents;
  const int64_t left = E - first;
  lc_tile<N, T, CHK>(bg_lc_lds, E, mom, hel, me2, first,
                     (int)(left < kTileEvents ? left : kTileEvents), chk);
}

// FP64 leading colour of the listed events: persistent blocks stride over
// 32-event tiles of the list, whose length is read on the device.
template <int N>
__global__ void __launch_bounds__(64) lc_fix_kernel(int64_t E, const double* __restrict__ mom,
                                                   const int8_t* __restrict__ hel,
                                                   const unsigned* __restrict__ count,
                                                   const unsigned* __restrict__ list,
                                                   double* __restrict__ me2) {
  extern __shared__ __align__(16) unsigned char bg_lc_lds[];
  const unsigned cnt = *count;
  for (unsigned first = blockIdx.x * kTileEvents; first < cnt; first += gridDim.x * kTileEvents) {
    const unsigned left = cnt - first;
    lc_tile<N, double, false, true>(bg_lc_lds, E, mom, hel, me2, first,
                                    (int)(left < (unsigned)kTileEvents ? left : (unsigned)kTileEvents),
                                    TileCheck{}, list);
  }
}

// FP64 leading colour on straight paths (cobg_path_impl.h), for n = 7, where
// the depth-first walk's FP64 state spills: 32 events per 64-lane block.
// idx (re-evaluation of listed events): the block's events are idx[j] for
// j < *cnt (blocks past the list return at once).
template <int N>
__global__ void __launch_bounds__(64) lc_path_kernel(int64_t E, const double* __restrict__ mom,
                                                    const int8_t* __restrict__ hel,
                                                    double* __restrict__ me2,
                                                    const unsigned* __restrict__ idx,
                                                    const unsigned* __restrict__ cnt) {
  extern __shared__ __align__(16) unsigned char bg_lcp_lds[];
  const int pair = (int)threadIdx.x >> 1, h = (int)threadIdx.x & 1;
  const int64_t j = (int64_t)blockIdx.x * kTileEvents + pair;
  bool live;
  int64_t e;
  if (idx) {
    const int64_t total = (int64_t)*cnt;
    const int64_t b0 = (int64_t)blockIdx.x * kTileEvents;
    if (b0 >= total) return;  // the whole block (uniform)
    live = j < total;
    e = (int64_t)idx[live ? j : b0];
  } else {
    live = j < E;
    e = live ? j : E - 1;
  }
  const double q = pathk::cobg_path_body<N, double, false, true>(bg_lcp_lds, E, mom, hel, 0, e,
                                                                 false, nullptr, 0, 0);
  double colour = 8.0;  // N^(n-2) (N^2 - 1)
#pragma unroll
  for (int i = 0; i < N - 2; ++i) colour *= 3.0;
  if (live && h == 0) me2[e] = q * colour;
}

template <int N, typename T>
int lc_launch(int64_t E, const double* mom, const int8_t* hel, double* me2, const CheckArgs* chk,
              int fix_grid, hipStream_t stream) {
  const unsigned tiles = (unsigned)((E + kTileEvents - 1) / kTileEvents);
  if constexpr (N == 7) {
    // FP64 (the plain path and the re-evaluation of listed events) on
    // straight paths
    const size_t lds = pathk::Lds<N>::template bytes<double>();
    if (!chk) {
      if constexpr (sizeof(T) == 8) {
        hipLaunchKernelGGL((lc_path_kernel<N>), dim3(tiles), dim3(64), lds, stream, E, mom, hel,
                           me2, nullptr, nullptr);
        return hipGetLastError() == hipSuccess ? 0 : -1;
      }
    } else {
      hipLaunchKernelGGL((lc_kernel<N, float, true>), dim3(tiles), dim3(64),
                         (pairk::Lds<N, true>::template bytes<float>()), stream, E, mom, hel, me2,
                         TileCheck{chk->tau, chk->count, chk->list});
      hipLaunchKernelGGL((lc_path_kernel<N>), dim3(tiles), dim3(64), lds, stream, E, mom, hel,
                         me2, chk->list, chk->count);
      return hipGetLastError() == hipSuccess ? 0 : -1;
    }
  }
  if (!chk) {
    hipLaunchKernelGGL((lc_kernel<N, T>), dim3(tiles), dim3(64),
                       (pairk::Lds<N, true>::template bytes<T>()), stream, E, mom, hel, me2,
                       TileCheck{});
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  hipLaunchKernelGGL((lc_kernel<N, float, true>), dim3(tiles), dim3(64),
                     (pairk::Lds<N, true>::template bytes<float>()), stream, E, mom, hel, me2,
                     TileCheck{chk->tau, chk->count, chk->list});
  hipLaunchKernelGGL((lc_fix_kernel<N>), dim3((unsigned)fix_grid), dim3(64),
                     (pairk::Lds<N, true>::template bytes<double>()), stream, E, mom, hel,
                     chk->count, chk->list, me2);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N>
int lc_fix_occupancy() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lc_fix_kernel<N>, 64,
                                                   pairk::Lds<N, true>::template bytes<double>()) !=
      hipSuccess)
    return -1;
  return nb;
}

__global__ void zero_counter_kernel(unsigned* c) {
  if (threadIdx.x == 0) c[0] = 0u;
}

// Tiles of the re-evaluation pass: segment s contributes ceil(fcount[s] /
// step) tiles over its list.  Colour-dressed segments come first and take one
// event per tile (a listed event is valid and costs a whole block for tens
// of microseconds, so the queue must spread them over all blocks);
// colour-ordered segments follow with tiles of 128 events (four 32-event
// sub-tiles, one per wave).  range[0..5]: the dressed tiles [0, n_cd), the
// colour-ordered tiles [n_cd, total) and all tiles [0, total).
__global__ void __launch_bounds__(256) fix_tiles_kernel(const BatchSegTable segs, int n_segs,
                                                       const unsigned* __restrict__ fcount,
                                                       BatchTile* __restrict__ tiles,
                                                       unsigned* __restrict__ range) {
  __shared__ unsigned start[kBatchMaxSegs];
  __shared__ unsigned ntile[kBatchMaxSegs];
  if (threadIdx.x == 0) {
    unsigned acc = 0, n_cd = 0;
    for (int pass = 0; pass < 2; ++pass) {  // dressed segments first
      for (int i = 0; i < n_segs; ++i) {
        const bool cd = segs.s[i].kind >= kBatchCdbg;
        if (cd != (pass == 0)) continue;
        const unsigned step = cd ? 1u : 128u;
        start[i] = acc;
        ntile[i] = (fcount[i] + step - 1) / step;
        acc += ntile[i];
      }
      if (pass == 0) n_cd = acc;
    }
    range[0] = 0u;
    range[1] = n_cd;
    range[2] = n_cd;
    range[3] = acc;
    range[4] = 0u;
    range[5] = acc;
  }
  __syncthreads();
  for (int i = 0; i < n_segs; ++i) {
    const unsigned step = segs.s[i].kind >= kBatchCdbg ? 1u : 128u;
    const unsigned cnt = fcount[i];
    for (unsigned k = threadIdx.x; k < ntile[i]; k += blockDim.x) {
      const unsigned f = k * step;
      tiles[start[i] + k] = BatchTile{(int64_t)f, i, (int)(cnt - f < step ? cnt - f : step)};
    }
  }
}

template <int N, typename T>
int fused_launch(int64_t E, const double* mom, const int8_t* hel, const double* Cb,
                 double* scratch, unsigned* counter, int grid, double* me2, const TileCheck* chk,
                 hipStream_t stream) {
  const size_t lds = Cobg<N>::template lds_bytes<T>();
  const TileCheck ck = chk ? *chk : TileCheck{};
  if constexpr (Cobg<N>::kLdsAmp) {
    (void)scratch;
    (void)counter;
    (void)grid;
    const unsigned tiles = (unsigned)((E + kTileEvents - 1) / kTileEvents);
#define BG_FUSED(HS, CK)                                                                      \
  hipLaunchKernelGGL((cobg_fused_kernel<N, T, HS, CK>), dim3(tiles), dim3(64), lds, stream, E, \
                     mom, hel, Cb, me2, ck)
    if constexpr (sizeof(T) == 4) {
      if (hel) {
        if (chk) BG_FUSED(false, true); else BG_FUSED(false, false);
      } else {
        if (chk) BG_FUSED(true, true); else BG_FUSED(true, false);
      }
    } else {
      if (hel) BG_FUSED(false, false); else BG_FUSED(true, false);
    }
#undef BG_FUSED
  } else {
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, stream, counter);
#define BG_QUEUE(HS, CK)                                                                      \
  hipLaunchKernelGGL((cobg_fused_queue_kernel<T, HS, CK>), dim3(grid), dim3(64), lds, stream, \
                     E, mom, hel, Cb, scratch, counter, me2, ck)
    if constexpr (sizeof(T) == 4) {
      if (hel) {
        if (chk) BG_QUEUE(false, true); else BG_QUEUE(false, false);
      } else {
        if (chk) BG_QUEUE(true, true); else BG_QUEUE(true, false);
      }
    } else {
      if (hel) BG_QUEUE(false, false); else BG_QUEUE(true, false);
    }
#undef BG_QUEUE
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N>
int fix_launch(int64_t E, const double* mom, const int8_t* hel, const double* Cb,
               double* scratch, const unsigned* count, const unsigned* list, int grid,
               double* me2, hipStream_t stream) {
  const size_t lds = Cobg<N>::template lds_bytes<double>();
  if (hel)
    hipLaunchKernelGGL((cobg_fix_kernel<N, false>), dim3(grid), dim3(64), lds, stream, E, mom, hel,
                       Cb, scratch, count, list, me2);
  else
    hipLaunchKernelGGL((cobg_fix_kernel<N, true>), dim3(grid), dim3(64), lds, stream, E, mom, hel,
                       Cb, scratch, count, list, me2);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N>
int fix_occupancy(bool hsum) {
  int nb = 0;
  const size_t lds = Cobg<N>::template lds_bytes<double>();
  const hipError_t e =
      hsum ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cobg_fix_kernel<N, true>, 64, lds)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cobg_fix_kernel<N, false>, 64, lds);
  return e == hipSuccess ? nb : -1;
}

// Blocks per CU of the persistent (n = 7) kernel.
template <typename T, bool CHK>
int fused_occupancy(bool hsum) {
  int nb = 0;
  const size_t lds = Cobg<7>::template lds_bytes<T>();
  const hipError_t e =
      hsum ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cobg_fused_queue_kernel<T, true, CHK>, 64, lds)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cobg_fused_queue_kernel<T, false, CHK>, 64, lds);
  return e == hipSuccess ? nb : -1;
}

}  // namespace fusedk

int lc_me2(int n, bool fp32, int64_t E, const double* mom, const int8_t* hel, double* me2,
           const CheckArgs* chk, int fix_grid, hipStream_t stream) {
  if (E <= 0) return 0;
  if (chk && !fp32) return -2;
  switch (n) {
#define BG_CASE(NN)                                                                           \
  case NN:                                                                                    \
    return fp32 ? fusedk::lc_launch<NN, float>(E, mom, hel, me2, chk, fix_grid, stream)       \
                : fusedk::lc_launch<NN, double>(E, mom, hel, me2, nullptr, 0, stream);
    BG_CASE(4)
    BG_CASE(5)
    BG_CASE(6)
    BG_CASE(7)
#undef BG_CASE
    default: return -2;
  }
}

int lc_fix_blocks_per_cu(int n) {
  switch (n) {
    case 4: return fusedk::lc_fix_occupancy<4>();
    case 5: return fusedk::lc_fix_occupancy<5>();
    case 6: return fusedk::lc_fix_occupancy<6>();
    case 7: return fusedk::lc_fix_occupancy<7>();
    default: return -2;
  }
}

int cobg_fused_scratch_doubles(int n) {
  switch (n) {
    case 4: return fusedk::Cobg<4>::kScratch;
    case 5: return fusedk::Cobg<5>::kScratch;
    case 6: return fusedk::Cobg<6>::kScratch;
    case 7: return fusedk::Cobg<7>::kScratch;
    default: return 0;
  }
}

size_t cobg_lds_bytes(int n, bool fp32) {
  switch (n) {
    case 4: return fp32 ? fusedk::Cobg<4>::lds_bytes<float>() : fusedk::Cobg<4>::lds_bytes<double>();
    case 5: return fp32 ? fusedk::Cobg<5>::lds_bytes<float>() : fusedk::Cobg<5>::lds_bytes<double>();
    case 6: return fp32 ? fusedk::Cobg<6>::lds_bytes<float>() : fusedk::Cobg<6>::lds_bytes<double>();
    case 7: return fp32 ? fusedk::Cobg<7>::lds_bytes<float>() : fusedk::Cobg<7>::lds_bytes<double>();
    default: return 0;
  }
}

int cobg_fused_persistent_blocks_per_cu(bool fp32, bool hsum, bool chk) {
  if (!fp32) return fusedk::fused_occupancy<double, false>(hsum);
  return chk ? fusedk::fused_occupancy<float, true>(hsum) : fusedk::fused_occupancy<float, false>(hsum);
}

int cobg_fused_me2(int n, bool fp32, int64_t E, const double* mom, const int8_t* hel,
                   const double* Cb, double* scratch, unsigned* counter, int grid, double* me2,
                   const CheckArgs* chk, hipStream_t stream) {
  if (E <= 0) return 0;
  fusedk::TileCheck tc{};
  if (chk) tc = fusedk::TileCheck{chk->tau, chk->count, chk->list};
  const fusedk::TileCheck* tp = chk && fp32 ? &tc : nullptr;
  switch (n) {
#define BG_CASE(NN)                                                                              \
  case NN:                                                                                       \
    return fp32 ? fusedk::fused_launch<NN, float>(E, mom, hel, Cb, scratch, counter, grid, me2,  \
                                                  tp, stream)                                    \
                : fusedk::fused_launch<NN, double>(E, mom, hel, Cb, scratch, counter, grid, me2, \
                                                   nullptr, stream);
    BG_CASE(4)
    BG_CASE(5)
    BG_CASE(6)
    BG_CASE(7)
#undef BG_CASE
    default:
      return -2;
  }
}

int cobg_fix_me2(int n, int64_t E, const double* mom, const int8_t* hel, const double* Cb,
                 double* scratch, const unsigned* count, const unsigned* list, int grid,
                 double* me2, hipStream_t stream) {
  if (E <= 0) return 0;
  switch (n) {
    case 4: return fusedk::fix_launch<4>(E, mom, hel, Cb, scratch, count, list, grid, me2, stream);
    case 5: return fusedk::fix_launch<5>(E, mom, hel, Cb, scratch, count, list, grid, me2, stream);
    case 6: return fusedk::fix_launch<6>(E, mom, hel, Cb, scratch, count, list, grid, me2, stream);
    case 7: return fusedk::fix_launch<7>(E, mom, hel, Cb, scratch, count, list, grid, me2, stream);
    default: return -2;
  }
}

int cobg_fix_blocks_per_cu(int n, bool hsum) {
  switch (n) {
    case 4: return fusedk::fix_occupancy<4>(hsum);
    case 5: return fusedk::fix_occupancy<5>(hsum);
    case 6: return fusedk::fix_occupancy<6>(hsum);
    case 7: return fusedk::fix_occupancy<7>(hsum);
    default: return -1;
  }
}

// LDS of the batch kernel for one segment kind (header included).
size_t batch_lds_bytes(int kind, int n, bool fp32, bool chk) {
  if (kind == kBatchCobg) {
    size_t per_wave = 0;
    switch (n) {
#define BG_CASE(NN)                                                                          \
  case NN:                                                                                   \
    per_wave = fp32 ? fusedk::Cobg<NN>::lds_bytes<float, fusedk::BatchP64G<NN>::value>()     \
                    : fusedk::Cobg<NN>::lds_bytes<double, fusedk::BatchP64G<NN>::value>();   \
    break;
      BG_CASE(4)
      BG_CASE(5)
      BG_CASE(6)
      BG_CASE(7)
#undef BG_CASE
      default:
        return 0;
    }
    return fusedk::kBatchHeader + fusedk::kBatchWaves * per_wave;
  }
  size_t c = 0;
  switch (n) {
#define BG_CASE(NN)                                                                         \
  case NN:                                                                                  \
    c = !fp32 ? cdbgk::Lay<NN, double>::bytes()                                             \
              : (chk ? cdbgk::Lay<NN, float, true>::bytes() : cdbgk::Lay<NN, float>::bytes()); \
    break;
    BG_CASE(4)
    BG_CASE(5)
    BG_CASE(6)
    BG_CASE(7)
    BG_CASE(8)
    BG_CASE(9)
#undef BG_CASE
    default:
      return 0;
  }
  return fusedk::kBatchHeader + c;
}

int batch_scratch_doubles(int n) { return fusedk::kBatchWaves * cobg_fused_scratch_doubles(n); }

int batch_blocks_per_cu(bool fp32, int waves, int pass, int kinds, size_t lds) {
  if ((fp32 && pass == kBatchFix) || (!fp32 && pass == kBatchCheck)) return -1;
  switch (kinds) {
    case kBatchKindsAll: return batch_occupancy_kinds<kBatchKindsAll>(fp32, waves, pass, lds);
    case kBatchKindsCobg: return batch_occupancy_kinds<kBatchKindsCobg>(fp32, waves, pass, lds);
    case kBatchKindsCdbg: return batch_occupancy_kinds<kBatchKindsCdbg>(fp32, waves, pass, lds);
    default: return -1;
  }
}

int batch_launch(bool fp32, int waves, int pass, int kinds, const BatchSegTable& segs,
                 const BatchTile* tiles, unsigned t_begin, unsigned t_end,
                 const unsigned* range_dev, unsigned* counter, double* scratch,
                 int64_t scratch_stride, int grid, size_t lds, hipStream_t stream) {
  if ((fp32 && pass == kBatchFix) || (!fp32 && pass == kBatchCheck)) return -2;
  if (kinds < kBatchKindsAll || kinds > kBatchKindsCdbg) return -2;
  hipLaunchKernelGGL(fusedk::zero_counter_kernel, dim3(1), dim3(64), 0, stream, counter);
#define BG_K(KK)                                                                             \
  batch_launch_kinds<KK>(fp32, waves, pass, segs, tiles, t_begin, t_end, range_dev, counter, \
                         scratch, scratch_stride, grid, lds, stream)
  if (kinds == kBatchKindsAll) BG_K(kBatchKindsAll);
  else if (kinds == kBatchKindsCobg) BG_K(kBatchKindsCobg);
  else BG_K(kBatchKindsCdbg);
#undef BG_K
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int batch_fix_tiles(const BatchSegTable& segs, int n_segs, const unsigned* fcount,
                    BatchTile* tiles, unsigned* range, hipStream_t stream) {
  hipLaunchKernelGGL(fusedk::fix_tiles_kernel, dim3(1), dim3(256), 0, stream, segs, n_segs, fcount,
                     tiles, range);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace bg
