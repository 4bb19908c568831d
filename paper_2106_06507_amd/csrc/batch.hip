// Fused colour-ordered kernel (recursion and colour sum in one pass) and the
// persistent mixed-multiplicity batch kernel.  Tile routines: fused_impl.h.
#include "fused_impl.h"

namespace bg {
namespace fusedk {

// n <= 6: one 32-event tile per block, amplitudes in LDS; the hardware
// dispatcher balances the blocks.
template <int N, typename T, bool HSUM>
__global__ void __launch_bounds__(64) cobg_fused_kernel(int64_t E, const double* __restrict__ mom,
                                                       const int8_t* __restrict__ hel,
                                                       const double* __restrict__ Cb,
                                                       double* __restrict__ me2) {
  extern __shared__ __align__(16) unsigned char bg_fused_lds[];
  const int64_t first = (int64_t)blockIdx.x * kTileEvents;
  const int64_t left = E - first;
  cobg_tile<N, T, HSUM>(bg_fused_lds, E, mom, hel, Cb, nullptr, me2, first,
                        (int)(left < kTileEvents ? left : kTileEvents));
}

// n = 7: persistent blocks, each with its own scratch slice, take tiles from
// an atomic queue (reset by zero_counter_kernel before the launch).
template <typename T, bool HSUM>
__global__ void __launch_bounds__(64) cobg_fused_queue_kernel(int64_t E,
                                                             const double* __restrict__ mom,
                                                             const int8_t* __restrict__ hel,
                                                             const double* __restrict__ Cb,
                                                             double* __restrict__ scratch,
                                                             unsigned* __restrict__ counter,
                                                             double* __restrict__ me2) {
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
    cobg_tile<7, T, HSUM>(bg_fused_lds, E, mom, hel, Cb, blk, me2, first,
                          (int)(left < kTileEvents ? left : kTileEvents));
  }
}

__global__ void zero_counter_kernel(unsigned* c) {
  if (threadIdx.x == 0) c[0] = 0u;
}

template <int N, typename T>
__device__ __forceinline__ void run_cobg(unsigned char* lds, const BatchSeg& s, double* blk,
                                         int64_t first, int count) {
  for (int off = 0; off < count; off += kTileEvents) {
    const int c = count - off < kTileEvents ? count - off : kTileEvents;
    cobg_tile<N, T, false>(lds, s.E, s.mom, s.hel, s.Cl, blk, s.me2, first + off, c);
  }
}

template <int N, typename T>
__device__ __forceinline__ void run_cdbg(unsigned char* lds, const BatchSeg& s, int64_t first,
                                         int count) {
  for (int off = 0; off < count; off += 64) {
    const int c = count - off < 64 ? count - off : 64;
    cdbg_chunk<N, T>(lds, s.E, s.mom, s.hel, s.col, s.me2, first + off, c);
  }
}

// Persistent: each one-wave block pops tile indices from an atomic counter
// until the queue is empty (every wave reaches the exit test).  Tiles are
// ordered by decreasing estimated cost on the host.
template <typename T>
__global__ void __launch_bounds__(64) batch_kernel(const BatchSegTable segs,
                                                  const BatchTile* __restrict__ tiles,
                                                  unsigned n_tiles, unsigned* __restrict__ counter,
                                                  double* __restrict__ scratch,
                                                  int64_t scratch_stride) {
  extern __shared__ __align__(16) unsigned char bg_batch_lds[];
  double* blk = scratch + (size_t)blockIdx.x * (size_t)scratch_stride;
  for (;;) {
    unsigned t = 0;
    if (threadIdx.x == 0) t = atomicAdd(counter, 1u);
    t = (unsigned)__builtin_amdgcn_readfirstlane((int)__shfl(t, 0));
    if (t >= n_tiles) break;
    const BatchTile tile = tiles[t];
    const BatchSeg s = segs.s[tile.seg];
    switch (s.kind) {
      case kBatchCobg + 4: run_cobg<4, T>(bg_batch_lds, s, blk, tile.first, tile.count); break;
      case kBatchCobg + 5: run_cobg<5, T>(bg_batch_lds, s, blk, tile.first, tile.count); break;
      case kBatchCobg + 6: run_cobg<6, T>(bg_batch_lds, s, blk, tile.first, tile.count); break;
      case kBatchCobg + 7: run_cobg<7, T>(bg_batch_lds, s, blk, tile.first, tile.count); break;
      case kBatchCdbg + 4: run_cdbg<4, T>(bg_batch_lds, s, tile.first, tile.count); break;
      case kBatchCdbg + 5: run_cdbg<5, T>(bg_batch_lds, s, tile.first, tile.count); break;
      case kBatchCdbg + 6: run_cdbg<6, T>(bg_batch_lds, s, tile.first, tile.count); break;
      case kBatchCdbg + 7: run_cdbg<7, T>(bg_batch_lds, s, tile.first, tile.count); break;
      case kBatchCdbg + 8: run_cdbg<8, T>(bg_batch_lds, s, tile.first, tile.count); break;
      case kBatchCdbg + 9: run_cdbg<9, T>(bg_batch_lds, s, tile.first, tile.count); break;
      default: break;
    }
    __syncthreads();  // the next tile rewrites LDS
  }
}

template <int N, typename T>
int fused_launch(int64_t E, const double* mom, const int8_t* hel, const double* Cb,
                 double* scratch, unsigned* counter, int grid, double* me2, hipStream_t stream) {
  const size_t lds = Cobg<N>::template lds_bytes<T>();
  if constexpr (Cobg<N>::kLdsAmp) {
    (void)scratch;
    (void)counter;
    (void)grid;
    const unsigned tiles = (unsigned)((E + kTileEvents - 1) / kTileEvents);
    if (hel)
      hipLaunchKernelGGL((cobg_fused_kernel<N, T, false>), dim3(tiles), dim3(64), lds, stream, E,
                         mom, hel, Cb, me2);
    else
      hipLaunchKernelGGL((cobg_fused_kernel<N, T, true>), dim3(tiles), dim3(64), lds, stream, E,
                         mom, hel, Cb, me2);
  } else {
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, stream, counter);
    if (hel)
      hipLaunchKernelGGL((cobg_fused_queue_kernel<T, false>), dim3(grid), dim3(64), lds, stream,
                         E, mom, hel, Cb, scratch, counter, me2);
    else
      hipLaunchKernelGGL((cobg_fused_queue_kernel<T, true>), dim3(grid), dim3(64), lds, stream,
                         E, mom, hel, Cb, scratch, counter, me2);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Blocks per CU of the persistent (n = 7) kernel.
template <typename T>
int fused_occupancy(bool hsum) {
  int nb = 0;
  const size_t lds = Cobg<7>::template lds_bytes<T>();
  const hipError_t e =
      hsum ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cobg_fused_queue_kernel<T, true>, 64, lds)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cobg_fused_queue_kernel<T, false>, 64, lds);
  return e == hipSuccess ? nb : -1;
}

}  // namespace fusedk

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

int cobg_fused_persistent_blocks_per_cu(bool fp32, bool hsum) {
  return fp32 ? fusedk::fused_occupancy<float>(hsum) : fusedk::fused_occupancy<double>(hsum);
}

int cobg_fused_me2(int n, bool fp32, int64_t E, const double* mom, const int8_t* hel,
                   const double* Cb, double* scratch, unsigned* counter, int grid, double* me2,
                   hipStream_t stream) {
  if (E <= 0) return 0;
  switch (n) {
#define BG_CASE(NN)                                                                              \
  case NN:                                                                                       \
    return fp32 ? fusedk::fused_launch<NN, float>(E, mom, hel, Cb, scratch, counter, grid, me2,  \
                                                  stream)                                        \
                : fusedk::fused_launch<NN, double>(E, mom, hel, Cb, scratch, counter, grid, me2, \
                                                   stream);
    BG_CASE(4)
    BG_CASE(5)
    BG_CASE(6)
    BG_CASE(7)
#undef BG_CASE
    default:
      return -2;
  }
}

int batch_blocks_per_cu(bool fp32, size_t lds) {
  int nb = 0;
  hipError_t e = fp32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &nb, fusedk::batch_kernel<float>, 64, lds)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &nb, fusedk::batch_kernel<double>, 64, lds);
  return e == hipSuccess ? nb : -1;
}

int batch_launch(bool fp32, const BatchSegTable& segs, const BatchTile* tiles, unsigned n_tiles,
                 unsigned* counter, double* scratch, int64_t scratch_stride, int grid, size_t lds,
                 hipStream_t stream) {
  hipLaunchKernelGGL(fusedk::zero_counter_kernel, dim3(1), dim3(64), 0, stream, counter);
  if (fp32)
    hipLaunchKernelGGL(fusedk::batch_kernel<float>, dim3(grid), dim3(64), lds, stream, segs, tiles,
                       n_tiles, counter, scratch, scratch_stride);
  else
    hipLaunchKernelGGL(fusedk::batch_kernel<double>, dim3(grid), dim3(64), lds, stream, segs,
                       tiles, n_tiles, counter, scratch, scratch_stride);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace bg
