// Persistent mixed-multiplicity batch kernel.  One template, instantiated per
// set of segment kinds it may meet (batch_kinds_all.hip, batch_kinds_cobg.hip,
// batch_kinds_cdbg.hip): a kernel that only ever runs colour-dressed tiles is
// compiled without the colour-ordered branches, so its register allocation
// and LDS are those of the dressed recursion alone.  Tile routines:
// fused_impl.h.
#pragma once

#include "fused_impl.h"

namespace bg {
namespace fusedk {

// Batch blocks: four waves.  A colour-ordered tile is split into 32-event
// sub-tiles, wave w taking sub-tiles w, w + 4, ... with its own LDS region and
// scratch slice; every wave runs the same number of rounds (a wave without a
// sub-tile evaluates a stand-in event and stores nothing), because the tile
// routine synchronises the block.  A colour-dressed tile is evaluated by all
// the block's lanes (256; 128 in the FP32 dressed-only kernel), one valid
// event at a time.  LDS: a 64-byte header (validity
// masks, tile broadcast) followed by the tile region.
constexpr int kBatchWaves = 4;
constexpr int kBatchLanes = 64 * kBatchWaves;
constexpr size_t kBatchHeader = 64;

// Lanes per block: 256, except the FP32 dressed-only kernel, which runs one
// event on 128 lanes (two waves), so that twice as many events are in flight
// per CU within the same LDS (measured best for FP32 dressed events alone).
template <typename T, int KINDS>
struct BatchLanes {
  static constexpr int value = (KINDS == kBatchKindsCdbg && sizeof(T) == 4) ? 128 : kBatchLanes;
};

// n >= 6 re-read FP64 momenta from global memory so that four waves of
// colour-ordered tiles fit in the LDS of one block.
template <int N>
struct BatchP64G {
  static constexpr bool value = N >= 6;
};

template <int N, typename T, int PASS>
__device__ __forceinline__ void run_cobg(unsigned char* lds, const BatchSeg& s, double* blk,
                                         int64_t first, int count) {
  constexpr bool G = BatchP64G<N>::value;
  const int w = threadIdx.x >> 6;
  unsigned char* mine = lds + (size_t)w * Cobg<N>::template lds_bytes<T, G>();
  double* myblk = blk + (size_t)w * Cobg<N>::kScratch;
  const int nsub = (count + kTileEvents - 1) / kTileEvents;
  for (int i = 0; i < nsub; i += kBatchWaves) {
    const int j = i + w;
    const int off = j * kTileEvents;
    const int c = j < nsub ? (count - off < kTileEvents ? count - off : kTileEvents) : 0;
    const int64_t f = first + (j < nsub ? off : 0);
    if constexpr (PASS == kBatchFix)
      cobg_tile<N, T, false, G, false, true>(mine, s.E, s.mom, s.hel, s.Cl, myblk, s.me2, f, c,
                                             TileCheck{}, s.idx);
    else if constexpr (PASS == kBatchCheck)
      cobg_tile<N, T, false, G, true>(mine, s.E, s.mom, s.hel, s.Cl, myblk, s.me2, f, c,
                                      TileCheck{s.tau, s.fcount, s.flist});
    else
      cobg_tile<N, T, false, G>(mine, s.E, s.mom, s.hel, s.Cl, myblk, s.me2, f, c);
  }
}

template <int N, typename T, int PASS, int NL>
__device__ __forceinline__ void run_cdbg(unsigned char* lds, unsigned long long* vmask,
                                         const BatchSeg& s, int64_t first, int count) {
  for (int off = 0; off < count; off += NL) {
    const int c = count - off < NL ? count - off : NL;
    cdbg_chunk<N, T, NL, PASS>(lds, vmask, s.E, s.mom, s.hel, s.col, s.me2, first + off,
                                        c, s.idx, cdbgk::DressedCheck{s.tau, s.fcount, s.flist});
  }
}

// Persistent: each block pops tile indices from an atomic counter (reset to 0
// before the launch) until the queue [begin, end) is empty (every block
// reaches the exit test).  The range is [t_begin, t_end), or read on the
// device from range_dev[0..1] when range_dev is given (the re-evaluation
// pass, whose tiles are built on the device).  Tiles are ordered by
// decreasing estimated cost on the host.
// WAVES: minimum waves per SIMD the register allocation must allow.  1: the
// largest branch (n = 7 colour-ordered) keeps all its registers and one
// block fits on a CU; 2: at most 256 registers per lane, two blocks per CU
// (the n = 7 colour-ordered branch spills a little).  KINDS (BatchKinds):
// the segment kinds this instance evaluates; tiles of another kind are
// skipped.  PASS: BatchPass.
template <typename T, int WAVES, int PASS, int KINDS>
__global__ void __launch_bounds__((BatchLanes<T, KINDS>::value), WAVES) batch_kernel(
                                                           const BatchSegTable segs,
                                                           const BatchTile* __restrict__ tiles,
                                                           unsigned t_begin, unsigned t_end,
                                                           const unsigned* __restrict__ range_dev,
                                                           unsigned* __restrict__ counter,
                                                           double* __restrict__ scratch,
                                                           int64_t scratch_stride) {
  extern __shared__ __align__(16) unsigned char bg_batch_lds[];
  unsigned long long* vmask = reinterpret_cast<unsigned long long*>(bg_batch_lds);
  unsigned* bcast = reinterpret_cast<unsigned*>(bg_batch_lds + 32);
  unsigned char* lds = bg_batch_lds + kBatchHeader;
  double* blk = scratch + (size_t)blockIdx.x * (size_t)scratch_stride;
  const unsigned begin = range_dev ? range_dev[0] : t_begin;
  const unsigned end = range_dev ? range_dev[1] : t_end;
  for (;;) {
    if (threadIdx.x == 0) bcast[0] = atomicAdd(counter, 1u);
    __syncthreads();
    const unsigned k = (unsigned)__builtin_amdgcn_readfirstlane((int)bcast[0]);
    __syncthreads();  // every lane has the index before the next pop
    if (k >= end - begin) break;
    const BatchTile tile = tiles[begin + k];
    const BatchSeg s = segs.s[tile.seg];
    constexpr bool kCo = KINDS != kBatchKindsCdbg, kCd = KINDS != kBatchKindsCobg;
    switch (s.kind) {
#define BG_CO(NN)                                                                       \
  case kBatchCobg + NN:                                                                 \
    if constexpr (kCo) run_cobg<NN, T, PASS>(lds, s, blk, tile.first, tile.count);      \
    break;
#define BG_CD(NN)                                                                       \
  case kBatchCdbg + NN:                                                                 \
    if constexpr (kCd)                                                                  \
      run_cdbg<NN, T, PASS, BatchLanes<T, KINDS>::value>(lds, vmask, s, tile.first,      \
                                                         tile.count);                    \
    break;
      BG_CO(4) BG_CO(5) BG_CO(6) BG_CO(7)
      BG_CD(4) BG_CD(5) BG_CD(6) BG_CD(7) BG_CD(8) BG_CD(9)
#undef BG_CO
#undef BG_CD
      default: break;
    }
    __syncthreads();  // the next tile rewrites LDS
  }
}

template <typename T, int WAVES, int PASS, int KINDS>
int occupancy_of(size_t lds) {
  int nb = 0;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel<T, WAVES, PASS, KINDS>,
                                                      BatchLanes<T, KINDS>::value,
                                                      lds) == hipSuccess
             ? nb
             : -1;
}

// FP32 plain and checked, FP64 plain and re-evaluation.
template <int WAVES, int KINDS>
int occupancy_pass(bool fp32, int pass, size_t lds) {
  if (fp32)
    return pass == kBatchCheck ? occupancy_of<float, WAVES, kBatchCheck, KINDS>(lds)
                               : occupancy_of<float, WAVES, kBatchPlain, KINDS>(lds);
  return pass == kBatchFix ? occupancy_of<double, WAVES, kBatchFix, KINDS>(lds)
                           : occupancy_of<double, WAVES, kBatchPlain, KINDS>(lds);
}

template <int WAVES, int KINDS>
void launch_pass(bool fp32, int pass, const BatchSegTable& segs, const BatchTile* tiles,
                 unsigned t_begin, unsigned t_end, const unsigned* range_dev, unsigned* counter,
                 double* scratch, int64_t scratch_stride, int grid, size_t lds,
                 hipStream_t stream) {
#define BG_L(TT, PP)                                                                          \
  hipLaunchKernelGGL((batch_kernel<TT, WAVES, PP, KINDS>), dim3(grid),                        \
                     dim3(BatchLanes<TT, KINDS>::value), lds,                                  \
                     stream, segs, tiles, t_begin, t_end, range_dev, counter, scratch,          \
                     scratch_stride)
  if (fp32) {
    if (pass == kBatchCheck) BG_L(float, kBatchCheck); else BG_L(float, kBatchPlain);
  } else {
    if (pass == kBatchFix) BG_L(double, kBatchFix); else BG_L(double, kBatchPlain);
  }
#undef BG_L
}

}  // namespace fusedk

// Colour-dressed-only instances exist for the two-waves budget only (the
// dressed branches need fewer than 256 registers per lane).
template <int KINDS>
int batch_occupancy_kinds(bool fp32, int waves, int pass, size_t lds) {
  if constexpr (KINDS != kBatchKindsCdbg) {
    if (waves == 1) return fusedk::occupancy_pass<1, KINDS>(fp32, pass, lds);
  }
  return fusedk::occupancy_pass<2, KINDS>(fp32, pass, lds);
}

template <int KINDS>
void batch_launch_kinds(bool fp32, int waves, int pass, const BatchSegTable& segs,
                        const BatchTile* tiles, unsigned t_begin, unsigned t_end,
                        const unsigned* range_dev, unsigned* counter, double* scratch,
                        int64_t scratch_stride, int grid, size_t lds, hipStream_t stream) {
  if constexpr (KINDS != kBatchKindsCdbg) {
    if (waves == 1) {
      fusedk::launch_pass<1, KINDS>(fp32, pass, segs, tiles, t_begin, t_end, range_dev, counter,
                                    scratch, scratch_stride, grid, lds, stream);
      return;
    }
  }
  fusedk::launch_pass<2, KINDS>(fp32, pass, segs, tiles, t_begin, t_end, range_dev, counter,
                                scratch, scratch_stride, grid, lds, stream);
}

}  // namespace bg
