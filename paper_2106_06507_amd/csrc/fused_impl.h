// Tile routines shared by the fused colour-ordered kernel and the persistent
// mixed-multiplicity batch kernel.
//
// Colour-ordered tile (n <= 7): 32 events on one 64-lane wave (lane pairs, as
// in cobg_pair_impl.h).  The (n-2)! partial amplitudes of the tile are staged
// as [2][K][32] (real and imaginary planes; where, see Cobg); then each lane
// forms the colour sum (eq. color_summed_analytic) of its plane,
//   q_h = a_h^T C a_h,  a_0 = Re A, a_1 = Im A,   |M|^2 = q_0 + q_1,
// with C given as its lower triangle with doubled off-diagonal entries (the
// same quadratic form for symmetric C at half the products), stored in row
// blocks (see lower_quadform).  A lane reads
// back only the amplitudes it wrote itself, so no cross-lane exchange of
// amplitudes is needed; the pair partner adds the other plane with one DPP
// move.  Without helicities the tile loops over all 2^n configurations and
// sums.
//
// Colour-dressed chunk (n >= 8 in the batch): up to 256 consecutive events
// are classified one per lane (closed colour circuit, as in cdbg_impl.h);
// invalid ones get exactly 0 and the valid ones are evaluated one at a time by
// all lanes of the block.
#pragma once

#include <stdint.h>

#include "cdbg_impl.h"
#include "cobg_pair_impl.h"
#include "cobg_path_impl.h"

namespace bg {
namespace fusedk {

constexpr int kTileEvents = 32;  // events per colour-ordered sub-tile (one per lane pair)

// Where a tile keeps its amplitudes: up to n = 6 in LDS, unscaled, in the
// recursion's type (at most 12 KB); at n = 7 (K = 120) in a block-private
// FP64 scratch slice of device memory, which stays in L2 because the block
// reuses it for every tile it takes.  The amplitudes come from the
// depth-first walk, except FP64 at n = 7: one straight path per ordering.
template <int N>
struct Cobg {
  static constexpr int K = (int)Factorial<N - 2>::value;
  static constexpr bool kLdsAmp = N <= 6;
  static constexpr int kScratch = kLdsAmp ? 0 : 2 * K * kTileEvents;  // doubles per block
  template <typename T, bool P64G = false>
  static constexpr size_t lds_bytes() {
    return pairk::Lds<N>::template bytes<T, P64G>() +
           (kLdsAmp ? sizeof(T) * 2 * (size_t)K * kTileEvents : 0);
  }
};

// Row block of the colour quadratic form (divides K = (n-2)!).
template <int K>
struct RowBlock {
  static constexpr int value = K < 8 ? K : 8;
};

// a^T C a for symmetric C given as its doubled lower triangle in row blocks:
// for row block b (rows b RB .. b RB + RB - 1) and every column
// j < (b + 1) RB the RB entries L[b RB + r][j], r = 0..RB-1, are contiguous,
// where L = 2 C below the diagonal, C on it and 0 above.  One scalar load of
// RB entries then serves the RB products of one loaded a_j.  a[j] is read at
// a[j * stride].
template <int K, typename A>
__device__ __forceinline__ double lower_quadform(const double* __restrict__ Cb, const A* a,
                                                 int stride) {
  constexpr int RB = RowBlock<K>::value;
  static_assert(K % RB == 0, "row block must divide K");
  double q = 0.0;
  const double* cb = Cb;
#pragma unroll 1
  for (int ib = 0; ib < K; ib += RB) {
    double y[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) y[r] = 0.0;
    const int jend = ib + RB;
#pragma unroll 2
    for (int j = 0; j < jend; ++j) {
      const double aj = (double)a[j * stride];
#pragma unroll
      for (int r = 0; r < RB; ++r) y[r] += cb[j * RB + r] * aj;
    }
    cb += jend * RB;
#pragma unroll
    for (int r = 0; r < RB; ++r) q += (double)a[(ib + r) * stride] * y[r];
  }
  return q;
}

// Re-evaluation of ill-conditioned events.  The FP32 pass (CHK) bounds,
// per event, the rounding error of its amplitudes relative to their size
// (pairk::State::Sb): the square of that bound is est = sum_sigma Sb_sigma^2 /
// sum_sigma |A_sigma|^2.  Events with est > tau (helicity configurations
// whose tree amplitude vanishes identically excepted: their |M|^2 is rounding
// noise at any precision) are appended to a list; a second pass in FP64 (IDX)
// evaluates the listed events again and overwrites their |M|^2.
struct TileCheck {
  float tau;          // threshold on est
  unsigned* count;    // number of listed events (device; zeroed before the FP32 pass)
  unsigned* list;     // listed event indices
};

// Appends the events of the lanes with f set to chk.list (one atomic per wave).
__device__ __forceinline__ void flag_events(bool f, unsigned e, const TileCheck& chk) {
  const unsigned long long m = __ballot(f);
  if (m == 0ull) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)m) - 1;
  unsigned base = 0u;
  if (lane == leader) base = atomicAdd(chk.count, (unsigned)__popcll(m));
  base = (unsigned)__shfl((int)base, leader);
  if (f) chk.list[base + (unsigned)__popcll(m & ((1ull << lane) - 1ull))] = e;
}

// Colour-summed |M|^2 of events [first, first + count) (0 <= count <= 32,
// event `first` must exist) of an [n][4][E] input, on one wave.  HSUM: sum
// over all 2^n helicity configurations (hel is ignored); otherwise one
// configuration per event from hel.  lds is the wave's Cobg<N>::lds_bytes<T>();
// blk its scratch slice (n = 7 only).  CHK: flag ill-conditioned events into
// chk (see TileCheck).  IDX: the events are idx[first .. first + count - 1]
// instead (idx[first] must exist).
template <int N, typename T, bool HSUM, bool P64G = false, bool CHK = false, bool IDX = false>
__device__ __forceinline__ void cobg_tile(unsigned char* lds, int64_t E,
                                          const double* __restrict__ mom,
                                          const int8_t* __restrict__ hel,
                                          const double* __restrict__ Cb, double* blk,
                                          double* __restrict__ me2, int64_t first, int count,
                                          TileCheck chk = TileCheck{},
                                          const unsigned* __restrict__ idx = nullptr) {
  constexpr int K = Cobg<N>::K;
  constexpr bool kL = Cobg<N>::kLdsAmp;
  T* amp_lds = reinterpret_cast<T*>(lds + pairk::Lds<N>::template bytes<T, P64G>());
  const int lane = threadIdx.x & 63;
  const int pair = lane >> 1;
  const int h = lane & 1;
  // count = 0: a wave without events in this round still takes part in the
  // block's barriers, evaluating event `first` without storing it
  const bool live = pair < count;
  const int64_t slot = first + (live ? pair : (count > 0 ? count - 1 : 0));
  int64_t e = IDX ? (int64_t)idx[slot] : slot;
  T est[2] = {T(0), T(0)};
  auto one = [&](const int8_t* hp, int hc) -> double {
    if constexpr (kL) {
      pairk::cobg_pair_body<N, T, true, P64G, false, CHK>(lds, E, mom, hp, hc, e, true, nullptr,
                                                          0, 0, amp_lds, est);
      return lower_quadform<K>(Cb, amp_lds + (size_t)h * K * kTileEvents + pair, kTileEvents);
    } else {
      if constexpr (sizeof(T) == 8) {
        // FP64 n = 7: one straight path per ordering (cobg_path_impl.h); the
        // walk's FP64 state does not fit the registers there (FP32: the
        // walk, 13% fewer vertices, is faster)
        static_assert(pathk::Lds<N>::template bytes<T>() <=
                          pairk::Lds<N>::template bytes<T, P64G>(),
                      "the path's LDS fits the wave's region");
        pathk::cobg_path_body<N, T, CHK>(lds, E, mom, hp, hc, e, true, blk, kTileEvents, pair,
                                         est);
      } else {
        pairk::cobg_pair_body<N, T, false, P64G, false, CHK>(lds, E, mom, hp, hc, e, true, blk,
                                                             kTileEvents, pair, nullptr, est);
      }
      return lower_quadform<K>(Cb, blk + (size_t)h * K * kTileEvents + pair, kTileEvents);
    }
  };
  double q = 0.0;
  if constexpr (HSUM) {
    for (int hc = 0; hc < (1 << N); ++hc) {
      // keep the momentum loads inside the loop: hoisting them would hold
      // 4n FP64 values live through the whole recursion
      asm volatile("" : "+v"(e));
      q += one(nullptr, hc);
      __syncthreads();  // the next configuration rewrites LDS and scratch
    }
  } else {
    q = one(hel, 0);
    __syncthreads();
  }
  if constexpr (kL) {
    double scale = 1.0;  // (g_s / sqrt2)^(n-2), squared: the amplitudes were stored unscaled
#pragma unroll
    for (int i = 0; i < N - 2; ++i) scale *= kGsOverSqrt2;
    q *= scale * scale;
  }
  const double tot = pairk::pair_sum(q);
  if (live && h == 0) me2[e] = tot;
  if constexpr (CHK) {
    bool f = false;
    if (live && h == 0) {
      bool vanishing = false;
      if constexpr (!HSUM) {
        int neg = 0;
#pragma unroll
        for (int i = 0; i < N; ++i) neg += hel[(int64_t)i * E + e] < 0 ? 1 : 0;
        vanishing = neg < 2 || neg > N - 2;
      }
      // the negated test also lists events whose estimate is not a number
      f = !vanishing && !(est[0] <= chk.tau * est[1]);
    }
    flag_events(f, (unsigned)e, chk);
  }
}

// Leading-colour |M|^2 (Section 3.1): N^(n-2) (N^2 - 1) sum over all (n-1)!
// orderings (1, rho) of |A(1, rho)|^2, N = 3, for events [first, first +
// count) (count <= 32), one helicity configuration per event.  lds holds
// pairk::Lds<N, true>::bytes<T>().  CHK: list the events whose
// sum_rho S_rho^2 > tau sum_rho |A_rho|^2 (running error bounds of the
// orderings' top currents; helicity configurations that vanish identically
// are never listed).  IDX: the events are idx[first .. first + count - 1].
template <int N, typename T, bool CHK = false, bool IDX = false>
__device__ __forceinline__ void lc_tile(unsigned char* lds, int64_t E,
                                        const double* __restrict__ mom,
                                        const int8_t* __restrict__ hel, double* __restrict__ me2,
                                        int64_t first, int count, TileCheck chk = TileCheck{},
                                        const unsigned* __restrict__ idx = nullptr) {
  const int lane = threadIdx.x & 63;
  const int pair = lane >> 1;
  const int h = lane & 1;
  const bool live = pair < count;
  const int64_t slot = first + (live ? pair : (count > 0 ? count - 1 : 0));
  const int64_t e = IDX ? (int64_t)idx[slot] : slot;
  T est[2] = {T(0), T(0)};
  const double q = pairk::cobg_pair_body<N, T, false, false, true, CHK>(
      lds, E, mom, hel, 0, e, false, nullptr, 0, 0, nullptr, est);
  __syncthreads();
  double scale = 1.0;  // (g_s / sqrt2)^(n-2) per amplitude, squared
#pragma unroll
  for (int i = 0; i < N - 2; ++i) scale *= kGsOverSqrt2;
  double colour = 8.0;  // N^(n-2) (N^2 - 1)
#pragma unroll
  for (int i = 0; i < N - 2; ++i) colour *= 3.0;
  const double tot = pairk::pair_sum(q) * scale * scale * colour;
  if (live && h == 0) me2[e] = tot;
  if constexpr (CHK) {
    bool f = false;
    if (live && h == 0) {
      int neg = 0;
#pragma unroll
      for (int i = 0; i < N; ++i) neg += hel[(int64_t)i * E + e] < 0 ? 1 : 0;
      // the negated test also lists events whose estimate is not a number
      f = neg >= 2 && neg <= N - 2 && !(est[0] <= chk.tau * est[1]);
    }
    flag_events(f, (unsigned)e, chk);
  }
}

// Colour-dressed |A|^2 of events [first, first + count), count <= NL, on
// the NL lanes of the block: one lane classifies each event (invalid flows
// get exactly 0), then the valid ones are evaluated in order by all lanes.
// vmask: NL/64 words of LDS for the validity masks.  PASS (BatchPass):
// kBatchCheck lists ill-conditioned events into chk; kBatchFix takes the
// events idx[first .. first + count - 1] instead.
template <int N, typename T, int NL, int PASS = kBatchPlain>
__device__ __forceinline__ void cdbg_chunk(unsigned char* lds, unsigned long long* vmask, int64_t E,
                                           const double* __restrict__ mom,
                                           const int8_t* __restrict__ hel,
                                           const int8_t* __restrict__ col,
                                           double* __restrict__ me2, int64_t first, int count,
                                           const unsigned* __restrict__ idx = nullptr,
                                           cdbgk::DressedCheck chk = cdbgk::DressedCheck{}) {
  constexpr bool kEst = PASS == kBatchCheck;
  const cdbgk::Sm<N, T> sm = cdbgk::carve<N, T, kEst>(lds);
  const int t = threadIdx.x;
  bool valid = false;
  if (t < count) {
    const int64_t ev = PASS == kBatchFix ? (int64_t)idx[first + t] : first + t;
    valid = cdbgk::flow_valid(N, E, col, ev);
    if (!valid) me2[ev] = 0.0;
  }
  const unsigned long long m = __ballot(valid);
  if ((t & 63) == 0) vmask[t >> 6] = m;
  __syncthreads();
  for (int w = 0; w < NL / 64; ++w) {
    unsigned long long mm = vmask[w];
    while (mm) {
      const int l = __builtin_ctzll(mm);
      mm &= mm - 1;
      const int64_t ev = PASS == kBatchFix ? (int64_t)idx[first + 64 * w + l] : first + 64 * w + l;
      cdbgk::cdbg_one_event<N, T, NL, kEst>(sm, E, mom, hel, col, ev, me2, chk);
    }
  }
  __syncthreads();  // vmask is rewritten by the next chunk
}

}  // namespace fusedk
}  // namespace bg
