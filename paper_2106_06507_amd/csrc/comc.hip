// Colour-sampled colour-ordered evaluation (Section 2.2,
// eq. color_decomposition_colorflow, with the colour-ordered amplitudes of
// Section 2.3): for one colour-flow assignment per event,
//   A = sum over orderings (1, sigma) of Tr(E_1 E_sigma2 ... E_sigman) A(1, sigma),
// E_k = e_{j_k i_k}.  The trace is 1 when the delta chain closes
// (i_prev = j_next along the ordering and i_last = j_1) and 0 otherwise, so
// only the closing orderings (the Euler circuits of the colour edges that
// start with gluon 1) are evaluated.
//
// Passes: (1) one thread per event classifies the flow and counts its closing
// orderings (depth-first over the colour chain; invalid flows get exactly 0),
// (2) one block scans the per-block counts, (3) one thread per event writes
// its (event, ordering) items at their ranks, (4) one lane pair per item
// evaluates A(1, sigma) with the lane-pair recursion of cobg_pair_impl.h on
// that single ordering (gluons of the ordering differ between pairs; 1/P^2
// from the FP64 prefix momenta), (5) one thread per event adds its items'
// amplitudes in order and writes |A|^2.  The item count is read back once
// (a synchronisation) to size the item arrays.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cdbg_impl.h"
#include "cobg_pair_impl.h"

namespace bg {
namespace comck {

using pairk::Cx;
using pairk::H;
using pairk::HR;

constexpr int kThreads = 256;

// colours packed two bits per gluon
template <int N>
struct Flow {
  int ci, cj;
  __device__ __forceinline__ int i(int g) const { return (ci >> (2 * g)) & 3; }
  __device__ __forceinline__ int j(int g) const { return (cj >> (2 * g)) & 3; }
};

template <int N>
__device__ __forceinline__ Flow<N> load_flow(int64_t E, const int8_t* __restrict__ col, int64_t e) {
  Flow<N> f{0, 0};
#pragma unroll
  for (int k = 0; k < N; ++k) {
    f.ci |= ((int)col[(int64_t)k * E + e] & 3) << (2 * k);
    f.cj |= ((int)col[((int64_t)N + k) * E + e] & 3) << (2 * k);
  }
  return f;
}

// Closing orderings: position D (1 .. N-1) takes an unused gluon g with
// j_g = i of the previous gluon; after position N-1, i_last must equal j_0.
// visit(code) with nibble D-1 of code = gluon at position D.
template <int N, int D, class V>
__device__ __forceinline__ void orderings(const Flow<N>& f, int used, int prev, uint32_t code,
                                          V& visit) {
  if constexpr (D == N) {
    if (f.i(prev) == f.j(0)) visit(code);
  } else {
    for (int g = 1; g < N; ++g) {
      if ((used >> g) & 1) continue;
      if (f.j(g) != f.i(prev)) continue;
      orderings<N, D + 1>(f, used | (1 << g), g, code | ((uint32_t)g << (4 * (D - 1))), visit);
    }
  }
}

// Pass 1
template <int N>
__global__ void __launch_bounds__(kThreads) count_kernel(int64_t E, const int8_t* __restrict__ col,
                                                        double* __restrict__ me2,
                                                        unsigned* __restrict__ counts,
                                                        uint64_t* __restrict__ block_count) {
  __shared__ unsigned part[kThreads];
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  unsigned c = 0;
  if (e < E) {
    if (cdbgk::flow_valid(N, E, col, e)) {
      const Flow<N> f = load_flow<N>(E, col, e);
      auto visit = [&](uint32_t) { ++c; };
      orderings<N, 1>(f, 1, 0, 0u, visit);
    }
    if (c == 0) me2[e] = 0.0;  // no closing ordering: the flow's amplitude is 0
    counts[e] = c;
  }
  part[threadIdx.x] = c;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) block_count[blockIdx.x] = part[0];
}

// Pass 2: exclusive scan of the block counts in place (one block); total at
// block_count[n_blocks].
__global__ void __launch_bounds__(1024) scan_kernel(uint64_t* __restrict__ block_count,
                                                    int n_blocks) {
  __shared__ uint64_t part[1024];
  const int t = threadIdx.x;
  const int per = (n_blocks + 1023) / 1024;
  const int lo = t * per;
  const int hi = lo + per < n_blocks ? lo + per : n_blocks;
  uint64_t s = 0;
  for (int k = lo; k < hi; ++k) s += block_count[k];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off *= 2) {
    const uint64_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint64_t run = part[t] - s;
  for (int k = lo; k < hi; ++k) {
    const uint64_t c = block_count[k];
    block_count[k] = run;
    run += c;
  }
  if (t == 1023) block_count[n_blocks] = part[1023];
}

// Pass 3: items (event << 32 | ordering code) at their ranks; the event's
// first item index goes to offsets[e].
template <int N>
__global__ void __launch_bounds__(kThreads) items_kernel(int64_t E, const int8_t* __restrict__ col,
                                                        const unsigned* __restrict__ counts,
                                                        const uint64_t* __restrict__ block_offset,
                                                        unsigned* __restrict__ offsets,
                                                        uint64_t* __restrict__ items) {
  __shared__ unsigned part[kThreads];
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const unsigned c = e < E ? counts[e] : 0u;
  part[threadIdx.x] = c;
  __syncthreads();
  for (int off = 1; off < kThreads; off *= 2) {
    const unsigned v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  if (e >= E) return;
  // the host admits only totals below 2^31, so the rank fits 32 bits
  const unsigned first = (unsigned)(block_offset[blockIdx.x] + part[threadIdx.x] - c);
  offsets[e] = first;
  if (c == 0) return;
  const Flow<N> f = load_flow<N>(E, col, e);
  unsigned k = first;
  auto visit = [&](uint32_t code) { items[k++] = ((uint64_t)e << 32) | code; };
  orderings<N, 1>(f, 1, 0, 0u, visit);
}

// Per-lane context for one ordering (see pairk::Ctx; 1/P^2 computed from the
// prefix momenta, V4 dot products recomputed when the Dt table would not fit
// in registers).
template <int N, typename T, bool NODT>
struct Ctx {
  static constexpr bool kRaw = false, kP64G = false, kLC = false;
  static constexpr bool kDirectP2 = true;
  static constexpr bool kNoDt = NODT;
  T* gl_slots;   // [6 (g-1) + x][lane]
  double* p64;   // [2 (g-1) + c][lane]
  T* tab;        // unused
  int lane, pair, h;
  T g0;
  H<T> epsN;
};

template <int N, typename T, int D, class C>
__device__ __forceinline__ void path(pairk::State<N, T>& s, C& c, uint32_t code, Cx<T>& top) {
  constexpr int M = N - 1;
  const int g = (int)((code >> (4 * (D - 1))) & 15u);
  s.gl[D] = g;
  const int base = 6 * (g - 1);
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    s.J[D][D].re[m] = c.gl_slots[(base + m) * 64 + c.lane];
    s.J[D][D].im[m] = c.gl_slots[(base + 2 + m) * 64 + c.lane];
    s.Pg[D].v[m] = c.gl_slots[(base + 4 + m) * 64 + c.lane];
    s.P0[D].v[m] = s.P0[D - 1].v[m] + c.p64[(2 * (g - 1) + m) * 64 + c.lane];
  }
  if constexpr (D == M - 1) {
    // the ordering's last gluon closes it
    const int gl = (int)((code >> (4 * (N - 2))) & 15u);
    const int lb = 6 * (gl - 1);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      c.epsN.re[m] = c.gl_slots[(lb + m) * 64 + c.lane];
      c.epsN.im[m] = c.gl_slots[(lb + 2 + m) * 64 + c.lane];
    }
  }
  pairk::build_column<N, T, D, D - 1>(s, c, 0, top);
  if constexpr (D < M - 1) path<N, T, D + 1>(s, c, code, top);
}

template <int N>
struct AmpLds {
  template <typename T>
  static constexpr size_t bytes() {
    return sizeof(T) * (size_t)6 * (N - 1) * 64 + sizeof(double) * (size_t)2 * (N - 1) * 64;
  }
};

// Pass 4: persistent blocks over 32-item tiles; amp[2 item + h] = plane h
// of A(1, sigma) including the couplings.
template <int N, typename T, bool NODT>
__global__ void __launch_bounds__(64) amp_kernel(int64_t E, const double* __restrict__ mom,
                                                const int8_t* __restrict__ hel,
                                                const uint64_t* __restrict__ items,
                                                const uint64_t* __restrict__ total_p,
                                                double* __restrict__ amp) {
  extern __shared__ __align__(16) unsigned char bg_comc_lds[];
  const unsigned total = (unsigned)*total_p;  // below 2^31 (host check)
  const int lane = threadIdx.x;
  const int pair = lane >> 1, h = lane & 1;
  const bool hi = h != 0;
  Ctx<N, T, NODT> c;
  c.gl_slots = reinterpret_cast<T*>(bg_comc_lds);
  c.p64 = reinterpret_cast<double*>(c.gl_slots + (size_t)6 * (N - 1) * 64);
  c.tab = nullptr;
  c.lane = lane;
  c.pair = pair;
  c.h = h;
  c.g0 = h == 0 ? T(1) : T(-1);
  double scale = 1.0;
#pragma unroll
  for (int i = 0; i < N - 2; ++i) scale *= kGsOverSqrt2;
  for (unsigned base = blockIdx.x * 32u; base < total; base += gridDim.x * 32u) {
    const unsigned it = base + pair < total ? base + pair : total - 1;
    const uint64_t item = items[it];
    const int64_t e = (int64_t)(item >> 32);
    const uint32_t code = (uint32_t)item;
    pairk::State<N, T> s;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double p[4], er[4], ei[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) p[m] = mom[((int64_t)i * 4 + m) * E + e];
      polarization(p, (int)hel[(int64_t)i * E + e], er, ei);
      T v[6];
      double ph[2];
      if (hi) {
        v[0] = (T)er[2]; v[1] = (T)er[3]; v[2] = (T)ei[2]; v[3] = (T)ei[3];
        ph[0] = p[2]; ph[1] = p[3];
      } else {
        v[0] = (T)er[0]; v[1] = (T)er[1]; v[2] = (T)ei[0]; v[3] = (T)ei[1];
        ph[0] = p[0]; ph[1] = p[1];
      }
      v[4] = (T)ph[0];
      v[5] = (T)ph[1];
      if (i == 0) {
        s.J[0][0].re[0] = v[0];
        s.J[0][0].re[1] = v[1];
        s.J[0][0].im[0] = v[2];
        s.J[0][0].im[1] = v[3];
        s.Pg[0].v[0] = v[4];
        s.Pg[0].v[1] = v[5];
        s.P0[0].v[0] = ph[0];
        s.P0[0].v[1] = ph[1];
      } else {
#pragma unroll
        for (int x = 0; x < 6; ++x) c.gl_slots[(6 * (i - 1) + x) * 64 + lane] = v[x];
        c.p64[(2 * (i - 1) + 0) * 64 + lane] = ph[0];
        c.p64[(2 * (i - 1) + 1) * 64 + lane] = ph[1];
      }
    }
    s.gl[0] = 0;
    Cx<T> top;
    path<N, T, 1>(s, c, code, top);
    if (base + pair < total) amp[2 * (size_t)it + h] = (double)(h == 0 ? top.re : top.im) * scale;
  }
}

// Pass 5: |sum of the event's item amplitudes|^2 (items in ordering order).
__global__ void __launch_bounds__(kThreads) reduce_kernel(int64_t E, const unsigned* __restrict__ counts,
                                                         const unsigned* __restrict__ offsets,
                                                         const double* __restrict__ amp,
                                                         double* __restrict__ me2) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= E) return;
  const unsigned c = counts[e];
  if (c == 0) return;  // invalid flow: already 0
  const unsigned o = offsets[e];
  double re = 0.0, im = 0.0;
  for (unsigned k = 0; k < c; ++k) {
    re += amp[2 * (size_t)(o + k)];
    im += amp[2 * (size_t)(o + k) + 1];
  }
  me2[e] = re * re + im * im;
}

template <int N, typename T>
int amp_launch(int64_t E, const double* mom, const int8_t* hel, const uint64_t* items,
               const uint64_t* total, double* amp, int grid, hipStream_t stream) {
  constexpr bool NODT = N >= 8;
  hipLaunchKernelGGL((amp_kernel<N, T, NODT>), dim3(grid), dim3(64), (AmpLds<N>::template bytes<T>()),
                     stream, E, mom, hel, items, total, amp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N>
int count_launch(int64_t E, const int8_t* col, double* me2, unsigned* counts, uint64_t* blocks,
                 hipStream_t stream) {
  const int64_t nb = (E + kThreads - 1) / kThreads;
  hipLaunchKernelGGL((count_kernel<N>), dim3((unsigned)nb), dim3(kThreads), 0, stream, E, col, me2,
                     counts, blocks);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, stream, blocks, (int)nb);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N>
int items_launch(int64_t E, const int8_t* col, const unsigned* counts, const uint64_t* blocks,
                 unsigned* offsets, uint64_t* items, hipStream_t stream) {
  const int64_t nb = (E + kThreads - 1) / kThreads;
  hipLaunchKernelGGL((items_kernel<N>), dim3((unsigned)nb), dim3(kThreads), 0, stream, E, col,
                     counts, blocks, offsets, items);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace comck

#define BG_COMC_SWITCH(CALL)              \
  switch (n) {                            \
    case 4: return CALL(4);               \
    case 5: return CALL(5);               \
    case 6: return CALL(6);               \
    case 7: return CALL(7);               \
    case 8: return CALL(8);               \
    case 9: return CALL(9);               \
    default: return -2;                   \
  }

int comc_count(int n, int64_t E, const int8_t* col, double* me2, unsigned* counts,
               uint64_t* blocks, hipStream_t stream) {
#define C_(NN) comck::count_launch<NN>(E, col, me2, counts, blocks, stream)
  BG_COMC_SWITCH(C_)
#undef C_
}

int comc_items(int n, int64_t E, const int8_t* col, const unsigned* counts, const uint64_t* blocks,
               unsigned* offsets, uint64_t* items, hipStream_t stream) {
#define C_(NN) comck::items_launch<NN>(E, col, counts, blocks, offsets, items, stream)
  BG_COMC_SWITCH(C_)
#undef C_
}

int comc_amplitudes(int n, bool fp32, int64_t E, const double* mom, const int8_t* hel,
                    const uint64_t* items, const uint64_t* total, double* amp, int grid,
                    hipStream_t stream) {
#define C_(NN)                                                                             \
  (fp32 ? comck::amp_launch<NN, float>(E, mom, hel, items, total, amp, grid, stream)       \
        : comck::amp_launch<NN, double>(E, mom, hel, items, total, amp, grid, stream))
  BG_COMC_SWITCH(C_)
#undef C_
}

int comc_reduce(int64_t E, const unsigned* counts, const unsigned* offsets, const double* amp,
                double* me2, hipStream_t stream) {
  const int64_t nb = (E + comck::kThreads - 1) / comck::kThreads;
  hipLaunchKernelGGL(comck::reduce_kernel, dim3((unsigned)nb), dim3(comck::kThreads), 0, stream, E,
                     counts, offsets, amp, me2);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

#undef BG_COMC_SWITCH

}  // namespace bg
