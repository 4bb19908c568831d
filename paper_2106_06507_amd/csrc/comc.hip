// Colour-sampled colour-ordered evaluation (Section 2.2,
// eq. color_decomposition_colorflow, with the colour-ordered amplitudes of
// Section 2.3): for one colour-flow assignment per event,
//   A = sum over orderings (1, sigma) of Tr(E_1 E_sigma2 ... E_sigman) A(1, sigma),
// E_k = e_{j_k i_k}.  The trace is 1 when the delta chain closes
// (i_prev = j_next along the ordering and i_last = j_1) and 0 otherwise, so
// only the closing orderings (the Euler circuits of the colour edges that
// start with gluon 1) are evaluated.
//
// Passes: (1) one thread per event counts its closing orderings without
// enumerating them: they are the Euler circuits of the colour multigraph
// (edge j_k -> i_k per gluon) that start with gluon 1's edge, whose number
// for distinguishable edges is, by the BEST theorem, the number of spanning
// arborescences towards any vertex (a 2x2 or 1x1 Laplacian minor over the
// three colours) times the product over vertices of (out-degree - 1)!;
// unbalanced or disconnected flows get 0 and exactly 0 for |A|^2.
// (2) one block scans the per-block item and valid-event counts.  (3) one
// thread per event writes its first item index and lists the valid events.
// (4) one wave per valid event enumerates its closing orderings, split over
// the lanes by the two gluons that follow gluon 1 (each prefix's share
// counted the same way), depth-first with candidate gluons from per-colour
// bit masks, and writes its (event, ordering) items at their ranks.
// (5) one lane pair per item
// evaluates A(1, sigma) with the lane-pair recursion of cobg_pair_impl.h on
// that single ordering (gluons of the ordering differ between pairs; 1/P^2
// from the FP64 prefix momenta).  (6) one wave per valid event adds its
// items' amplitudes and writes |A|^2.  The totals are read back once (a
// synchronisation) to size the item arrays and the enumeration grid.
//
// FP32 check: with the FP32 recursion each item also carries the running
// error bound of its top current (State::Sb of cobg_pair_impl.h, scaled like
// the amplitude); the flow amplitude's FP32 error is bounded by the sum of
// its items' bounds B, so pass 6 lists the event when B^2 > tau |A|^2
// (helicity configurations whose tree amplitude vanishes identically are
// never listed), together with its items.  The listed items are evaluated
// again in FP64 (pass 5 over the item list, its length read on the device)
// and the listed events reduced again (pass 6 over the event list).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cdbg_impl.h"
#include "cobg_path_impl.h"
#include "cobg_quad_impl.h"

namespace bg {
namespace comck {

using pairk::Cx;
using pairk::H;
using pairk::HR;

constexpr int kThreads = 256;
constexpr int kWave = 64;

// colours packed two bits per gluon; jm[c] = gluons 1..N-1 whose j is c
template <int N>
struct Flow {
  int ci, cj;
  unsigned jm[3];
  __host__ __device__ __forceinline__ int i(int g) const { return (ci >> (2 * g)) & 3; }
  __host__ __device__ __forceinline__ int j(int g) const { return (cj >> (2 * g)) & 3; }
};

template <int N>
__host__ __device__ __forceinline__ Flow<N> load_flow(int64_t E, const int8_t* __restrict__ col, int64_t e,
                                             bool& in_range) {
  Flow<N> f{0, 0, {0u, 0u, 0u}};
  in_range = true;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int ii = col[(int64_t)k * E + e];
    const int jj = col[((int64_t)N + k) * E + e];
    in_range = in_range && ii >= 0 && ii <= 2 && jj >= 0 && jj <= 2;
    f.ci |= (ii & 3) << (2 * k);
    f.cj |= (jj & 3) << (2 * k);
    if (k > 0) {
      f.jm[0] |= (unsigned)(jj == 0) << k;
      f.jm[1] |= (unsigned)(jj == 1) << k;
      f.jm[2] |= (unsigned)(jj == 2) << k;
    }
  }
  return f;
}

// Euler circuits (as cyclic sequences of distinguishable edges) of the
// multigraph made of the colour edges j_k -> i_k of the gluons k not in
// `skip`, plus the edge vu -> vv when vu >= 0; 0 when it is unbalanced or
// disconnected.  BEST theorem: spanning arborescences towards any vertex (a
// Laplacian minor over the three colours) times the product over vertices
// of (out-degree - 1)!.
template <int N>
__host__ __device__ __forceinline__ unsigned euler_count(const Flow<N>& f, unsigned skip, int vu,
                                                         int vv) {
  int out[3] = {0, 0, 0}, in[3] = {0, 0, 0};
  int a[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // non-loop edges u -> v
#pragma unroll
  for (int k = 0; k <= N; ++k) {
    int u, v;
    if (k < N) {
      if ((skip >> k) & 1u) continue;
      u = f.j(k);
      v = f.i(k);
    } else {
      if (vu < 0) continue;
      u = vu;
      v = vv;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      out[c] += u == c;
      in[c] += v == c;
#pragma unroll
      for (int d = 0; d < 3; ++d) a[c][d] += (u == c && v == d && c != d);
    }
  }
  if (out[0] != in[0] || out[1] != in[1] || out[2] != in[2]) return 0u;
  constexpr unsigned fact[10] = {1u, 1u, 2u, 6u, 24u, 120u, 720u, 5040u, 40320u, 362880u};
  // Laplacian L[c][d]: out-degree without loops on the diagonal, -a[c][d]
  // off it; the count towards the first active vertex is the determinant of
  // L restricted to the other active vertices
  int act[3], na = 0;
  unsigned prod = 1u;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (out[c] > 0) {
      act[na++] = c;
      prod *= fact[out[c] - 1];
    }
  }
  if (na == 0) return 0u;
  int t;
  if (na == 1) {
    t = 1;
  } else {
    int l[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int d = 0; d < 3; ++d) l[c][d] = c == d ? a[c][0] + a[c][1] + a[c][2] : -a[c][d];
    }
    if (na == 2) {
      t = l[act[1]][act[1]];
    } else {
      t = l[1][1] * l[2][2] - l[1][2] * l[2][1];
    }
  }
  return t > 0 ? (unsigned)t * prod : 0u;
}

// Number of closing orderings: the Euler circuits of all colour edges (each
// read from gluon 1's edge on).  At most (N-1)!.
template <int N>
__host__ __device__ __forceinline__ unsigned closing_count(const Flow<N>& f) {
  return euler_count<N>(f, 0u, -1, -1);
}

// Closing orderings that start (1, a, b): the chain holds through b, and the
// remaining edges form an Euler trail from i_b back to j_1, i.e. an Euler
// circuit once the edge j_1 -> i_b is added.
template <int N>
__host__ __device__ __forceinline__ unsigned prefix_count(const Flow<N>& f, int a, int b) {
  if (f.j(a) != f.i(0) || f.j(b) != f.i(a)) return 0u;
  const unsigned skip = 1u | (1u << a) | (1u << b);
  if (N == 3) return f.i(b) == f.j(0) ? 1u : 0u;
  return euler_count<N>(f, skip, f.j(0), f.i(b));
}

// The prefix (a, b) of lane l < (N-1)(N-2), in the depth-first order of the
// orderings: a ascending, then b ascending.
template <int N>
__host__ __device__ __forceinline__ void prefix_of(int l, int& a, int& b) {
  a = 1 + l / (N - 2);
  b = 1 + l % (N - 2);
  b += b >= a;
}

// Closing orderings: position D (1 .. N-1) takes an unused gluon g with
// j_g = i of the previous gluon; after position N-1, i_last must equal j_0.
// visit(code) with nibble D-1 of code = gluon at position D.
template <int N, int D, class V>
__host__ __device__ __forceinline__ void orderings(const Flow<N>& f, unsigned used, int prev, uint32_t code,
                                          V& visit) {
  if constexpr (D == N) {
    if (f.i(prev) == f.j(0)) visit(code);
  } else {
    for (unsigned m = f.jm[f.i(prev)] & ~used; m != 0u; m &= m - 1u) {
      const int g = __builtin_ctz(m);
      orderings<N, D + 1>(f, used | (1u << g), g, code | ((uint32_t)g << (4 * (D - 1))), visit);
    }
  }
}

__device__ __forceinline__ void block_sum_2(uint64_t x, uint64_t y, uint64_t* out_x,
                                            uint64_t* out_y) {
  __shared__ uint64_t px[kThreads], py[kThreads];
  px[threadIdx.x] = x;
  py[threadIdx.x] = y;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      px[threadIdx.x] += px[threadIdx.x + off];
      py[threadIdx.x] += py[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out_x[blockIdx.x] = px[0];
    out_y[blockIdx.x] = py[0];
  }
}

// Pass 1
template <int N>
__global__ void __launch_bounds__(kThreads) count_kernel(int64_t E, const int8_t* __restrict__ col,
                                                        double* __restrict__ me2,
                                                        unsigned* __restrict__ counts,
                                                        uint64_t* __restrict__ block_items,
                                                        uint64_t* __restrict__ block_valid) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  unsigned c = 0;
  if (e < E) {
    bool in_range;
    const Flow<N> f = load_flow<N>(E, col, e, in_range);
    if (in_range) c = closing_count<N>(f);
    if (c == 0) me2[e] = 0.0;  // no closing ordering: the flow's amplitude is 0
    counts[e] = c;
  }
  block_sum_2(c, c != 0, block_items, block_valid);
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

// Pass 3: offsets[e] = the event's first item index; valid events listed in
// event order.  Item ranks fit 32 bits: the host admits only totals below
// 2^31 to the later passes.
__global__ void __launch_bounds__(kThreads) offsets_kernel(int64_t E,
                                                          const unsigned* __restrict__ counts,
                                                          const uint64_t* __restrict__ block_items,
                                                          const uint64_t* __restrict__ block_valid,
                                                          unsigned* __restrict__ offsets,
                                                          unsigned* __restrict__ valid) {
  __shared__ unsigned pc[kThreads], pv[kThreads];
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const unsigned c = e < E ? counts[e] : 0u;
  pc[threadIdx.x] = c;
  pv[threadIdx.x] = c != 0u;
  __syncthreads();
  for (int off = 1; off < kThreads; off *= 2) {
    const bool take = (int)threadIdx.x >= off;
    const unsigned vc = take ? pc[threadIdx.x - off] : 0u;
    const unsigned vv = take ? pv[threadIdx.x - off] : 0u;
    __syncthreads();
    pc[threadIdx.x] += vc;
    pv[threadIdx.x] += vv;
    __syncthreads();
  }
  if (e >= E) return;
  offsets[e] = (unsigned)(block_items[blockIdx.x] + pc[threadIdx.x] - c);
  if (c != 0u) valid[block_valid[blockIdx.x] + pv[threadIdx.x] - 1u] = (unsigned)e;
}

// Pass 4: one wave per valid event writes its closing orderings
// (event << 32 | ordering code) from offsets[e] on, never more than
// counts[e]: lane l takes the orderings that start (1, a, b) (prefix_of),
// counts them (prefix_count), finds its first rank by a prefix sum over the
// wave and enumerates the rest of its subtree depth-first, so the items are
// in the same order as one depth-first walk over the whole event.
template <int N>
__global__ void __launch_bounds__(kThreads) enumerate_kernel(int64_t E, const int8_t* __restrict__ col,
                                                            const unsigned* __restrict__ valid,
                                                            unsigned n_valid,
                                                            const unsigned* __restrict__ counts,
                                                            const unsigned* __restrict__ offsets,
                                                            uint64_t* __restrict__ items) {
  static_assert((N - 1) * (N - 2) <= kWave, "one prefix per lane");
  const int lane = threadIdx.x & (kWave - 1);
  const unsigned v = blockIdx.x * (kThreads / kWave) + threadIdx.x / kWave;
  if (v >= n_valid) return;  // whole waves leave together
  const int64_t e = valid[v];
  bool in_range;
  const Flow<N> f = load_flow<N>(E, col, e, in_range);
  int a = 1, b = 2;
  unsigned c = 0u;
  if (lane < (N - 1) * (N - 2)) {
    prefix_of<N>(lane, a, b);
    c = prefix_count<N>(f, a, b);
  }
  // inclusive prefix sum over the wave
  unsigned incl = c;
#pragma unroll
  for (int off = 1; off < kWave; off *= 2) {
    const unsigned t = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += t;
  }
  if (c == 0u) return;
  const unsigned first = offsets[e];
  const unsigned end = first + counts[e];
  unsigned k = first + incl - c;
  const unsigned stop = k + c < end ? k + c : end;
  auto visit = [&](uint32_t code) {
    if (k < stop) items[k++] = ((uint64_t)e << 32) | code;
  };
  orderings<N, 3>(f, 1u | (1u << a) | (1u << b), b, (uint32_t)a | ((uint32_t)b << 4), visit);
}

template <int N, typename T, bool NODT, bool EST = false>
using Ctx = pathk::Ctx<N, T, NODT, EST>;
template <int N>
using AmpLds = pathk::Lds<N>;
using pathk::path;

// Pass 4: persistent blocks over 32-item tiles; amp[2 item + h] = plane h
// of A(1, sigma) including the couplings; EST: bnd[item] = the running error
// bound of the top current times the same couplings.  sel (re-evaluation of
// listed items): the items are sel[0 .. *sel_count) instead of all.
template <int N, typename T, bool NODT, bool EST>
__global__ void __launch_bounds__(64) amp_kernel(int64_t E, const double* __restrict__ mom,
                                                const int8_t* __restrict__ hel,
                                                const uint64_t* __restrict__ items,
                                                const uint64_t* __restrict__ total_p,
                                                double* __restrict__ amp,
                                                float* __restrict__ bnd,
                                                const unsigned* __restrict__ sel,
                                                const unsigned* __restrict__ sel_count) {
  extern __shared__ __align__(16) unsigned char bg_comc_lds[];
  const unsigned total = sel ? *sel_count : (unsigned)*total_p;  // below 2^31 (host check)
  const int lane = threadIdx.x;
  const int pair = lane >> 1, h = lane & 1;
  const bool hi = h != 0;
  Ctx<N, T, NODT, EST> c;
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
    const unsigned slot = base + pair < total ? base + pair : total - 1;
    const unsigned it = sel ? sel[slot] : slot;
    const uint64_t item = items[it];
    int64_t e = (int64_t)(item >> 32);
    e = e < E ? e : E - 1;  // items always hold e < E; the clamp keeps reads in bounds regardless
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
        if constexpr (EST) {
          s.Ep[0] = (T)fabs(p[0]);
          s.Sb[0][0] = T(1);
        }
      } else {
#pragma unroll
        for (int x = 0; x < 6; ++x) c.gl_slots[(6 * (i - 1) + x) * 64 + lane] = v[x];
        c.p64[(2 * (i - 1) + 0) * 64 + lane] = ph[0];
        c.p64[(2 * (i - 1) + 1) * 64 + lane] = ph[1];
      }
    }
    s.gl[0] = 0;
    Cx<T> top;
    T topb = T(0);
    path<N, T, 1>(s, c, code, top, topb);
    if (base + pair < total) {
      amp[2 * (size_t)it + h] = (double)(h == 0 ? top.re : top.im) * scale;
      if (EST && h == 0) bnd[it] = (float)((double)topb * scale);
    }
  }
}

// Pass 6: |sum of the event's item amplitudes|^2, one wave per valid event
// (the others were set to 0 by pass 1): lane l adds items l, l + 64, ...,
// then a fixed butterfly adds the lanes, so the result does not depend on
// the launch.
__global__ void __launch_bounds__(kThreads) reduce_kernel(const unsigned* __restrict__ valid,
                                                         unsigned n_valid,
                                                         const unsigned* __restrict__ counts,
                                                         const unsigned* __restrict__ offsets,
                                                         const double* __restrict__ amp,
                                                         double* __restrict__ me2) {
  const int lane = threadIdx.x & (kWave - 1);
  const unsigned v = blockIdx.x * (kThreads / kWave) + threadIdx.x / kWave;
  if (v >= n_valid) return;  // whole waves leave together
  const unsigned e = valid[v];
  const unsigned c = counts[e];
  const unsigned o = offsets[e];
  double re = 0.0, im = 0.0;
  for (unsigned k = lane; k < c; k += kWave) {
    re += amp[2 * (size_t)(o + k)];
    im += amp[2 * (size_t)(o + k) + 1];
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, kWave);
    im += __shfl_xor(im, off, kWave);
  }
  if (lane == 0) me2[e] = re * re + im * im;
}

// Pass 6 with the FP32 check: as reduce_kernel, and the sum B of the items'
// error bounds; the event is listed when B^2 > tau |A|^2 (or the test is not
// a number) unless its helicity configuration vanishes identically: appended
// to flist (count fcount[0]) and its items to sel (count fcount[1]).
__global__ void __launch_bounds__(kThreads) reduce_check_kernel(
    int n, int64_t E, const int8_t* __restrict__ hel, const unsigned* __restrict__ valid,
    unsigned n_valid, const unsigned* __restrict__ counts, const unsigned* __restrict__ offsets,
    const double* __restrict__ amp, const float* __restrict__ bnd, double* __restrict__ me2,
    float tau, unsigned* __restrict__ fcount, unsigned* __restrict__ flist,
    unsigned* __restrict__ sel) {
  const int lane = threadIdx.x & (kWave - 1);
  const unsigned v = blockIdx.x * (kThreads / kWave) + threadIdx.x / kWave;
  if (v >= n_valid) return;  // whole waves leave together
  const unsigned e = valid[v];
  const unsigned c = counts[e];
  const unsigned o = offsets[e];
  double re = 0.0, im = 0.0, b = 0.0;
  for (unsigned k = lane; k < c; k += kWave) {
    re += amp[2 * (size_t)(o + k)];
    im += amp[2 * (size_t)(o + k) + 1];
    b += (double)bnd[o + k];
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, kWave);
    im += __shfl_xor(im, off, kWave);
    b += __shfl_xor(b, off, kWave);
  }
  const double a2 = re * re + im * im;
  int neg = 0;
  for (int k = 0; k < n; ++k) neg += hel[(int64_t)k * E + e] < 0 ? 1 : 0;
  const bool listed = neg >= 2 && neg <= n - 2 && !(b * b <= (double)tau * a2);
  if (lane == 0) me2[e] = a2;
  if (!listed) return;  // uniform over the wave
  unsigned ib = 0u;
  if (lane == 0) {
    flist[atomicAdd(fcount, 1u)] = e;
    ib = atomicAdd(fcount + 1, c);
  }
  ib = (unsigned)__shfl((int)ib, 0, kWave);
  for (unsigned k = lane; k < c; k += kWave) sel[ib + k] = o + k;
}

// Pass 6 again for the listed events flist[0 .. *fcount) after their items'
// FP64 re-evaluation (waves past the count leave at once).
__global__ void __launch_bounds__(kThreads) reduce_listed_kernel(
    const unsigned* __restrict__ flist, const unsigned* __restrict__ fcount,
    const unsigned* __restrict__ counts, const unsigned* __restrict__ offsets,
    const double* __restrict__ amp, double* __restrict__ me2) {
  const int lane = threadIdx.x & (kWave - 1);
  const unsigned v = blockIdx.x * (kThreads / kWave) + threadIdx.x / kWave;
  if (v >= *fcount) return;  // whole waves leave together
  const unsigned e = flist[v];
  const unsigned c = counts[e];
  const unsigned o = offsets[e];
  double re = 0.0, im = 0.0;
  for (unsigned k = lane; k < c; k += kWave) {
    re += amp[2 * (size_t)(o + k)];
    im += amp[2 * (size_t)(o + k) + 1];
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, kWave);
    im += __shfl_xor(im, off, kWave);
  }
  if (lane == 0) me2[e] = re * re + im * im;
}

// Colour-ordered amplitudes A(1, sigma, n) of every ordering sigma for
// events e0 .. e0 + count - 1 of an [n][4][E] input, into amp [2][K][count]
// (the layout of cobg_pair_kernel), one straight path per ordering
// (cobg_path_impl.h).  idx (re-evaluation of listed events): column j holds
// event idx[e0 + j] for e0 + j < *cnt (blocks past the list length return at
// once).  gridDim.y splits the orderings: block (x, y) evaluates ranks
// [y K / gridDim.y, (y + 1) K / gridDim.y) of its 32 events (more, shorter
// tasks when few events are listed).
template <int N, typename T>
__global__ void __launch_bounds__(64) cobg_path_kernel(int64_t E, int64_t e0, int64_t count,
                                                      const double* __restrict__ mom,
                                                      const int8_t* __restrict__ hel, int hconf,
                                                      double* __restrict__ amp,
                                                      const unsigned* __restrict__ idx,
                                                      const unsigned* __restrict__ cnt) {
  extern __shared__ __align__(16) unsigned char bg_path_lds[];
  const int pair = (int)threadIdx.x >> 1;
  const int64_t j = (int64_t)blockIdx.x * 32 + pair;
  bool live = j < count;
  int64_t e;
  if (idx) {
    const int64_t total = (int64_t)*cnt;
    const int64_t b0 = e0 + (int64_t)blockIdx.x * 32;
    if (b0 >= total) return;  // the whole block (uniform)
    live = live && e0 + j < total;
    e = (int64_t)idx[live ? e0 + j : b0];
  } else {
    e = e0 + (live ? j : count - 1);
  }
  constexpr int K = (int)Factorial<N - 2>::value;
  const int sig0 = (int)(blockIdx.y * K / gridDim.y), sig1 = (int)((blockIdx.y + 1) * K / gridDim.y);
  pathk::cobg_path_body<N, T>(bg_path_lds, E, mom, hel, hconf, e, live, amp, count, j, nullptr,
                              sig0, sig1);
}

template <int N, typename T>
int path_launch(int64_t E, int64_t e0, int64_t count, const double* mom, const int8_t* hel,
                int hconf, double* amp, const unsigned* idx, const unsigned* cnt, int osplit,
                hipStream_t stream) {
  const unsigned grid = (unsigned)((count + 31) / 32);
  hipLaunchKernelGGL((cobg_path_kernel<N, T>), dim3(grid, (unsigned)osplit), dim3(64),
                     (pathk::Lds<N>::template bytes<T>()), stream, E, e0, count, mom, hel, hconf,
                     amp, idx, cnt);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Pass 4 for FP64 at n >= 8 on quads (cobg_quad_impl.h): 16 items per
// 64-lane block and round, one Lorentz component per lane.
template <int N>
__global__ void __launch_bounds__(64) amp_kernel_q(int64_t E, const double* __restrict__ mom,
                                                  const int8_t* __restrict__ hel,
                                                  const uint64_t* __restrict__ items,
                                                  const uint64_t* __restrict__ total_p,
                                                  double* __restrict__ amp,
                                                  const unsigned* __restrict__ sel,
                                                  const unsigned* __restrict__ sel_count) {
  extern __shared__ __align__(16) unsigned char bg_quad_lds[];
  const unsigned total = sel ? *sel_count : (unsigned)*total_p;  // below 2^31 (host check)
  const int lane = threadIdx.x;
  const int quad = lane >> 2, cc = lane & 3;
  double scale = 1.0;
#pragma unroll
  for (int i = 0; i < N - 2; ++i) scale *= kGsOverSqrt2;
  for (unsigned base = blockIdx.x * 16u; base < total; base += gridDim.x * 16u) {
    const unsigned slot = base + quad < total ? base + quad : total - 1;
    const unsigned it = sel ? sel[slot] : slot;
    const uint64_t item = items[it];
    int64_t e = (int64_t)(item >> 32);
    e = e < E ? e : E - 1;  // items always hold e < E; the clamp keeps reads in bounds regardless
    quadk::State<N> s;
    quadk::Ctx c;
    quadk::setup<N>(s, c, reinterpret_cast<double*>(bg_quad_lds), E, mom, hel, 0, e);
    quadk::Q top;
    quadk::path<N, 1>(s, c, (uint32_t)item, top);
    if (base + quad < total && cc < 2) amp[2 * (size_t)it + cc] = (cc == 0 ? top.re : top.im) * scale;
  }
}

template <int N>
int amp_launch_q(int64_t E, const double* mom, const int8_t* hel, const uint64_t* items,
                 const uint64_t* total, double* amp, const unsigned* sel, const unsigned* sel_count,
                 int grid, hipStream_t stream) {
  hipLaunchKernelGGL((amp_kernel_q<N>), dim3(2 * grid), dim3(64), quadk::Lds<N>::bytes(), stream,
                     E, mom, hel, items, total, amp, sel, sel_count);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Colour-ordered amplitudes of every ordering on quads (FP64, n = 8): as
// cobg_path_kernel, 16 events per block.
template <int N>
__global__ void __launch_bounds__(64) cobg_path_kernel_q(int64_t E, int64_t e0, int64_t count,
                                                        const double* __restrict__ mom,
                                                        const int8_t* __restrict__ hel, int hconf,
                                                        double* __restrict__ amp,
                                                        const unsigned* __restrict__ idx,
                                                        const unsigned* __restrict__ cnt) {
  extern __shared__ __align__(16) unsigned char bg_quad_lds[];
  constexpr int K = (int)Factorial<N - 2>::value;
  const int lane = threadIdx.x;
  const int quad = lane >> 2, cc = lane & 3;
  const int64_t j = (int64_t)blockIdx.x * 16 + quad;
  bool live = j < count;
  int64_t e;
  if (idx) {
    const int64_t tot = (int64_t)*cnt;
    const int64_t b0 = e0 + (int64_t)blockIdx.x * 16;
    if (b0 >= tot) return;  // the whole block (uniform)
    live = live && e0 + j < tot;
    e = (int64_t)idx[live ? e0 + j : b0];
  } else {
    e = e0 + (live ? j : count - 1);
  }
  double scale = 1.0;
#pragma unroll
  for (int i = 0; i < N - 2; ++i) scale *= kGsOverSqrt2;
  quadk::State<N> s;
  quadk::Ctx c;
  quadk::setup<N>(s, c, reinterpret_cast<double*>(bg_quad_lds), E, mom, hel, hconf, e);
#pragma unroll 1
  for (int sig = 0; sig < K; ++sig) {  // wave-uniform
    quadk::Q top;
    quadk::path<N, 1>(s, c, pathk::lex_code<N>(sig), top);
    if (live && cc < 2)
      amp[((int64_t)cc * K + sig) * count + j] = (cc == 0 ? top.re : top.im) * scale;
  }
}

template <int N>
int path_launch_q(int64_t E, int64_t e0, int64_t count, const double* mom, const int8_t* hel,
                  int hconf, double* amp, const unsigned* idx, const unsigned* cnt,
                  hipStream_t stream) {
  const unsigned grid = (unsigned)((count + 15) / 16);
  hipLaunchKernelGGL((cobg_path_kernel_q<N>), dim3(grid), dim3(64), quadk::Lds<N>::bytes(), stream,
                     E, e0, count, mom, hel, hconf, amp, idx, cnt);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N, typename T, bool EST = false>
int amp_launch(int64_t E, const double* mom, const int8_t* hel, const uint64_t* items,
               const uint64_t* total, double* amp, float* bnd, const unsigned* sel,
               const unsigned* sel_count, int grid, hipStream_t stream) {
  constexpr bool NODT = N >= 8;
  hipLaunchKernelGGL((amp_kernel<N, T, NODT, EST>), dim3(grid), dim3(64),
                     (AmpLds<N>::template bytes<T>()), stream, E, mom, hel, items, total, amp, bnd,
                     sel, sel_count);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N>
int count_launch(int64_t E, const int8_t* col, double* me2, unsigned* counts, unsigned* offsets,
                 unsigned* valid, uint64_t* block_items, uint64_t* block_valid,
                 hipStream_t stream) {
  const int64_t nb = (E + kThreads - 1) / kThreads;
  hipLaunchKernelGGL((count_kernel<N>), dim3((unsigned)nb), dim3(kThreads), 0, stream, E, col, me2,
                     counts, block_items, block_valid);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, stream, block_items, (int)nb);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, stream, block_valid, (int)nb);
  hipLaunchKernelGGL(offsets_kernel, dim3((unsigned)nb), dim3(kThreads), 0, stream, E, counts,
                     block_items, block_valid, offsets, valid);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N>
int enumerate_launch(int64_t E, const int8_t* col, const unsigned* valid, unsigned n_valid,
                     const unsigned* counts, const unsigned* offsets, uint64_t* items,
                     hipStream_t stream) {
  constexpr unsigned per_block = kThreads / kWave;  // one wave per valid event
  const unsigned nb = (n_valid + per_block - 1) / per_block;
  hipLaunchKernelGGL((enumerate_kernel<N>), dim3(nb), dim3(kThreads), 0, stream, E, col, valid,
                     n_valid, counts, offsets, items);
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
               unsigned* offsets, unsigned* valid, uint64_t* block_items, uint64_t* block_valid,
               hipStream_t stream) {
#define C_(NN) \
  comck::count_launch<NN>(E, col, me2, counts, offsets, valid, block_items, block_valid, stream)
  BG_COMC_SWITCH(C_)
#undef C_
}

int comc_items(int n, int64_t E, const int8_t* col, const unsigned* valid, unsigned n_valid,
               const unsigned* counts, const unsigned* offsets, uint64_t* items,
               hipStream_t stream) {
#define C_(NN) \
  comck::enumerate_launch<NN>(E, col, valid, n_valid, counts, offsets, items, stream)
  BG_COMC_SWITCH(C_)
#undef C_
}

int comc_amplitudes(int n, bool fp32, int64_t E, const double* mom, const int8_t* hel,
                    const uint64_t* items, const uint64_t* total, double* amp, float* bnd,
                    int grid, hipStream_t stream) {
#define C_(NN)                                                                              \
  (!fp32 ? (NN >= 8 ? comck::amp_launch_q<NN>(E, mom, hel, items, total, amp, nullptr,       \
                                              nullptr, grid, stream)                         \
                    : comck::amp_launch<NN, double>(E, mom, hel, items, total, amp, nullptr, \
                                                    nullptr, nullptr, grid, stream))         \
   : bnd ? comck::amp_launch<NN, float, true>(E, mom, hel, items, total, amp, bnd, nullptr,  \
                                              nullptr, grid, stream)                         \
         : comck::amp_launch<NN, float>(E, mom, hel, items, total, amp, nullptr, nullptr,    \
                                        nullptr, grid, stream))
  BG_COMC_SWITCH(C_)
#undef C_
}

int comc_amplitudes_listed(int n, int64_t E, const double* mom, const int8_t* hel,
                           const uint64_t* items, const unsigned* sel, const unsigned* sel_count,
                           double* amp, int grid, hipStream_t stream) {
#define C_(NN)                                                                               \
  (NN >= 8 ? comck::amp_launch_q<NN>(E, mom, hel, items, nullptr, amp, sel, sel_count, grid,  \
                                     stream)                                                  \
           : comck::amp_launch<NN, double>(E, mom, hel, items, nullptr, amp, nullptr, sel,    \
                                           sel_count, grid, stream))
  BG_COMC_SWITCH(C_)
#undef C_
}

int cobg_path_amplitudes(int n, int64_t E, int64_t e0, int64_t count, const double* mom,
                         const int8_t* hel, int hconf, double* amp, const unsigned* idx,
                         const unsigned* cnt, hipStream_t stream, int osplit) {
  if (count <= 0) return 0;
  if (osplit < 1 || osplit > 120 || 120 % osplit != 0) return -2;
  switch (n) {
    case 7:
      return comck::path_launch<7, double>(E, e0, count, mom, hel, hconf, amp, idx, cnt, osplit,
                                           stream);
    case 8: return comck::path_launch_q<8>(E, e0, count, mom, hel, hconf, amp, idx, cnt, stream);
    default: return -2;
  }
}

int comc_reduce(const unsigned* valid, unsigned n_valid, const unsigned* counts,
                const unsigned* offsets, const double* amp, double* me2, hipStream_t stream) {
  constexpr unsigned per_block = comck::kThreads / comck::kWave;  // one wave per valid event
  const unsigned nb = (n_valid + per_block - 1) / per_block;
  hipLaunchKernelGGL(comck::reduce_kernel, dim3(nb), dim3(comck::kThreads), 0, stream, valid,
                     n_valid, counts, offsets, amp, me2);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int comc_reduce_check(int n, int64_t E, const int8_t* hel, const unsigned* valid, unsigned n_valid,
                      const unsigned* counts, const unsigned* offsets, const double* amp,
                      const float* bnd, double* me2, float tau, unsigned* fcount, unsigned* flist,
                      unsigned* sel, hipStream_t stream) {
  constexpr unsigned per_block = comck::kThreads / comck::kWave;  // one wave per valid event
  const unsigned nb = (n_valid + per_block - 1) / per_block;
  hipLaunchKernelGGL(comck::reduce_check_kernel, dim3(nb), dim3(comck::kThreads), 0, stream, n, E,
                     hel, valid, n_valid, counts, offsets, amp, bnd, me2, tau, fcount, flist, sel);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int comc_reduce_listed(const unsigned* flist, const unsigned* fcount, unsigned max_listed,
                       const unsigned* counts, const unsigned* offsets, const double* amp,
                       double* me2, hipStream_t stream) {
  constexpr unsigned per_block = comck::kThreads / comck::kWave;  // one wave per listed event
  const unsigned nb = (max_listed + per_block - 1) / per_block;
  if (nb == 0) return 0;
  hipLaunchKernelGGL(comck::reduce_listed_kernel, dim3(nb), dim3(comck::kThreads), 0, stream, flist,
                     fcount, counts, offsets, amp, me2);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

#undef BG_COMC_SWITCH

}  // namespace bg
