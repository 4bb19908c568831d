// Colour-ordered Berends-Giele recursion (Section 2.3, eqs. cobg and
// cobg_full_amplitude) for all (n-2)! orderings A(1, sigma, n) of the adjoint
// basis (Section 2.2, eq. color_decomposition_adjoint), one event per lane.
//
// Design (gfx950, wave64):
//  * Momenta and helicities are read coalesced from the [n][4][E] / [n][E]
//    structure-of-arrays inputs.  Polarizations and the invariants 1/P_S^2 of
//    every subset S of gluons 1..n-1 are computed once per event in FP64; the
//    invariant table and the polarizations/momenta of the n-2 permuted gluons
//    are parked in LDS, lane-major ([slot][lane]) so that a wave-uniform slot
//    index gives conflict-free accesses.
//  * The orderings are walked depth-first in lexicographic order.  Position d
//    of the ordering (1, sigma_2, .., sigma_{n-1}) is a template level; the
//    gluon chosen there is a wave-uniform loop variable, so every lane of a
//    wave takes the same branch.  Entering level d computes the column of
//    range currents J(a..d), a = d-1..0, from the columns of the shallower
//    levels, which stay live in VGPRs (all register indices are compile-time
//    constants).  Prefixes are shared between orderings: column d is computed
//    once per distinct prefix of length d+1.
//  * The full range (0..n-2) is amputated (its propagator is the inverse of
//    the on-shell p_n^2 = 0 factor) and contracted with eps_n.
//  * T = double: plain FP64.  T = float: FP32 complex currents and momenta;
//    1/P^2 is formed in FP64 and rounded once, which avoids the cancellation in
//    E^2 - |p|^2 for nearly light-like subsets.
#include "bg_device.h"
#include "bg_kernels.h"

namespace bg {

template <int N, typename T>
struct CobgState {
  static constexpr int M = N - 1;  // gluons that enter currents (positions 0..M-1)
  C4<T> J[M][M];                   // J[a][b]: range current of positions a..b
  R4<T> P[M][M];                   // P[a][b]: range momentum
  int gl[M];                       // gluon index at each position (wave-uniform)
};

template <int N, typename T>
struct CobgCtx {
  T* sm;              // dynamic LDS, [slot][BLK]
  int tid;            // lane slot index in the block
  int blk;            // block size (LDS stride)
  C4<T> epsN;         // external current of the last gluon
  double* amp;        // [2][K][E]
  int64_t E;
  int64_t e;
  int sigma;          // running ordering index (lexicographic)
};

// LDS slot map: gluon g in 1..N-2 stores eps (8 T) and p (4 T) at 12*(g-1);
// the invariant table 1/P_S^2 follows at kTab + mask.
template <int N>
struct CobgSlots {
  static constexpr int kGluon = 12;
  static constexpr int kTab = 12 * (N - 2);
  static constexpr int kTotal = kTab + (1 << (N - 1));
};

template <int N, typename T>
__device__ __forceinline__ T lds_get(const CobgCtx<N, T>& c, int slot) {
  return c.sm[slot * c.blk + c.tid];
}

template <int N, typename T>
__device__ __forceinline__ void lds_put(CobgCtx<N, T>& c, int slot, T v) {
  c.sm[slot * c.blk + c.tid] = v;
}

// Compute column D: ranges (a..D) for a = D-1 .. 0.  gl[D] has been set and
// J[D][D], P[D][D] hold the new gluon.  For D == M-1 the range (0..D) is the
// amputated top current, returned in `top`.
template <int N, typename T, int D>
__device__ __forceinline__ void cobg_column(CobgState<N, T>& s, const CobgCtx<N, T>& c,
                                            C4<T>& top) {
  constexpr int M = N - 1;
  int mask = 1 << s.gl[D];
#pragma unroll
  for (int a = D - 1; a >= 0; --a) {
    mask |= 1 << s.gl[a];
    s.P[a][D] = radd(s.P[a][D - 1], s.P[D][D]);
    C4<T> acc;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      acc.re[m] = T(0);
      acc.im[m] = T(0);
    }
#pragma unroll
    for (int k = a; k < D; ++k) v3_acc(acc, s.P[a][k], s.P[k + 1][D], s.J[a][k], s.J[k + 1][D]);
#pragma unroll
    for (int j = a; j < D; ++j) {
#pragma unroll
      for (int k = j + 1; k < D; ++k) v4_acc(acc, s.J[a][j], s.J[j + 1][k], s.J[k + 1][D]);
    }
    if (a == 0 && D == M - 1) {
      top = acc;
    } else {
      const T ip2 = lds_get(c, CobgSlots<N>::kTab + mask);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        s.J[a][D].re[m] = acc.re[m] * ip2;
        s.J[a][D].im[m] = acc.im[m] * ip2;
      }
    }
  }
}

template <int N, typename T, int D>
__device__ __forceinline__ void cobg_level(CobgState<N, T>& s, CobgCtx<N, T>& c, int used) {
  constexpr int M = N - 1;
  for (int g = 1; g <= N - 2; ++g) {  // wave-uniform
    if (used & (1 << g)) continue;
    s.gl[D] = g;
    const int base = CobgSlots<N>::kGluon * (g - 1);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      s.J[D][D].re[m] = lds_get(c, base + m);
      s.J[D][D].im[m] = lds_get(c, base + 4 + m);
      s.P[D][D].v[m] = lds_get(c, base + 8 + m);
    }
    C4<T> top;
    cobg_column<N, T, D>(s, c, top);
    if constexpr (D == M - 1) {
      T ar, ai;
      cdot(c.epsN, top, ar, ai);
      double scale = 1.0;
#pragma unroll
      for (int i = 0; i < N - 2; ++i) scale *= kGsOverSqrt2;
      constexpr int64_t K = Factorial<N - 2>::value;
      c.amp[(int64_t)c.sigma * c.E + c.e] = (double)ar * scale;
      c.amp[(K + c.sigma) * c.E + c.e] = (double)ai * scale;
      ++c.sigma;
    } else {
      cobg_level<N, T, D + 1>(s, c, used | (1 << g));
    }
  }
}

template <int N, typename T>
__global__ void __launch_bounds__(64) cobg_amp_kernel(int64_t E, const double* __restrict__ mom,
                                                     const int8_t* __restrict__ hel, int hconf,
                                                     double* __restrict__ amp) {
  extern __shared__ __align__(16) unsigned char bg_lds_raw[];
  constexpr int M = N - 1;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;

  CobgCtx<N, T> c;
  c.sm = reinterpret_cast<T*>(bg_lds_raw);
  c.tid = threadIdx.x;
  c.blk = blockDim.x;
  c.amp = amp;
  c.E = E;
  c.e = e;
  c.sigma = 0;

  double p[N][4];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int m = 0; m < 4; ++m) p[i][m] = mom[((int64_t)i * 4 + m) * E + e];

  CobgState<N, T> s;
  // external currents
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double er[4], ei[4];
    const int h = hel ? (int)hel[(int64_t)i * E + e] : (((hconf >> (N - 1 - i)) & 1) ? -1 : 1);
    polarization(p[i], h, er, ei);
    C4<T> cur;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      cur.re[m] = (T)er[m];
      cur.im[m] = (T)ei[m];
    }
    if (i == 0) {
      s.J[0][0] = cur;
#pragma unroll
      for (int m = 0; m < 4; ++m) s.P[0][0].v[m] = (T)p[0][m];
    } else if (i == N - 1) {
      c.epsN = cur;
    } else {
      const int base = CobgSlots<N>::kGluon * (i - 1);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        lds_put(c, base + m, cur.re[m]);
        lds_put(c, base + 4 + m, cur.im[m]);
        lds_put(c, base + 8 + m, (T)p[i][m]);
      }
    }
  }
  // invariant table 1/P_S^2 over subsets S of gluons 0..M-1 (FP64, rounded once)
  for (int mask = 0; mask < (1 << M); ++mask) {
    double q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < M; ++i) {
      if (mask & (1 << i)) {
#pragma unroll
        for (int m = 0; m < 4; ++m) q[m] += p[i][m];
      }
    }
    const double p2 = q[0] * q[0] - q[1] * q[1] - q[2] * q[2] - q[3] * q[3];
    lds_put(c, CobgSlots<N>::kTab + mask, (T)(1.0 / p2));
  }
  s.gl[0] = 0;
  cobg_level<N, T, 1>(s, c, 1);
}

template <int N, typename T>
int launch_cobg_amp(int64_t E, const double* mom, const int8_t* hel, int hconf, double* amp,
                    hipStream_t stream) {
  const int blk = 64;
  const int64_t grid = (E + blk - 1) / blk;
  const size_t lds = sizeof(T) * (size_t)CobgSlots<N>::kTotal * blk;
  hipLaunchKernelGGL((cobg_amp_kernel<N, T>), dim3((unsigned)grid), dim3(blk), lds, stream, E, mom,
                     hel, hconf, amp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int cobg_amplitudes(int n, bool fp32, int64_t E, const double* mom, const int8_t* hel, int hconf,
                    double* amp, hipStream_t stream) {
  if (E <= 0) return 0;
  switch (n) {
    case 4: return fp32 ? launch_cobg_amp<4, float>(E, mom, hel, hconf, amp, stream)
                        : launch_cobg_amp<4, double>(E, mom, hel, hconf, amp, stream);
    case 5: return fp32 ? launch_cobg_amp<5, float>(E, mom, hel, hconf, amp, stream)
                        : launch_cobg_amp<5, double>(E, mom, hel, hconf, amp, stream);
    case 6: return fp32 ? launch_cobg_amp<6, float>(E, mom, hel, hconf, amp, stream)
                        : launch_cobg_amp<6, double>(E, mom, hel, hconf, amp, stream);
    case 7: return fp32 ? launch_cobg_amp<7, float>(E, mom, hel, hconf, amp, stream)
                        : launch_cobg_amp<7, double>(E, mom, hel, hconf, amp, stream);
    default: return -2;
  }
}

}  // namespace bg
