// Colour-ordered amplitudes along one straight path per ordering (Section
// 2.3, eqs. cobg and cobg_full_amplitude), on the lane-pair layout of
// cobg_pair_impl.h: the ranges of one ordering (1, sigma, n) are built column
// by column with the same vertex code as the depth-first walk, but nothing is
// shared with the orderings of the same prefix.  That costs 13 % more vertex
// work at n = 7 and 21 % at n = 8, and keeps only one path's currents live:
// in FP64 the walk's state overflows the register file from n = 7 on.  1/P^2
// comes from the FP64 prefix momenta of the path (halves plus one partner
// exchange), the V4 dot products are recomputed when a table would not fit.
#pragma once

#include <stdint.h>

#include "cobg_pair_impl.h"

namespace bg {
namespace pathk {

using pairk::Cx;
using pairk::H;

// Per-lane context (see pairk::Ctx).  The gluons 1..n-1 of the lane's event
// sit in LDS: six T values per gluon and lane (polarization halves and
// momentum half) and two FP64 momentum halves.
template <int N, typename T, bool NODT, bool EST = false>
struct Ctx {
  static constexpr bool kRaw = false, kP64G = false, kLC = false, kEst = EST;
  static constexpr bool kDirectP2 = true;
  static constexpr bool kNoDt = NODT;
  T* gl_slots;   // [6 (g-1) + x][lane]
  double* p64;   // [2 (g-1) + c][lane]
  T* tab;        // unused
  int lane, pair, h;
  T g0;
  H<T> epsN;
};

template <int N>
struct Lds {
  template <typename T>
  static constexpr size_t bytes() {
    return sizeof(T) * (size_t)6 * (N - 1) * 64 + sizeof(double) * (size_t)2 * (N - 1) * 64;
  }
};

// Positions D .. n-2 of the ordering coded 4 bits per position (position D
// in bits 4 (D - 1)), the closing gluon in bits 4 (n - 2): the ranges ending
// at position D, then the next position.  top: the amputated top current
// contracted with the closing gluon; topb (EST): its running error bound.
template <int N, typename T, int D, class C>
__device__ __forceinline__ void path(pairk::State<N, T>& s, C& c, uint32_t code, Cx<T>& top,
                                     T& topb) {
  constexpr int M = N - 1;
  int g = (int)((code >> (4 * (D - 1))) & 15u);
  g = g < 1 ? 1 : (g > N - 1 ? N - 1 : g);  // codes hold 1..N-1; keeps LDS reads in bounds
  s.gl[D] = g;
  const int base = 6 * (g - 1);
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    s.J[D][D].re[m] = c.gl_slots[(base + m) * 64 + c.lane];
    s.J[D][D].im[m] = c.gl_slots[(base + 2 + m) * 64 + c.lane];
    s.Pg[D].v[m] = c.gl_slots[(base + 4 + m) * 64 + c.lane];
    s.P0[D].v[m] = s.P0[D - 1].v[m] + c.p64[(2 * (g - 1) + m) * 64 + c.lane];
  }
  if constexpr (C::kEst) {
    // |p^0| of the gluon: the h = 0 lane holds it, the h = 1 lane takes it
    // from its partner (both lanes run this exchange)
    const double pg = c.p64[(2 * (g - 1)) * 64 + c.lane];
    const double px = pairk::xswap(pg);
    s.Ep[D] = s.Ep[D - 1] + (T)fabs(c.h == 0 ? pg : px);
    s.Sb[D][D] = T(1);
  }
  pairk::set_gd<N, T, D, D>(s, c);
  if constexpr (D == M - 1) {
    // the ordering's last gluon closes it
    int gl = (int)((code >> (4 * (N - 2))) & 15u);
    gl = gl < 1 ? 1 : (gl > N - 1 ? N - 1 : gl);
    const int lb = 6 * (gl - 1);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      c.epsN.re[m] = c.gl_slots[(lb + m) * 64 + c.lane];
      c.epsN.im[m] = c.gl_slots[(lb + 2 + m) * 64 + c.lane];
    }
  }
  pairk::build_column<N, T, D, D - 1>(s, c, 0, top, topb);
  if constexpr (D < M - 1) path<N, T, D + 1>(s, c, code, top, topb);
}

// Code of the sigma-th ordering (1, sigma, n) of the adjoint basis in
// lexicographic order of the middle gluons 1..n-2: the permutation is
// unranked digit by digit (factorial number system), the closing gluon n-1
// appended.  Wave-uniform when sigma is.
template <int N>
__device__ __forceinline__ uint32_t lex_code(int sigma) {
  constexpr int KM = N - 2;
  uint32_t code = (uint32_t)(N - 1) << (4 * KM);
  int avail = ((1 << KM) - 1) << 1;  // bits 1..KM: gluons not yet placed
  int f = (int)Factorial<KM - 1>::value;
  int r = sigma;
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    const int d = r / f;
    r -= d * f;
    if (k < KM - 1) f /= (KM - 1 - k);
    // the (d+1)-th set bit of avail is the gluon at position k + 1
    int a = avail;
    for (int i = 0; i < d; ++i) a &= a - 1;
    const int gl = __builtin_ctz(a);
    avail &= ~(1 << gl);
    code |= (uint32_t)gl << (4 * k);
  }
  return code;
}

// Code of the rho-th ordering (1, rho) of gluons 1..n-1 in lexicographic
// order, every gluon allowed at every position including the closing one
// (the (n-1)! orderings of the leading-colour sum, Section 3.1): the
// permutation unranked in the factorial number system.  Wave-uniform when
// rho is.
template <int N>
__device__ __forceinline__ uint32_t lc_code(int rho) {
  constexpr int KM = N - 1;
  uint32_t code = 0u;
  int avail = ((1 << KM) - 1) << 1;  // bits 1..KM: gluons not yet placed
  int f = (int)Factorial<KM - 1>::value;
  int r = rho;
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    const int d = r / f;
    r -= d * f;
    if (k < KM - 1) f /= (KM - 1 - k);
    int a = avail;
    for (int i = 0; i < d; ++i) a &= a - 1;
    const int gl = __builtin_ctz(a);
    avail &= ~(1 << gl);
    code |= (uint32_t)gl << (4 * k);
  }
  return code;
}

// The amplitudes A(1, sigma, n) of event e on this lane pair for the
// orderings of lexicographic rank sig0 <= sigma < sig1 (default: all K =
// (n-2)!), scaled by the couplings, in FP64 to amp[((h K + sigma) astride) +
// acol] when live (plane h of the lane).  lds: this wave's Lds<N>::bytes<T>();
// each lane reads back only its own slots, so no barrier is needed.  EST (T =
// float): est[0] += S_top^2 and est[1] += |A|^2 over the orderings (see
// pairk::cobg_pair_body).  LC: instead, the sum of |A(1, rho)|^2 over the
// (n-1)! leading-colour orderings (lc_code), scaled by the couplings and
// returned (both lanes of the pair); nothing is written.
template <int N, typename T, bool EST = false, bool LC = false>
__device__ __forceinline__ double cobg_path_body(unsigned char* lds, int64_t E,
                                               const double* __restrict__ mom,
                                               const int8_t* __restrict__ hel, int hconf,
                                               int64_t e, bool live, double* __restrict__ amp,
                                               int64_t astride, int64_t acol, T* est = nullptr,
                                               int sig0 = 0,
                                               int sig1 = (int)Factorial<N - 2>::value) {
  constexpr int K = (int)Factorial<N - 2>::value;
  constexpr bool NODT = N >= 8;
  const int lane = threadIdx.x & 63;
  const int pair = lane >> 1, h = lane & 1;
  const bool hi = h != 0;
  Ctx<N, T, NODT, EST> c;
  c.gl_slots = reinterpret_cast<T*>(lds);
  c.p64 = reinterpret_cast<double*>(c.gl_slots + (size_t)6 * (N - 1) * 64);
  c.tab = nullptr;
  c.lane = lane;
  c.pair = pair;
  c.h = h;
  c.g0 = h == 0 ? T(1) : T(-1);
  double scale = 1.0;
#pragma unroll
  for (int i = 0; i < N - 2; ++i) scale *= kGsOverSqrt2;
  pairk::State<N, T> s;
  T e0p = T(0);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double p[4], er[4], ei[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) p[m] = mom[((int64_t)i * 4 + m) * E + e];
    const int hh = hel ? (int)hel[(int64_t)i * E + e] : (((hconf >> (N - 1 - i)) & 1) ? -1 : 1);
    polarization(p, hh, er, ei);
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
      e0p = (T)fabs(p[0]);
    } else {
#pragma unroll
      for (int x = 0; x < 6; ++x) c.gl_slots[(6 * (i - 1) + x) * 64 + lane] = v[x];
      c.p64[(2 * (i - 1) + 0) * 64 + lane] = ph[0];
      c.p64[(2 * (i - 1) + 1) * 64 + lane] = ph[1];
    }
  }
  s.gl[0] = 0;
  if constexpr (EST) {
    s.Sb[0][0] = T(1);
    s.Ep[0] = e0p;
  }
  if constexpr (LC) {
    double q = 0.0;
#pragma unroll 1
    for (int rho = 0; rho < (int)Factorial<N - 1>::value; ++rho) {  // wave-uniform
      Cx<T> top;
      T topb = T(0);
      path<N, T, 1>(s, c, lc_code<N>(rho), top, topb);
      q += (double)top.re * (double)top.re + (double)top.im * (double)top.im;
    }
    return q * scale * scale;
  }
  T s2 = T(0), a2 = T(0);
#pragma unroll 1
  for (int sig = sig0; sig < sig1; ++sig) {  // wave-uniform
    Cx<T> top;
    T topb = T(0);
    path<N, T, 1>(s, c, lex_code<N>(sig), top, topb);
    if constexpr (EST) {
      s2 += topb * topb;
      a2 += top.re * top.re + top.im * top.im;
    }
    if (live) amp[((int64_t)h * K + sig) * astride + acol] = (double)(h == 0 ? top.re : top.im) * scale;
  }
  if constexpr (EST) {
    est[0] += s2;
    est[1] += a2;
  }
  return 0.0;
}

}  // namespace pathk
}  // namespace bg
