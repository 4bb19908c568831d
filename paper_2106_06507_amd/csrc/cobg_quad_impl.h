// Colour-ordered amplitude of one ordering on four lanes (one Lorentz
// component per lane), FP64, for n >= 8 (Section 2.3, eqs. cobg and
// cobg_full_amplitude).  The lane-pair layout of cobg_pair_impl.h keeps two
// components of every current of a path in each lane; in FP64 at n = 8, 9
// that state (28 / 36 currents) overflows the register file and spills up
// to 1.8 KB per lane, which goes to HBM.  Here each lane of a quad holds one
// component, so a path's state halves, and every Minkowski product is the
// sum of the four lanes' partials, formed with two DPP quad_perm moves
// ([1,0,3,2] then [2,3,0,1]).  The sum is ((x0 + x1) + (x2 + x3)) in every
// lane (IEEE addition commutes), so all four lanes hold identical values.
// The vertex arithmetic is that of pairk::build_range, term by term; 1/P^2
// comes from the FP64 prefix momenta of the path, the V4 dot products are
// recomputed.
#pragma once

#include <stdint.h>

#include "bg_device.h"
#include "bg_kernels.h"

namespace bg {
namespace quadk {

struct Q {  // the lane's component of a complex four-vector, or a complex scalar
  double re, im;
};

__device__ __forceinline__ double dpp_d(double x, int ctrl) {
  // quad_perm moves stay inside the quad: every source lane exists
  const int lo = ctrl == 0xB1 ? __builtin_amdgcn_mov_dpp(__double2loint(x), 0xB1, 0xF, 0xF, true)
                              : __builtin_amdgcn_mov_dpp(__double2loint(x), 0x4E, 0xF, 0xF, true);
  const int hi = ctrl == 0xB1 ? __builtin_amdgcn_mov_dpp(__double2hiint(x), 0xB1, 0xF, 0xF, true)
                              : __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x4E, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// sum over the quad: ((x0 + x1) + (x2 + x3)) in all four lanes
__device__ __forceinline__ double qsum(double x) {
  const double y = x + dpp_d(x, 0xB1);
  return y + dpp_d(y, 0x4E);
}

// complex Minkowski product a.b from the lanes' components, with b's
// component already multiplied by the lane's metric sign (bg = g_c b_c)
__device__ __forceinline__ Q qdot_g(const Q& a, const Q& bg) {
  double pr = a.re * bg.re;
  pr -= a.im * bg.im;
  double pi = a.re * bg.im;
  pi += a.im * bg.re;
  return Q{qsum(pr), qsum(pi)};
}

__device__ __forceinline__ Q qdot(const Q& a, const Q& b, double g) {
  return qdot_g(a, Q{g * b.re, g * b.im});
}

// real-complex product p.a (p: the lane's component)
__device__ __forceinline__ Q qrdot(double p, const Q& a, double g) {
  const double gp = g * p;
  return Q{qsum(gp * a.re), qsum(gp * a.im)};
}

// acc += s v (complex scalar s, complex component v)
__device__ __forceinline__ void cax(Q& acc, const Q& s, const Q& v) {
  acc.re += s.re * v.re;
  acc.re -= s.im * v.im;
  acc.im += s.re * v.im;
  acc.im += s.im * v.re;
}

template <int N>
struct State {
  static constexpr int M = N - 1;
  Q J[M][M];      // [a][b]: the lane's component of J(a..b), a <= b
  double P0[M];   // prefix momentum P(0..b), the lane's component
  double Pg[M];   // momentum of the gluon at each position
  Q Gd[M];        // [a]: g_c times the component of J(a..d), d the column being built
};

// Per-lane context: gluons 1..n-1 of the lane's item in LDS, three FP64
// values per gluon and lane (polarization component re, im; momentum
// component).
struct Ctx {
  double* gl;  // [3 (g-1) + x][lane]
  int lane;
  double g;    // metric sign of the lane's component: +1 for c = 0, -1 otherwise
  Q epsN;      // the closing gluon's polarization component
};

template <int N>
struct Lds {
  static constexpr size_t bytes() { return sizeof(double) * (size_t)3 * (N - 1) * 64; }
};

template <int N, int A, int B>
__device__ __forceinline__ double range_mom(const State<N>& s) {
  if constexpr (A == B) return s.Pg[A];
  else if constexpr (A == 0) return s.P0[B];
  else return s.P0[B] - s.P0[A - 1];
}

// J(A..D) from the ranges of columns < D and the ranges (k+1..D), k >= A, of
// column D (pairk::build_range in one component per lane)
template <int N, int D, int A>
__device__ __forceinline__ void build_range(State<N>& s, const Ctx& c, Q& top) {
  constexpr int M = N - 1;
  constexpr bool kTop = (A == 0 && D == M - 1);
  constexpr int NS = D - A;
  // keep each range's code together: scheduling across ranges of the fully
  // unrolled path raises the register demand past the file (n = 8: 527
  // registers and spills without the barrier, 460 with it)
  __builtin_amdgcn_sched_barrier(0);
  Q coefL[NS], coefR[NS];
  Q acc{0.0, 0.0};
  // splits: three-gluon vertices
#pragma unroll
  for (int k = A; k < D; ++k) {
    double PL, PR;
    // range momenta through the template helper (k is a compile-time index
    // after unrolling; the prefix form covers every case)
    PL = (k == A) ? s.Pg[A] : (A == 0 ? s.P0[k] : s.P0[k] - s.P0[A - 1]);
    PR = (k + 1 == D) ? s.Pg[D] : s.P0[D] - s.P0[k];
    const Q d = qdot_g(s.J[A][k], s.Gd[k + 1]);
    coefR[k - A] = qrdot(2.0 * PR + PL, s.J[A][k], c.g);
    const Q c2 = qrdot(2.0 * PL + PR, s.J[k + 1][D], c.g);
    coefL[k - A] = Q{-c2.re, -c2.im};
    const double dif = PL - PR;
    acc.re += d.re * dif;
    acc.im += d.im * dif;
  }
  // triples: four-gluon vertices
#pragma unroll
  for (int j = A; j < D; ++j) {
#pragma unroll
    for (int k = j + 1; k < D; ++k) {
      const Q xy = qdot(s.J[A][j], s.J[j + 1][k], c.g);
      const Q yz = qdot_g(s.J[j + 1][k], s.Gd[k + 1]);
      const Q xz = qdot_g(s.J[A][j], s.Gd[k + 1]);
      coefL[j - A].re -= yz.re;
      coefL[j - A].im -= yz.im;
      coefR[k - A].re -= xy.re;
      coefR[k - A].im -= xy.im;
      cax(acc, Q{2.0 * xz.re, 2.0 * xz.im}, s.J[j + 1][k]);
    }
  }
#pragma unroll
  for (int k = A; k < D; ++k) {
    cax(acc, coefL[k - A], s.J[A][k]);
    cax(acc, coefR[k - A], s.J[k + 1][D]);
  }
  if constexpr (kTop) {
    top = qdot(c.epsN, acc, c.g);
  } else {
    const double pv = A == 0 ? s.P0[D] : s.P0[D] - s.P0[A - 1];
    const double ip2 = 1.0 / qsum(c.g * pv * pv);
    s.J[A][D] = Q{acc.re * ip2, acc.im * ip2};
    s.Gd[A] = Q{c.g * s.J[A][D].re, c.g * s.J[A][D].im};
  }
}

template <int N, int D, int A>
__device__ __forceinline__ void build_column(State<N>& s, const Ctx& c, Q& top) {
  if constexpr (A >= 0) {
    build_range<N, D, A>(s, c, top);
    build_column<N, D, A - 1>(s, c, top);
  }
}

// Positions D .. n-2 of the ordering coded 4 bits per position (position D
// in bits 4 (D - 1)), the closing gluon in bits 4 (n - 2), as pathk::path.
template <int N, int D>
__device__ __forceinline__ void path(State<N>& s, Ctx& c, uint32_t code, Q& top) {
  constexpr int M = N - 1;
  int g = (int)((code >> (4 * (D - 1))) & 15u);
  g = g < 1 ? 1 : (g > N - 1 ? N - 1 : g);  // codes hold 1..N-1; keeps LDS reads in bounds
  const int base = 3 * (g - 1);
  s.J[D][D] = Q{c.gl[(base + 0) * 64 + c.lane], c.gl[(base + 1) * 64 + c.lane]};
  s.Pg[D] = c.gl[(base + 2) * 64 + c.lane];
  s.P0[D] = s.P0[D - 1] + s.Pg[D];
  s.Gd[D] = Q{c.g * s.J[D][D].re, c.g * s.J[D][D].im};
  if constexpr (D == M - 1) {
    int gl = (int)((code >> (4 * (N - 2))) & 15u);
    gl = gl < 1 ? 1 : (gl > N - 1 ? N - 1 : gl);
    c.epsN = Q{c.gl[(3 * (gl - 1) + 0) * 64 + c.lane], c.gl[(3 * (gl - 1) + 1) * 64 + c.lane]};
  }
  build_column<N, D, D - 1>(s, c, top);
  if constexpr (D < M - 1) path<N, D + 1>(s, c, code, top);
}

// The lane's component c of a four-vector held in a register array (no
// indexed stack access)
__device__ __forceinline__ double comp(const double v[4], int c) {
  return c == 0 ? v[0] : (c == 1 ? v[1] : (c == 2 ? v[2] : v[3]));
}

// Set-up for event e on this quad: gluon 0 into the state, gluons 1..n-1 into
// the lane's LDS slots (each lane reads back only its own slots).
template <int N>
__device__ __forceinline__ void setup(State<N>& s, Ctx& c, double* lds, int64_t E,
                                      const double* __restrict__ mom,
                                      const int8_t* __restrict__ hel, int hconf, int64_t e) {
  const int lane = threadIdx.x & 63;
  const int cc = lane & 3;
  c.gl = lds;
  c.lane = lane;
  c.g = cc == 0 ? 1.0 : -1.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double p[4], er[4], ei[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) p[m] = mom[((int64_t)i * 4 + m) * E + e];
    const int hh = hel ? (int)hel[(int64_t)i * E + e] : (((hconf >> (N - 1 - i)) & 1) ? -1 : 1);
    polarization(p, hh, er, ei);
    const double vr = comp(er, cc), vi = comp(ei, cc), vp = comp(p, cc);
    if (i == 0) {
      s.J[0][0] = Q{vr, vi};
      s.Pg[0] = vp;
      s.P0[0] = vp;
    } else {
      c.gl[(3 * (i - 1) + 0) * 64 + lane] = vr;
      c.gl[(3 * (i - 1) + 1) * 64 + lane] = vi;
      c.gl[(3 * (i - 1) + 2) * 64 + lane] = vp;
    }
  }
}

}  // namespace quadk
}  // namespace bg
