// Colour-ordered Berends-Giele recursion (Section 2.3, eqs. cobg and
// cobg_full_amplitude) for all (n-2)! orderings A(1, sigma, n) of the adjoint
// basis (Section 2.2, eq. color_decomposition_adjoint), one event per lane
// PAIR.
//
// Layout.  Lanes 2p and 2p+1 of a wave hold event p of the block's 32 events.
// Lane half h = lane & 1 owns Lorentz components 2h and 2h+1 of every current
// and momentum, so the per-lane register and LDS state is half that of one
// event per lane.  A Minkowski product is the sum of the two halves'
// partials, exchanged between partners with one DPP quad_perm [1,0,3,2]
// move (a + b and b + a are the same IEEE result, so both lanes hold
// bit-identical scalars).  The metric sign of the lane's first component is a
// per-lane constant g0 (+1 for h = 0, -1 for h = 1); the second is always -1.
//
// Walk.  Orderings are visited depth first in lexicographic order; position d
// of (1, sigma_2, .., sigma_{n-1}) is a template level and the gluon placed
// there a wave-uniform loop variable.  Entering level d builds the ranges
// (a..d), a = d-1 .. 0; the shallower columns stay live in VGPRs and are
// shared by every ordering with the same prefix.
//
// Per range R = (a..b) (couplings factored out, see bg_device.h):
//   Jhat(R) = sum_k [ d_k (P_L - P_R) + c1_k J_R - c2_k J_L ]
//           + sum_{j<k} [ 2 (X.Z) J_Y - (Y.Z) J_X - (X.Y) J_Z ],
// L = (a..k), R = (k+1..b), X = (a..j), Y = (j+1..k), Z = (k+1..b),
// d_k = J_L.J_R, c1_k = (2P_R + P_L).J_L, c2_k = (2P_L + P_R).J_R.  This is
// V3 summed over splits plus V4 summed over triples with the coefficients of
// each sub-current collected.  X.Y and Y.Z are the d's of ranges (a..k) and
// (j+1..b), kept in a table when those ranges are built, so a V4 needs one new
// product.  J(R) = Jhat(R) / P_R^2 with 1/P^2 taken from a per-event table
// formed in FP64 from the FP64 momenta (rounded once for T = float); the full
// range is amputated and contracted with eps_n.  Range momenta are
// differences of FP64 prefix sums, rounded once to T.
#pragma once

#include <stdint.h>

#include <utility>

#include "bg_device.h"
#include "bg_kernels.h"
#include "bg_pair.h"

namespace bg {
namespace pairk {

// LDS map per 64-lane block (32 events), NG movable gluons (1..NG):
//   T region, [slot][lane]: gluon g in 1..NG has eps half (4) and p half (2)
//     at slots 6 (g-1) .. 6 (g-1) + 5;
//   T region, [mask][pair]: 1/P_S^2 for subsets S of gluons 0..NG;
//   double region, [2 (g-1) + c][lane]: FP64 momentum halves of gluons 1..NG.
// Adjoint basis (LC = false): NG = N-2, gluon N-1 closes every ordering.
// Leading colour (LC = true): NG = N-1, all orderings (1, rho) of gluons
// 1..N-1; the gluon left after the others are placed closes the ordering.
// P64G: the FP64 momentum halves are re-read from global memory (L1/L2
// hits) instead of being kept in LDS, which saves 2 NG x 64 doubles where
// LDS is the occupancy limit.
template <int N, bool LC = false>
struct Lds {
  static constexpr int kLanes = 64;
  static constexpr int kPairs = 32;
  static constexpr int NG = LC ? N - 1 : N - 2;
  static constexpr int kGluonSlots = 6 * NG;
  static constexpr int kTabEntries = 1 << (NG + 1);
  template <typename T, bool P64G = false>
  static constexpr size_t bytes() {
    return sizeof(T) * ((size_t)kGluonSlots * kLanes + (size_t)kTabEntries * kPairs) +
           (P64G ? 0 : sizeof(double) * (size_t)(2 * NG) * kLanes);
  }
};

// RAW: amplitudes go unscaled, in T, to amp_raw[(h K + sigma) 32 + pair]
// (block-private LDS); otherwise scaled, in FP64, to
// amp[(h K + sigma) astride + acol].  P64G, LC: see Lds; with LC nothing is
// stored, lcsum accumulates this lane's plane of |A|^2 over the orderings.
template <int N, typename T, bool RAW, bool P64G, bool LC = false, bool EST = false>
struct Ctx {
  static constexpr bool kRaw = RAW;
  static constexpr bool kP64G = P64G;
  static constexpr bool kLC = LC;
  static constexpr bool kEst = EST;  // carry the rounding-error bounds (see State::Sb)
  static constexpr bool kDirectP2 = false;  // 1/P^2 from the per-event table
  static constexpr bool kNoDt = N >= 8;     // V4 dot products from the Dt table (n <= 7) or
                                            // recomputed (n = 8: the table would not fit)
  double lcsum;
  T est_s2, est_a2;   // EST: sum over orderings of Sb(top)^2 and of |A|^2
  const double* mom;
  T* gl_slots;      // [slot][lane]
  T* tab;           // [mask][pair]
  double* p64;      // [2 (g-1) + c][lane]
  int lane, pair;
  T g0;
  H<T> epsN;
  double* amp;
  T* amp_raw;
  int64_t E, e;       // input stride and event index
  int64_t astride;    // amplitude array stride (events per plane row)
  int64_t acol;       // amplitude column of this event
  bool live;          // false for padding pairs: compute, do not store
  int sigma;
  int h;
};

template <int N, typename T>
struct State {
  static constexpr int M = N - 1;
  H<T> J[M][M];
  Cx<T> Dt[M][M][M];  // [a][b][k] = J(a..k).J(k+1..b)
  HR<double> P0[M];   // prefix momenta P(0..b), FP64 halves
  HR<T> Pg[M];        // momentum half of the gluon at each position
  Cx<T> Gd[M];        // [a]: g0 times the lane's first component of J(a..d), d the
                      // column being built (the right operand of its products)
  int gl[M];          // gluon at each position (wave-uniform)
  // Rounding-error bounds (only with Ctx::kEst).  Sb[a][b] bounds the
  // components of J(a..b) as the recursion would if every product were taken
  // in modulus: Sb = 1 for a gluon (unit polarization components), and for a
  // range Sb = |1/P^2| (E(a..b) sum_k Sb_L Sb_R + sum_{j<k} Sb_X Sb_Y Sb_Z),
  // where E(a..b) = sum of |p^0| over the range bounds every momentum
  // component of a sub-range (the constant factors of the vertices are
  // dropped; only ratios of such bounds are used).  Ep[b] = E(0..b).
  T Sb[M][M];
  T Ep[M];
};

template <int N, typename T, int A, int D, class CtxT>
__device__ __forceinline__ void set_gd(State<N, T>& s, const CtxT& c) {
  s.Gd[A] = Cx<T>{c.g0 * s.J[A][D].re[0], c.g0 * s.J[A][D].im[0]};
}

template <int N, typename T, int A, int B>
__device__ __forceinline__ HR<T> range_mom(const State<N, T>& s) {
  HR<T> r;
  if constexpr (A == B) {
    r = s.Pg[A];
  } else if constexpr (A == 0) {
#pragma unroll
    for (int m = 0; m < 2; ++m) r.v[m] = (T)s.P0[B].v[m];
  } else {
#pragma unroll
    for (int m = 0; m < 2; ++m) r.v[m] = (T)(s.P0[B].v[m] - s.P0[A - 1].v[m]);
  }
  return r;
}

template <int N, typename T, int D, int A, class CtxT>
__device__ __forceinline__ void build_range(State<N, T>& s, const CtxT& c, int mask,
                                            Cx<T>& top, T& topb) {
  constexpr int M = N - 1;
  constexpr bool kTop = (A == 0 && D == M - 1);
  constexpr int NS = D - A;
  Cx<T> coefL[NS], coefR[NS];
  H<T> acc;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    acc.re[m] = T(0);
    acc.im[m] = T(0);
  }
  // splits: three-gluon vertices
  [&]<int... Ks>(std::integer_sequence<int, Ks...>) {
    (
        [&] {
          constexpr int k = A + Ks;
          const HR<T> PL = range_mom<N, T, A, k>(s);
          const HR<T> PR = range_mom<N, T, k + 1, D>(s);
          const Cx<T> d = hdot_g(s.J[A][k], s.J[k + 1][D], s.Gd[k + 1]);
          if constexpr (!kTop && !CtxT::kNoDt) s.Dt[A][D][k] = d;
          HR<T> q2p, p2q, dif;
#pragma unroll
          for (int m = 0; m < 2; ++m) {
            q2p.v[m] = T(2) * PR.v[m] + PL.v[m];
            p2q.v[m] = T(2) * PL.v[m] + PR.v[m];
            dif.v[m] = PL.v[m] - PR.v[m];
          }
          coefR[Ks] = hrdot(q2p, s.J[A][k], c.g0);
          const Cx<T> c2 = hrdot(p2q, s.J[k + 1][D], c.g0);
          coefL[Ks] = Cx<T>{-c2.re, -c2.im};
          craxpy(acc, d, dif);
        }(),
        ...);
  }(std::make_integer_sequence<int, NS>{});
  // triples: four-gluon vertices
#pragma unroll
  for (int j = A; j < D; ++j) {
#pragma unroll
    for (int k = j + 1; k < D; ++k) {
      Cx<T> xy, yz;
      if constexpr (CtxT::kNoDt) {
        xy = hdot(s.J[A][j], s.J[j + 1][k], c.g0);
        yz = hdot_g(s.J[j + 1][k], s.J[k + 1][D], s.Gd[k + 1]);
      } else {
        xy = s.Dt[A][k][j];
        yz = s.Dt[j + 1][D][k];
      }
      const Cx<T> xz = hdot_g(s.J[A][j], s.J[k + 1][D], s.Gd[k + 1]);
      coefL[j - A].re -= yz.re;
      coefL[j - A].im -= yz.im;
      coefR[k - A].re -= xy.re;
      coefR[k - A].im -= xy.im;
      caxpy(acc, Cx<T>{T(2) * xz.re, T(2) * xz.im}, s.J[j + 1][k]);
    }
  }
#pragma unroll
  for (int k = A; k < D; ++k) {
    caxpy(acc, coefL[k - A], s.J[A][k]);
    caxpy(acc, coefR[k - A], s.J[k + 1][D]);
  }
  T sb = T(0);
  if constexpr (CtxT::kEst) {
    T v3 = T(0), v4 = T(0);
#pragma unroll
    for (int k = A; k < D; ++k) v3 += s.Sb[A][k] * s.Sb[k + 1][D];
#pragma unroll
    for (int j = A; j < D; ++j)
#pragma unroll
      for (int k = j + 1; k < D; ++k) v4 += s.Sb[A][j] * s.Sb[j + 1][k] * s.Sb[k + 1][D];
    const T er = A == 0 ? s.Ep[D] : s.Ep[D] - s.Ep[A - 1];
    sb = er * v3 + v4;
  }
  if constexpr (kTop) {
    top = hdot(c.epsN, acc, c.g0);
    topb = sb;
  } else {
    T ip2;
    if constexpr (CtxT::kDirectP2) {
      // P(A..D)^2 from the FP64 prefix momenta (halves + partner exchange)
      double pv[2];
#pragma unroll
      for (int m = 0; m < 2; ++m)
        pv[m] = A == 0 ? s.P0[D].v[m] : s.P0[D].v[m] - s.P0[A - 1].v[m];
      const double part = (double)c.g0 * pv[0] * pv[0] - pv[1] * pv[1];
      ip2 = (T)(1.0 / pair_sum(part));
    } else {
      ip2 = c.tab[mask * Lds<N>::kPairs + c.pair];
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      s.J[A][D].re[m] = acc.re[m] * ip2;
      s.J[A][D].im[m] = acc.im[m] * ip2;
    }
    if constexpr (CtxT::kEst) s.Sb[A][D] = sb * fabs(ip2);
    set_gd<N, T, A, D>(s, c);
  }
}

template <int N, typename T, int D, int A, class CtxT>
__device__ __forceinline__ void build_column(State<N, T>& s, const CtxT& c, int mask,
                                             Cx<T>& top, T& topb) {
  if constexpr (A >= 0) {
    mask |= 1 << s.gl[A];
    build_range<N, T, D, A>(s, c, mask, top, topb);
    build_column<N, T, D, A - 1>(s, c, mask, top, topb);
  }
}

template <int N, typename T, int D, class CtxT>
__device__ __forceinline__ void level(State<N, T>& s, CtxT& c, int used) {
  constexpr int M = N - 1;
  constexpr int NG = CtxT::kLC ? N - 1 : N - 2;
  for (int g = 1; g <= NG; ++g) {  // wave-uniform
    if (used & (1 << g)) continue;
    s.gl[D] = g;
    const int base = 6 * (g - 1);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      s.J[D][D].re[m] = c.gl_slots[(base + m) * Lds<N>::kLanes + c.lane];
      s.J[D][D].im[m] = c.gl_slots[(base + 2 + m) * Lds<N>::kLanes + c.lane];
      s.Pg[D].v[m] = c.gl_slots[(base + 4 + m) * Lds<N>::kLanes + c.lane];
      double pg;
      if constexpr (CtxT::kP64G)
        pg = c.mom[((int64_t)g * 4 + 2 * c.h + m) * c.E + c.e];
      else
        pg = c.p64[(2 * (g - 1) + m) * Lds<N>::kLanes + c.lane];
      s.P0[D].v[m] = s.P0[D - 1].v[m] + pg;
      if constexpr (CtxT::kEst) {
        if (m == 0) {
          // |p^0| of the gluon: the h = 0 lane holds it, the h = 1 lane
          // takes it from its partner
          const double px = xswap(pg);
          s.Ep[D] = s.Ep[D - 1] + (T)fabs(c.h == 0 ? pg : px);
        }
      }
    }
    if constexpr (CtxT::kEst) s.Sb[D][D] = T(1);
    set_gd<N, T, D, D>(s, c);
    Cx<T> top;
    T topb = T(0);
    if constexpr (CtxT::kLC && D == M - 1) {
      // the one gluon not yet placed closes the ordering
      const int all = ((1 << (NG + 1)) - 1) & ~1;
      const int rem = __builtin_ctz(all & ~(used | (1 << g)));
      const int rb = 6 * (rem - 1);
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        c.epsN.re[m] = c.gl_slots[(rb + m) * Lds<N>::kLanes + c.lane];
        c.epsN.im[m] = c.gl_slots[(rb + 2 + m) * Lds<N>::kLanes + c.lane];
      }
    }
    build_column<N, T, D, D - 1>(s, c, 1 << g, top, topb);
    if constexpr (D == M - 1) {
      constexpr int64_t K = Factorial<N - 2>::value;
      if constexpr (CtxT::kEst) {
        c.est_s2 += topb * topb;
        c.est_a2 += top.re * top.re + top.im * top.im;
      }
      if constexpr (CtxT::kLC) {
        const double v = (double)(c.h == 0 ? top.re : top.im);
        c.lcsum += v * v;
      } else if constexpr (CtxT::kRaw) {
        c.amp_raw[(c.h * (int)K + c.sigma) * Lds<N>::kPairs + c.pair] = c.h == 0 ? top.re : top.im;
      } else {
        double scale = 1.0;
#pragma unroll
        for (int i = 0; i < N - 2; ++i) scale *= kGsOverSqrt2;
        const double v = (double)(c.h == 0 ? top.re : top.im) * scale;
        if (c.live) c.amp[((int64_t)c.h * K + c.sigma) * c.astride + c.acol] = v;
      }
      ++c.sigma;
    } else {
      level<N, T, D + 1>(s, c, used | (1 << g));
    }
  }
}

// Amplitudes of the event pair of this lane (event e of an [n][4][E] input);
// padding pairs (live = false) repeat a valid event and store nothing.  The
// block's waves must all call it (it synchronises the block); lds is this
// wave's region of Lds<N>::bytes<T>().  RAW: the
// unscaled amplitudes go to amp_raw (see Ctx), amp is unused.
//
// EST: also accumulate, over the orderings, est[0] += Sb(top)^2 and
// est[1] += |A|^2 (State::Sb); est[0] / est[1] is then the square of a
// bound on the amplitudes' rounding error relative to their size, the
// conditioning of this event's evaluation (identical in both lanes).
template <int N, typename T, bool RAW = false, bool P64G = false, bool LC = false,
          bool EST = false>
__device__ __forceinline__ double cobg_pair_body(unsigned char* lds, int64_t E,
                                               const double* __restrict__ mom,
                                               const int8_t* __restrict__ hel, int hconf,
                                               int64_t e, bool live, double* __restrict__ amp,
                                               int64_t astride, int64_t acol,
                                               T* amp_raw = nullptr, T* est = nullptr) {
  const int lane = threadIdx.x & 63;  // lane within this wave (the wave owns lds)
  const int pair = lane >> 1;
  const int h = lane & 1;
  using L = Lds<N, LC>;
  Ctx<N, T, RAW, P64G, LC, EST> c;
  c.lcsum = 0.0;
  c.est_s2 = T(0);
  c.est_a2 = T(0);
  c.mom = mom;
  c.gl_slots = reinterpret_cast<T*>(lds);
  c.tab = c.gl_slots + (size_t)L::kGluonSlots * L::kLanes;
  c.p64 = reinterpret_cast<double*>(c.tab + (size_t)L::kTabEntries * L::kPairs);
  c.lane = lane;
  c.pair = pair;
  c.h = h;
  c.g0 = h == 0 ? T(1) : T(-1);
  c.amp = amp;
  c.amp_raw = amp_raw;
  c.E = E;
  c.e = e;
  c.astride = astride;
  c.acol = acol;
  c.live = live;
  c.sigma = 0;

  double p[N][4];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int m = 0; m < 4; ++m) p[i][m] = mom[((int64_t)i * 4 + m) * E + e];

  State<N, T> s;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double er[4], ei[4];
    const int hh = hel ? (int)hel[(int64_t)i * E + e] : (((hconf >> (N - 1 - i)) & 1) ? -1 : 1);
    polarization(p[i], hh, er, ei);
    // select this lane's two components as values (no indexed stack array)
    const bool hi = h != 0;
    H<T> cur;
    cur.re[0] = (T)(hi ? er[2] : er[0]);
    cur.re[1] = (T)(hi ? er[3] : er[1]);
    cur.im[0] = (T)(hi ? ei[2] : ei[0]);
    cur.im[1] = (T)(hi ? ei[3] : ei[1]);
    double ph[2];
    ph[0] = hi ? p[i][2] : p[i][0];
    ph[1] = hi ? p[i][3] : p[i][1];
    if (i == 0) {
      s.J[0][0] = cur;
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        s.Pg[0].v[m] = (T)ph[m];
        s.P0[0].v[m] = ph[m];
      }
    } else if (i == N - 1 && !LC) {
      c.epsN = cur;
    } else {
      const int base = 6 * (i - 1);
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        c.gl_slots[(base + m) * Lds<N>::kLanes + lane] = cur.re[m];
        c.gl_slots[(base + 2 + m) * Lds<N>::kLanes + lane] = cur.im[m];
        c.gl_slots[(base + 4 + m) * Lds<N>::kLanes + lane] = (T)ph[m];
        if constexpr (!P64G) c.p64[(2 * (i - 1) + m) * Lds<N>::kLanes + lane] = ph[m];
      }
    }
  }
  // 1/P_S^2 table: the two lanes of a pair fill alternate subsets
  constexpr int MT = L::NG + 1;  // gluons that can appear in a range
  for (int mask = h; mask < (1 << MT); mask += 2) {
    double q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < MT; ++i) {
      if (mask & (1 << i)) {
#pragma unroll
        for (int m = 0; m < 4; ++m) q[m] += p[i][m];
      }
    }
    const double p2 = q[0] * q[0] - q[1] * q[1] - q[2] * q[2] - q[3] * q[3];
    c.tab[mask * Lds<N>::kPairs + pair] = (T)(1.0 / p2);
  }
  __syncthreads();
  s.gl[0] = 0;
  if constexpr (EST) {
    s.Sb[0][0] = T(1);
    s.Ep[0] = (T)fabs(p[0][0]);
  }
  level<N, T, 1>(s, c, 1);
  if constexpr (EST) {
    est[0] += c.est_s2;
    est[1] += c.est_a2;
  }
  return c.lcsum;
}

// Amplitudes of events e0 .. e0 + count - 1 of an [n][4][E] input into
// amp [2][K][count] (real plane, imaginary plane).
template <int N, typename T>
__global__ void __launch_bounds__(64) cobg_pair_kernel(int64_t E, int64_t e0, int64_t count,
                                                      const double* __restrict__ mom,
                                                      const int8_t* __restrict__ hel, int hconf,
                                                      double* __restrict__ amp) {
  extern __shared__ __align__(16) unsigned char bg_pair_lds[];
  const int64_t j = (int64_t)blockIdx.x * Lds<N>::kPairs + (threadIdx.x >> 1);
  const bool live = j < count;
  cobg_pair_body<N, T>(bg_pair_lds, E, mom, hel, hconf, e0 + (live ? j : count - 1), live, amp,
                       count, j);
}

}  // namespace pairk
}  // namespace bg
