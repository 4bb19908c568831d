// Adjoint of the colour-summed |M|^2 of the colour-ordered recursion with
// respect to the momenta (reverse mode, recomputed currents).
//
// me2 = sum_{s,t} C_st Re(A_s conj(A_t)) (Section 2.2, eq. color_summed_analytic),
// A_s from the recursion of Section 2.3 (eqs. cobg, cobg_full_amplitude).
// Adjoints follow dL = Re(zbar dz) for every complex intermediate z, so that
// for z = u v: ubar += zbar v, vbar += zbar u, and for a real r entering
// z = r u: rbar += Re(zbar u).  With Y = C A the seed is
// Abar_s = 2 g_e conj(Y_s), g_e the upstream gradient of event e.
//
// Per ordering the range currents are recomputed (nothing of the 2^n subset
// space is stored), the top amplitude is seeded and the ranges are swept from
// the longest to the shortest, back-propagating through the propagator
// (1/P^2 from the FP64 invariant table), the three- and four-gluon vertices
// and the range momenta.  Adjoints of the external currents are finally pulled
// back to the momenta through the Jacobian of the polarization construction
// (forward-mode dual numbers in FP64).  Gluon adjoints are accumulated in
// FP64.  Layout: one event per lane pair, as in the forward kernel.
#include <stdint.h>

#include "bg_device.h"
#include "bg_kernels.h"
#include "bg_pair.h"

namespace bg {
namespace adjk {

using pairk::Cx;
using pairk::H;
using pairk::HR;
using pairk::hdot;
using pairk::hrdot;
using pairk::pair_sum;

// LDS per 64-lane block (32 events), all in the recursion type T:
//   [6 g + x][lane]     eps half (4) and p half (2) of every gluon g
//   [mask][pair]        1/P_S^2 (formed in FP64)
//   [6 g + x][lane]     adjoint accumulators: eps_bar half (4), p_bar half (2)
//   [4 r + x][lane]     forward current halves of range r = tri(a, b), a < b
//   [2 r + x][lane]     range momentum halves of range r
// Single-gluon ranges are read from the gluon slots.  FP64 momenta for the
// range-momentum prefix sums are re-read from global memory (L1/L2 hits).
template <int N>
struct Lds {
  static constexpr int kLanes = 64, kPairs = 32;
  static constexpr int kTab = 1 << (N - 1);
  static constexpr int M = N - 1;
  static constexpr int kR = M * (M - 1) / 2;  // ranges (a, b), a < b
  template <typename T>
  static constexpr size_t bytes() {
    return sizeof(T) * ((size_t)12 * N * kLanes + (size_t)kTab * kPairs + (size_t)6 * kR * kLanes);
  }
};

// index of range (a, b), a < b, among the ranges of positions 0..M-1
template <int M>
__device__ __forceinline__ constexpr int tri(int a, int b) {
  return a * (2 * M - a - 1) / 2 + (b - a - 1);
}

template <int N, typename T>
struct Ctx {
  T* jl;        // [4 r + x][lane]
  T* pl;        // [2 r + x][lane]
  T* gsl;       // [6 g + x][lane]
  T* ip2;       // [mask][pair]
  T* acc;       // [6 g + x][lane]
  int lane, pair, h;
  T g0;
};

template <typename T>
__device__ __forceinline__ void zero(H<T>& v) {
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    v.re[m] = T(0);
    v.im[m] = T(0);
  }
}

// metric factor of the lane's component m
template <typename T>
__device__ __forceinline__ T gm(T g0, int m) {
  return m == 0 ? g0 : T(-1);
}

// plain (non-metric) complex sum over all four components of a.b
template <typename T>
__device__ __forceinline__ Cx<T> psum(const H<T>& a, const H<T>& b) {
  T r = 0, i = 0;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    r += a.re[m] * b.re[m];
    r -= a.im[m] * b.im[m];
    i += a.re[m] * b.im[m];
    i += a.im[m] * b.re[m];
  }
  return Cx<T>{pair_sum(r), pair_sum(i)};
}

template <typename T>
__device__ __forceinline__ Cx<T> psumr(const H<T>& a, const HR<T>& d) {
  T r = 0, i = 0;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    r += a.re[m] * d.v[m];
    i += a.im[m] * d.v[m];
  }
  return Cx<T>{pair_sum(r), pair_sum(i)};
}

// y += s * x (complex scalar times half vector)
template <typename T>
__device__ __forceinline__ void axpy(H<T>& y, Cx<T> s, const H<T>& x) {
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    y.re[m] += s.re * x.re[m];
    y.re[m] -= s.im * x.im[m];
    y.im[m] += s.re * x.im[m];
    y.im[m] += s.im * x.re[m];
  }
}

// y += s * g * x (metric-weighted)
template <typename T>
__device__ __forceinline__ void axpyg(H<T>& y, Cx<T> s, const H<T>& x, T g0) {
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const T g = gm(g0, m);
    const T gr = g * s.re, gi = g * s.im;
    y.re[m] += gr * x.re[m];
    y.re[m] -= gi * x.im[m];
    y.im[m] += gr * x.im[m];
    y.im[m] += gi * x.re[m];
  }
}

template <typename T>
__device__ __forceinline__ void axpygr(H<T>& y, Cx<T> s, const HR<T>& x, T g0) {
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const T g = gm(g0, m);
    y.re[m] += g * s.re * x.v[m];
    y.im[m] += g * s.im * x.v[m];
  }
}

template <typename T>
__device__ __forceinline__ void v3(H<T>& acc, const HR<T>& P, const HR<T>& Q, const H<T>& A,
                                   const H<T>& B, T g0) {
  HR<T> q2p, p2q;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    q2p.v[m] = T(2) * Q.v[m] + P.v[m];
    p2q.v[m] = T(2) * P.v[m] + Q.v[m];
  }
  const Cx<T> s = hdot(A, B, g0);
  const Cx<T> c1 = hrdot(q2p, A, g0);
  const Cx<T> c2 = hrdot(p2q, B, g0);
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const T d = P.v[m] - Q.v[m];
    acc.re[m] += s.re * d;
    acc.re[m] += c1.re * B.re[m];
    acc.re[m] -= c1.im * B.im[m];
    acc.re[m] -= c2.re * A.re[m];
    acc.re[m] += c2.im * A.im[m];
    acc.im[m] += s.im * d;
    acc.im[m] += c1.re * B.im[m];
    acc.im[m] += c1.im * B.re[m];
    acc.im[m] -= c2.re * A.im[m];
    acc.im[m] -= c2.im * A.re[m];
  }
}

template <typename T>
__device__ __forceinline__ void v4(H<T>& acc, const H<T>& J1, const H<T>& J2, const H<T>& J3,
                                   T g0) {
  Cx<T> d13 = hdot(J1, J3, g0);
  const Cx<T> d23 = hdot(J2, J3, g0);
  const Cx<T> d12 = hdot(J1, J2, g0);
  d13.re *= T(2);
  d13.im *= T(2);
  axpy(acc, d13, J2);
  axpy(acc, Cx<T>{-d23.re, -d23.im}, J1);
  axpy(acc, Cx<T>{-d12.re, -d12.im}, J3);
}

// Back-propagate V = V3(P, Q; A, B) with adjoint Vb.
template <typename T>
__device__ __forceinline__ void v3_adj(const H<T>& Vb, const HR<T>& P, const HR<T>& Q,
                                       const H<T>& A, const H<T>& B, H<T>& Ab, H<T>& Bb,
                                       HR<double>& Pb, HR<double>& Qb, T g0) {
  HR<T> q2p, p2q, d;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    q2p.v[m] = T(2) * Q.v[m] + P.v[m];
    p2q.v[m] = T(2) * P.v[m] + Q.v[m];
    d.v[m] = P.v[m] - Q.v[m];
  }
  const Cx<T> s = hdot(A, B, g0);
  const Cx<T> c1 = hrdot(q2p, A, g0);
  const Cx<T> c2 = hrdot(p2q, B, g0);
  const Cx<T> sb = psumr(Vb, d);
  const Cx<T> c1b = psum(Vb, B);
  Cx<T> c2b = psum(Vb, A);
  c2b.re = -c2b.re;
  c2b.im = -c2b.im;
  axpy(Bb, c1, Vb);
  axpy(Ab, Cx<T>{-c2.re, -c2.im}, Vb);
  axpyg(Ab, sb, B, g0);
  axpyg(Bb, sb, A, g0);
  axpygr(Ab, c1b, q2p, g0);
  axpygr(Bb, c2b, p2q, g0);
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const T g = gm(g0, m);
    const double db = (double)(s.re * Vb.re[m] - s.im * Vb.im[m]);
    const double qb = (double)(g * (c1b.re * A.re[m] - c1b.im * A.im[m]));
    const double pb = (double)(g * (c2b.re * B.re[m] - c2b.im * B.im[m]));
    Pb.v[m] += db + qb + 2.0 * pb;
    Qb.v[m] += -db + 2.0 * qb + pb;
  }
}

// Back-propagate V = 2 (J1.J3) J2 - (J2.J3) J1 - (J1.J2) J3.
template <typename T>
__device__ __forceinline__ void v4_adj(const H<T>& Vb, const H<T>& J1, const H<T>& J2,
                                       const H<T>& J3, H<T>& B1, H<T>& B2, H<T>& B3, T g0) {
  const Cx<T> d13 = hdot(J1, J3, g0);
  const Cx<T> d23 = hdot(J2, J3, g0);
  const Cx<T> d12 = hdot(J1, J2, g0);
  Cx<T> d13b = psum(Vb, J2);
  d13b.re *= T(2);
  d13b.im *= T(2);
  Cx<T> d23b = psum(Vb, J1);
  d23b.re = -d23b.re;
  d23b.im = -d23b.im;
  Cx<T> d12b = psum(Vb, J3);
  d12b.re = -d12b.re;
  d12b.im = -d12b.im;
  axpy(B2, Cx<T>{T(2) * d13.re, T(2) * d13.im}, Vb);
  axpy(B1, Cx<T>{-d23.re, -d23.im}, Vb);
  axpy(B3, Cx<T>{-d12.re, -d12.im}, Vb);
  axpyg(B1, d13b, J3, g0);
  axpyg(B3, d13b, J1, g0);
  axpyg(B2, d23b, J3, g0);
  axpyg(B3, d23b, J2, g0);
  axpyg(B1, d12b, J2, g0);
  axpyg(B2, d12b, J1, g0);
}

template <int N, typename T>
struct St {
  static constexpr int M = N - 1;
  H<T> Jb[M][M];
  HR<double> pb[M];  // momentum adjoint per position
  int gl[M];
};

// current of range (a, b): a gluon slot for a == b, else the stored range
template <int N, typename T>
__device__ __forceinline__ H<T> ldJ(const Ctx<N, T>& c, const St<N, T>& s, int a, int b) {
  H<T> v;
  if (a == b) {
    const T* g = c.gsl + (size_t)6 * s.gl[a] * 64 + c.lane;
    v.re[0] = g[0];
    v.re[1] = g[64];
    v.im[0] = g[128];
    v.im[1] = g[192];
  } else {
    const int r = tri<N - 1>(a, b);
    v.re[0] = c.jl[(4 * r + 0) * 64 + c.lane];
    v.re[1] = c.jl[(4 * r + 1) * 64 + c.lane];
    v.im[0] = c.jl[(4 * r + 2) * 64 + c.lane];
    v.im[1] = c.jl[(4 * r + 3) * 64 + c.lane];
  }
  return v;
}

template <int N, typename T>
__device__ __forceinline__ void stJ(const Ctx<N, T>& c, int a, int b, const H<T>& v) {
  const int r = tri<N - 1>(a, b);
  c.jl[(4 * r + 0) * 64 + c.lane] = v.re[0];
  c.jl[(4 * r + 1) * 64 + c.lane] = v.re[1];
  c.jl[(4 * r + 2) * 64 + c.lane] = v.im[0];
  c.jl[(4 * r + 3) * 64 + c.lane] = v.im[1];
}

template <int N, typename T>
__device__ __forceinline__ HR<T> ldP(const Ctx<N, T>& c, const St<N, T>& s, int a, int b) {
  HR<T> v;
  if (a == b) {
    const T* g = c.gsl + (size_t)(6 * s.gl[a] + 4) * 64 + c.lane;
    v.v[0] = g[0];
    v.v[1] = g[64];
  } else {
    const int r = tri<N - 1>(a, b);
    v.v[0] = c.pl[(2 * r + 0) * 64 + c.lane];
    v.v[1] = c.pl[(2 * r + 1) * 64 + c.lane];
  }
  return v;
}

template <int N, typename T>
__device__ __forceinline__ void stP(const Ctx<N, T>& c, int a, int b, const HR<T>& v) {
  const int r = tri<N - 1>(a, b);
  c.pl[(2 * r + 0) * 64 + c.lane] = v.v[0];
  c.pl[(2 * r + 1) * 64 + c.lane] = v.v[1];
}

template <int N, typename T>
__device__ __forceinline__ int range_mask(const St<N, T>& s, int a, int b) {
  int m = 0;
#pragma unroll
  for (int i = 0; i < N - 1; ++i)
    if (i >= a && i <= b) m |= 1 << s.gl[i];
  return m;
}

template <int N, typename T>
__global__ void __launch_bounds__(64) cobg_adj_kernel(int64_t E, const double* __restrict__ mom,
                                                     const int8_t* __restrict__ hel,
                                                     const double* __restrict__ Y,
                                                     const double* __restrict__ gme2,
                                                     const uint8_t* __restrict__ perms,
                                                     double* __restrict__ grad) {
  extern __shared__ __align__(16) unsigned char bg_adj_lds[];
  constexpr int M = N - 1;
  constexpr int K = (int)Factorial<N - 2>::value;
  using L = Lds<N>;
  const int lane = threadIdx.x, pair = lane >> 1, h = lane & 1;
  const int64_t e = (int64_t)blockIdx.x * L::kPairs + pair;
  if (e >= E) return;
  Ctx<N, T> c;
  c.gsl = reinterpret_cast<T*>(bg_adj_lds);
  c.acc = c.gsl + (size_t)6 * N * L::kLanes;
  c.ip2 = c.acc + (size_t)6 * N * L::kLanes;
  c.jl = c.ip2 + (size_t)L::kTab * L::kPairs;
  c.pl = c.jl + (size_t)4 * L::kR * L::kLanes;
  c.lane = lane;
  c.pair = pair;
  c.h = h;
  c.g0 = h == 0 ? T(1) : T(-1);
  const bool hi = h != 0;

  // set-up: the momenta and helicities are read again for the final
  // pull-back instead of being held in registers through the orderings
  {
  double p[N][4];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int m = 0; m < 4; ++m) p[i][m] = mom[((int64_t)i * 4 + m) * E + e];
  int hv[N];
#pragma unroll
  for (int i = 0; i < N; ++i) hv[i] = (int)hel[(int64_t)i * E + e];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double er[4], ei[4];
    polarization(p[i], hv[i], er, ei);
    // lane-dependent halves by branch (constant indices on both sides)
    double v[6];
    if (hi) {
      v[0] = er[2]; v[1] = er[3]; v[2] = ei[2]; v[3] = ei[3]; v[4] = p[i][2]; v[5] = p[i][3];
    } else {
      v[0] = er[0]; v[1] = er[1]; v[2] = ei[0]; v[3] = ei[1]; v[4] = p[i][0]; v[5] = p[i][1];
    }
#pragma unroll
    for (int x = 0; x < 6; ++x) c.gsl[(6 * i + x) * L::kLanes + lane] = (T)v[x];
#pragma unroll
    for (int x = 0; x < 6; ++x) c.acc[(6 * i + x) * L::kLanes + lane] = T(0);
  }
  for (int mask = h; mask < L::kTab; mask += 2) {
    double q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < M; ++i)
      if (mask & (1 << i)) {
#pragma unroll
        for (int m = 0; m < 4; ++m) q[m] += p[i][m];
      }
    const double p2 = q[0] * q[0] - q[1] * q[1] - q[2] * q[2] - q[3] * q[3];
    c.ip2[mask * L::kPairs + pair] = (T)(1.0 / p2);
  }
  }
  __syncthreads();

  const double ge = gme2 ? gme2[e] : 1.0;
  double scale = 1.0;
#pragma unroll
  for (int i = 0; i < N - 2; ++i) scale *= kGsOverSqrt2;
  H<T> epsN;
  epsN.re[0] = c.gsl[(6 * (N - 1) + 0) * L::kLanes + lane];
  epsN.re[1] = c.gsl[(6 * (N - 1) + 1) * L::kLanes + lane];
  epsN.im[0] = c.gsl[(6 * (N - 1) + 2) * L::kLanes + lane];
  epsN.im[1] = c.gsl[(6 * (N - 1) + 3) * L::kLanes + lane];
  H<double> epsNb;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    epsNb.re[m] = 0.0;
    epsNb.im[m] = 0.0;
  }

  St<N, T> s;
  for (int sig = 0; sig < K; ++sig) {  // wave-uniform
    s.gl[0] = 0;
#pragma unroll
    for (int k = 1; k < M; ++k) s.gl[k] = perms[sig * (N - 2) + (k - 1)];
    // range momenta: FP64 prefix sums of the positions' momenta (re-read
    // from global memory), differences rounded once to T
    HR<double> P0[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const int g = s.gl[k];
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const double pg = mom[((int64_t)g * 4 + 2 * h + m) * E + e];
        P0[k].v[m] = k == 0 ? pg : P0[k - 1].v[m] + pg;
      }
      s.pb[k].v[0] = 0.0;
      s.pb[k].v[1] = 0.0;
    }
#pragma unroll
    for (int a = 0; a < M; ++a)
#pragma unroll
      for (int b = a + 1; b < M; ++b) {
        if (a == 0 && b == M - 1) continue;  // the top range's momentum is not needed
        HR<T> pr;
#pragma unroll
        for (int m = 0; m < 2; ++m)
          pr.v[m] = (T)(a == 0 ? P0[b].v[m] : P0[b].v[m] - P0[a - 1].v[m]);
        stP(c, a, b, pr);
      }
    // forward
    H<T> top;
#pragma unroll
    for (int len = 2; len <= M; ++len) {
#pragma unroll
      for (int a = 0; a + len - 1 < M; ++a) {
        const int b = a + len - 1;
        H<T> acc;
        zero(acc);
#pragma unroll
        for (int k = a; k < b; ++k)
          v3(acc, ldP(c, s, a, k), ldP(c, s, k + 1, b), ldJ(c, s, a, k), ldJ(c, s, k + 1, b), c.g0);
#pragma unroll
        for (int j = a; j < b; ++j)
#pragma unroll
          for (int k = j + 1; k < b; ++k)
            v4(acc, ldJ(c, s, a, j), ldJ(c, s, j + 1, k), ldJ(c, s, k + 1, b), c.g0);
        if (len == M) {
          top = acc;
        } else {
          const T ip = c.ip2[range_mask(s, a, b) * L::kPairs + pair];
          H<T> jn;
#pragma unroll
          for (int m = 0; m < 2; ++m) {
            jn.re[m] = acc.re[m] * ip;
            jn.im[m] = acc.im[m] * ip;
          }
          stJ(c, a, b, jn);
        }
      }
    }
    // seed: Abar = 2 g_e conj(Y_sigma); A = scale * eps_N . top
    const double yr = Y[(int64_t)sig * E + e], yi = Y[((int64_t)K + sig) * E + e];
    const Cx<T> ab{(T)(2.0 * ge * yr * scale), (T)(-2.0 * ge * yi * scale)};
#pragma unroll
    for (int a = 0; a < M; ++a)
#pragma unroll
      for (int b = a; b < M; ++b) zero(s.Jb[a][b]);
    H<T> topb;
    zero(topb);
    axpyg(topb, ab, epsN, c.g0);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const T g = gm(c.g0, m);
      epsNb.re[m] += (double)(g * (ab.re * top.re[m] - ab.im * top.im[m]));
      epsNb.im[m] += (double)(g * (ab.re * top.im[m] + ab.im * top.re[m]));
    }
    // backward sweep, longest ranges first
#pragma unroll
    for (int len = M; len >= 2; --len) {
#pragma unroll
      for (int a = 0; a + len - 1 < M; ++a) {
        const int b = a + len - 1;
        H<T> accb;
        if (len == M) {
          accb = topb;
        } else {
          const int mk = range_mask(s, a, b);
          const T ip = c.ip2[mk * L::kPairs + pair];
#pragma unroll
          for (int m = 0; m < 2; ++m) {
            accb.re[m] = s.Jb[a][b].re[m] * ip;
            accb.im[m] = s.Jb[a][b].im[m] * ip;
          }
          // J = acc ip, ip = 1/(P.P): ip_bar = Re sum Jb acc = Re(sum Jb J) P^2 and
          // Pbar_m += ip_bar d ip / dP_m = Re(sum Jb J) (-2 g_m P_m) ip
          const Cx<T> jj = psum(s.Jb[a][b], ldJ(c, s, a, b));
          const HR<T> pab = ldP(c, s, a, b);
#pragma unroll
          for (int m = 0; m < 2; ++m) {
            const double v =
                (double)jj.re * (-2.0 * (double)gm(c.g0, m) * (double)pab.v[m]) * (double)ip;
#pragma unroll
            for (int i = a; i <= b; ++i) s.pb[i].v[m] += v;
          }
        }
#pragma unroll
        for (int k = a; k < b; ++k) {
          HR<double> PLb{{0.0, 0.0}}, PRb{{0.0, 0.0}};
          v3_adj(accb, ldP(c, s, a, k), ldP(c, s, k + 1, b), ldJ(c, s, a, k), ldJ(c, s, k + 1, b), s.Jb[a][k],
                 s.Jb[k + 1][b], PLb, PRb, c.g0);
#pragma unroll
          for (int m = 0; m < 2; ++m) {
#pragma unroll
            for (int i = a; i <= k; ++i) s.pb[i].v[m] += PLb.v[m];
#pragma unroll
            for (int i = k + 1; i <= b; ++i) s.pb[i].v[m] += PRb.v[m];
          }
        }
#pragma unroll
        for (int j = a; j < b; ++j)
#pragma unroll
          for (int k = j + 1; k < b; ++k)
            v4_adj(accb, ldJ(c, s, a, j), ldJ(c, s, j + 1, k), ldJ(c, s, k + 1, b), s.Jb[a][j],
                   s.Jb[j + 1][k], s.Jb[k + 1][b], c.g0);
      }
    }
    // gluon accumulators (type T; the per-ordering momentum adjoints are
    // summed in FP64 first)
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const int g = s.gl[k];
      T* ac = c.acc + (size_t)6 * g * L::kLanes + lane;
      ac[0 * L::kLanes] += s.Jb[k][k].re[0];
      ac[1 * L::kLanes] += s.Jb[k][k].re[1];
      ac[2 * L::kLanes] += s.Jb[k][k].im[0];
      ac[3 * L::kLanes] += s.Jb[k][k].im[1];
      ac[4 * L::kLanes] += (T)s.pb[k].v[0];
      ac[5 * L::kLanes] += (T)s.pb[k].v[1];
    }
  }
  // pull the external-current adjoints back to the momenta
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const T* ac = c.acc + (size_t)6 * i * L::kLanes + lane;
    double ebr0 = ac[0], ebr1 = ac[L::kLanes], ebi0 = ac[2 * L::kLanes], ebi1 = ac[3 * L::kLanes];
    if (i == N - 1) {
      ebr0 += epsNb.re[0];
      ebr1 += epsNb.re[1];
      ebi0 += epsNb.im[0];
      ebi1 += epsNb.im[1];
    }
    double pi[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) pi[m] = mom[((int64_t)i * 4 + m) * E + e];
    double dre[4][4], dim[4][4];
    polarization_jacobian(pi, (int)hel[(int64_t)i * E + e], dre, dim);
    // this lane's eps_bar as a full four-vector with zeros in the partner's slots
    double ebr[4], ebi[4];
    if (hi) {
      ebr[0] = 0.0; ebr[1] = 0.0; ebr[2] = ebr0; ebr[3] = ebr1;
      ebi[0] = 0.0; ebi[1] = 0.0; ebi[2] = ebi0; ebi[3] = ebi1;
    } else {
      ebr[0] = ebr0; ebr[1] = ebr1; ebr[2] = 0.0; ebr[3] = 0.0;
      ebi[0] = ebi0; ebi[1] = ebi1; ebi[2] = 0.0; ebi[3] = 0.0;
    }
    double part[4];
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
      double t = 0.0;
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) t += ebr[mu] * dre[nu][mu] - ebi[mu] * dim[nu][mu];
      part[nu] = pair_sum(t);
    }
    const double pb0 = (double)ac[4 * L::kLanes], pb1 = (double)ac[5 * L::kLanes];
    if (hi) {
      grad[((int64_t)i * 4 + 2) * E + e] = pb0 + part[2];
      grad[((int64_t)i * 4 + 3) * E + e] = pb1 + part[3];
    } else {
      grad[((int64_t)i * 4 + 0) * E + e] = pb0 + part[0];
      grad[((int64_t)i * 4 + 1) * E + e] = pb1 + part[1];
    }
  }
}

template <int N, typename T>
int launch(int64_t E, const double* mom, const int8_t* hel, const double* Y, const double* gme2,
           const uint8_t* perms, double* grad, hipStream_t stream) {
  const unsigned grid = (unsigned)((E + Lds<N>::kPairs - 1) / Lds<N>::kPairs);
  hipLaunchKernelGGL((cobg_adj_kernel<N, T>), dim3(grid), dim3(64), (Lds<N>::template bytes<T>()),
                     stream, E, mom, hel, Y, gme2, perms, grad);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace adjk

int cobg_gradient(int n, bool fp32, int64_t E, const double* mom, const int8_t* hel,
                  const double* Y, const double* gme2, const uint8_t* perms, double* grad,
                  hipStream_t stream) {
  if (E <= 0) return 0;
  switch (n) {
    case 4: return fp32 ? adjk::launch<4, float>(E, mom, hel, Y, gme2, perms, grad, stream)
                        : adjk::launch<4, double>(E, mom, hel, Y, gme2, perms, grad, stream);
    case 5: return fp32 ? adjk::launch<5, float>(E, mom, hel, Y, gme2, perms, grad, stream)
                        : adjk::launch<5, double>(E, mom, hel, Y, gme2, perms, grad, stream);
    case 6: return fp32 ? adjk::launch<6, float>(E, mom, hel, Y, gme2, perms, grad, stream)
                        : adjk::launch<6, double>(E, mom, hel, Y, gme2, perms, grad, stream);
    case 7: return fp32 ? adjk::launch<7, float>(E, mom, hel, Y, gme2, perms, grad, stream)
                        : adjk::launch<7, double>(E, mom, hel, Y, gme2, perms, grad, stream);
    default: return -2;
  }
}

}  // namespace bg
