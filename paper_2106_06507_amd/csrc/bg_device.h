// Device building blocks shared by the HIP kernels: complex Lorentz vectors,
// the colour-ordered three- and four-gluon vertices (Section 2.3) and the
// external polarization vectors (Section 2.1 projector eq. tensor_axial and its
// helicity split eq. helicity_axial).
//
// Everything here is templated on the arithmetic type T (float or double).
// Couplings are factored out of the recursion: with g' = g_s/sqrt2 every
// n-gluon diagram carries g'^(n-2), since V3 ~ g' and V4 ~ g_s^2/2 = g'^2.  The
// kernels therefore use V3 = (A.B)(P-Q) + ((2Q+P).A)B - ((2P+Q).B)A and
// V4 = 2(J1.J3)J2 - (J2.J3)J1 - (J1.J2)J3 without couplings or factors of i
// (the -i of each propagator cancels the i of each vertex) and multiply the
// amplitude by g'^(n-2) at the end.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bg {

// g_s = sqrt(4 pi alpha_s) with alpha_s = 0.118, and g_s / sqrt(2).
constexpr double kGs = 1.2177157847767197;        // sqrt(4*pi*0.118)
constexpr double kGsOverSqrt2 = 0.8610550889735169;

// Unit three-vector orienting the transverse plane of the polarizations.
constexpr double kR1 = 3.0 / 7.0, kR2 = -6.0 / 7.0, kR3 = 2.0 / 7.0;
constexpr double kInvSqrt2 = 0.70710678118654752440;

template <typename T>
struct R4 {
  T v[4];
};

template <typename T>
struct C4 {
  T re[4];
  T im[4];
};

template <typename T>
__device__ __forceinline__ R4<T> radd(const R4<T>& a, const R4<T>& b) {
  R4<T> r;
#pragma unroll
  for (int m = 0; m < 4; ++m) r.v[m] = a.v[m] + b.v[m];
  return r;
}

// complex Minkowski product a.b (no conjugation)
template <typename T>
__device__ __forceinline__ void cdot(const C4<T>& a, const C4<T>& b, T& re, T& im) {
  re = a.re[0] * b.re[0] - a.im[0] * b.im[0];
  im = a.re[0] * b.im[0] + a.im[0] * b.re[0];
#pragma unroll
  for (int m = 1; m < 4; ++m) {
    re -= a.re[m] * b.re[m] - a.im[m] * b.im[m];
    im -= a.re[m] * b.im[m] + a.im[m] * b.re[m];
  }
}

// real-complex Minkowski product p.a
template <typename T>
__device__ __forceinline__ void rdot(const R4<T>& p, const C4<T>& a, T& re, T& im) {
  re = p.v[0] * a.re[0] - p.v[1] * a.re[1] - p.v[2] * a.re[2] - p.v[3] * a.re[3];
  im = p.v[0] * a.im[0] - p.v[1] * a.im[1] - p.v[2] * a.im[2] - p.v[3] * a.im[3];
}

template <typename T>
__device__ __forceinline__ T mdot(const R4<T>& a, const R4<T>& b) {
  return a.v[0] * b.v[0] - a.v[1] * b.v[1] - a.v[2] * b.v[2] - a.v[3] * b.v[3];
}

// acc += V3(P, Q; A, B) = (A.B)(P-Q) + ((2Q+P).A) B - ((2P+Q).B) A
template <typename T>
__device__ __forceinline__ void v3_acc(C4<T>& acc, const R4<T>& P, const R4<T>& Q,
                                       const C4<T>& A, const C4<T>& B) {
  T abr, abi;
  cdot(A, B, abr, abi);
  R4<T> q2p, p2q;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    q2p.v[m] = T(2) * Q.v[m] + P.v[m];
    p2q.v[m] = T(2) * P.v[m] + Q.v[m];
  }
  T c1r, c1i, c2r, c2i;
  rdot(q2p, A, c1r, c1i);
  rdot(p2q, B, c2r, c2i);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const T d = P.v[m] - Q.v[m];
    acc.re[m] += abr * d + (c1r * B.re[m] - c1i * B.im[m]) - (c2r * A.re[m] - c2i * A.im[m]);
    acc.im[m] += abi * d + (c1r * B.im[m] + c1i * B.re[m]) - (c2r * A.im[m] + c2i * A.re[m]);
  }
}

// acc += V4(J1, J2, J3) = 2 (J1.J3) J2 - (J2.J3) J1 - (J1.J2) J3
template <typename T>
__device__ __forceinline__ void v4_acc(C4<T>& acc, const C4<T>& J1, const C4<T>& J2,
                                       const C4<T>& J3) {
  T d13r, d13i, d23r, d23i, d12r, d12i;
  cdot(J1, J3, d13r, d13i);
  cdot(J2, J3, d23r, d23i);
  cdot(J1, J2, d12r, d12i);
  d13r *= T(2);
  d13i *= T(2);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    acc.re[m] += (d13r * J2.re[m] - d13i * J2.im[m]) - (d23r * J1.re[m] - d23i * J1.im[m]) -
                 (d12r * J3.re[m] - d12i * J3.im[m]);
    acc.im[m] += (d13r * J2.im[m] + d13i * J2.re[m]) - (d23r * J1.im[m] + d23i * J1.re[m]) -
                 (d12r * J3.im[m] + d12i * J3.re[m]);
  }
}

// First-order dual number for forward-mode derivatives of the polarization.
struct Dual {
  double v, d;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
__device__ __forceinline__ Dual dsqrt_inv(Dual a) {  // 1/sqrt(a)
  const double r = 1.0 / sqrt(a.v);
  return {r, -0.5 * r * r * r * a.d};
}
__device__ __forceinline__ double dval(double x) { return x; }
__device__ __forceinline__ double dval(Dual x) { return x.v; }
__device__ __forceinline__ double dsqrt_inv(double a) { return 1.0 / sqrt(a); }

// External current (eps^h(k))* = (e1 - i h e2)/sqrt2 for the all-outgoing
// momentum p, in the light-cone gauge whose gauge vector q = (|k|, -k) points
// against the gluon (purely spatial, unit polarizations):
//   k = sign(p^0) p,  e1 = (r |k|^2 - (r.k) k) / |r |k|^2 - (r.k) k|,
//   e2 = (k x e1) / |k|,  e1^0 = e2^0 = 0,  r = (3, -6, 2)/7.
// R = double, or Dual for derivatives.
template <typename R>
__device__ __forceinline__ void polarization_t(const R p[4], int h, R er[4], R ei[4]) {
  const double s = dval(p[0]) > 0.0 ? 1.0 : -1.0;
  const R k1 = s * p[1], k2 = s * p[2], k3 = s * p[3];
  const R kk = k1 * k1 + k2 * k2 + k3 * k3;
  const R rk = kR1 * k1 + kR2 * k2 + kR3 * k3;
  const R v1 = kR1 * kk - rk * k1, v2 = kR2 * kk - rk * k2, v3 = kR3 * kk - rk * k3;
  const R inv_nv = dsqrt_inv(v1 * v1 + v2 * v2 + v3 * v3);
  const R e1x = v1 * inv_nv, e1y = v2 * inv_nv, e1z = v3 * inv_nv;
  const R inv_kap = dsqrt_inv(kk);
  const R e2x = (k2 * e1z - k3 * e1y) * inv_kap;
  const R e2y = (k3 * e1x - k1 * e1z) * inv_kap;
  const R e2z = (k1 * e1y - k2 * e1x) * inv_kap;
  const double c = -(h > 0 ? 1.0 : -1.0) * kInvSqrt2;
  er[0] = 0.0 * e1x;
  er[1] = kInvSqrt2 * e1x;
  er[2] = kInvSqrt2 * e1y;
  er[3] = kInvSqrt2 * e1z;
  ei[0] = 0.0 * e2x;
  ei[1] = c * e2x;
  ei[2] = c * e2y;
  ei[3] = c * e2z;
}

__device__ __forceinline__ void polarization(const double p[4], int h, double er[4],
                                             double ei[4]) {
  polarization_t<double>(p, h, er, ei);
}

// d eps_mu / d p^nu: dre[nu][mu], dim[nu][mu]
__device__ __forceinline__ void polarization_jacobian(const double p[4], int h, double dre[4][4],
                                                      double dim[4][4]) {
#pragma unroll
  for (int nu = 0; nu < 4; ++nu) {
    Dual pd[4], er[4], ei[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) pd[m] = Dual{p[m], m == nu ? 1.0 : 0.0};
    polarization_t<Dual>(pd, h, er, ei);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      dre[nu][m] = er[m].d;
      dim[nu][m] = ei[m].d;
    }
  }
}

}  // namespace bg
