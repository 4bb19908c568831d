// Lane-pair building blocks: an event's Lorentz components are split over
// two adjacent lanes (lane half h = lane & 1 owns components 2h, 2h+1).  A
// Minkowski product is the sum of the halves' partials, exchanged with one
// DPP quad_perm [1,0,3,2] move; the metric sign of the lane's first component
// is g0 = +1 (h = 0) or -1 (h = 1), the second is always -1.  The sum a + b is
// formed in both lanes in opposite operand order, which IEEE addition makes
// bit-identical.
#pragma once

#include <hip/hip_runtime.h>

namespace bg {
namespace pairk {

template <typename T>
struct H {  // the lane's half of a complex four-vector
  T re[2], im[2];
};

template <typename T>
struct HR {  // the lane's half of a real four-vector
  T v[2];
};

template <typename T>
struct Cx {
  T re, im;
};

// quad_perm [1,0,3,2] reads a lane of the same quad, so no lane is out of
// bounds and the value written for out-of-bounds lanes (bound_ctrl) never
// matters; with an undefined old value the compiler can fold the move into
// the consuming add (v_add_f32_dpp).
__device__ __forceinline__ float xswap(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, true));
}

__device__ __forceinline__ double xswap(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0xB1, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0xB1, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// full complex Minkowski product of two currents from the lane halves
template <typename T>
__device__ __forceinline__ Cx<T> hdot(const H<T>& a, const H<T>& b, T g0) {
  const T r0 = a.re[0] * b.re[0] - a.im[0] * b.im[0];
  const T i0 = a.re[0] * b.im[0] + a.im[0] * b.re[0];
  const T r1 = a.re[1] * b.re[1] - a.im[1] * b.im[1];
  const T i1 = a.re[1] * b.im[1] + a.im[1] * b.re[1];
  const T pr = g0 * r0 - r1;
  const T pi = g0 * i0 - i1;
  return Cx<T>{pr + xswap(pr), pi + xswap(pi)};
}

// hdot(a, b, g0) with the lane's first component of b pre-multiplied by its
// metric sign: bg = g0 (b.re[0], b.im[0]); one multiply-add per real product
template <typename T>
__device__ __forceinline__ Cx<T> hdot_g(const H<T>& a, const H<T>& b, const Cx<T>& bg) {
  T pr = a.im[1] * b.im[1];
  pr -= a.re[1] * b.re[1];
  pr -= a.im[0] * bg.im;
  pr += a.re[0] * bg.re;
  T pi = a.re[0] * bg.im;
  pi += a.im[0] * bg.re;
  pi -= a.re[1] * b.im[1];
  pi -= a.im[1] * b.re[1];
  return Cx<T>{pr + xswap(pr), pi + xswap(pi)};
}

// full product p.J of a real and a complex four-vector
template <typename T>
__device__ __forceinline__ Cx<T> hrdot(const HR<T>& p, const H<T>& a, T g0) {
  const T pr = g0 * p.v[0] * a.re[0] - p.v[1] * a.re[1];
  const T pi = g0 * p.v[0] * a.im[0] - p.v[1] * a.im[1];
  return Cx<T>{pr + xswap(pr), pi + xswap(pi)};
}

// acc += s v with one multiply-add per real product
template <typename T>
__device__ __forceinline__ void caxpy(H<T>& acc, const Cx<T>& s, const H<T>& v) {
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    acc.re[m] += s.re * v.re[m];
    acc.re[m] -= s.im * v.im[m];
    acc.im[m] += s.re * v.im[m];
    acc.im[m] += s.im * v.re[m];
  }
}

template <typename T>
__device__ __forceinline__ void craxpy(H<T>& acc, const Cx<T>& s, const HR<T>& v) {
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    acc.re[m] += s.re * v.v[m];
    acc.im[m] += s.im * v.v[m];
  }
}


// full sum over the pair of a per-lane partial (no metric)
template <typename T>
__device__ __forceinline__ T pair_sum(T x) {
  return x + xswap(x);
}

}  // namespace pairk
}  // namespace bg
