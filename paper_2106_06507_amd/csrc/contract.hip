// Colour contraction |M|^2 = sum_{s,t} C_st Re(A_s conj(A_t))
// (Section 2.2, eq. color_summed_analytic) in FP64.
//
// C is real and symmetric, so with x = Re A and y = Im A the contraction is
// x^T C x + y^T C y.  Matrix-core path (K = 24, 120): a wave takes 16
// consecutive events, the columns of X (one plane at a time), and forms
// Z = C' X on v_mfma_f64_16x16x4f64.  C' is C in block-triangular form over
// blocks of 16 rows and columns: the diagonal blocks as they are, the blocks
// right of the diagonal doubled, those left of it dropped, so that
// x^T C x = sum over row blocks b of x_b . (C' x)_b by the symmetry of C;
// row block b runs over the k range from 16 b to K only (K = 24: 6 + 2 k
// steps of 4 instead of 2 x 6; K = 120: 128 instead of 240).  Operand layout
// (wave64): lane l supplies A[l%16][l/16] and B[l/16][l%16]; accumulator
// element r of lane l is D[l/16 + 4 r][l%16] (bg_mfma_layout_probe; the
// tests assert rows and columns).  The X operands of all K/4 k steps are
// loaded once from global memory into registers (16 events of one row are
// 128 contiguous bytes); the k dimension needs no padding.  Lane l holds
// X rows 4 ks + l/16, which are also the rows of its accumulator elements in
// row block b (ks = 4 b + r), so x . Z needs no second read.  C' sits in LDS
// as FP32 (entries are integers below 2^24 in modulus, also when doubled:
// exact), rows padded with zeros to a multiple of 16 and the row stride odd
// (K + 1) against bank conflicts.  The four lane groups of a column are
// added with two cross-lane exchanges.  Listed form (idx non-null): column e
// of the amplitude array belongs to event idx[first + e], written only for
// first + e < *cnt.
#include "bg_kernels.h"

namespace bg {

typedef double d4_t __attribute__((ext_vector_type(4)));

// One thread per event; C read through the scalar cache (uniform addresses).
__global__ void __launch_bounds__(256) contract_valu_kernel(int K, int64_t E,
                                                           const double* __restrict__ amp,
                                                           const double* __restrict__ C,
                                                           double* __restrict__ me2,
                                                           int accumulate) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  double acc = 0.0;
  for (int s = 0; s < K; ++s) {
    const double xs = amp[(int64_t)s * E + e];
    const double ys = amp[((int64_t)K + s) * E + e];
    double zx = 0.0, zy = 0.0;
    for (int t = 0; t < K; ++t) {
      const double c = C[s * K + t];
      zx += c * amp[(int64_t)t * E + e];
      zy += c * amp[((int64_t)K + t) * E + e];
    }
    acc += xs * zx + ys * zy;
  }
  me2[e] = accumulate ? me2[e] + acc : acc;
}

template <int K>
struct MfmaShape {
  static constexpr int KS = K / 4;          // k steps of 4
  static constexpr int RB = (K + 15) / 16;  // row blocks of 16
  static constexpr int RP = RB * 16;
  static constexpr int KL = K + 1;          // LDS row stride (odd)
  static constexpr size_t lds = sizeof(float) * (size_t)RP * KL;
  static constexpr int kBlock = K <= 32 ? 256 : 768;  // threads per block (K = 120: 3 waves/SIMD)
};

template <int K>
__global__ void __launch_bounds__(MfmaShape<K>::kBlock) contract_mfma_kernel(
    int64_t E, const double* __restrict__ amp, const double* __restrict__ C,
    double* __restrict__ me2, int accumulate, const unsigned* __restrict__ idx,
    const unsigned* __restrict__ cnt, int64_t first) {
  using S = MfmaShape<K>;
  static_assert(K % 4 == 0, "k steps of four");
  extern __shared__ float bg_contract_c[];  // C' [RP][KL], rows >= K zero
  for (int i = threadIdx.x; i < S::RP * K; i += S::kBlock) {
    const int r = i / K, t = i % K;
    const int br = r >> 4, bt = t >> 4;
    const float c = r < K ? (float)C[r * K + t] : 0.0f;
    bg_contract_c[r * S::KL + t] = bt == br ? c : (bt > br ? 2.0f * c : 0.0f);
  }
  __syncthreads();
  const int l = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int c16 = l & 15, g = l >> 4;
  const int64_t e = ((int64_t)blockIdx.x * (S::kBlock / 64) + w) * 16 + c16;
  const bool live = e < E;
  const int64_t ee = live ? e : E - 1;  // lanes past the end read a valid event, store nothing
  double bx[S::KS], by[S::KS];
#pragma unroll
  for (int ks = 0; ks < S::KS; ++ks) {
    bx[ks] = amp[(int64_t)(4 * ks + g) * E + ee];
    by[ks] = amp[(int64_t)(K + 4 * ks + g) * E + ee];
  }
  double q = 0.0;
#pragma unroll
  for (int rb = 0; rb < S::RB; ++rb) {
    d4_t ax = d4_t{0.0, 0.0, 0.0, 0.0}, ay = d4_t{0.0, 0.0, 0.0, 0.0};
    const float* crow = bg_contract_c + (16 * rb + c16) * S::KL + g;
#pragma unroll
    for (int ks = 4 * rb; ks < S::KS; ++ks) {
      const double a = (double)crow[4 * ks];
      ax = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bx[ks], ax, 0, 0, 0);
      ay = __builtin_amdgcn_mfma_f64_16x16x4f64(a, by[ks], ay, 0, 0, 0);
    }
    // element r: row 16 rb + g + 4 r = 4 (4 rb + r) + g, held in bx/by[4 rb + r]
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (4 * rb + r < S::KS) q += bx[4 * rb + r] * ax[r] + by[4 * rb + r] * ay[r];
    }
  }
  q += __shfl_xor(q, 16);
  q += __shfl_xor(q, 32);
  if (g == 0 && live) {
    if (idx) {
      if (first + e < (int64_t)*cnt) {
        const int64_t o = idx[first + e];
        me2[o] = accumulate ? me2[o] + q : q;
      }
    } else {
      me2[e] = accumulate ? me2[e] + q : q;
    }
  }
}

// Layout self-test: D = A x B with A[i][k] = i + 1 + 100 k and B[k][j] =
// (j + 1) * 1000^(k+1) mod-free encodings; every accumulator element is
// written with its lane and register so the host can check the column mapping.
__global__ void mfma_probe_kernel(double* out) {
  const int l = threadIdx.x;
  const double a = (double)((l & 15) + 1) + 100.0 * (double)(l >> 4);
  const double b = (double)((l & 15) + 1) * (double)(1 << (3 * (l >> 4)));
  d4_t d = d4_t{0.0, 0.0, 0.0, 0.0};
  d = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, d, 0, 0, 0);
#pragma unroll
  for (int r = 0; r < 4; ++r) out[l * 4 + r] = d[r];
}

int mfma_probe(double* out_dev, hipStream_t stream) {
  hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, stream, out_dev);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Y = C A per event (both planes) and me2 = x.Cx + y.Cy, for the gradient.
__global__ void __launch_bounds__(256) contract_y_kernel(int K, int64_t E,
                                                        const double* __restrict__ amp,
                                                        const double* __restrict__ C,
                                                        double* __restrict__ Y,
                                                        double* __restrict__ me2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  double acc = 0.0;
  for (int s = 0; s < K; ++s) {
    double zx = 0.0, zy = 0.0;
    for (int t = 0; t < K; ++t) {
      const double c = C[s * K + t];
      zx += c * amp[(int64_t)t * E + e];
      zy += c * amp[((int64_t)K + t) * E + e];
    }
    Y[(int64_t)s * E + e] = zx;
    Y[((int64_t)K + s) * E + e] = zy;
    acc += amp[(int64_t)s * E + e] * zx + amp[((int64_t)K + s) * E + e] * zy;
  }
  if (me2) me2[e] = acc;
}

// The same for K <= 24 with the event's 2K amplitudes held in registers:
// each is read from HBM once (the loop above re-reads every amplitude K
// times, and the blocks' working sets overflow L2), and the sums run in the
// same order, so the results are identical.
template <int K>
__global__ void __launch_bounds__(256) contract_y_reg_kernel(int64_t E,
                                                             const double* __restrict__ amp,
                                                             const double* __restrict__ C,
                                                             double* __restrict__ Y,
                                                             double* __restrict__ me2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  double x[K], y[K];
#pragma unroll
  for (int t = 0; t < K; ++t) {
    x[t] = amp[(int64_t)t * E + e];
    y[t] = amp[((int64_t)K + t) * E + e];
  }
  double acc = 0.0;
#pragma unroll
  for (int s = 0; s < K; ++s) {
    double zx = 0.0, zy = 0.0;
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const double c = C[s * K + t];
      zx += c * x[t];
      zy += c * y[t];
    }
    Y[(int64_t)s * E + e] = zx;
    Y[((int64_t)K + s) * E + e] = zy;
    acc += x[s] * zx + y[s] * zy;
  }
  if (me2) me2[e] = acc;
}

int contract_y(int K, int64_t E, const double* amp, const double* C, double* Y, double* me2,
               hipStream_t stream) {
  if (E <= 0) return 0;
  const dim3 grid((unsigned)((E + 255) / 256));
  switch (K) {
    case 2: hipLaunchKernelGGL(contract_y_reg_kernel<2>, grid, dim3(256), 0, stream, E, amp, C, Y, me2); break;
    case 6: hipLaunchKernelGGL(contract_y_reg_kernel<6>, grid, dim3(256), 0, stream, E, amp, C, Y, me2); break;
    case 24: hipLaunchKernelGGL(contract_y_reg_kernel<24>, grid, dim3(256), 0, stream, E, amp, C, Y, me2); break;
    default:
      hipLaunchKernelGGL(contract_y_kernel, grid, dim3(256), 0, stream, K, E, amp, C, Y, me2);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int contract_valu(int K, int64_t E, const double* amp, const double* C, double* me2,
                  int accumulate, hipStream_t stream) {
  if (E <= 0) return 0;
  const int blk = 256;
  hipLaunchKernelGGL(contract_valu_kernel, dim3((unsigned)((E + blk - 1) / blk)), dim3(blk), 0,
                     stream, K, E, amp, C, me2, accumulate);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int contract_mfma(int K, int64_t E, const double* amp, const double* C, double* me2,
                  int accumulate, hipStream_t stream, const unsigned* idx, const unsigned* cnt,
                  int64_t first) {
  if (E <= 0) return 0;
  switch (K) {
#define BG_CASE(KK)                                                                           \
  case KK: {                                                                                  \
    using S = MfmaShape<KK>;                                                                  \
    const int64_t per_block = (S::kBlock / 64) * 16;                                          \
    const unsigned grid = (unsigned)((E + per_block - 1) / per_block);                        \
    hipLaunchKernelGGL(contract_mfma_kernel<KK>, dim3(grid), dim3(S::kBlock), S::lds, stream, \
                       E, amp, C, me2, accumulate, idx, cnt, first);                          \
    break;                                                                                    \
  }
    BG_CASE(24)
    BG_CASE(120)
#undef BG_CASE
    default:
      return -2;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace bg
