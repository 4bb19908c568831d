// Colour contraction |M|^2 = sum_{s,t} C_st Re(A_s conj(A_t))
// (Section 2.2, eq. color_summed_analytic) in FP64.
//
// C is real and symmetric, so with x = Re A and y = Im A the contraction is
// x^T C x + y^T C y.  For a tile of 64 events the 2x64 vectors form the
// columns of X (K x 128); Z = C X is a dense FP64 product done on the matrix
// cores with v_mfma_f64_16x16x4f64, and me2_e = sum_s X_se Z_se + X_s,e+64 Z_s,e+64.
// K is padded to KP (a multiple of 16) with zero rows/columns of C.
//
// Operand layout of v_mfma_f64_16x16x4f64 (wave64, one block): lane l supplies
// A[l%16][l/16] and B[l/16][l%16].  The accumulator layout is not assumed:
// the same instruction multiplies X by an identity tile, which places X in
// exactly the accumulator layout of Z, so the elementwise products X*Z line up
// whatever the row order.  Only the column of an accumulator element is used
// (lanes with equal l%16 share a column), and bg_mfma_selftest checks it.
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

template <int KP>
__global__ void __launch_bounds__(64) contract_mfma_kernel(int K, int64_t E,
                                                          const double* __restrict__ amp,
                                                          const double* __restrict__ Cp,
                                                          double* __restrict__ me2,
                                                          int accumulate) {
  // X tile in LDS: [KP][128] (columns 0..63 real parts, 64..127 imaginary parts)
  __shared__ double X[KP][128];
  const int l = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * 64;
  const int64_t e = e0 + l;
  const bool live = e < E;
  for (int s = 0; s < KP; ++s) {
    double xr = 0.0, xi = 0.0;
    if (s < K && live) {
      xr = amp[(int64_t)s * E + e];
      xi = amp[((int64_t)K + s) * E + e];
    }
    X[s][l] = xr;
    X[s][64 + l] = xi;
  }
  __syncthreads();

  const int li = l & 15;  // row of A / column of B and D
  const int lk = l >> 4;  // k of A and B
  double part[4] = {0.0, 0.0, 0.0, 0.0};  // per column group (events li + 16 g)
#pragma unroll 1
  for (int rt = 0; rt < KP / 16; ++rt) {
    d4_t acc[8], xd[8];
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) {
      acc[ct] = d4_t{0.0, 0.0, 0.0, 0.0};
      xd[ct] = d4_t{0.0, 0.0, 0.0, 0.0};
    }
#pragma unroll 4
    for (int ks = 0; ks < KP / 4; ++ks) {
      const double a = Cp[(rt * 16 + li) * KP + ks * 4 + lk];
#pragma unroll
      for (int ct = 0; ct < 8; ++ct) {
        const double b = X[ks * 4 + lk][ct * 16 + li];
        acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[ct], 0, 0, 0);
      }
    }
    // X rows rt*16..rt*16+15 in accumulator layout: I(16x16) x X_tile
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const double a = (li == ks * 4 + lk) ? 1.0 : 0.0;
#pragma unroll
      for (int ct = 0; ct < 8; ++ct) {
        const double b = X[rt * 16 + ks * 4 + lk][ct * 16 + li];
        xd[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, xd[ct], 0, 0, 0);
      }
    }
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) {
#pragma unroll
      for (int r = 0; r < 4; ++r) part[ct & 3] += xd[ct][r] * acc[ct][r];
    }
  }
  // reduce over the four row groups (lanes li, li+16, li+32, li+48)
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    part[g] += __shfl_xor(part[g], 16);
    part[g] += __shfl_xor(part[g], 32);
  }
  // lane l writes event l: its column group is l/16 (== lk), column li
  const double v = part[lk];
  if (live) me2[e] = accumulate ? me2[e] + v : v;
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

int contract_y(int K, int64_t E, const double* amp, const double* C, double* Y, double* me2,
               hipStream_t stream) {
  if (E <= 0) return 0;
  hipLaunchKernelGGL(contract_y_kernel, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, stream, K,
                     E, amp, C, Y, me2);
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

int contract_mfma(int K, int64_t E, const double* amp, const double* C_pad, int KP, double* me2,
                  int accumulate, hipStream_t stream) {
  if (E <= 0) return 0;
  const unsigned grid = (unsigned)((E + 63) / 64);
  switch (KP) {
    case 32:
      hipLaunchKernelGGL(contract_mfma_kernel<32>, dim3(grid), dim3(64), 0, stream, K, E, amp,
                         C_pad, me2, accumulate);
      break;
    default:
      return -2;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace bg
