// Full-colour colour-ordered |M|^2 at n = 8 (K = 720 orderings) with the
// colour matrix stored as its first row (Section 2.2, eqs.
// color_decomposition_adjoint and color_coefficient_adjoint).
//
// Relabelled storage.  Renaming the summed colour labels of gluons 2..n-1
// maps ordering s to the identity, so C_{s t} = C_{id, pi_s(t)}: pi_s(t) is t
// with every label x replaced by its position in s (1-based), and the row
// index of that permutation is its lexicographic (Lehmer) rank.  The context
// keeps the K entries of row 0 and the K orderings (labels and, for each s,
// the position of every label); a block rebuilds the 64 x 16 tile of C that
// it needs from them in LDS.  Storage O((n-2)!) instead of O((n-2)!^2).
//
// Contraction.  me2_e = x^T C x + y^T C y for x = Re A, y = Im A (C real
// symmetric) with A [2][K][E] from the colour-ordered recursion.  By the
// symmetry of C only the block upper triangle over blocks of 64 rows and
// columns is used: block row rb takes the columns from 64 rb on, the
// diagonal block as it is and the blocks to its right doubled, so that
// x^T C x = sum over rb of x_rb . (C' x)_rb (about half of the products).
// Block (cx, rb): rows 64 rb .. 64 rb + 63 of C' times the 64 columns of X
// formed by 32 events (both planes), on v_mfma_f64_16x16x4f64: wave w owns
// rows 64 rb + 16 w .. + 15 and the four 16-column tiles; k runs over
// chunks of 16 columns of C (each chunk's C' tile is rebuilt in LDS from
// row 0, 1024 entries, four per thread).  Operand layout (wave64): lane l
// supplies A[l%16][l/16] and B[l/16][l%16]; accumulator element r of lane l
// is D[l/16 + 4 r][l%16] (bg_mfma_layout_probe).  The X operands are staged
// through LDS (16 events of one row are 128 contiguous bytes of global
// memory).  The block's share of the quadratic form, sum over its 64 rows
// of X .* (C' X), is written per event to part[rb][e]; a second kernel adds
// the row blocks in a fixed order.  Entries of C(8) and their doubles are
// integers below 2^24 in modulus: exact in FP32.
#include "bg_kernels.h"

namespace bg {
namespace fck {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;  // four waves
constexpr int kRows = 64;      // rows of C per block (16 per wave)
constexpr int kEvents = 32;    // events per block: 64 columns (both planes)
constexpr int kKc = 16;        // columns of C per chunk

// LDS of one block for KM middle gluons (K = KM!).
template <int KM>
struct Shape {
  static constexpr int K = (int)Factorial<KM>::value;
  static constexpr int KC = (K + kKc - 1) / kKc;     // k chunks
  static constexpr int RBK = (K + kRows - 1) / kRows;  // row blocks of 64
};

// C_{s t} from row 0: v_j = position of t's j-th label in s, the entry is
// row0[rank(v)] with the lexicographic (Lehmer) rank accumulated in Horner
// form, rank = ((d_0 (KM-1) + d_1) (KM-2) + d_2) ..., d_j = number of
// positions not yet used that are smaller than v_j.
template <int KM>
__device__ __forceinline__ float entry(int s, int t, const unsigned char* labels,
                                       const unsigned char* pos, const float* row0) {
  int avail = (1 << KM) - 1, r = 0;
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    const int v = pos[s * KM + labels[t * KM + j] - 1];
    r = r * (KM - j) + __popc(avail & ((1 << v) - 1));
    avail &= ~(1 << v);
  }
  return row0[r];
}

// part[rb][e] = sum over rows 64 rb .. 64 rb + 63 of x_s (C' x)_s + y_s (C' y)_s
// for the block's 32 events, C' the block upper triangle of C with the
// off-diagonal blocks doubled (see the file comment).
template <int KM>
__global__ void __launch_bounds__(kThreads) relabel_contract_kernel(
    int64_t E, const double* __restrict__ amp, const float* __restrict__ row0_g,
    const unsigned char* __restrict__ labels_g, const unsigned char* __restrict__ pos_g,
    double* __restrict__ part) {
  using S = Shape<KM>;
  constexpr int K = S::K;
  __shared__ float row0[K];
  __shared__ unsigned char labels[K * KM];
  __shared__ unsigned char pos[K * KM];
  __shared__ float ct[kRows][kKc];          // C' tile of the chunk
  __shared__ double xc[kKc][2 * kEvents];   // X rows of the chunk: [k][plane * 32 + event]
  __shared__ double red[4][2 * kEvents];    // per-wave column sums
  const int tid = threadIdx.x;
  for (int i = tid; i < K; i += kThreads) row0[i] = row0_g[i];
  for (int i = tid; i < K * KM; i += kThreads) {
    labels[i] = labels_g[i];
    pos[i] = pos_g[i];
  }
  const int rb = blockIdx.y;
  const int64_t e0 = (int64_t)blockIdx.x * kEvents;
  const int l = tid & 63, w = tid >> 6;
  const int c16 = l & 15, g = l >> 4;
  d4_t acc[4];
#pragma unroll
  for (int ct4 = 0; ct4 < 4; ++ct4) acc[ct4] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
  for (int kc = rb * (kRows / kKc); kc < S::KC; ++kc) {
    __syncthreads();  // tables loaded; the previous chunk's tiles are consumed
#pragma unroll
    for (int q = 0; q < (kRows * kKc) / kThreads; ++q) {
      const int idx = tid + q * kThreads;
      const int r = idx / kKc, j = idx % kKc;
      const int s = rb * kRows + r, t = kc * kKc + j;
      const float c = (s < K && t < K) ? entry<KM>(s, t, labels, pos, row0) : 0.0f;
      ct[r][j] = t < (rb + 1) * kRows ? c : 2.0f * c;  // t >= 64 rb here
    }
#pragma unroll
    for (int q = 0; q < (kKc * 2 * kEvents) / kThreads; ++q) {
      const int idx = tid + q * kThreads;
      const int k = idx / (2 * kEvents), col = idx % (2 * kEvents);
      const int plane = col / kEvents, ev = col % kEvents;
      const int t = kc * kKc + k;
      const int64_t e = e0 + ev;
      xc[k][col] = (t < K && e < E) ? amp[((int64_t)plane * K + t) * E + e] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kKc / 4; ++ks) {
      const double a = (double)ct[16 * w + c16][4 * ks + g];
#pragma unroll
      for (int ct4 = 0; ct4 < 4; ++ct4) {
        const double b = xc[4 * ks + g][16 * ct4 + c16];
        acc[ct4] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[ct4], 0, 0, 0);
      }
    }
  }
  // accumulator element r of lane l: row 16 w + g + 4 r of the block, column
  // 16 ct4 + c16 (plane ct4 / 2, event 16 (ct4 % 2) + c16)
#pragma unroll
  for (int ct4 = 0; ct4 < 4; ++ct4) {
    const int plane = ct4 >> 1;
    const int64_t e = e0 + 16 * (ct4 & 1) + c16;
    double q = 0.0;
    if (e < E) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int s = rb * kRows + 16 * w + g + 4 * r;
        if (s < K) q += amp[((int64_t)plane * K + s) * E + e] * acc[ct4][r];
      }
    }
    q += __shfl_xor(q, 16);
    q += __shfl_xor(q, 32);
    if (g == 0) red[w][16 * ct4 + c16] = q;
  }
  __syncthreads();
  if (tid < kEvents) {
    const int64_t e = e0 + tid;
    const int cx = 16 * (tid >> 4) + (tid & 15);  // plane 0 column of the event
    double q = 0.0;
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) q += red[ww][cx] + red[ww][kEvents + cx];
    if (e < E) part[(int64_t)rb * E + e] = q;
  }
}

// me2[e] (+)= sum over row blocks of part[rb][e], in row-block order.
__global__ void __launch_bounds__(256) relabel_reduce_kernel(int64_t E, int rbk,
                                                             const double* __restrict__ part,
                                                             double* __restrict__ me2,
                                                             int accumulate) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= E) return;
  double q = 0.0;
  for (int rb = 0; rb < rbk; ++rb) q += part[(int64_t)rb * E + e];
  me2[e] = accumulate ? me2[e] + q : q;
}

}  // namespace fck

int relabel_row_blocks(int n) { return n == 8 ? fck::Shape<6>::RBK : 0; }

int relabel_contract(int n, int64_t E, const double* amp, const float* row0,
                     const unsigned char* labels, const unsigned char* pos, double* part,
                     double* me2, int accumulate, hipStream_t stream) {
  if (E <= 0) return 0;
  if (n != 8) return -2;
  using S = fck::Shape<6>;
  const dim3 grid((unsigned)((E + fck::kEvents - 1) / fck::kEvents), (unsigned)S::RBK);
  hipLaunchKernelGGL(fck::relabel_contract_kernel<6>, grid, dim3(fck::kThreads), 0, stream, E, amp,
                     row0, labels, pos, part);
  hipLaunchKernelGGL(fck::relabel_reduce_kernel, dim3((unsigned)((E + 255) / 256)), dim3(256), 0,
                     stream, E, S::RBK, part, me2, accumulate);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace bg
