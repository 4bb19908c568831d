// Continuous colour and polarization sampling with the colour-dressed
// recursion (Section 2.1, eqs. polarization_simple and
// gluon_color_polarization; Section 2.3, eq. color_dressed_currents): every
// number is real.
//
// Gluon k enters with the real polarization e_k = sqrt2 (cos phi_k e1 +
// sin phi_k e2) (the phi-average of e e^T is the helicity sum of the
// external currents (e1 -+ i e2)/sqrt2) and the colour matrix
// etabar_k eta_k^T (the trace-basis contraction of eta T^a etabar; its
// unit-matrix part decouples).  The dressed current of a subset S is a real
// 3x3 colour matrix of four-vectors J(S)[i][j][mu] together with the
// antisymmetric tensor current T(S)[i][j][mu nu] (six components).  With
// J1, T1 = J(A), T(A) and J2, T2 = J(B), T(B) for an ordered split (A, B) of
// S, and k summed (colour-matrix products), the entry (i, j) is
//   J(S)^nu = 1/P_S^2 sum over splits of
//       (J1_ik . J2_kj)(P_A - P_B)^nu + ((2 P_B + P_A) . J1_ik) J2_kj^nu
//     - ((2 P_A + P_B) . J2_kj) J1_ik^nu
//     + sum_b g_bb J1_ik^b T2_kj^{nu b} + sum_a g_aa T1_ik^{a nu} J2_kj^a
//   T(S)^{ab} = sum over splits of J1_ik^a J2_kj^b - J1_ik^b J2_kj^a.
// The factors i of the vertices cancel the -i of the propagators and the
// tensor's -i; the couplings g_s/sqrt2 are taken out (each current of |S|
// gluons carries (g_s/sqrt2)^(|S|-1)) and applied to the amplitude
//   A = (g_s/sqrt2)^(n-2) eta_n^T (e_n . J(1..n-1)) etabar_n
// (J of the full set amputated).  The kernel returns A^2; 9^n times its
// average over uniform phi and sphere vectors is the colour- and
// helicity-summed |M|^2.
//
// Layout: one event per block of NW waves; within a wave, groups of nine
// lanes hold the nine colour entries (i, j) (lane 63 idles).  Subsets are
// processed by size; the targets of one size are spread over the groups,
// with q groups per target taking contiguous ranges of its ordered splits
// when targets are fewer than groups, and the q partial sums added in a
// fixed order.  The
// subset state (J, T, P as T, 1/P^2 from FP64 momenta) lives in LDS, or for
// FP64 at n = 9 in a global slab per block (it exceeds the LDS).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bg_device.h"

namespace bg {
namespace cdmck {

constexpr int kWave = 64;
constexpr int kGroup = 9;                      // colour entries per group
constexpr int kGroupsPerWave = kWave / kGroup;  // 7

template <int N>
struct Waves {
  static constexpr int value = N <= 5 ? 1 : (N == 6 ? 2 : (N == 7 ? 4 : 8));
};

// state of one event, in elements of T
template <int N>
struct State {
  static constexpr int M = N - 1;
  static constexpr int NS = 1 << M;
  static constexpr size_t oJ = 0;                       // J[S][i][j][mu]
  static constexpr size_t oT = oJ + (size_t)NS * 36;    // T[S][i][j][pair]
  static constexpr size_t oP = oT + (size_t)NS * 54;    // P[S][mu]
  static constexpr size_t oIp = oP + (size_t)NS * 4;    // 1/P^2 [S]
  static constexpr size_t size = oIp + NS;
};

template <int N, typename T, bool GS>
struct Lds {
  static constexpr int NW = Waves<N>::value;
  static constexpr int G = NW * kGroupsPerWave;
  static constexpr size_t state_bytes = GS ? 0 : sizeof(T) * State<N>::size;
  static constexpr size_t part_bytes = sizeof(T) * (size_t)G * kGroup * 10;
  static constexpr size_t red_bytes = sizeof(double) * (size_t)NW * kWave;
  static constexpr size_t ext_bytes = sizeof(double) * 16;   // e_n[4], eta_n[3], etabar_n[3]
  static constexpr size_t sub_bytes = sizeof(int) * ((1 << (N - 1)) + N + 2);
  static constexpr size_t bytes() {
    return state_bytes + part_bytes + red_bytes + ext_bytes + sub_bytes;
  }
};

__device__ __forceinline__ int binom(int m, int k) {
  int r = 1;
  for (int t = 1; t <= k; ++t) r = r * (m - k + t) / t;
  return r;
}

// the x-th (1-based) sub-mask of S in increasing order of its bit pattern
__device__ __forceinline__ int submask(int S, int x) {
  int out = 0;
  for (int s = S; s != 0; s &= s - 1) {
    const int low = s & -s;
    if (x & 1) out |= low;
    x >>= 1;
  }
  return out;
}

// pair index of (a, b), a < b, in (01, 02, 03, 12, 13, 23)
__device__ __forceinline__ constexpr int pidx(int a, int b) {
  return a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
}

// out[nu] += sgn sum_b g_bb J^b T^{nu b} for the antisymmetric T given by
// t[6] (pairs 01, 02, 03, 12, 13, 23); one multiply-add per term
template <typename T>
__device__ __forceinline__ void jt_accumulate(const T J[4], const T t[6], T sgn, T out[4]) {
  const T j0 = sgn * J[0], j1 = sgn * J[1], j2 = sgn * J[2], j3 = sgn * J[3];
  out[0] -= j1 * t[0];
  out[0] -= j2 * t[1];
  out[0] -= j3 * t[2];
  out[1] -= j0 * t[0];
  out[1] -= j2 * t[3];
  out[1] -= j3 * t[4];
  out[2] -= j0 * t[1];
  out[2] += j1 * t[3];
  out[2] -= j3 * t[5];
  out[3] -= j0 * t[2];
  out[3] += j1 * t[4];
  out[3] += j2 * t[5];
}

// Accumulate the contribution of the ordered split (A, B) to entry (i, j).
// Every product is accumulated with its own multiply-add.
template <int N, typename T>
__device__ __forceinline__ void split_term(const T* __restrict__ st, int A, int B, int i, int j,
                                           bool want_t, T outJ[4], T outT[6]) {
  using L = State<N>;
  T a[3][4], b[3][4], P1[4], P2[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    P1[m] = st[L::oP + 4 * A + m];
    P2[m] = st[L::oP + 4 * B + m];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      a[k][m] = st[L::oJ + 36 * A + 12 * i + 4 * k + m];
      b[k][m] = st[L::oJ + 36 * B + 12 * k + 4 * j + m];
    }
  }
  // metric folded into the momenta: qg = g (2 P_B + P_A), pg = g (2 P_A + P_B)
  T qg[4], pg[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const T sg = m == 0 ? T(1) : T(-1);
    qg[m] = sg * (T(2) * P2[m] + P1[m]);
    pg[m] = sg * (T(2) * P1[m] + P2[m]);
  }
  T ab = T(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    ab += a[k][0] * b[k][0];
    ab -= a[k][1] * b[k][1];
    ab -= a[k][2] * b[k][2];
    ab -= a[k][3] * b[k][3];
    T qa = qg[0] * a[k][0];
    T pb = pg[0] * b[k][0];
#pragma unroll
    for (int m = 1; m < 4; ++m) {
      qa += qg[m] * a[k][m];
      pb += pg[m] * b[k][m];
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      outJ[m] += qa * b[k][m];
      outJ[m] -= pb * a[k][m];
    }
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) outJ[m] += ab * (P1[m] - P2[m]);
  if (__popc(B) >= 2) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T t[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) t[c] = st[L::oT + 54 * B + 18 * k + 6 * j + c];
      jt_accumulate(a[k], t, T(1), outJ);
    }
  }
  if (__popc(A) >= 2) {
    // sum_a g_aa T1^{a nu} J2^a = -sum_a g_aa T1^{nu a} J2^a
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T t[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) t[c] = st[L::oT + 54 * A + 18 * i + 6 * k + c];
      jt_accumulate(b[k], t, T(-1), outJ);
    }
  }
  if (want_t) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
      for (int x = 0; x < 4; ++x) {
#pragma unroll
        for (int y = x + 1; y < 4; ++y) {
          outT[pidx(x, y)] += a[k][x] * b[k][y];
          outT[pidx(x, y)] -= a[k][y] * b[k][x];
        }
      }
    }
  }
}

// One event per block; persistent over events.
template <int N, typename T, bool GS>
__global__ void __launch_bounds__(Waves<N>::value * kWave)
cdmc_kernel(int64_t E, const double* __restrict__ mom, const double* __restrict__ phi,
            const double* __restrict__ eta, T* __restrict__ gstate, double* __restrict__ me2) {
  using L = State<N>;
  using Y = Lds<N, T, GS>;
  constexpr int M = L::M, NS = L::NS, NW = Y::NW, G = Y::G;
  constexpr int NT = NW * kWave;
  extern __shared__ __align__(16) unsigned char bg_cdmc_lds[];
  unsigned char* lp = bg_cdmc_lds;
  T* st = GS ? gstate + (size_t)blockIdx.x * L::size : reinterpret_cast<T*>(lp);
  lp += Y::state_bytes;
  T* part = reinterpret_cast<T*>(lp);
  lp += Y::part_bytes;
  double* red = reinterpret_cast<double*>(lp);
  lp += Y::red_bytes;
  double* ext = reinterpret_cast<double*>(lp);
  lp += Y::ext_bytes;
  int* sub = reinterpret_cast<int*>(lp);  // subsets ordered by size, then value
  int* off = sub + NS;                    // off[s] = first index of size s

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  const int grp = lane / kGroup;
  const bool active = grp < kGroupsPerWave;
  const int gid = wave * kGroupsPerWave + grp;  // < G when active
  const int e9 = lane - grp * kGroup;
  const int ci = e9 / 3, cj = e9 - 3 * (e9 / 3);

  for (int s = tid; s < NS; s += NT) {
    const int pc = __popc(s);
    int r = 0;
    for (int u = 0; u < s; ++u) r += __popc(u) == pc;
    int o = 0;
    for (int z = 0; z < pc; ++z) o += binom(M, z);
    sub[o + r] = s;
  }
  if (tid <= M + 1) {
    int o = 0;
    for (int z = 0; z < tid; ++z) o += binom(M, z);
    off[tid] = o;
  }
  __syncthreads();

  double coup = 1.0;
#pragma unroll
  for (int z = 0; z < N - 2; ++z) coup *= kGsOverSqrt2;

  for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
    // external currents of gluons 1..n-1, and e_n, eta_n, etabar_n
    for (int k = tid; k < N; k += NT) {
      double p[4], er[4], ei[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) p[m] = mom[((int64_t)k * 4 + m) * E + e];
      polarization(p, 1, er, ei);
      const double f = phi[(int64_t)k * E + e];
      const double c = cos(f), sn = sin(f);
      double ev[4], h[3], hb[3];
#pragma unroll
      for (int m = 0; m < 4; ++m) ev[m] = 2.0 * (c * er[m] - sn * ei[m]);
#pragma unroll
      for (int x = 0; x < 3; ++x) {
        h[x] = eta[((int64_t)k * 3 + x) * E + e];
        hb[x] = eta[((int64_t)(N + k) * 3 + x) * E + e];
      }
      if (k < M) {
        const int S = 1 << k;
#pragma unroll
        for (int x = 0; x < 3; ++x) {
#pragma unroll
          for (int y = 0; y < 3; ++y) {
#pragma unroll
            for (int m = 0; m < 4; ++m) st[L::oJ + 36 * S + 12 * x + 4 * y + m] = (T)(hb[x] * h[y] * ev[m]);
          }
        }
#pragma unroll
        for (int c2 = 0; c2 < 54; ++c2) st[L::oT + 54 * S + c2] = T(0);
      } else {
#pragma unroll
        for (int m = 0; m < 4; ++m) ext[m] = ev[m];
#pragma unroll
        for (int x = 0; x < 3; ++x) {
          ext[4 + x] = h[x];
          ext[7 + x] = hb[x];
        }
      }
    }
    // subset momenta (FP64 sums) and 1/P^2
    for (int S = tid + 1; S < NS; S += NT) {
      double P[4] = {0.0, 0.0, 0.0, 0.0};
      for (int k = 0; k < M; ++k) {
        if ((S >> k) & 1) {
#pragma unroll
          for (int m = 0; m < 4; ++m) P[m] += mom[((int64_t)k * 4 + m) * E + e];
        }
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) st[L::oP + 4 * S + m] = (T)P[m];
      const double p2 = P[0] * P[0] - P[1] * P[1] - P[2] * P[2] - P[3] * P[3];
      st[L::oIp + S] = __popc(S) >= 2 && S != NS - 1 ? (T)(1.0 / p2) : T(0);
    }
    __syncthreads();

    double amp_part = 0.0;
    for (int sz = 2; sz <= M; ++sz) {
      const int nt = off[sz + 1] - off[sz];
      const int nsplit = (1 << sz) - 2;
      int q = G / nt;
      q = q < 1 ? 1 : (q > nsplit ? nsplit : q);
      const bool top = sz == M;
      for (int task = gid; task < nt * q; task += G) {
        const int r = task / q, slice = task - r * q;
        const int S = sub[off[sz] + r];
        T outJ[4] = {T(0), T(0), T(0), T(0)};
        T outT[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
        if (active) {
          // a contiguous range of splits per slice; the next sub-mask of S
          // in increasing order is (A - S) & S
          const int per = (nsplit + q - 1) / q;
          const int x0 = 1 + slice * per;
          const int x1 = x0 + per - 1 < nsplit ? x0 + per - 1 : nsplit;
          int A = x0 <= x1 ? submask(S, x0) : 0;
          for (int x = x0; x <= x1; ++x) {
            split_term<N, T>(st, A, S ^ A, ci, cj, !top, outJ, outT);
            A = (A - S) & S;
          }
        }
        if (top) {
          if (active) {
            const double v = (double)outJ[0] * ext[0] - (double)outJ[1] * ext[1] -
                             (double)outJ[2] * ext[2] - (double)outJ[3] * ext[3];
            amp_part += v * ext[4 + ci] * ext[7 + cj];
          }
        } else if (q == 1) {
          if (active) {
            const T ip = st[L::oIp + S];
#pragma unroll
            for (int m = 0; m < 4; ++m) st[L::oJ + 36 * S + 4 * e9 + m] = outJ[m] * ip;
#pragma unroll
            for (int c2 = 0; c2 < 6; ++c2) st[L::oT + 54 * S + 6 * e9 + c2] = outT[c2];
          }
        } else if (active) {
          T* pp = part + ((size_t)task * kGroup + e9) * 10;
#pragma unroll
          for (int m = 0; m < 4; ++m) pp[m] = outJ[m];
#pragma unroll
          for (int c2 = 0; c2 < 6; ++c2) pp[4 + c2] = outT[c2];
        }
      }
      if (!top && q > 1) {
        __syncthreads();
        for (int w = tid; w < nt * kGroup * 10; w += NT) {
          const int r = w / (kGroup * 10);
          const int rest = w - r * kGroup * 10;
          const int x9 = rest / 10, comp = rest - 10 * x9;
          const int S = sub[off[sz] + r];
          T acc = T(0);
          for (int sl = 0; sl < q; ++sl) acc += part[((size_t)(r * q + sl) * kGroup + x9) * 10 + comp];
          if (comp < 4) {
            st[L::oJ + 36 * S + 4 * x9 + comp] = acc * st[L::oIp + S];
          } else {
            st[L::oT + 54 * S + 6 * x9 + comp - 4] = acc;
          }
        }
      }
      __syncthreads();
    }
    // block sum of the top-level entries (fixed order)
    red[tid] = amp_part;
    __syncthreads();
    if (tid == 0) {
      double a = 0.0;
      for (int t = 0; t < NT; ++t) a += red[t];
      a *= coup;
      me2[e] = a * a;
    }
    __syncthreads();
  }
}

template <int N, typename T, bool GS>
int launch(int64_t E, const double* mom, const double* phi, const double* eta, void* gstate,
           int grid, double* me2, hipStream_t stream) {
  using Y = Lds<N, T, GS>;
  hipLaunchKernelGGL((cdmc_kernel<N, T, GS>), dim3(grid), dim3(Y::NW * kWave), (Y::bytes()), stream,
                     E, mom, phi, eta, reinterpret_cast<T*>(gstate), me2);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N, typename T, bool GS>
int occupancy() {
  using Y = Lds<N, T, GS>;
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, cdmc_kernel<N, T, GS>, Y::NW * kWave,
                                                   Y::bytes()) != hipSuccess)
    return 0;
  return b;
}

// FP64 state at n = 9 does not fit the LDS
template <int N, typename T>
struct Global {
  static constexpr bool value = sizeof(T) * State<N>::size + 48 * 1024 > 160 * 1024;
};

}  // namespace cdmck

#define BG_CDMC_SWITCH(CALL) \
  switch (n) {               \
    case 4: return CALL(4);  \
    case 5: return CALL(5);  \
    case 6: return CALL(6);  \
    case 7: return CALL(7);  \
    case 8: return CALL(8);  \
    case 9: return CALL(9);  \
    default: return -2;      \
  }

size_t cdmc_state_bytes(int n, bool fp32) {
  if (n < 4 || n > 9) return 0;
  return (fp32 ? sizeof(float) : sizeof(double)) * (size_t)(1 << (n - 1)) * 95;
}

bool cdmc_global_state(int n, bool fp32) {
#define C_(NN) (fp32 ? cdmck::Global<NN, float>::value : cdmck::Global<NN, double>::value)
  switch (n) {
    case 4: return C_(4);
    case 5: return C_(5);
    case 6: return C_(6);
    case 7: return C_(7);
    case 8: return C_(8);
    case 9: return C_(9);
    default: return false;
  }
#undef C_
}

int cdmc_blocks_per_cu(int n, bool fp32) {
#define C_(NN)                                                                                  \
  (fp32 ? cdmck::occupancy<NN, float, cdmck::Global<NN, float>::value>()                        \
        : cdmck::occupancy<NN, double, cdmck::Global<NN, double>::value>())
  BG_CDMC_SWITCH(C_)
#undef C_
}

int cdmc_me2(int n, bool fp32, int64_t E, const double* mom, const double* phi, const double* eta,
             void* gstate, int grid, double* me2, hipStream_t stream) {
#define C_(NN)                                                                                   \
  (fp32 ? cdmck::launch<NN, float, cdmck::Global<NN, float>::value>(E, mom, phi, eta, gstate,     \
                                                                    grid, me2, stream)            \
        : cdmck::launch<NN, double, cdmck::Global<NN, double>::value>(E, mom, phi, eta, gstate,   \
                                                                      grid, me2, stream))
  BG_CDMC_SWITCH(C_)
#undef C_
}

#undef BG_CDMC_SWITCH

}  // namespace bg
