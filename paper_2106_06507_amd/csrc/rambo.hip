// Phase-space generation on the device: RAMBO (Kleiss, Stirling, Ellis,
// Comput. Phys. Commun. 40 (1986) 359), massless, with the p_T and Delta R
// cuts of Section 5, helicities and colour-flow pairs, all from a keyed
// counter-based SplitMix64 stream (Steele, Lea, Flood, OOPSLA 2014).
//
// Attempt t draws uniforms u_j = ((z >> 11) + 0.5) 2^-53 with
//   z = mix64(mix64(seed + G (t + 1)) + G (j + 1)),  G = 0x9E3779B97F4A7C15,
// j = 0 .. 4 n_out - 1 for RAMBO (four per outgoing gluon: cos theta, phi,
// and the two factors of the energy -log(r3 r4)), then n for the helicities
// (u < 1/2 -> +1), then 2n for the colour pairs (i_k, j_k) = min(3u, 2).
// The accepted events are the attempts that pass the cuts, in attempt order:
// pass 1 marks and counts them per block, pass 2 scans the block counts,
// pass 3 regenerates each accepted attempt and writes it at its rank.
// Incoming beams (sqrt(s)/2)(1, 0, 0, +-1) enter negated as gluons 1 and 2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bg_kernels.h"

namespace bg {
namespace genk {

constexpr int kThreads = 256;
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct Stream {
  uint64_t base;
  __device__ __forceinline__ double uniform(int j) const {
    const uint64_t z = mix64(base + kGamma * (uint64_t)(j + 1));
    return ((double)(z >> 11) + 0.5) * 0x1p-53;
  }
};

__device__ __forceinline__ Stream stream_of(uint64_t seed, uint64_t t) {
  return Stream{mix64(seed + kGamma * (t + 1))};
}

// RAMBO momenta p[i][mu] of the NO outgoing gluons of attempt t.
template <int NO>
__device__ __forceinline__ void rambo(const Stream& st, double sqrt_s, double p[NO][4]) {
  double q[NO][4];
  double Q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < NO; ++i) {
    const double c = 2.0 * st.uniform(4 * i) - 1.0;
    const double s = sqrt(fmax(0.0, 1.0 - c * c));
    const double f = 2.0 * M_PI * st.uniform(4 * i + 1);
    const double e = -log(st.uniform(4 * i + 2) * st.uniform(4 * i + 3));
    q[i][0] = e;
    q[i][1] = e * s * cos(f);
    q[i][2] = e * s * sin(f);
    q[i][3] = e * c;
#pragma unroll
    for (int m = 0; m < 4; ++m) Q[m] += q[i][m];
  }
  const double M = sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
  const double b[3] = {-Q[1] / M, -Q[2] / M, -Q[3] / M};
  const double x = sqrt_s / M;
  const double gam = Q[0] / M;
  const double a = 1.0 / (1.0 + gam);
#pragma unroll
  for (int i = 0; i < NO; ++i) {
    const double bq = b[0] * q[i][1] + b[1] * q[i][2] + b[2] * q[i][3];
    p[i][0] = x * (gam * q[i][0] + bq);
#pragma unroll
    for (int k = 0; k < 3; ++k) p[i][k + 1] = x * (q[i][k + 1] + b[k] * q[i][0] + a * bq * b[k]);
  }
}

// p_T > pt_min for every outgoing gluon, Delta R > dr_min for every pair
// (rapidity = pseudo-rapidity for massless momenta, Delta phi folded into
// [0, pi]).
template <int NO>
__device__ __forceinline__ bool pass_cuts(const double p[NO][4], double pt_min, double dr_min) {
  double eta[NO], phi[NO];
  bool ok = true;
#pragma unroll
  for (int i = 0; i < NO; ++i) {
    const double pt = hypot(p[i][1], p[i][2]);
    ok = ok && pt > pt_min;
    eta[i] = asinh(p[i][3] / pt);
    phi[i] = atan2(p[i][2], p[i][1]);
  }
  const double dr2 = dr_min * dr_min;
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = i + 1; j < NO; ++j) {
      double dphi = fabs(phi[i] - phi[j]);
      if (dphi > M_PI) dphi = 2.0 * M_PI - dphi;
      const double deta = eta[i] - eta[j];
      ok = ok && (deta * deta + dphi * dphi) > dr2;
    }
  return ok;
}

// Pass 1: acceptance bit per attempt (one 32-bit word per 32 attempts) and
// accepted count per block.
template <int NO>
__global__ void __launch_bounds__(kThreads) flags_kernel(GenParams gp, int64_t n_attempts,
                                                        unsigned* __restrict__ bits,
                                                        unsigned* __restrict__ block_count) {
  __shared__ unsigned wave_count[kThreads / 64];
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  bool ok = false;
  if (i < n_attempts) {
    ok = true;
    if (gp.cuts) {
      double p[NO][4];
      rambo<NO>(stream_of(gp.seed, gp.first_attempt + (uint64_t)i), gp.sqrt_s, p);
      ok = pass_cuts<NO>(p, gp.pt_min, gp.dr_min);
    }
  }
  const unsigned long long m = __ballot(ok);
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  // two 32-bit words per wave
  if (lane == 0 && i < n_attempts) bits[i >> 5] = (unsigned)(m & 0xffffffffull);
  if (lane == 32 && i < n_attempts) bits[i >> 5] = (unsigned)(m >> 32);
  if (lane == 0) wave_count[w] = (unsigned)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned c = 0;
    for (int v = 0; v < kThreads / 64; ++v) c += wave_count[v];
    block_count[blockIdx.x] = c;
  }
}

// Pass 2: exclusive scan of the block counts in place (one block); total at
// block_count[n_blocks].
__global__ void __launch_bounds__(1024) scan_kernel(unsigned* __restrict__ block_count,
                                                    int n_blocks) {
  __shared__ unsigned part[1024];
  const int t = threadIdx.x;
  const int per = (n_blocks + 1023) / 1024;
  const int lo = t * per;
  const int hi = lo + per < n_blocks ? lo + per : n_blocks;
  unsigned s = 0;
  for (int k = lo; k < hi; ++k) s += block_count[k];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off *= 2) {
    const unsigned v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  unsigned run = part[t] - s;  // exclusive prefix of this thread's range
  for (int k = lo; k < hi; ++k) {
    const unsigned c = block_count[k];
    block_count[k] = run;
    run += c;
  }
  if (t == 1023) block_count[n_blocks] = part[1023];
}

// Pass 3: regenerate accepted attempts and write them at their rank.
template <int NO>
__global__ void __launch_bounds__(kThreads) write_kernel(GenParams gp, int64_t n_attempts,
                                                        const unsigned* __restrict__ bits,
                                                        const unsigned* __restrict__ block_offset,
                                                        int64_t max_events, double* __restrict__ mom,
                                                        int8_t* __restrict__ hel,
                                                        int8_t* __restrict__ col,
                                                        int64_t* __restrict__ attempt,
                                                        int64_t* __restrict__ n_out) {
  constexpr int N = NO + 2;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t total = block_offset[gridDim.x];
    n_out[0] = total < max_events ? total : max_events;
  }
  if (i >= n_attempts) return;
  const unsigned word = bits[i >> 5];
  const int b = (int)(i & 31);
  if (!((word >> b) & 1u)) return;
  // rank within the block: accepted attempts of the block before this one
  const int64_t blk0 = (int64_t)blockIdx.x * kThreads;
  int64_t r = block_offset[blockIdx.x];
  for (int64_t wv = blk0 >> 5; wv < (i >> 5); ++wv) r += __popc(bits[wv]);
  r += __popc(word & ((1u << b) - 1u));
  if (r >= max_events) return;
  const Stream st = stream_of(gp.seed, gp.first_attempt + (uint64_t)i);
  double p[NO][4];
  rambo<NO>(st, gp.sqrt_s, p);
  const int64_t E = max_events;
  const double half = 0.5 * gp.sqrt_s;
  mom[(0 * 4 + 0) * E + r] = -half;
  mom[(0 * 4 + 1) * E + r] = 0.0;
  mom[(0 * 4 + 2) * E + r] = 0.0;
  mom[(0 * 4 + 3) * E + r] = -half;
  mom[(1 * 4 + 0) * E + r] = -half;
  mom[(1 * 4 + 1) * E + r] = 0.0;
  mom[(1 * 4 + 2) * E + r] = 0.0;
  mom[(1 * 4 + 3) * E + r] = half;
#pragma unroll
  for (int k = 0; k < NO; ++k)
#pragma unroll
    for (int m = 0; m < 4; ++m) mom[((int64_t)(k + 2) * 4 + m) * E + r] = p[k][m];
  if (hel) {
#pragma unroll
    for (int k = 0; k < N; ++k)
      hel[(int64_t)k * E + r] = st.uniform(4 * NO + k) < 0.5 ? (int8_t)1 : (int8_t)-1;
  }
  if (col) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const int ci = (int)(st.uniform(4 * NO + N + 2 * k) * 3.0);
      const int cj = (int)(st.uniform(4 * NO + N + 2 * k + 1) * 3.0);
      col[(int64_t)k * E + r] = (int8_t)(ci < 2 ? ci : 2);
      col[((int64_t)N + k) * E + r] = (int8_t)(cj < 2 ? cj : 2);
    }
  }
  if (attempt) attempt[r] = (int64_t)(gp.first_attempt + (uint64_t)i);
}

template <int NO>
int launch(const GenParams& gp, int64_t n_attempts, int64_t max_events, unsigned* ws,
           double* mom, int8_t* hel, int8_t* col, int64_t* attempt, int64_t* n_out,
           hipStream_t stream) {
  const int64_t blocks = (n_attempts + kThreads - 1) / kThreads;
  unsigned* bits = ws;
  unsigned* counts = ws + (n_attempts + 31) / 32;
  hipLaunchKernelGGL((flags_kernel<NO>), dim3((unsigned)blocks), dim3(kThreads), 0, stream, gp,
                     n_attempts, bits, counts);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, stream, counts, (int)blocks);
  hipLaunchKernelGGL((write_kernel<NO>), dim3((unsigned)blocks), dim3(kThreads), 0, stream, gp,
                     n_attempts, bits, counts, max_events, mom, hel, col, attempt, n_out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace genk

namespace genk {

// Continuous colour and polarization variables of event t = first + e:
// draws 5k .. 5k+4 of the event's stream for gluon k: phi = 2 pi u, then
// (cos theta, azimuth) of eta(z_k) and of eta(zbar_k) with
// cos theta = 2u - 1, azimuth 2 pi u (uniform on the unit sphere, Section
// 2.1 eq. color_angles).  phi [n][E], eta [2][n][3][E].
__global__ void __launch_bounds__(kThreads) continuous_kernel(int n, uint64_t seed, uint64_t first,
                                                             int64_t E, double* __restrict__ phi,
                                                             double* __restrict__ eta) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= E) return;
  const Stream st = stream_of(seed, first + (uint64_t)e);
  for (int k = 0; k < n; ++k) {
    phi[(int64_t)k * E + e] = 2.0 * M_PI * st.uniform(5 * k);
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const double c = 2.0 * st.uniform(5 * k + 1 + 2 * v) - 1.0;
      const double sn = sqrt(fmax(0.0, 1.0 - c * c));
      const double a = 2.0 * M_PI * st.uniform(5 * k + 2 + 2 * v);
      double* out = eta + ((int64_t)(v * n + k) * 3) * E + e;
      out[0] = c;
      out[E] = sn * cos(a);
      out[2 * E] = sn * sin(a);
    }
  }
}

}  // namespace genk

int generate_continuous(int n, uint64_t seed, uint64_t first, int64_t E, double* phi, double* eta,
                        hipStream_t stream) {
  if (E <= 0) return 0;
  const int64_t blocks = (E + genk::kThreads - 1) / genk::kThreads;
  hipLaunchKernelGGL(genk::continuous_kernel, dim3((unsigned)blocks), dim3(genk::kThreads), 0, stream,
                     n, seed, first, E, phi, eta);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

size_t generate_workspace_words(int64_t n_attempts) {
  const int64_t blocks = (n_attempts + genk::kThreads - 1) / genk::kThreads;
  return (size_t)((n_attempts + 31) / 32 + blocks + 1);
}

int generate_events(const GenParams& gp, int64_t n_attempts, int64_t max_events, unsigned* ws,
                    double* mom, int8_t* hel, int8_t* col, int64_t* attempt, int64_t* n_out,
                    hipStream_t stream) {
  switch (gp.n) {
#define BG_CASE(NN) \
  case NN:          \
    return genk::launch<NN - 2>(gp, n_attempts, max_events, ws, mom, hel, col, attempt, n_out, stream);
    BG_CASE(4)
    BG_CASE(5)
    BG_CASE(6)
    BG_CASE(7)
    BG_CASE(8)
    BG_CASE(9)
#undef BG_CASE
    default:
      return -2;
  }
}

}  // namespace bg
