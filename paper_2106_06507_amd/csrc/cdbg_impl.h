// Colour-dressed Berends-Giele recursion (Section 2.3, eqs. cdcurrents and
// color_dressed_currents, with the tensor auxiliary field of eqs. prop_pseudo,
// cobg_tensor_current and cobg_tensor_vertex) for one sampled colour-flow
// assignment per event (Section 2.2, eq. color_decomposition_colorflow).
//
// Colour structure.  Gluon k carries E_k = e_{j_k i_k}, a directed edge
// j_k -> i_k between the three colours.  The dressed current of a subset S is
// the sum over orderings of E_s1..E_sk J(s), so its 3x3 colour matrix is
// non-zero only in entries (r, c) such that the edges of S form a trail from
// r to c: if S is balanced (in = out degree at every colour) only diagonal
// entries (v, v) with v touched by S survive; otherwise exactly one entry
// (r, c) with out-in = +1 at r and -1 at c.  A subset whose edges are not
// connected, or whose degrees allow no trail, has a zero current.  Each subset
// therefore stores three slots: slot v = entry (v, v) when balanced, slot 0 =
// entry (r, c) otherwise.  Only the slots a subset can hold are stored: one
// for a trail, one per touched colour for a balanced subset, none for a zero
// current, packed in mask order (the subset's code word carries the index of
// its first slot).  Over every valid flow (all 9^n colour assignments that
// close, enumerated exhaustively for n = 4..9) the total is at most
// (2^(n-1) - 1) + 2^(n-1)/4, against 3 (2^(n-1) - 1) for three slots per
// subset.  The matrix product J(S1) J(S2) in the recursion
// then selects one operand pair per target slot:
//   S1 (r1,c1), S2 (r2,c2):  needs c1 = r2, gives (r1, c2)
//   S1 (r1,c1), S2 balanced: slots (0, c1) -> (r1, c1)
//   S1 balanced, S2 (r2,c2): slots (r2, 0) -> (r2, c2)
//   both balanced:           slots (v, v) -> (v, v).
// An event's full amplitude is non-zero only if all n edges form a closed
// circuit (balanced and connected); other events get exactly 0.
//
// Recursion (couplings g_s/sqrt2 factored out as in bg_device.h), summed over
// ordered splits (S1, S2) of S:
//   J(S) = 1/P_S^2 sum [ V3(P1, P2; J1, J2) + T2.J1 - T1.J2 ],
//   T(S) = sum [ J1^a J2^b - J1^b J2^a ],     (T.J)^nu = T^{nu beta} J_beta,
// and A = (g_s/sqrt2)^(n-2) eps_n . (P^2 J)_{i_n j_n}(1..n-1).  The bracket
// and the tensor term change sign when the two operands (with their momenta)
// are exchanged, so the kernel sums over unordered splits with the colour
// commutator [J1, J2] instead (pair_slots): splits of two balanced subsets
// drop out, a trail and a balanced subset take one evaluation, and half the
// candidate splits are visited.
//
// Parallel layout (gfx950): one 64-lane wave per valid event, persistent
// blocks pulling events from a compacted list.  Currents, tensors, momenta and
// 1/P^2 of all subsets live in LDS.  Subsets are processed by size; the
// (subset, slot) targets of a size are spread over the lanes, and when there
// are fewer targets than lanes each target's splits are shared by q lanes
// whose partial sums are added in a fixed order (deterministic results).
#pragma once

#include <stdint.h>

#include "bg_device.h"
#include "bg_kernels.h"

namespace bg {
namespace cdbgk {

constexpr int kWave = 64;

// LDS layout of one event (T = float or double), M = n - 1 gluons in subsets.
// EST: also the rounding-error bounds of every current and tensor slot and
// the energy sum of every subset (see cdbg_one_event).
template <int N, typename T, bool EST = false>
struct Lay {
  static constexpr int M = N - 1;
  static constexpr int NS = 1 << M;          // subsets (mask 0 unused)
  static constexpr int kCap = NS - 1 + NS / 4;  // stored slots of a valid flow, at most
  static constexpr int kJ = kCap * 8;        // currents [slot][re0..3, im0..3]
  static constexpr int kT = kCap * 12;       // tensors  [slot][re6, im6]
  static constexpr int kP = NS * 4;          // momenta  [mask][mu]
  static constexpr int kI = NS;              // 1/P^2    [mask]
  static constexpr int kB = EST ? kCap * 2 + NS : 0;  // bounds [slot] of J and T, E [mask]
  static constexpr int kItems = kCap;        // target list of one size
  static constexpr int kPm = 4 * N;          // FP64 momenta of the event [gluon][mu]
  static constexpr size_t bytes() {
    return sizeof(double) * (size_t)kPm + sizeof(T) * (size_t)(kJ + kT + kP + kI + kB) +
           sizeof(int) * (size_t)(NS + kItems + 2 * N + 16);
  }
};

template <int N, typename T>
struct Sm {
  double* pm;
  T* J;
  T* Tt;
  T* P;
  T* ip2;
  T* bJ;       // EST: bound of each current slot [slot]
  T* bT;       // EST: bound of each tensor slot [slot]
  T* en;       // EST: sum of |p^0| over the subset [mask]
  int* code;   // per mask: 0 zero; 1 | r << 2 | c << 4 unbalanced; 2 | touched << 6
               // balanced; | first slot << 9 (see slot_index)
  int* items;
  int* ci;     // colours i_k
  int* cj;     // colours j_k
  int* misc;   // [3 w + t]: items of slot t found by wave w; [12]: broadcast
};

template <int N, typename T, bool EST = false>
__device__ __forceinline__ Sm<N, T> carve(unsigned char* raw) {
  using L = Lay<N, T, EST>;
  Sm<N, T> s;
  s.pm = reinterpret_cast<double*>(raw);
  T* t = reinterpret_cast<T*>(s.pm + L::kPm);
  s.J = t;
  s.Tt = s.J + L::kJ;
  s.P = s.Tt + L::kT;
  s.ip2 = s.P + L::kP;
  s.bJ = s.ip2 + L::kI;
  s.bT = s.bJ + (EST ? L::kCap : 0);
  s.en = s.bT + (EST ? L::kCap : 0);
  int* ip = reinterpret_cast<int*>(s.ip2 + L::kI + L::kB);
  s.code = ip;
  s.items = s.code + L::NS;
  s.ci = s.items + L::kItems;
  s.cj = s.ci + N;
  s.misc = s.cj + N;
  return s;
}

// g += s t j for complex t, j and a real sign s, one multiply-add per real
// product
template <typename T>
__device__ __forceinline__ void cmac(T& gr, T& gi, T s, T tr, T ti, T jr, T ji) {
  const T str = s * tr, sti = s * ti;
  gr += str * jr;
  gr -= sti * ji;
  gi += str * ji;
  gi += sti * jr;
}

// (T.J)^nu = T^{nu beta} g_beta beta J^beta for antisymmetric T stored as
// components (01, 02, 03, 12, 13, 23); acc += sgn * T.J (complex).
template <typename T>
__device__ __forceinline__ void tdotj_acc(T* gre, T* gim, const T* tre, const T* tim,
                                          const T* jre, const T* jim, T sgn) {
  const T m = -sgn;
  // nu = 0: -(T01 J1 + T02 J2 + T03 J3)
  cmac(gre[0], gim[0], m, tre[0], tim[0], jre[1], jim[1]);
  cmac(gre[0], gim[0], m, tre[1], tim[1], jre[2], jim[2]);
  cmac(gre[0], gim[0], m, tre[2], tim[2], jre[3], jim[3]);
  // nu = 1: -T01 J0 - T12 J2 - T13 J3
  cmac(gre[1], gim[1], m, tre[0], tim[0], jre[0], jim[0]);
  cmac(gre[1], gim[1], m, tre[3], tim[3], jre[2], jim[2]);
  cmac(gre[1], gim[1], m, tre[4], tim[4], jre[3], jim[3]);
  // nu = 2: -T02 J0 + T12 J1 - T23 J3
  cmac(gre[2], gim[2], m, tre[1], tim[1], jre[0], jim[0]);
  cmac(gre[2], gim[2], sgn, tre[3], tim[3], jre[1], jim[1]);
  cmac(gre[2], gim[2], m, tre[5], tim[5], jre[3], jim[3]);
  // nu = 3: -T03 J0 + T13 J1 + T23 J2
  cmac(gre[3], gim[3], m, tre[2], tim[2], jre[0], jim[0]);
  cmac(gre[3], gim[3], sgn, tre[4], tim[4], jre[1], jim[1]);
  cmac(gre[3], gim[3], sgn, tre[5], tim[5], jre[2], jim[2]);
}

// The x-th subset of S in the order of the binary counter over S's bits
// (bit b of x selects the b-th lowest member of S): x = 1 .. 2^|S| - 2 runs
// over the non-empty proper subsets.  Fixed trip count (no divergence).
template <int M>
__device__ __forceinline__ int subset_of(int x, int S) {
  int r = 0, j = 0;
#pragma unroll
  for (int b = 0; b < M; ++b) {
    const bool in = (S >> b) & 1;
    r |= (in && ((x >> j) & 1)) ? (1 << b) : 0;
    j += in ? 1 : 0;
  }
  return r;
}

// v from lane + off (own value where that lane does not exist).
template <typename T>
__device__ __forceinline__ T shfl_down_t(T v, int off) {
  return __shfl_down(v, (unsigned)off, kWave);
}

// Unordered split {m1, m2} of S feeding target slot t of S.  The ordered
// contribution F(P1, P2; X1, X2) (X = current and tensor field) is bilinear
// and changes sign when the two operands are exchanged, so the two orders of
// a split combine into one evaluation F(P_L, P_R; X_L, X_R) with the colour
// commutator in the right operand:
//   two trails:           at most one order gives entry t (both orders
//                         give different diagonal entries of a balanced S);
//   trail (r, c) U and balanced D:  X_R = X_D(c, c) - X_D(r, r), L = U
//                         (entry (r, c) of [X_U, X_D]);
//   both balanced:        diagonal matrices commute, the orders cancel.
// Returns false if the split contributes nothing; otherwise swap tells
// whether L is m2, iL is L's slot and X_R = X[ip] - X[im] (an index < 0
// stands for a colour the balanced operand does not touch: a zero entry).
__device__ __forceinline__ bool pair_slots(int c1, int c2, int t, bool& swap, int& iL, int& ip,
                                           int& im) {
  if ((c1 & 3) == 0 || (c2 & 3) == 0) return false;  // zero currents
  const bool b1 = (c1 & 3) == 2, b2 = (c2 & 3) == 2;
  if (b1 && b2) return false;
  if (!b1 && !b2) {
    const int r1 = (c1 >> 2) & 3, k1 = (c1 >> 4) & 3;
    const int r2 = (c2 >> 2) & 3, k2 = (c2 >> 4) & 3;
    if (k1 == r2 && (r1 == k2 ? r1 : 0) == t) swap = false;
    else if (k2 == r1 && (r2 == k1 ? r2 : 0) == t) swap = true;
    else return false;
    iL = (swap ? c2 : c1) >> 9;
    ip = (swap ? c1 : c2) >> 9;
    im = -1;
    return true;
  }
  if (t != 0) return false;
  swap = b1;
  const int cu = b1 ? c2 : c1, cd = b1 ? c1 : c2;
  const int r = (cu >> 2) & 3, c = (cu >> 4) & 3, touched = (cd >> 6) & 7;
  const int first = cd >> 9;
  ip = (touched >> c) & 1 ? first + __popc(touched & ((1 << c) - 1)) : -1;
  im = (touched >> r) & 1 ? first + __popc(touched & ((1 << r) - 1)) : -1;
  iL = cu >> 9;
  return ip >= 0 || im >= 0;
}

// Packed index of colour slot s of a subset with code word c (s a slot the
// subset holds): its first slot, plus for a balanced subset the touched
// colours below s.
__device__ __forceinline__ int slot_index(int c, int s) {
  const int first = c >> 9;
  return (c & 3) == 2 ? first + __popc(((c >> 6) & 7) & ((1 << s) - 1)) : first;
}

// Number of slots a subset with code c holds.
__device__ __forceinline__ int slot_count(int c) {
  return (c & 3) == 1 ? 1 : ((c & 3) == 2 ? __popc((c >> 6) & 7) : 0);
}

// Accumulate F(P_L, P_R; X_L, X_R) for left operand slot iL of subset mL
// and right operand X[ip] - X[im] of subset mR (see pair_slots).
template <int N, typename T>
__device__ __forceinline__ void split_contrib(const Sm<N, T>& sm, int mL, int mR, int iL, int ip,
                                              int im, bool want_tensor, T* gre, T* gim, T* tre,
                                              T* tim) {
  const T* J1 = sm.J + iL * 8;
  T a_re[4], a_im[4], b_re[4], b_im[4], P1[4], P2[4];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    a_re[mu] = J1[mu];
    a_im[mu] = J1[4 + mu];
    P1[mu] = sm.P[mL * 4 + mu];
    P2[mu] = sm.P[mR * 4 + mu];
  }
  if (ip >= 0) {
    const T* J2 = sm.J + ip * 8;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      b_re[mu] = J2[mu];
      b_im[mu] = J2[4 + mu];
    }
  } else {
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) b_re[mu] = b_im[mu] = T(0);
  }
  if (im >= 0) {
    const T* J2 = sm.J + im * 8;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      b_re[mu] -= J2[mu];
      b_im[mu] -= J2[4 + mu];
    }
  }
  // V3(P1, P2; J1, J2) = (J1.J2)(P1-P2) + ((2P2+P1).J1) J2 - ((2P1+P2).J2) J1
  T abr = a_re[0] * b_re[0] - a_im[0] * b_im[0];
  T abi = a_re[0] * b_im[0] + a_im[0] * b_re[0];
  T c1r = (T(2) * P2[0] + P1[0]) * a_re[0], c1i = (T(2) * P2[0] + P1[0]) * a_im[0];
  T c2r = (T(2) * P1[0] + P2[0]) * b_re[0], c2i = (T(2) * P1[0] + P2[0]) * b_im[0];
#pragma unroll
  for (int mu = 1; mu < 4; ++mu) {
    abr -= a_re[mu] * b_re[mu];
    abr += a_im[mu] * b_im[mu];
    abi -= a_re[mu] * b_im[mu];
    abi -= a_im[mu] * b_re[mu];
    const T q = T(2) * P2[mu] + P1[mu], p = T(2) * P1[mu] + P2[mu];
    c1r -= q * a_re[mu];
    c1i -= q * a_im[mu];
    c2r -= p * b_re[mu];
    c2i -= p * b_im[mu];
  }
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const T d = P1[mu] - P2[mu];
    gre[mu] += abr * d;
    gre[mu] += c1r * b_re[mu];
    gre[mu] -= c1i * b_im[mu];
    gre[mu] -= c2r * a_re[mu];
    gre[mu] += c2i * a_im[mu];
    gim[mu] += abi * d;
    gim[mu] += c1r * b_im[mu];
    gim[mu] += c1i * b_re[mu];
    gim[mu] -= c2r * a_im[mu];
    gim[mu] -= c2i * a_re[mu];
  }
  // tensor couplings: + T2.J1 - T1.J2
  const T* T1 = sm.Tt + iL * 12;
  {
    T t_re[6], t_im[6];
    if (ip >= 0) {
      const T* T2 = sm.Tt + ip * 12;
#pragma unroll
      for (int x = 0; x < 6; ++x) {
        t_re[x] = T2[x];
        t_im[x] = T2[6 + x];
      }
    } else {
#pragma unroll
      for (int x = 0; x < 6; ++x) t_re[x] = t_im[x] = T(0);
    }
    if (im >= 0) {
      const T* T2 = sm.Tt + im * 12;
#pragma unroll
      for (int x = 0; x < 6; ++x) {
        t_re[x] -= T2[x];
        t_im[x] -= T2[6 + x];
      }
    }
    tdotj_acc(gre, gim, t_re, t_im, a_re, a_im, T(1));
#pragma unroll
    for (int x = 0; x < 6; ++x) {
      t_re[x] = T1[x];
      t_im[x] = T1[6 + x];
    }
    tdotj_acc(gre, gim, t_re, t_im, b_re, b_im, T(-1));
  }
  if (want_tensor) {
    // antisymmetric J1^a J2^b - J1^b J2^a for (ab) = 01, 02, 03, 12, 13, 23
    const int ia[6] = {0, 0, 0, 1, 1, 2};
    const int ib[6] = {1, 2, 3, 2, 3, 3};
#pragma unroll
    for (int x = 0; x < 6; ++x) {
      const int a = ia[x], b = ib[x];
      tre[x] += a_re[a] * b_re[b];
      tre[x] -= a_im[a] * b_im[b];
      tre[x] -= a_re[b] * b_re[a];
      tre[x] += a_im[b] * b_im[a];
      tim[x] += a_re[a] * b_im[b];
      tim[x] += a_im[a] * b_re[b];
      tim[x] -= a_re[b] * b_im[a];
      tim[x] -= a_im[b] * b_re[a];
    }
  }
}

// Degrees, touched colours and connectivity of a set of colour edges
// j -> i over the three colours, kept in registers (packed union-find: two
// bits of parent per colour).
struct ColourGraph {
  int d0 = 0, d1 = 0, d2 = 0;  // out - in degree per colour
  int par = 0 | (1 << 2) | (2 << 4);
  int touched = 0;

  __device__ __forceinline__ int find(int a) const {
    int p = (par >> (2 * a)) & 3;
    while (p != a) {
      a = p;
      p = (par >> (2 * a)) & 3;
    }
    return a;
  }
  __device__ __forceinline__ void add(int jj, int ii) {
    d0 += (jj == 0) - (ii == 0);
    d1 += (jj == 1) - (ii == 1);
    d2 += (jj == 2) - (ii == 2);
    touched |= (1 << ii) | (1 << jj);
    const int a = find(jj), b = find(ii);
    if (a != b) par = (par & ~(3 << (2 * a))) | (b << (2 * a));
  }
  __device__ __forceinline__ bool connected() const {
    int root = -1;
    bool conn = true;
    for (int v = 0; v < 3; ++v) {
      if (!(touched & (1 << v))) continue;
      const int a = find(v);
      if (root < 0) root = a;
      else if (a != root) conn = false;
    }
    return conn;
  }
  __device__ __forceinline__ bool balanced() const { return d0 == 0 && d1 == 0 && d2 == 0; }
  // subset code: 0 zero current; 1 | r << 2 | c << 4 single trail r -> c;
  // 2 | touched << 6 balanced
  __device__ __forceinline__ int code() const {
    if (!connected()) return 0;
    if (balanced()) return 2 | (touched << 6);
    const int dv[3] = {d0, d1, d2};
    int r = -1, c = -1;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      if (dv[v] == 1) r = v;
      else if (dv[v] == -1) c = v;
      else if (dv[v] != 0) return 0;
    }
    return (r >= 0 && c >= 0) ? (1 | (r << 2) | (c << 4)) : 0;
  }
};

// True if the colour-flow edges j_k -> i_k of event e are balanced (in =
// out degree at every colour) and connected, i.e. form one closed circuit.
// Indices outside 0..2 make the event invalid.
__device__ __forceinline__ bool flow_valid(int n, int64_t E, const int8_t* __restrict__ col,
                                           int64_t e) {
  ColourGraph g;
  bool in_range = true;
  for (int k = 0; k < n; ++k) {
    int ii = col[(int64_t)k * E + e];
    int jj = col[((int64_t)n + k) * E + e];
    if (ii < 0 || ii > 2 || jj < 0 || jj > 2) {
      in_range = false;
      ii = 0;
      jj = 0;
    }
    g.add(jj, ii);
  }
  return in_range && g.balanced() && g.connected();
}

// Check of the FP32 recursion (EST): alongside every current and tensor slot
// the recursion carries a bound on its components computed as if every
// product were taken in modulus: 1 for an external polarization; for a slot
// of subset S, with E_S the sum of |p^0| over S (a bound on every momentum
// component of a sub-subset) and the split operands' bounds bJ, bT,
//   bT(S) = sum_splits bJ1 bJ2,
//   bJ(S) = |1/P_S^2| sum_splits (E_S bJ1 bJ2 + bT2 bJ1 + bT1 bJ2),
// constant factors of the vertices dropped.  An event whose amplitude
// A = eps_n . Jhat satisfies bJ(top)^2 > tau |A|^2 cancels strongly, so FP32
// rounding is amplified; it is appended to list for an FP64 re-evaluation.
struct DressedCheck {
  float tau;
  unsigned* count;
  unsigned* list;
};

// One valid event (colour flow closes into a circuit) on the NL lanes of this
// block (NL = 64: one wave; NL = 256: four waves sharing the event's LDS).
template <int N, typename T, int NL = kWave, bool EST = false>
__device__ __forceinline__ void cdbg_one_event(const Sm<N, T>& sm, int64_t E,
                                               const double* __restrict__ mom,
                                               const int8_t* __restrict__ hel,
                                               const int8_t* __restrict__ col, int64_t e,
                                               double* __restrict__ me2,
                                               DressedCheck chk = DressedCheck{}) {
  using L = Lay<N, T, EST>;
  constexpr int M = N - 1;
  constexpr int NS = L::NS;
  constexpr int NW = NL / kWave;
  static_assert(NL % kWave == 0 && NW <= 4, "one to four waves per event");
  const int lane = threadIdx.x;
  const int w = lane / kWave, lw = lane % kWave;
  // ---- event set-up -------------------------------------------------
  if (lane < N) {
    sm.ci[lane] = col[(int64_t)lane * E + e];
    sm.cj[lane] = col[((int64_t)N + lane) * E + e];
  }
  if (lane < 4 * N) sm.pm[lane] = mom[(int64_t)lane * E + e];  // [k][mu] = row 4k + mu
  __syncthreads();
  // subset codes, momenta, 1/P^2 (FP64 sums); subset index x + 1 for
  // x = lane, lane + NL, ...
  for (int mask = lane + 1; mask < NS; mask += NL) {
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    double en = 0.0;
    ColourGraph g;
    for (int k = 0; k < M; ++k) {
      if (!(mask & (1 << k))) continue;
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) q[mu] += sm.pm[k * 4 + mu];
      en += fabs(sm.pm[k * 4]);
      g.add(sm.cj[k], sm.ci[k]);
    }
    if constexpr (EST) sm.en[mask] = (T)en;
    sm.code[mask] = g.code();
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) sm.P[mask * 4 + mu] = (T)q[mu];
    const double p2 = q[0] * q[0] - q[1] * q[1] - q[2] * q[2] - q[3] * q[3];
    sm.ip2[mask] = (T)(1.0 / p2);
  }
  __syncthreads();
  // first packed slot of every subset: exclusive prefix sum of the slot
  // counts in subset order, NL subsets per round (a shuffle scan per wave,
  // then the wave totals), carried over the rounds
  int total = 0;
  for (int base = 1; base < NS; base += NL) {
    const int mask = base + lane;
    const int code = mask < NS ? sm.code[mask] : 0;
    const int cnt = slot_count(code);
    int incl = cnt;
#pragma unroll
    for (int off = 1; off < kWave; off *= 2) {
      const int v = __shfl_up(incl, (unsigned)off, kWave);
      if (lw >= off) incl += v;
    }
    if (lw == kWave - 1) sm.misc[w] = incl;
    __syncthreads();
    int first = total + incl - cnt;
#pragma unroll
    for (int v = 0; v < NW; ++v) {
      const int tv = sm.misc[v];
      first += v < w ? tv : 0;
      total += tv;
    }
    __syncthreads();  // misc is read by every lane before the next round rewrites it
    if (mask < NS) sm.code[mask] = code | (first << 9);
  }
  // a valid flow holds at most kCap slots (exhaustive count over all flows);
  // the guard keeps the packed arrays in bounds regardless
  if (total > L::kCap) {
    if (lane == 0) me2[e] = __builtin_nan("");
    return;  // uniform over the block
  }
  __syncthreads();
  // external currents of gluons 0..M-1 into their colour slot (the tensor
  // of a single gluon is 0)
  if (lane < M) {
    double p[4], er[4], ei[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) p[mu] = sm.pm[lane * 4 + mu];
    polarization(p, (int)hel[(int64_t)lane * E + e], er, ei);
    const int si = sm.code[1 << lane] >> 9;  // the gluon's only slot
    T* dst = sm.J + si * 8;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      dst[mu] = (T)er[mu];
      dst[4 + mu] = (T)ei[mu];
    }
    T* dt = sm.Tt + si * 12;
#pragma unroll
    for (int x = 0; x < 12; ++x) dt[x] = T(0);
    if constexpr (EST) {
      sm.bJ[si] = T(1);
      sm.bT[si] = T(0);
    }
  }
  __syncthreads();

  // ---- recursion by subset size ---------------------------------------
  for (int size = 2; size <= M; ++size) {
    const bool top = size == M;
    // targets (mask, slot) of this size
    int nitems = 0;
    if (top) {
      if (lane == 0) {
        const int ii = sm.ci[M], jj = sm.cj[M];  // last gluon: entry (i_n, j_n)
        sm.items[0] = (NS - 1) * 4 + (ii == jj ? ii : 0);
      }
      nitems = 1;
    } else {
      // compaction of the (mask, slot) targets: slot-major, waves in order
      for (int base = 0; base < NS; base += NL) {
        const int tm = base + lane;
        int tc = 0;
        if (tm > 0 && tm < NS && __popc(tm) == size) tc = sm.code[tm];
        bool ok[3];
        unsigned long long bal[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          ok[t] = false;
          if ((tc & 3) == 1) ok[t] = (t == 0);
          else if ((tc & 3) == 2) ok[t] = ((tc >> 6) >> t) & 1;
          bal[t] = __ballot(ok[t]);
        }
        if (lw == 0) {
#pragma unroll
          for (int t = 0; t < 3; ++t) sm.misc[3 * w + t] = __popcll(bal[t]);
        }
        __syncthreads();
        const unsigned long long below = lw ? ((~0ull) >> (kWave - lw)) : 0ull;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          int before = 0, all = 0;
#pragma unroll
          for (int v = 0; v < NW; ++v) {
            const int cnt = sm.misc[3 * v + t];
            if (v < w) before += cnt;
            all += cnt;
          }
          if (ok[t]) sm.items[nitems + before + __popcll(bal[t] & below)] = tm * 4 + t;
          nitems += all;
        }
        __syncthreads();  // misc is rewritten by the next base
      }
    }
    __syncthreads();
    // q adjacent lanes of one wave per target (no more than it has splits),
    // each taking a contiguous range of its splits
    const int nsplit = (1 << (size - 1)) - 1;  // unordered splits (pair_slots)
    int q = nitems == 0 ? 1 : NL / nitems;
    q = q > nsplit ? nsplit : q;
    q = q < 1 ? 1 : (q > kWave ? kWave : q);
    const int gpw = kWave / q;  // targets per wave and round
    const int per_round = gpw * NW;
    for (int r0 = 0; r0 < nitems; r0 += per_round) {
      const int grp = lw / q;
      const int it = r0 + w * gpw + grp;
      const int sub = lw % q;
      T gre[4] = {0, 0, 0, 0}, gim[4] = {0, 0, 0, 0};
      T tre[6] = {0, 0, 0, 0, 0, 0}, tim[6] = {0, 0, 0, 0, 0, 0};
      T bv = T(0), bt = T(0);  // EST: bounds of this lane's share of the current and tensor
      int S = 0, t = 0;
      const bool active = grp < gpw && it < nitems;
      if (active) {
        const int item = sm.items[it];
        S = item >> 2;
        t = item & 3;
        T enS = T(0);
        if constexpr (EST) enS = sm.en[S];
        // a contiguous range of splits per lane: the first sub-mask (of
        // S's members below its highest one, so each unordered split comes
        // once) is deposited into S's bits, the next ones follow as
        // (m1 - S) & S
        const int per = (nsplit + q - 1) / q;
        const int k0 = sub * per;
        const int k1 = k0 + per < nsplit ? k0 + per : nsplit;
        int m1 = k0 < k1 ? subset_of<M>(k0 + 1, S) : 0;
        for (int k = k0; k < k1; ++k, m1 = (m1 - S) & S) {
          const int m2 = S ^ m1;
          bool swap;
          int iL, ip, im;
          if (!pair_slots(sm.code[m1], sm.code[m2], t, swap, iL, ip, im)) continue;
          split_contrib<N, T>(sm, swap ? m2 : m1, swap ? m1 : m2, iL, ip, im, !top, gre, gim, tre,
                              tim);
          if constexpr (EST) {
            const T j1 = sm.bJ[iL];
            const T j2 = (ip >= 0 ? sm.bJ[ip] : T(0)) + (im >= 0 ? sm.bJ[im] : T(0));
            const T t2 = (ip >= 0 ? sm.bT[ip] : T(0)) + (im >= 0 ? sm.bT[im] : T(0));
            const T jj = j1 * j2;
            bv += enS * jj;
            bv += t2 * j1;
            bv += sm.bT[iL] * j2;
            bt += jj;
          }
        }
      }
      // fixed-order tree over the q lanes of a target (all lanes take part)
      for (int off = 1; off < q; off *= 2) {
        const bool take = (sub % (2 * off)) == 0 && sub + off < q;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const T a = shfl_down_t(gre[x], off), b = shfl_down_t(gim[x], off);
          if (take) {
            gre[x] += a;
            gim[x] += b;
          }
        }
        if (!top) {
#pragma unroll
          for (int x = 0; x < 6; ++x) {
            const T a = shfl_down_t(tre[x], off), b = shfl_down_t(tim[x], off);
            if (take) {
              tre[x] += a;
              tim[x] += b;
            }
          }
        }
        if constexpr (EST) {
          const T a = shfl_down_t(bv, off), b = shfl_down_t(bt, off);
          if (take) {
            bv += a;
            bt += b;
          }
        }
      }
      if (active && sub == 0) {
        if (top) {
          double p[4], er[4], ei[4];
#pragma unroll
          for (int mu = 0; mu < 4; ++mu) p[mu] = sm.pm[M * 4 + mu];
          polarization(p, (int)hel[(int64_t)M * E + e], er, ei);
          double ar = 0.0, ai = 0.0;
#pragma unroll
          for (int mu = 0; mu < 4; ++mu) {
            const double sg = mu == 0 ? 1.0 : -1.0;
            ar += sg * (er[mu] * (double)gre[mu] - ei[mu] * (double)gim[mu]);
            ai += sg * (er[mu] * (double)gim[mu] + ei[mu] * (double)gre[mu]);
          }
          if constexpr (EST) {
            // helicity configurations whose tree amplitude vanishes
            // identically are never listed; the negated test also lists an
            // estimate that is not a number
            int neg = 0;
#pragma unroll
            for (int k = 0; k < N; ++k) neg += hel[(int64_t)k * E + e] < 0 ? 1 : 0;
            const double b2 = (double)bv * (double)bv;
            if (neg >= 2 && neg <= N - 2 && !(b2 <= (double)chk.tau * (ar * ar + ai * ai)))
              chk.list[atomicAdd(chk.count, 1u)] = (unsigned)e;
          }
          double scale = 1.0;
#pragma unroll
          for (int i = 0; i < N - 2; ++i) scale *= kGsOverSqrt2;
          ar *= scale;
          ai *= scale;
          me2[e] = ar * ar + ai * ai;
        } else {
          const T ip = sm.ip2[S];
          const int si = slot_index(sm.code[S], t);
          T* dj = sm.J + si * 8;
          T* dt = sm.Tt + si * 12;
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            dj[x] = gre[x] * ip;
            dj[4 + x] = gim[x] * ip;
          }
#pragma unroll
          for (int x = 0; x < 6; ++x) {
            dt[x] = tre[x];
            dt[6 + x] = tim[x];
          }
          if constexpr (EST) {
            sm.bJ[si] = bv * fabs(ip);
            sm.bT[si] = bt;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Persistent blocks of NL lanes, one valid event at a time from the
// compacted list.  EST: list ill-conditioned events into chk (FP32 pass).
template <int N, typename T, int NL, bool EST = false>
__global__ void __launch_bounds__(NL) cdbg_event_kernel(int64_t E, const double* __restrict__ mom,
                                                       const int8_t* __restrict__ hel,
                                                       const int8_t* __restrict__ col,
                                                       const unsigned* __restrict__ list,
                                                       const unsigned* __restrict__ count,
                                                       unsigned* __restrict__ work,
                                                       double* __restrict__ me2,
                                                       DressedCheck chk) {
  extern __shared__ __align__(16) unsigned char bg_cdbg_lds[];
  Sm<N, T> sm = carve<N, T, EST>(bg_cdbg_lds);
  const int lane = threadIdx.x;
  const unsigned total = *count;
  for (;;) {
    if (lane == 0) sm.misc[12] = (int)atomicAdd(work, 1u);
    __syncthreads();
    const unsigned idx = (unsigned)sm.misc[12];
    __syncthreads();  // every lane has read the index before the next pop
    if (idx >= total) break;
    cdbg_one_event<N, T, NL, EST>(sm, E, mom, hel, col, (int64_t)list[idx], me2, chk);
  }
}

}  // namespace cdbgk
}  // namespace bg
