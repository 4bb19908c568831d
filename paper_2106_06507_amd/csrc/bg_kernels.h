// Internal launch interface between the C-ABI layer (bg_api.cpp) and the
// HIP kernels.  Launchers return 0 on success, -1 on a launch error and -2 for
// an unsupported size.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bg {

template <int K>
struct Factorial {
  static constexpr int64_t value = K * Factorial<K - 1>::value;
};
template <>
struct Factorial<0> {
  static constexpr int64_t value = 1;
};

inline int64_t factorial(int k) {
  int64_t r = 1;
  for (int i = 2; i <= k; ++i) r *= i;
  return r;
}

// Allocation-free entry point: size of the per-device static workspace
// (noalloc.hip) and its layout.  Words [0, 64) counters; from byte 256 the
// event lists (at most 2 x kNoallocMaxEvents words); from kNoallocBlockOffset
// the per-block scratch of the persistent n = 7 kernels.
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
constexpr int64_t kNoallocMaxEvents = (int64_t)1 << 22;
constexpr size_t kNoallocBlockOffset = (size_t)33 << 20;
// Device address of this device's copy of the array (device must be current).
int noalloc_scratch_address(void** out);

// p[0..n) = v on `stream` (a kernel, so it can be recorded into a graph).
int fill_u32(unsigned* p, int n, unsigned v, hipStream_t stream);
// bad[0] |= 1 when one of the nh bytes of hel is not +-1 or one of the nc
// bytes of col is not 0, 1 or 2 (either pointer may be null with size 0).
int validate_inputs(int64_t nh, const int8_t* hel, int64_t nc, const int8_t* col, unsigned* bad,
                    hipStream_t stream);

// Partial amplitudes amp [2][K][E] for one helicity per event.  hel may be
// null, in which case helicity configuration `hconf` is used for every event
// (bit n-1-i set means gluon i has helicity -1).
int cobg_amplitudes(int n, bool fp32, int64_t E, const double* mom, const int8_t* hel, int hconf,
                    double* amp, hipStream_t stream);
// The same for events e0 .. e0 + count - 1 only, into amp [2][K][count].
// n in [4, 8].
int cobg_amplitudes_range(int n, bool fp32, int64_t E, int64_t e0, int64_t count,
                          const double* mom, const int8_t* hel, int hconf, double* amp,
                          hipStream_t stream);

// Helicity-summed colour-ordered |M|^2 in FP64 for n = 4..6 (hsum.hip): one
// block per (32-event tile, configuration), part [2^n][2][E] doubles of
// workspace, then the per-event sums; the fused kernel's bits.
int cobg_hsum_split(int n, int64_t E, const double* mom, const double* Cb, double* part,
                    double* me2, hipStream_t stream);

// Gradient of sum_st C_st Re(A_s conj(A_t)) scaled by gme2[e] (null = 1),
// given Y = C A [2][K][E]; perms [K][n-2] lists the middle gluons of each
// ordering; grad [n][4][E].
int cobg_gradient(int n, bool fp32, int64_t E, const double* mom, const int8_t* hel,
                  const double* Y, const double* gme2, const uint8_t* perms, double* grad,
                  hipStream_t stream);

// Y = C A [2][K][E] and me2 = Re sum A^* Y (FP64, one event per lane).
int contract_y(int K, int64_t E, const double* amp, const double* C, double* Y, double* me2,
               hipStream_t stream);

// me2[e] (+)= sum_st C_st Re(A_s conj(A_t)); C is K x K row-major on device.
int contract_valu(int K, int64_t E, const double* amp, const double* C, double* me2,
                  int accumulate, hipStream_t stream);
int mfma_probe(double* out_dev, hipStream_t stream);
// Colour sum with the colour matrix stored as its first row (n = 8, K = 720;
// full_colour.hip): row0 [K] (FP32, exact integers), labels [K][n-2] (the
// middle gluons of each ordering, 1..n-2), pos [K][n-2] (pos[s][x-1] = the
// position of label x in ordering s), part [relabel_row_blocks(n)][E]
// workspace; me2 (+)= x^T C x + y^T C y for amp [2][K][E].
int relabel_row_blocks(int n);
int relabel_contract(int n, int64_t E, const double* amp, const float* row0,
                     const unsigned char* labels, const unsigned char* pos, double* part,
                     double* me2, int accumulate, hipStream_t stream);

// Matrix-core contraction for K in {24, 120} (-2 otherwise); C is K x K
// row-major on device.
// idx non-null (listed form): column e is event idx[first + e], stored only
// for first + e < *cnt.
int contract_mfma(int K, int64_t E, const double* amp, const double* C, double* me2,
                  int accumulate, hipStream_t stream, const unsigned* idx = nullptr,
                  const unsigned* cnt = nullptr, int64_t first = 0);

// Check of an FP32 pass: events whose rounding-error estimate exceeds tau
// are appended to list (count must be zero before the pass; list holds E
// entries).
struct CheckArgs {
  float tau;
  unsigned* count;
  unsigned* list;
};

// Colour-dressed |A|^2 for one colour-flow assignment per event.  ws holds
// 4 + 2 E unsigned (counters, compacted list of valid events, list of events
// for the FP64 re-evaluation); grid is the number of persistent blocks
// (NL lanes each, one event at a time).  chk (FP32 only, may be null): list
// the ill-conditioned events and evaluate them again in FP64 on fix_grid
// blocks.
int cdbg_me2(int n, bool fp32, int64_t E, const double* mom, const int8_t* hel, const int8_t* col,
             unsigned* ws, double* me2, int grid, const CheckArgs* chk, int fix_grid,
             hipStream_t stream);
size_t cdbg_lds_bytes(int n, bool fp32);
int cdbg_blocks_per_cu(int n, bool fp32, bool chk);

// Fused colour-ordered |M|^2: recursion and colour sum in one kernel.  Cb is
// the colour matrix as doubled lower triangle in row blocks.  n <= 6: one
// block per 32-event tile (scratch, counter and grid unused).  n = 7:
// persistent grid of `grid` blocks over an atomic tile queue; scratch holds
// grid * cobg_fused_scratch_doubles(7) doubles, counter one unsigned.  chk
// (FP32 only, may be null): list the ill-conditioned events.
int cobg_fused_me2(int n, bool fp32, int64_t E, const double* mom, const int8_t* hel,
                   const double* Cb, double* scratch, unsigned* counter, int grid, double* me2,
                   const CheckArgs* chk, hipStream_t stream);
// FP64 re-evaluation of the *count events in list (persistent grid; scratch:
// grid * cobg_fused_scratch_doubles(n) doubles).
int cobg_fix_me2(int n, int64_t E, const double* mom, const int8_t* hel, const double* Cb,
                 double* scratch, const unsigned* count, const unsigned* list, int grid,
                 double* me2, hipStream_t stream);
int cobg_fix_blocks_per_cu(int n, bool hsum);
int cobg_fused_scratch_doubles(int n);
// Leading-colour |M|^2 over all (n-1)! orderings, one helicity per event.
// Leading colour; chk (FP32 only): list ill-conditioned events into
// chk->count / chk->list (count zeroed beforehand), then evaluate them again
// in FP64 on fix_grid persistent blocks.
int lc_me2(int n, bool fp32, int64_t E, const double* mom, const int8_t* hel, double* me2,
           const CheckArgs* chk, int fix_grid, hipStream_t stream);
int lc_fix_blocks_per_cu(int n);
int cobg_fused_persistent_blocks_per_cu(bool fp32, bool hsum, bool chk);
// LDS of a colour-ordered tile (recursion state plus staged amplitudes).
size_t cobg_lds_bytes(int n, bool fp32);

// Mixed-multiplicity batch.  kind = kBatchCobg + n or kBatchCdbg + n.
constexpr int kBatchCobg = 0;
constexpr int kBatchCdbg = 16;

struct BatchSeg {
  const double* mom;   // [n][4][E]
  const int8_t* hel;   // [n][E]
  const int8_t* col;   // [2][n][E] (colour-dressed only)
  double* me2;         // [E]
  const double* Cl;    // doubled lower-triangle colour matrix (colour-ordered only)
  const unsigned* idx; // re-evaluation pass: the tile's events are idx[first ..]
  unsigned* flist;     // checked FP32 pass: ill-conditioned events of the segment
  unsigned* fcount;    // checked FP32 pass: their number
  int64_t E;
  int kind;
  float tau;           // checked FP32 pass: threshold of the segment's mode and n
};

struct BatchTile {
  int64_t first;  // first event of the tile within its segment
  int seg;
  int count;      // events in the tile
};

constexpr int kBatchMaxSegs = 32;

// Passed by value as a kernel argument, so that a launch (or a recorded graph
// node) carries the caller's pointers without any device-side table.
struct BatchSegTable {
  BatchSeg s[kBatchMaxSegs];
};

// Batch blocks are 256 lanes.  LDS for a segment kind (kBatchCobg or
// kBatchCdbg, without n) and per-block scratch doubles for colour-ordered n;
// chk: the checked FP32 pass (the colour-dressed state carries its bounds).
size_t batch_lds_bytes(int kind, int n, bool fp32, bool chk = false);
int batch_scratch_doubles(int n);
// Pass of the batch kernel: plain, checked FP32 (lists ill-conditioned
// events per segment), or the FP64 re-evaluation of the listed events.
enum BatchPass { kBatchPlain = 0, kBatchCheck = 1, kBatchFix = 2 };
// Segment kinds a batch kernel instance evaluates: every kind, colour-ordered
// only, colour-dressed only (tiles of other kinds are skipped).
enum BatchKinds { kBatchKindsAll = 0, kBatchKindsCobg = 1, kBatchKindsCdbg = 2 };
// waves: register budget variant, 1 (one wave per SIMD, no cap) or 2 (at
// most 256 registers per lane; the only variant of the dressed-only kernel).
int batch_blocks_per_cu(bool fp32, int waves, int pass, int kinds, size_t lds);
// Enqueues the counter reset and the persistent kernel on stream over the
// tiles [t_begin, t_end), or [range_dev[0], range_dev[1]) read on the device
// when range_dev is given.
int batch_launch(bool fp32, int waves, int pass, int kinds, const BatchSegTable& segs,
                 const BatchTile* tiles, unsigned t_begin, unsigned t_end,
                 const unsigned* range_dev, unsigned* counter, double* scratch,
                 int64_t scratch_stride, int grid, size_t lds, hipStream_t stream);
// Per-kinds instances (batch_kinds_*.hip).
template <int KINDS>
int batch_occupancy_kinds(bool fp32, int waves, int pass, size_t lds);
template <int KINDS>
void batch_launch_kinds(bool fp32, int waves, int pass, const BatchSegTable& segs,
                        const BatchTile* tiles, unsigned t_begin, unsigned t_end,
                        const unsigned* range_dev, unsigned* counter, double* scratch,
                        int64_t scratch_stride, int grid, size_t lds, hipStream_t stream);
// Tiles of the re-evaluation pass from the per-segment counts fcount[s] of
// listed events: colour-dressed tiles of one listed event (queued first),
// colour-ordered tiles of up to 128; tiles[] and range[0..5] on the device:
// the dressed tiles, the colour-ordered tiles, all tiles (begin, end each).
int batch_fix_tiles(const BatchSegTable& segs, int n_segs, const unsigned* fcount,
                    BatchTile* tiles, unsigned* range, hipStream_t stream);

// Colour-sampled colour-ordered |A|^2 (comc.hip).  count: counts, offsets
// and the valid-event list [E] each, block_items and block_valid
// [ceil(E/256) + 1] (exclusive offsets, totals last; the item total must be
// below 2^31 before items runs); items: items [total] for the n_valid
// listed events; amplitudes: amp [2 total] (persistent grid); reduce.
int comc_count(int n, int64_t E, const int8_t* col, double* me2, unsigned* counts,
               unsigned* offsets, unsigned* valid, uint64_t* block_items, uint64_t* block_valid,
               hipStream_t stream);
int comc_items(int n, int64_t E, const int8_t* col, const unsigned* valid, unsigned n_valid,
               const unsigned* counts, const unsigned* offsets, uint64_t* items,
               hipStream_t stream);
int comc_amplitudes(int n, bool fp32, int64_t E, const double* mom, const int8_t* hel,
                    const uint64_t* items, const uint64_t* total, double* amp, float* bnd,
                    int grid, hipStream_t stream);
int comc_reduce(const unsigned* valid, unsigned n_valid, const unsigned* counts,
                const unsigned* offsets, const double* amp, double* me2, hipStream_t stream);
// FP64 colour-ordered amplitudes for n = 7, 8 with one straight path per
// ordering (comc.hip, cobg_path_impl.h): amp [2][K][count] as
// cobg_amplitudes_range.  idx non-null: column j is event idx[e0 + j] for
// e0 + j < *cnt (listed events; other columns untouched).  osplit (n = 7):
// blocks per 32 events, each taking a contiguous range of the orderings
// (divides 120).
int cobg_path_amplitudes(int n, int64_t E, int64_t e0, int64_t count, const double* mom,
                         const int8_t* hel, int hconf, double* amp, const unsigned* idx,
                         const unsigned* cnt, hipStream_t stream, int osplit = 1);
// FP32 check (bnd from comc_amplitudes with fp32 and bnd non-null): events
// with B^2 > tau |A|^2 are appended to flist (count fcount[0]) and their
// items to sel (count fcount[1]; both zeroed beforehand); then the listed
// items again in FP64 and the listed events reduced again (max_listed: an
// upper bound on fcount[0] that sizes the grid).
int comc_reduce_check(int n, int64_t E, const int8_t* hel, const unsigned* valid, unsigned n_valid,
                      const unsigned* counts, const unsigned* offsets, const double* amp,
                      const float* bnd, double* me2, float tau, unsigned* fcount, unsigned* flist,
                      unsigned* sel, hipStream_t stream);
int comc_amplitudes_listed(int n, int64_t E, const double* mom, const int8_t* hel,
                           const uint64_t* items, const unsigned* sel, const unsigned* sel_count,
                           double* amp, int grid, hipStream_t stream);
int comc_reduce_listed(const unsigned* flist, const unsigned* fcount, unsigned max_listed,
                       const unsigned* counts, const unsigned* offsets, const double* amp,
                       double* me2, hipStream_t stream);

// Continuous colour / real-polarization sampling with the dressed recursion
// (cdmc.hip).  gstate: blocks x cdmc_state_bytes when cdmc_global_state.
size_t cdmc_state_bytes(int n, bool fp32);
bool cdmc_global_state(int n, bool fp32);
int cdmc_blocks_per_cu(int n, bool fp32);
int cdmc_me2(int n, bool fp32, int64_t E, const double* mom, const double* phi, const double* eta,
             void* gstate, int grid, double* me2, hipStream_t stream);

// Continuous colour / polarization variables on the device (rambo.hip).
int generate_continuous(int n, uint64_t seed, uint64_t first, int64_t E, double* phi, double* eta,
                        hipStream_t stream);

// On-device phase-space generation (rambo.hip).
struct GenParams {
  int n;
  int cuts;
  double sqrt_s, pt_min, dr_min;
  uint64_t seed, first_attempt;
};
size_t generate_workspace_words(int64_t n_attempts);
// Attempts [first_attempt, first_attempt + n_attempts): accepted ones, in
// attempt order, written at ranks < max_events (arrays of stride
// max_events); *n_out (device) = min(accepted, max_events).  hel, col and
// attempt may be null.
int generate_events(const GenParams& gp, int64_t n_attempts, int64_t max_events, unsigned* ws,
                    double* mom, int8_t* hel, int8_t* col, int64_t* attempt, int64_t* n_out,
                    hipStream_t stream);

}  // namespace bg
