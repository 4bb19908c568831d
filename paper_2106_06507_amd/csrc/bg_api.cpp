// C-ABI layer: argument validation, context (colour matrices, workspace) and
// dispatch to the HIP kernels.  See include/bg.h for the contract.
#include "bg.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "bg_kernels.h"

namespace bg {
int64_t colour_matrix(int n, double* C);
int64_t colour_matrix_row0(int n, double* row);
}

namespace {

// Cached tile table of one batch shape (segment kinds and sizes, precision,
// config).
struct BatchPlan {
  std::vector<int64_t> key;
  bg::BatchTile* tiles = nullptr;
  unsigned n_tiles = 0;
  unsigned n_tiles_cobg = 0;  // split plans: colour-ordered tiles first, then the dressed ones
  uint64_t last_use = 0;
  // FP32 plans: workspace of the check and of the FP64 re-evaluation pass:
  // words [0, 32) listed-event counts per segment, words [32, 38) the
  // re-evaluation tile ranges (dressed, colour-ordered, all), from word 64
  // the per-segment lists (list_off), then the re-evaluation tiles (at most
  // max_fix_cd dressed ones, then at most max_fix_co colour-ordered ones).
  unsigned* chk_ws = nullptr;
  std::vector<size_t> list_off;
  bg::BatchTile* fix_tiles = nullptr;
  unsigned max_fix_cd = 0, max_fix_co = 0;
};

void free_plan(BatchPlan& pl) {
  if (pl.tiles) (void)hipFree(pl.tiles);
  if (pl.chk_ws) (void)hipFree(pl.chk_ws);
  pl.tiles = nullptr;
  pl.chk_ws = nullptr;
}

}  // namespace

struct bg_context {
  int device = 0;
  int num_cus = 0;
  size_t lds_per_cu = 0;
  size_t lds_per_block = 0;
  unsigned* cws = nullptr;                   // colour-dressed workspace (counters + event list)
  size_t cws_bytes = 0;
  double* C_dev[BG_N_MAX + 1] = {};          // K x K colour matrix per n (lazy)
  double* Cb_dev[BG_N_MAX + 1] = {};         // doubled lower triangle in row blocks (fused path)
  float* row0_dev[BG_N_MAX + 1] = {};        // n = 8: row 0 of C (relabelled storage)
  unsigned char* labels_dev[BG_N_MAX + 1] = {};  // n = 8: [K][n-2] middle gluons per ordering
  unsigned char* pos_dev[BG_N_MAX + 1] = {};     // n = 8: [K][n-2] position of each label
  double* ws = nullptr;                      // workspace (partial amplitudes)
  size_t ws_bytes = 0;
  double* part = nullptr;                    // n = 8 colour sum: per-row-block partial sums
  size_t part_bytes = 0;
  uint8_t* perms_dev[BG_N_MAX + 1] = {};     // [K][n-2] middle gluons of each ordering (gradient)
  double* scratch = nullptr;                 // per-block scratch of the fused and batch kernels
  size_t scratch_bytes = 0;
  std::vector<void*> retired;                // outgrown scratch buffers, freed on destroy
  unsigned* counter = nullptr;               // tile-queue heads: [0] batch, [1] fused n = 7
  unsigned* gen_ws = nullptr;                // phase-space generator: acceptance bits, counts
  size_t gen_ws_words = 0;
  uint64_t* comc_ws = nullptr;               // colour-sampled COBG: block offsets, counts, offsets
  size_t comc_ws_words = 0;
  uint64_t* comc_items = nullptr;            // (event, ordering) items
  double* comc_amp = nullptr;                // their amplitudes
  float* comc_bnd = nullptr;                 // their FP32 error bounds (checked FP32)
  unsigned* comc_sel = nullptr;              // items listed for FP64 re-evaluation
  size_t comc_cap = 0;
  void* cdmc_state = nullptr;                // per-block state slabs (FP64, n = 9)
  size_t cdmc_state_bytes = 0;
  int occ_cdmc[BG_N_MAX + 1][2] = {};
  bg_batch_config bcfg[2] = {{0, 128, 256, 2, 1}, {0, 128, 256, 2, 1}};
  std::vector<BatchPlan> plans;
  uint64_t clock = 0;
  int occ_fused[2][2][2] = {};               // blocks per CU of the persistent fused kernel
                                             // [fp32][helicity sum][checked], 0 = unknown
  int occ_batch[3][4][2] = {};               // of the batch kernel [kinds][fp32 * 2 + (pass != plain)][waves - 1]
                                             // [variant] at its last LDS size
  int occ_cdbg[BG_N_MAX + 1][2] = {};        // of the colour-dressed event kernel
  size_t occ_batch_lds[3][4][2] = {};
  uint32_t flags = 0;                        // BG_FLAG_* applied to every request
  float fp32_tau[4][BG_N_MAX + 1] = {};      // FP32 check thresholds [COBG, CDBG, COMC, LC][n]
  int occ_lc_fix[BG_N_MAX + 1] = {};         // of the FP64 leading-colour re-evaluation
  unsigned* flag_ws = nullptr;               // FP32 check: [0] count, list from word 64
  size_t flag_ws_words = 0;
  int occ_fix[BG_N_MAX + 1][2] = {};         // blocks per CU of the FP64 re-evaluation [n][hsum]
  int occ_cdbg_chk[BG_N_MAX + 1] = {};       // of the checked FP32 colour-dressed event kernel
  unsigned* val_dev = nullptr;               // BG_FLAG_VALIDATE result word
  unsigned char* noalloc = nullptr;          // this device's static workspace (bg_me2_noalloc)
  hipEvent_t ws_event = nullptr;             // recorded after each call that uses the workspace
  hipStream_t ws_stream = nullptr;           // stream of that call
  bool ws_pending = false;
  // batch: side stream of the concurrent per-kind launches, fork/join events
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
};

namespace {

bool log_enabled() {
  static int v = -1;
  if (v < 0) {
    const char* s = getenv("BG_LOG");
    v = (s && s[0] && s[0] != '0') ? 1 : 0;
  }
  return v == 1;
}

#define BG_LOG(...)                         \
  do {                                      \
    if (log_enabled()) {                    \
      fprintf(stderr, "[bg] " __VA_ARGS__); \
      fputc('\n', stderr);                  \
    }                                       \
  } while (0)

int hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return BG_OK;
  BG_LOG("%s failed: %s", what, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? BG_ENOMEM : BG_EDEVICE;
}

int launch_status(int r) {
  if (r == 0) return BG_OK;
  if (r == -2) return BG_EUNSUPPORTED;
  return BG_EDEVICE;
}

// Make the context's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Symmetric C as its doubled lower triangle, row blocks of RB rows: for each
// block and each column j below the block's end, the RB entries of the block's
// rows are contiguous (the layout the fused colour sum reads).
std::vector<double> row_blocked_lower(const std::vector<double>& C, int K) {
  const int RB = K < 8 ? K : 8;
  std::vector<double> out;
  for (int ib = 0; ib < K; ib += RB)
    for (int j = 0; j < ib + RB; ++j)
      for (int r = 0; r < RB; ++r) {
        const int i = ib + r;
        const double c = C[(size_t)i * K + j];
        out.push_back(j < i ? 2.0 * c : (j == i ? c : 0.0));
      }
  return out;
}

int upload(const std::vector<double>& v, double** out, const char* what) {
  double* d = nullptr;
  int st = hip_status(hipMalloc(&d, sizeof(double) * v.size()), what);
  if (st) return st;
  st = hip_status(hipMemcpy(d, v.data(), sizeof(double) * v.size(), hipMemcpyHostToDevice), what);
  if (st) {
    (void)hipFree(d);
    return st;
  }
  *out = d;
  return BG_OK;
}

int ensure_colour(bg_context* ctx, int n) {
  if (ctx->C_dev[n]) return BG_OK;
  const int64_t K = bg::factorial(n - 2);
  std::vector<double> C((size_t)(K * K));
  bg::colour_matrix(n, C.data());
  if (!ctx->Cb_dev[n]) {
    int st = upload(row_blocked_lower(C, (int)K), &ctx->Cb_dev[n], "colour matrix (row blocks)");
    if (st) return st;
  }
  int st = upload(C, &ctx->C_dev[n], "colour matrix");
  if (st) return st;
  BG_LOG("colour matrix n=%d K=%lld uploaded", n, (long long)K);
  return BG_OK;
}

// Per-row-block partial sums of the n = 8 colour sum (grown with a device
// synchronisation, like the other workspaces).
int ensure_part(bg_context* ctx, int64_t E) {
  const size_t bytes = sizeof(double) * (size_t)bg::relabel_row_blocks(8) * (size_t)E;
  if (ctx->part_bytes >= bytes) return BG_OK;
  if (ctx->part) {
    int st = hip_status(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (st) return st;
    (void)hipFree(ctx->part);
    ctx->part = nullptr;
    ctx->part_bytes = 0;
  }
  int st = hip_status(hipMalloc(&ctx->part, bytes), "hipMalloc(colour sum partials)");
  if (st) return st;
  ctx->part_bytes = bytes;
  return BG_OK;
}

// Relabelled storage of C(n) for n = 8 (K = 720): row 0 and the orderings
// (labels and, per ordering, the position of each label), K (1 + 2 (n-2))
// numbers instead of K^2.
int ensure_relabel(bg_context* ctx, int n) {
  if (ctx->row0_dev[n]) return BG_OK;
  const int k = n - 2;
  const int64_t K = bg::factorial(k);
  std::vector<double> row((size_t)K);
  bg::colour_matrix_row0(n, row.data());
  std::vector<float> rowf(row.begin(), row.end());  // integers below 2^24: exact
  std::vector<unsigned char> labels((size_t)(K * k)), pos((size_t)(K * k));
  std::vector<int> p(k);
  for (int i = 0; i < k; ++i) p[i] = i + 1;
  for (int64_t s = 0; s < K; ++s) {
    for (int i = 0; i < k; ++i) {
      labels[(size_t)(s * k + i)] = (unsigned char)p[i];
      pos[(size_t)(s * k + p[i] - 1)] = (unsigned char)i;
    }
    std::next_permutation(p.begin(), p.end());
  }
  float* r = nullptr;
  unsigned char* lb = nullptr;
  unsigned char* ps = nullptr;
  int st = hip_status(hipMalloc(&r, sizeof(float) * K), "hipMalloc(row0)");
  if (!st) st = hip_status(hipMalloc(&lb, labels.size()), "hipMalloc(labels)");
  if (!st) st = hip_status(hipMalloc(&ps, pos.size()), "hipMalloc(positions)");
  if (!st) st = hip_status(hipMemcpy(r, rowf.data(), sizeof(float) * K, hipMemcpyHostToDevice),
                           "hipMemcpy(row0)");
  if (!st) st = hip_status(hipMemcpy(lb, labels.data(), labels.size(), hipMemcpyHostToDevice),
                           "hipMemcpy(labels)");
  if (!st) st = hip_status(hipMemcpy(ps, pos.data(), pos.size(), hipMemcpyHostToDevice),
                           "hipMemcpy(positions)");
  if (st) {
    if (r) (void)hipFree(r);
    if (lb) (void)hipFree(lb);
    if (ps) (void)hipFree(ps);
    return st;
  }
  ctx->row0_dev[n] = r;
  ctx->labels_dev[n] = lb;
  ctx->pos_dev[n] = ps;
  return BG_OK;
}

int ensure_ws(bg_context* ctx, size_t bytes) {
  if (ctx->ws_bytes >= bytes) return BG_OK;
  if (ctx->ws) {
    // the previous workspace may still be read by queued kernels
    int st = hip_status(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (st) return st;
    (void)hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  int st = hip_status(hipMalloc(&ctx->ws, bytes), "hipMalloc(workspace)");
  if (st) return st;
  ctx->ws_bytes = bytes;
  return BG_OK;
}

bool valid_n(int n) { return n >= BG_N_MIN && n <= BG_N_MAX; }

// Default FP32 check thresholds on est = sum S^2 / sum |A|^2 per n (the bound
// S grows with the number of terms, so the threshold grows with n), measured
// on 2^20 (n = 7: 2^18) sampled-helicity RAMBO events against the FP64 path.
// Colour-ordered:
//   n = 5: tau 3e5 lists 12% of the events, per-event error p99 6.8e-6;
//   n = 6: tau 3e6 lists 17%, p99 5.9e-6;
//   n = 7: tau 1e8 lists 15%, p99 6.9e-6;
//   n = 4 is not checked: without the check its largest per-event error over
//   2^20 events is 1.3e-6.
// Colour-dressed, on the valid flows of 2^20 sampled-flow events (sampled
// helicities), interpolating a sweep in decades of tau:
//   n = 4: tau 1e8 lists 0.6% (p99 2.1e-6: already small without the check);
//   n = 5: 3e5, ~17% (p99 ~7e-6);  n = 6: 2e6, ~27% (~6e-6);
//   n = 7: 3e7, ~35% (~7e-6);      n = 8: 3e8, ~44% (~6e-6);
//   n = 9: 5e9, ~48% (~6e-6).
// The dressed bound is looser than the colour-ordered one (many more terms
// per current), so larger fractions are listed.
// Colour-sampled colour-ordered, same flows (the flow amplitude sums a few
// orderings that cancel: p99 without the check 3e-4 .. 7e-4 for n >= 5):
//   n = 4: 1e6 (p99 2.1e-6, max 2.7e-5; without: max 5.4e-4);
//   n = 5: 1e5, ~20% re-evaluated (5.9e-6);  n = 6: 1e6, ~28% (6.8e-6);
//   n = 7: 1e7, ~35% (7.3e-6);  n = 8: 1e8, ~42% (7.0e-6);
//   n = 9: 1e9, ~51% (6.1e-6).
// Leading colour (2^18 events, n = 7: 2^15):
//   n = 4 is not checked (largest error 7.5e-7);  n = 5: 1e6, ~9% (6.0e-6);
//   n = 6: 3e7, ~10% (6.2e-6);  n = 7: 1e9, ~9% (6.1e-6).
constexpr float kDefaultFp32Tau[4][BG_N_MAX + 1] = {
    {0.f, 0.f, 0.f, 0.f, INFINITY, 3e5f, 3e6f, 1e8f, 0.f, 0.f},
    {0.f, 0.f, 0.f, 0.f, 1e8f, 3e5f, 2e6f, 3e7f, 3e8f, 5e9f},
    {0.f, 0.f, 0.f, 0.f, 1e6f, 1e5f, 1e6f, 1e7f, 1e8f, 1e9f},
    {0.f, 0.f, 0.f, 0.f, INFINITY, 1e6f, 3e7f, 1e9f, 0.f, 0.f}};

// Grows the per-block scratch.  An outgrown buffer is kept until the context
// is destroyed, since a recorded graph may still refer to it.
int ensure_scratch(bg_context* ctx, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (ctx->scratch_bytes >= bytes) return BG_OK;
  size_t want = std::max(bytes, 2 * ctx->scratch_bytes);
  double* d = nullptr;
  int st = hip_status(hipMalloc(&d, want), "hipMalloc(scratch)");
  if (st) return st;
  if (ctx->scratch) ctx->retired.push_back(ctx->scratch);
  ctx->scratch = d;
  ctx->scratch_bytes = want;
  return BG_OK;
}

// Workspace of one call when it must not allocate (bg_me2_noalloc): views
// into the per-device static array of noalloc.hip (layout in bg_kernels.h).
struct FixedWs {
  unsigned* flag_ws;     // check: count at word 0, list from word kFlagListOffset
  unsigned* counter;     // [0] batch queue (unused), [1] n = 7 tile queue
  unsigned* cws;         // colour-dressed counters and lists
  unsigned* val;         // BG_FLAG_VALIDATE result word
  double* scratch;       // per-block scratch (n = 7)
  size_t scratch_bytes;
};

FixedWs fixed_ws(unsigned char* base) {
  FixedWs w;
  unsigned* words = reinterpret_cast<unsigned*>(base);
  w.counter = words + 32;
  w.val = words + 48;
  w.flag_ws = words + 64;  // its list starts 64 words further: within the list region
  w.cws = words + 64;
  w.scratch = reinterpret_cast<double*>(base + bg::kNoallocBlockOffset);
  w.scratch_bytes = bg::kNoallocScratchBytes - bg::kNoallocBlockOffset;
  return w;
}

// FP32 check workspace: a count word and a list of up to E event indices.
constexpr size_t kFlagListOffset = 64;  // words: the list starts 256 bytes in
int ensure_flags(bg_context* ctx, int64_t E) {
  const size_t words = kFlagListOffset + (size_t)E;
  if (ctx->flag_ws_words >= words) return BG_OK;
  if (ctx->flag_ws) {
    int st = hip_status(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (st) return st;
    (void)hipFree(ctx->flag_ws);
    ctx->flag_ws = nullptr;
    ctx->flag_ws_words = 0;
  }
  const size_t want = std::max(words, (size_t)1024);
  int st = hip_status(hipMalloc(&ctx->flag_ws, sizeof(unsigned) * want), "hipMalloc(check list)");
  if (st) return st;
  ctx->flag_ws_words = want;
  return BG_OK;
}

bool capturing_stream(hipStream_t stream) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return false;
  return cs == hipStreamCaptureStatusActive;
}

// Orders calls that share the context workspace across streams: a call on a
// stream other than the previous call's waits for the event recorded after
// that call.  Skipped while the stream captures (a graph cannot wait on an
// event recorded outside it; replays are ordered by the caller).
int ws_acquire(bg_context* ctx, hipStream_t stream) {
  if (!ctx->ws_pending || ctx->ws_stream == stream || capturing_stream(stream)) return BG_OK;
  return hip_status(hipStreamWaitEvent(stream, ctx->ws_event, 0), "hipStreamWaitEvent");
}

int ws_release(bg_context* ctx, hipStream_t stream, int status) {
  if (status != BG_OK || capturing_stream(stream)) return status;
  int st = hip_status(hipEventRecord(ctx->ws_event, stream), "hipEventRecord");
  if (st) return st;
  ctx->ws_stream = stream;
  ctx->ws_pending = true;
  return BG_OK;
}

// BG_FLAG_VALIDATE: every hel entry +-1, every col entry in {0, 1, 2}.
// fixed: the result word of the static workspace instead of a context buffer.
int validate_values(bg_context* ctx, int n, int64_t E, const int8_t* hel, const int8_t* col,
                    hipStream_t stream, const FixedWs* fixed = nullptr) {
  if (capturing_stream(stream)) return BG_EINVAL;
  unsigned* word = fixed ? fixed->val : ctx->val_dev;
  if (!word) {
    int st = hip_status(hipMalloc(&ctx->val_dev, 256), "hipMalloc(validate)");
    if (st) return st;
    word = ctx->val_dev;
  }
  int st = launch_status(bg::fill_u32(word, 1, 0u, stream));
  if (!st)
    st = launch_status(bg::validate_inputs(hel ? (int64_t)n * E : 0, hel,
                                           col ? (int64_t)2 * n * E : 0, col, word, stream));
  unsigned bad = 0;
  if (!st)
    st = hip_status(hipMemcpyAsync(&bad, word, sizeof(unsigned), hipMemcpyDeviceToHost,
                                   stream), "hipMemcpyAsync(validate)");
  if (!st) st = hip_status(hipStreamSynchronize(stream), "hipStreamSynchronize");
  if (st) return st;
  return bad ? BG_EINVAL : BG_OK;
}

int grad_run(bg_context* ctx, const bg_request* r, const double* grad_me2, double* grad_mom,
             hipStream_t s);

// Device address of each device's copy of the static workspace of
// bg_me2_noalloc, looked up once per device (with that device current).
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
unsigned char* g_noalloc_ptr[kMaxDevices] = {};

int noalloc_address(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return BG_ENODEV;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    void* p = nullptr;
    if (bg::noalloc_scratch_address(&p) != 0) {
      BG_LOG("hipGetSymbolAddress of the static workspace failed on device %d", device);
      return BG_EDEVICE;
    }
    g_noalloc_ptr[device] = static_cast<unsigned char*>(p);
  }
  *out = g_noalloc_ptr[device];
  return BG_OK;
}

// Lexicographic orderings of the middle gluons 1..n-2, as bytes [K][n-2].
int ensure_perms(bg_context* ctx, int n) {
  if (ctx->perms_dev[n]) return BG_OK;
  const int k = n - 2;
  const int64_t K = bg::factorial(k);
  std::vector<uint8_t> tab((size_t)(K * k));
  std::vector<int> p(k);
  for (int i = 0; i < k; ++i) p[i] = i + 1;
  for (int64_t s = 0; s < K; ++s) {
    for (int i = 0; i < k; ++i) tab[(size_t)(s * k + i)] = (uint8_t)p[i];
    // next lexicographic permutation
    int i = k - 2;
    while (i >= 0 && p[i] > p[i + 1]) --i;
    if (i < 0) break;
    int j = k - 1;
    while (p[j] < p[i]) --j;
    std::swap(p[i], p[j]);
    for (int a = i + 1, b = k - 1; a < b; ++a, --b) std::swap(p[a], p[b]);
  }
  uint8_t* d = nullptr;
  int st = hip_status(hipMalloc(&d, tab.size()), "hipMalloc(perms)");
  if (st) return st;
  st = hip_status(hipMemcpy(d, tab.data(), tab.size(), hipMemcpyHostToDevice), "hipMemcpy(perms)");
  if (st) {
    (void)hipFree(d);
    return st;
  }
  ctx->perms_dev[n] = d;
  return BG_OK;
}

int check_events(int n, int64_t E) {
  if (E < 0) return BG_EINVAL;
  // [n][4][E] doubles must be addressable
  if (E > ((int64_t)1 << 40) / (4 * n)) return BG_ERANGE;
  return BG_OK;
}

// part: workspace of relabel_row_blocks(8) x E doubles for n = 8 (may be null
// for n <= 7).
int contract_dispatch(bg_context* ctx, int n, int64_t E, const double* amp, double* me2,
                      int accumulate, hipStream_t stream, double* part = nullptr) {
  if (n == 8) {
    int st = ensure_relabel(ctx, n);
    if (st) return st;
    return launch_status(bg::relabel_contract(n, E, amp, ctx->row0_dev[n], ctx->labels_dev[n],
                                              ctx->pos_dev[n], part, me2, accumulate, stream));
  }
  int st = ensure_colour(ctx, n);
  if (st) return st;
  const int K = (int)bg::factorial(n - 2);
  if (K == 24 || K == 120)
    return launch_status(bg::contract_mfma(K, E, amp, ctx->C_dev[n], me2, accumulate, stream));
  return launch_status(bg::contract_valu(K, E, amp, ctx->C_dev[n], me2, accumulate, stream));
}

// Colour-ordered amplitudes [2][K][count] of events e0 .. e0 + count - 1:
// the depth-first walk with shared prefixes, except FP64 at n >= 7, where
// one straight path per ordering avoids the walk's register spills.
int amplitudes_dispatch(bg_context* ctx, int n, bool fp32, int64_t E, int64_t e0, int64_t count,
                        const double* mom, const int8_t* hel, int hconf, double* amp,
                        hipStream_t stream) {
  if (!fp32 && n >= 7)
    return launch_status(bg::cobg_path_amplitudes(n, E, e0, count, mom, hel, hconf, amp, nullptr,
                                                  nullptr, stream));
  return launch_status(bg::cobg_amplitudes_range(n, fp32, E, e0, count, mom, hel, hconf, amp,
                                                 stream));
}

// Events per chunk of the two-stage colour-ordered path at n = 8 (amplitudes
// 11.5 KB per event in FP64 through the context workspace).
constexpr int64_t kN8Chunk = (int64_t)1 << 17;  // events per two-stage n = 8 chunk (1.5 GB of amplitudes)
constexpr int64_t kN7Chunk = (int64_t)1 << 18;  // n = 7: 0.5 GB

}  // namespace

extern "C" {

const char* bg_status_string(int status) {
  switch (status) {
    case BG_OK: return "ok";
    case BG_EINVAL: return "invalid argument";
    case BG_ERANGE: return "size out of range";
    case BG_ENODEV: return "no usable gfx950 device";
    case BG_EDEVICE: return "HIP runtime error";
    case BG_ENOMEM: return "device out of memory";
    case BG_EUNSUPPORTED: return "unsupported request";
    default: return "unknown status";
  }
}

int64_t bg_num_orderings(int n) { return valid_n(n) ? bg::factorial(n - 2) : 0; }

int bg_color_matrix(int n, double* out, int64_t cap) {
  if (!out || n < 4 || n > 8) return BG_EINVAL;
  const int64_t K = bg::factorial(n - 2);
  if (cap < K * K) return BG_ERANGE;
  bg::colour_matrix(n, out);
  return BG_OK;
}

int bg_context_create(bg_context** out, int device, uint32_t flags) {
  if (!out) return BG_EINVAL;
  if (flags & ~(BG_FLAG_VALIDATE | BG_FLAG_FP32_UNCHECKED)) return BG_EINVAL;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return BG_ENODEV;
  if (device < 0 || device >= count) return BG_ENODEV;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return BG_ENODEV;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    BG_LOG("device %d is %s, not gfx950", device, prop.gcnArchName);
    return BG_ENODEV;
  }
  bg_context* ctx = new (std::nothrow) bg_context();
  if (!ctx) return BG_ENOMEM;
  ctx->device = device;
  ctx->num_cus = prop.multiProcessorCount;
  ctx->lds_per_cu = prop.maxSharedMemoryPerMultiProcessor;
  ctx->lds_per_block = prop.sharedMemPerBlock;
  ctx->flags = flags;
  for (int m = 0; m < 4; ++m)
    for (int n = 0; n <= BG_N_MAX; ++n) ctx->fp32_tau[m][n] = kDefaultFp32Tau[m][n];
  {
    DeviceGuard g(device);
    if (!g.ok || hipEventCreateWithFlags(&ctx->ws_event, hipEventDisableTiming) != hipSuccess) {
      delete ctx;
      return BG_EDEVICE;
    }
    int st = noalloc_address(device, &ctx->noalloc);
    // the colour matrices of the colour-ordered path, so that bg_me2_noalloc
    // never has to upload one
    for (int n = 4; n <= 7 && !st; ++n) st = ensure_colour(ctx, n);
    if (st) {
      bg_context_destroy(ctx);
      return st;
    }
  }
  *out = ctx;
  return BG_OK;
}

void bg_context_destroy(bg_context* ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  (void)hipDeviceSynchronize();
  for (int n = 0; n <= BG_N_MAX; ++n) {
    if (ctx->C_dev[n]) (void)hipFree(ctx->C_dev[n]);
    if (ctx->Cb_dev[n]) (void)hipFree(ctx->Cb_dev[n]);
    if (ctx->row0_dev[n]) (void)hipFree(ctx->row0_dev[n]);
    if (ctx->labels_dev[n]) (void)hipFree(ctx->labels_dev[n]);
    if (ctx->pos_dev[n]) (void)hipFree(ctx->pos_dev[n]);
    if (ctx->perms_dev[n]) (void)hipFree(ctx->perms_dev[n]);
  }
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->part) (void)hipFree(ctx->part);
  if (ctx->cws) (void)hipFree(ctx->cws);
  if (ctx->scratch) (void)hipFree(ctx->scratch);
  for (void* p : ctx->retired) (void)hipFree(p);
  if (ctx->gen_ws) (void)hipFree(ctx->gen_ws);
  if (ctx->comc_ws) (void)hipFree(ctx->comc_ws);
  if (ctx->comc_items) (void)hipFree(ctx->comc_items);
  if (ctx->comc_amp) (void)hipFree(ctx->comc_amp);
  if (ctx->comc_bnd) (void)hipFree(ctx->comc_bnd);
  if (ctx->comc_sel) (void)hipFree(ctx->comc_sel);
  if (ctx->cdmc_state) (void)hipFree(ctx->cdmc_state);
  if (ctx->counter) (void)hipFree(ctx->counter);
  if (ctx->flag_ws) (void)hipFree(ctx->flag_ws);
  if (ctx->val_dev) (void)hipFree(ctx->val_dev);
  if (ctx->ws_event) (void)hipEventDestroy(ctx->ws_event);
  if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
  if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  for (BatchPlan& pl : ctx->plans) free_plan(pl);
  delete ctx;
}

int bg_currents(bg_context* ctx, int n, int64_t E, const double* mom, const int8_t* hel,
                int precision, double* amp, void* stream) {
  if (!ctx || n < 4 || n > 8) return n > 8 && n <= BG_N_MAX ? BG_EUNSUPPORTED : BG_EINVAL;
  int st = check_events(n, E);
  if (st) return st;
  if (precision != BG_PREC_FP64 && precision != BG_PREC_FP32_MIXED) return BG_EINVAL;
  if (E == 0) return BG_OK;
  if (!mom || !hel || !amp) return BG_EINVAL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return BG_EDEVICE;
  return amplitudes_dispatch(ctx, n, precision == BG_PREC_FP32_MIXED, E, 0, E, mom, hel, 0, amp,
                             (hipStream_t)stream);
}

int bg_color_contract(bg_context* ctx, int n, int64_t E, const double* amp, double* me2,
                      int accumulate, void* stream) {
  if (!ctx || n < 4 || n > 8) return n > 8 && n <= BG_N_MAX ? BG_EUNSUPPORTED : BG_EINVAL;
  int st = check_events(n, E);
  if (st) return st;
  if (E == 0) return BG_OK;
  if (!amp || !me2) return BG_EINVAL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return BG_EDEVICE;
  hipStream_t s = (hipStream_t)stream;
  if (n <= 7) return contract_dispatch(ctx, n, E, amp, me2, accumulate, s);
  st = ws_acquire(ctx, s);
  if (!st) st = ensure_part(ctx, E);
  if (!st) st = contract_dispatch(ctx, n, E, amp, me2, accumulate, s, ctx->part);
  return ws_release(ctx, s, st);
}

static int ensure_counters(bg_context* ctx) {
  if (ctx->counter) return BG_OK;
  return hip_status(hipMalloc(&ctx->counter, 256), "hipMalloc(counters)");
}

// fixed (may be null): use the static workspace, allocate nothing (the
// colour matrix must then be uploaded already, see bg_context_create).
// Colour-ordered FP64 at n = 7 (K = 120) and n = 8 (K = 720): the
// amplitudes of a chunk of events into the workspace (one straight path per
// ordering), then the colour sum (matrix cores with C in LDS at K = 120;
// through the relabelled first row of C at K = 720); over all 2^n helicity
// configurations (accumulated) when hel is null.  Each event's arithmetic
// does not depend on the chunk, so any chunk size gives the same bits.
// fixed: n = 7 only, chunks that fit the static workspace.
static int me2_cobg_two_stage(bg_context* ctx, const bg_request* r, hipStream_t stream,
                              const FixedWs* fixed) {
  const int n = r->n;
  const int64_t E = r->n_events;
  const int64_t K = bg::factorial(n - 2);
  const size_t per_event = sizeof(double) * 2 * (size_t)K;
  int64_t chunk;
  double* ws;
  int st = BG_OK;
  if (fixed) {
    if (n != 7 || !ctx->C_dev[n]) return BG_EUNSUPPORTED;
    chunk = std::min<int64_t>(E, (int64_t)(fixed->scratch_bytes / per_event));
    ws = fixed->scratch;
  } else {
    chunk = std::min<int64_t>(E, n == 7 ? kN7Chunk : kN8Chunk);
    st = n == 8 ? ensure_relabel(ctx, n) : ensure_colour(ctx, n);
    if (!st) st = ensure_ws(ctx, per_event * (size_t)chunk);
    if (!st && n == 8) st = ensure_part(ctx, chunk);
    if (st) return st;
    ws = ctx->ws;
  }
  const int nh = r->hel ? 1 : 1 << n;
  for (int64_t e0 = 0; e0 < E && !st; e0 += chunk) {
    const int64_t c = std::min<int64_t>(chunk, E - e0);
    for (int hc = 0; hc < nh && !st; ++hc) {
      st = amplitudes_dispatch(ctx, n, false, E, e0, c, r->mom, r->hel, hc, ws, stream);
      if (!st)
        st = contract_dispatch(ctx, n, c, ws, r->me2 + e0, hc > 0 ? 1 : 0, stream, ctx->part);
    }
  }
  return st;
}

// FP64 re-evaluation of the n = 7 events listed by the FP32 check (count and
// list on the device) through the same two stages as the FP64 path, so that
// each listed event gets the FP64 path's result bit for bit: the listed
// events' amplitudes into a compact workspace, then the matrix-core colour
// sum written to their me2 (accumulated over the helicity configurations
// when hel is null).  The list is covered in slices of the workspace's
// capacity; slices past the list length return at once.
static int fix_listed_two_stage(bg_context* ctx, const bg_request* r, const unsigned* count,
                                const unsigned* list, hipStream_t stream, const FixedWs* fixed) {
  const int n = 7;
  const int64_t E = r->n_events;
  const int64_t K = bg::factorial(n - 2);
  const size_t per_event = sizeof(double) * 2 * (size_t)K;
  int64_t slice;
  double* ws;
  int st = BG_OK;
  if (fixed) {
    slice = std::min<int64_t>(E, (int64_t)(fixed->scratch_bytes / per_event));
    ws = fixed->scratch;
  } else {
    slice = std::min<int64_t>(E, kN7Chunk);
    st = ensure_ws(ctx, per_event * (size_t)slice);
    if (st) return st;
    ws = ctx->ws;
  }
  const int nh = r->hel ? 1 : 1 << n;
  for (int64_t f0 = 0; f0 < E && !st; f0 += slice) {
    const int64_t c = std::min<int64_t>(slice, E - f0);
    for (int hc = 0; hc < nh && !st; ++hc) {
      // the listed events are a small share: four ordering ranges per block
      // of 32 of them, so that the short list still spreads over the CUs
      st = launch_status(bg::cobg_path_amplitudes(n, E, f0, c, r->mom, r->hel, hc, ws, list,
                                                  count, stream, 4));
      if (!st)
        st = launch_status(bg::contract_mfma((int)K, c, ws, ctx->C_dev[n], r->me2, hc > 0 ? 1 : 0,
                                             stream, list, count, f0));
    }
  }
  return st;
}

// Helicity-summed requests up to this many events take the split path
// (below ~16 k events the tiles of the fused kernel do not fill the GPU).
constexpr int64_t kHsumSplitEvents = 16384;

static int me2_cobg(bg_context* ctx, const bg_request* r, uint32_t flags, hipStream_t stream,
                    const FixedWs* fixed = nullptr) {
  const int n = r->n;
  if (n == 8) {
    if (fixed || r->precision != BG_PREC_FP64) return BG_EUNSUPPORTED;
    return me2_cobg_two_stage(ctx, r, stream, nullptr);
  }
  if (n > 8) return BG_EUNSUPPORTED;
  if (n == 7 && r->precision == BG_PREC_FP64) return me2_cobg_two_stage(ctx, r, stream, fixed);
  const int64_t E = r->n_events;
  if (fixed && !ctx->Cb_dev[n]) return BG_EINVAL;
  int st = ensure_colour(ctx, n);
  if (st) return st;
  const bool fp32 = r->precision == BG_PREC_FP32_MIXED;
  const bool hsum = r->hel == nullptr;
  const float tau = ctx->fp32_tau[0][n];
  const bool check = fp32 && !(flags & BG_FLAG_FP32_UNCHECKED) && !(tau == INFINITY) &&
                     E <= (int64_t)0xffffffffLL;
  // blocks whose per-block scratch fits the static workspace (n = 7)
  const int64_t fixed_blocks =
      fixed ? (int64_t)(fixed->scratch_bytes /
                        (sizeof(double) * (size_t)std::max(1, bg::cobg_fused_scratch_doubles(n))))
            : INT64_MAX;
  // few events with the helicities summed (FP64, n <= 6): one block per
  // (tile, configuration) instead of the configurations in turn on one block
  // per tile, which would leave most CUs idle; the same bits
  if (hsum && !fp32 && !fixed && n <= 6 && E <= kHsumSplitEvents) {
    st = ensure_ws(ctx, sizeof(double) * 2 * ((size_t)1 << n) * (size_t)E);
    if (st) return st;
    return launch_status(
        bg::cobg_hsum_split(n, E, r->mom, ctx->Cb_dev[n], ctx->ws, r->me2, stream));
  }
  int64_t grid = 0, fix_grid = 0;
  if (check) {
    int& occ = ctx->occ_fix[n][hsum ? 1 : 0];
    if (occ <= 0) occ = bg::cobg_fix_blocks_per_cu(n, hsum);
    if (occ <= 0) return BG_EDEVICE;
    fix_grid = std::min<int64_t>({(E + 31) / 32, (int64_t)ctx->num_cus * occ, fixed_blocks});
    if (!fixed) {
      st = ensure_flags(ctx, E);
      if (st) return st;
    }
  }
  double* scratch = fixed ? fixed->scratch : ctx->scratch;
  unsigned* counter = fixed ? fixed->counter : ctx->counter;
  if (n == 7) {  // persistent kernel with per-block scratch
    int& occ = ctx->occ_fused[fp32 ? 1 : 0][hsum ? 1 : 0][check ? 1 : 0];
    if (occ <= 0) occ = bg::cobg_fused_persistent_blocks_per_cu(fp32, hsum, check);
    if (occ <= 0) return BG_EDEVICE;
    grid = std::min<int64_t>({(E + 31) / 32, (int64_t)ctx->num_cus * occ, fixed_blocks});
    if (!fixed) {
      st = ensure_scratch(ctx, sizeof(double) * (size_t)std::max(grid, fix_grid) *
                                   bg::cobg_fused_scratch_doubles(n));
      if (!st) st = ensure_counters(ctx);
      if (st) return st;
      scratch = ctx->scratch;
      counter = ctx->counter;
    }
  }
  bg::CheckArgs ca{tau, nullptr, nullptr};
  if (check) {
    unsigned* ws = fixed ? fixed->flag_ws : ctx->flag_ws;
    ca.count = ws;
    ca.list = ws + kFlagListOffset;
    st = launch_status(bg::fill_u32(ca.count, 1, 0u, stream));
    if (st) return st;
  }
  st = launch_status(bg::cobg_fused_me2(n, fp32, E, r->mom, r->hel, ctx->Cb_dev[n], scratch,
                                        counter ? counter + 1 : nullptr, (int)grid, r->me2,
                                        check ? &ca : nullptr, stream));
  if (st || !check) return st;
  if (n == 7) return fix_listed_two_stage(ctx, r, ca.count, ca.list, stream, fixed);
  return launch_status(bg::cobg_fix_me2(n, E, r->mom, r->hel, ctx->Cb_dev[n], scratch, ca.count,
                                        ca.list, (int)fix_grid, r->me2, stream));
}

static int me2_cdbg(bg_context* ctx, const bg_request* r, uint32_t flags, hipStream_t stream,
                    const FixedWs* fixed = nullptr) {
  const int n = r->n;
  const int64_t E = r->n_events;
  const bool fp32 = r->precision == BG_PREC_FP32_MIXED;
  const float tau = ctx->fp32_tau[1][n];
  const bool check = fp32 && !(flags & BG_FLAG_FP32_UNCHECKED) && !(tau == INFINITY) &&
                     E <= (int64_t)0x7fffffffLL;
  const size_t lds = bg::cdbg_lds_bytes(n, fp32);
  if (lds == 0 || lds > ctx->lds_per_block) return BG_EUNSUPPORTED;
  const size_t need = sizeof(unsigned) * (size_t)(4 + 2 * E);
  if (!fixed && ctx->cws_bytes < need) {
    if (ctx->cws) {
      int st = hip_status(hipDeviceSynchronize(), "hipDeviceSynchronize");
      if (st) return st;
      (void)hipFree(ctx->cws);
      ctx->cws = nullptr;
      ctx->cws_bytes = 0;
    }
    int st = hip_status(hipMalloc(&ctx->cws, need), "hipMalloc(cdbg workspace)");
    if (st) return st;
    ctx->cws_bytes = need;
  }
  int& per_cu = check ? ctx->occ_cdbg_chk[n] : ctx->occ_cdbg[n][fp32 ? 1 : 0];
  if (per_cu <= 0) per_cu = bg::cdbg_blocks_per_cu(n, fp32, check);
  if (per_cu <= 0) return BG_EUNSUPPORTED;
  int64_t grid = std::min<int64_t>((int64_t)ctx->num_cus * (int64_t)per_cu, E);
  if (grid < 1) grid = 1;
  int64_t fix_grid = 0;
  if (check) {
    int& per_cu64 = ctx->occ_cdbg[n][0];
    if (per_cu64 <= 0) per_cu64 = bg::cdbg_blocks_per_cu(n, false, false);
    if (per_cu64 <= 0) return BG_EUNSUPPORTED;
    fix_grid = std::max<int64_t>(1, std::min<int64_t>((int64_t)ctx->num_cus * per_cu64, E));
  }
  bg::CheckArgs ca{tau, nullptr, nullptr};
  return launch_status(bg::cdbg_me2(n, fp32, E, r->mom, r->hel, r->col,
                                    fixed ? fixed->cws : ctx->cws, r->me2, (int)grid,
                                    check ? &ca : nullptr, (int)fix_grid, stream));
}

static int me2_comc(bg_context* ctx, const bg_request* r, uint32_t flags, hipStream_t stream) {
  const int n = r->n;
  const int64_t E = r->n_events;
  if (E > 0x7fffffffLL) return BG_ERANGE;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive)
    return BG_EINVAL;  // needs a synchronisation
  const bool fp32 = r->precision == BG_PREC_FP32_MIXED;
  const float tau = ctx->fp32_tau[2][n];
  const bool check = fp32 && !(flags & BG_FLAG_FP32_UNCHECKED) && tau != INFINITY;
  // workspace in 8-byte words: block item and valid-event offsets [nb + 1]
  // each, then as 32-bit words counts, offsets and the valid-event list [E]
  // each, the listed-event count and work counter, the listed events [E]
  const int64_t nb = (E + 255) / 256;
  const size_t words = (size_t)(2 * (nb + 1) + (4 * E + 2 + 1) / 2);
  int st;
  if (ctx->comc_ws_words < words) {
    st = hip_status(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (st) return st;
    if (ctx->comc_ws) (void)hipFree(ctx->comc_ws);
    ctx->comc_ws = nullptr;
    ctx->comc_ws_words = 0;
    st = hip_status(hipMalloc(&ctx->comc_ws, sizeof(uint64_t) * words), "hipMalloc(comc)");
    if (st) return st;
    ctx->comc_ws_words = words;
  }
  uint64_t* block_items = ctx->comc_ws;
  uint64_t* block_valid = block_items + nb + 1;
  unsigned* counts = reinterpret_cast<unsigned*>(block_valid + nb + 1);
  unsigned* offsets = counts + E;
  unsigned* valid = offsets + E;
  unsigned* fcount = valid + E;  // [0] listed events, [1] listed items
  unsigned* flist = fcount + 2;
  st = launch_status(bg::comc_count(n, E, r->col, r->me2, counts, offsets, valid, block_items,
                                    block_valid, stream));
  if (st) return st;
  uint64_t total[2] = {0, 0};
  st = hip_status(hipMemcpyAsync(&total[0], block_items + nb, sizeof(uint64_t),
                                 hipMemcpyDeviceToHost, stream), "hipMemcpyAsync(comc total)");
  if (!st)
    st = hip_status(hipMemcpyAsync(&total[1], block_valid + nb, sizeof(uint64_t),
                                   hipMemcpyDeviceToHost, stream), "hipMemcpyAsync(comc valid)");
  if (!st) st = hip_status(hipStreamSynchronize(stream), "hipStreamSynchronize");
  if (st) return st;
  const uint64_t n_items = total[0], n_valid = total[1];
  if (n_items == 0) return BG_OK;
  if (n_items >= (1ull << 31) || n_valid > (uint64_t)E) return BG_ERANGE;  // split the call
  if (ctx->comc_cap < n_items) {
    st = hip_status(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (st) return st;
    const size_t cap = std::max<size_t>((size_t)n_items, 2 * ctx->comc_cap);
    if (ctx->comc_items) (void)hipFree(ctx->comc_items);
    if (ctx->comc_amp) (void)hipFree(ctx->comc_amp);
    if (ctx->comc_bnd) (void)hipFree(ctx->comc_bnd);
    if (ctx->comc_sel) (void)hipFree(ctx->comc_sel);
    ctx->comc_items = nullptr;
    ctx->comc_amp = nullptr;
    ctx->comc_bnd = nullptr;
    ctx->comc_sel = nullptr;
    ctx->comc_cap = 0;
    st = hip_status(hipMalloc(&ctx->comc_items, sizeof(uint64_t) * cap), "hipMalloc(comc items)");
    if (!st) st = hip_status(hipMalloc(&ctx->comc_amp, 2 * sizeof(double) * cap), "hipMalloc(comc amp)");
    if (!st) st = hip_status(hipMalloc(&ctx->comc_bnd, sizeof(float) * cap), "hipMalloc(comc bounds)");
    if (!st) st = hip_status(hipMalloc(&ctx->comc_sel, sizeof(unsigned) * cap), "hipMalloc(comc list)");
    if (st) return st;
    ctx->comc_cap = cap;
  }
  st = launch_status(bg::comc_items(n, E, r->col, valid, (unsigned)n_valid, counts, offsets,
                                    ctx->comc_items, stream));
  if (st) return st;
  const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((n_items + 31) / 32,
                                                                 (uint64_t)ctx->num_cus * 8));
  st = launch_status(bg::comc_amplitudes(n, fp32, E, r->mom, r->hel, ctx->comc_items,
                                         block_items + nb, ctx->comc_amp,
                                         check ? ctx->comc_bnd : nullptr, grid, stream));
  if (st) return st;
  if (!check)
    return launch_status(bg::comc_reduce(valid, (unsigned)n_valid, counts, offsets, ctx->comc_amp,
                                         r->me2, stream));
  // FP32 check: the listed events' items again in FP64, then those events
  // reduced again (counts stay on the device)
  st = launch_status(bg::fill_u32(fcount, 2, 0u, stream));
  if (!st)
    st = launch_status(bg::comc_reduce_check(n, E, r->hel, valid, (unsigned)n_valid, counts,
                                             offsets, ctx->comc_amp, ctx->comc_bnd, r->me2, tau,
                                             fcount, flist, ctx->comc_sel, stream));
  if (!st)
    st = launch_status(bg::comc_amplitudes_listed(n, E, r->mom, r->hel, ctx->comc_items,
                                                  ctx->comc_sel, fcount + 1, ctx->comc_amp, grid,
                                                  stream));
  if (!st)
    st = launch_status(bg::comc_reduce_listed(flist, fcount, (unsigned)n_valid, counts, offsets,
                                              ctx->comc_amp, r->me2, stream));
  return st;
}

static int validate_request(const bg_request* r) {
  if (!r) return BG_EINVAL;
  if (!valid_n(r->n)) return BG_EINVAL;
  if (r->mode < BG_MODE_COBG || r->mode > BG_MODE_COMC) return BG_EINVAL;
  if (r->precision != BG_PREC_FP64 && r->precision != BG_PREC_FP32_MIXED) return BG_EINVAL;
  if (r->flags & ~(BG_FLAG_VALIDATE | BG_FLAG_FP32_UNCHECKED)) return BG_EINVAL;
  int st = check_events(r->n, r->n_events);
  if (st) return st;
  if (r->n_events == 0) return BG_OK;
  if (!r->mom) return BG_EINVAL;
  const int mode = r->mode == BG_MODE_AUTO ? (r->n <= 7 ? BG_MODE_COBG : BG_MODE_CDBG) : r->mode;
  if ((mode == BG_MODE_CDBG || mode == BG_MODE_COMC) && (!r->col || !r->hel)) return BG_EINVAL;
  return BG_OK;
}

// Leading colour (fused, n <= 7), with the FP32 check of the colour-ordered
// path (running error bounds summed over the (n-1)! orderings).
static int me2_lc(bg_context* ctx, const bg_request* r, uint32_t flags, hipStream_t stream,
                  const FixedWs* fixed) {
  const int n = r->n;
  const int64_t E = r->n_events;
  if (n > 7) return BG_EUNSUPPORTED;
  if (!r->hel) return BG_EINVAL;
  const bool fp32 = r->precision == BG_PREC_FP32_MIXED;
  const float tau = ctx->fp32_tau[3][n];
  const bool check = fp32 && !(flags & BG_FLAG_FP32_UNCHECKED) && !(tau == INFINITY) &&
                     E <= (int64_t)0xffffffffLL;
  if (!check)
    return launch_status(bg::lc_me2(n, fp32, E, r->mom, r->hel, r->me2, nullptr, 0, stream));
  int& occ = ctx->occ_lc_fix[n];
  if (occ <= 0) occ = bg::lc_fix_blocks_per_cu(n);
  if (occ <= 0) return BG_EDEVICE;
  const int64_t fix_grid = std::min<int64_t>((E + 31) / 32, (int64_t)ctx->num_cus * occ);
  if (!fixed) {
    int st = ensure_flags(ctx, E);
    if (st) return st;
  }
  unsigned* ws = fixed ? fixed->flag_ws : ctx->flag_ws;
  bg::CheckArgs ca{tau, ws, ws + kFlagListOffset};
  int st = launch_status(bg::fill_u32(ca.count, 1, 0u, stream));
  if (st) return st;
  return launch_status(bg::lc_me2(n, true, E, r->mom, r->hel, r->me2, &ca, (int)fix_grid, stream));
}

static int me2_dispatch(bg_context* ctx, const bg_request* r, uint32_t flags, hipStream_t stream,
                        const FixedWs* fixed = nullptr) {
  const int mode = r->mode == BG_MODE_AUTO ? (r->n <= 7 ? BG_MODE_COBG : BG_MODE_CDBG) : r->mode;
  if (mode == BG_MODE_COBG) return me2_cobg(ctx, r, flags, stream, fixed);
  if (mode == BG_MODE_COMC) return fixed ? BG_EUNSUPPORTED : me2_comc(ctx, r, flags, stream);
  if (mode == BG_MODE_LC) return me2_lc(ctx, r, flags, stream, fixed);
  return me2_cdbg(ctx, r, flags, stream, fixed);
}

int bg_me2(bg_context* ctx, const bg_request* r, void* stream) {
  if (!ctx) return BG_EINVAL;
  int st = validate_request(r);
  if (st) return st;
  if (r->n_events > 0 && !r->me2) return BG_EINVAL;
  if (r->n_events == 0) return BG_OK;
  DeviceGuard g(ctx->device);
  if (!g.ok) return BG_EDEVICE;
  hipStream_t s = (hipStream_t)stream;
  const uint32_t flags = r->flags | ctx->flags;
  st = ws_acquire(ctx, s);
  if (!st && (flags & BG_FLAG_VALIDATE))
    st = validate_values(ctx, r->n, r->n_events, r->hel, r->col, s);
  if (!st) st = me2_dispatch(ctx, r, flags, s);
  return ws_release(ctx, s, st);
}

int bg_me2_noalloc(bg_context* ctx, const bg_request* r, void* stream) {
  if (!ctx) return BG_EINVAL;
  int st = validate_request(r);
  if (st) return st;
  if (r->n_events > 0 && !r->me2) return BG_EINVAL;
  if (r->n_events > bg::kNoallocMaxEvents) return BG_ERANGE;
  if (r->n_events == 0) return BG_OK;
  if (!ctx->noalloc) return BG_EDEVICE;
  DeviceGuard g(ctx->device);
  if (!g.ok) return BG_EDEVICE;
  hipStream_t s = (hipStream_t)stream;
  const FixedWs w = fixed_ws(ctx->noalloc);
  const uint32_t flags = r->flags | ctx->flags;
  if (flags & BG_FLAG_VALIDATE) {
    st = validate_values(ctx, r->n, r->n_events, r->hel, r->col, s, &w);
    if (st) return st;
  }
  return me2_dispatch(ctx, r, flags, s, &w);
}

static int check_slot(int mode, int n) {
  if (mode == BG_MODE_COBG && n >= 4 && n <= 7) return 0;
  if (mode == BG_MODE_CDBG && valid_n(n)) return 1;
  if (mode == BG_MODE_COMC && valid_n(n)) return 2;
  if (mode == BG_MODE_LC && n >= 4 && n <= 7) return 3;
  return -1;
}

int bg_fp32_check_set(bg_context* ctx, int mode, int n, float tau) {
  const int m = check_slot(mode, n);
  if (!ctx || m < 0 || !(tau >= 0.0f)) return BG_EINVAL;
  ctx->fp32_tau[m][n] = tau;
  return BG_OK;
}

int bg_fp32_check_get(bg_context* ctx, int mode, int n, float* tau) {
  const int m = check_slot(mode, n);
  if (!ctx || !tau || m < 0) return BG_EINVAL;
  *tau = ctx->fp32_tau[m][n];
  return BG_OK;
}

int bg_me2_grad(bg_context* ctx, const bg_request* r, const double* grad_me2, double* grad_mom,
                void* stream) {
  if (!ctx) return BG_EINVAL;
  int st = validate_request(r);
  if (st) return st;
  if (r->n_events > 0 && !grad_mom) return BG_EINVAL;
  const int mode = r->mode == BG_MODE_AUTO ? (r->n <= 7 ? BG_MODE_COBG : BG_MODE_CDBG) : r->mode;
  if (mode != BG_MODE_COBG || r->n > 7) return BG_EUNSUPPORTED;
  if (r->n_events > 0 && !r->hel) return BG_EINVAL;
  if (r->n_events == 0) return BG_OK;
  DeviceGuard g(ctx->device);
  if (!g.ok) return BG_EDEVICE;
  hipStream_t s = (hipStream_t)stream;
  st = ws_acquire(ctx, s);
  if (!st && ((r->flags | ctx->flags) & BG_FLAG_VALIDATE))
    st = validate_values(ctx, r->n, r->n_events, r->hel, r->col, s);
  if (!st) st = grad_run(ctx, r, grad_me2, grad_mom, s);
  return ws_release(ctx, s, st);
}

}  // extern "C"

namespace {

int grad_run(bg_context* ctx, const bg_request* r, const double* grad_me2, double* grad_mom,
             hipStream_t s) {
  int st = BG_OK;
  const int n = r->n;
  const int64_t K = bg::factorial(n - 2);
  const int64_t E = r->n_events;
  const bool fp32 = r->precision == BG_PREC_FP32_MIXED;
  st = ensure_colour(ctx, n);
  if (!st) st = ensure_perms(ctx, n);
  if (!st) st = ensure_ws(ctx, sizeof(double) * 4 * K * E);
  if (st) return st;
  double* amp = ctx->ws;
  double* Y = ctx->ws + 2 * K * E;
  st = amplitudes_dispatch(ctx, n, fp32, E, 0, E, r->mom, r->hel, 0, amp, s);
  if (!st) st = launch_status(bg::contract_y((int)K, E, amp, ctx->C_dev[n], Y, r->me2, s));
  if (!st)
    st = launch_status(
        bg::cobg_gradient(n, fp32, E, r->mom, r->hel, Y, grad_me2, ctx->perms_dev[n], grad_mom, s));
  return st;
}

int resolved_mode(const bg_request* r) {
  return r->mode == BG_MODE_AUTO ? (r->n <= 7 ? BG_MODE_COBG : BG_MODE_CDBG) : r->mode;
}

// Estimated cost of one event in wave-time units (FP32 flops of one lane),
// used only to order the tiles.  Colour-ordered: the recursion's vertex counts
// (prefix sharing of the depth-first walk) over 64 lanes (32 events, each
// split over two lanes) plus the FP64 colour sum.  Colour-dressed: a valid
// event occupies the whole wave for ~3x its flops / 64; about 5% of uniformly
// sampled colour assignments are valid.
double event_cost(int n, bool cdbg, bool fp32) {
  const double prec = fp32 ? 1.0 : 2.0;
  if (!cdbg) {
    const int M = n - 1;
    double v3 = 0, v4 = 0;
    for (int d = 1; d < M; ++d) {
      const double times = (double)bg::factorial(n - 2) / (double)bg::factorial(n - 2 - d);
      for (int a = d - 1; a >= 0; --a) {
        const int L = d - a + 1;
        v3 += times * (L - 1);
        v4 += times * ((L - 1) * (L - 2) / 2);
      }
    }
    const double K = (double)bg::factorial(n - 2);
    return (166.0 * v3 + 188.0 * v4) * prec / 64.0 + 2.0 * (K * K / 2.0 + 8.0 * K);
  }
  const int M = n - 1;
  double splits = 1.0;
  for (int i = 0; i < M; ++i) splits *= 3.0;
  splits -= 2.0 * (double)(1 << M) - 1.0;
  return 20.0 * n + 0.05 * 3.0 * splits * 450.0 * prec / 64.0;
}

int validate_batch(bg_context* ctx, const bg_request* segs, int n_segs) {
  if (!ctx || n_segs < 0 || (n_segs > 0 && !segs)) return BG_EINVAL;
  if (n_segs > BG_BATCH_MAX_SEGS) return BG_ERANGE;
  for (int i = 0; i < n_segs; ++i) {
    const bg_request* r = &segs[i];
    int st = validate_request(r);
    if (st) return st;
    if (r->precision != segs[0].precision) return BG_EINVAL;
    if (r->n_events == 0) continue;
    if (!r->me2 || !r->hel) return BG_EINVAL;
    const int mode = resolved_mode(r);
    if (mode == BG_MODE_LC || mode == BG_MODE_COMC) return BG_EUNSUPPORTED;
    if (mode == BG_MODE_COBG && r->n > 7) return BG_EUNSUPPORTED;
    const bool fp32 = r->precision == BG_PREC_FP32_MIXED;
    const size_t lds = bg::batch_lds_bytes(mode == BG_MODE_COBG ? bg::kBatchCobg : bg::kBatchCdbg,
                                           r->n, fp32);
    if (lds == 0 || lds > ctx->lds_per_block) return BG_EUNSUPPORTED;
  }
  return BG_OK;
}

bool stream_capturing(hipStream_t stream) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return false;
  return cs == hipStreamCaptureStatusActive;
}

// Finds or builds the tile table of this batch shape.  Building allocates
// and uploads synchronously, so it is refused while the stream records.
int batch_plan(bg_context* ctx, const bg_request* segs, int n_segs, const bg_batch_config& cfg,
               bool capturing, BatchPlan** out) {
  const int prec = segs[0].precision;
  const bool fp32 = prec == BG_PREC_FP32_MIXED;
  std::vector<int64_t> key = {prec, cfg.cobg_tile_events, cfg.cdbg_tile_events, cfg.split_kinds};
  for (int i = 0; i < n_segs; ++i) {
    key.push_back(segs[i].n * 2 + (resolved_mode(&segs[i]) == BG_MODE_CDBG ? 1 : 0));
    key.push_back(segs[i].n_events);
  }
  for (BatchPlan& pl : ctx->plans) {
    if (pl.key == key) {
      pl.last_use = ++ctx->clock;
      *out = &pl;
      return BG_OK;
    }
  }
  if (capturing) {
    BG_LOG("bg_me2_batch: shape not prepared before graph capture");
    return BG_EINVAL;
  }
  struct Item {
    double cost;
    bool cd;
    bg::BatchTile t;
  };
  std::vector<Item> items;
  for (int i = 0; i < n_segs; ++i) {
    const bg_request* r = &segs[i];
    if (r->n_events == 0) continue;
    const bool cd = resolved_mode(r) == BG_MODE_CDBG;
    int64_t step = cd ? cfg.cdbg_tile_events : cfg.cobg_tile_events;
    if (cd) {
      // a colour-dressed tile costs about its number of valid events (~5 %)
      // times one event on the whole block: small segments get small tiles
      // (multiples of 16 raw events) so that ~4 tiles per block exist
      const int64_t want = (int64_t)ctx->num_cus * 2 * 4;
      const int64_t t = ((r->n_events + want - 1) / want + 15) / 16 * 16;
      step = std::max<int64_t>(16, std::min<int64_t>(step, t));
    }
    const double c = event_cost(r->n, cd, fp32);
    for (int64_t f = 0; f < r->n_events; f += step) {
      const int cnt = (int)std::min<int64_t>(step, r->n_events - f);
      items.push_back(Item{c * cnt, cd, bg::BatchTile{f, i, cnt}});
    }
  }
  if (items.size() > 0x7fffffffu) return BG_ERANGE;
  // by decreasing cost; split plans keep the colour-ordered tiles ahead of
  // the dressed ones (one persistent launch each)
  const bool split = cfg.split_kinds != 0;
  std::stable_sort(items.begin(), items.end(), [split](const Item& a, const Item& b) {
    if (split && a.cd != b.cd) return !a.cd;
    return a.cost > b.cost;
  });
  std::vector<bg::BatchTile> tiles(items.size());
  unsigned n_co = 0;
  for (size_t i = 0; i < items.size(); ++i) {
    tiles[i] = items[i].t;
    n_co += items[i].cd ? 0u : 1u;
  }
  BatchPlan pl;
  pl.key = key;
  pl.n_tiles = (unsigned)tiles.size();
  pl.n_tiles_cobg = n_co;
  if (!tiles.empty()) {
    int st = hip_status(hipMalloc(&pl.tiles, sizeof(bg::BatchTile) * tiles.size()),
                        "hipMalloc(tiles)");
    if (st) return st;
    st = hip_status(hipMemcpy(pl.tiles, tiles.data(), sizeof(bg::BatchTile) * tiles.size(),
                              hipMemcpyHostToDevice),
                    "hipMemcpy(tiles)");
    if (st) {
      free_plan(pl);
      return st;
    }
  }
  if (fp32) {
    size_t words = 64;
    uint64_t fix_cd = 0, fix_co = 0;
    for (int i = 0; i < n_segs; ++i) {
      pl.list_off.push_back(words);
      words += (size_t)segs[i].n_events;
      if (resolved_mode(&segs[i]) == BG_MODE_CDBG)
        fix_cd += (uint64_t)segs[i].n_events;
      else
        fix_co += (uint64_t)((segs[i].n_events + 127) / 128);
    }
    const uint64_t fix_tiles = fix_cd + fix_co;
    if (fix_tiles > 0x7fffffffu) {
      free_plan(pl);
      return BG_ERANGE;
    }
    words = (words + 3) / 4 * 4;  // 16-byte alignment of the tile array
    pl.max_fix_cd = (unsigned)fix_cd;
    pl.max_fix_co = (unsigned)fix_co;
    const size_t bytes = sizeof(unsigned) * words + sizeof(bg::BatchTile) * (fix_tiles + 1);
    int st = hip_status(hipMalloc(&pl.chk_ws, bytes), "hipMalloc(batch check)");
    if (st) {
      free_plan(pl);
      return st;
    }
    pl.fix_tiles = reinterpret_cast<bg::BatchTile*>(pl.chk_ws + words);
  }
  if (ctx->plans.size() >= BG_BATCH_MAX_PLANS) {
    auto lru = std::min_element(ctx->plans.begin(), ctx->plans.end(),
                                [](const BatchPlan& a, const BatchPlan& b) {
                                  return a.last_use < b.last_use;
                                });
    int st = hip_status(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (st) {
      free_plan(pl);
      return st;
    }
    free_plan(*lru);
    ctx->plans.erase(lru);
  }
  pl.last_use = ++ctx->clock;
  ctx->plans.push_back(std::move(pl));
  *out = &ctx->plans.back();
  BG_LOG("batch plan: %u tiles, %d segments", ctx->plans.back().n_tiles, n_segs);
  return BG_OK;
}

// Blocks per CU of a batch pass at an LDS size (cached per kinds, pass and
// variant).  The dressed-only kernel exists for the two-waves budget only.
int batch_occ(bg_context* ctx, bool fp32, int waves, int pass, int kinds, size_t lds,
              bool capturing) {
  if (kinds == bg::kBatchKindsCdbg) waves = 2;
  const int wi = waves - 1;
  const int k = (fp32 ? 2 : 0) + (pass != bg::kBatchPlain ? 1 : 0);
  int& occ = ctx->occ_batch[kinds][k][wi];
  size_t& at = ctx->occ_batch_lds[kinds][k][wi];
  if (occ <= 0 || at != lds) {
    if (capturing) return -1;
    occ = bg::batch_blocks_per_cu(fp32, waves, pass, kinds, lds);
    at = lds;
  }
  return occ;
}

int batch_run(bg_context* ctx, const bg_request* segs, int n_segs, const bg_batch_config& cfg,
              hipStream_t stream) {
  const bool capturing = stream_capturing(stream);
  const bool fp32 = segs[0].precision == BG_PREC_FP32_MIXED;
  bool check = false;
  if (fp32)
    for (int i = 0; i < n_segs; ++i)
      if (segs[i].n_events > 0 && !((segs[i].flags | ctx->flags) & BG_FLAG_FP32_UNCHECKED))
        check = true;
  bg::BatchSegTable tab;
  memset(&tab, 0, sizeof(tab));
  size_t lds[2] = {0, 0}, lds64[2] = {0, 0};  // [colour-ordered, colour-dressed]
  int64_t stride = 0;
  for (int i = 0; i < n_segs; ++i) {
    const bg_request* r = &segs[i];
    const bool cd = resolved_mode(r) == BG_MODE_CDBG;
    bg::BatchSeg& b = tab.s[i];
    b.mom = r->mom;
    b.hel = r->hel;
    b.col = r->col;
    b.me2 = r->me2;
    b.E = r->n_events;
    b.kind = (cd ? bg::kBatchCdbg : bg::kBatchCobg) + r->n;
    if (r->n_events == 0) continue;
    const int kind = cd ? bg::kBatchCdbg : bg::kBatchCobg;
    if (!cd) {
      if (!ctx->Cb_dev[r->n]) {
        if (capturing) return BG_EINVAL;
        int st = ensure_colour(ctx, r->n);
        if (st) return st;
      }
      b.Cl = ctx->Cb_dev[r->n];
      stride = std::max<int64_t>(stride, bg::batch_scratch_doubles(r->n));
    }
    lds[cd] = std::max(lds[cd], bg::batch_lds_bytes(kind, r->n, fp32, check));
    lds64[cd] = std::max(lds64[cd], bg::batch_lds_bytes(kind, r->n, false));
  }
  BatchPlan* pl = nullptr;
  int st = batch_plan(ctx, segs, n_segs, cfg, capturing, &pl);
  if (st) return st;
  if (pl->n_tiles == 0) return BG_OK;
  // One persistent launch per pass over every tile, or (split_kinds) one
  // over the colour-ordered tiles and one over the dressed tiles, each with
  // the LDS and register budget of its own kind.  The re-evaluation pass
  // runs the FP64 variant with the FP64 config's register budget, over tile
  // ranges built on the device.
  struct Launch {
    int kinds, waves;
    unsigned b, e;              // host tile range, or
    const unsigned* range;      // the device one
    uint64_t max_tiles;
    size_t lds;
    int64_t grid;
  };
  const bg_batch_config& cfg64 = ctx->bcfg[0];
  const int waves = cfg.waves_per_simd == 1 ? 1 : 2;
  const int waves64 = cfg64.waves_per_simd == 1 ? 1 : 2;
  unsigned* const range = fp32 && pl->chk_ws ? pl->chk_ws + 32 : nullptr;
  Launch main_l[2], fix_l[2];
  int n_main = 0, n_fix = 0;
  if (!cfg.split_kinds) {
    main_l[n_main++] = Launch{bg::kBatchKindsAll, waves, 0u, pl->n_tiles, nullptr, pl->n_tiles,
                              std::max(lds[0], lds[1]), 0};
    if (check)
      fix_l[n_fix++] = Launch{bg::kBatchKindsAll, waves64, 0u, 0u, range + 4,
                              (uint64_t)pl->max_fix_cd + pl->max_fix_co,
                              std::max(lds64[0], lds64[1]), 0};
  } else {
    if (pl->n_tiles_cobg > 0)
      main_l[n_main++] = Launch{bg::kBatchKindsCobg, waves, 0u, pl->n_tiles_cobg, nullptr,
                                pl->n_tiles_cobg, lds[0], 0};
    if (pl->n_tiles > pl->n_tiles_cobg)
      main_l[n_main++] = Launch{bg::kBatchKindsCdbg, 2, pl->n_tiles_cobg, pl->n_tiles, nullptr,
                                pl->n_tiles - pl->n_tiles_cobg, lds[1], 0};
    if (check && pl->max_fix_cd > 0)
      fix_l[n_fix++] = Launch{bg::kBatchKindsCdbg, 2, 0u, 0u, range + 0, pl->max_fix_cd,
                              lds64[1], 0};
    if (check && pl->max_fix_co > 0)
      fix_l[n_fix++] = Launch{bg::kBatchKindsCobg, waves64, 0u, 0u, range + 2, pl->max_fix_co,
                              lds64[0], 0};
  }
  size_t need = 256;
  auto size_grid = [&](Launch& l, bool f32, int ps, const bg_batch_config& c) -> int {
    const int occ = batch_occ(ctx, f32, l.waves, ps, l.kinds, l.lds, capturing);
    if (occ == -1 && capturing) return BG_EINVAL;
    if (occ <= 0) return BG_EUNSUPPORTED;
    const int bpc = c.blocks_per_cu > 0 ? std::min(c.blocks_per_cu, occ) : occ;
    l.grid = std::max<int64_t>(
        1, std::min<int64_t>((int64_t)ctx->num_cus * bpc, (int64_t)std::max<uint64_t>(l.max_tiles, 1)));
    if (l.kinds != bg::kBatchKindsCdbg)
      need = std::max(need, sizeof(double) * (size_t)l.grid * (size_t)stride);
    return BG_OK;
  };
  const int pass = check ? bg::kBatchCheck : bg::kBatchPlain;
  for (int i = 0; i < n_main; ++i)
    if ((st = size_grid(main_l[i], fp32, pass, cfg))) return st;
  for (int i = 0; i < n_fix; ++i)
    if ((st = size_grid(fix_l[i], false, bg::kBatchFix, cfg64))) return st;
  if (ctx->scratch_bytes < need || !ctx->counter) {
    if (capturing) {
      BG_LOG("bg_me2_batch: workspace not prepared before graph capture");
      return BG_EINVAL;
    }
    st = ensure_scratch(ctx, need);
    if (!st) st = ensure_counters(ctx);
    if (st) return st;
  }
  auto run = [&](const Launch& l, bool f32, int ps, hipStream_t on, unsigned* head) -> int {
    // the dressed-only kernel never touches the colour-ordered scratch
    const int64_t sstride = l.kinds == bg::kBatchKindsCdbg ? 0 : stride;
    return launch_status(bg::batch_launch(f32, l.waves, ps, l.kinds, tab, ps == bg::kBatchFix
                                                                          ? pl->fix_tiles
                                                                          : pl->tiles,
                                          l.b, l.e, l.range, head, ctx->scratch, sstride,
                                          (int)l.grid, l.lds, on));
  };
  // The launches of one pass.  Split into kinds, the two run concurrently:
  // the colour-ordered one on `stream`, the dressed one on the context's side
  // stream (forked and joined through events, so a graph records both), each
  // with its own queue head.  The colour-ordered launch is enqueued first: its
  // blocks (the larger LDS) take their CUs before the dressed blocks fill the
  // rest, and as each CU's colour-ordered block runs out of tiles (the long
  // n = 7 tasks end at different times) dressed blocks take its place.
  if (cfg.split_kinds && !ctx->side && !capturing) {
    st = hip_status(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking), "hipStreamCreate");
    if (!st) st = hip_status(hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming), "hipEventCreate");
    if (!st) st = hip_status(hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming), "hipEventCreate");
    if (st) return st;
  }
  auto run_pass = [&](const Launch* ls, int nl, bool f32, int ps) -> int {
    if (nl == 2 && ctx->side && ctx->fork_ev && ctx->join_ev) {
      const int a = ls[0].kinds == bg::kBatchKindsCobg ? 0 : 1;  // colour-ordered first
      int r = hip_status(hipEventRecord(ctx->fork_ev, stream), "hipEventRecord");
      if (!r) r = hip_status(hipStreamWaitEvent(ctx->side, ctx->fork_ev, 0), "hipStreamWaitEvent");
      if (!r) r = run(ls[a], f32, ps, stream, ctx->counter);
      if (!r) r = run(ls[1 - a], f32, ps, ctx->side, ctx->counter + 2);
      if (!r) r = hip_status(hipEventRecord(ctx->join_ev, ctx->side), "hipEventRecord");
      if (!r) r = hip_status(hipStreamWaitEvent(stream, ctx->join_ev, 0), "hipStreamWaitEvent");
      return r;
    }
    int r = BG_OK;
    for (int i = 0; i < nl && !r; ++i) r = run(ls[i], f32, ps, stream, ctx->counter);
    return r;
  };
  if (!check) return run_pass(main_l, n_main, fp32, bg::kBatchPlain);
  for (int i = 0; i < n_segs; ++i) {
    const bg_request* r = &segs[i];
    bg::BatchSeg& b = tab.s[i];
    const bool cd = resolved_mode(r) == BG_MODE_CDBG;
    b.fcount = pl->chk_ws + i;
    b.flist = pl->chk_ws + pl->list_off[i];
    b.tau = ((r->flags | ctx->flags) & BG_FLAG_FP32_UNCHECKED) ? INFINITY
                                                               : ctx->fp32_tau[cd ? 1 : 0][r->n];
  }
  st = launch_status(bg::fill_u32(pl->chk_ws, 38, 0u, stream));
  if (!st) st = run_pass(main_l, n_main, true, bg::kBatchCheck);
  if (!st)
    st = launch_status(bg::batch_fix_tiles(tab, n_segs, pl->chk_ws, pl->fix_tiles, range, stream));
  if (st) return st;
  for (int i = 0; i < n_segs; ++i) tab.s[i].idx = tab.s[i].flist;
  return run_pass(fix_l, n_fix, false, bg::kBatchFix);
}

bool valid_config(const bg_batch_config* c) {
  return c && c->blocks_per_cu >= 0 && c->blocks_per_cu <= 64 && c->cobg_tile_events >= 128 &&
         c->cobg_tile_events <= 8192 && c->cobg_tile_events % 128 == 0 &&
         c->cdbg_tile_events >= 32 && c->cdbg_tile_events <= 8192 &&
         c->cdbg_tile_events % 32 == 0 && (c->waves_per_simd == 1 || c->waves_per_simd == 2) &&
         (c->split_kinds == 0 || c->split_kinds == 1);
}

}  // namespace

extern "C" {

int bg_me2_batch(bg_context* ctx, const bg_request* segs, int n_segs, void* stream) {
  int st = validate_batch(ctx, segs, n_segs);
  if (st) return st;
  if (n_segs == 0) return BG_OK;
  DeviceGuard g(ctx->device);
  if (!g.ok) return BG_EDEVICE;
  const int fi = segs[0].precision == BG_PREC_FP32_MIXED ? 1 : 0;
  hipStream_t s = (hipStream_t)stream;
  st = ws_acquire(ctx, s);
  for (int i = 0; i < n_segs && !st; ++i)
    if ((segs[i].flags | ctx->flags) & BG_FLAG_VALIDATE)
      st = validate_values(ctx, segs[i].n, segs[i].n_events, segs[i].hel, segs[i].col, s);
  if (!st) st = batch_run(ctx, segs, n_segs, ctx->bcfg[fi], s);
  return ws_release(ctx, s, st);
}

int bg_batch_config_get(bg_context* ctx, int precision, bg_batch_config* out) {
  if (!ctx || !out) return BG_EINVAL;
  if (precision != BG_PREC_FP64 && precision != BG_PREC_FP32_MIXED) return BG_EINVAL;
  *out = ctx->bcfg[precision == BG_PREC_FP32_MIXED ? 1 : 0];
  return BG_OK;
}

int bg_batch_config_set(bg_context* ctx, int precision, const bg_batch_config* cfg) {
  if (!ctx || !valid_config(cfg)) return BG_EINVAL;
  if (precision != BG_PREC_FP64 && precision != BG_PREC_FP32_MIXED) return BG_EINVAL;
  ctx->bcfg[precision == BG_PREC_FP32_MIXED ? 1 : 0] = *cfg;
  return BG_OK;
}

int bg_me2_batch_tune(bg_context* ctx, const bg_request* segs, int n_segs, bg_batch_config* best,
                      double* best_ms, void* stream) {
  int st = validate_batch(ctx, segs, n_segs);
  if (st) return st;
  if (n_segs == 0) return BG_EINVAL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return BG_EDEVICE;
  hipStream_t s = (hipStream_t)stream;
  if (stream_capturing(s)) return BG_EINVAL;
  const int fi = segs[0].precision == BG_PREC_FP32_MIXED ? 1 : 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  st = hip_status(hipEventCreate(&e0), "hipEventCreate");
  if (!st) st = hip_status(hipEventCreate(&e1), "hipEventCreate");
  bg_batch_config cur = {0, 128, 256, 2, 1};
  double cur_ms = 1e300;
  auto time_cfg = [&](const bg_batch_config& c, double* ms) -> int {
    int r = batch_run(ctx, segs, n_segs, c, s);  // warm-up, builds the plan
    if (r) return r;
    double bestt = 1e300;
    for (int rep = 0; rep < 2; ++rep) {
      r = hip_status(hipEventRecord(e0, s), "hipEventRecord");
      if (!r) r = batch_run(ctx, segs, n_segs, c, s);
      if (!r) r = hip_status(hipEventRecord(e1, s), "hipEventRecord");
      if (!r) r = hip_status(hipEventSynchronize(e1), "hipEventSynchronize");
      float t = 0.f;
      if (!r) r = hip_status(hipEventElapsedTime(&t, e0, e1), "hipEventElapsedTime");
      if (r) return r;
      bestt = std::min(bestt, (double)t);
    }
    *ms = bestt;
    return BG_OK;
  };
  auto try_cfg = [&](const bg_batch_config& c) -> int {
    double ms = 0.0;
    int r = time_cfg(c, &ms);
    if (r) return r;
    BG_LOG("tune: split %d waves/SIMD %d blocks/CU %d cobg tile %d cdbg tile %d -> %.3f ms",
           c.split_kinds, c.waves_per_simd, c.blocks_per_cu, c.cobg_tile_events,
           c.cdbg_tile_events, ms);
    if (ms < cur_ms) {
      cur_ms = ms;
      cur = c;
    }
    return BG_OK;
  };
  if (!st) {
    const bg_batch_config base = cur;
    for (int sp : {1, 0}) {
      for (int v : {2, 1}) {
        for (int b : {0, 1}) {
          bg_batch_config c = base;
          c.split_kinds = sp;
          c.waves_per_simd = v;
          c.blocks_per_cu = b;
          if ((st = try_cfg(c))) break;
        }
        if (st) break;
      }
      if (st) break;
    }
  }
  if (!st) {
    const bg_batch_config base = cur;
    for (int t : {128, 256, 512, 1024}) {
      bg_batch_config c = base;
      c.cobg_tile_events = t;
      if ((st = try_cfg(c))) break;
    }
  }
  if (!st) {
    const bg_batch_config base = cur;
    for (int t : {32, 64, 128, 256, 512}) {
      bg_batch_config c = base;
      c.cdbg_tile_events = t;
      if ((st = try_cfg(c))) break;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) return st;
  ctx->bcfg[fi] = cur;
  if (best) *best = cur;
  if (best_ms) *best_ms = cur_ms;
  return BG_OK;
}

int bg_me2_continuous(bg_context* ctx, int n, int precision, int64_t n_events, const double* mom,
                      const double* phi, const double* eta, double* me2, void* stream) {
  if (!ctx) return BG_EINVAL;
  if (!valid_n(n)) return BG_EINVAL;
  if (precision != BG_PREC_FP64 && precision != BG_PREC_FP32_MIXED) return BG_EINVAL;
  int st = check_events(n, n_events);
  if (st) return st;
  if (n_events == 0) return BG_OK;
  if (!mom || !phi || !eta || !me2) return BG_EINVAL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return BG_EDEVICE;
  const bool fp32 = precision == BG_PREC_FP32_MIXED;
  int& per_cu = ctx->occ_cdmc[n][fp32 ? 1 : 0];
  if (per_cu <= 0) per_cu = bg::cdmc_blocks_per_cu(n, fp32);
  if (per_cu <= 0) return BG_EUNSUPPORTED;
  int64_t grid = (int64_t)ctx->num_cus * (int64_t)per_cu;
  if (grid > n_events) grid = n_events;
  void* gstate = nullptr;
  if (bg::cdmc_global_state(n, fp32)) {
    // one slab per block of the largest grid, allocated once per context
    const size_t need = bg::cdmc_state_bytes(n, fp32) * (size_t)ctx->num_cus * (size_t)per_cu;
    if (ctx->cdmc_state_bytes < need) {
      st = hip_status(hipDeviceSynchronize(), "hipDeviceSynchronize");
      if (st) return st;
      if (ctx->cdmc_state) (void)hipFree(ctx->cdmc_state);
      ctx->cdmc_state = nullptr;
      ctx->cdmc_state_bytes = 0;
      st = hip_status(hipMalloc(&ctx->cdmc_state, need), "hipMalloc(continuous state)");
      if (st) return st;
      ctx->cdmc_state_bytes = need;
    }
    gstate = ctx->cdmc_state;
  }
  st = ws_acquire(ctx, (hipStream_t)stream);
  if (!st)
    st = launch_status(bg::cdmc_me2(n, fp32, n_events, mom, phi, eta, gstate, (int)grid, me2,
                                    (hipStream_t)stream));
  return ws_release(ctx, (hipStream_t)stream, st);
}

int bg_generate_continuous(bg_context* ctx, int n, uint64_t seed, uint64_t first_event,
                           int64_t n_events, double* phi, double* eta, void* stream) {
  if (!ctx) return BG_EINVAL;
  if (!valid_n(n)) return BG_EINVAL;
  int st = check_events(n, n_events);
  if (st) return st;
  if (n_events == 0) return BG_OK;
  if (!phi || !eta) return BG_EINVAL;
  if (n_events > ((int64_t)1 << 31) * 256) return BG_ERANGE;  // grid limit
  DeviceGuard g(ctx->device);
  if (!g.ok) return BG_EDEVICE;
  return launch_status(bg::generate_continuous(n, seed, first_event, n_events, phi, eta,
                                               (hipStream_t)stream));
}

int bg_generate(bg_context* ctx, const bg_gen_params* gp, int64_t n_attempts, int64_t max_events,
                double* mom, int8_t* hel, int8_t* col, int64_t* attempt, int64_t* n_generated,
                void* stream) {
  if (!ctx || !gp || !mom || !n_generated) return BG_EINVAL;
  if (!valid_n(gp->n)) return BG_EINVAL;
  if (gp->flags & ~(BG_GEN_CUTS | BG_GEN_HEL | BG_GEN_COL)) return BG_EINVAL;
  if (((gp->flags & BG_GEN_HEL) && !hel) || ((gp->flags & BG_GEN_COL) && !col)) return BG_EINVAL;
  if (!(gp->sqrt_s > 0.0) || !(gp->pt_min >= 0.0) || !(gp->dr_min >= 0.0)) return BG_EINVAL;
  if (n_attempts < 1 || max_events < 1) return BG_EINVAL;
  if (n_attempts > ((int64_t)1 << 31)) return BG_ERANGE;
  int st = check_events(gp->n, max_events);
  if (st) return st;
  DeviceGuard g(ctx->device);
  if (!g.ok) return BG_EDEVICE;
  const size_t words = bg::generate_workspace_words(n_attempts);
  if (ctx->gen_ws_words < words) {
    if (stream_capturing((hipStream_t)stream)) return BG_EINVAL;
    unsigned* w = nullptr;
    st = hip_status(hipMalloc(&w, sizeof(unsigned) * words), "hipMalloc(generator workspace)");
    if (st) return st;
    if (ctx->gen_ws) ctx->retired.push_back(ctx->gen_ws);  // queued work may still read it
    ctx->gen_ws = w;
    ctx->gen_ws_words = words;
  }
  bg::GenParams p;
  p.n = gp->n;
  p.cuts = (gp->flags & BG_GEN_CUTS) ? 1 : 0;
  p.sqrt_s = gp->sqrt_s;
  p.pt_min = gp->pt_min;
  p.dr_min = gp->dr_min;
  p.seed = gp->seed;
  p.first_attempt = gp->first_attempt;
  st = ws_acquire(ctx, (hipStream_t)stream);
  if (!st)
    st = launch_status(bg::generate_events(p, n_attempts, max_events, ctx->gen_ws, mom,
                                           (gp->flags & BG_GEN_HEL) ? hel : nullptr,
                                           (gp->flags & BG_GEN_COL) ? col : nullptr, attempt,
                                           n_generated, (hipStream_t)stream));
  return ws_release(ctx, (hipStream_t)stream, st);
}

int bg_mfma_layout_probe(bg_context* ctx, double* out) {
  if (!ctx || !out) return BG_EINVAL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return BG_EDEVICE;
  double* d = nullptr;
  int st = hip_status(hipMalloc(&d, 256 * sizeof(double)), "hipMalloc(probe)");
  if (st) return st;
  st = launch_status(bg::mfma_probe(d, nullptr));
  if (!st) st = hip_status(hipMemcpy(out, d, 256 * sizeof(double), hipMemcpyDeviceToHost),
                           "hipMemcpy(probe)");
  (void)hipFree(d);
  return st;
}

}  // extern "C"
