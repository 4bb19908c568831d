// C-ABI layer: argument validation, context (colour matrices, workspace) and
// dispatch to the HIP kernels.  See include/bg.h for the contract.
#include "bg.h"

#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <utility>
#include <vector>

#include "bg_kernels.h"

namespace bg {
int64_t colour_matrix(int n, double* C);
}

struct bg_context {
  int device;
  int num_cus;
  size_t lds_per_cu;
  size_t lds_per_block;
  unsigned* cws;                   // colour-dressed workspace (counters + event list)
  size_t cws_bytes;
  double* C_dev[BG_N_MAX + 1];     // K x K colour matrix per n (lazy)
  double* Cpad_dev[BG_N_MAX + 1];  // KP x KP zero-padded copy for the matrix-core path
  int KP[BG_N_MAX + 1];
  double* ws;                      // workspace (partial amplitudes)
  size_t ws_bytes;
  uint8_t* perms_dev[BG_N_MAX + 1];  // [K][n-2] middle gluons of each ordering (gradient)
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

int ensure_colour(bg_context* ctx, int n) {
  if (ctx->C_dev[n]) return BG_OK;
  const int64_t K = bg::factorial(n - 2);
  std::vector<double> C((size_t)(K * K));
  bg::colour_matrix(n, C.data());
  int KP = (int)((K + 15) / 16 * 16);
  std::vector<double> Cp((size_t)KP * KP, 0.0);
  for (int64_t i = 0; i < K; ++i)
    for (int64_t j = 0; j < K; ++j) Cp[(size_t)(i * KP + j)] = C[(size_t)(i * K + j)];
  double* d = nullptr;
  double* dp = nullptr;
  int st = hip_status(hipMalloc(&d, sizeof(double) * K * K), "hipMalloc(C)");
  if (st) return st;
  st = hip_status(hipMalloc(&dp, sizeof(double) * KP * KP), "hipMalloc(Cpad)");
  if (st) {
    (void)hipFree(d);
    return st;
  }
  st = hip_status(hipMemcpy(d, C.data(), sizeof(double) * K * K, hipMemcpyHostToDevice),
                  "hipMemcpy(C)");
  if (!st)
    st = hip_status(hipMemcpy(dp, Cp.data(), sizeof(double) * KP * KP, hipMemcpyHostToDevice),
                    "hipMemcpy(Cpad)");
  if (st) {
    (void)hipFree(d);
    (void)hipFree(dp);
    return st;
  }
  ctx->C_dev[n] = d;
  ctx->Cpad_dev[n] = dp;
  ctx->KP[n] = KP;
  BG_LOG("colour matrix n=%d K=%lld uploaded", n, (long long)K);
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

int contract_dispatch(bg_context* ctx, int n, int64_t E, const double* amp, double* me2,
                      int accumulate, hipStream_t stream) {
  int st = ensure_colour(ctx, n);
  if (st) return st;
  const int K = (int)bg::factorial(n - 2);
  if (ctx->KP[n] == 32)
    return launch_status(
        bg::contract_mfma(K, E, amp, ctx->Cpad_dev[n], ctx->KP[n], me2, accumulate, stream));
  return launch_status(bg::contract_valu(K, E, amp, ctx->C_dev[n], me2, accumulate, stream));
}

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

int bg_context_create(bg_context** out, int device) {
  if (!out) return BG_EINVAL;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return BG_ENODEV;
  if (device < 0 || device >= count) return BG_ENODEV;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return BG_ENODEV;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    BG_LOG("device %d is %s, not gfx950", device, prop.gcnArchName);
    return BG_ENODEV;
  }
  bg_context* ctx = (bg_context*)calloc(1, sizeof(bg_context));
  if (!ctx) return BG_ENOMEM;
  ctx->device = device;
  ctx->num_cus = prop.multiProcessorCount;
  ctx->lds_per_cu = prop.maxSharedMemoryPerMultiProcessor;
  ctx->lds_per_block = prop.sharedMemPerBlock;
  *out = ctx;
  return BG_OK;
}

void bg_context_destroy(bg_context* ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  (void)hipDeviceSynchronize();
  for (int n = 0; n <= BG_N_MAX; ++n) {
    if (ctx->C_dev[n]) (void)hipFree(ctx->C_dev[n]);
    if (ctx->Cpad_dev[n]) (void)hipFree(ctx->Cpad_dev[n]);
    if (ctx->perms_dev[n]) (void)hipFree(ctx->perms_dev[n]);
  }
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->cws) (void)hipFree(ctx->cws);
  free(ctx);
}

int bg_currents(bg_context* ctx, int n, int64_t E, const double* mom, const int8_t* hel,
                int precision, double* amp, void* stream) {
  if (!ctx || n < 4 || n > 7) return n > 7 && n <= BG_N_MAX ? BG_EUNSUPPORTED : BG_EINVAL;
  int st = check_events(n, E);
  if (st) return st;
  if (precision != BG_PREC_FP64 && precision != BG_PREC_FP32_MIXED) return BG_EINVAL;
  if (E == 0) return BG_OK;
  if (!mom || !hel || !amp) return BG_EINVAL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return BG_EDEVICE;
  return launch_status(bg::cobg_amplitudes(n, precision == BG_PREC_FP32_MIXED, E, mom, hel, 0,
                                           amp, (hipStream_t)stream));
}

int bg_color_contract(bg_context* ctx, int n, int64_t E, const double* amp, double* me2,
                      int accumulate, void* stream) {
  if (!ctx || n < 4 || n > 7) return n > 7 && n <= BG_N_MAX ? BG_EUNSUPPORTED : BG_EINVAL;
  int st = check_events(n, E);
  if (st) return st;
  if (E == 0) return BG_OK;
  if (!amp || !me2) return BG_EINVAL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return BG_EDEVICE;
  return contract_dispatch(ctx, n, E, amp, me2, accumulate, (hipStream_t)stream);
}

static int me2_cobg(bg_context* ctx, const bg_request* r, hipStream_t stream) {
  const int n = r->n;
  if (n > 7) return BG_EUNSUPPORTED;
  const int64_t K = bg::factorial(n - 2);
  const int64_t E = r->n_events;
  int st = ensure_colour(ctx, n);
  if (st) return st;
  st = ensure_ws(ctx, sizeof(double) * 2 * K * E);
  if (st) return st;
  const bool fp32 = r->precision == BG_PREC_FP32_MIXED;
  if (r->hel) {
    st = launch_status(bg::cobg_amplitudes(n, fp32, E, r->mom, r->hel, 0, ctx->ws, stream));
    if (st) return st;
    return contract_dispatch(ctx, n, E, ctx->ws, r->me2, 0, stream);
  }
  for (int h = 0; h < (1 << n); ++h) {
    st = launch_status(bg::cobg_amplitudes(n, fp32, E, r->mom, nullptr, h, ctx->ws, stream));
    if (st) return st;
    st = contract_dispatch(ctx, n, E, ctx->ws, r->me2, h > 0, stream);
    if (st) return st;
  }
  return BG_OK;
}

static int me2_cdbg(bg_context* ctx, const bg_request* r, hipStream_t stream) {
  const int n = r->n;
  const bool fp32 = r->precision == BG_PREC_FP32_MIXED;
  const size_t lds = bg::cdbg_lds_bytes(n, fp32);
  if (lds == 0 || lds > ctx->lds_per_block) return BG_EUNSUPPORTED;
  const size_t need = sizeof(unsigned) * (size_t)(2 + r->n_events);
  if (ctx->cws_bytes < need) {
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
  size_t per_cu = ctx->lds_per_cu ? ctx->lds_per_cu / lds : 1;
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 8) per_cu = 8;
  int64_t grid = (int64_t)ctx->num_cus * (int64_t)per_cu;
  if (grid > r->n_events) grid = r->n_events;
  if (grid < 1) grid = 1;
  return launch_status(bg::cdbg_me2(n, fp32, r->n_events, r->mom, r->hel, r->col, ctx->cws, r->me2,
                                    (int)grid, stream));
}

static int validate_request(const bg_request* r) {
  if (!r) return BG_EINVAL;
  if (!valid_n(r->n)) return BG_EINVAL;
  if (r->mode < BG_MODE_COBG || r->mode > BG_MODE_AUTO) return BG_EINVAL;
  if (r->precision != BG_PREC_FP64 && r->precision != BG_PREC_FP32_MIXED) return BG_EINVAL;
  if (r->reserved != 0) return BG_EINVAL;
  int st = check_events(r->n, r->n_events);
  if (st) return st;
  if (r->n_events == 0) return BG_OK;
  if (!r->mom) return BG_EINVAL;
  const int mode = r->mode == BG_MODE_AUTO ? (r->n <= 7 ? BG_MODE_COBG : BG_MODE_CDBG) : r->mode;
  if (mode == BG_MODE_CDBG && (!r->col || !r->hel)) return BG_EINVAL;
  return BG_OK;
}

int bg_me2(bg_context* ctx, const bg_request* r, void* stream) {
  if (!ctx) return BG_EINVAL;
  int st = validate_request(r);
  if (st) return st;
  if (r->n_events > 0 && !r->me2) return BG_EINVAL;
  if (r->n_events == 0) return BG_OK;
  DeviceGuard g(ctx->device);
  if (!g.ok) return BG_EDEVICE;
  const int mode = r->mode == BG_MODE_AUTO ? (r->n <= 7 ? BG_MODE_COBG : BG_MODE_CDBG) : r->mode;
  if (mode == BG_MODE_COBG) return me2_cobg(ctx, r, (hipStream_t)stream);
  return me2_cdbg(ctx, r, (hipStream_t)stream);
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
  st = launch_status(bg::cobg_amplitudes(n, fp32, E, r->mom, r->hel, 0, amp, s));
  if (!st) st = launch_status(bg::contract_y((int)K, E, amp, ctx->C_dev[n], Y, r->me2, s));
  if (!st)
    st = launch_status(
        bg::cobg_gradient(n, fp32, E, r->mom, r->hel, Y, grad_me2, ctx->perms_dev[n], grad_mom, s));
  return st;
}

int bg_me2_batch(bg_context* ctx, const bg_request* segs, int n_segs, void* stream) {
  (void)stream;
  if (!ctx || n_segs < 0 || (n_segs > 0 && !segs)) return BG_EINVAL;
  for (int i = 0; i < n_segs; ++i) {
    int st = validate_request(&segs[i]);
    if (st) return st;
  }
  return BG_EUNSUPPORTED;
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
