// api.cpp -- the C ABI (include/eapdtw.h): argument checks, device scratch,
// launch sequencing and result read-back.  All arithmetic of the method runs
// in the device kernels; the host only validates, plans memory and launches.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/eapdtw.h"
#include "dispatch.h"
#include "wide.h"
#include "wf.h"
#include "batch.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

using namespace eapdtw;

struct eapdtw_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  bool poisoned = false;
  char *scratch = nullptr;
  size_t scratch_cap = 0;
  char *pinned = nullptr;
  size_t pinned_cap = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr;
  hipEvent_t ev_lb[4] = {nullptr, nullptr, nullptr, nullptr};  // cascade: pass boundaries
  // options
  int64_t check_interval = 0;  // 0: chosen per window
  int64_t seed = 1;
  int64_t rows_per_group = 0;
  int64_t wide_rows = 0;
  int64_t graph = 1;
  int64_t force_wide = 0;
  int64_t seed_stride = 0;  // 0: about kSeedBlocks blocks per search
  uint32_t epoch = 0;  // numbers the searches (non-finite flag values)
  int64_t border = 1;
  int64_t ed = 1;
  int64_t autotune = 0;
  int64_t lanes = 0;  // band search with lane refill where it applies
  int64_t wf_lanes = 0;  // wavefront pair kernels: lanes per pair (0 = by size, 16, 32 or 64)
  // test hooks (host only; no device work): a cap on the scratch the context
  // may allocate (0: none), and a device fault reported by the next call
  int64_t scratch_limit = 0;
  int64_t inject_fault = 0;
  int64_t log = 0;  // one stderr line per kernel choice (EAPDTW_LOG=1 at create sets it)
  int64_t lb_ec = 0;         // cascade: apply the candidate-envelope LB_Keogh
  int64_t lb_probe_div = 0;  // cascade: first pass over K / div candidates (0: one pass)
  float lb_ms = 0.f, lb_dp_ms = 0.f;  // cascade timing of the last timed call
  bool lb_probe_two = false;          // the last cascade ran a probe range first
  std::map<int64_t, eapdtw_tune> tune;  // autotuning cache, by (length, window) bucket
  int64_t seed_window = 8;
  int64_t batch_grid = 2048;
  int64_t batch_chunk = 4;
  int64_t batch_seed_stride = 0;
  int64_t batch_branches = 4;  // streams the batched search's band launches spread over
  // batched search: dedicated device buffer and the captured graph
  char *batch_buf = nullptr;
  size_t batch_cap = 0;
  hipGraphExec_t batch_exec = nullptr;
  uint64_t batch_key = 0;
  hipStream_t cap_stream = nullptr;  // private stream used only to record graphs
  // second stream on which the seeding workgroup runs beside the search
  hipStream_t seed_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // side streams of the batched search's concurrent band launches, with the
  // fork event and one join event each
  static constexpr int kMaxBranches = 8;
  hipStream_t branch[kMaxBranches] = {};
  hipEvent_t ev_bfork = nullptr;
  hipEvent_t ev_bjoin[kMaxBranches] = {};
  // device address of this GPU's fixed scratch array (eapdtw_nn_search_noalloc)
  char *noalloc = nullptr;
};

static thread_local std::string g_create_error;

namespace {

int fail(eapdtw_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

bool is_fault(hipError_t e) {
  return e == hipErrorIllegalAddress || e == hipErrorLaunchFailure ||
         e == hipErrorIllegalState || e == hipErrorAssert;
}

// Launch log: which kernel (template parameters, class) and launch shape a
// call took, one line on stderr each, when the context's option "log" is set.
__attribute__((format(printf, 2, 3))) void log_launch(const eapdtw_ctx *c, const char *fmt, ...) {
  if (!c || !c->log) return;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  fprintf(stderr, "[eapdtw] %s\n", buf);
}

int fail_hip(eapdtw_ctx *c, hipError_t e, const char *what) {
  if (is_fault(e)) c->poisoned = true;
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
  return fail(c, EAPDTW_EDEVICE, buf);
}

#define HIPCHK(call)                                    \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return fail_hip(ctx, e_, #call); \
  } while (0)

#define CHECK_CTX()                                                          \
  do {                                                                       \
    if (!ctx) return EAPDTW_EINVAL;                                          \
    if (ctx->poisoned) return fail(ctx, EAPDTW_EPOISONED, "context poisoned by an earlier device fault"); \
    ctx->err.clear();                                                        \
    if (ctx->inject_fault) {                                                 \
      ctx->inject_fault = 0;                                                 \
      return fail_hip(ctx, hipErrorLaunchFailure, "injected device fault (test hook)"); \
    }                                                                        \
  } while (0)

// Byte offsets of the sub-buffers of one call inside the context scratch.
struct Plan {
  size_t off = 0;
  size_t add(size_t bytes) {
    size_t o = (off + 255) & ~size_t(255);
    off = o + bytes;
    return o;
  }
};

int ensure_scratch(eapdtw_ctx *ctx, size_t need) {
  if (need <= ctx->scratch_cap) return EAPDTW_OK;
  if (ctx->scratch_limit > 0 && need > (size_t)ctx->scratch_limit)
    return fail(ctx, EAPDTW_ENOMEM, "device scratch above the context's scratch_limit");
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (ctx->scratch) HIPCHK(hipFree(ctx->scratch));
  ctx->scratch = nullptr;
  ctx->scratch_cap = 0;
  size_t cap = need + need / 2 + (1 << 20);
  if (hipMalloc((void **)&ctx->scratch, cap) != hipSuccess) {
    (void)hipGetLastError();
    ctx->scratch = nullptr;
    return fail(ctx, EAPDTW_ENOMEM, "device scratch allocation failed");
  }
  ctx->scratch_cap = cap;
  // the non-finite flag word after the counters: no epoch matches zero
  HIPCHK(launch_fill_u64(reinterpret_cast<unsigned long long *>(ctx->scratch) + kCntWords, 0ull, 1,
                         ctx->stream));
  return EAPDTW_OK;
}

int ensure_pinned(eapdtw_ctx *ctx, size_t need) {
  if (need <= ctx->pinned_cap) return EAPDTW_OK;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (ctx->pinned) HIPCHK(hipHostFree(ctx->pinned));
  ctx->pinned = nullptr;
  ctx->pinned_cap = 0;
  size_t cap = need < 4096 ? 4096 : need;
  HIPCHK(hipHostMalloc((void **)&ctx->pinned, cap, hipHostMallocDefault));
  ctx->pinned_cap = cap;
  return EAPDTW_OK;
}

template <class T>
T *at(eapdtw_ctx *ctx, size_t off) {
  return reinterpret_cast<T *>(ctx->scratch + off);
}

// float32 bound that keeps exactly the float32 results <= ub (rounded down)
float bound_down(double ub) {
  if (std::isinf(ub)) return ub > 0 ? INFINITY : -INFINITY;
  float f = (float)ub;
  if ((double)f > ub) f = std::nextafter(f, -INFINITY);
  return f;
}

int64_t band_cells_total(int64_t lrow, int64_t lcol, int64_t r) {
  int64_t c = 0;
  for (int64_t i = 0; i < lrow; ++i) {
    int64_t lo = i - r < 0 ? 0 : i - r;
    int64_t hi = i + r > lcol - 1 ? lcol - 1 : i + r;
    if (hi >= lo) c += hi - lo + 1;
  }
  return c;
}

// Persistent single-wave workgroups of the wide kernels: enough to fill the
// chip, each with its own boundary row in the scratch.
int64_t wide_grid(int64_t ntasks) {
  const int64_t cap = 4096;
  return ntasks < cap ? ntasks : cap;
}

int pick_rows(const eapdtw_ctx *ctx, int r) {
  if (ctx->rows_per_group) return (int)ctx->rows_per_group;
  return r == 0 ? 8 : 4;
}

// Tile height the tiled kernel takes for a problem (the launch's choice).
int wide_h(const eapdtw_ctx *ctx, int64_t r, int64_t lrow, int64_t lcol) {
  const int h = wide_rows_for((int)r, (int)lrow, (int)lcol);
  return h == kWideFullRows && ctx->wide_rows == 32 ? 32 : h;
}

// Reads `nbytes` at scratch offset `off` back into the pinned buffer and waits.
int readback(eapdtw_ctx *ctx, size_t off, size_t nbytes) {
  int rc = ensure_pinned(ctx, nbytes);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(ctx->pinned, ctx->scratch + off, nbytes, hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return EAPDTW_OK;
}

// sum of one counter over its stripes
uint64_t counter_sum(const unsigned long long *cnt, int slot) {
  uint64_t t = 0;
  for (int s = 0; s < kCntStripes; ++s) t += cnt[s * kCntStride + slot];
  return t;
}

void fill_stats(eapdtw_stats *st, const unsigned long long *cnt, uint64_t nominal,
                uint64_t problems, float ms, float main_ms = -1.f) {
  if (!st) return;
  st->cells_nominal = nominal;
  st->cells_evaluated = counter_sum(cnt, kCntEvaluated);
  st->cells_computed = counter_sum(cnt, kCntComputed);
  st->problems = problems;
  st->abandoned = counter_sum(cnt, kCntAbandoned);
  st->kernel_ms = ms;
  st->main_kernel_ms = main_ms < 0.f ? ms : main_ms;
}

// elapsed time between two recorded events (0 when unavailable)
float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    ms = 0.f;
  }
  return ms;
}

}  // namespace

extern "C" {

const char *eapdtw_version(void) { return "eapdtw 0.1 gfx950"; }

// ---------------------------------------------------------------------------
// Scratch of eapdtw_nn_search_noalloc: a fixed device array (one copy per GPU,
// held until the process ends) instead of the context's allocated scratch.
// Host code uses the device address hipGetSymbolAddress returns for the GPU,
// never the array's name (which is a host-side stand-in).
constexpr size_t kNoAllocScratchBytes = 64 * 1024;
constexpr int64_t kNoAllocMaxM = 4096;
constexpr int kNoAllocMaxDevices = 64;
static __device__ __align__(256) unsigned char g_noalloc_scratch[kNoAllocScratchBytes];
static std::mutex g_noalloc_mu;
static char *g_noalloc_ptr[kNoAllocMaxDevices] = {};

// Looks the array's address up once per device (the device must be current).
static char *noalloc_scratch(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_noalloc_scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_noalloc_ptr[device] = static_cast<char *>(p);
  }
  return g_noalloc_ptr[device];
}

int eapdtw_create(int device, void *hip_stream, eapdtw_ctx **out) {
  g_create_error.clear();
  if (!out) {
    g_create_error = "out is NULL";
    return EAPDTW_EINVAL;
  }
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    g_create_error = "no HIP device";
    return EAPDTW_ENODEV;
  }
  if (device < 0 || device >= n) {
    g_create_error = "device index out of range";
    return EAPDTW_ENODEV;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    g_create_error = "hipGetDeviceProperties failed";
    return EAPDTW_ENODEV;
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    g_create_error = std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950";
    return EAPDTW_ENODEV;
  }
  if (hipSetDevice(device) != hipSuccess) {
    g_create_error = "hipSetDevice failed";
    return EAPDTW_ENODEV;
  }
  eapdtw_ctx *c = new eapdtw_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (const char *lv = std::getenv("EAPDTW_LOG")) c->log = lv[0] && strcmp(lv, "0") != 0;
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
      hipEventCreate(&c->ev2) != hipSuccess || hipEventCreate(&c->ev3) != hipSuccess ||
      hipEventCreate(&c->ev_lb[0]) != hipSuccess || hipEventCreate(&c->ev_lb[1]) != hipSuccess ||
      hipEventCreate(&c->ev_lb[2]) != hipSuccess || hipEventCreate(&c->ev_lb[3]) != hipSuccess) {
    g_create_error = "hipEventCreate failed";
    delete c;
    return EAPDTW_EDEVICE;
  }
  // set-up of the allocation-free search: the device's scratch address and a
  // pinned read-back buffer large enough for its results
  c->noalloc = noalloc_scratch(device);
  if (ensure_pinned(c, 4096) != EAPDTW_OK) {
    g_create_error = "pinned host buffer allocation failed";
    eapdtw_destroy(c);
    return EAPDTW_ENOMEM;
  }
  *out = c;
  return EAPDTW_OK;
}

void eapdtw_destroy(eapdtw_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (!ctx->poisoned) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->scratch) (void)hipFree(ctx->scratch);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  if (ctx->ev2) (void)hipEventDestroy(ctx->ev2);
  if (ctx->ev3) (void)hipEventDestroy(ctx->ev3);
  for (hipEvent_t e : ctx->ev_lb)
    if (e) (void)hipEventDestroy(e);
  if (ctx->batch_exec) (void)hipGraphExecDestroy(ctx->batch_exec);
  if (ctx->batch_buf) (void)hipFree(ctx->batch_buf);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->seed_stream) {
    if (!ctx->poisoned) (void)hipStreamSynchronize(ctx->seed_stream);
    (void)hipStreamDestroy(ctx->seed_stream);
  }
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  for (int b = 0; b < eapdtw_ctx::kMaxBranches; ++b) {
    if (ctx->branch[b]) {
      if (!ctx->poisoned) (void)hipStreamSynchronize(ctx->branch[b]);
      (void)hipStreamDestroy(ctx->branch[b]);
    }
    if (ctx->ev_bjoin[b]) (void)hipEventDestroy(ctx->ev_bjoin[b]);
  }
  if (ctx->ev_bfork) (void)hipEventDestroy(ctx->ev_bfork);
  delete ctx;
}

int eapdtw_set_stream(eapdtw_ctx *ctx, void *hip_stream) {
  CHECK_CTX();
  if ((hipStream_t)hip_stream != ctx->stream) {
    // scratch may still be in use on the old stream; a stream that is being
    // captured into a graph cannot wait here (no synchronisation is allowed
    // during a capture): the capturing caller orders the two streams itself
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPCHK(hipStreamIsCapturing((hipStream_t)hip_stream, &cs));
    if (cs == hipStreamCaptureStatusNone) HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->stream = (hipStream_t)hip_stream;
  }
  return EAPDTW_OK;
}

const char *eapdtw_last_error(const eapdtw_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

static int64_t *option_slot(eapdtw_ctx *ctx, const char *key) {
  if (!key) return nullptr;
  if (!strcmp(key, "check_interval")) return &ctx->check_interval;
  if (!strcmp(key, "seed")) return &ctx->seed;
  if (!strcmp(key, "rows_per_group")) return &ctx->rows_per_group;
  if (!strcmp(key, "wide_rows")) return &ctx->wide_rows;
  if (!strcmp(key, "graph")) return &ctx->graph;
  if (!strcmp(key, "force_wide")) return &ctx->force_wide;
  if (!strcmp(key, "seed_stride")) return &ctx->seed_stride;
  if (!strcmp(key, "seed_window")) return &ctx->seed_window;
  if (!strcmp(key, "batch_grid")) return &ctx->batch_grid;
  if (!strcmp(key, "batch_chunk")) return &ctx->batch_chunk;
  if (!strcmp(key, "batch_seed_stride")) return &ctx->batch_seed_stride;
  if (!strcmp(key, "batch_branches")) return &ctx->batch_branches;
  if (!strcmp(key, "border")) return &ctx->border;
  if (!strcmp(key, "ed")) return &ctx->ed;
  if (!strcmp(key, "autotune")) return &ctx->autotune;
  if (!strcmp(key, "lanes")) return &ctx->lanes;
  if (!strcmp(key, "lb_ec")) return &ctx->lb_ec;
  if (!strcmp(key, "lb_probe_div")) return &ctx->lb_probe_div;
  if (!strcmp(key, "wf_lanes")) return &ctx->wf_lanes;
  if (!strcmp(key, "scratch_limit")) return &ctx->scratch_limit;
  if (!strcmp(key, "inject_fault")) return &ctx->inject_fault;
  if (!strcmp(key, "log")) return &ctx->log;
  return nullptr;
}

int eapdtw_set_option(eapdtw_ctx *ctx, const char *key, int64_t value) {
  if (!ctx) return EAPDTW_EINVAL;
  int64_t *slot = option_slot(ctx, key);
  if (!slot) return fail(ctx, EAPDTW_EINVAL, std::string("unknown option ") + (key ? key : "(null)"));
  bool ok = true;
  if (!strcmp(key, "check_interval")) ok = value >= 0 && value <= (1 << 20);
  else if (!strcmp(key, "seed") || !strcmp(key, "graph") || !strcmp(key, "force_wide") ||
           !strcmp(key, "border") || !strcmp(key, "ed") || !strcmp(key, "autotune") ||
           !strcmp(key, "lanes") || !strcmp(key, "lb_ec") || !strcmp(key, "log"))
    ok = value == 0 || value == 1;
  else if (!strcmp(key, "lb_probe_div")) ok = value == 0 || (value >= 2 && value <= 4096);
  else if (!strcmp(key, "wf_lanes")) ok = value == 0 || value == 16 || value == 32 || value == 64;
  else if (!strcmp(key, "scratch_limit")) ok = value >= 0;
  else if (!strcmp(key, "inject_fault")) ok = value == 0 || value == 1;
  else if (!strcmp(key, "rows_per_group")) ok = value == 0 || value == 2 || value == 4 || value == 8;
  else if (!strcmp(key, "wide_rows")) ok = value == 0 || value == 32 || value == 64;
  else if (!strcmp(key, "seed_stride")) ok = value >= 0 && value <= (1 << 20);
  else if (!strcmp(key, "seed_window")) ok = value >= 0 && value <= kBandRMax;
  else if (!strcmp(key, "batch_grid")) ok = value >= 64 && value <= 65536;
  else if (!strcmp(key, "batch_chunk")) ok = value >= 1 && value <= 1024;
  else if (!strcmp(key, "batch_seed_stride")) ok = value >= 0 && value <= (1 << 20);
  else if (!strcmp(key, "batch_branches")) ok = value >= 1 && value <= eapdtw_ctx::kMaxBranches;
  if (!ok) return fail(ctx, EAPDTW_EINVAL, std::string("bad value for option ") + key);
  *slot = value;
  return EAPDTW_OK;
}

int eapdtw_get_option(const eapdtw_ctx *ctx, const char *key, int64_t *value) {
  if (!ctx || !value) return EAPDTW_EINVAL;
  int64_t *slot = option_slot(const_cast<eapdtw_ctx *>(ctx), key);
  if (!slot) return EAPDTW_EINVAL;
  *value = *slot;
  return EAPDTW_OK;
}

// --------------------------------------------------------------------------- pair engine

// Every call's scratch starts with the striped counters.
// ... followed by one 256-byte line holding the non-finite flag word.
constexpr size_t kCntBytes = sizeof(unsigned long long) * kCntWords + 256;

static bool use_band(const eapdtw_ctx *ctx, int64_t r) { return r <= kBandRMax && !ctx->force_wide; }

// The window-0 seeding pass visits about this many blocks of 64 candidates
// (spread evenly over the series) unless a stride is set: one wave's
// 256-row pass costs ~11 us whatever the grid, so a pass over more blocks
// only adds waves, while the seeding workgroup tightens the bound anyway.
constexpr int64_t kSeedBlocks = 128;
static int64_t seed_stride_for(int64_t opt, int64_t nblk) {
  if (opt > 0) return opt;
  const int64_t s = nblk / kSeedBlocks;
  return s > 1 ? s : 1;
}

// DTW of pairs (rows X[p] of length lrow, columns Y[p] of length lcol), window
// r (already clipped to max(lrow,lcol)-1), bound per ub_mode.  Queues all
// device work on the context stream; with `stats` it also waits and fills them.
static int pairs_engine(eapdtw_ctx *ctx, const float *X, const float *Y, int64_t npairs,
                        int64_t lrow, int64_t lcol, int64_t r, int ub_mode, const float *ub,
                        float ub_scalar, float *out, eapdtw_stats *stats) {
  hipStream_t st = ctx->stream;
  const int64_t ld = (npairs + kWave - 1) / kWave * kWave;
  const bool band = use_band(ctx, r);
  Plan pl;
  const size_t o_cnt = pl.add(kCntBytes);
  const size_t o_rows = pl.add(sizeof(float) * lrow * ld);
  const size_t o_cols = pl.add(sizeof(float) * (lcol + (band ? 2 * kColPad : 0)) * ld);
  const int64_t ntasks = ld / kWave;
  const int64_t grid = wide_grid(ntasks);
  const size_t o_bnd = band ? 0 : pl.add(sizeof(float) * grid * (lcol + 1) * kWave);
  int rc = ensure_scratch(ctx, pl.off);
  if (rc) return rc;
  unsigned long long *cnt = at<unsigned long long>(ctx, o_cnt);
  if (stats) HIPCHK(hipEventRecord(ctx->ev0, st));
  HIPCHK(launch_fill_u64(cnt, 0ull, kCntWords, st));
  HIPCHK(launch_transpose_pad(X, npairs, (int)lrow, ld, 0, 0.0f, at<float>(ctx, o_rows), st));
  HIPCHK(launch_transpose_pad(Y, npairs, (int)lcol, ld, band ? kColPad : 0, INFINITY,
                              at<float>(ctx, o_cols), st));
  if (stats) HIPCHK(hipEventRecord(ctx->ev2, st));
  if (band) {
    PairArgs a{};
    a.rowsT = at<float>(ctx, o_rows);
    a.colsT = at<float>(ctx, o_cols);
    a.ld = ld;
    a.npairs = npairs;
    a.lrow = (int)lrow;
    a.lcol = (int)lcol;
    a.ub_mode = ub_mode;
    a.ub = ub;
    a.ub_scalar = ub_scalar;
    a.out = out;
    a.counters = cnt;
    HIPCHK(pair_band_launcher((int)r)(a, ntasks, pick_rows(ctx, (int)r), st));
    log_launch(ctx, "pairs %lld x (%lld, %lld) r=%lld: pair_band_kernel<%lld,%d> grid=%lld", (long long)npairs,
               (long long)lrow, (long long)lcol, (long long)r, (long long)r, pick_rows(ctx, (int)r),
               (long long)ntasks);
  } else {
    WideArgs w{};
    w.lrow = (int)lrow;
    w.lcol = (int)lcol;
    w.r = (int)r;
    w.RT = at<float>(ctx, o_rows);
    w.XT = at<float>(ctx, o_cols);
    w.N = npairs;
    w.ld = ld;
    w.ub_mode = ub_mode;
    w.ub = ub;
    w.ub_scalar = ub_scalar;
    w.out = out;
    w.ntasks = ntasks;
    w.bnd = at<float>(ctx, o_bnd);
    w.bnd_stride = (lcol + 1) * kWave;
    w.counters = cnt;
    w.check_interval = 1;
    HIPCHK(launch_wide(kWidePairs, (int)ctx->wide_rows, w, (int)grid, st));
    log_launch(ctx, "pairs %lld x (%lld, %lld) r=%lld: wide_kernel<%d,pairs> %lld blocks of 64 on %lld waves",
               (long long)npairs, (long long)lrow, (long long)lcol, (long long)r, wide_h(ctx, r, lrow, lcol),
               (long long)ntasks, (long long)grid);
  }
  if (stats) {
    HIPCHK(hipEventRecord(ctx->ev3, st));
    HIPCHK(hipEventRecord(ctx->ev1, st));
    rc = readback(ctx, o_cnt, kCntBytes);
    if (rc) return rc;
    fill_stats(stats, reinterpret_cast<unsigned long long *>(ctx->pinned),
               (uint64_t)(band_cells_total(lrow, lcol, r) * npairs), (uint64_t)npairs,
               elapsed(ctx->ev0, ctx->ev1), elapsed(ctx->ev2, ctx->ev3));
  }
  return EAPDTW_OK;
}

// --------------------------------------------------------------------------- single pair

int eapdtw_dtw(eapdtw_ctx *ctx, const float *S, int64_t lS, const float *T, int64_t lT,
               int64_t window, double ub, double *out_dist, eapdtw_stats *stats) {
  CHECK_CTX();
  if (!out_dist) return fail(ctx, EAPDTW_EINVAL, "out_dist is NULL");
  if (lS < 0 || lT < 0) return fail(ctx, EAPDTW_EINVAL, "negative length");
  if (window < 0) return fail(ctx, EAPDTW_EINVAL, "window < 0");
  if (std::isnan(ub)) return fail(ctx, EAPDTW_EINVAL, "ub is NaN");
  if ((lS > 0 && !S) || (lT > 0 && !T)) return fail(ctx, EAPDTW_EINVAL, "NULL series");
  if (lS > INT_MAX / 2 || lT > INT_MAX / 2) return fail(ctx, EAPDTW_EINVAL, "series too long");
  if (stats) std::memset(stats, 0, sizeof *stats);
  // Eq. 2-4 borders and the empty-window case need no device work
  if (lS == 0 && lT == 0) {
    *out_dist = ub >= 0 ? 0.0 : INFINITY;
    return EAPDTW_OK;
  }
  if (lS == 0 || lT == 0 || std::llabs(lS - lT) > window || ub < 0) {
    *out_dist = INFINITY;
    return EAPDTW_OK;
  }
  const int64_t lmax = lS > lT ? lS : lT;
  const int64_t r = window < lmax - 1 ? window : lmax - 1;
  HIPCHK(hipSetDevice(ctx->device));
  // the single result is written into a scratch word placed after the engine's buffers
  Plan pl;
  pl.add(kCntBytes);
  const int64_t ld = kWave;
  pl.add(sizeof(float) * lS * ld);
  pl.add(sizeof(float) * (lT + 2 * kColPad) * ld);
  if (!use_band(ctx, r)) pl.add(sizeof(float) * 1 * (lT + 1) * kWave);
  const size_t o_out = pl.add(sizeof(float));
  int rc = ensure_scratch(ctx, pl.off);
  if (rc) return rc;
  rc = pairs_engine(ctx, S, T, 1, lS, lT, r, 3, nullptr, bound_down(ub), at<float>(ctx, o_out),
                    stats);
  if (rc) return rc;
  rc = readback(ctx, o_out, sizeof(float));
  if (rc) return rc;
  *out_dist = (double)*reinterpret_cast<float *>(ctx->pinned);
  return EAPDTW_OK;
}

// --------------------------------------------------------------------------- pairs

static int pairs_common(eapdtw_ctx *ctx, const float *X, const float *Y, int64_t npairs,
                        int64_t len, int64_t window, int ub_mode, const float *ub, float *out,
                        eapdtw_stats *stats) {
  if (npairs < 0 || len < 0) return fail(ctx, EAPDTW_EINVAL, "negative size");
  if (window < 0) return fail(ctx, EAPDTW_EINVAL, "window < 0");
  if (ub_mode < 0 || ub_mode > 2) return fail(ctx, EAPDTW_EINVAL, "ub_mode must be 0, 1 or 2");
  if (npairs > 0 && (!X || !Y || !out)) return fail(ctx, EAPDTW_EINVAL, "NULL pointer");
  if (ub_mode == 1 && npairs > 0 && !ub) return fail(ctx, EAPDTW_EINVAL, "ub is NULL with ub_mode 1");
  if (len > INT_MAX / 2) return fail(ctx, EAPDTW_EINVAL, "series too long");
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (npairs == 0) return EAPDTW_OK;
  HIPCHK(hipSetDevice(ctx->device));
  if (len == 0) {
    HIPCHK(launch_fill_f32(out, 0.0f, npairs, ctx->stream));
    return EAPDTW_OK;
  }
  const int64_t r = window < len - 1 ? window : len - 1;
  return pairs_engine(ctx, X, Y, npairs, len, len, r, ub_mode, ub, 0.0f, out, stats);
}

int eapdtw_dtw_pairs(eapdtw_ctx *ctx, const float *X, const float *Y, int64_t npairs, int64_t len,
                     int64_t window, int ub_mode, const float *ub, float *out, eapdtw_stats *stats) {
  CHECK_CTX();
  return pairs_common(ctx, X, Y, npairs, len, window, ub_mode, ub, out, stats);
}

int eapdtw_erp_pairs(eapdtw_ctx *ctx, const float *X, const float *Y, int64_t npairs, int64_t len,
                     int64_t window, double g, const float *ub, float *out, eapdtw_stats *stats) {
  CHECK_CTX();
  if (npairs < 0 || len < 0) return fail(ctx, EAPDTW_EINVAL, "negative size");
  if (window < 0) return fail(ctx, EAPDTW_EINVAL, "window < 0");
  if (npairs > 0 && (!out || (len > 0 && (!X || !Y)))) return fail(ctx, EAPDTW_EINVAL, "NULL pointer");
  if (!std::isfinite(g) || std::fabs(g) > FLT_MAX) return fail(ctx, EAPDTW_EINVAL, "g must be a finite float32");
  if (len > INT_MAX / 2) return fail(ctx, EAPDTW_EINVAL, "series too long");
  if (npairs > (int64_t)INT_MAX - kWave) return fail(ctx, EAPDTW_EINVAL, "too many pairs");
  const int64_t r = len > 0 && window > len - 1 ? len - 1 : window;
  if (len > 0 && r > kErpMaxR)
    return fail(ctx, EAPDTW_EINVAL, "ERP takes windows up to 64 (after clamping to len - 1)");
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (npairs == 0) return EAPDTW_OK;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  if (len == 0) {
    HIPCHK(launch_fill_f32(out, 0.0f, npairs, st));
    return EAPDTW_OK;
  }
  const int64_t ld = (npairs + kWave - 1) / kWave * kWave;
  Plan pl;
  const size_t o_cnt = pl.add(kCntBytes);
  const size_t o_xt = pl.add(sizeof(float) * len * ld);
  const size_t o_yt = pl.add(sizeof(float) * len * ld);
  int rc = ensure_scratch(ctx, pl.off);
  if (rc) return rc;
  unsigned long long *cnt = at<unsigned long long>(ctx, o_cnt);
  if (stats) HIPCHK(hipEventRecord(ctx->ev0, st));
  HIPCHK(launch_fill_u64(cnt, 0ull, kCntWords, st));
  HIPCHK(launch_transpose_pad(X, npairs, (int)len, ld, 0, 0.0f, at<float>(ctx, o_xt), st));
  HIPCHK(launch_transpose_pad(Y, npairs, (int)len, ld, 0, 0.0f, at<float>(ctx, o_yt), st));
  if (stats) HIPCHK(hipEventRecord(ctx->ev2, st));
  ErpArgs e{};
  e.Xt = at<float>(ctx, o_xt);
  e.Yt = at<float>(ctx, o_yt);
  e.ld = ld;
  e.npairs = npairs;
  e.len = (int)len;
  e.g = (float)g;
  e.ub = ub;
  e.out = out;
  e.counters = cnt;
  HIPCHK(launch_erp_pairs((int)r, e, st));
  log_launch(ctx, "erp pairs: %lld pairs of length %lld, r=%lld: erp_pairs_kernel<%lld> grid=%lld",
             (long long)npairs, (long long)len, (long long)r, (long long)r, (long long)(ld / kWave));
  if (stats) {
    HIPCHK(hipEventRecord(ctx->ev3, st));
    HIPCHK(hipEventRecord(ctx->ev1, st));
    rc = readback(ctx, o_cnt, kCntBytes);
    if (rc) return rc;
    fill_stats(stats, reinterpret_cast<unsigned long long *>(ctx->pinned),
               (uint64_t)(band_cells_total(len, len, r) * npairs), (uint64_t)npairs,
               elapsed(ctx->ev0, ctx->ev1), elapsed(ctx->ev2, ctx->ev3));
  }
  return EAPDTW_OK;
}

int eapdtw_pairwise(eapdtw_ctx *ctx, const float *X, int64_t N, int64_t len, int64_t window,
                    float *out_D, eapdtw_stats *stats) {
  CHECK_CTX();
  if (N < 0 || len < 0) return fail(ctx, EAPDTW_EINVAL, "negative size");
  if (window < 0) return fail(ctx, EAPDTW_EINVAL, "window < 0");
  if (N > 1 && (!X || !out_D)) return fail(ctx, EAPDTW_EINVAL, "NULL pointer");
  if (len > INT_MAX / 2 || N > (int64_t)1 << 31) return fail(ctx, EAPDTW_EINVAL, "too large");
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (N < 2) return EAPDTW_OK;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const int64_t npairs = N * (N - 1) / 2;
  if (len == 0) {
    HIPCHK(launch_fill_f32(out_D, 0.0f, npairs, st));
    return EAPDTW_OK;
  }
  const int64_t r = window < len - 1 ? window : len - 1;
  const int64_t ldN = (N + kWave - 1) / kWave * kWave;
  const int64_t nblk_j = ldN / kWave;
  const int64_t ntasks = N * nblk_j;
  const int64_t grid = wide_grid(ntasks);
  Plan pl;
  const size_t o_cnt = pl.add(kCntBytes);
  const size_t o_xt = pl.add(sizeof(float) * len * ldN);
  const size_t o_bnd = pl.add(sizeof(float) * grid * (len + 1) * kWave);
  int rc = ensure_scratch(ctx, pl.off);
  if (rc) return rc;
  unsigned long long *cnt = at<unsigned long long>(ctx, o_cnt);
  if (stats) HIPCHK(hipEventRecord(ctx->ev0, st));
  HIPCHK(launch_fill_u64(cnt, 0ull, kCntWords, st));
  HIPCHK(launch_transpose_pad(X, N, (int)len, ldN, 0, 0.0f, at<float>(ctx, o_xt), st));
  WideArgs w{};
  w.lrow = (int)len;
  w.lcol = (int)len;
  w.r = (int)r;
  w.X = X;
  w.XT = at<float>(ctx, o_xt);
  w.N = N;
  w.ld = ldN;
  w.nblk_j = nblk_j;
  w.ub_mode = 2;
  w.out = out_D;
  w.ntasks = ntasks;
  w.bnd = at<float>(ctx, o_bnd);
  w.bnd_stride = (len + 1) * kWave;
  w.counters = cnt;
  w.check_interval = 1;
  if (stats) HIPCHK(hipEventRecord(ctx->ev2, st));
  HIPCHK(launch_wide(kWidePairwise, (int)ctx->wide_rows, w, (int)grid, st));
  log_launch(ctx, "%s rows %lld x %lld columns of length %d, r=%d: wide_kernel<%d,pairwise> %lld tasks on %lld waves",
             w.nn1 ? "nn1" : "pairwise", (long long)(w.nq ? w.nq : w.N), (long long)w.N, w.lrow, w.r,
             wide_h(ctx, w.r, w.lrow, w.lcol), (long long)w.ntasks, (long long)grid);
  if (stats) {
    HIPCHK(hipEventRecord(ctx->ev3, st));
    HIPCHK(hipEventRecord(ctx->ev1, st));
    rc = readback(ctx, o_cnt, kCntBytes);
    if (rc) return rc;
    fill_stats(stats, reinterpret_cast<unsigned long long *>(ctx->pinned),
               (uint64_t)(band_cells_total(len, len, r) * npairs), (uint64_t)npairs,
               elapsed(ctx->ev0, ctx->ev1), elapsed(ctx->ev2, ctx->ev3));
  }
  return EAPDTW_OK;
}

// --------------------------------------------------------------------------- search

static int search_validate(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                           int64_t n, int64_t window) {
  if (!query || !series) return fail(ctx, EAPDTW_EINVAL, "NULL series");
  if (m <= 0) return fail(ctx, EAPDTW_EINVAL, "query length must be positive");
  if (n < m) return fail(ctx, EAPDTW_EINVAL, "series shorter than the query");
  if (window < 0) return fail(ctx, EAPDTW_EINVAL, "window < 0");
  if (m > INT_MAX / 4) return fail(ctx, EAPDTW_EINVAL, "query too long");
  if (n - m + 1 > (int64_t)0xfffffffe) return fail(ctx, EAPDTW_EINVAL, "too many candidate offsets");
  return EAPDTW_OK;
}

// Queues the search of one query: query normalisation into qpad, bound
// seeding, and the DP pass over offsets [0, n-m].  dists != nullptr selects the
// per-candidate mode against fixed_ub (no best-so-far).  bsf points at two
// words (search, seeding pass); cnt at cleared counters.
// Device buffers of the lower-bound cascade (see LBArgs / NNArgs list mode).
struct LbBufs {
  float *ux, *lx, *uq, *lq;                           // envelopes [n], [n], [m], [m]
  uint32_t *lk;                                       // survivor list [K]
  float *lmh, *lml, *linv, *lbq, *lbmax;              // [K] each
};

static void lb_plan(Plan &pl, size_t *offs, int64_t n, int64_t m, int64_t K) {
  offs[0] = pl.add(sizeof(float) * n);
  offs[1] = pl.add(sizeof(float) * n);
  offs[2] = pl.add(sizeof(float) * m);
  offs[3] = pl.add(sizeof(float) * m);
  for (int i = 0; i < 6; ++i) offs[4 + i] = pl.add(sizeof(float) * K);
}

static LbBufs lb_bind(eapdtw_ctx *ctx, const size_t *offs) {
  return LbBufs{at<float>(ctx, offs[0]), at<float>(ctx, offs[1]), at<float>(ctx, offs[2]),
                at<float>(ctx, offs[3]), at<uint32_t>(ctx, offs[4]), at<float>(ctx, offs[5]),
                at<float>(ctx, offs[6]), at<float>(ctx, offs[7]), at<float>(ctx, offs[8]),
                at<float>(ctx, offs[9])};
}

// Device buffers of the k-nearest-neighbour search: the kept candidates and
// their count (a counter word, cleared by the set-up kernel).
struct KnnBufs {
  int k;
  unsigned long long *buf, *n;
};

// The second stream (and its fork/join events) of the concurrent seeding.
static hipError_t ensure_seed_stream(eapdtw_ctx *ctx) {
  if (ctx->seed_stream) return hipSuccess;
  hipError_t e = hipStreamCreateWithFlags(&ctx->seed_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming);
  return e;
}

// The cascade serves band windows from 1 on (at window 0 LB_Keogh is the
// squared Euclidean distance itself, which the window-0 kernel computes).
// The cascade runs in front of the band kernels' list mode, and for windows
// above them (up to kEnvMaxR) in front of the tiled kernel's list kernel.
static bool lb_applies(const eapdtw_ctx *ctx, int64_t r) {
  return r >= 1 && (use_band(ctx, r) || (r > kBandRMax && r <= kEnvMaxR));
}

static int search_queue(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                        int64_t n, int64_t r, float *qpad, unsigned long long *bsf,
                        unsigned long long *cnt, float *dists, float fixed_ub, float *bnd,
                        int64_t bnd_waves, bool time_main, const LbBufs *lb = nullptr,
                        const KnnBufs *kb = nullptr, const float *wgt = nullptr,
                        bool one_stream = false, const float *wt_dev = nullptr) {
  hipStream_t st = ctx->stream;
  const int64_t K = n - m + 1;
  const int64_t nblk = (K + kWave - 1) / kWave;
  if (++ctx->epoch == 0) ++ctx->epoch;
  HIPCHK(launch_search_prep(query, (int)m, qpad, dists ? nullptr : series, n, cnt,
                            dists ? nullptr : bsf, dists ? 0 : 2,
                            reinterpret_cast<unsigned *>(cnt + kCntWords), ctx->epoch, st));
  NNArgs a{};
  a.x = series;
  a.n = n;
  a.m = (int)m;
  a.qpad = qpad;
  a.k_begin = 0;
  a.k_end = K;
  a.check_interval = (int)ctx->check_interval;
  a.block_stride = 1;
  // weighted DTW: the weights of phase differences 0..r (the unweighted
  // window-0 seeding pass stays valid: every weight is at most 1, so the
  // squared Euclidean distance bounds the weighted diagonal path's cost)
  // (above the band kernels' windows only the seeding workgroup's narrower
  // window reads them; the tiled kernel takes wt_dev)
  if (wgt) std::memcpy(a.wgt, wgt, sizeof(float) * (size_t)((r < kBandRMax ? r : kBandRMax) + 1));
  bool joined = true;
  if (!dists && ctx->seed) {
    // Bound seeding.  A candidate's DTW under a narrower window is never below
    // its DTW under the search window (fewer admissible paths), so
    //  1. the window-0 (squared Euclidean) pass over every seed_stride-th
    //     block of candidates yields a valid distance bound and an offset;
    //  2. one workgroup over the search's 64-offset block holding that
    //     offset, under window min(r, seed_window), tightens it.
    // Both record distance-only bounds; the search itself then finds the
    // exact minimum and its offset.  The true minimum is never abandoned:
    // the seeding workgroup normalises its candidates with the search's own
    // block statistics (the same float32 z-values), and float32 addition is
    // monotone, so its distance for any candidate is never below the
    // search's distance for that candidate.
    // The band search starts from the window-0 bound and the seeding
    // workgroup runs beside it on a second stream: its bound reaches the
    // search's waves through their periodic reads of the best-so-far.
    // (Running this pass beside the search too, so that the search's waves
    // start at once from +inf, was slower on C2: 2.24-2.31 against 2.11-2.32
    // ms per step.)
    const int64_t sstr = seed_stride_for(ctx->seed_stride, nblk);
    NNArgs e = a;
    e.bsf = bsf + 1;
    e.block_stride = (int)sstr;
    if (ctx->ed)
      HIPCHK(launch_ed_search(e, (nblk + sstr - 1) / sstr, false, st));
    else
      HIPCHK(nn_band_launcher(0)(e, (nblk + sstr - 1) / sstr, 8, false, false, st));
    const int64_t rs = r < ctx->seed_window ? r : ctx->seed_window;
    NNArgs s = a;
    s.bsf = bsf;
    s.center = bsf + 1;
    s.bsf_init = bsf + 1;
    s.bound_only = 1;
    if (kb) {
      // k nearest neighbours: the window-0 pass only locates the seeding
      // workgroup (its minimum bounds the best, not the k-th best); the
      // workgroup publishes the k-th best of its 64 distances and appends
      // nothing (its distances are under a narrower window)
      s.bsf_init = nullptr;
      s.knn = kb->k;
    }
    hipStream_t ss = st;
    // (a k-NN search behind the cascade seeds on the search stream: its bound
    // pass has no window-0 bound to start from, the seed's k-th best is it)
    if (use_band(ctx, r) && !one_stream && !(kb && lb && lb_applies(ctx, r))) {
      HIPCHK(ensure_seed_stream(ctx));
      HIPCHK(hipEventRecord(ctx->ev_fork, st));
      HIPCHK(hipStreamWaitEvent(ctx->seed_stream, ctx->ev_fork, 0));
      ss = ctx->seed_stream;
      if (!kb) a.bsf_init = bsf + 1;  // the search's waves start from the window-0 bound
    }
    if (wgt)
      HIPCHK(nn_wband_launcher((int)rs)(s, 1, false, false, ss));
    else if (rs == 0 && ctx->ed && !kb)  // (the window-0 kernel publishes only the best)
      HIPCHK(launch_ed_search(s, 1, false, ss));
    else
      HIPCHK(nn_band_launcher((int)rs)(s, 1, pick_rows(ctx, (int)rs), false, false, ss));
    if (ss != st) {
      HIPCHK(hipEventRecord(ctx->ev_join, ss));
      joined = false;
    }
    log_launch(ctx, "search seeding: %s grid=%lld (every %lld-th block of 64), then %s window %lld, 1 workgroup%s",
               ctx->ed ? "ed_search_kernel" : "nn_band_kernel<0,8>", (long long)((nblk + sstr - 1) / sstr),
               (long long)sstr, wgt ? "nn_wband_kernel" : (rs == 0 && ctx->ed && !kb) ? "ed_search_kernel" : "nn_band_kernel",
               (long long)rs, ss != st ? " on the seed stream" : "");
  }
  if (time_main) HIPCHK(hipEventRecord(ctx->ev2, st));
  if (lb && lb_applies(ctx, r)) {
    // envelopes, then per range of candidates the bound pass (survivor list)
    // and the DP over the list.  A search first takes a probe range of
    // K / lb_probe_div candidates: its DP brings the best-so-far near its
    // final value before the bound pass over the remaining candidates, which
    // compares with the best-so-far of its start.
    HIPCHK(launch_envelopes(series, n, qpad + kColPad, (int)m, (int)r, lb->ux, lb->lx, lb->uq,
                            lb->lq, st));
    int64_t cut = 0;
    if (!dists && ctx->lb_probe_div > 0) {
      cut = (K / ctx->lb_probe_div + kWave - 1) / kWave * kWave;
      if (cut >= K) cut = 0;
    }
    const int64_t edges[3] = {0, cut ? cut : K, K};
    const int nranges = cut ? 2 : 1;
    ctx->lb_probe_two = cut != 0;
    for (int pi = 0, e = 0; pi < nranges; ++pi) {
      const int64_t lo = edges[pi], hi = edges[pi + 1];
      LBArgs la{};
      la.x = series;
      la.n = n;
      la.m = (int)m;
      la.r = (int)r;
      la.qz = qpad + kColPad;
      la.uq = lb->uq;
      la.lq = lb->lq;
      la.ux = lb->ux;
      la.lx = lb->lx;
      la.k_begin = lo;
      la.k_end = hi;
      la.mode = dists ? 1 : 0;
      la.bsf = bsf;
      la.bsf_init = a.bsf_init;
      la.fixed_ub = fixed_ub;
      la.dists = dists;
      la.use_ec = ctx->lb_ec != 0;
      la.counters = cnt;
      la.list_n = cnt + pi * kCntStride + kCntListN;
      la.list_k = lb->lk + lo;
      la.list_mh = lb->lmh + lo;
      la.list_ml = lb->lml + lo;
      la.list_inv = lb->linv + lo;
      la.list_lbq = lb->lbq + lo;
      la.list_lbmax = lb->lbmax + lo;
      HIPCHK(launch_lb_pass(la, st));
      if (time_main) HIPCHK(hipEventRecord(ctx->ev_lb[e++], st));
      NNArgs b = a;
      b.bsf = bsf;
      b.counters = cnt;
      b.fixed_ub = fixed_ub;
      b.dists = dists;
      b.list_n = la.list_n;
      b.list_k = la.list_k;
      b.list_mh = la.list_mh;
      b.list_ml = la.list_ml;
      b.list_inv = la.list_inv;
      b.list_lbq = la.list_lbq;
      b.list_lbmax = la.list_lbmax;
      b.uq = lb->uq;
      b.lq = lb->lq;
      if (kb) {
        b.knn = kb->k;
        b.knn_buf = kb->buf;
        b.knn_n = kb->n;
      }
      if (use_band(ctx, r)) {
        HIPCHK(nn_list_launcher((int)r)(b, (hi - lo + kWave - 1) / kWave, dists != nullptr,
                                        ctx->border != 0, st));
        log_launch(ctx, "search m=%lld r=%lld candidates %lld..%lld: envelope_kernel, lb_pass_kernel, "
                   "nn_list_kernel<%lld,4,border=%d> grid=%lld", (long long)m, (long long)r,
                   (long long)lo, (long long)hi, (long long)r, ctx->border != 0,
                   (long long)((hi - lo + kWave - 1) / kWave));
      } else {
        // windows above the band kernels': the tiled kernel over the list
        WideArgs w{};
        w.lrow = (int)m;
        w.lcol = (int)m;
        w.r = (int)r;
        w.x = series;
        w.n = n;
        w.qpad = qpad;
        w.bsf = bsf;
        w.k_begin = 0;
        w.k_end = K;
        w.fixed_ub = fixed_ub;
        w.dists = dists;
        w.dists_mode = dists != nullptr;
        w.ntasks = (hi - lo + kWave - 1) / kWave;
        w.bnd = bnd;
        w.bnd_stride = (m + 1) * kWave;
        w.counters = cnt;
        w.check_interval = (int)ctx->check_interval;
        w.list_n = la.list_n;
        w.list_k = la.list_k;
        w.list_mh = la.list_mh;
        w.list_ml = la.list_ml;
        w.list_inv = la.list_inv;
        w.list_lbmax = la.list_lbmax;
        w.list_lbq = la.list_lbq;
        w.uq = lb->uq;
        w.lq = lb->lq;
        if (kb) {
          w.knn = kb->k;
          w.knn_buf = kb->buf;
          w.knn_n = kb->n;
        }
        const int64_t g = bnd_waves < w.ntasks ? bnd_waves : w.ntasks;
        HIPCHK(launch_wide_list((int)ctx->wide_rows, w, (int)g, st));
        log_launch(ctx, "search m=%lld r=%lld candidates %lld..%lld: envelope_kernel, lb_pass_kernel, "
                   "wide_list_kernel<%d> on %lld persistent waves", (long long)m, (long long)r,
                   (long long)lo, (long long)hi, wide_h(ctx, r, m, m), (long long)g);
      }
      if (time_main && pi + 1 < nranges) HIPCHK(hipEventRecord(ctx->ev_lb[e++], st));
    }
  } else if (use_band(ctx, r) || (wgt && r <= kBandRMax)) {
    a.bsf = bsf;
    a.counters = cnt;
    a.fixed_ub = fixed_ub;
    a.dists = dists;
    const bool bord = ctx->border != 0 && r >= kBorderMinR;
    if (wgt) {
      HIPCHK(nn_wband_launcher((int)r)(a, nblk, dists != nullptr, ctx->border != 0, st));
      log_launch(ctx, "search m=%lld r=%lld: nn_wband_kernel<%lld,4,border=%d> grid=%lld", (long long)m,
                 (long long)r, (long long)r, bord, (long long)nblk);
    } else if (kb) {
      a.knn = kb->k;
      a.knn_buf = kb->buf;
      a.knn_n = kb->n;
      HIPCHK(nn_band_launcher((int)r)(a, nblk, 4, false, ctx->border != 0, st));
      log_launch(ctx, "search m=%lld r=%lld k=%d: nn_band_kernel<%lld,4,border=%d> grid=%lld", (long long)m,
                 (long long)r, kb->k, (long long)r, bord, (long long)nblk);
    } else if (r == 0 && ctx->ed) {
      HIPCHK(launch_ed_search(a, nblk, dists != nullptr, st));
      log_launch(ctx, "search m=%lld r=0: ed_search_kernel grid=%lld", (long long)m, (long long)nblk);
    } else if (!dists && ctx->lanes && lane_search_supported((int)r, (int)m)) {
      HIPCHK(launch_lane_search((int)r, a, st));
      log_launch(ctx, "search m=%lld r=%lld: lane-refill kernel", (long long)m, (long long)r);
    } else {
      const int u = dists ? 4 : pick_rows(ctx, (int)r);
      HIPCHK(nn_band_launcher((int)r)(a, nblk, u, dists != nullptr, ctx->border != 0, st));
      log_launch(ctx, "search m=%lld r=%lld: nn_band_kernel<%lld,%d,border=%d> grid=%lld", (long long)m,
                 (long long)r, (long long)r, u, bord, (long long)nblk);
    }
  } else {
    WideArgs w{};
    w.lrow = (int)m;
    w.lcol = (int)m;
    w.r = (int)r;
    w.x = series;
    w.n = n;
    w.qpad = qpad;
    w.bsf = bsf;
    w.k_begin = 0;
    w.k_end = K;
    w.fixed_ub = fixed_ub;
    w.dists = dists;
    w.dists_mode = dists != nullptr;
    w.ntasks = nblk;
    w.bnd = bnd;
    w.bnd_stride = (m + 1) * kWave;
    w.counters = cnt;
    w.check_interval = (int)ctx->check_interval;
    if (kb) {
      w.knn = kb->k;
      w.knn_buf = kb->buf;
      w.knn_n = kb->n;
    }
    w.wt_band = wt_dev;
    HIPCHK(launch_wide(wgt ? kWideSearchW : kWideSearch, (int)ctx->wide_rows, w,
                       (int)(bnd_waves < nblk ? bnd_waves : nblk), st));
    log_launch(ctx, "search m=%lld r=%lld: wide_kernel<%d,search> %lld blocks of 64 on %lld persistent waves",
               (long long)m, (long long)r, wide_h(ctx, r, m, m), (long long)nblk,
               (long long)(bnd_waves < nblk ? bnd_waves : nblk));
  }
  if (time_main) HIPCHK(hipEventRecord(ctx->ev3, st));
  if (!joined) HIPCHK(hipStreamWaitEvent(st, ctx->ev_join, 0));
  return EAPDTW_OK;
}

// --------------------------------------------------------------------------- tuning

int64_t eapdtw_tune_bucket(int64_t m, int64_t window) {
  if (m < 1 || window < 0) return -1;
  auto bits = [](int64_t v) { int b = 0; while (v) { ++b; v >>= 1; } return (int64_t)b; };
  const int64_t r = window < m - 1 ? window : m - 1;
  int64_t rb;
  if (m > 1 && r >= m - 1) rb = 31;
  else if (r == 0) rb = 0;
  else if (r <= kBandRMax) rb = bits(r);
  else rb = 8 + bits(r);
  return 32 * bits(m) + rb;
}

namespace {

// Applies a bucket's tuned choices to the context for one call and restores
// the previous ones afterwards.
struct KnobGuard {
  eapdtw_ctx *ctx;
  int64_t rows, border, ci, wide, lanes;
  explicit KnobGuard(eapdtw_ctx *c)
      : ctx(c), rows(c->rows_per_group), border(c->border), ci(c->check_interval),
        wide(c->wide_rows), lanes(c->lanes) {}
  void apply(const eapdtw_tune &t) {
    ctx->rows_per_group = t.rows_per_group;
    ctx->border = t.border;
    ctx->check_interval = t.check_interval;
    ctx->wide_rows = t.wide_rows;
    ctx->lanes = t.lanes;
  }
  void apply_cached(int64_t m, int64_t window) {
    if (!ctx->autotune) return;
    auto it = ctx->tune.find(eapdtw_tune_bucket(m, window));
    if (it != ctx->tune.end()) apply(it->second);
  }
  ~KnobGuard() {
    ctx->rows_per_group = rows;
    ctx->border = border;
    ctx->check_interval = ci;
    ctx->wide_rows = wide;
    ctx->lanes = lanes;
  }
};

}  // namespace

// Splits a timed cascade call into bound passes and DP passes: events ev2,
// ev_lb[0] (after the first bound pass), then with a probe range ev_lb[1]
// (after its DP), ev_lb[2] (after the second bound pass), and ev3.
static void lb_split_times(eapdtw_ctx *ctx) {
  const float total = elapsed(ctx->ev2, ctx->ev3);
  float lbt = elapsed(ctx->ev2, ctx->ev_lb[0]);
  if (ctx->lb_probe_two) lbt += elapsed(ctx->ev_lb[1], ctx->ev_lb[2]);
  ctx->lb_ms = lbt;
  ctx->lb_dp_ms = total - lbt;
}

static void fill_lb_stats(eapdtw_lb_stats *ls, const unsigned long long *cnt, bool applied,
                          uint64_t K, float lb_ms) {
  if (!ls) return;
  std::memset(ls, 0, sizeof *ls);
  if (!applied) {
    ls->dtw_candidates = K;
    return;
  }
  ls->pruned_kim = counter_sum(cnt, kCntLbKim);
  ls->pruned_keogh_eq = counter_sum(cnt, kCntLbEq);
  ls->pruned_keogh_ec = counter_sum(cnt, kCntLbEc);
  ls->pruned_recheck = counter_sum(cnt, kCntLbRecheck);
  ls->dtw_candidates = counter_sum(cnt, kCntListN) - ls->pruned_recheck;
  ls->lb_ms = lb_ms;
}

static int upload(eapdtw_ctx *ctx, size_t off, const void *src, size_t nbytes);

// Weighted search above the band kernels' windows: the 2r + 1 weights w(|d|),
// d = -r..r, for the tiled kernel's LDS (wgt holds w(0..r)), with kWtPad
// entries of 1 on each side.
static size_t band_weight_words(int64_t r) { return (size_t)(2 * r + 1 + 2 * kWtPad); }
static int upload_band_weights(eapdtw_ctx *ctx, size_t off, const float *wgt, int64_t r) {
  std::vector<float> t(band_weight_words(r), 1.0f);
  for (int64_t d = -r; d <= r; ++d) t[(size_t)(d + r + kWtPad)] = wgt[d < 0 ? -d : d];
  return upload(ctx, off, t.data(), sizeof(float) * t.size());
}

static int nn_search_impl(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                          int64_t n, int64_t window, int64_t *out_offset, double *out_dist,
                          eapdtw_stats *stats, bool use_lb, eapdtw_lb_stats *lbstats,
                          const float *wgt = nullptr) {
  CHECK_CTX();
  KnobGuard knobs(ctx);
  knobs.apply_cached(m, window);
  if (!out_offset || !out_dist) return fail(ctx, EAPDTW_EINVAL, "NULL output");
  int rc = search_validate(ctx, query, m, series, n, window);
  if (rc) return rc;
  if (stats) std::memset(stats, 0, sizeof *stats);
  const int64_t r = window < m - 1 ? window : m - 1;
  const int64_t K = n - m + 1;
  const int64_t grid = use_band(ctx, r) ? 0 : wide_grid((K + kWave - 1) / kWave);
  const bool lb_on = use_lb && lb_applies(ctx, r);
  const bool timed = stats != nullptr || lbstats != nullptr;
  Plan pl;
  const size_t o_cnt = pl.add(kCntBytes);
  const size_t o_bsf = pl.add(sizeof(unsigned long long) * 2);  // [0] search, [1] seeding pass
  const size_t o_q = pl.add(sizeof(float) * (m + 2 * kColPad));
  const size_t o_bnd = grid ? pl.add(sizeof(float) * grid * (m + 1) * kWave) : 0;
  const bool wide_w = wgt && r > kBandRMax;
  const size_t o_wt = wide_w ? pl.add(sizeof(float) * band_weight_words(r)) : 0;
  size_t o_lb[10];
  if (lb_on) lb_plan(pl, o_lb, n, m, K);
  rc = ensure_scratch(ctx, pl.off);
  if (rc) return rc;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  if (wide_w && (rc = upload_band_weights(ctx, o_wt, wgt, r))) return rc;
  unsigned long long *bsf = at<unsigned long long>(ctx, o_bsf);
  unsigned long long *cnt = at<unsigned long long>(ctx, o_cnt);
  LbBufs lbb{};
  if (lb_on) lbb = lb_bind(ctx, o_lb);
  if (timed) HIPCHK(hipEventRecord(ctx->ev0, st));
  rc = search_queue(ctx, query, m, series, n, r, at<float>(ctx, o_q), bsf, cnt, nullptr, 0.f,
                    grid ? at<float>(ctx, o_bnd) : nullptr, grid, timed, lb_on ? &lbb : nullptr,
                    nullptr, wgt, false, wide_w ? at<float>(ctx, o_wt) : nullptr);
  if (rc) return rc;
  if (timed) HIPCHK(hipEventRecord(ctx->ev1, st));
  // counters and the two best-so-far words are contiguous
  rc = readback(ctx, o_cnt, o_bsf + 2 * sizeof(unsigned long long) - o_cnt);
  if (rc) return rc;
  const unsigned long long *hc = reinterpret_cast<unsigned long long *>(ctx->pinned);
  const unsigned long long best = *reinterpret_cast<unsigned long long *>(ctx->pinned + (o_bsf - o_cnt));
  if (*reinterpret_cast<const unsigned *>(hc + kCntWords) == ctx->epoch)
    return fail(ctx, EAPDTW_ENONFINITE, "non-finite value in query or series");
  *out_offset = best_offset(best) == 0xffffffffu ? -1 : (int64_t)best_offset(best);
  *out_dist = (double)best_dist(best);
  if (lb_on && timed) lb_split_times(ctx);
  if (stats)
    fill_stats(stats, hc, (uint64_t)(band_cells_total(m, m, r) * K), (uint64_t)K,
               elapsed(ctx->ev0, ctx->ev1), lb_on ? ctx->lb_dp_ms : elapsed(ctx->ev2, ctx->ev3));
  fill_lb_stats(lbstats, hc, lb_on, (uint64_t)K, ctx->lb_ms);
  return EAPDTW_OK;
}

int eapdtw_nn_search(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                     int64_t n, int64_t window, int64_t *out_offset, double *out_dist,
                     eapdtw_stats *stats) {
  return nn_search_impl(ctx, query, m, series, n, window, out_offset, out_dist, stats, false,
                        nullptr);
}

int eapdtw_nn_search_lb(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                        int64_t n, int64_t window, int64_t *out_offset, double *out_dist,
                        eapdtw_stats *stats, eapdtw_lb_stats *lbstats) {
  return nn_search_impl(ctx, query, m, series, n, window, out_offset, out_dist, stats, true,
                        lbstats);
}

int eapdtw_nn_search_noalloc(eapdtw_ctx *ctx, const float *query, int64_t m,
                             const float *series, int64_t n, int64_t window, int64_t *out_offset,
                             double *out_dist) {
  CHECK_CTX();
  KnobGuard knobs(ctx);
  knobs.apply_cached(m, window);
  if (!out_offset || !out_dist) return fail(ctx, EAPDTW_EINVAL, "NULL output");
  int rc = search_validate(ctx, query, m, series, n, window);
  if (rc) return rc;
  const int64_t r = window < m - 1 ? window : m - 1;
  if (!use_band(ctx, r))
    return fail(ctx, EAPDTW_EINVAL, "the allocation-free search takes windows up to 64");
  if (m > kNoAllocMaxM)
    return fail(ctx, EAPDTW_EINVAL, "the allocation-free search takes queries up to 4096 points");
  Plan pl;
  const size_t o_cnt = pl.add(kCntBytes);
  const size_t o_bsf = pl.add(sizeof(unsigned long long) * 2);
  const size_t o_q = pl.add(sizeof(float) * (m + 2 * kColPad));
  if (pl.off > kNoAllocScratchBytes)
    return fail(ctx, EAPDTW_EINVAL, "the query exceeds the allocation-free scratch");
  // flag word .. best-so-far words: what the host reads back
  const size_t o_rd = sizeof(unsigned long long) * kCntWords;
  const size_t rd_bytes = o_bsf + 2 * sizeof(unsigned long long) - o_rd;
  if (!ctx->noalloc) return fail(ctx, EAPDTW_EDEVICE, "no address for the fixed scratch array");
  if (rd_bytes > ctx->pinned_cap) return fail(ctx, EAPDTW_EDEVICE, "pinned read-back buffer too small");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  char *base = ctx->noalloc;
  unsigned long long *cnt = reinterpret_cast<unsigned long long *>(base + o_cnt);
  unsigned long long *bsf = reinterpret_cast<unsigned long long *>(base + o_bsf);
  // the array keeps the last call's contents (of any context on this GPU):
  // clear the non-finite flag word; the set-up kernel clears the rest
  HIPCHK(launch_fill_u64(cnt + kCntWords, 0ull, 1, st));
  rc = search_queue(ctx, query, m, series, n, r, reinterpret_cast<float *>(base + o_q), bsf, cnt,
                    nullptr, 0.f, nullptr, 0, false, nullptr, nullptr, nullptr, true);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(ctx->pinned, base + o_rd, rd_bytes, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (*reinterpret_cast<const unsigned *>(ctx->pinned) == ctx->epoch)
    return fail(ctx, EAPDTW_ENONFINITE, "non-finite value in query or series");
  const unsigned long long best =
      *reinterpret_cast<const unsigned long long *>(ctx->pinned + (o_bsf - o_rd));
  *out_offset = best_offset(best) == 0xffffffffu ? -1 : (int64_t)best_offset(best);
  *out_dist = (double)best_dist(best);
  return EAPDTW_OK;
}

static int nn_dists_impl(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                         int64_t n, int64_t window, float ub, float *out, eapdtw_stats *stats,
                         bool use_lb, eapdtw_lb_stats *lbstats, const float *wgt = nullptr) {
  CHECK_CTX();
  KnobGuard knobs(ctx);
  knobs.apply_cached(m, window);
  if (!out) return fail(ctx, EAPDTW_EINVAL, "NULL output");
  if (std::isnan(ub)) return fail(ctx, EAPDTW_EINVAL, "ub is NaN");
  int rc = search_validate(ctx, query, m, series, n, window);
  if (rc) return rc;
  if (stats) std::memset(stats, 0, sizeof *stats);
  const int64_t r = window < m - 1 ? window : m - 1;
  const int64_t K = n - m + 1;
  const int64_t grid = use_band(ctx, r) ? 0 : wide_grid((K + kWave - 1) / kWave);
  const bool lb_on = use_lb && lb_applies(ctx, r);
  const bool timed = stats != nullptr || lbstats != nullptr;
  Plan pl;
  const size_t o_cnt = pl.add(kCntBytes);
  const size_t o_bsf = pl.add(sizeof(unsigned long long) * 2);
  const size_t o_q = pl.add(sizeof(float) * (m + 2 * kColPad));
  const size_t o_bnd = grid ? pl.add(sizeof(float) * grid * (m + 1) * kWave) : 0;
  const bool wide_w = wgt && r > kBandRMax;
  const size_t o_wt = wide_w ? pl.add(sizeof(float) * band_weight_words(r)) : 0;
  size_t o_lb[10];
  if (lb_on) lb_plan(pl, o_lb, n, m, K);
  rc = ensure_scratch(ctx, pl.off);
  if (rc) return rc;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  if (wide_w && (rc = upload_band_weights(ctx, o_wt, wgt, r))) return rc;
  unsigned long long *cnt = at<unsigned long long>(ctx, o_cnt);
  LbBufs lbb{};
  if (lb_on) lbb = lb_bind(ctx, o_lb);
  if (timed) HIPCHK(hipEventRecord(ctx->ev0, st));
  rc = search_queue(ctx, query, m, series, n, r, at<float>(ctx, o_q),
                    at<unsigned long long>(ctx, o_bsf), cnt, out, ub,
                    grid ? at<float>(ctx, o_bnd) : nullptr, grid, timed, lb_on ? &lbb : nullptr,
                    nullptr, wgt, false, wide_w ? at<float>(ctx, o_wt) : nullptr);
  if (rc) return rc;
  if (timed) {
    HIPCHK(hipEventRecord(ctx->ev1, st));
    rc = readback(ctx, o_cnt, kCntBytes);
    if (rc) return rc;
    const unsigned long long *hc = reinterpret_cast<unsigned long long *>(ctx->pinned);
    if (lb_on) lb_split_times(ctx);
    fill_stats(stats, hc, (uint64_t)(band_cells_total(m, m, r) * K), (uint64_t)K,
               elapsed(ctx->ev0, ctx->ev1), lb_on ? ctx->lb_dp_ms : elapsed(ctx->ev2, ctx->ev3));
    fill_lb_stats(lbstats, hc, lb_on, (uint64_t)K, ctx->lb_ms);
  }
  return EAPDTW_OK;
}

int eapdtw_nn_dists(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                    int64_t n, int64_t window, float ub, float *out, eapdtw_stats *stats) {
  return nn_dists_impl(ctx, query, m, series, n, window, ub, out, stats, false, nullptr);
}

int eapdtw_nn_dists_lb(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                       int64_t n, int64_t window, float ub, float *out, eapdtw_stats *stats,
                       eapdtw_lb_stats *lbstats) {
  return nn_dists_impl(ctx, query, m, series, n, window, ub, out, stats, true, lbstats);
}

// Weights of weighted DTW for phase differences 0..r of a query of length m
// (modified logistic weight, maximum 1, midpoint m / 2).  Fails for windows
// the band kernels do not serve.
// The weights w(0..r) (at least kBandRMax + 1 entries) of a weighted search.
static int wdtw_prepare(eapdtw_ctx *ctx, int64_t m, int64_t window, float g, std::vector<float> &wt) {
  if (!std::isfinite(g)) return fail(ctx, EAPDTW_EINVAL, "weighted DTW: g must be finite");
  wt.assign(kBandRMax + 1, 0.0f);
  if (m <= 0 || window < 0) return EAPDTW_OK;  // left to the search's own checks
  const int64_t r = window < m - 1 ? window : m - 1;
  if (r > kWtMaxR) return fail(ctx, EAPDTW_EINVAL, "weighted DTW: window above 4095");
  if (r + 1 > (int64_t)wt.size()) wt.resize((size_t)(r + 1));
  for (int64_t k = 0; k <= r; ++k)
    wt[(size_t)k] = (float)(1.0 / (1.0 + std::exp(-(double)g * ((double)k - (double)m / 2.0))));
  return EAPDTW_OK;
}

int eapdtw_nn_search_w(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                       int64_t n, int64_t window, float g, int64_t *out_offset, double *out_dist,
                       eapdtw_stats *stats) {
  CHECK_CTX();
  std::vector<float> wt;
  int rc = wdtw_prepare(ctx, m, window, g, wt);
  if (rc) return rc;
  return nn_search_impl(ctx, query, m, series, n, window, out_offset, out_dist, stats, false,
                        nullptr, wt.data());
}

int eapdtw_nn_dists_w(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                      int64_t n, int64_t window, float g, float ub, float *out,
                      eapdtw_stats *stats) {
  CHECK_CTX();
  std::vector<float> wt;
  int rc = wdtw_prepare(ctx, m, window, g, wt);
  if (rc) return rc;
  return nn_dists_impl(ctx, query, m, series, n, window, ub, out, stats, false, nullptr, wt.data());
}

int eapdtw_nn_lower_bounds(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                           int64_t n, int64_t window, float *out_kim, float *out_eq,
                           float *out_ec) {
  CHECK_CTX();
  if (!out_kim || !out_eq || !out_ec) return fail(ctx, EAPDTW_EINVAL, "NULL output");
  int rc = search_validate(ctx, query, m, series, n, window);
  if (rc) return rc;
  const int64_t r = window < m - 1 ? window : m - 1;
  if (r > kEnvMaxR) return fail(ctx, EAPDTW_EINVAL, "lower bounds: window above 2048");
  const int64_t K = n - m + 1;
  Plan pl;
  const size_t o_cnt = pl.add(kCntBytes);
  const size_t o_q = pl.add(sizeof(float) * (m + 2 * kColPad));
  size_t o_lb[10];
  lb_plan(pl, o_lb, n, m, K);
  rc = ensure_scratch(ctx, pl.off);
  if (rc) return rc;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  unsigned long long *cnt = at<unsigned long long>(ctx, o_cnt);
  float *qpad = at<float>(ctx, o_q);
  const LbBufs lbb = lb_bind(ctx, o_lb);
  if (++ctx->epoch == 0) ++ctx->epoch;
  HIPCHK(launch_search_prep(query, (int)m, qpad, series, n, cnt, nullptr, 0,
                            reinterpret_cast<unsigned *>(cnt + kCntWords), ctx->epoch, st));
  HIPCHK(launch_envelopes(series, n, qpad + kColPad, (int)m, (int)r, lbb.ux, lbb.lx, lbb.uq, lbb.lq,
                          st));
  LBArgs la{};
  la.x = series;
  la.n = n;
  la.m = (int)m;
  la.r = (int)r;
  la.qz = qpad + kColPad;
  la.uq = lbb.uq;
  la.lq = lbb.lq;
  la.ux = lbb.ux;
  la.lx = lbb.lx;
  la.k_begin = 0;
  la.k_end = K;
  la.mode = 2;
  la.out_kim = out_kim;
  la.out_eq = out_eq;
  la.out_ec = out_ec;
  HIPCHK(launch_lb_pass(la, st));
  rc = readback(ctx, o_cnt, kCntBytes);
  if (rc) return rc;
  if (*reinterpret_cast<const unsigned *>(reinterpret_cast<unsigned long long *>(ctx->pinned) +
                                          kCntWords) == ctx->epoch)
    return fail(ctx, EAPDTW_ENONFINITE, "non-finite value in query or series");
  return EAPDTW_OK;
}

int eapdtw_nn1(eapdtw_ctx *ctx, const float *X, int64_t N, int64_t len, int64_t window,
               int64_t *out_index, double *out_dist, eapdtw_stats *stats) {
  CHECK_CTX();
  if (N < 2 || len < 1) return fail(ctx, EAPDTW_EINVAL, "need at least 2 series of length >= 1");
  if (window < 0) return fail(ctx, EAPDTW_EINVAL, "window < 0");
  if (!X || !out_index || !out_dist) return fail(ctx, EAPDTW_EINVAL, "NULL pointer");
  if (len > INT_MAX / 2 || N > (int64_t)0xfffffffe) return fail(ctx, EAPDTW_EINVAL, "too large");
  if (stats) std::memset(stats, 0, sizeof *stats);
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const int64_t npairs = N * (N - 1) / 2;
  const int64_t r = window < len - 1 ? window : len - 1;
  const int64_t ldN = (N + kWave - 1) / kWave * kWave;
  const int64_t nblk_j = ldN / kWave;
  const int64_t ntasks = N * nblk_j;
  const int64_t grid = wide_grid(ntasks);
  Plan pl;
  const size_t o_cnt = pl.add(kCntBytes);
  const size_t o_nn = pl.add(sizeof(unsigned long long) * N);
  const size_t o_xt = pl.add(sizeof(float) * len * ldN);
  const size_t o_bnd = pl.add(sizeof(float) * grid * (len + 1) * kWave);
  int rc = ensure_scratch(ctx, pl.off);
  if (rc) return rc;
  unsigned long long *cnt = at<unsigned long long>(ctx, o_cnt);
  unsigned long long *nn = at<unsigned long long>(ctx, o_nn);
  if (stats) HIPCHK(hipEventRecord(ctx->ev0, st));
  HIPCHK(launch_fill_u64(cnt, 0ull, kCntWords, st));
  HIPCHK(launch_fill_u64(nn, pack_best(INFINITY, 0xffffffffu), N, st));
  HIPCHK(launch_transpose_pad(X, N, (int)len, ldN, 0, 0.0f, at<float>(ctx, o_xt), st));
  WideArgs w{};
  w.lrow = (int)len;
  w.lcol = (int)len;
  w.r = (int)r;
  w.X = X;
  w.XT = at<float>(ctx, o_xt);
  w.N = N;
  w.ld = ldN;
  w.nblk_j = nblk_j;
  w.ub_mode = 2;
  w.nn1 = nn;
  w.ntasks = ntasks;
  w.bnd = at<float>(ctx, o_bnd);
  w.bnd_stride = (len + 1) * kWave;
  w.counters = cnt;
  w.check_interval = 1;
  HIPCHK(launch_nn1_seed(w, (int)grid, st));
  if (stats) HIPCHK(hipEventRecord(ctx->ev2, st));
  HIPCHK(launch_wide(kWidePairwise, (int)ctx->wide_rows, w, (int)grid, st));
  log_launch(ctx, "%s rows %lld x %lld columns of length %d, r=%d: wide_kernel<%d,pairwise> %lld tasks on %lld waves",
             w.nn1 ? "nn1" : "pairwise", (long long)(w.nq ? w.nq : w.N), (long long)w.N, w.lrow, w.r,
             wide_h(ctx, w.r, w.lrow, w.lcol), (long long)w.ntasks, (long long)grid);
  if (stats) {
    HIPCHK(hipEventRecord(ctx->ev3, st));
    HIPCHK(hipEventRecord(ctx->ev1, st));
  }
  // counters then the per-series words
  rc = readback(ctx, o_cnt, o_nn + sizeof(unsigned long long) * N - o_cnt);
  if (rc) return rc;
  const unsigned long long *words =
      reinterpret_cast<const unsigned long long *>(ctx->pinned + (o_nn - o_cnt));
  for (int64_t i = 0; i < N; ++i) {
    out_index[i] = best_offset(words[i]) == 0xffffffffu ? -1 : (int64_t)best_offset(words[i]);
    out_dist[i] = (double)best_dist(words[i]);
  }
  if (stats)
    fill_stats(stats, reinterpret_cast<unsigned long long *>(ctx->pinned),
               (uint64_t)(band_cells_total(len, len, r) * npairs), (uint64_t)npairs,
               elapsed(ctx->ev0, ctx->ev1), elapsed(ctx->ev2, ctx->ev3));
  return EAPDTW_OK;
}

int eapdtw_nn1_ref(eapdtw_ctx *ctx, const float *Q, int64_t nq, const float *R, int64_t nr,
                   int64_t len, int64_t window, int64_t *out_index, double *out_dist,
                   eapdtw_stats *stats) {
  CHECK_CTX();
  if (nq < 1 || nr < 1 || len < 1) return fail(ctx, EAPDTW_EINVAL, "empty test or reference set");
  if (window < 0) return fail(ctx, EAPDTW_EINVAL, "window < 0");
  if (!Q || !R || !out_index || !out_dist) return fail(ctx, EAPDTW_EINVAL, "NULL pointer");
  if (len > INT_MAX / 2 || nr > (int64_t)0xfffffffe || nq > ((int64_t)1 << 40))
    return fail(ctx, EAPDTW_EINVAL, "too large");
  if (stats) std::memset(stats, 0, sizeof *stats);
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const int64_t npairs = nq * nr;
  const int64_t r = window < len - 1 ? window : len - 1;
  const int64_t ldN = (nr + kWave - 1) / kWave * kWave;
  const int64_t nblk_j = ldN / kWave;
  const int64_t ntasks = nq * nblk_j;
  const int64_t grid = wide_grid(ntasks);
  Plan pl;
  const size_t o_cnt = pl.add(kCntBytes);
  const size_t o_nn = pl.add(sizeof(unsigned long long) * nq);
  const size_t o_xt = pl.add(sizeof(float) * len * ldN);
  const size_t o_bnd = pl.add(sizeof(float) * grid * (len + 1) * kWave);
  int rc = ensure_scratch(ctx, pl.off);
  if (rc) return rc;
  unsigned long long *cnt = at<unsigned long long>(ctx, o_cnt);
  unsigned long long *nn = at<unsigned long long>(ctx, o_nn);
  if (stats) HIPCHK(hipEventRecord(ctx->ev0, st));
  HIPCHK(launch_fill_u64(cnt, 0ull, kCntWords, st));
  HIPCHK(launch_fill_u64(nn, pack_best(INFINITY, 0xffffffffu), nq, st));
  HIPCHK(launch_transpose_pad(R, nr, (int)len, ldN, 0, 0.0f, at<float>(ctx, o_xt), st));
  WideArgs w{};
  w.lrow = (int)len;
  w.lcol = (int)len;
  w.r = (int)r;
  w.X = Q;
  w.XT = at<float>(ctx, o_xt);
  w.N = nr;
  w.nq = nq;
  w.ld = ldN;
  w.nblk_j = nblk_j;
  w.ub_mode = 2;
  w.nn1 = nn;
  w.ntasks = ntasks;
  w.bnd = at<float>(ctx, o_bnd);
  w.bnd_stride = (len + 1) * kWave;
  w.counters = cnt;
  w.check_interval = 1;
  HIPCHK(launch_nn1_seed(w, (int)grid, st));
  if (stats) HIPCHK(hipEventRecord(ctx->ev2, st));
  HIPCHK(launch_wide(kWidePairwise, (int)ctx->wide_rows, w, (int)grid, st));
  log_launch(ctx, "%s rows %lld x %lld columns of length %d, r=%d: wide_kernel<%d,pairwise> %lld tasks on %lld waves",
             w.nn1 ? "nn1" : "pairwise", (long long)(w.nq ? w.nq : w.N), (long long)w.N, w.lrow, w.r,
             wide_h(ctx, w.r, w.lrow, w.lcol), (long long)w.ntasks, (long long)grid);
  if (stats) {
    HIPCHK(hipEventRecord(ctx->ev3, st));
    HIPCHK(hipEventRecord(ctx->ev1, st));
  }
  rc = readback(ctx, o_cnt, o_nn + sizeof(unsigned long long) * nq - o_cnt);
  if (rc) return rc;
  const unsigned long long *words =
      reinterpret_cast<const unsigned long long *>(ctx->pinned + (o_nn - o_cnt));
  for (int64_t i = 0; i < nq; ++i) {
    out_index[i] = best_offset(words[i]) == 0xffffffffu ? -1 : (int64_t)best_offset(words[i]);
    out_dist[i] = (double)best_dist(words[i]);
  }
  if (stats)
    fill_stats(stats, reinterpret_cast<unsigned long long *>(ctx->pinned),
               (uint64_t)(band_cells_total(len, len, r) * npairs), (uint64_t)npairs,
               elapsed(ctx->ev0, ctx->ev1), elapsed(ctx->ev2, ctx->ev3));
  return EAPDTW_OK;
}

static int knn_search_impl(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                           int64_t n, int64_t window, int64_t k, int64_t *out_offsets,
                           double *out_dists, eapdtw_stats *stats, bool use_lb,
                           eapdtw_lb_stats *lbstats) {
  CHECK_CTX();
  KnobGuard knobs(ctx);
  knobs.apply_cached(m, window);
  if (!out_offsets || !out_dists) return fail(ctx, EAPDTW_EINVAL, "NULL output");
  if (k < 1 || k > kKnnMax) return fail(ctx, EAPDTW_EINVAL, "k must be in 1..64");
  int rc = search_validate(ctx, query, m, series, n, window);
  if (rc) return rc;
  const int64_t r = window < m - 1 ? window : m - 1;
  if (stats) std::memset(stats, 0, sizeof *stats);
  const int64_t K = n - m + 1;
  const int64_t grid = use_band(ctx, r) ? 0 : wide_grid((K + kWave - 1) / kWave);
  const bool lb_on = use_lb && lb_applies(ctx, r);
  const bool timed = stats != nullptr || lbstats != nullptr;
  Plan pl;
  const size_t o_cnt = pl.add(kCntBytes);
  const size_t o_bsf = pl.add(sizeof(unsigned long long) * 2);
  const size_t o_res = pl.add(sizeof(unsigned long long) * kKnnMax);
  const size_t o_q = pl.add(sizeof(float) * (m + 2 * kColPad));
  const size_t o_buf = pl.add(sizeof(unsigned long long) * K);
  const size_t o_tmp = pl.add(sizeof(unsigned long long) * K);
  const size_t o_bnd = grid ? pl.add(sizeof(float) * grid * (m + 1) * kWave) : 0;
  size_t o_lb[10];
  if (lb_on) lb_plan(pl, o_lb, n, m, K);
  rc = ensure_scratch(ctx, pl.off);
  if (rc) return rc;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  unsigned long long *cnt = at<unsigned long long>(ctx, o_cnt);
  unsigned long long *bsf = at<unsigned long long>(ctx, o_bsf);
  // the kept-candidate count and the filtered count live in counter words
  // (stripe 0 and 1, slot kCntKnnN), cleared by the set-up kernel
  const KnnBufs kb{(int)k, at<unsigned long long>(ctx, o_buf), cnt + kCntKnnN};
  LbBufs lbb{};
  if (lb_on) lbb = lb_bind(ctx, o_lb);
  if (timed) HIPCHK(hipEventRecord(ctx->ev0, st));
  rc = search_queue(ctx, query, m, series, n, r, at<float>(ctx, o_q), bsf, cnt, nullptr, 0.f,
                    grid ? at<float>(ctx, o_bnd) : nullptr, grid, timed, lb_on ? &lbb : nullptr, &kb);
  if (rc) return rc;
  HIPCHK(launch_knn_select(kb.buf, kb.n, bsf, at<unsigned long long>(ctx, o_tmp),
                           cnt + kCntStride + kCntKnnN, (int)k,
                           at<unsigned long long>(ctx, o_res), st));
  if (timed) HIPCHK(hipEventRecord(ctx->ev1, st));
  // counters, the best-so-far words and the results are contiguous
  rc = readback(ctx, o_cnt, o_res + sizeof(unsigned long long) * kKnnMax - o_cnt);
  if (rc) return rc;
  const unsigned long long *hc = reinterpret_cast<unsigned long long *>(ctx->pinned);
  if (*reinterpret_cast<const unsigned *>(hc + kCntWords) == ctx->epoch)
    return fail(ctx, EAPDTW_ENONFINITE, "non-finite value in query or series");
  const unsigned long long *res =
      reinterpret_cast<const unsigned long long *>(ctx->pinned + (o_res - o_cnt));
  for (int64_t i = 0; i < k; ++i) {
    const bool have = i < K && res[i] != ~0ull;
    out_offsets[i] = have ? (int64_t)best_offset(res[i]) : -1;
    out_dists[i] = have ? (double)best_dist(res[i]) : INFINITY;
  }
  if (lb_on && timed) lb_split_times(ctx);
  if (stats)
    fill_stats(stats, hc, (uint64_t)(band_cells_total(m, m, r) * K), (uint64_t)K,
               elapsed(ctx->ev0, ctx->ev1), lb_on ? ctx->lb_dp_ms : elapsed(ctx->ev2, ctx->ev3));
  fill_lb_stats(lbstats, hc, lb_on, (uint64_t)K, ctx->lb_ms);
  return EAPDTW_OK;
}

int eapdtw_knn_search(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                      int64_t n, int64_t window, int64_t k, int64_t *out_offsets,
                      double *out_dists, eapdtw_stats *stats) {
  return knn_search_impl(ctx, query, m, series, n, window, k, out_offsets, out_dists, stats,
                         false, nullptr);
}

int eapdtw_knn_search_lb(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                         int64_t n, int64_t window, int64_t k, int64_t *out_offsets,
                         double *out_dists, eapdtw_stats *stats, eapdtw_lb_stats *lbstats) {
  return knn_search_impl(ctx, query, m, series, n, window, k, out_offsets, out_dists, stats,
                         true, lbstats);
}

int eapdtw_nn_search_erp(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                         int64_t n, int64_t window, double g, int64_t *out_offset, double *out_dist,
                         eapdtw_stats *stats) {
  CHECK_CTX();
  if (!out_offset || !out_dist) return fail(ctx, EAPDTW_EINVAL, "NULL output");
  if (!std::isfinite(g) || std::fabs(g) > FLT_MAX) return fail(ctx, EAPDTW_EINVAL, "g must be a finite float32");
  int rc = search_validate(ctx, query, m, series, n, window);
  if (rc) return rc;
  const int64_t r = window < m - 1 ? window : m - 1;
  if (r > kErpMaxR) return fail(ctx, EAPDTW_EINVAL, "ERP takes windows up to 64 (after clamping to m - 1)");
  if (stats) std::memset(stats, 0, sizeof *stats);
  const int64_t K = n - m + 1;
  Plan pl;
  const size_t o_cnt = pl.add(kCntBytes);
  const size_t o_bsf = pl.add(sizeof(unsigned long long) * 2);
  const size_t o_q = pl.add(sizeof(float) * (m + 2 * kColPad));
  rc = ensure_scratch(ctx, pl.off);
  if (rc) return rc;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  unsigned long long *cnt = at<unsigned long long>(ctx, o_cnt);
  unsigned long long *bsf = at<unsigned long long>(ctx, o_bsf);
  float *qpad = at<float>(ctx, o_q);
  if (stats) HIPCHK(hipEventRecord(ctx->ev0, st));
  if (++ctx->epoch == 0) ++ctx->epoch;
  HIPCHK(launch_search_prep(query, (int)m, qpad, series, n, cnt, bsf, 2,
                            reinterpret_cast<unsigned *>(cnt + kCntWords), ctx->epoch, st));
  if (stats) HIPCHK(hipEventRecord(ctx->ev2, st));
  ErpSearchArgs e{};
  e.x = series;
  e.n = n;
  e.K = K;
  e.qz = qpad + kColPad;
  e.m = (int)m;
  e.g = (float)g;
  e.bsf = bsf;
  e.check_interval = (int)(ctx->check_interval > 0 ? ctx->check_interval : 4);
  e.counters = cnt;
  HIPCHK(launch_erp_search((int)r, e, st));
  log_launch(ctx, "erp search m=%lld r=%lld: erp_search_kernel<%lld> grid=%lld", (long long)m,
             (long long)r, (long long)r, (long long)((K + kWave - 1) / kWave));
  if (stats) {
    HIPCHK(hipEventRecord(ctx->ev3, st));
    HIPCHK(hipEventRecord(ctx->ev1, st));
  }
  // counters, the flag word and the best-so-far words are contiguous
  rc = readback(ctx, o_cnt, o_bsf + 2 * sizeof(unsigned long long) - o_cnt);
  if (rc) return rc;
  const unsigned long long *hc = reinterpret_cast<unsigned long long *>(ctx->pinned);
  if (*reinterpret_cast<const unsigned *>(hc + kCntWords) == ctx->epoch)
    return fail(ctx, EAPDTW_ENONFINITE, "non-finite value in query or series");
  const unsigned long long best = *reinterpret_cast<unsigned long long *>(ctx->pinned + (o_bsf - o_cnt));
  *out_offset = best_offset(best) == 0xffffffffu ? -1 : (int64_t)best_offset(best);
  *out_dist = (double)best_dist(best);
  if (stats)
    fill_stats(stats, hc, (uint64_t)(band_cells_total(m, m, r) * K), (uint64_t)K,
               elapsed(ctx->ev0, ctx->ev1), elapsed(ctx->ev2, ctx->ev3));
  return EAPDTW_OK;
}

static uint64_t fnv1a(uint64_t h, const void *p, size_t n) {
  const unsigned char *b = static_cast<const unsigned char *>(p);
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}

// Queues the whole batched search on stream st, forking side streams from it
// and joining them back (used directly, or once under stream capture to build
// the graph).
// Queries with band windows (the descriptors from nband_first on) each get
// one launch of their band (or window-0) kernel after the batched seeding;
// the others share the persistent tiled launch.
static int batch_queue(eapdtw_ctx *ctx, const BatchArgs &ba, int grid,
                       const std::vector<BatchQuery> &desc, const std::vector<eapdtw_tune> &knob,
                       int64_t nband_first, hipStream_t st) {
  HIPCHK(launch_fill_u64(ba.counters, 0ull, kCntWords, st));
  HIPCHK(launch_batch_prep(ba, st));
  HIPCHK(launch_check_finite(ba.x, ba.n, ba.counters, st));
  if (ctx->seed) HIPCHK(launch_batch_seed(ba, st));
  // Band-window queries are independent searches (own best-so-far word; the
  // shared counters are atomics): they go round-robin, most expensive first,
  // onto up to batch_branches streams forked from st.  The launches then run
  // side by side, and the CUs that one launch's late waves (the candidates
  // abandoned last) leave idle take the others' waves.  st itself takes the
  // persistent tiled launch, or the first branch when there is none.
  const int64_t nband = (int64_t)desc.size() - nband_first;
  const bool own_main = ba.total_units > 0;
  // band-launch branches on side streams (st takes one more when it has no
  // tiled launch of its own)
  const int nside = (int)std::max<int64_t>(
      0, own_main ? std::min<int64_t>(ctx->batch_branches - 1, nband)
                  : std::min<int64_t>(ctx->batch_branches, nband) - 1);
  if (nside > 0) {
    if (!ctx->ev_bfork) HIPCHK(hipEventCreateWithFlags(&ctx->ev_bfork, hipEventDisableTiming));
    for (int b = 0; b < nside; ++b) {
      if (!ctx->branch[b]) HIPCHK(hipStreamCreateWithFlags(&ctx->branch[b], hipStreamNonBlocking));
      if (!ctx->ev_bjoin[b]) HIPCHK(hipEventCreateWithFlags(&ctx->ev_bjoin[b], hipEventDisableTiming));
    }
    HIPCHK(hipEventRecord(ctx->ev_bfork, st));
    for (int b = 0; b < nside; ++b) HIPCHK(hipStreamWaitEvent(ctx->branch[b], ctx->ev_bfork, 0));
  }
  // branch j of the band launches: side stream j (or j - 1 after st's own
  // first branch when there is no tiled launch)
  auto branch_stream = [&](int64_t j) -> hipStream_t {
    if (own_main) return ctx->branch[j % nside];
    const int64_t b = j % (nside + 1);
    return b == 0 ? st : ctx->branch[b - 1];
  };
  for (int64_t i = nband_first; i < (int64_t)desc.size(); ++i) {
    const hipStream_t bs = nside > 0 ? branch_stream(i - nband_first) : st;
    const BatchQuery &d = desc[i];
    NNArgs a{};
    a.x = ba.x;
    a.n = ba.n;
    a.m = d.m;
    a.qpad = d.qpad;
    a.bsf = d.bsf;
    a.k_begin = 0;
    a.k_end = d.K;
    a.counters = ba.counters;
    a.check_interval = ba.check_interval;
    a.block_stride = 1;
    const int64_t nblk = (d.K + kWave - 1) / kWave;
    const eapdtw_tune &t = knob[i];
    a.check_interval = (int)t.check_interval;
    const int rows = t.rows_per_group ? (int)t.rows_per_group : pick_rows(ctx, d.r);
    if (ba.knn > 0) {
      a.knn = ba.knn;
      a.knn_buf = d.knn_buf;
      a.knn_n = d.knn_n;
      a.knn_slots = d.knn_slots;
      // (the window-0 kernel publishes only the best)
      HIPCHK(nn_band_launcher(d.r)(a, nblk, 4, false, t.border != 0, bs));
    } else if (d.r == 0 && ctx->ed) {
      HIPCHK(launch_ed_search(a, nblk, false, bs));
    } else {
      HIPCHK(nn_band_launcher(d.r)(a, nblk, rows, false, t.border != 0, bs));
    }
  }
  if (ba.total_units > 0) HIPCHK(launch_batch_main(ba, grid, st));
  for (int b = 0; b < nside; ++b) {
    HIPCHK(hipEventRecord(ctx->ev_bjoin[b], ctx->branch[b]));
    HIPCHK(hipStreamWaitEvent(st, ctx->ev_bjoin[b], 0));
  }
  // k nearest neighbours: per query, the kept candidates at or below its
  // final bound, then the k best of them (knn_res, k words per query)
  for (size_t i = 0; ba.knn > 0 && i < desc.size(); ++i) {
    const BatchQuery &d = desc[i];
    HIPCHK(launch_knn_select(d.knn_buf, d.knn_n, d.bsf, d.knn_buf + d.K, d.knn_nsel, ba.knn,
                             d.knn_res, st));
  }
  return EAPDTW_OK;
}

// The batched search: nearest neighbour of every query (k == 0, results in
// out) or its k nearest neighbours (k >= 1, offsets and distances [nq][k]).
static int batch_impl(eapdtw_ctx *ctx, const eapdtw_query *qs, int64_t nq, const float *series,
                      int64_t n, int64_t k, eapdtw_result *out, int64_t *out_offsets,
                      double *out_dists, eapdtw_stats *stats) {
  CHECK_CTX();
  if (nq < 0 || (nq > 0 && (!qs || (k == 0 ? !out : (!out_offsets || !out_dists)))))
    return fail(ctx, EAPDTW_EINVAL, "bad query array");
  if (k < 0 || k > kKnnMax) return fail(ctx, EAPDTW_EINVAL, "k must be in 1..64");
  if (nq > 65536) return fail(ctx, EAPDTW_EINVAL, "too many queries");
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (nq == 0) return EAPDTW_OK;
  int64_t max_m = 0;
  for (int64_t q = 0; q < nq; ++q) {
    int rc = search_validate(ctx, qs[q].query, qs[q].m, series, n, qs[q].window);
    if (rc) return rc;
    max_m = std::max(max_m, qs[q].m);
  }
  if (ctx->autotune) {
    // tune each (length, window) bucket the cache has no record for
    for (int64_t q = 0; q < nq; ++q) {
      if (ctx->tune.count(eapdtw_tune_bucket(qs[q].m, qs[q].window))) continue;
      int rc = eapdtw_autotune(ctx, qs[q].query, qs[q].m, series, n, qs[q].window, 1 << 18, nullptr);
      if (rc) return rc;
    }
  }
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  // most expensive queries first (band cells per candidate x candidates)
  std::vector<int64_t> order(nq);
  std::vector<double> cost(nq);
  uint64_t nominal = 0, problems = 0;
  for (int64_t q = 0; q < nq; ++q) {
    const int64_t m = qs[q].m, r = std::min(qs[q].window, m - 1), K = n - m + 1;
    const int64_t bc = band_cells_total(m, m, r);
    cost[q] = (double)bc * (double)K;
    nominal += (uint64_t)(bc * K);
    problems += (uint64_t)K;
    order[q] = q;
  }
  // tiled-kernel queries first (they share the persistent launch's work
  // queue), then band-window queries; each part most expensive first
  auto banded = [&](int64_t q) { return use_band(ctx, std::min(qs[q].window, qs[q].m - 1)); };
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    if (banded(a) != banded(b)) return !banded(a);
    return cost[a] > cost[b];
  });
  const int grid = (int)ctx->batch_grid;
  Plan pl;
  const size_t o_cnt = pl.add(kCntBytes);
  const size_t o_work = pl.add(sizeof(unsigned long long));
  const size_t o_desc = pl.add(sizeof(BatchQuery) * nq);
  const size_t o_bsf = pl.add(sizeof(unsigned long long) * 2 * nq);
  // k nearest neighbours: the k result words of every query (read back with
  // the counters and best-so-far words)
  const size_t o_kres = k > 0 ? pl.add(sizeof(unsigned long long) * kKnnMax * nq) : 0;
  std::vector<size_t> o_q(nq), o_knn(nq);
  for (int64_t i = 0; i < nq; ++i) o_q[i] = pl.add(sizeof(float) * (qs[order[i]].m + 2 * kColPad));
  // k nearest neighbours, per query: the slot words (k, kCntStride apart),
  // the two counts, and the kept candidates with their filtered copy (K words
  // each)
  constexpr size_t kKnnHead = (size_t)kKnnMax * kCntStride + 2;
  if (k > 0)
    for (int64_t i = 0; i < nq; ++i)
      o_knn[i] = pl.add(sizeof(unsigned long long) * (kKnnHead + 2 * (size_t)(n - qs[order[i]].m + 1)));
  const size_t o_bnd = pl.add(sizeof(float) * (size_t)grid * (max_m + 1) * kWave);
  if (pl.off > ctx->batch_cap) {
    HIPCHK(hipStreamSynchronize(st));
    if (ctx->batch_exec) {
      (void)hipGraphExecDestroy(ctx->batch_exec);
      ctx->batch_exec = nullptr;
    }
    if (ctx->batch_buf) HIPCHK(hipFree(ctx->batch_buf));
    ctx->batch_buf = nullptr;
    ctx->batch_cap = 0;
    if (hipMalloc((void **)&ctx->batch_buf, pl.off) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, EAPDTW_ENOMEM, "batch buffer allocation failed");
    }
    ctx->batch_cap = pl.off;
  }
  char *bb = ctx->batch_buf;
  // descriptors in the sorted order
  std::vector<BatchQuery> desc(nq);
  int64_t units = 0, seeds = 0, nband_first = nq;
  for (int64_t i = 0; i < nq; ++i) {
    const eapdtw_query &h = qs[order[i]];
    BatchQuery &d = desc[i];
    d.query = h.query;
    d.qpad = reinterpret_cast<float *>(bb + o_q[i]);
    d.bsf = reinterpret_cast<unsigned long long *>(bb + o_bsf) + 2 * i;
    d.m = (int)h.m;
    d.r = (int)std::min(h.window, h.m - 1);
    d.K = n - h.m + 1;
    d.unit_begin = units;
    d.seed_begin = seeds;
    const int64_t nblk = (d.K + kWave - 1) / kWave;
    const int64_t sstr = seed_stride_for(ctx->batch_seed_stride, nblk);
    d.seed_stride = (int)sstr;
    if (k > 0) {
      unsigned long long *kw = reinterpret_cast<unsigned long long *>(bb + o_knn[i]);
      d.knn_slots = kw;
      d.knn_n = kw + (size_t)kKnnMax * kCntStride;
      d.knn_nsel = d.knn_n + 1;
      d.knn_buf = d.knn_n + 2;
      d.knn_res = reinterpret_cast<unsigned long long *>(bb + o_kres) + (size_t)kKnnMax * i;
    }
    if (use_band(ctx, d.r)) {
      if (nband_first == nq) nband_first = i;
    } else {
      units += nblk;  // band queries own no units (their unit_begin is past the last)
    }
    seeds += (nblk + sstr - 1) / sstr;
  }
  // per-query choices for the band launches: the tuned ones of the query's
  // bucket when autotuning, else the context's
  std::vector<eapdtw_tune> knob(nq, eapdtw_tune{ctx->rows_per_group, ctx->border,
                                                ctx->check_interval, ctx->wide_rows, 0, 0.f});
  if (ctx->autotune) {
    for (int64_t i = 0; i < nq; ++i) {
      auto it = ctx->tune.find(eapdtw_tune_bucket(qs[order[i]].m, qs[order[i]].window));
      if (it != ctx->tune.end()) knob[i] = it->second;
      knob[i].ms = 0.f;
    }
  }
  BatchArgs ba{};
  ba.qs = reinterpret_cast<const BatchQuery *>(bb + o_desc);
  ba.nq = (int)nq;
  ba.x = series;
  ba.n = n;
  ba.total_units = units;
  ba.work = reinterpret_cast<unsigned long long *>(bb + o_work);
  ba.chunk = (int)ctx->batch_chunk;
  ba.total_seed_blocks = seeds;
  ba.seed_window = (int)std::min<int64_t>(ctx->seed_window, 8);
  ba.bnd = reinterpret_cast<float *>(bb + o_bnd);
  ba.bnd_stride = (max_m + 1) * kWave;
  ba.counters = reinterpret_cast<unsigned long long *>(bb + o_cnt);
  ba.check_interval = (int)ctx->check_interval;
  ba.knn = (int)k;
  // graph key: everything the captured launches depend on
  uint64_t key = 1469598103934665603ull;
  key = fnv1a(key, &bb, sizeof bb);
  key = fnv1a(key, &ctx->stream, sizeof ctx->stream);
  key = fnv1a(key, &ba, sizeof ba);
  key = fnv1a(key, desc.data(), sizeof(BatchQuery) * nq);
  key = fnv1a(key, &grid, sizeof grid);
  key = fnv1a(key, &ctx->seed, sizeof ctx->seed);
  key = fnv1a(key, &ctx->border, sizeof ctx->border);
  key = fnv1a(key, &ctx->ed, sizeof ctx->ed);
  key = fnv1a(key, &ctx->rows_per_group, sizeof ctx->rows_per_group);
  key = fnv1a(key, &ctx->force_wide, sizeof ctx->force_wide);
  key = fnv1a(key, &ctx->batch_branches, sizeof ctx->batch_branches);
  for (const eapdtw_tune &t : knob) {
    const int64_t f[4] = {t.rows_per_group, t.border, t.check_interval, t.wide_rows};
    key = fnv1a(key, f, sizeof f);
  }
  const bool use_graph = ctx->graph != 0;
  const bool rebuild = !use_graph || !ctx->batch_exec || ctx->batch_key != key;
  log_launch(ctx, "batch %lld queries: %lld band launches on up to %lld streams, %lld units of 64 offsets in "
             "the persistent batch_main_kernel (%d waves), %lld seeding blocks; %s",
             (long long)nq, (long long)(nq - nband_first), (long long)ctx->batch_branches, (long long)units,
             grid, (long long)seeds, use_graph ? (rebuild ? "graph captured" : "graph replayed") : "no graph");
  if (rebuild) {
    // descriptors are constant for a given key: upload them outside the graph
    int rc = ensure_pinned(ctx, sizeof(BatchQuery) * nq);
    if (rc) return rc;
    std::memcpy(ctx->pinned, desc.data(), sizeof(BatchQuery) * nq);
    HIPCHK(hipMemcpyAsync(bb + o_desc, ctx->pinned, sizeof(BatchQuery) * nq, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  if (stats) HIPCHK(hipEventRecord(ctx->ev0, st));
  if (use_graph) {
    if (rebuild) {
      if (ctx->batch_exec) {
        (void)hipGraphExecDestroy(ctx->batch_exec);
        ctx->batch_exec = nullptr;
      }
      // the caller's stream may be the null stream, which cannot be
      // captured: record on a private stream, replay on the caller's
      if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
      int rc = batch_queue(ctx, ba, grid, desc, knob, nband_first, ctx->cap_stream);
      hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (ec != hipSuccess) return fail_hip(ctx, ec, "hipStreamEndCapture");
      ec = hipGraphInstantiate(&ctx->batch_exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ec != hipSuccess) {
        ctx->batch_exec = nullptr;
        return fail_hip(ctx, ec, "hipGraphInstantiate");
      }
      ctx->batch_key = key;
    }
    HIPCHK(hipGraphLaunch(ctx->batch_exec, st));
  } else {
    int rc = batch_queue(ctx, ba, grid, desc, knob, nband_first, st);
    if (rc) return rc;
  }
  if (stats) HIPCHK(hipEventRecord(ctx->ev1, st));
  // counters, work counter, descriptors and best-so-far words read back at once
  const size_t nbytes = k > 0 ? o_kres + sizeof(unsigned long long) * kKnnMax * nq
                              : o_bsf + sizeof(unsigned long long) * 2 * nq;
  int rc = ensure_pinned(ctx, nbytes);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(ctx->pinned, bb, nbytes, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const unsigned long long *hc = reinterpret_cast<unsigned long long *>(ctx->pinned + o_cnt);
  if (counter_sum(hc, kCntNonFinite)) return fail(ctx, EAPDTW_ENONFINITE, "non-finite value in a query or the series");
  const unsigned long long *hb = reinterpret_cast<unsigned long long *>(ctx->pinned + o_bsf);
  for (int64_t i = 0; k == 0 && i < nq; ++i) {
    const unsigned long long b = hb[2 * i];
    eapdtw_result &r = out[order[i]];
    r.offset = best_offset(b) == 0xffffffffu ? -1 : (int64_t)best_offset(b);
    r.dist = (double)best_dist(b);
  }
  if (k > 0) {
    const unsigned long long *hr = reinterpret_cast<unsigned long long *>(ctx->pinned + o_kres);
    for (int64_t i = 0; i < nq; ++i) {
      const int64_t q = order[i];
      const int64_t Kq = n - qs[q].m + 1;
      for (int64_t j = 0; j < k; ++j) {
        const unsigned long long w = hr[(size_t)kKnnMax * i + j];
        const bool have = j < Kq && w != ~0ull;
        out_offsets[q * k + j] = have ? (int64_t)best_offset(w) : -1;
        out_dists[q * k + j] = have ? (double)best_dist(w) : INFINITY;
      }
    }
  }
  if (stats) {
    const float ms = elapsed(ctx->ev0, ctx->ev1);
    fill_stats(stats, hc, nominal, problems, ms, ms);
  }
  return EAPDTW_OK;
}

int eapdtw_nn_search_batch(eapdtw_ctx *ctx, const eapdtw_query *qs, int64_t nq,
                           const float *series, int64_t n, eapdtw_result *out,
                           eapdtw_stats *stats) {
  return batch_impl(ctx, qs, nq, series, n, 0, out, nullptr, nullptr, stats);
}

int eapdtw_knn_search_batch(eapdtw_ctx *ctx, const eapdtw_query *qs, int64_t nq,
                            const float *series, int64_t n, int64_t k, int64_t *out_offsets,
                            double *out_dists, eapdtw_stats *stats) {
  if (ctx && (k < 1 || k > kKnnMax)) return fail(ctx, EAPDTW_EINVAL, "k must be in 1..64");
  return batch_impl(ctx, qs, nq, series, n, k, nullptr, out_offsets, out_dists, stats);
}

int eapdtw_autotune(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                    int64_t n, int64_t window, int64_t sample_n, eapdtw_tune *out) {
  CHECK_CTX();
  int rc = search_validate(ctx, query, m, series, n, window);
  if (rc) return rc;
  int64_t ns = std::max<int64_t>(sample_n, m + 65536);
  ns = std::min(ns, n);
  const int64_t r = window < m - 1 ? window : m - 1;
  std::vector<eapdtw_tune> cand;
  const int64_t cis[3] = {0, 1, 4};
  if (use_band(ctx, r)) {
    for (int64_t ci : cis) {
      if (r >= kBorderMinR) {
        for (int64_t b : {1, 0}) cand.push_back({0, b, ci, 0, 0, 0.f});
      } else {
        for (int64_t u : {4, 2, 8}) cand.push_back({u, 1, ci, 0, 0, 0.f});
      }
      // the other mapping of lanes to candidates: each lane streams its own
      if (lane_search_supported((int)r, (int)m)) cand.push_back({0, 1, ci, 0, 1, 0.f});
    }
  } else {
    const bool full = m > 1 && r >= m - 1;
    for (int64_t ci : cis) {
      if (full) {
        for (int64_t h : {64, 32}) cand.push_back({0, 1, ci, h, 0, 0.f});
      } else {
        cand.push_back({0, 1, ci, 0, 0, 0.f});
      }
    }
  }
  KnobGuard knobs(ctx);
  const int64_t at = ctx->autotune;
  ctx->autotune = 0;
  eapdtw_tune best{};
  best.ms = INFINITY;
  for (eapdtw_tune &t : cand) {
    knobs.apply(t);
    float ms = INFINITY;
    for (int rep = 0; rep < 3 && rc == 0; ++rep) {
      int64_t off;
      double d;
      eapdtw_stats st;
      rc = eapdtw_nn_search(ctx, query, m, series, ns, window, &off, &d, &st);
      if (rep > 0) ms = std::min(ms, st.kernel_ms);  // the first run warms up
    }
    if (rc) break;
    t.ms = ms;
    if (ms < best.ms) best = t;
  }
  ctx->autotune = at;
  if (rc) return rc;
  ctx->tune[eapdtw_tune_bucket(m, window)] = best;
  if (out) *out = best;
  return EAPDTW_OK;
}

int eapdtw_tune_get(const eapdtw_ctx *ctx, int64_t bucket, eapdtw_tune *out) {
  if (!ctx || !out) return EAPDTW_EINVAL;
  auto it = ctx->tune.find(bucket);
  if (it == ctx->tune.end()) return EAPDTW_EINVAL;
  *out = it->second;
  return EAPDTW_OK;
}

int eapdtw_tune_save(const eapdtw_ctx *ctx, const char *path) {
  if (!ctx || !path) return EAPDTW_EINVAL;
  FILE *f = std::fopen(path, "w");
  if (!f) return EAPDTW_EINVAL;
  std::fprintf(f, "{\"arch\": \"gfx950\", \"entries\": [");
  bool first = true;
  for (const auto &kv : ctx->tune) {
    const eapdtw_tune &t = kv.second;
    std::fprintf(f,
                 "%s\n  {\"bucket\": %lld, \"rows_per_group\": %lld, \"border\": %lld, "
                 "\"check_interval\": %lld, \"wide_rows\": %lld, \"lanes\": %lld, \"ms\": %.6g}",
                 first ? "" : ",", (long long)kv.first, (long long)t.rows_per_group,
                 (long long)t.border, (long long)t.check_interval, (long long)t.wide_rows,
                 (long long)t.lanes, (double)t.ms);
    first = false;
  }
  std::fprintf(f, "\n]}\n");
  return std::fclose(f) == 0 ? EAPDTW_OK : EAPDTW_EINVAL;
}

// Reads the file written by eapdtw_tune_save: the arch string, then one
// entry per object; every value must be in the range its option accepts.
int eapdtw_tune_load(eapdtw_ctx *ctx, const char *path) {
  if (!ctx || !path) return EAPDTW_EINVAL;
  FILE *f = std::fopen(path, "r");
  if (!f) return fail(ctx, EAPDTW_EINVAL, "cannot open tuning file");
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
  std::fclose(f);
  if (text.find("\"arch\": \"gfx950\"") == std::string::npos)
    return fail(ctx, EAPDTW_EINVAL, "tuning file is not for gfx950");
  std::map<int64_t, eapdtw_tune> add;
  size_t pos = 0;
  while ((pos = text.find("{\"bucket\"", pos)) != std::string::npos) {
    long long b, u, bo, ci, w, ln = 0;
    double ms;
    // entries written before the lanes choice existed have no "lanes" field
    if (std::sscanf(text.c_str() + pos,
                    "{\"bucket\": %lld, \"rows_per_group\": %lld, \"border\": %lld, "
                    "\"check_interval\": %lld, \"wide_rows\": %lld, \"lanes\": %lld, \"ms\": %lf}",
                    &b, &u, &bo, &ci, &w, &ln, &ms) != 7 &&
        std::sscanf(text.c_str() + pos,
                    "{\"bucket\": %lld, \"rows_per_group\": %lld, \"border\": %lld, "
                    "\"check_interval\": %lld, \"wide_rows\": %lld, \"ms\": %lf}",
                    &b, &u, &bo, &ci, &w, &ms) != 6)
      return fail(ctx, EAPDTW_EINVAL, "malformed tuning entry");
    const bool ok = b >= 0 && (u == 0 || u == 2 || u == 4 || u == 8) && (bo == 0 || bo == 1) &&
                    ci >= 0 && ci <= (1 << 20) && (w == 0 || w == 32 || w == 64) &&
                    (ln == 0 || ln == 1);
    if (!ok) return fail(ctx, EAPDTW_EINVAL, "tuning entry out of range");
    add[b] = eapdtw_tune{u, bo, ci, w, ln, (float)ms};
    ++pos;
  }
  for (const auto &kv : add) ctx->tune[kv.first] = kv.second;
  return EAPDTW_OK;
}

// --------------------------------------------------------------------------- wavefront pair batches

// Host view of one pair of a wavefront batch (window already clipped).
struct WfHostPair {
  int64_t s_off, t_off, ls, lt, r;
};

static int64_t clip_window(int64_t window, int64_t ls, int64_t lt) {
  const int64_t lmax = ls > lt ? ls : lt;
  return lmax > 0 && window > lmax - 1 ? lmax - 1 : window;
}

static bool wf_has_path(const WfHostPair &h) {
  return h.ls > 0 && h.lt > 0 && std::llabs(h.ls - h.lt) <= h.r;
}

// Validates a host array of eapdtw_pair against the pools and clips the
// windows.  `disjoint`: the pairs' S regions must not overlap, nor their T
// regions (their gradients and path ranges are written in place).
static int wf_validate(eapdtw_ctx *ctx, const float *S, int64_t s_total, const float *T,
                       int64_t t_total, const eapdtw_pair *pairs, int64_t npairs, bool disjoint,
                       std::vector<WfHostPair> &hp) {
  if (npairs < 0 || s_total < 0 || t_total < 0) return fail(ctx, EAPDTW_EINVAL, "negative size");
  if (npairs > 0 && !pairs) return fail(ctx, EAPDTW_EINVAL, "pairs is NULL");
  if ((s_total > 0 && !S) || (t_total > 0 && !T)) return fail(ctx, EAPDTW_EINVAL, "NULL pool");
  if (npairs > INT_MAX) return fail(ctx, EAPDTW_EINVAL, "too many pairs");
  hp.resize((size_t)npairs);
  for (int64_t p = 0; p < npairs; ++p) {
    const eapdtw_pair &q = pairs[p];
    if (q.s_len < 0 || q.t_len < 0 || q.window < 0 || q.s_off < 0 || q.t_off < 0)
      return fail(ctx, EAPDTW_EINVAL, "pair " + std::to_string(p) + ": negative field");
    if (q.s_len > kWfMaxLen || q.t_len > kWfMaxLen)
      return fail(ctx, EAPDTW_EINVAL, "pair " + std::to_string(p) + ": series longer than 8191");
    if (q.s_off > s_total - q.s_len || q.t_off > t_total - q.t_len)
      return fail(ctx, EAPDTW_EINVAL, "pair " + std::to_string(p) + ": outside its pool");
    const int64_t r = clip_window(q.window, q.s_len, q.t_len);
    if (q.s_len > 0 && q.t_len > 0 && wf_class_for((int)q.s_len, (int)q.t_len, (int)r) < 0)
      return fail(ctx, EAPDTW_EINVAL,
                  "pair " + std::to_string(p) +
                      ": more than 511 rows active at once, or s_len + t_len above 16318");
    hp[(size_t)p] = WfHostPair{q.s_off, q.t_off, q.s_len, q.t_len, r};
  }
  if (disjoint) {
    for (int side = 0; side < 2; ++side) {
      std::vector<std::pair<int64_t, int64_t>> iv;
      iv.reserve(hp.size());
      for (const auto &h : hp) {
        const int64_t o = side ? h.t_off : h.s_off, l = side ? h.lt : h.ls;
        if (l > 0) iv.emplace_back(o, o + l);
      }
      std::sort(iv.begin(), iv.end());
      for (size_t k = 1; k < iv.size(); ++k)
        if (iv[k].first < iv[k - 1].second)
          return fail(ctx, EAPDTW_EINVAL, side ? "pairs overlap in T" : "pairs overlap in S");
    }
  }
  return EAPDTW_OK;
}

// Kernel class of a distance-only sweep in a launch of npairs pairs: by size
// and launch width, or with the lanes per pair that option wf_lanes asks for,
// if such a class holds the pair.
static int wf_pick(const eapdtw_ctx *ctx, int64_t ls, int64_t lt, int64_t r, int64_t npairs) {
  if (ls == 0 || lt == 0) return 0;
  if (ctx && ctx->wf_lanes) {
    const int c = wf_choose((int)ls, (int)lt, (int)r, npairs, (int)ctx->wf_lanes, false);
    if (c >= 0) return c;
  }
  return wf_choose((int)ls, (int)lt, (int)r, npairs, 0, false);
}

// Launch groups of a planned batch: (class, mode); mode 0 distances, 1 codes
// to memory (then the walk kernel), 2 codes in LDS and the backtrack in the
// forward.
constexpr int kWfGroups = 3 * kWfClasses;

// A recorded batch in one device buffer (the caller's record or scratch):
// the status word of every pair, the path ranges in the layout of the two
// pools (pair p's rows at s_off, columns at t_off) and the code words of the
// pairs whose sweep keeps them in memory (mode 1).
struct WfRecLayout {
  size_t status = 0, rowrng = 0, colrng = 0, codes = 0, bytes = 0;
};

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

static WfRecLayout wf_layout(int64_t npairs, int64_t s_extent, int64_t t_extent,
                             int64_t code_words) {
  WfRecLayout L;
  L.status = 0;
  L.rowrng = align256(sizeof(unsigned) * (size_t)npairs);
  L.colrng = L.rowrng + align256(sizeof(unsigned) * (size_t)s_extent);
  L.codes = L.colrng + align256(sizeof(unsigned) * (size_t)t_extent);
  L.bytes = L.codes + sizeof(unsigned) * (size_t)code_words;
  if (L.bytes < 4) L.bytes = 4;
  return L;
}

// Per-pair device descriptors and per-group launch orders (most steps first).
struct WfBatchPlan {
  std::vector<WfPair> desc;
  std::vector<int32_t> order;       // pairs grouped by launch group
  int64_t begin[kWfGroups + 1] = {};
  int lds_stride[kWfGroups] = {};
  int max_chunks[kWfGroups] = {};   // record chunks of the group's longest pair
  int max_ranges[kWfGroups] = {};   // ls + lt of the group's longest pair
  int64_t code_words = 0;
  int64_t s_extent = 0, t_extent = 0;
  uint64_t band_cells = 0;
};

// path = false: distance-only classes (mode 0, ctx options apply); true:
// recorded classes (mode 2 where the codes fit in LDS, else mode 1).
static void wf_plan(const eapdtw_ctx *ctx, const std::vector<WfHostPair> &hp, bool path,
                    WfBatchPlan &pl) {
  const int64_t n = (int64_t)hp.size();
  pl.desc.resize((size_t)n);
  std::vector<int> grp((size_t)n);
  int64_t cnt[kWfGroups] = {};
  for (int64_t p = 0; p < n; ++p) {
    const WfHostPair &h = hp[(size_t)p];
    int c = 0, mode = 0;
    if (h.ls > 0 && h.lt > 0) {
      if (path) {
        bool fused = false;
        c = wf_path_class((int)h.ls, (int)h.lt, (int)h.r, n, ctx ? (int)ctx->wf_lanes : 0, &fused);
        mode = fused ? 2 : 1;
      } else {
        c = wf_pick(ctx, h.ls, h.lt, h.r, n);
      }
    } else if (path) {
      mode = 2;  // no sweep: the status word only
    }
    const int gi = mode * kWfClasses + c;
    grp[(size_t)p] = gi;
    ++cnt[gi];
    WfPair &d = pl.desc[(size_t)p];
    d.s_off = h.s_off;
    d.t_off = h.t_off;
    d.rec_off = pl.code_words;
    d.ls = (int32_t)h.ls;
    d.lt = (int32_t)h.lt;
    d.r = (int32_t)h.r;
    d.pad = 0;
    if (mode == 1) pl.code_words += wf_rec_words((int)h.ls, (int)h.lt, c);
    const int need = (int)(mode == 2 ? wf_fused_words((int)h.ls, (int)h.lt, c)
                                     : h.ls + h.lt + 2 * kWfPad);
    if (need > pl.lds_stride[gi]) pl.lds_stride[gi] = need;
    const int nch = wf_chunks((int)h.ls, (int)h.lt);
    if (nch > pl.max_chunks[gi]) pl.max_chunks[gi] = nch;
    if (h.ls + h.lt > pl.max_ranges[gi]) pl.max_ranges[gi] = (int)(h.ls + h.lt);
    if (h.s_off + h.ls > pl.s_extent) pl.s_extent = h.s_off + h.ls;
    if (h.t_off + h.lt > pl.t_extent) pl.t_extent = h.t_off + h.lt;
    if (wf_has_path(h)) pl.band_cells += (uint64_t)band_cells_total(h.ls, h.lt, h.r);
  }
  for (int gi = 0; gi < kWfGroups; ++gi) pl.begin[gi + 1] = pl.begin[gi] + cnt[gi];
  pl.order.resize((size_t)n);
  std::vector<int64_t> fill(pl.begin, pl.begin + kWfGroups);
  std::vector<int32_t> idx((size_t)n);
  for (int64_t p = 0; p < n; ++p) idx[(size_t)p] = (int32_t)p;
  std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) {
    return hp[(size_t)x].ls + hp[(size_t)x].lt > hp[(size_t)y].ls + hp[(size_t)y].lt;
  });
  for (int32_t p : idx) pl.order[(size_t)fill[grp[(size_t)p]]++] = p;
}

// Uploads a host array into the scratch at `off` (stream-ordered; the host
// array may be reused once this returns).
static int upload(eapdtw_ctx *ctx, size_t off, const void *src, size_t nbytes) {
  if (nbytes == 0) return EAPDTW_OK;
  HIPCHK(hipMemcpyAsync(ctx->scratch + off, src, nbytes, hipMemcpyHostToDevice, ctx->stream));
  return EAPDTW_OK;
}

// Device pointers of one recorded batch.
struct WfRecPtrs {
  unsigned *status = nullptr, *rowrng = nullptr, *colrng = nullptr, *codes = nullptr;
};

static WfRecPtrs wf_rec_ptrs(void *base, const WfRecLayout &L) {
  char *b = static_cast<char *>(base);
  WfRecPtrs r;
  r.status = reinterpret_cast<unsigned *>(b + L.status);
  r.rowrng = reinterpret_cast<unsigned *>(b + L.rowrng);
  r.colrng = reinterpret_cast<unsigned *>(b + L.colrng);
  r.codes = reinterpret_cast<unsigned *>(b + L.codes);
  return r;
}

// Forward launches of a planned batch, one per launch group present; with a
// record, the recorded modes write into it (ranges to rowrng/colrng).
static int wf_launch_batch(eapdtw_ctx *ctx, const float *S, const float *T, const WfBatchPlan &pl,
                           const WfPair *d_desc, const int32_t *d_order, float *out,
                           const WfRecPtrs *rec, unsigned *rowrng, unsigned *colrng,
                           const float *ub, unsigned long long *cnt) {
  for (int gi = 0; gi < kWfGroups; ++gi) {
    const int64_t n = pl.begin[gi + 1] - pl.begin[gi];
    if (n == 0) continue;
    const int mode = gi / kWfClasses, c = gi % kWfClasses;
    WfArgs a{};
    a.S = S;
    a.T = T;
    a.pairs = d_desc;
    a.order = d_order + pl.begin[gi];
    a.nitems = n;
    a.out = out;
    if (rec) {
      a.rec = rec->codes;
      a.status = rec->status;
      a.rowrng = rowrng;
      a.colrng = colrng;
    }
    a.lds_stride = pl.lds_stride[gi];
    a.ub = ub;
    a.counters = cnt;
    HIPCHK(launch_wf_fwd(c, mode, a, ctx->stream));
    log_launch(ctx, "pair batch: wf_fwd_kernel<%d,%d,%d> %lld pairs", kWfG[c], kWfNC[c], mode, (long long)n);
  }
  return EAPDTW_OK;
}

// The walk kernel for the pairs of mode 1, one launch per class.
static int wf_walk_batch(eapdtw_ctx *ctx, const WfBatchPlan &pl, const WfPair *d_desc,
                         const int32_t *d_order, const WfRecPtrs &rec, unsigned *rowrng,
                         unsigned *colrng) {
  for (int c = 0; c < kWfClasses; ++c) {
    const int gi = kWfClasses + c;
    const int64_t n = pl.begin[gi + 1] - pl.begin[gi];
    if (n == 0) continue;
    WfWalkArgs w{};
    w.pairs = d_desc;
    w.npairs = (int64_t)pl.desc.size();
    w.order = d_order + pl.begin[gi];
    w.nitems = n;
    w.rec = rec.codes;
    w.status = rec.status;
    w.rowrng = rowrng;
    w.colrng = colrng;
    w.max_chunks = pl.max_chunks[gi];
    w.max_ranges = pl.max_ranges[gi];
    HIPCHK(launch_wf_walk(kWfG[c] * kWfNC[c], w, ctx->stream));
    log_launch(ctx, "pair batch: wf_walk_kernel<%d> %lld pairs", kWfG[c] * kWfNC[c], (long long)n);
  }
  return EAPDTW_OK;
}

int eapdtw_dtw_pairs_batch(eapdtw_ctx *ctx, const float *S, int64_t s_total, const float *T,
                           int64_t t_total, const eapdtw_pair *pairs, int64_t npairs,
                           const float *ub, float *out, eapdtw_stats *stats) {
  CHECK_CTX();
  std::vector<WfHostPair> hp;
  int rc = wf_validate(ctx, S, s_total, T, t_total, pairs, npairs, false, hp);
  if (rc) return rc;
  if (npairs > 0 && !out) return fail(ctx, EAPDTW_EINVAL, "out is NULL");
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (npairs == 0) return EAPDTW_OK;
  HIPCHK(hipSetDevice(ctx->device));
  WfBatchPlan pl;
  wf_plan(ctx, hp, false, pl);
  Plan sp;
  const size_t o_cnt = sp.add(kCntBytes);
  const size_t o_desc = sp.add(sizeof(WfPair) * pl.desc.size());
  const size_t o_ord = sp.add(sizeof(int32_t) * pl.order.size());
  rc = ensure_scratch(ctx, sp.off);
  if (rc) return rc;
  unsigned long long *cnt = at<unsigned long long>(ctx, o_cnt);
  if (stats) HIPCHK(hipEventRecord(ctx->ev0, ctx->stream));
  HIPCHK(launch_fill_u64(cnt, 0ull, kCntWords, ctx->stream));
  if ((rc = upload(ctx, o_desc, pl.desc.data(), sizeof(WfPair) * pl.desc.size()))) return rc;
  if ((rc = upload(ctx, o_ord, pl.order.data(), sizeof(int32_t) * pl.order.size()))) return rc;
  if (stats) HIPCHK(hipEventRecord(ctx->ev2, ctx->stream));
  rc = wf_launch_batch(ctx, S, T, pl, at<WfPair>(ctx, o_desc), at<int32_t>(ctx, o_ord), out,
                       nullptr, nullptr, nullptr, ub, cnt);
  if (rc) return rc;
  if (stats) {
    HIPCHK(hipEventRecord(ctx->ev3, ctx->stream));
    HIPCHK(hipEventRecord(ctx->ev1, ctx->stream));
    rc = readback(ctx, o_cnt, kCntBytes);
    if (rc) return rc;
    fill_stats(stats, reinterpret_cast<unsigned long long *>(ctx->pinned), pl.band_cells,
               (uint64_t)npairs, elapsed(ctx->ev0, ctx->ev1), elapsed(ctx->ev2, ctx->ev3));
  }
  return EAPDTW_OK;
}

// Validation of a recorded batch's pairs without a context (for the size query).
static bool wf_plan_of(const eapdtw_pair *pairs, int64_t npairs, std::vector<WfHostPair> &hp) {
  if (npairs < 0 || (npairs > 0 && !pairs)) return false;
  hp.resize((size_t)npairs);
  for (int64_t p = 0; p < npairs; ++p) {
    const eapdtw_pair &q = pairs[p];
    if (q.s_len < 0 || q.t_len < 0 || q.window < 0 || q.s_off < 0 || q.t_off < 0 ||
        q.s_len > kWfMaxLen || q.t_len > kWfMaxLen)
      return false;
    const int64_t r = clip_window(q.window, q.s_len, q.t_len);
    if (q.s_len > 0 && q.t_len > 0 && wf_class_for((int)q.s_len, (int)q.t_len, (int)r) < 0)
      return false;
    hp[(size_t)p] = WfHostPair{q.s_off, q.t_off, q.s_len, q.t_len, r};
  }
  return true;
}

int64_t eapdtw_dtw_batch_record_bytes(const eapdtw_pair *pairs, int64_t npairs) {
  std::vector<WfHostPair> hp;
  if (!wf_plan_of(pairs, npairs, hp)) return -1;
  WfBatchPlan pl;
  wf_plan(nullptr, hp, true, pl);
  return (int64_t)wf_layout(npairs, pl.s_extent, pl.t_extent, pl.code_words).bytes;
}

// A recorded batch: descriptors in scratch and the record's pointers (the
// caller's record, or scratch when `record` is NULL).
struct WfBatchRun {
  WfBatchPlan pl;
  WfPair *desc = nullptr;
  int32_t *order = nullptr;
  WfRecPtrs rec;
  float *dist = nullptr;
};

// `extra` bytes of scratch are reserved after the batch's buffers (offset in
// *o_extra).
static int wf_batch_prepare(eapdtw_ctx *ctx, const std::vector<WfHostPair> &hp, void *record,
                            WfBatchRun &run, size_t extra = 0, size_t *o_extra = nullptr) {
  wf_plan(ctx, hp, true, run.pl);
  const WfRecLayout L = wf_layout((int64_t)hp.size(), run.pl.s_extent, run.pl.t_extent,
                                  run.pl.code_words);
  Plan sp;
  const size_t o_desc = sp.add(sizeof(WfPair) * run.pl.desc.size());
  const size_t o_ord = sp.add(sizeof(int32_t) * run.pl.order.size());
  const size_t o_dist = sp.add(sizeof(float) * run.pl.desc.size());
  const size_t o_rec = record ? 0 : sp.add(L.bytes);
  const size_t o_x = sp.add(extra);
  if (o_extra) *o_extra = o_x;
  int rc = ensure_scratch(ctx, sp.off);
  if (rc) return rc;
  run.desc = at<WfPair>(ctx, o_desc);
  run.order = at<int32_t>(ctx, o_ord);
  run.dist = at<float>(ctx, o_dist);
  run.rec = wf_rec_ptrs(record ? record : ctx->scratch + o_rec, L);
  if ((rc = upload(ctx, o_desc, run.pl.desc.data(), sizeof(WfPair) * run.pl.desc.size())))
    return rc;
  return upload(ctx, o_ord, run.pl.order.data(), sizeof(int32_t) * run.pl.order.size());
}

int eapdtw_dtw_batch_fwd(eapdtw_ctx *ctx, const float *S, int64_t s_total, const float *T,
                         int64_t t_total, const eapdtw_pair *pairs, int64_t npairs, float *out,
                         void *record) {
  CHECK_CTX();
  std::vector<WfHostPair> hp;
  int rc = wf_validate(ctx, S, s_total, T, t_total, pairs, npairs, record != nullptr, hp);
  if (rc) return rc;
  if (npairs > 0 && !out) return fail(ctx, EAPDTW_EINVAL, "out is NULL");
  if (npairs == 0) return EAPDTW_OK;
  HIPCHK(hipSetDevice(ctx->device));
  if (!record) {
    WfBatchPlan pl;
    wf_plan(ctx, hp, false, pl);
    Plan sp;
    const size_t o_desc = sp.add(sizeof(WfPair) * pl.desc.size());
    const size_t o_ord = sp.add(sizeof(int32_t) * pl.order.size());
    if ((rc = ensure_scratch(ctx, sp.off))) return rc;
    if ((rc = upload(ctx, o_desc, pl.desc.data(), sizeof(WfPair) * pl.desc.size()))) return rc;
    if ((rc = upload(ctx, o_ord, pl.order.data(), sizeof(int32_t) * pl.order.size()))) return rc;
    return wf_launch_batch(ctx, S, T, pl, at<WfPair>(ctx, o_desc), at<int32_t>(ctx, o_ord), out,
                           nullptr, nullptr, nullptr, nullptr, nullptr);
  }
  WfBatchRun run;
  if ((rc = wf_batch_prepare(ctx, hp, record, run))) return rc;
  return wf_launch_batch(ctx, S, T, run.pl, run.desc, run.order, out, &run.rec, run.rec.rowrng,
                         run.rec.colrng, nullptr, nullptr);
}

// Walk (mode-1 pairs) + gradient; without a record the recording forward
// runs first into scratch.  With rowrng_out the ranges go to the caller's
// arrays and no gradient is made.
static int wf_batch_backward(eapdtw_ctx *ctx, const float *S, const float *T,
                             const std::vector<WfHostPair> &hp, void *record,
                             const float *grad_out, float *grad_S, float *grad_T,
                             unsigned *rowrng_out, unsigned *colrng_out) {
  WfBatchRun run;
  int rc = wf_batch_prepare(ctx, hp, record, run);
  if (rc) return rc;
  unsigned *rr = rowrng_out ? rowrng_out : run.rec.rowrng;
  unsigned *cr = colrng_out ? colrng_out : run.rec.colrng;
  if (!record || rowrng_out) {
    rc = wf_launch_batch(ctx, S, T, run.pl, run.desc, run.order, run.dist, &run.rec, rr, cr,
                         nullptr, nullptr);
    if (rc) return rc;
  }
  if ((rc = wf_walk_batch(ctx, run.pl, run.desc, run.order, run.rec, rr, cr))) return rc;
  if (!grad_S) return EAPDTW_OK;
  WfGradArgs g{};
  g.pairs = run.desc;
  g.npairs = (int64_t)hp.size();
  for (const WfHostPair &h : hp) {
    if (h.ls > g.max_ls) g.max_ls = (int)h.ls;
    if (h.lt > g.max_lt) g.max_lt = (int)h.lt;
  }
  g.status = run.rec.status;
  g.S = S;
  g.T = T;
  g.rowrng = rr;
  g.colrng = cr;
  g.gout = grad_out;
  g.gS = grad_S;
  g.gT = grad_T;
  HIPCHK(launch_wf_grad(g, ctx->stream));
  log_launch(ctx, "wf_grad_kernel %lld pairs", (long long)g.npairs);
  return EAPDTW_OK;
}

int eapdtw_dtw_batch_bwd(eapdtw_ctx *ctx, const float *S, int64_t s_total, const float *T,
                         int64_t t_total, const eapdtw_pair *pairs, int64_t npairs,
                         const void *record, const float *grad_out, float *grad_S,
                         float *grad_T) {
  CHECK_CTX();
  std::vector<WfHostPair> hp;
  int rc = wf_validate(ctx, S, s_total, T, t_total, pairs, npairs, true, hp);
  if (rc) return rc;
  if (npairs == 0) return EAPDTW_OK;
  if (!grad_out || !grad_S || !grad_T) return fail(ctx, EAPDTW_EINVAL, "NULL gradient buffer");
  HIPCHK(hipSetDevice(ctx->device));
  return wf_batch_backward(ctx, S, T, hp, const_cast<void *>(record), grad_out, grad_S, grad_T,
                           nullptr, nullptr);
}

int eapdtw_dtw_batch_path(eapdtw_ctx *ctx, const float *S, int64_t s_total, const float *T,
                          int64_t t_total, const eapdtw_pair *pairs, int64_t npairs,
                          unsigned *rowrng, unsigned *colrng) {
  CHECK_CTX();
  std::vector<WfHostPair> hp;
  int rc = wf_validate(ctx, S, s_total, T, t_total, pairs, npairs, true, hp);
  if (rc) return rc;
  if (npairs == 0) return EAPDTW_OK;
  if (!rowrng || !colrng) return fail(ctx, EAPDTW_EINVAL, "NULL range buffer");
  HIPCHK(hipSetDevice(ctx->device));
  return wf_batch_backward(ctx, S, T, hp, nullptr, nullptr, nullptr, nullptr, rowrng, colrng);
}

// --------------------------------------------------------------------------- differentiable batch (equal lengths)

// Class of a distance-only sweep of uniform pairs (-1: unsupported).
static int wf_uniform_class(const eapdtw_ctx *ctx, int64_t npairs, int64_t len, int64_t window,
                            int64_t *r_out) {
  const int64_t r = clip_window(window, len, len);
  if (r_out) *r_out = r;
  if (len == 0) return 0;
  if (len > kWfMaxLen) return -1;
  return wf_pick(ctx, len, len, r, npairs);
}

// Class, mode (1 or 2) and record layout of a recorded sweep of uniform pairs.
struct WfUniformRec {
  int cls = 0, mode = 2;
  int64_t r = 0, words = 0;
  WfRecLayout L;
};

static bool wf_uniform_rec(int64_t npairs, int64_t len, int64_t window, int lanes,
                           WfUniformRec &u) {
  u.r = clip_window(window, len, len);
  if (len > kWfMaxLen) return false;
  if (len > 0) {
    if (wf_class_for((int)len, (int)len, (int)u.r) < 0) return false;
    bool fused = false;
    u.cls = wf_path_class((int)len, (int)len, (int)u.r, npairs, lanes, &fused);
    u.mode = fused ? 2 : 1;
  }
  u.words = u.mode == 1 ? wf_rec_words((int)len, (int)len, u.cls) : 0;
  u.L = wf_layout(npairs, npairs * len, npairs * len, npairs * u.words);
  return true;
}

int64_t eapdtw_dtw_ckpt_bytes(int64_t npairs, int64_t len, int64_t window) {
  if (npairs < 0 || len < 0 || window < 0) return -1;
  WfUniformRec u;
  if (!wf_uniform_rec(npairs, len, window, 0, u)) return -1;
  return (int64_t)u.L.bytes;
}

static int diff_validate(eapdtw_ctx *ctx, const float *S, const float *T, int64_t npairs,
                         int64_t len, int64_t window) {
  if (npairs < 0 || len < 0) return fail(ctx, EAPDTW_EINVAL, "negative size");
  if (window < 0) return fail(ctx, EAPDTW_EINVAL, "window < 0");
  if (npairs > INT_MAX) return fail(ctx, EAPDTW_EINVAL, "too many pairs");
  if (npairs > 0 && len > 0 && (!S || !T)) return fail(ctx, EAPDTW_EINVAL, "NULL pointer");
  WfUniformRec u;
  if (!wf_uniform_rec(npairs, len, window, 0, u))
    return fail(ctx, EAPDTW_EINVAL,
                "the differentiable batch supports lengths up to 8159 (both series in a "
                "wave's LDS) with at most 511 rows active at once (min(window + 1, len) <= 511)");
  return EAPDTW_OK;
}

// Recorded forward of uniform pairs into the layout u at `base`; ranges to
// rr / cr (the record's own unless given).
static int wf_uniform_rec_fwd(eapdtw_ctx *ctx, const float *S, const float *T, int64_t npairs,
                              int64_t len, const WfUniformRec &u, void *base, float *out,
                              unsigned *rr, unsigned *cr) {
  const WfRecPtrs p = wf_rec_ptrs(base, u.L);
  WfArgs a{};
  a.S = S;
  a.T = T;
  a.nitems = npairs;
  a.ls = a.lt = (int)len;
  a.r = (int)u.r;
  a.rec_words_u = u.words;
  a.out = out;
  a.rec = p.codes;
  a.status = p.status;
  a.rowrng = rr ? rr : p.rowrng;
  a.colrng = cr ? cr : p.colrng;
  a.lds_stride = (int)(u.mode == 2 ? wf_fused_words((int)len, (int)len, u.cls)
                                   : 2 * len + 2 * kWfPad);
  HIPCHK(launch_wf_fwd(u.cls, u.mode, a, ctx->stream));
  log_launch(ctx, "pairs %lld x %lld r=%d: wf_fwd_kernel<%d,%d,%d>", (long long)a.nitems, (long long)len, a.r,
             kWfG[u.cls], kWfNC[u.cls], u.mode);
  return EAPDTW_OK;
}

int eapdtw_dtw_kernel_class(eapdtw_ctx *ctx, int64_t npairs, int64_t len, int64_t window,
                            int recorded, int64_t *lanes, int64_t *slots, int64_t *codes_in_lds) {
  CHECK_CTX();
  if (npairs < 0 || len < 0 || window < 0) return fail(ctx, EAPDTW_EINVAL, "negative size");
  int c = 0;
  bool lds = false;
  if (recorded) {
    WfUniformRec u;
    if (!wf_uniform_rec(npairs, len, window, (int)ctx->wf_lanes, u))
      return fail(ctx, EAPDTW_EINVAL, "unsupported sizes for the differentiable batch");
    c = u.cls;
    lds = u.mode == 2;
  } else {
    int64_t r = 0;
    c = wf_uniform_class(ctx, npairs, len, window, &r);
    if (c < 0) return fail(ctx, EAPDTW_EINVAL, "unsupported sizes for the differentiable batch");
  }
  if (lanes) *lanes = kWfG[c];
  if (slots) *slots = kWfNC[c];
  if (codes_in_lds) *codes_in_lds = lds ? 1 : 0;
  return EAPDTW_OK;
}

int eapdtw_dtw_fwd(eapdtw_ctx *ctx, const float *S, const float *T, int64_t npairs, int64_t len,
                   int64_t window, float *out_dist, void *ckpt) {
  CHECK_CTX();
  int rc = diff_validate(ctx, S, T, npairs, len, window);
  if (rc) return rc;
  if (npairs == 0) return EAPDTW_OK;
  if (!out_dist) return fail(ctx, EAPDTW_EINVAL, "NULL output");
  HIPCHK(hipSetDevice(ctx->device));
  if (ckpt) {
    WfUniformRec u;
    wf_uniform_rec(npairs, len, window, (int)ctx->wf_lanes, u);
    return wf_uniform_rec_fwd(ctx, S, T, npairs, len, u, ckpt, out_dist, nullptr, nullptr);
  }
  int64_t r = 0;
  const int c = wf_uniform_class(ctx, npairs, len, window, &r);
  WfArgs a{};
  a.S = S;
  a.T = T;
  a.nitems = npairs;
  a.ls = a.lt = (int)len;
  a.r = (int)r;
  a.out = out_dist;
  a.lds_stride = (int)(2 * len + 2 * kWfPad);
  HIPCHK(launch_wf_fwd(c, 0, a, ctx->stream));
  log_launch(ctx, "pairs %lld x %lld r=%lld: wf_fwd_kernel<%d,%d,0>", (long long)npairs, (long long)len,
             (long long)r, kWfG[c], kWfNC[c]);
  return EAPDTW_OK;
}

// Walk (mode 1) + gradient of uniform pairs; without a record the recorded
// forward runs first into scratch.  With rowrng_out the ranges go there and
// no gradient is made.
static int wf_uniform_backward(eapdtw_ctx *ctx, const float *S, const float *T, int64_t npairs,
                               int64_t len, int64_t window, const void *record,
                               const float *grad_out, float *grad_S, float *grad_T,
                               unsigned *rowrng_out, unsigned *colrng_out, float *dist_out) {
  WfUniformRec u;
  wf_uniform_rec(npairs, len, window, (int)ctx->wf_lanes, u);
  Plan sp;
  const size_t o_dist = sp.add(sizeof(float) * (size_t)npairs);
  const size_t o_rec = record ? 0 : sp.add(u.L.bytes);
  int rc = ensure_scratch(ctx, sp.off);
  if (rc) return rc;
  void *base = record ? const_cast<void *>(record) : ctx->scratch + o_rec;
  const WfRecPtrs p = wf_rec_ptrs(base, u.L);
  unsigned *rr = rowrng_out ? rowrng_out : p.rowrng;
  unsigned *cr = colrng_out ? colrng_out : p.colrng;
  if (!record) {
    rc = wf_uniform_rec_fwd(ctx, S, T, npairs, len, u, base,
                            dist_out ? dist_out : at<float>(ctx, o_dist), rr, cr);
    if (rc) return rc;
  }
  if (u.mode == 1) {
    WfWalkArgs w{};
    w.npairs = npairs;
    w.nitems = npairs;
    w.ls = w.lt = (int)len;
    w.r = (int)u.r;
    w.rec_words_u = u.words;
    w.rec = p.codes;
    w.status = p.status;
    w.rowrng = rr;
    w.colrng = cr;
    w.max_chunks = wf_chunks((int)len, (int)len);
    w.max_ranges = (int)(2 * len);
    HIPCHK(launch_wf_walk(kWfG[u.cls] * kWfNC[u.cls], w, ctx->stream));
    log_launch(ctx, "wf_walk_kernel<%d> %lld pairs", kWfG[u.cls] * kWfNC[u.cls], (long long)w.nitems);
  }
  if (!grad_S) return EAPDTW_OK;
  WfGradArgs g{};
  g.npairs = npairs;
  g.ls = g.lt = (int)len;
  g.status = p.status;
  g.S = S;
  g.T = T;
  g.rowrng = rr;
  g.colrng = cr;
  g.gout = grad_out;
  g.gS = grad_S;
  g.gT = grad_T;
  HIPCHK(launch_wf_grad(g, ctx->stream));
  log_launch(ctx, "wf_grad_kernel %lld pairs", (long long)g.npairs);
  return EAPDTW_OK;
}

int eapdtw_dtw_bwd(eapdtw_ctx *ctx, const float *S, const float *T, int64_t npairs, int64_t len,
                   int64_t window, const void *ckpt, const float *grad_out, float *grad_S,
                   float *grad_T) {
  CHECK_CTX();
  int rc = diff_validate(ctx, S, T, npairs, len, window);
  if (rc) return rc;
  if (npairs == 0 || len == 0) return EAPDTW_OK;
  if (!grad_out || !grad_S || !grad_T) return fail(ctx, EAPDTW_EINVAL, "NULL gradient buffer");
  HIPCHK(hipSetDevice(ctx->device));
  return wf_uniform_backward(ctx, S, T, npairs, len, window, ckpt, grad_out, grad_S, grad_T,
                             nullptr, nullptr, nullptr);
}

int eapdtw_dtw_path(eapdtw_ctx *ctx, const float *S, const float *T, int64_t npairs, int64_t len,
                    int64_t window, float *out_dist, unsigned *rowrng, unsigned *colrng) {
  CHECK_CTX();
  int rc = diff_validate(ctx, S, T, npairs, len, window);
  if (rc) return rc;
  if (npairs == 0 || len == 0) return EAPDTW_OK;
  if (!rowrng || !colrng) return fail(ctx, EAPDTW_EINVAL, "NULL range buffer");
  HIPCHK(hipSetDevice(ctx->device));
  return wf_uniform_backward(ctx, S, T, npairs, len, window, nullptr, nullptr, nullptr, nullptr,
                             rowrng, colrng, out_dist);
}

// --------------------------------------------------------------------------- DBA

int eapdtw_dba_step(eapdtw_ctx *ctx, const float *B, int64_t lb, const float *X, int64_t n,
                    int64_t len, int64_t window, float *out_B, float *out_count) {
  CHECK_CTX();
  if (lb <= 0 || len <= 0 || n <= 0) return fail(ctx, EAPDTW_EINVAL, "empty barycentre or set");
  if (window < 0) return fail(ctx, EAPDTW_EINVAL, "window < 0");
  if (!B || !X || !out_B) return fail(ctx, EAPDTW_EINVAL, "NULL pointer");
  if (n > INT_MAX / 2) return fail(ctx, EAPDTW_EINVAL, "too many series");
  const int64_t r = clip_window(window, lb, len);
  if (std::llabs(lb - len) > r)
    return fail(ctx, EAPDTW_EINVAL, "no warping path: |lb - len| exceeds the window");
  if (lb > kWfMaxLen || len > kWfMaxLen || wf_class_for((int)lb, (int)len, (int)r) < 0)
    return fail(ctx, EAPDTW_EINVAL,
                "more than 511 rows active at once, or series too long for a wave's LDS");
  HIPCHK(hipSetDevice(ctx->device));
  // the pairs (B, X[p]) as a batch over a broadcast copy of B
  std::vector<WfHostPair> hp((size_t)n);
  for (int64_t p = 0; p < n; ++p) hp[(size_t)p] = WfHostPair{p * lb, p * len, lb, len, r};
  const int64_t nchunk = (n + kDbaPairs - 1) / kDbaPairs;
  // scratch beside the batch: the broadcast copy of B and the partial sums
  const size_t b_Bx = align256(sizeof(float) * (size_t)(n * lb));
  const size_t b_p = align256(sizeof(double) * (size_t)(nchunk * lb));
  WfBatchRun run;
  size_t o_x = 0;
  int rc = wf_batch_prepare(ctx, hp, nullptr, run, b_Bx + 2 * b_p, &o_x);
  if (rc) return rc;
  const size_t o_Bx = o_x, o_ps = o_x + b_Bx, o_pc = o_ps + b_p;
  float *Bx = at<float>(ctx, o_Bx);
  HIPCHK(launch_broadcast_rows(B, lb, n, Bx, ctx->stream));
  rc = wf_launch_batch(ctx, Bx, X, run.pl, run.desc, run.order, run.dist, &run.rec,
                       run.rec.rowrng, run.rec.colrng, nullptr, nullptr);
  if (rc) return rc;
  if ((rc = wf_walk_batch(ctx, run.pl, run.desc, run.order, run.rec, run.rec.rowrng,
                          run.rec.colrng)))
    return rc;
  HIPCHK(launch_wf_dba(X, n, (int)len, (int)lb, run.rec.rowrng, run.rec.status,
                       at<double>(ctx, o_ps), at<double>(ctx, o_pc), nchunk, out_B, out_count,
                       ctx->stream));
  return EAPDTW_OK;
}

// --------------------------------------------------------------------------- exposed steps

int eapdtw_window_stats(eapdtw_ctx *ctx, const float *series, int64_t n, int64_t m, double *mean,
                        double *sigma) {
  CHECK_CTX();
  if (!series || !mean || !sigma) return fail(ctx, EAPDTW_EINVAL, "NULL pointer");
  if (m <= 0 || n < m || m > INT_MAX / 4) return fail(ctx, EAPDTW_EINVAL, "bad sizes");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(launch_window_stats(series, n, (int)m, mean, sigma, ctx->stream));
  return EAPDTW_OK;
}

int eapdtw_znorm(eapdtw_ctx *ctx, const float *x, int64_t m, float *out) {
  CHECK_CTX();
  if (!x || !out) return fail(ctx, EAPDTW_EINVAL, "NULL pointer");
  if (m <= 0 || m > INT_MAX / 4) return fail(ctx, EAPDTW_EINVAL, "bad length");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(launch_znorm(x, (int)m, out, ctx->stream));
  return EAPDTW_OK;
}

}  // extern "C"
