// api.cpp -- the C ABI (include/eapdtw.h): argument checks, device scratch,
// launch sequencing and result read-back.  All arithmetic of the method runs
// in the device kernels; the host only validates, plans memory and launches.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/eapdtw.h"
#include "dispatch.h"

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
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // options
  int64_t check_interval = 1;
  int64_t seed = 1;
  int64_t rows_per_group = 0;
  int64_t wide_rows = 0;
  int64_t lanes_per_problem = 1;
  int64_t graph = 1;
  int64_t force_wide = 0;
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

int pick_rows(const eapdtw_ctx *ctx, int r) {
  if (ctx->rows_per_group) return (int)ctx->rows_per_group;
  return r == 0 ? 8 : 4;
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

void fill_stats(eapdtw_stats *st, const unsigned long long *cnt, uint64_t nominal,
                uint64_t problems, float ms) {
  if (!st) return;
  st->cells_nominal = nominal;
  st->cells_evaluated = cnt[kCntEvaluated];
  st->cells_computed = cnt[kCntComputed];
  st->problems = problems;
  st->abandoned = cnt[kCntAbandoned];
  st->kernel_ms = ms;
}

}  // namespace

extern "C" {

const char *eapdtw_version(void) { return "eapdtw 0.1 gfx950"; }

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
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    g_create_error = "hipEventCreate failed";
    delete c;
    return EAPDTW_EDEVICE;
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
  delete ctx;
}

int eapdtw_set_stream(eapdtw_ctx *ctx, void *hip_stream) {
  CHECK_CTX();
  if ((hipStream_t)hip_stream != ctx->stream) {
    // scratch may still be in use on the old stream
    HIPCHK(hipStreamSynchronize(ctx->stream));
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
  if (!strcmp(key, "lanes_per_problem")) return &ctx->lanes_per_problem;
  if (!strcmp(key, "graph")) return &ctx->graph;
  if (!strcmp(key, "force_wide")) return &ctx->force_wide;
  return nullptr;
}

int eapdtw_set_option(eapdtw_ctx *ctx, const char *key, int64_t value) {
  if (!ctx) return EAPDTW_EINVAL;
  int64_t *slot = option_slot(ctx, key);
  if (!slot) return fail(ctx, EAPDTW_EINVAL, std::string("unknown option ") + (key ? key : "(null)"));
  bool ok = true;
  if (!strcmp(key, "check_interval")) ok = value >= 1 && value <= (1 << 20);
  else if (!strcmp(key, "seed") || !strcmp(key, "graph") || !strcmp(key, "force_wide")) ok = value == 0 || value == 1;
  else if (!strcmp(key, "rows_per_group")) ok = value == 0 || value == 2 || value == 4 || value == 8;
  else if (!strcmp(key, "wide_rows")) ok = value == 0 || value == 8 || value == 16 || value == 32;
  else if (!strcmp(key, "lanes_per_problem")) ok = value == 1;
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
  PairLaunchFn fn = pair_band_launcher((int)r);
  if (!fn) return fail(ctx, EAPDTW_EINVAL, "window wider than the band kernels (wide-window path not built yet)");
  const int64_t ld = kWave;
  Plan pl;
  size_t o_rows = pl.add(sizeof(float) * lS * ld);
  size_t o_cols = pl.add(sizeof(float) * (lT + 2 * kColPad) * ld);
  size_t o_out = pl.add(sizeof(float) * ld);
  size_t o_cnt = pl.add(sizeof(unsigned long long) * kCntSlots);
  int rc = ensure_scratch(ctx, pl.off);
  if (rc) return rc;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  HIPCHK(hipEventRecord(ctx->ev0, st));
  HIPCHK(launch_fill_u64(at<unsigned long long>(ctx, o_cnt), 0ull, kCntSlots, st));
  HIPCHK(launch_transpose_pad(S, 1, (int)lS, ld, 0, 0.0f, at<float>(ctx, o_rows), st));
  HIPCHK(launch_transpose_pad(T, 1, (int)lT, ld, kColPad, INFINITY, at<float>(ctx, o_cols), st));
  PairArgs a{};
  a.rowsT = at<float>(ctx, o_rows);
  a.colsT = at<float>(ctx, o_cols);
  a.ld = ld;
  a.npairs = 1;
  a.lrow = (int)lS;
  a.lcol = (int)lT;
  a.ub_mode = 3;
  a.ub_scalar = bound_down(ub);
  a.out = at<float>(ctx, o_out);
  a.counters = at<unsigned long long>(ctx, o_cnt);
  HIPCHK(fn(a, 1, pick_rows(ctx, (int)r), st));
  HIPCHK(hipEventRecord(ctx->ev1, st));
  // out (one float) and the counters are read back together
  rc = readback(ctx, o_out, (o_cnt - o_out) + sizeof(unsigned long long) * kCntSlots);
  if (rc) return rc;
  const float d = *reinterpret_cast<float *>(ctx->pinned);
  *out_dist = (double)d;
  if (stats) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    fill_stats(stats, reinterpret_cast<unsigned long long *>(ctx->pinned + (o_cnt - o_out)),
               (uint64_t)band_cells_total(lS, lT, r), 1, ms);
  }
  return EAPDTW_OK;
}

// --------------------------------------------------------------------------- pairs

static int pairs_common(eapdtw_ctx *ctx, const float *X, const float *Y, int64_t npairs,
                        int64_t len, int64_t window, int ub_mode, const float *ub, float *out,
                        eapdtw_stats *stats, float *ckpt, int ckpt_every) {
  if (npairs < 0 || len < 0) return fail(ctx, EAPDTW_EINVAL, "negative size");
  if (window < 0) return fail(ctx, EAPDTW_EINVAL, "window < 0");
  if (ub_mode < 0 || ub_mode > 2) return fail(ctx, EAPDTW_EINVAL, "ub_mode must be 0, 1 or 2");
  if (npairs > 0 && (!X || !Y || !out)) return fail(ctx, EAPDTW_EINVAL, "NULL pointer");
  if (ub_mode == 1 && npairs > 0 && !ub) return fail(ctx, EAPDTW_EINVAL, "ub is NULL with ub_mode 1");
  if (len > INT_MAX / 2) return fail(ctx, EAPDTW_EINVAL, "series too long");
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (npairs == 0) return EAPDTW_OK;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  if (len == 0) {
    HIPCHK(launch_fill_f32(out, 0.0f, npairs, st));
    return EAPDTW_OK;
  }
  const int64_t r = window < len - 1 ? window : len - 1;
  PairLaunchFn fn = pair_band_launcher((int)r);
  if (!fn) return fail(ctx, EAPDTW_EINVAL, "window wider than the band kernels (wide-window path not built yet)");
  const int64_t ld = (npairs + kWave - 1) / kWave * kWave;
  Plan pl;
  size_t o_rows = pl.add(sizeof(float) * len * ld);
  size_t o_cols = pl.add(sizeof(float) * (len + 2 * kColPad) * ld);
  size_t o_cnt = pl.add(sizeof(unsigned long long) * kCntSlots);
  int rc = ensure_scratch(ctx, pl.off);
  if (rc) return rc;
  if (stats) HIPCHK(hipEventRecord(ctx->ev0, st));
  HIPCHK(launch_fill_u64(at<unsigned long long>(ctx, o_cnt), 0ull, kCntSlots, st));
  HIPCHK(launch_transpose_pad(X, npairs, (int)len, ld, 0, 0.0f, at<float>(ctx, o_rows), st));
  HIPCHK(launch_transpose_pad(Y, npairs, (int)len, ld, kColPad, INFINITY, at<float>(ctx, o_cols), st));
  PairArgs a{};
  a.rowsT = at<float>(ctx, o_rows);
  a.colsT = at<float>(ctx, o_cols);
  a.ld = ld;
  a.npairs = npairs;
  a.lrow = (int)len;
  a.lcol = (int)len;
  a.ub_mode = ub_mode;
  a.ub = ub;
  a.out = out;
  a.ckpt = ckpt;
  a.ckpt_every = ckpt_every;
  a.counters = at<unsigned long long>(ctx, o_cnt);
  HIPCHK(fn(a, ld / kWave, pick_rows(ctx, (int)r), st));
  if (stats) {
    HIPCHK(hipEventRecord(ctx->ev1, st));
    rc = readback(ctx, o_cnt, sizeof(unsigned long long) * kCntSlots);
    if (rc) return rc;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    fill_stats(stats, reinterpret_cast<unsigned long long *>(ctx->pinned),
               (uint64_t)(band_cells_total(len, len, r) * npairs), (uint64_t)npairs, ms);
  }
  return EAPDTW_OK;
}

int eapdtw_dtw_pairs(eapdtw_ctx *ctx, const float *X, const float *Y, int64_t npairs, int64_t len,
                     int64_t window, int ub_mode, const float *ub, float *out, eapdtw_stats *stats) {
  CHECK_CTX();
  return pairs_common(ctx, X, Y, npairs, len, window, ub_mode, ub, out, stats, nullptr, 0);
}

int eapdtw_pairwise(eapdtw_ctx *ctx, const float *X, int64_t N, int64_t len, int64_t window,
                    float *out_D, eapdtw_stats *stats) {
  CHECK_CTX();
  (void)X; (void)N; (void)len; (void)window; (void)out_D; (void)stats;
  return fail(ctx, EAPDTW_EINVAL, "pairwise: not built yet");
}

// --------------------------------------------------------------------------- search

struct SearchBufs {
  size_t o_q, o_bsf, o_cnt, o_dists;
};

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

int eapdtw_nn_search(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                     int64_t n, int64_t window, int64_t *out_offset, double *out_dist,
                     eapdtw_stats *stats) {
  CHECK_CTX();
  if (!out_offset || !out_dist) return fail(ctx, EAPDTW_EINVAL, "NULL output");
  int rc = search_validate(ctx, query, m, series, n, window);
  if (rc) return rc;
  if (stats) std::memset(stats, 0, sizeof *stats);
  const int64_t r = window < m - 1 ? window : m - 1;
  NNLaunchFn fn = nn_band_launcher((int)r);
  if (!fn) return fail(ctx, EAPDTW_EINVAL, "window wider than the band kernels (wide-window path not built yet)");
  NNLaunchFn fn0 = nn_band_launcher(0);
  const int64_t K = n - m + 1;
  Plan pl;
  size_t o_bsf = pl.add(sizeof(unsigned long long) * 2);  // [0] search, [1] window-0 pass
  size_t o_cnt = pl.add(sizeof(unsigned long long) * kCntSlots);
  size_t o_q = pl.add(sizeof(float) * (m + 2 * kColPad));
  rc = ensure_scratch(ctx, pl.off);
  if (rc) return rc;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  unsigned long long *bsf = at<unsigned long long>(ctx, o_bsf);
  unsigned long long *cnt = at<unsigned long long>(ctx, o_cnt);
  if (stats) HIPCHK(hipEventRecord(ctx->ev0, st));
  HIPCHK(launch_fill_u64(bsf, pack_best(INFINITY, 0xffffffffu), 2, st));
  HIPCHK(launch_fill_u64(cnt, 0ull, kCntSlots, st));
  HIPCHK(launch_query_prep(query, (int)m, at<float>(ctx, o_q), cnt, st));
  HIPCHK(launch_check_finite(series, n, cnt, st));
  NNArgs a{};
  a.x = series;
  a.n = n;
  a.m = (int)m;
  a.qpad = at<float>(ctx, o_q);
  a.k_begin = 0;
  a.k_end = K;
  a.check_interval = (int)ctx->check_interval;
  const int64_t nblk = (K + kWave - 1) / kWave;
  if (ctx->seed && r > 0) {
    // bound seeding: the window-0 distance (squared Euclidean) of any
    // candidate bounds its DTW, so the best window-0 candidate gives a valid
    // starting bound; one workgroup of candidates around it tightens it.
    NNArgs e = a;
    e.bsf = bsf + 1;
    e.counters = nullptr;
    HIPCHK(fn0(e, nblk, 8, false, st));
    NNArgs s = a;
    s.bsf = bsf;
    s.center = bsf + 1;
    s.bsf_init = bsf + 1;
    s.counters = nullptr;
    HIPCHK(fn(s, 1, pick_rows(ctx, (int)r), false, st));
  }
  a.bsf = bsf;
  a.counters = cnt;
  HIPCHK(fn(a, nblk, pick_rows(ctx, (int)r), false, st));
  if (stats) HIPCHK(hipEventRecord(ctx->ev1, st));
  rc = readback(ctx, o_bsf, (o_cnt - o_bsf) + sizeof(unsigned long long) * kCntSlots);
  if (rc) return rc;
  const unsigned long long best = *reinterpret_cast<unsigned long long *>(ctx->pinned);
  const unsigned long long *hc = reinterpret_cast<unsigned long long *>(ctx->pinned + (o_cnt - o_bsf));
  if (hc[kCntNonFinite]) return fail(ctx, EAPDTW_ENONFINITE, "non-finite value in query or series");
  *out_offset = best_offset(best) == 0xffffffffu ? -1 : (int64_t)best_offset(best);
  *out_dist = (double)best_dist(best);
  if (stats) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    fill_stats(stats, hc, (uint64_t)(band_cells_total(m, m, r) * K), (uint64_t)K, ms);
  }
  return EAPDTW_OK;
}

int eapdtw_nn_dists(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                    int64_t n, int64_t window, float ub, float *out, eapdtw_stats *stats) {
  CHECK_CTX();
  if (!out) return fail(ctx, EAPDTW_EINVAL, "NULL output");
  if (std::isnan(ub)) return fail(ctx, EAPDTW_EINVAL, "ub is NaN");
  int rc = search_validate(ctx, query, m, series, n, window);
  if (rc) return rc;
  if (stats) std::memset(stats, 0, sizeof *stats);
  const int64_t r = window < m - 1 ? window : m - 1;
  NNLaunchFn fn = nn_band_launcher((int)r);
  if (!fn) return fail(ctx, EAPDTW_EINVAL, "window wider than the band kernels (wide-window path not built yet)");
  const int64_t K = n - m + 1;
  Plan pl;
  size_t o_cnt = pl.add(sizeof(unsigned long long) * kCntSlots);
  size_t o_q = pl.add(sizeof(float) * (m + 2 * kColPad));
  rc = ensure_scratch(ctx, pl.off);
  if (rc) return rc;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  unsigned long long *cnt = at<unsigned long long>(ctx, o_cnt);
  if (stats) HIPCHK(hipEventRecord(ctx->ev0, st));
  HIPCHK(launch_fill_u64(cnt, 0ull, kCntSlots, st));
  HIPCHK(launch_query_prep(query, (int)m, at<float>(ctx, o_q), cnt, st));
  NNArgs a{};
  a.x = series;
  a.n = n;
  a.m = (int)m;
  a.qpad = at<float>(ctx, o_q);
  a.k_begin = 0;
  a.k_end = K;
  a.fixed_ub = ub;
  a.dists = out;
  a.counters = cnt;
  a.check_interval = 1;
  HIPCHK(fn(a, (K + kWave - 1) / kWave, 4, true, st));
  if (stats) {
    HIPCHK(hipEventRecord(ctx->ev1, st));
    rc = readback(ctx, o_cnt, sizeof(unsigned long long) * kCntSlots);
    if (rc) return rc;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    fill_stats(stats, reinterpret_cast<unsigned long long *>(ctx->pinned),
               (uint64_t)(band_cells_total(m, m, r) * K), (uint64_t)K, ms);
  }
  return EAPDTW_OK;
}

int eapdtw_nn_search_batch(eapdtw_ctx *ctx, const eapdtw_query *qs, int64_t nq,
                           const float *series, int64_t n, eapdtw_result *out,
                           eapdtw_stats *stats) {
  CHECK_CTX();
  (void)qs; (void)nq; (void)series; (void)n; (void)out; (void)stats;
  return fail(ctx, EAPDTW_EINVAL, "batch search: not built yet");
}

// --------------------------------------------------------------------------- differentiable batch

int64_t eapdtw_dtw_ckpt_bytes(int64_t npairs, int64_t len, int64_t window) {
  (void)npairs; (void)len; (void)window;
  return -1;
}

int eapdtw_dtw_fwd(eapdtw_ctx *ctx, const float *S, const float *T, int64_t npairs, int64_t len,
                   int64_t window, float *out_dist, void *ckpt) {
  CHECK_CTX();
  (void)S; (void)T; (void)npairs; (void)len; (void)window; (void)out_dist; (void)ckpt;
  return fail(ctx, EAPDTW_EINVAL, "forward: not built yet");
}

int eapdtw_dtw_bwd(eapdtw_ctx *ctx, const float *S, const float *T, int64_t npairs, int64_t len,
                   int64_t window, const void *ckpt, const float *grad_out, float *grad_S,
                   float *grad_T) {
  CHECK_CTX();
  (void)S; (void)T; (void)npairs; (void)len; (void)window; (void)ckpt; (void)grad_out;
  (void)grad_S; (void)grad_T;
  return fail(ctx, EAPDTW_EINVAL, "backward: not built yet");
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
