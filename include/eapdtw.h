/*
 * eapdtw.h -- C ABI of the MI355X (gfx950) early-abandoning pruned DTW library.
 *
 * Method: Herrmann & Webb, "Early Abandoning PrunedDTW and its application to
 * similarity search", arXiv 2010.05371.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - DTW is the recurrence of Section 2 (Eq. 1-5): rows i index the first
 *    series S, columns j index the second series T, cost(a,b) = (a-b)^2 in
 *    float32, M(0,0)=0, M(i,0)=M(0,j)=+inf.
 *  - window r is the Sakoe-Chiba window of Section 2.1: a cell is admissible
 *    iff |i-j| <= r.  r >= max(lS,lT)-1 is unconstrained DTW.  |lS-lT| > r has
 *    no admissible path and yields +inf.  r < 0 is EINVAL.
 *  - ub is the early-abandoning bound of Section 2.2: a result <= ub is the
 *    exact DTW value (bit-identical to the unpruned float32 computation); a
 *    result that would strictly exceed ub is returned as +inf (ties are kept).
 *    ub = +inf computes plain DTW.  ub < 0 returns +inf.  NaN ub is EINVAL.
 *  - Pointers documented as DEVICE point to memory on the context's device
 *    (e.g. torch tensors on ROCm); they are owned by the caller and must stay
 *    valid until the stream reaches the call's end.  HOST pointers are owned by
 *    the caller.  Series are contiguous float32.
 *  - Every call is ordered on the context's stream.  Calls that return values
 *    through HOST pointers synchronise that stream before returning; calls
 *    whose outputs are DEVICE buffers are asynchronous.
 *  - No exception or abort crosses the ABI: every failure is a negative status
 *    code and eapdtw_last_error() describes it.  Argument errors are detected on
 *    the host before any device work is queued.  After a device fault the
 *    context is poisoned and every later call returns EAPDTW_EPOISONED.
 *  - A context is not thread-safe; use one per host thread.
 */
#ifndef EAPDTW_H
#define EAPDTW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EAPDTW_OK 0
#define EAPDTW_EINVAL (-1)     /* invalid argument (checked before any device work) */
#define EAPDTW_ENOMEM (-2)     /* device scratch allocation failed */
#define EAPDTW_EDEVICE (-3)    /* HIP runtime error */
#define EAPDTW_ENODEV (-4)     /* no usable gfx950 device */
#define EAPDTW_ENONFINITE (-5) /* NaN or infinity in the input series */
#define EAPDTW_EPOISONED (-6)  /* an earlier device fault poisoned the context */

typedef struct eapdtw_ctx eapdtw_ctx;

/* Work counters of one call (all optional: pass NULL to skip them).
 *  cells_nominal   : admissible (in-window) cells of every problem
 *  cells_evaluated : cells computed for problems that were still alive
 *  cells_computed  : every cell a SIMD lane computed (>= evaluated)
 *  problems        : candidates (search) or pairs
 *  abandoned       : problems that ended as +inf (strictly above the bound)
 *  kernel_ms       : device time of the whole call between two stream events
 *  main_kernel_ms  : device time of the call's dominant DP kernel alone
 *                    (stream events around that launch)                      */
typedef struct {
  uint64_t cells_nominal;
  uint64_t cells_evaluated;
  uint64_t cells_computed;
  uint64_t problems;
  uint64_t abandoned;
  float kernel_ms;
  float main_kernel_ms;
} eapdtw_stats;

/* One query of a batched search: HOST struct, `query` is a DEVICE pointer. */
typedef struct {
  const float *query;
  int64_t m;
  int64_t window;
} eapdtw_query;

/* One result of a batched search (HOST). */
typedef struct {
  int64_t offset;
  double dist;
} eapdtw_result;

/* Version string of the library. */
const char *eapdtw_version(void);

/* Creates a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * order work on (NULL: the device's null stream).  *out receives the context.
 * Returns ENODEV if the device does not exist or is not gfx950. */
int eapdtw_create(int device, void *hip_stream, eapdtw_ctx **out);

/* Releases the context and its device scratch.  NULL is ignored. */
void eapdtw_destroy(eapdtw_ctx *ctx);

/* Re-targets the context's stream (hipStream_t, NULL = null stream).  The
 * context first waits for its old stream (its scratch may still be in use
 * there), except when the new stream is being captured into a graph, where no
 * wait is allowed: the caller then orders the two streams (as graph capture
 * requires anyway).  Entry points that read results back to the host, or
 * whose scratch must grow, cannot run under capture; the differentiable
 * batch's forward with a record and its backward can, once a first call has
 * sized the scratch. */
int eapdtw_set_stream(eapdtw_ctx *ctx, void *hip_stream);

/* Text of the context's last failure ("" if none).  With ctx == NULL: the
 * calling thread's last eapdtw_create() failure. */
const char *eapdtw_last_error(const eapdtw_ctx *ctx);

/* Tuning knobs (for tests and the autotuner).  Keys:
 *   "check_interval" : row groups between reloads of the shared best-so-far
 *                      (>= 1; 0 = chosen per window, the default)
 *   "seed"           : 1 = seed the best-so-far from a window-0 pass and one
 *                      workgroup of candidates around its best offset (default),
 *                      0 = start the search from +inf
 *   "rows_per_group" : rows handled per group by the band search kernel (2,4,8; 0=auto)
 *   "seed_stride"    : the window-0 seeding pass visits every seed_stride-th block
 *                      of 64 candidates (0 = about 128 blocks per search, the default)
 *   "seed_window"    : window of the seeding workgroup (<= search window)
 *   "batch_grid"     : persistent workgroups of the batched search
 *   "batch_chunk"    : work units taken per queue access in the batched search
 *   "batch_seed_stride": seed_stride of the batched search
 *   "batch_branches" : streams over which the batched search spreads its
 *                      band-window launches, which then run concurrently
 *                      (1-8, default 4; 1 = one after the other)
 *   "wide_rows"      : rows per tile of the whole-matrix-window kernel (32, 64; 0=auto)
 *   "graph"          : 1 = replay batched searches from a captured hipGraph
 *   "force_wide"     : 1 = use the wide-window kernel even for narrow windows
 *   "border"         : 1 = the band search sweeps each row group only between
 *                      its pruning borders (windows >= 24; default), 0 = the
 *                      whole band with row-minimum abandoning; both give the
 *                      same bits for every distance at most the bound
 *   "autotune"       : 1 = searches apply the tuning cache (see eapdtw_autotune)
 *   "ed"             : 1 = window-0 searches and seeding passes use the
 *                      squared-Euclidean kernel (default), 0 = the band kernel
 *                      (same bits)
 *   "lanes"          : 1 = band searches (windows 1-64, query length a multiple
 *                      of 4 up to 2048) give each lane its own stream of
 *                      candidates, refilling a lane as soon as its candidate is
 *                      abandoned, over the whole band; 0 = wave-synchronous
 *                      row groups (default).  Same answers; the refill kernel
 *                      keeps more lanes busy but is slower on this hardware
 *   "lb_ec"          : 1 = the cascade searches (eapdtw_nn_search_lb,
 *                      eapdtw_nn_dists_lb) also apply LB_Keogh with the
 *                      candidate's envelope; 0 = LB_Kim and LB_Keogh with the
 *                      query's envelope only (default: a wave evaluates the third
 *                      bound whenever one of its lanes passed the second, for
 *                      few additional skips)
 *   "lb_probe_div"   : the cascade search first runs bounds and DTW over the
 *                      first K / lb_probe_div candidates, so that the bound pass
 *                      over the rest compares with a tightened best-so-far
 *                      (2..4096; 0 = one pass over all candidates, the default:
 *                      the DTW pass re-checks each survivor's bounds against
 *                      its own best-so-far anyway, and a second pair of
 *                      launches costs more than the probe saves)
 *   "wf_lanes"       : lanes per pair of the wavefront pair kernels (the
 *                      equal-length and uneven batches): 0 = chosen by the
 *                      pair's size and the number of pairs (default), or 16,
 *                      32, 64 when a class with that many lanes holds the pair
 *                      (recorded sweeps: only among the classes that keep the
 *                      pair's codes in LDS, so the record size never depends
 *                      on it).  Same results for every value
 *   "scratch_limit"  : test hook: the largest device scratch (bytes) the
 *                      context may allocate; a call that needs more returns
 *                      ENOMEM without allocating (0 = no limit, the default)
 *   "inject_fault"   : test hook: 1 = the next call on the context fails as if
 *                      the device had reported a fault (EDEVICE, no device
 *                      work is done) and poisons the context: every later
 *                      call returns EPOISONED
 *   "log"            : 1 = one line on stderr per kernel choice ("[eapdtw] "
 *                      then the kernel, its template parameters or class and
 *                      the launch shape); 0 = silent (default, unless the
 *                      environment variable EAPDTW_LOG is set to a value
 *                      other than 0 when the context is created)
 * Returns EINVAL for an unknown key or value. */
int eapdtw_set_option(eapdtw_ctx *ctx, const char *key, int64_t value);
int eapdtw_get_option(const eapdtw_ctx *ctx, const char *key, int64_t *value);

/* ---------------------------------------------------------------------------
 * Single pair: DTW(S, T) under window r and early-abandoning bound ub
 * (Section 2 Eq. 1-5; Section 2.1 window; Section 2.2 bound).
 *   S [lS], T [lT] : DEVICE float32, not normalised by the call.
 *   window         : r >= 0.
 *   ub             : bound (+INFINITY = plain DTW); compared in float32,
 *                    rounded down so that a float32 result <= ub is kept.
 *   out_dist       : HOST, the distance or +INFINITY.
 * lS == lT == 0 gives 0; exactly one empty series gives +inf (Eq. 2-4).
 * Synchronous. */
int eapdtw_dtw(eapdtw_ctx *ctx, const float *S, int64_t lS, const float *T, int64_t lT,
               int64_t window, double ub, double *out_dist, eapdtw_stats *stats);

/* ---------------------------------------------------------------------------
 * Batch of independent pairs of equal length `len` (Section 2 Eq. 1-5).
 *   X, Y [npairs][len] : DEVICE float32 row-major; pair p = (X[p], Y[p]).
 *   ub_mode 0          : no bound (plain DTW), `ub` ignored.
 *   ub_mode 1          : ub [npairs] DEVICE float32, one bound per pair.
 *   ub_mode 2          : the PrunedDTW setting of Section 2.3 -- the bound of
 *                        each pair is its squared Euclidean distance (the
 *                        diagonal path), computed with the same float32
 *                        operations as the diagonal cells, so it never binds.
 *   out [npairs]       : DEVICE float32 distances (+inf when abandoned).
 * Asynchronous on the context's stream. */
int eapdtw_dtw_pairs(eapdtw_ctx *ctx, const float *X, const float *Y, int64_t npairs, int64_t len,
                     int64_t window, int ub_mode, const float *ub, float *out, eapdtw_stats *stats);

/* ---------------------------------------------------------------------------
 * ERP, the edit distance with real penalty (Chen & Ng, VLDB 2004), of a batch
 * of pairs of equal length: an elastic distance with DTW's three moves (the
 * kind the paper's closing outlook carries the method over to) in which a
 * diagonal move costs |S_i - T_j| and a vertical or horizontal move aligns
 * its point with the gap value g at cost |S_i - g| or |T_j - g|.  The
 * Sakoe-Chiba window applies to every cell, borders included: M(0,0) = 0,
 * M(0,j) = M(0,j-1) + |T_j - g| and M(i,0) = M(i-1,0) + |S_i - g| while
 * |i - j| <= r, cells outside the window +inf.  Early abandoning as
 * Section 2.2: a pair whose row of cells all exceed its bound returns +inf.
 *   X, Y [npairs][len] : DEVICE float32 row-major; pair p = (X[p], Y[p]),
 *                        used as given (not normalised).
 *   window             : r >= 0, clamped to len - 1; at most 64 after the
 *                        clamp (EINVAL beyond).
 *   g                  : gap value (finite, taken as float32).
 *   ub                 : DEVICE float32 [npairs], one bound per pair (the
 *                        distance if <= ub[p], else +inf), or NULL: no bound.
 *   out [npairs]       : DEVICE float32 distances.
 * len 0 gives 0 (X and Y may then be NULL).  Values are float32 sums in the recurrence's order; inputs
 * are not checked for non-finite values.  Asynchronous on the context's
 * stream (synchronous when stats is given). */
int eapdtw_erp_pairs(eapdtw_ctx *ctx, const float *X, const float *Y, int64_t npairs, int64_t len,
                     int64_t window, double g, const float *ub, float *out, eapdtw_stats *stats);

/* Nearest-neighbour search under ERP (Section 2.2's search with the outlook's
 * other distance; the matrix and window of eapdtw_erp_pairs): the offset k of
 * series with the smallest ERP between z(series[k..k+m)) (rows) and z(query)
 * (columns), under eapdtw_nn_search's normalisation and tie rule (smallest
 * offset among equal float32 distances).  Every candidate is early-abandoned
 * against the shared best-so-far.
 *   query [m], series [n] : DEVICE float32; window clamped to m - 1, at most
 *                           64 after the clamp (EINVAL beyond).
 *   g                     : gap value in normalised units (finite).
 *   out_offset, out_dist  : HOST.
 * Errors as eapdtw_nn_search (non-finite input: ENONFINITE).  Synchronous. */
int eapdtw_nn_search_erp(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                         int64_t n, int64_t window, double g, int64_t *out_offset, double *out_dist,
                         eapdtw_stats *stats);

/* ---------------------------------------------------------------------------
 * All pairwise distances of N series (Section 2.3: pruning with the squared
 * Euclidean distance as the only bound, e.g. for 1-NN classification).
 *   X [N][len] : DEVICE float32 row-major.
 *   out_D      : DEVICE float32 [N*(N-1)/2], the strict upper triangle in
 *                row-major order: pair (i,j), i<j, at
 *                i*N - i*(i+1)/2 + (j-i-1); the pair's rows are X[i], columns X[j].
 * Asynchronous. */
int eapdtw_pairwise(eapdtw_ctx *ctx, const float *X, int64_t N, int64_t len, int64_t window,
                    float *out_D, eapdtw_stats *stats);

/* ---------------------------------------------------------------------------
 * Nearest-neighbour subsequence search (Section 2.2 early abandoning against
 * the best-so-far; Section 5, the "no lower bound" configuration: every
 * candidate is evaluated with the pruned, early-abandoned DTW).
 *   query [m]   : DEVICE float32; z-normalised by the call (population sigma).
 *   series [n]  : DEVICE float32; every offset k in [0, n-m] is a candidate
 *                 z-normalised on the fly; a window with zero deviation
 *                 normalises to all zeros.
 *   window      : r >= 0.
 *   out_offset  : HOST, the smallest offset among the minimal distances.
 *   out_dist    : HOST, that distance (float32 value widened).
 * m == 0, n < m: EINVAL.  Non-finite values in query or series: ENONFINITE.
 * Synchronous. */
int eapdtw_nn_search(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                     int64_t n, int64_t window, int64_t *out_offset, double *out_dist,
                     eapdtw_stats *stats);

/* ---------------------------------------------------------------------------
 * Many queries of uneven length and window against one series (Section 2.2's
 * search per query; each query's answer is that of eapdtw_nn_search), replayed
 * as one captured hipGraph.  Queries with windows above 64 share one
 * persistent launch whose workgroups take 64-offset units from a device work
 * queue; queries with windows up to 64 each get their own band-kernel launch,
 * spread over concurrent streams (option "batch_branches"): measured faster
 * than feeding those windows through the persistent tiled kernel, whose
 * per-tile boundary traffic the band kernels do not pay.
 *   qs [nq] : HOST array of queries (query pointers are DEVICE).
 *   out [nq]: HOST results.
 * Synchronous. */
int eapdtw_nn_search_batch(eapdtw_ctx *ctx, const eapdtw_query *qs, int64_t nq,
                           const float *series, int64_t n, eapdtw_result *out,
                           eapdtw_stats *stats);

/* ---------------------------------------------------------------------------
 * The batched search with a top-k bound per query: the k nearest neighbours
 * (Section 2.2's NN search with the k-th best distance as the bound, as in
 * eapdtw_knn_search) of every query of the batch, in the same launches as
 * eapdtw_nn_search_batch (band launches, persistent tiled launch, hipGraph
 * replay) with a bound word, k slot words and a buffer of kept candidates per
 * query, then per query the filter and the k-best selection.
 *   k           : 1..64, the same for every query.
 *   out_offsets : HOST [nq][k], query q's k offsets ascending by (distance,
 *                 offset), in the order of qs; -1 past the n-m+1 offsets.
 *   out_dists   : HOST [nq][k], their distances; +inf past the offsets.
 * The kept-candidate buffers take 16 bytes per candidate offset of every
 * query (device memory of the context's batch buffer).  Errors as
 * eapdtw_nn_search_batch; k outside 1..64: EINVAL.  Synchronous. */
int eapdtw_knn_search_batch(eapdtw_ctx *ctx, const eapdtw_query *qs, int64_t nq,
                            const float *series, int64_t n, int64_t k, int64_t *out_offsets,
                            double *out_dists, eapdtw_stats *stats);

/* ---------------------------------------------------------------------------
 * Autotuning of the search kernels (a tuning aid; the paper has no
 * counterpart).  Choices are kept per bucket of (query length, window):
 * length bucket = bit length of m; window bucket = 0 for r = 0, bit length of
 * r for 1 <= r <= 64 (band kernels), 8 + bit length of r beyond (tiled
 * kernel), 31 for a window covering the whole query; bucket = 32 x length
 * bucket + window bucket.
 *   rows_per_group : band kernel rows per group (2, 4, 8; 0 = default)
 *   border         : bordered band sweep on/off (windows >= 24)
 *   check_interval : row groups between best-so-far reads (0 = automatic)
 *   wide_rows      : tile height of the whole-window tiled kernel (0, 32, 64)
 *   lanes          : band windows: 0 = 64 candidates per wave in lockstep row
 *                    groups, 1 = each lane streams its own candidates (option
 *                    "lanes"; single searches only, the batch ignores it)
 *   ms             : measured time of the sample search with these choices */
typedef struct {
  int64_t rows_per_group, border, check_interval, wide_rows;
  int64_t lanes;
  float ms;
} eapdtw_tune;

/* Times every candidate choice for `query` [m] (DEVICE) under `window` on the
 * first sample_n points of `series` (DEVICE; at least m + 64 Ki points are
 * used when available), records the fastest in the context's cache under the
 * query's bucket and returns it in *out (may be NULL).  With option
 * "autotune" = 1, eapdtw_nn_search, eapdtw_nn_dists and eapdtw_nn_search_batch
 * apply the recorded choices of each query's bucket, and the batch tunes a
 * bucket it has no record for on first use.  Off by default: the defaults
 * were chosen from the same sweeps, and on the 64-query batched workload the
 * tuned choices were not faster than them.  Synchronous. */
int eapdtw_autotune(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                    int64_t n, int64_t window, int64_t sample_n, eapdtw_tune *out);

/* Bucket of (m, window) as described above, and the cached record of a bucket
 * (EINVAL when none). */
int64_t eapdtw_tune_bucket(int64_t m, int64_t window);
int eapdtw_tune_get(const eapdtw_ctx *ctx, int64_t bucket, eapdtw_tune *out);

/* The cache as JSON, {"arch": "gfx950", "entries": [{"bucket": b, ...}, ...]}:
 * save writes the file; load merges a file written for the same arch
 * (EINVAL for another arch or an unreadable file).  Host-only. */
int eapdtw_tune_save(const eapdtw_ctx *ctx, const char *path);
int eapdtw_tune_load(eapdtw_ctx *ctx, const char *path);

/* ---------------------------------------------------------------------------
 * Differentiable batch of equal-length pairs (Section 2: DTW is the cost of an
 * optimal warping path; its gradient is the gradient of that path's cost,
 * dD/dS(i) = 2 sum_j (S(i)-T(j)), dD/dT(j) = -2 sum_i (S(i)-T(j)) over the
 * path cells).  Each pair is swept by 16, 32 or 64 SIMD lanes along the
 * anti-diagonals of its band, one matrix row per lane and cell slot (1-8
 * slots); no bound, plain DTW.
 *   S, T [npairs][len] : DEVICE float32, row-major.
 *   window             : r >= 0 (clipped to len - 1).  Supported: len <= 8159
 *                        (a pair's two series sit in one wave's 64 KB of
 *                        LDS) and min(window + 1, len) <= 511 (rows active
 *                        at once); otherwise EINVAL.
 *
 * eapdtw_dtw_ckpt_bytes: size of the record the forward leaves for the
 *   backward: a status word per pair and the optimal path as one column range
 *   per row and one row range per column (ties: the diagonal, then (i-1,j),
 *   then (i,j-1)); when a pair's 2-bit argmin codes (one per swept cell) do
 *   not fit in LDS beside its series, also those codes, which the backward
 *   then follows.  The len x len matrix is never stored.  -1 for unsupported
 *   sizes.
 * eapdtw_dtw_fwd: out_dist [npairs] DEVICE.  ckpt: DEVICE buffer of
 *   eapdtw_dtw_ckpt_bytes bytes that receives the record (consumed by
 *   eapdtw_dtw_bwd), or NULL for the distances alone (the backward then
 *   sweeps the forward again).  With a record, each pair's forward follows its
 *   codes back from (len,len) to (1,1) when they are held in LDS.  A pair with
 *   a non-finite value gets NaN.  Asynchronous.
 * eapdtw_dtw_bwd: takes the path from the record (following the recorded
 *   codes first where the forward kept them in memory; ckpt = NULL: the
 *   forward is swept again with a record in the context's scratch) and writes
 *   grad_S[p][i] = 2 g sum over the path cells (i,j) of (S(i)-T(j)),
 *   grad_T[p][j] = -2 g sum over the path cells (i,j) of (S(i)-T(j)),
 *   g = grad_out[p]; a pair with a non-finite value gets NaN gradients.
 *   grad_out [npairs], grad_S, grad_T [npairs][len]: DEVICE float32
 *   (overwritten).  Asynchronous. */
int64_t eapdtw_dtw_ckpt_bytes(int64_t npairs, int64_t len, int64_t window);
int eapdtw_dtw_fwd(eapdtw_ctx *ctx, const float *S, const float *T, int64_t npairs, int64_t len,
                   int64_t window, float *out_dist, void *ckpt);
int eapdtw_dtw_bwd(eapdtw_ctx *ctx, const float *S, const float *T, int64_t npairs, int64_t len,
                   int64_t window, const void *ckpt, const float *grad_out, float *grad_S,
                   float *grad_T);

/* The kernel class eapdtw_dtw_fwd would use for this batch: lanes per pair
 * (16, 32, 64) and matrix rows per lane and anti-diagonal step (1-8); for a
 * recorded forward (recorded != 0) also whether the argmin codes stay in LDS
 * (the forward then recovers the path itself).  Any output may be NULL.
 * Host only; depends on option "wf_lanes".  EINVAL for unsupported sizes. */
int eapdtw_dtw_kernel_class(eapdtw_ctx *ctx, int64_t npairs, int64_t len, int64_t window,
                            int recorded, int64_t *lanes, int64_t *slots, int64_t *codes_in_lds);

/* The optimal warping path of each pair of an equal-length batch, as the
 * backward follows it (Section 2; ties as above), and the distances.
 *   out_dist [npairs] : DEVICE float32 (may be NULL).
 *   rowrng, colrng [npairs][len] : DEVICE uint32.  rowrng[p][i] =
 *     jlo | jhi << 16: the path cells of row i (0-based) are the columns
 *     jlo..jhi; colrng[p][j] = ilo | ihi << 16 likewise for column j.  A path
 *     is monotone, so these ranges describe it completely.  Pairs with a
 *     non-finite value are left untouched.
 * Asynchronous. */
int eapdtw_dtw_path(eapdtw_ctx *ctx, const float *S, const float *T, int64_t npairs, int64_t len,
                    int64_t window, float *out_dist, unsigned *rowrng, unsigned *colrng);

/* ---------------------------------------------------------------------------
 * Batches of pairs of uneven length and window (Section 2, Eq. 1-5 for
 * lS != lT; Section 2.1 window per pair).  Series live in two DEVICE pools:
 * pair p is S[s_off .. s_off + s_len) against T[t_off .. t_off + t_len) under
 * window r_p (clipped to max(s_len, t_len) - 1; |s_len - t_len| > r_p has no
 * warping path: +inf).  Pairs are grouped by kernel class (16, 32 or 64 lanes
 * per pair, 1-8 rows per lane) and run longest first, one launch per group.
 * Supported: lengths up to 8191 with s_len + t_len <= 16318 (a pair's two
 * series sit in one wave's 64 KB of LDS) and min(r_p + 1, s_len, t_len) <=
 * 511 (rows active at once); otherwise EINVAL.  Both series empty: 0; one empty: +inf (Eq. 2-4).
 *   pairs [npairs] : HOST array (copied before the call returns). */
typedef struct {
  int64_t s_off, s_len;
  int64_t t_off, t_len;
  int64_t window;
} eapdtw_pair;

/* Distances with an optional early-abandoning bound (Section 2.2): ub [npairs]
 * DEVICE float32 or NULL; a distance strictly above its bound is +inf, and a
 * pair stops as soon as every cell of two consecutive anti-diagonals exceeds
 * its bound (every warping path crosses one of them).  A pair with a
 * non-finite value gets NaN.  out [npairs]: DEVICE.  Asynchronous unless
 * stats are requested. */
int eapdtw_dtw_pairs_batch(eapdtw_ctx *ctx, const float *S, int64_t s_total, const float *T,
                           int64_t t_total, const eapdtw_pair *pairs, int64_t npairs,
                           const float *ub, float *out, eapdtw_stats *stats);

/* Differentiable form (as eapdtw_dtw_fwd / eapdtw_dtw_bwd): the record size
 * (-1 when unsupported), the forward (record may be NULL) and the backward
 * into pool-shaped gradients grad_S [s_total], grad_T [t_total] (elements
 * outside every pair are not written).  A forward with a record and the
 * backward need pairs whose S regions do not overlap, nor their T regions
 * (EINVAL otherwise: the record holds the path ranges in the pools' layout);
 * the backward must get the same pairs as the forward that wrote the record. */
int64_t eapdtw_dtw_batch_record_bytes(const eapdtw_pair *pairs, int64_t npairs);
int eapdtw_dtw_batch_fwd(eapdtw_ctx *ctx, const float *S, int64_t s_total, const float *T,
                         int64_t t_total, const eapdtw_pair *pairs, int64_t npairs, float *out,
                         void *record);
int eapdtw_dtw_batch_bwd(eapdtw_ctx *ctx, const float *S, int64_t s_total, const float *T,
                         int64_t t_total, const eapdtw_pair *pairs, int64_t npairs,
                         const void *record, const float *grad_out, float *grad_S,
                         float *grad_T);
/* Path ranges of each pair, pool-shaped: rowrng [s_total], colrng [t_total]
 * DEVICE uint32 (as eapdtw_dtw_path; disjoint pairs).  Asynchronous. */
int eapdtw_dtw_batch_path(eapdtw_ctx *ctx, const float *S, int64_t s_total, const float *T,
                          int64_t t_total, const eapdtw_pair *pairs, int64_t npairs,
                          unsigned *rowrng, unsigned *colrng);

/* ---------------------------------------------------------------------------
 * One DTW barycentre averaging (DBA) update (the barycentre use of the path
 * named in Section 6's outlook; Petitjean, Ketterlin & Gancarski, 2011): with
 * the optimal warping path of every pair (B, X[p]) under the window (Section
 * 2; ties as above), each point i of B becomes the mean of the values X[p][j]
 * its paths align with it.
 *   B [lb], X [n][len] : DEVICE float32.
 *   out_B [lb]         : DEVICE float32, sum / count (sums in float64).
 *   out_count [lb]     : DEVICE float32 or NULL, the number of aligned values.
 * |lb - len| beyond the window, empty inputs or unsupported sizes (as the
 * differentiable batch): EINVAL.  Asynchronous. */
int eapdtw_dba_step(eapdtw_ctx *ctx, const float *B, int64_t lb, const float *X, int64_t n,
                    int64_t len, int64_t window, float *out_B, float *out_count);

/* ---------------------------------------------------------------------------
 * Exposed steps of the search, for tests.
 * Window statistics of every offset k in [0, n-m]: mean and population
 * standard deviation of series[k..k+m), as the search computes them.
 *   mean, sigma [n-m+1] : DEVICE float64.  Asynchronous. */
int eapdtw_window_stats(eapdtw_ctx *ctx, const float *series, int64_t n, int64_t m, double *mean,
                        double *sigma);

/* z-normalised copy of x [m] (population sigma, zero deviation -> zeros).
 *   x, out [m] : DEVICE float32.  Asynchronous. */
int eapdtw_znorm(eapdtw_ctx *ctx, const float *x, int64_t m, float *out);

/* Per-candidate early-abandoned distances of a search against a fixed bound:
 *   out[k] = EAP(z(query), z(series[k..k+m)), window, ub) for k in [0, n-m].
 *   out [n-m+1] : DEVICE float32.  Asynchronous. */
int eapdtw_nn_dists(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                    int64_t n, int64_t window, float ub, float *out, eapdtw_stats *stats);

/* ---------------------------------------------------------------------------
 * Search with the lower-bound cascade in front of the DTW (Section 2.2: a
 * lower bound strictly above the bound skips the candidate; Section 5: the
 * search experiments' configuration with the UCR Suite's bounds, and the bound
 * tightened row by row with the cumulative lower bound).
 *
 * Per candidate k, on z-normalised values, in this order:
 *   LB_Kim   : three levels from each end: level a adds the cheapest cell with
 *              max(i,j) = a-1 and the cheapest with min(i,j) = m-a (every warping
 *              path crosses both sets; they are disjoint for 2a <= m);
 *   LB_Keogh : sum over t of the squared distance from z(c_t) to
 *              [L_t, U_t], the envelope (running min / max over t-r..t+r, clipped)
 *              of z(query);
 *   LB_Keogh : sum over t of the squared distance from z(q_t) to the
 *              candidate's envelope: the envelope of the whole series at k+t,
 *              z-normalised with the candidate's mean and sigma (near the
 *              candidate's ends it covers values past them: a wider, still valid
 *              envelope).
 * The third bound is applied with option "lb_ec" = 1 (it is always reported by
 * eapdtw_nn_lower_bounds).
 * Bounds are computed in float32 and lowered by a relative 2^-18 before the
 * comparison (their sums round differently from the DP's).  A candidate that
 * passes all three gets the pruned, early-abandoned DTW, whose bound in row t
 * is the best-so-far minus the rest of its query-envelope LB_Keogh (the terms
 * of the rows below t).  The answer is the eapdtw_nn_search answer; a
 * candidate whose distance is within float32 rounding of the best-so-far may be
 * skipped, which can only change which of two such near-equal candidates is
 * reported.
 *
 * Windows 1..64 take the cascade in front of the band kernels, windows
 * 65..2048 in front of the tiled kernel (survivors swept 64 per wave with
 * their stored normalisation, re-checked against the bound in force, and
 * tightened per tile of rows by the rest of their LB_Keogh below the tile);
 * window 0 (where LB_Keogh is the squared Euclidean
 * distance the window-0 kernel computes anyway), windows above 2048 and
 * option force_wide with a window up to 64 run eapdtw_nn_search's path,
 * reported as every candidate reaching the DTW.
 *
 * Counters of one call (lbstats may be NULL):
 *   pruned_kim, pruned_keogh_eq, pruned_keogh_ec : candidates skipped by
 *     LB_Kim, by LB_Keogh with the query's envelope, with the candidate's
 *     (the bound pass compares with the best-so-far at its start);
 *   pruned_recheck : candidates that passed, skipped when the DTW pass
 *     compares their largest bound with its own, tighter, best-so-far;
 *   dtw_candidates : candidates whose DTW was started;
 *   lb_ms          : device time of the envelopes and the bound pass.
 * In eapdtw_stats, main_kernel_ms is then the DTW pass over the survivors. */
typedef struct {
  uint64_t pruned_kim, pruned_keogh_eq, pruned_keogh_ec, pruned_recheck, dtw_candidates;
  float lb_ms;
} eapdtw_lb_stats;

/* Allocation-free form of eapdtw_nn_search, for callers that cannot allocate
 * device memory (code under graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): same arguments and results (offset and distance,
 * bit for bit), no stats.  It calls no hipMalloc, hipFree or other
 * allocating routine: its counters, best-so-far words and normalised query
 * live in a fixed 64 KiB device array, one per GPU, held until the process
 * ends (looked up at eapdtw_create), and the result comes back through the
 * pinned buffer eapdtw_create allocates.  Limits: window <= 64 (the band and
 * window-0 kernels) and m <= 4096; larger sizes return EINVAL before any
 * device work.  The bound-seeding pass runs on the context's stream before
 * the search.  Every call on one GPU uses that GPU's one array, from any
 * context: calls that overlap in time on one GPU (two streams, two threads)
 * race and must be serialised by the caller.  Synchronous. */
int eapdtw_nn_search_noalloc(eapdtw_ctx *ctx, const float *query, int64_t m,
                             const float *series, int64_t n, int64_t window, int64_t *out_offset,
                             double *out_dist);

/* As eapdtw_nn_search, with the cascade.  Synchronous. */
int eapdtw_nn_search_lb(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                        int64_t n, int64_t window, int64_t *out_offset, double *out_dist,
                        eapdtw_stats *stats, eapdtw_lb_stats *lbstats);

/* As eapdtw_nn_dists, with the cascade against the fixed bound ub: a skipped
 * candidate reads +inf (its distance is above ub).  Asynchronous unless stats
 * or lbstats are requested. */
int eapdtw_nn_dists_lb(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                       int64_t n, int64_t window, float ub, float *out, eapdtw_stats *stats,
                       eapdtw_lb_stats *lbstats);

/* The three bounds of every candidate k in [0, n-m], in full (no skipping):
 *   out_kim, out_eq, out_ec [n-m+1] : DEVICE float32 (LB_Kim, LB_Keogh with
 *   the query's envelope, LB_Keogh with the candidate's envelope).
 * window above 2048 (after clamping to m-1): EINVAL.  Non-finite values:
 * ENONFINITE.  Synchronous. */
int eapdtw_nn_lower_bounds(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                           int64_t n, int64_t window, float *out_kim, float *out_eq,
                           float *out_ec);

/* ---------------------------------------------------------------------------
 * k nearest neighbours of the search (Section 2.2 names NN search and NN1
 * classification; k > 1 keeps an upper bound of the k-th best distance as
 * the early-abandoning bound).  The k smallest (distance, offset) pairs in
 * lexicographic order over every offset k in [0, n-m] (overlapping offsets are
 * not excluded), under eapdtw_nn_search's normalisation and window.
 *   k           : 1..64.
 *   out_offsets : HOST [k], ascending by (distance, offset); -1 past the
 *                 n-m+1 available offsets.
 *   out_dists   : HOST [k], the distances (float32 values widened); +inf past
 *                 the available offsets.
 * Each wave appends its kept candidates to a device buffer and lowers the
 * bound (its own k-th smallest distance when it kept at least k; the largest
 * of k slot words that hold distances of k distinct candidates); a filter and
 * a one-workgroup LDS sort then select the k best.  Every window (band kernels
 * up to 64, the tiled kernel beyond).  Synchronous. */
int eapdtw_knn_search(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                      int64_t n, int64_t window, int64_t k, int64_t *out_offsets,
                      double *out_dists, eapdtw_stats *stats);

/* eapdtw_knn_search behind the lower-bound cascade of eapdtw_nn_search_lb
 * (Section 5's UCR Suite bounds with the k-th best distance as the bound
 * in force): LB_Kim and LB_Keogh skip a candidate whose bound exceeds the
 * bound word, the survivors run the DTW of the list kernels (per-row
 * tightening as in eapdtw_nn_search_lb) and append to the buffer as above.
 * Arguments, outputs and errors as eapdtw_knn_search; lbstats (may be NULL)
 * as eapdtw_nn_search_lb.  The k results are eapdtw_knn_search's, except that
 * a candidate whose distance lies within float32 rounding of the k-th best
 * may be skipped (only the order among such near-equal candidates can
 * change).  Windows 0 and above 2048 run eapdtw_knn_search's path.
 * Synchronous. */
int eapdtw_knn_search_lb(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                         int64_t n, int64_t window, int64_t k, int64_t *out_offsets,
                         double *out_dists, eapdtw_stats *stats, eapdtw_lb_stats *lbstats);

/* ---------------------------------------------------------------------------
 * Leave-one-out nearest neighbour of every series of a set (the NN1
 * classification use of Section 2.2): for each series i, the series j != i with
 * the smallest DTW under the window, the smaller j among equal distances.
 * Every unordered pair is computed once, early-abandoned above the larger of
 * its two series' best distances so far (and pruned with the squared
 * Euclidean distance as in eapdtw_pairwise); a kept distance lowers both
 * series' best.
 *   X [N][len]  : DEVICE float32 row-major, used as given (not normalised).
 *   out_index   : HOST [N] int64, out_dist : HOST [N] (float32 values widened).
 * N < 2 or len < 1: EINVAL.  Synchronous. */
int eapdtw_nn1(eapdtw_ctx *ctx, const float *X, int64_t N, int64_t len, int64_t window,
               int64_t *out_index, double *out_dist, eapdtw_stats *stats);

/* Nearest neighbour of every series of a test set among a separate reference
 * set (NN1 classification): for each test series i, the reference series j with
 * the smallest DTW(Q_i, R_j) under the window, the smaller j on ties.  Every
 * pair is early-abandoned above its test series' best distance so far (and
 * pruned with the squared Euclidean distance); a seeding pass starts each
 * test series from its smallest squared Euclidean distance.
 *   Q [nq][len], R [nr][len] : DEVICE float32 row-major, used as given.
 *   out_index : HOST [nq] int64, out_dist : HOST [nq].
 * Empty sets or len < 1: EINVAL.  Synchronous. */
int eapdtw_nn1_ref(eapdtw_ctx *ctx, const float *Q, int64_t nq, const float *R, int64_t nr,
                   int64_t len, int64_t window, int64_t *out_index, double *out_dist,
                   eapdtw_stats *stats);

/* ---------------------------------------------------------------------------
 * Weighted DTW search, an elastic distance with DTW's recurrence and another
 * cost (the paper's outlook, Section 6: EAPrunedDTW carries over to such
 * distances unchanged, since costs stay non-negative): cell (i, j) costs
 * w(|i-j|) (q_i - c_j)^2 with the modified logistic weight of weighted DTW
 * (Jeong, Jeong & Omitaomu, 2011), w(k) = 1 / (1 + exp(-g (k - m/2))), maximum
 * weight 1, m the query length; weights are computed in double and rounded to
 * float32.  Otherwise as eapdtw_nn_search / eapdtw_nn_dists (z-normalisation,
 * early abandoning, pruning, ties, errors).  Windows up to 64 run the band
 * kernels, wider ones the tiled kernel with the 2r + 1 weights in LDS.  g
 * must be finite; windows above 4095 (after clamping to m-1): EINVAL.
 * eapdtw_nn_search_w: synchronous.  eapdtw_nn_dists_w: asynchronous unless
 * stats are requested. */
int eapdtw_nn_search_w(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                       int64_t n, int64_t window, float g, int64_t *out_offset, double *out_dist,
                       eapdtw_stats *stats);
int eapdtw_nn_dists_w(eapdtw_ctx *ctx, const float *query, int64_t m, const float *series,
                      int64_t n, int64_t window, float g, float ub, float *out,
                      eapdtw_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* EAPDTW_H */
