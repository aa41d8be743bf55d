// common.h -- shared device/host definitions of the gfx950 EAPrunedDTW kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eapdtw {

constexpr float kInf = __builtin_huge_valf();
constexpr int kWave = 64;

// Largest window handled by the band-in-registers kernels; wider windows go to
// the tiled wide-window kernel.
constexpr int kBandRMax = 64;
// Padding (in elements) on each side of a padded column series: out-of-matrix
// columns hold +inf so that their cells evaluate to +inf.  Twice the largest
// band window, because a row-longer-than-column pair reaches 2r past the end.
constexpr int kColPad = 2 * kBandRMax + 16;
// Widest window of the weighted search (its tiled kernel keeps the 2 r + 1
// weights in LDS).
constexpr int kWtMaxR = 4095;
// Widest window of the lower-bound cascade (its envelopes keep a window of
// 2 r + 1 values per output in LDS).
constexpr int kEnvMaxR = 2048;
// Smallest band window swept between pruning borders (narrower bands gain
// too little to pay for the borders).
constexpr int kBorderMinR = 24;
// Tile heights of the wide-window kernels (banded / whole-matrix windows).
// Banded windows take the tall tiles when 2r + 2 >= kWideBandRowsTall (every
// search window above 64): per column, the boundary load and store, the
// liveness ballot and the counters are shared by twice the cells, which made
// windows 100-150 1.2-1.7x faster than with 16-row tiles.
constexpr int kWideBandRowsTall = 32;
constexpr int kWideBandRows = 16;
constexpr int kWideFullRows = 64;

// Counter slots written by the kernels.  The device array holds kCntStripes
// copies kCntStride words apart (one 128-byte line each); a workgroup adds
// into stripe blockIdx % kCntStripes so that the end-of-wave atomics of tens
// of thousands of workgroups do not serialise on one address.  The host sums
// the stripes.
enum Counter : int {
  kCntEvaluated = 0,  // cells computed for problems still alive
  kCntComputed = 1,   // all lane-cells computed
  kCntAbandoned = 2,  // problems finished as +inf
  kCntNonFinite = 3,  // non-finite input values seen
  kCntLbKim = 4,      // candidates skipped by LB_Kim
  kCntLbEq = 5,       // ... by LB_Keogh with the query's envelope
  kCntLbEc = 6,       // ... by LB_Keogh with the candidate's envelope
  kCntListN = 7,      // survivor list lengths (one word per pass, in stripes 0, 1, ...)
  kCntLbRecheck = 8,  // list entries dropped when the DP pass re-checks their bound
  kCntSlots = 9,
  // not a counter: a k-nearest-neighbour search's kept-candidate count
  // (stripe 0) and its selection's filtered count (stripe 1)
  kCntKnnN = 10,
  // not a counter: word j of the k-nearest-neighbour slots sits at slot
  // kCntKnnSlot of stripe j (own 128-byte line each; cleared with the counters)
  kCntKnnSlot = 15
};
constexpr int kCntStripes = 64;
constexpr int kCntStride = 16;
constexpr int kCntWords = kCntStripes * kCntStride;

__host__ __device__ inline unsigned long long *counter_stripe(unsigned long long *c, unsigned b) {
  return c + (b % kCntStripes) * kCntStride;
}

// Workgroups are dealt to the chip's eight XCDs (each with its own L2) in
// turn: workgroup b runs on XCD b % 8.  xcd_block maps the dispatch index to
// a logical block so that each XCD works through runs of kXcdRun consecutive
// logical blocks (runs dealt to the XCDs in turn): a run's waves share one
// stretch of the series in one L2, while the work along the series stays
// spread evenly over the XCDs.  A bijection on [0, nblocks): blocks past the
// last whole round of runs keep their index.
constexpr int kXcds = 8;
constexpr int kXcdRun = 64;
__host__ __device__ inline int64_t xcd_block(int64_t b, int64_t nblocks) {
  const int64_t round = (int64_t)kXcds * kXcdRun;
  if (b >= nblocks / round * round) return b;
  const int64_t x = b % kXcds, j = b / kXcds;
  return (j / kXcdRun) * round + x * kXcdRun + j % kXcdRun;
}

// The shared best-so-far of a search packs (distance, offset) into one u64 so
// that a single 64-bit atomic min keeps the lexicographic minimum: distances
// are non-negative float32, whose bit patterns order like unsigned integers.
__host__ __device__ inline unsigned long long pack_best(float d, uint32_t k) {
  return ((unsigned long long)__builtin_bit_cast(uint32_t, d) << 32) | k;
}
__host__ __device__ inline float best_dist(unsigned long long b) {
  return __builtin_bit_cast(float, (uint32_t)(b >> 32));
}
__host__ __device__ inline uint32_t best_offset(unsigned long long b) { return (uint32_t)b; }

// Arguments of the subsequence-search band kernel.
struct NNArgs {
  const float *x;                    // series [n]
  int64_t n;
  int m;                             // query length
  const float *qpad;                 // z(query) with kColPad +inf on each side
  unsigned long long *bsf;           // shared best-so-far (packed)
  int64_t k_begin, k_end;            // candidate offsets [k_begin, k_end)
  const unsigned long long *center;  // optional: restrict to the 64-offset block holding center's offset
  const unsigned long long *bsf_init;// optional: start from this word's distance as the bound
                                     // (with center: also min it into bsf first)
  float fixed_ub;                    // per-candidate-distance mode: fixed bound
  float *dists;                      // per-candidate-distance mode: out[k - k_begin]
  unsigned long long *counters;      // kCntWords (nullable)
  int check_interval;                // row groups between best-so-far reloads
  int block_stride;                  // workgroup b covers offsets from k_begin + 64 b stride
  int bound_only;                    // record distance-only bounds (offset field all ones)
  // List mode (candidates that passed the lower bounds): lane l of workgroup b
  // takes list entry 64 b + l of list_n entries (entries from the list
  // arrays' start, which the caller offsets); the entry carries the offset,
  // the z-normalisation constants and the lower bounds of the candidate.
  const unsigned long long *list_n;
  const uint32_t *list_k;
  const float *list_mh, *list_ml, *list_inv;
  const float *list_lbq;             // LB_Keogh with the query's envelope (full sum)
  const float *list_lbmax;           // largest of the three bounds
  const float *uq, *lq;              // envelope of z(query) [m]: tightening of the bound per row
  // k nearest neighbours (knn > 0): bsf holds an upper bound of the k-th best
  // distance (offset field all ones); kept candidates are appended to knn_buf
  // (when given) as packed (distance, offset) words, knn_n counting them.
  int knn;
  unsigned long long *knn_buf;
  unsigned long long *knn_n;
  // the k slot words (kCntStride apart; nullptr: those of the counter array)
  unsigned long long *knn_slots;
  // weighted DTW kernels: the weight of phase difference |i - j| = 0..kBandRMax
  float wgt[kBandRMax + 1];
};

// Largest k of the k-nearest-neighbour search (one wave sorts 64 candidates).
constexpr int kKnnMax = 64;

// Where a k-nearest-neighbour search publishes (see publish_knn).
struct KnnOut {
  unsigned long long *bound;      // upper bound of the k-th best distance (packed)
  int k;
  unsigned long long *buf;        // kept candidates (nullable)
  unsigned long long *n;          // their count
  unsigned long long *counters;   // counter array holding the k slot words (nullable)
  unsigned long long *slots;      // the k slot words instead (nullable)
};

// Relative margin by which float32 lower bounds are lowered before they are
// compared with a distance: their sums round differently from the DP's.
constexpr float kLbMargin = 1.0f / 262144.0f;  // 2^-18

// Arguments of the lower-bound pass (lb.hip).
struct LBArgs {
  const float *x;                    // series [n]
  int64_t n;
  int m, r;
  const float *qz;                   // z(query) [m]
  const float *uq, *lq;              // envelope of z(query) under r [m]
  const float *ux, *lx;              // envelope of the series under r [n]
  int64_t k_begin, k_end;
  int mode;                          // 0 search (bound = best-so-far), 1 fixed bound, 2 bounds only
  unsigned long long *bsf;           // mode 0
  const unsigned long long *bsf_init;// mode 0, optional
  float fixed_ub;                    // mode 1
  float *dists;                      // mode 1: +inf written for skipped candidates
  float *out_kim, *out_eq, *out_ec;  // mode 2: [k - k_begin]
  int use_ec;                        // modes 0, 1: apply the candidate-envelope bound
  unsigned long long *counters;      // kCntWords
  unsigned long long *list_n;        // modes 0, 1: entries appended so far (one word)
  uint32_t *list_k;                  // modes 0, 1: survivor list
  float *list_mh, *list_ml, *list_inv, *list_lbq, *list_lbmax;
};

// Arguments of the pair band kernel.  Row and column series are stored
// transposed (element t of pair p at [t * ld + p]) so that a wave's loads are
// coalesced; the column series is padded with kColPad +inf rows on each side.
struct PairArgs {
  const float *rowsT;     // [lrow][ld]
  const float *colsT;     // [lcol + 2*kColPad][ld]
  int64_t ld;
  int64_t npairs;
  int lrow, lcol;
  int ub_mode;            // 0 none, 1 per-pair array, 2 squared Euclidean distance
  const float *ub;        // [npairs] when ub_mode == 1
  float ub_scalar;        // bound for every pair when ub_mode == 3
  float *out;             // [npairs]
  unsigned long long *counters;
};

// Number of admissible in-matrix cells of row i (0-based) of an lrow x lcol
// matrix under window r.
__host__ __device__ inline int row_cells(int i, int lcol, int r) {
  int lo = i - r < 0 ? 0 : i - r;
  int hi = i + r > lcol - 1 ? lcol - 1 : i + r;
  return hi >= lo ? hi - lo + 1 : 0;
}

}  // namespace eapdtw
