// dispatch.h -- host-side entry points of the device kernels.
#pragma once
#include "common.h"

namespace eapdtw {

// border selects the bordered sweep (windows of at least kBorderMinR only).
typedef hipError_t (*NNLaunchFn)(const NNArgs &, int64_t nblocks, int rows_per_group, bool dists,
                                 bool border, hipStream_t);
// List mode: the candidates of the survivor list (see NNArgs); nblocks covers
// the largest possible list, workgroups past its end return at once.
typedef hipError_t (*NNListLaunchFn)(const NNArgs &, int64_t nblocks, bool dists, bool border,
                                     hipStream_t);
typedef hipError_t (*PairLaunchFn)(const PairArgs &, int64_t nblocks, int rows_per_group,
                                   hipStream_t);

// Band search with lane refill (lanes.hip): windows 1..kBandRMax, query
// lengths that are multiples of 4 up to kLaneMaxM, offsets from 0.
constexpr int kLaneMaxM = 2048;
bool lane_search_supported(int r, int m);
hipError_t launch_lane_search(int r, const NNArgs &a, hipStream_t st);

// Window 0: early-abandoned squared Euclidean distance (ed.hip).
hipError_t launch_ed_search(const NNArgs &a, int64_t nblocks, bool dists, hipStream_t st);

// Band-in-registers kernels for windows 0..kBandRMax (nullptr otherwise).
NNLaunchFn nn_band_launcher(int r);
NNListLaunchFn nn_list_launcher(int r);
// Weighted-DTW band search (same signature as the list launcher).
NNListLaunchFn nn_wband_launcher(int r);
PairLaunchFn pair_band_launcher(int r);

// Lower bounds (lb.hip): envelopes of the series and of z(query) under window
// r, then the per-candidate LB_Kim / LB_Keogh pass.
hipError_t launch_envelopes(const float *x, int64_t n, const float *qz, int m, int r, float *ux,
                            float *lx, float *uq, float *lq, hipStream_t st);
hipError_t launch_lb_pass(const LBArgs &a, hipStream_t st);

// k nearest neighbours (knn.hip): from the n_buf words of buf, the k <= kKnnMax
// smallest at or below *bound's distance, ascending, into out[k] (all-ones
// words past the available ones); tmp holds as many words as buf, *n_tmp = 0.
hipError_t launch_knn_select(const unsigned long long *buf, const unsigned long long *n_buf,
                             const unsigned long long *bound, unsigned long long *tmp,
                             unsigned long long *n_tmp, int k, unsigned long long *out,
                             hipStream_t st);

// Wide-window kernels (wide_inst.hip): kind is a WideKind, rows the tile height
// (16, 32 or 64), grid the number of persistent single-wave workgroups.
struct WideArgs;
hipError_t launch_wide(int kind, int rows, const WideArgs &a, int grid, hipStream_t st);
int wide_rows_for(int r, int lrow, int lcol);
// The lower-bound cascade's search over a survivor list with the tiled kernel
// (windows above kBandRMax; WideArgs::list_* set).
hipError_t launch_wide_list(int rows, const WideArgs &a, int grid, hipStream_t st);
// NN1 seeding: every pair's squared Euclidean distance min-ed into both series'
// nearest-neighbour words (pairwise geometry of WideArgs).
hipError_t launch_nn1_seed(const WideArgs &a, int grid, hipStream_t st);

// ERP of a batch of pairs (erp.hip): windows 0..kErpMaxR (r <= len - 1).
constexpr int kErpMaxR = 64;
struct ErpArgs {
  const float *Xt, *Yt;          // [len][ld] transposed series (pair p at column p)
  int64_t ld;                    // row stride of Xt, Yt: at least npairs rounded up to 64
  int64_t npairs;
  int len;
  float g;                       // gap value
  const float *ub;               // [npairs] bound per pair, or nullptr (no bound)
  float *out;                    // [npairs]
  unsigned long long *counters;  // kCntWords (nullable)
};
hipError_t launch_erp_pairs(int r, const ErpArgs &a, hipStream_t st);
// Nearest-neighbour search under ERP (one candidate offset per lane).
struct ErpSearchArgs {
  const float *x;                // series [n]
  int64_t n, K;                  // K = n - m + 1 candidate offsets
  const float *qz;               // z-normalised query [m]
  int m;
  float g;                       // gap value
  unsigned long long *bsf;       // packed (distance, offset) best-so-far, +inf on entry
  int check_interval;            // row groups between best-so-far reads
  unsigned long long *counters;  // kCntWords (nullable)
};
hipError_t launch_erp_search(int r, const ErpSearchArgs &a, hipStream_t st);

// Auxiliary kernels (aux.hip).
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t st);
hipError_t launch_check_finite(const float *x, int64_t n, unsigned long long *counters,
                               hipStream_t st);
// Search set-up in one launch (counters, best-so-far words, padded query,
// series check; x may be null to skip the check).
hipError_t launch_search_prep(const float *q, int m, float *qpad, const float *x, int64_t n,
                              unsigned long long *cnt, unsigned long long *bsf, int nbsf,
                              unsigned *flag, unsigned epoch, hipStream_t st);
hipError_t launch_transpose_pad(const float *src, int64_t npairs, int len, int64_t ld,
                                int pad, float padval, float *dst, hipStream_t st);
hipError_t launch_window_stats(const float *x, int64_t n, int m, double *mean, double *sd,
                               hipStream_t st);
hipError_t launch_znorm(const float *x, int m, float *out, hipStream_t st);
hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t st);
// n copies of src [len] into dst [n][len]
hipError_t launch_broadcast_rows(const float *src, int64_t len, int64_t n, float *dst,
                                 hipStream_t st);

}  // namespace eapdtw
