// batch.h -- many queries of uneven length and window against one series in
// one persistent launch.
#pragma once
#include "common.h"

namespace eapdtw {

// Device descriptor of one query of a batch.
struct BatchQuery {
  const float *query;          // raw query [m]
  float *qpad;                 // z(query) with kColPad +inf on each side
  unsigned long long *bsf;     // [0] search, [1] seeding pass
  int m, r;
  int64_t K;                   // candidate offsets n - m + 1
  int64_t unit_begin;          // first work unit (64 offsets each) of the main pass
  int64_t seed_begin;          // first workgroup of the window-0 seeding pass
  int seed_stride;             // that pass visits every seed_stride-th block of the query
  // k nearest neighbours (BatchArgs::knn > 0): bsf[0] bounds the k-th best;
  // kept candidates go to knn_buf (knn_n counting them), the k slot words
  // are knn_slots (kCntStride apart), knn_nsel counts the selection's filter
  unsigned long long *knn_buf, *knn_n, *knn_slots, *knn_nsel;
  unsigned long long *knn_res;  // the k best, packed (distance, offset), ascending
};

struct BatchArgs {
  const BatchQuery *qs;
  int nq;
  const float *x;
  int64_t n;
  int64_t total_units;
  unsigned long long *work;    // work-queue counter (cleared by the graph)
  int chunk;                   // units taken per queue access
  int64_t total_seed_blocks;
  int seed_window;
  float *bnd;
  int64_t bnd_stride;
  unsigned long long *counters;
  int check_interval;
  int knn;                     // 0: nearest neighbour; 1..kKnnMax: k nearest neighbours
};

hipError_t launch_batch_prep(const BatchArgs &a, hipStream_t st);
hipError_t launch_batch_seed(const BatchArgs &a, hipStream_t st);
hipError_t launch_batch_main(const BatchArgs &a, int grid, hipStream_t st);

}  // namespace eapdtw
