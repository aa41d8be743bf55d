// batch.hip -- batched uneven nearest-neighbour search (gfx950).
//
// Every query of the batch searches the same series (Section 2.2's scan with a
// per-query best-so-far).  The candidates of all queries are cut into work
// units of 64 consecutive offsets; the units of the most expensive queries come
// first.  Persistent single-wave workgroups pull chunks of units from a
// device-wide counter and run the tiled kernel of wide.h on them, so queries
// of any length and window share one launch and the expensive ones are not
// left for the tail.  Bound seeding for all queries is batched in two
// launches before it (window-0 pass, then one workgroup per query).
#include "batch.h"
#include "wide.h"
#include "znorm.h"

namespace eapdtw {

// Last query whose first unit (or seeding workgroup) is <= u.
__device__ __forceinline__ int batch_find(const BatchQuery *qs, int nq, int64_t u, bool seed) {
  int lo = 0, hi = nq - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t b = seed ? qs[mid].seed_begin : qs[mid].unit_begin;
    if (b <= u) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ NNArgs batch_nnargs(const BatchArgs &a, const BatchQuery &q) {
  NNArgs n{};
  n.x = a.x;
  n.n = a.n;
  n.m = q.m;
  n.qpad = q.qpad;
  n.k_begin = 0;
  n.k_end = q.K;
  n.check_interval = a.check_interval;
  n.block_stride = 1;
  return n;
}

// One workgroup per query: normalise it, reset its best-so-far words; the
// first workgroup also resets the work-queue counter.
__global__ void batch_prep_kernel(BatchArgs a) {
  __shared__ double sh[16];
  const BatchQuery &q = a.qs[blockIdx.x];
  const int bad = znorm_block(q.query, q.m, q.qpad, kColPad, sh);
  if (a.knn > 0) {
    // the kept-candidate and filter counts and the k slot words start at 0
    for (int s = threadIdx.x; s < a.knn; s += blockDim.x) q.knn_slots[s * kCntStride] = 0ull;
    if (threadIdx.x == 0) {
      *q.knn_n = 0ull;
      *q.knn_nsel = 0ull;
    }
  }
  if (threadIdx.x == 0) {
    q.bsf[0] = pack_best(kInf, 0xffffffffu);
    q.bsf[1] = pack_best(kInf, 0xffffffffu);
    if (bad && a.counters) atomicAdd(&a.counters[kCntNonFinite], (unsigned long long)bad);
    if (blockIdx.x == 0) *a.work = 0ull;
  }
}

// Window-0 seeding pass over every seed_stride-th block of every query.
__global__ __launch_bounds__(64) void batch_seed0_kernel(BatchArgs a) {
  const int q = batch_find(a.qs, a.nq, blockIdx.x, true);
  const BatchQuery &bq = a.qs[q];
  if (bq.r == 0) return;
  NNArgs n = batch_nnargs(a, bq);
  n.bsf = bq.bsf + 1;
  n.block_stride = bq.seed_stride;
  nn_band_body<0, 8, false>(n, blockIdx.x - bq.seed_begin);
}

// One workgroup per query: the 64-offset block holding the window-0 best, window
// min(r, seed_window); records a distance-only bound.
template <int RS>
__device__ __forceinline__ void batch_seed_rs(const NNArgs &n) {
  nn_band_body<RS, 4, false>(n, 0);
}

__global__ __launch_bounds__(64) void batch_seed_kernel(BatchArgs a) {
  const BatchQuery &bq = a.qs[blockIdx.x];
  if (bq.r == 0) return;
  NNArgs n = batch_nnargs(a, bq);
  n.bsf = bq.bsf;
  n.center = bq.bsf + 1;
  n.bsf_init = bq.bsf + 1;
  n.bound_only = 1;
  if (a.knn > 0) {
    // k nearest neighbours: the window-0 pass only locates this workgroup (its
    // minimum bounds the best, not the k-th best); the workgroup publishes the
    // k-th best of its 64 distances and appends nothing (they are distances
    // under a narrower window)
    n.bsf_init = nullptr;
    n.knn = a.knn;
  }
  const int rs = bq.r < a.seed_window ? bq.r : a.seed_window;
  switch (rs) {
    case 1: batch_seed_rs<1>(n); break;
    case 2: batch_seed_rs<2>(n); break;
    case 3: batch_seed_rs<3>(n); break;
    case 4: batch_seed_rs<4>(n); break;
    case 5: batch_seed_rs<5>(n); break;
    case 6: batch_seed_rs<6>(n); break;
    case 7: batch_seed_rs<7>(n); break;
    default: batch_seed_rs<8>(n); break;
  }
}

// Persistent main pass.
__global__ __launch_bounds__(64) void batch_main_kernel(BatchArgs a) {
  const int lane = threadIdx.x;
  float *Bw = a.bnd + (int64_t)blockIdx.x * a.bnd_stride;
  uint64_t evaluated = 0, computed = 0, abandoned = 0;
  for (;;) {
    unsigned long long u0 = 0;
    if (lane == 0) u0 = atomicAdd(a.work, (unsigned long long)a.chunk);
    u0 = __shfl(u0, 0, kWave);
    if ((int64_t)u0 >= a.total_units) break;
    for (int c = 0; c < a.chunk; ++c) {
      const int64_t unit = (int64_t)u0 + c;
      if (unit >= a.total_units) break;
      const int q = batch_find(a.qs, a.nq, unit, false);
      const BatchQuery &bq = a.qs[q];
      WideArgs w{};
      w.lrow = bq.m;
      w.lcol = bq.m;
      w.r = bq.r < bq.m - 1 ? bq.r : bq.m - 1;
      w.x = a.x;
      w.n = a.n;
      w.qpad = bq.qpad;
      w.bsf = bq.bsf;
      w.k_begin = 0;
      w.k_end = bq.K;
      w.check_interval = a.check_interval;
      if (a.knn > 0) {
        w.knn = a.knn;
        w.knn_buf = bq.knn_buf;
        w.knn_n = bq.knn_n;
        w.knn_slots = bq.knn_slots;
      }
      const int64_t task = unit - bq.unit_begin;
      if (2 * w.r + 2 >= kWideBandRowsTall)
        wide_search_task<kWideBandRowsTall, true>(w, task, Bw, lane, evaluated, computed, abandoned);
      else if (2 * w.r + 2 >= kWideBandRows)
        wide_search_task<kWideBandRows, true>(w, task, Bw, lane, evaluated, computed, abandoned);
      else if (2 * w.r + 2 >= 4)
        wide_search_task<4, true>(w, task, Bw, lane, evaluated, computed, abandoned);
      else
        wide_search_task<2, true>(w, task, Bw, lane, evaluated, computed, abandoned);
    }
  }
  if (a.counters && lane == 0) {
    unsigned long long *cc = counter_stripe(a.counters, blockIdx.x);
    atomicAdd(&cc[kCntEvaluated], (unsigned long long)evaluated);
    atomicAdd(&cc[kCntComputed], (unsigned long long)computed);
    atomicAdd(&cc[kCntAbandoned], (unsigned long long)abandoned);
  }
}

hipError_t launch_batch_prep(const BatchArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(batch_prep_kernel, dim3(a.nq), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_batch_seed(const BatchArgs &a, hipStream_t st) {
  if (a.total_seed_blocks > 0)
    hipLaunchKernelGGL(batch_seed0_kernel, dim3((unsigned)a.total_seed_blocks), dim3(kWave), 0, st, a);
  hipLaunchKernelGGL(batch_seed_kernel, dim3(a.nq), dim3(kWave), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_batch_main(const BatchArgs &a, int grid, hipStream_t st) {
  hipLaunchKernelGGL(batch_main_kernel, dim3(grid), dim3(kWave), 0, st, a);
  return hipGetLastError();
}

}  // namespace eapdtw
