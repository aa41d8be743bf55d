// ed.hip -- the search at window 0: early-abandoned squared Euclidean distance
// of every z-normalised candidate (Section 2.1: a window of zero leaves only
// the diagonal path; Section 2.2: abandon once the running sum passes the
// bound).  Same arithmetic, cell by cell, as the band kernel at window 0, so
// the two give identical bits; this kernel drops the band machinery, whose
// per-row bookkeeping dominates when a row is a single cell.
#include "band.h"
#include "dispatch.h"

namespace eapdtw {

namespace {

constexpr int kEdBlock = 16;  // rows between abandon checks

// Lane l of the workgroup owns candidate kb + l (kb as in the band kernel).
// Per staged stretch of kStageRows rows: the 64 + rows - 1 series values the
// wave reads and the query rows go to LDS with one coalesced copy each.
template <bool DISTS>
__global__ __launch_bounds__(64) void ed_search_kernel(NNArgs a) {
  const int lane = threadIdx.x;
  int64_t kbeg = a.k_begin, kend = a.k_end;
  if (a.center) {
    const unsigned long long c = *a.center;
    int64_t ck = (int64_t)best_offset(c);
    if (ck > kend - 1) ck = kend - 1;
    // the 64-offset block of the search that holds ck: its window statistics
    // (pivot, summation order) and so its z-values are the search's bit for bit
    if (ck < kbeg) ck = kbeg;
    const int64_t lo = kbeg + ((ck - kbeg) & ~(int64_t)(kWave - 1));
    if (lo + 64 < kend) kend = lo + 64;
    kbeg = lo;
    if (a.bsf_init && lane == 0) atomicMin(a.bsf, pack_best(best_dist(*a.bsf_init), 0xffffffffu));
  }
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t kb = kbeg + blk * kWave * (a.block_stride > 1 ? a.block_stride : 1);
  if (kb >= kend) return;
  const int64_t k = kb + lane;
  const bool active = k < kend;
  const int m = a.m;

  double mean, sd;
  wave_window_stats(a.x, a.n, m, kb, lane, mean, sd);
  float mu_hi, mu_lo, inv;
  znorm_params(mean, sd, mu_hi, mu_lo, inv);

  float ub = (DISTS ? a.fixed_ub : load_bsf_dist(a.bsf)) + 0.0f;
  if (!DISTS && a.bsf_init) ub = fminf(ub, best_dist(*a.bsf_init));
  bool alive = active && ub >= 0.0f;
  bool stopped = !wave_any(alive);

  __shared__ float sx[kWave + kStageRows - 1];
  __shared__ __attribute__((aligned(16))) float sq[kStageRows];
  const float *__restrict__ qz = a.qpad + kColPad;  // z(query)

  // bound reads, each applied kEdCheck blocks after it is issued
  constexpr int kEdCheck = 8;
  int since = 0;
  bool pending = false;
  unsigned long long bpend = 0;

  float acc = 0.0f;
  uint64_t evaluated = 0, computed = 0;
  for (int base = 0; base < m && !stopped; base += kStageRows) {
    const int rows = m - base < kStageRows ? m - base : kStageRows;
    __syncthreads();
    stage_copy<kWave + kStageRows - 1>(sx, a.x + kb + base, a.n - 1 - (kb + base), lane);
    stage_copy<kStageRows>(sq, qz + base, m - 1 - base, lane);
    __syncthreads();
    for (int i = 0; i < rows && !stopped; i += kEdBlock) {
      if (!DISTS && !pending) {
        bpend = __hip_atomic_load(a.bsf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        pending = true;
        since = 0;
      }
      const int nr = rows - i < kEdBlock ? rows - i : kEdBlock;
      if (nr == kEdBlock) {
#pragma unroll
        for (int t = 0; t < kEdBlock; t += 4) {
          const float4 q4 = *reinterpret_cast<const float4 *>(&sq[i + t]);
          const float qv[4] = {q4.x, q4.y, q4.z, q4.w};
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float diff = qv[j] - znorm_value(sx[lane + i + t + j], mu_hi, mu_lo, inv);
            acc = __builtin_fmaf(diff, diff, acc);
          }
        }
      } else {
        for (int t = 0; t < nr; ++t) {
          const float diff = sq[i + t] - znorm_value(sx[lane + i + t], mu_hi, mu_lo, inv);
          acc = __builtin_fmaf(diff, diff, acc);
        }
      }
      evaluated += (uint64_t)nr * (uint64_t)__popcll(__builtin_amdgcn_ballot_w64(alive));
      computed += (uint64_t)nr * kWave;
      if (!DISTS && ++since >= kEdCheck) {
        ub = fminf(ub, best_dist(bpend));
        pending = false;
      }
      alive = alive && acc <= ub;
      if (!wave_any(alive)) stopped = true;
    }
  }

  const bool keep = alive && !stopped && acc <= ub;
  if (DISTS) {
    if (active) a.dists[k - a.k_begin] = keep ? acc : kInf;
  } else {
    publish_best(a.bsf, keep, acc, a.bound_only ? 0xffffffffu : (uint32_t)k);
  }
  if (a.counters) {
    const uint64_t aband = (uint64_t)__popcll(__builtin_amdgcn_ballot_w64(active && !keep));
    if (lane == 0) {
      unsigned long long *c = counter_stripe(a.counters, blockIdx.x);
      atomicAdd(&c[kCntEvaluated], (unsigned long long)evaluated);
      atomicAdd(&c[kCntComputed], (unsigned long long)computed);
      atomicAdd(&c[kCntAbandoned], (unsigned long long)aband);
    }
  }
}

}  // namespace

hipError_t launch_ed_search(const NNArgs &a, int64_t nblocks, bool dists, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (dists)
    hipLaunchKernelGGL(ed_search_kernel<true>, dim3((unsigned)nblocks), dim3(kWave), 0, st, a);
  else
    hipLaunchKernelGGL(ed_search_kernel<false>, dim3((unsigned)nblocks), dim3(kWave), 0, st, a);
  return hipGetLastError();
}

}  // namespace eapdtw
