// band.h -- band-in-registers DTW kernels for gfx950 (windows r <= kBandRMax).
//
// One SIMD lane owns one problem (a search candidate or a pair).  The DP
// state of the lane is one matrix row of the Sakoe-Chiba band, held in
// 2r+1 VGPRs indexed by the diagonal d = j - i + r (Section 2 Eq. 1-5 with
// the window of Section 2.1).  In these coordinates cell (i,d) reads
//   diag (i-1,j-1) -> v[d]   (previous row, same register)
//   top  (i-1,j)   -> v[d+1] (previous row)
//   left (i,j-1)   -> v[d-1] (current row)
// so a row can be updated in place.  Rows are processed U at a time and the
// U rows of a group are swept column by column (a column s of the group holds
// cells (u, d = s-u)); that order respects the three dependencies and lets
// all U cells of a column share one column value, so the per-cell work is
// one subtraction, one 3-way min and one fused multiply-add.
//
// Early abandoning (Section 2.2): after each row group every lane checks the
// minimum of its last row; a row whose cells all exceed the bound means every
// later cell does too, so the lane is dead, and a wave whose lanes are all
// dead stops.  The value of a cell <= ub never depends on a cell > ub, so the
// surviving values are exactly those of the unpruned float32 recurrence.
#pragma once
#include "common.h"

namespace eapdtw {

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

// Wave-uniform read-only data (the normalised query) is read through the
// scalar cache: addresses in the constant address space select s_load.
typedef const __attribute__((address_space(4))) float ConstF;
__device__ __forceinline__ ConstF *as_const(const float *p) {
  return (ConstF *)(const __attribute__((address_space(4))) void *)p;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// exclusive prefix sum over the wave (lane l gets the sum of lanes < l)
__device__ __forceinline__ double wave_excl_scan_f64(double v, int lane) {
  double incl = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    double t = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += t;
  }
  return incl - v;
}

__device__ __forceinline__ float fmin3(float a, float b, float c) { return fminf(fminf(a, b), c); }

// Window statistics of the 64 consecutive offsets kb..kb+63 (lane l <-> kb+l),
// window length m.  Sums are taken in float64 relative to the pivot x[kb] so
// that long random walks do not lose the variance to cancellation:
//   sum over [l, l+m) = P(m) + (sum of y[m..m+l)) - (sum of y[0..l)),
// with P(m) = sum of y[0..m) reduced over the wave and the two partial sums
// from wave scans.  Loads past the end of the series are clamped; they only
// reach lanes whose offset is itself past the end.
__device__ __forceinline__ void wave_window_stats(const float *__restrict__ x, int64_t n, int m,
                                                  int64_t kb, int lane, double &mean,
                                                  double &sd) {
  const double pivot = (double)x[kb];
  double s1 = 0.0, s2 = 0.0;
  for (int t = lane; t < m; t += kWave) {
    int64_t idx = kb + t;
    idx = idx < n ? idx : n - 1;
    double y = (double)x[idx] - pivot;
    s1 += y;
    s2 += y * y;
  }
  s1 = wave_sum_f64(s1);
  s2 = wave_sum_f64(s2);
  int64_t ia = kb + lane, ib = kb + m + lane;
  ia = ia < n ? ia : n - 1;
  ib = ib < n ? ib : n - 1;
  const double ya = (double)x[ia] - pivot;
  const double yb = (double)x[ib] - pivot;
  const double e1 = wave_excl_scan_f64(ya, lane), e2 = wave_excl_scan_f64(ya * ya, lane);
  const double f1 = wave_excl_scan_f64(yb, lane), f2 = wave_excl_scan_f64(yb * yb, lane);
  const double sum1 = s1 + f1 - e1, sum2 = s2 + f2 - e2;
  const double my = sum1 / (double)m;
  const double ey2 = sum2 / (double)m;
  double var = ey2 - my * my;
  // a window whose deviation is only rounding noise is flat: normalise to 0
  if (!(var > 1e-14 * ey2)) var = 0.0;
  mean = pivot + my;
  sd = sqrt(var);
}

// Split of the window mean into float32 hi + lo parts and the inverse
// deviation: z = ((x - mu_hi) - mu_lo) * inv keeps the subtraction accurate
// to a few float32 ulps of the normalised value even for |x| >> sigma.
__device__ __forceinline__ void znorm_params(double mean, double sd, float &mu_hi, float &mu_lo,
                                             float &inv) {
  mu_hi = (float)mean;
  mu_lo = (float)(mean - (double)mu_hi);
  double iv = sd > 0.0 ? 1.0 / sd : 0.0;
  inv = (iv > 3.0e38) ? 0.0f : (float)iv;
}

__device__ __forceinline__ float znorm_value(float xv, float mu_hi, float mu_lo, float inv) {
  return ((xv - mu_hi) - mu_lo) * inv;
}

// Hides a pointer's provenance from the optimiser so that loads through it
// cannot be merged with, or hoisted above, loads of other column chunks.
__device__ __forceinline__ ConstF *opaque(ConstF *p) {
  asm volatile("" : "+s"(p));
  return p;
}
__device__ __forceinline__ const float *opaque(const float *p) {
  asm volatile("" : "+s"(p));
  return p;
}

// Column values of a group sweep: the value of group column s is
// base[s * stride + lane_off].  base is wave-uniform (kept in SGPRs);
// lane_off is 0 for a uniform column series (the query) and the lane's pair
// index for per-lane series, so the loads use a scalar base and a 32-bit
// lane offset.
template <class Ptr>
struct Cols {
  Ptr base;
  int64_t stride;
  int lane_off;
};

// One group of U rows, swept column by column (group column s is matrix
// column j = i0 + s - R).  Column values are fetched one chunk of kColChunk
// columns ahead of their use, which bounds the registers that hold them.
constexpr int kColChunk = 16;

template <int R, int U, class Ptr>
__device__ __forceinline__ void sweep_group(float (&v)[2 * R + 1], const float (&rv)[U],
                                            Cols<Ptr> cs) {
  constexpr int W = 2 * R + 1;
  constexpr int NS = W + U - 1;
  constexpr int CH = kColChunk;
  constexpr int NCH = (NS + CH - 1) / CH;
  const int64_t stride = cs.stride;
  float cur[CH];
  {
    Ptr p0 = opaque(cs.base);
#pragma unroll
    for (int t = 0; t < CH; ++t) cur[t] = (t < NS) ? p0[t * stride + cs.lane_off] : 0.0f;
  }
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    float nxt[CH];
    if (c + 1 < NCH) {
      Ptr pn = opaque(cs.base + (int64_t)(c + 1) * CH * stride);
#pragma unroll
      for (int t = 0; t < CH; ++t)
        nxt[t] = ((c + 1) * CH + t < NS) ? pn[t * stride + cs.lane_off] : 0.0f;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int s = c * CH + t;
      if (s >= NS) continue;
      const float cv = cur[t];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int d = s - u;
        if (d < 0 || d >= W) continue;
        const float left = (d > 0) ? v[d > 0 ? d - 1 : 0] : kInf;
        const float top = (d < W - 1) ? v[d < W - 1 ? d + 1 : 0] : kInf;
        const float diff = cv - rv[u];
        v[d] = __builtin_fmaf(diff, diff, fmin3(left, top, v[d]));
      }
    }
    // Pin this chunk's results before the next chunk's loads are issued:
    // volatile asm statements keep their order, so the loads of chunk c+2
    // (behind the next opaque()) cannot move above the cells of chunk c.
#pragma unroll
    for (int d = 0; d < W; ++d) {
      if (d + U - 1 < c * CH || d > c * CH + CH - 1) continue;  // untouched by this chunk
      asm volatile("" : "+v"(v[d]));
    }
    __builtin_amdgcn_sched_barrier(0);
    if (c + 1 < NCH) {
#pragma unroll
      for (int t = 0; t < CH; ++t) cur[t] = nxt[t];
    }
  }
}

template <int R>
__device__ __forceinline__ float band_min(const float (&v)[2 * R + 1]) {
  float m = v[0];
#pragma unroll
  for (int d = 1; d < 2 * R + 1; ++d) m = fminf(m, v[d]);
  return m;
}

// In-matrix cells of rows [i0, i0+u) (scalar bookkeeping for the counters).
template <int U>
__device__ __forceinline__ int rows_cells(int i0, int lcol, int r) {
  int c = 0;
#pragma unroll
  for (int u = 0; u < U; ++u) c += row_cells(i0 + u, lcol, r);
  return c;
}

__device__ __forceinline__ float load_bsf_dist(const unsigned long long *bsf) {
  unsigned long long b = __hip_atomic_load(bsf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return best_dist(b);
}

// ---------------------------------------------------------------------------
// Subsequence search: lane l of workgroup b owns candidate offset
// k = k_begin + 64 b + l.  Rows run over the candidate (one z-normalised
// value per row and lane), columns over the z-normalised query (one uniform
// value per column, read through the scalar cache).
// DISTS = true writes every candidate's early-abandoned distance against the
// fixed bound instead of updating the shared best-so-far.
template <int R, int U, bool DISTS>
__device__ __forceinline__ void nn_band_body(const NNArgs &a, int64_t blk) {
  constexpr int W = 2 * R + 1;
  const int lane = threadIdx.x;
  int64_t kbeg = a.k_begin, kend = a.k_end;
  if (a.center) {
    // seed launch: 64 offsets centred on the best offset of an earlier pass
    const unsigned long long c = *a.center;
    int64_t ck = (int64_t)best_offset(c);
    if (ck > kend - 1) ck = kend - 1;
    int64_t lo = ck - 32;
    if (lo < kbeg) lo = kbeg;
    if (lo + 64 < kend) kend = lo + 64;
    kbeg = lo;
    if (a.bsf_init && lane == 0) atomicMin(a.bsf, pack_best(best_dist(*a.bsf_init), 0xffffffffu));
  }
  const int64_t kb = kbeg + blk * kWave * (a.block_stride > 1 ? a.block_stride : 1);
  if (kb >= kend) return;
  const int64_t k = kb + lane;
  const bool active = k < kend;
  const int64_t kc = active ? k : kend - 1;
  const int m = a.m;

  double mean, sd;
  wave_window_stats(a.x, a.n, m, kb, lane, mean, sd);
  float mu_hi, mu_lo, inv;
  znorm_params(mean, sd, mu_hi, mu_lo, inv);
  const float *__restrict__ xk = a.x + kc;

  float v[W];
#pragma unroll
  for (int d = 0; d < W; ++d) v[d] = kInf;
  v[R] = 0.0f;  // M(0,0) lies on diagonal R of the row above the first row

  float ub = DISTS ? a.fixed_ub : load_bsf_dist(a.bsf);
  if (!DISTS && a.center && a.bsf_init) ub = fminf(ub, best_dist(*a.bsf_init));
  bool alive = active && ub >= 0.0f;
  int since = 0;
  uint64_t evaluated = 0, computed = 0;
  const int mg = m - m % U;  // rows covered by full groups
  int i0 = 0;
  bool stopped = !wave_any(alive);

  float rv_next[U];
#pragma unroll
  for (int u = 0; u < U; ++u) rv_next[u] = (u < mg) ? xk[u] : 0.0f;

  for (; i0 < mg && !stopped; i0 += U) {
    float rv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) rv[u] = znorm_value(rv_next[u], mu_hi, mu_lo, inv);
    if (i0 + U < mg) {
#pragma unroll
      for (int u = 0; u < U; ++u) rv_next[u] = xk[i0 + U + u];
    }
    sweep_group<R, U>(v, rv, Cols<ConstF *>{as_const(a.qpad + kColPad + i0 - R), 1, 0});
    const int cells = rows_cells<U>(i0, m, R);
    evaluated += (uint64_t)cells * (uint64_t)__popcll(__ballot(alive));
    computed += (uint64_t)cells * kWave;
    if (!DISTS && ++since >= a.check_interval) {
      since = 0;
      ub = load_bsf_dist(a.bsf);
    }
    alive = alive && band_min<R>(v) <= ub;
    if (!wave_any(alive)) stopped = true;
  }
  // remaining rows, one at a time
  for (int i = mg; i < m && !stopped; ++i) {
    float rv1[1] = {znorm_value(xk[i], mu_hi, mu_lo, inv)};
    sweep_group<R, 1>(v, rv1, Cols<ConstF *>{as_const(a.qpad + kColPad + i - R), 1, 0});
    const int cells = row_cells(i, m, R);
    evaluated += (uint64_t)cells * (uint64_t)__popcll(__ballot(alive));
    computed += (uint64_t)cells * kWave;
    alive = alive && band_min<R>(v) <= ub;
    if (!wave_any(alive)) stopped = true;
  }

  const float d = v[R];
  const bool keep = alive && !stopped && d <= ub;
  if (DISTS) {
    if (active) a.dists[k - a.k_begin] = keep ? d : kInf;
  } else if (keep) {
    atomicMin(a.bsf, pack_best(d, a.bound_only ? 0xffffffffu : (uint32_t)k));
  }
  if (a.counters) {
    const uint64_t aband = (uint64_t)__popcll(__ballot(active && !keep));
    if (lane == 0) {
      unsigned long long *c = counter_stripe(a.counters, blockIdx.x);
      atomicAdd(&c[kCntEvaluated], (unsigned long long)evaluated);
      atomicAdd(&c[kCntComputed], (unsigned long long)computed);
      atomicAdd(&c[kCntAbandoned], (unsigned long long)aband);
    }
  }
}

template <int R, int U, bool DISTS>
__global__ __launch_bounds__(64) void nn_band_kernel(NNArgs a) {
  nn_band_body<R, U, DISTS>(a, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Independent pairs: lane l of workgroup b owns pair p = 64 b + l.  Row and
// column values come from the transposed copies (coalesced per wave).
template <int R, int U>
__global__ __launch_bounds__(64) void pair_band_kernel(PairArgs a) {
  constexpr int W = 2 * R + 1;
  const int lane = threadIdx.x;
  const int64_t p = (int64_t)blockIdx.x * kWave + lane;
  const bool active = p < a.npairs;
  const int64_t pc = active ? p : a.npairs - 1;
  const int64_t ld = a.ld;
  const int lrow = a.lrow, lcol = a.lcol;
  const float *__restrict__ rows = a.rowsT + pc;
  const float *__restrict__ cols = a.colsT + (int64_t)kColPad * ld + pc;
  const float *colu = a.colsT + (int64_t)kColPad * ld;  // wave-uniform column base

  float ub;
  float ed = kInf;
  if (a.ub_mode == 1) {
    ub = a.ub[pc];
  } else if (a.ub_mode == 2) {
    // squared Euclidean distance along the diagonal, with the same operations
    // as the diagonal cells of the recurrence (so DTW <= ED holds bitwise)
    float acc = 0.0f;
    for (int i = 0; i < lrow; ++i) {
      const float diff = cols[(int64_t)i * ld] - rows[(int64_t)i * ld];
      acc = __builtin_fmaf(diff, diff, acc);
    }
    ed = acc;
    ub = acc;
  } else if (a.ub_mode == 3) {
    ub = a.ub_scalar;
  } else {
    ub = kInf;
  }
  const bool bounded = wave_any(active && ub < kInf);

  float v[W];
#pragma unroll
  for (int d = 0; d < W; ++d) v[d] = kInf;
  v[R] = 0.0f;
  bool alive = active && ub >= 0.0f;
  bool stopped = !wave_any(alive);
  uint64_t evaluated = 0, computed = 0;
  const int mg = lrow - lrow % U;
  int ck = 0;
  for (int i0 = 0; i0 < mg && !stopped; i0 += U) {
    float rv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) rv[u] = rows[(int64_t)(i0 + u) * ld];
    sweep_group<R, U>(v, rv, Cols<const float *>{colu + (int64_t)(i0 - R) * ld, ld, (int)pc});
    const int cells = rows_cells<U>(i0, lcol, R);
    evaluated += (uint64_t)cells * (uint64_t)__popcll(__ballot(alive));
    computed += (uint64_t)cells * kWave;
    if (a.ckpt && ((i0 + U) % a.ckpt_every) == 0 && i0 + U < lrow) {
      float *cp = a.ckpt + (int64_t)ck * W * ld + p;
      if (active) {
#pragma unroll
        for (int d = 0; d < W; ++d) cp[(int64_t)d * ld] = v[d];
      }
      ++ck;
    }
    if (bounded) {
      alive = alive && band_min<R>(v) <= ub;
      if (!wave_any(alive)) stopped = true;
    }
  }
  for (int i = mg; i < lrow && !stopped; ++i) {
    float rv1[1] = {rows[(int64_t)i * ld]};
    sweep_group<R, 1>(v, rv1, Cols<const float *>{colu + (int64_t)(i - R) * ld, ld, (int)pc});
    const int cells = row_cells(i, lcol, R);
    evaluated += (uint64_t)cells * (uint64_t)__popcll(__ballot(alive));
    computed += (uint64_t)cells * kWave;
    if (bounded) {
      alive = alive && band_min<R>(v) <= ub;
      if (!wave_any(alive)) stopped = true;
    }
  }
  // result cell (lrow-1, lcol-1) sits on diagonal R + lcol - lrow
  const int dans = R + lcol - lrow;
  float d = kInf;
#pragma unroll
  for (int q = 0; q < W; ++q)
    if (q == dans) d = v[q];
  const bool keep = alive && !stopped && d <= ub;
  if (active) {
    float o = keep ? d : kInf;
    if (a.ub_mode == 2 && !keep) o = ed;  // the diagonal path is always admissible
    a.out[p] = o;
  }
  if (a.counters) {
    const uint64_t aband = (uint64_t)__popcll(__ballot(active && !keep));
    if (lane == 0) {
      unsigned long long *c = counter_stripe(a.counters, blockIdx.x);
      atomicAdd(&c[kCntEvaluated], (unsigned long long)evaluated);
      atomicAdd(&c[kCntComputed], (unsigned long long)computed);
      atomicAdd(&c[kCntAbandoned], (unsigned long long)aband);
    }
  }
}

// Host-side launchers (explicitly instantiated per window in band_r*.hip).
template <int R>
hipError_t launch_nn_band(const NNArgs &a, int64_t nblocks, int rows_per_group, bool dists,
                          hipStream_t st);
template <int R>
hipError_t launch_pair_band(const PairArgs &a, int64_t nblocks, int rows_per_group,
                            hipStream_t st);

}  // namespace eapdtw
