// erp.hip -- ERP, the edit distance with real penalty (Chen & Ng, VLDB 2004),
// over a batch of pairs: an elastic distance with DTW's three moves where the
// vertical and horizontal moves align a point with the gap value g (the kind
// of distance the paper's closing outlook carries the method over to).
//
// One SIMD lane owns one pair; the Sakoe-Chiba band of the current row lives
// in 2r+1 VGPRs indexed by the diagonal d = j - i + r, as in the DTW band
// kernels: cell (i,d) reads diag v[d], top v[d+1] (previous row) and left
// v[d-1] (current row).  Rows are swept U at a time, column by column, so a
// column value T_j and its gap cost |T_j - g| serve the U cells of the column.
// Both series are read transposed ([len][ld], pair p at column p), so a wave's
// loads are coalesced.
//
// Matrix (1-based cells, borders in the window only):
//   M(0,0) = 0, M(0,j) = M(0,j-1) + |T_j - g|, M(i,0) = M(i-1,0) + |S_i - g|,
//   M(i,j) = min(M(i-1,j-1) + |S_i - T_j|, M(i-1,j) + |S_i - g|,
//                M(i,j-1) + |T_j - g|),
// every cell with |i - j| > r at +inf.  Every cost is non-negative, so a row
// whose cells all exceed the bound ub means the result does too (each
// alignment path crosses every row): the pair is abandoned (Section 2.2's
// early abandoning carried over), and cells are never changed, so a kept
// result has the plain float32 recurrence's bits.
#include <array>
#include <utility>

#include "band.h"
#include "dispatch.h"

namespace eapdtw {

namespace {

constexpr int kErpU = 4;
constexpr int kErpChunk = 16;

__device__ __forceinline__ int erp_clamp(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

__device__ __forceinline__ bool erp_wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0ull; }

// One group: rows i0+1 .. i0+U, group column s holds matrix column
// j = i0 + 1 + s - R, cells (u, d = s - u).  EDGE: the group has cells on
// column 0, left of it, right of column L, or rows past L (its column loads
// are clamped into the series; the values they bring there are not used).
// Column values are fetched one chunk of kErpChunk ahead of their use, which
// bounds the registers that hold them.
template <int R, bool EDGE, class ColFn>
__device__ __forceinline__ void erp_group(float (&v)[2 * R + 1], const float (&av)[kErpU],
                                          const float (&ga)[kErpU], const float (&cs)[kErpU],
                                          ColFn col, int i0, int L, float g) {
  constexpr int W = 2 * R + 1;
  constexpr int NS = W + kErpU - 1;
  constexpr int CH = kErpChunk;
  constexpr int NCH = (NS + CH - 1) / CH;
  const int jb = i0 - R;  // series index (j - 1) of group column 0
  auto load = [&](int s) -> float {
    int idx = jb + s;
    if (EDGE) idx = erp_clamp(idx, 0, L - 1);
    return col(idx);
  };
  float cur[CH], nxt[CH];
#pragma unroll
  for (int t = 0; t < CH; ++t) cur[t] = (t < NS) ? load(t) : 0.0f;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    if (c + 1 < NCH) {
#pragma unroll
      for (int t = 0; t < CH; ++t) nxt[t] = ((c + 1) * CH + t < NS) ? load((c + 1) * CH + t) : 0.0f;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int s = c * CH + t;
      if (s >= NS) continue;
      const int j = i0 + 1 + s - R;
      const float b = cur[t];
      const float gb = __builtin_fabsf(b - g);
#pragma unroll
      for (int u = 0; u < kErpU; ++u) {
        const int d = s - u;
        if (d < 0 || d >= W) continue;
        const float diag = v[d];
        const float top = (d + 1 < W) ? v[d + 1 < W ? d + 1 : 0] : kInf;
        const float left = (d > 0) ? v[d > 0 ? d - 1 : 0] : kInf;
        float nv = fminf(fminf(diag + __builtin_fabsf(av[u] - b), top + ga[u]), left + gb);
        if constexpr (EDGE) {
          if (i0 + 1 + u > L) continue;  // rows past the end (last group): unchanged
          if (j < 0 || j > L) nv = kInf;
          else if (j == 0) nv = cs[u];
        }
        v[d] = nv;
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    if (c + 1 < NCH) {
#pragma unroll
      for (int t = 0; t < CH; ++t) cur[t] = nxt[t];
    }
  }
}

// The whole sweep of one problem per lane: row values row(i) (0-based), column
// values col(j) (0-based, L of each), gap value g; the bound is ub_at(group)
// (re-read by the caller's rule).  Returns M(L, L), and alive = false once a
// swept row had no cell at or below the bound.
template <int R, class RowFn, class ColFn, class UbFn>
__device__ __forceinline__ float erp_sweep(RowFn row, ColFn col, UbFn ub_at, int L, float g,
                                           bool &alive, uint64_t &evaluated, uint64_t &computed) {
  constexpr int W = 2 * R + 1;
  float v[W];
  // row 0: M(0,j) for j = d - R in 0..R (R <= L - 1), +inf left of column 0
  float acc = 0.0f;
#pragma unroll
  for (int d = 0; d < W; ++d) {
    const int j = d - R;
    if (j > 0) acc += __builtin_fabsf(col(j - 1) - g);
    v[d] = j < 0 ? kInf : acc;
  }
  float cum = 0.0f;  // M(i,0) of the rows swept so far (read while i <= R)
  int grp = 0;
  for (int i0 = 0; i0 < L; i0 += kErpU, ++grp) {
    float av[kErpU], ga[kErpU], cs[kErpU];
    int cells = 0;
#pragma unroll
    for (int u = 0; u < kErpU; ++u) {
      const int i = i0 + 1 + u;
      av[u] = row(erp_clamp(i - 1, 0, L - 1));
      ga[u] = __builtin_fabsf(av[u] - g);
      cum += ga[u];
      cs[u] = cum;
      if (i <= L) cells += (i + R < L ? i + R : L) - (i - R > 1 ? i - R : 1) + 1;
    }
    if (i0 + 1 <= R || i0 + kErpU + R > L)
      erp_group<R, true>(v, av, ga, cs, col, i0, L, g);
    else
      erp_group<R, false>(v, av, ga, cs, col, i0, L, g);
    computed += (uint64_t)cells;
    if (alive) evaluated += (uint64_t)cells;
    // the last swept row (cells outside the matrix hold +inf)
    float mn = v[0];
#pragma unroll
    for (int d = 1; d < W; ++d) mn = fminf(mn, v[d]);
    alive = alive && mn <= ub_at(grp);
    if (!erp_wave_any(alive)) break;
  }
  return v[R];
}

__device__ __forceinline__ void erp_count(unsigned long long *counters, uint64_t evaluated,
                                          uint64_t computed, bool active, bool keep) {
  for (int o = 32; o >= 1; o >>= 1) {
    evaluated += (uint64_t)__shfl_xor((long long)evaluated, o, kWave);
    computed += (uint64_t)__shfl_xor((long long)computed, o, kWave);
  }
  const uint64_t aband = (uint64_t)__popcll(__builtin_amdgcn_ballot_w64(active && !keep));
  if (threadIdx.x == 0) {
    unsigned long long *c = counter_stripe(counters, blockIdx.x);
    atomicAdd(&c[kCntEvaluated], (unsigned long long)evaluated);
    atomicAdd(&c[kCntComputed], (unsigned long long)computed);
    atomicAdd(&c[kCntAbandoned], (unsigned long long)aband);
  }
}

// Windows 40..57 are held to two waves per SIMD (up to 16 bytes of scratch
// per lane at 56..57); from 58 the spills would cost more than the second wave
// brings, and the kernel runs one wave per SIMD.
template <int R>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu((R >= 40 && R <= 57) ? 2 : 1)))
void erp_pairs_kernel(ErpArgs a) {
  const int lane = threadIdx.x;
  const int64_t p = (int64_t)blockIdx.x * kWave + lane;
  const bool active = p < a.npairs;
  // [len][ld] transposed series: row pointers are wave-uniform, the lane
  // reads column lp (ld >= the pair count rounded up to 64)
  const int lp = (int)p;
  const float *Xt = a.Xt, *Yt = a.Yt;
  const int64_t ld = a.ld;
  const float ub = (a.ub && active) ? a.ub[p] : kInf;
  bool alive = active;
  uint64_t evaluated = 0, computed = 0;
  const float dist = erp_sweep<R>([&](int i) { return (Xt + (int64_t)i * ld)[lp]; },
                                  [&](int j) { return (Yt + (int64_t)j * ld)[lp]; },
                                  [&](int) { return ub; }, a.len, a.g, alive, evaluated, computed);
  const bool keep = alive && dist <= ub;
  if (active) a.out[p] = keep ? dist : kInf;
  if (a.counters) erp_count(a.counters, evaluated, computed, active, keep);
}

// Nearest-neighbour search under ERP: lane l of workgroup b takes candidate
// offset k = 64 b + l, its window z-normalised on the fly with the statistics
// the DTW search kernels use (rows), against the z-normalised query (columns,
// one wave-uniform value each); the bound is the shared best-so-far, re-read
// every check_interval row groups; the wave publishes its best with one atomic.
template <int R>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu((R >= 40 && R <= 57) ? 2 : 1)))
void erp_search_kernel(ErpSearchArgs a) {
  const int lane = threadIdx.x;
  const int64_t kb = (int64_t)blockIdx.x * kWave;
  const int64_t k = kb + lane;
  const bool active = k < a.K;
  const int m = a.m;
  double mean, sd;
  wave_window_stats(a.x, a.n, m, kb, lane, mean, sd);
  float mu_hi, mu_lo, inv;
  znorm_params(mean, sd, mu_hi, mu_lo, inv);
  const float *xk = a.x + (active ? k : a.K - 1);
  const float *qz = a.qz;
  float ub = load_bsf_dist(a.bsf);
  const int ci = a.check_interval > 0 ? a.check_interval : 1;
  bool alive = active;
  uint64_t evaluated = 0, computed = 0;
  const float dist = erp_sweep<R>(
      [&](int i) { return znorm_value(xk[i], mu_hi, mu_lo, inv); }, [&](int j) { return qz[j]; },
      [&](int grp) {
        if ((grp + 1) % ci == 0) ub = fminf(ub, load_bsf_dist(a.bsf));
        return ub;
      },
      m, a.g, alive, evaluated, computed);
  const bool keep = alive && dist <= ub;
  publish_best(a.bsf, keep, dist, (uint32_t)k);
  if (a.counters) erp_count(a.counters, evaluated, computed, active, keep);
}

typedef hipError_t (*ErpFn)(const ErpArgs &, int64_t, hipStream_t);

template <int R>
hipError_t erp_launch_r(const ErpArgs &a, int64_t nblk, hipStream_t st) {
  hipLaunchKernelGGL(erp_pairs_kernel<R>, dim3((unsigned)nblk), dim3(kWave), 0, st, a);
  return hipGetLastError();
}

template <int... Rs>
constexpr std::array<ErpFn, sizeof...(Rs)> erp_table(std::integer_sequence<int, Rs...>) {
  return {&erp_launch_r<Rs>...};
}

constexpr auto kErpLaunch = erp_table(std::make_integer_sequence<int, kErpMaxR + 1>{});

typedef hipError_t (*ErpSearchFn)(const ErpSearchArgs &, int64_t, hipStream_t);

template <int R>
hipError_t erp_search_launch_r(const ErpSearchArgs &a, int64_t nblk, hipStream_t st) {
  hipLaunchKernelGGL(erp_search_kernel<R>, dim3((unsigned)nblk), dim3(kWave), 0, st, a);
  return hipGetLastError();
}

template <int... Rs>
constexpr std::array<ErpSearchFn, sizeof...(Rs)> erp_search_table(std::integer_sequence<int, Rs...>) {
  return {&erp_search_launch_r<Rs>...};
}

constexpr auto kErpSearchLaunch =
    erp_search_table(std::make_integer_sequence<int, kErpMaxR + 1>{});

}  // namespace

hipError_t launch_erp_pairs(int r, const ErpArgs &a, hipStream_t st) {
  if (r < 0 || r > kErpMaxR || a.len < 1 || r > a.len - 1) return hipErrorInvalidValue;
  if (a.npairs <= 0) return hipSuccess;
  const int64_t nblk = (a.npairs + kWave - 1) / kWave;
  if (nblk * kWave > 0x7fffffff || a.ld < nblk * kWave) return hipErrorInvalidValue;
  return kErpLaunch[r](a, nblk, st);
}

hipError_t launch_erp_search(int r, const ErpSearchArgs &a, hipStream_t st) {
  if (r < 0 || r > kErpMaxR || a.m < 1 || r > a.m - 1 || a.K < 1) return hipErrorInvalidValue;
  const int64_t nblk = (a.K + kWave - 1) / kWave;
  if (nblk > 0x7fffffff || a.K > 0xffffffffll) return hipErrorInvalidValue;
  return kErpSearchLaunch[r](a, nblk, st);
}

}  // namespace eapdtw
