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

#include "dispatch.h"

namespace eapdtw {

namespace {

constexpr int kErpU = 4;
constexpr int kErpChunk = 16;

__device__ __forceinline__ int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

__device__ __forceinline__ bool erp_wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0ull; }

// One group: rows i0+1 .. i0+U, group column s holds matrix column
// j = i0 + 1 + s - R, cells (u, d = s - u).  EDGE: the group has cells on
// column 0, left of it, right of column L, or rows past L (its column loads
// are clamped into the series; the values they bring there are not used).
// Column values are fetched one chunk of kErpChunk ahead of their use, which
// bounds the registers that hold them.
template <int R, bool EDGE>
__device__ __forceinline__ void erp_group(float (&v)[2 * R + 1], const float (&av)[kErpU],
                                          const float (&ga)[kErpU], const float (&cs)[kErpU],
                                          const float *Yt, int64_t ld, int lp, int i0, int L,
                                          float g) {
  constexpr int W = 2 * R + 1;
  constexpr int NS = W + kErpU - 1;
  constexpr int CH = kErpChunk;
  constexpr int NCH = (NS + CH - 1) / CH;
  const int jb = i0 - R;  // series index (j - 1) of group column 0
  auto load = [&](int s) -> float {
    int idx = jb + s;
    if (EDGE) idx = clampi(idx, 0, L - 1);
    return (Yt + (int64_t)idx * ld)[lp];  // wave-uniform row, the lane's column
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

// Windows 40..57 are held to two waves per SIMD (up to 16 bytes of scratch
// per lane at 56..57); from 58 the spills would cost more than the second wave
// brings, and the kernel runs one wave per SIMD.
template <int R>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu((R >= 40 && R <= 57) ? 2 : 1)))
void erp_pairs_kernel(ErpArgs a) {
  constexpr int W = 2 * R + 1;
  const int lane = threadIdx.x;
  const int64_t p = (int64_t)blockIdx.x * kWave + lane;
  const bool active = p < a.npairs;
  const int L = a.len;
  const float g = a.g;
  // [len][ld] transposed series: row pointers are wave-uniform, the lane
  // reads column lp (ld >= the pair count rounded up to 64)
  const int lp = (int)p;
  const float *Xt = a.Xt, *Yt = a.Yt;
  const float ub = (a.ub && active) ? a.ub[p] : kInf;
  float v[W];
  // row 0: M(0,j) for j = d - R in 0..R (R <= L - 1), +inf left of column 0
  float acc = 0.0f;
#pragma unroll
  for (int d = 0; d < W; ++d) {
    const int j = d - R;
    if (j > 0) acc += __builtin_fabsf((Yt + (int64_t)(j - 1) * a.ld)[lp] - g);
    v[d] = j < 0 ? kInf : acc;
  }
  float cum = 0.0f;  // M(i,0) of the rows swept so far (read while i <= R)
  bool alive = active;
  uint64_t evaluated = 0, computed = 0;
  for (int i0 = 0; i0 < L; i0 += kErpU) {
    float av[kErpU], ga[kErpU], cs[kErpU];
    int cells = 0;
#pragma unroll
    for (int u = 0; u < kErpU; ++u) {
      const int i = i0 + 1 + u;
      av[u] = (Xt + (int64_t)clampi(i - 1, 0, L - 1) * a.ld)[lp];
      ga[u] = __builtin_fabsf(av[u] - g);
      cum += ga[u];
      cs[u] = cum;
      if (i <= L) cells += (i + R < L ? i + R : L) - (i - R > 1 ? i - R : 1) + 1;
    }
    if (i0 + 1 <= R || i0 + kErpU + R > L)
      erp_group<R, true>(v, av, ga, cs, Yt, a.ld, lp, i0, L, g);
    else
      erp_group<R, false>(v, av, ga, cs, Yt, a.ld, lp, i0, L, g);
    computed += (uint64_t)cells;
    if (alive) evaluated += (uint64_t)cells;
    // the last swept row (cells outside the matrix hold +inf)
    float mn = v[0];
#pragma unroll
    for (int d = 1; d < W; ++d) mn = fminf(mn, v[d]);
    alive = alive && mn <= ub;
    if (!erp_wave_any(alive)) break;
  }
  const float dist = v[R];
  const bool keep = alive && dist <= ub;
  if (active) a.out[p] = keep ? dist : kInf;
  if (a.counters) {
    for (int o = 32; o >= 1; o >>= 1) {
      evaluated += (uint64_t)__shfl_xor((long long)evaluated, o, kWave);
      computed += (uint64_t)__shfl_xor((long long)computed, o, kWave);
    }
    const uint64_t aband = (uint64_t)__popcll(__builtin_amdgcn_ballot_w64(active && !keep));
    if (lane == 0) {
      unsigned long long *c = counter_stripe(a.counters, blockIdx.x);
      atomicAdd(&c[kCntEvaluated], (unsigned long long)evaluated);
      atomicAdd(&c[kCntComputed], (unsigned long long)computed);
      atomicAdd(&c[kCntAbandoned], (unsigned long long)aband);
    }
  }
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

}  // namespace

hipError_t launch_erp_pairs(int r, const ErpArgs &a, hipStream_t st) {
  if (r < 0 || r > kErpMaxR || a.len < 1 || r > a.len - 1) return hipErrorInvalidValue;
  if (a.npairs <= 0) return hipSuccess;
  const int64_t nblk = (a.npairs + kWave - 1) / kWave;
  if (nblk * kWave > 0x7fffffff || a.ld < nblk * kWave) return hipErrorInvalidValue;
  return kErpLaunch[r](a, nblk, st);
}

}  // namespace eapdtw
