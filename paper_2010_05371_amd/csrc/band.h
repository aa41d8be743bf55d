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
#include <type_traits>

#include "common.h"

namespace eapdtw {

// A window whose variance is at most kFlatRel of its mean square is flat.
constexpr double kFlatRel = 1e-14;

__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0ull; }

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

// Minimum of cell values through their bit patterns: cells are never negative
// (or NaN), and for such floats the unsigned order of the bits is the numeric
// order, so the integer minimum needs no NaN quieting of its operands.
__device__ __forceinline__ uint32_t cell_bits(float x) { return __float_as_uint(x); }
__device__ __forceinline__ uint32_t umin3(uint32_t a, uint32_t b, uint32_t c) {
  const uint32_t t = a < b ? a : b;
  return t < c ? t : c;
}

// Window statistics of the 64 consecutive offsets kb..kb+63 (lane l <-> kb+l),
// window length m.  Sums are taken in float64 relative to the pivot x[kb] so
// that long random walks do not lose the variance to cancellation:
//   sum over [l, l+m) = P(m) + (sum of y[m..m+l)) - (sum of y[0..l)),
// with P(m) = sum of y[0..m) reduced over the wave and the two partial sums
// from wave scans.  Loads past the end of the series are clamped; they only
// reach lanes whose offset is itself past the end.
// X: anything indexable by a series position (a global pointer, or a view of
// a stretch staged in LDS); every caller gets the same float64 arithmetic.
template <class X>
__device__ __forceinline__ void wave_window_stats(X x, int64_t n, int m, int64_t kb, int lane,
                                                  double &mean, double &sd) {
  const double pivot = (double)x[kb];
  int64_t ia = kb + lane, ib = kb + m + lane;
  ia = ia < n ? ia : n - 1;
  ib = ib < n ? ib : n - 1;
  const float xa = x[ia], xb = x[ib];
  // four loads in flight per step (the sums keep the lane's order t, t + 64, ...)
  double s1 = 0.0, s2 = 0.0;
  for (int t0 = 0; t0 < m; t0 += 4 * kWave) {
    float xv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int64_t idx = kb + t0 + j * kWave + lane;
      idx = idx < n ? idx : n - 1;
      xv[j] = x[idx];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (t0 + j * kWave + lane < m) {
        const double y = (double)xv[j] - pivot;
        s1 += y;
        s2 += y * y;
      }
    }
  }
  s1 = wave_sum_f64(s1);
  s2 = wave_sum_f64(s2);
  const double ya = (double)xa - pivot;
  const double yb = (double)xb - pivot;
  const double e1 = wave_excl_scan_f64(ya, lane), e2 = wave_excl_scan_f64(ya * ya, lane);
  const double f1 = wave_excl_scan_f64(yb, lane), f2 = wave_excl_scan_f64(yb * yb, lane);
  const double sum1 = s1 + f1 - e1, sum2 = s2 + f2 - e2;
  const double my = sum1 / (double)m;
  const double ey2 = sum2 / (double)m;
  double var = ey2 - my * my;
  double mu = pivot + my;
  // E[x^2] = E[(x-p)^2] + p (2 E[x-p] + p)
  double ex2 = ey2 + pivot * (2.0 * my + pivot);
  // The moments about the shared pivot p lose about log10(E[(x-p)^2] / var)
  // digits of the variance; a window far from p with a small spread (a
  // plateau after a step) takes a second pass over its own values about its
  // first mean instead.
  if (var < 1e-6 * ey2) {
    double c1 = 0.0, c2 = 0.0;
    for (int t = 0; t < m; ++t) {
      int64_t idx = kb + lane + t;
      idx = idx < n ? idx : n - 1;
      const double y = (double)x[idx] - mu;
      c1 += y;
      c2 += y * y;
    }
    const double d1 = c1 / (double)m;
    var = c2 / (double)m - d1 * d1;
    mu += d1;
    ex2 = var + mu * mu;
  }
  // Flat window (normalised to 0): variance at most kFlatRel of the window's
  // mean square, i.e. variation at the float32 rounding level of its values.
  if (!(var > kFlatRel * ex2)) var = 0.0;
  mean = mu;
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

// Waits for the scalar loads of a column chunk before the next chunk's loads
// are issued.  Scalar loads may return out of order, so a wait for an older
// one is a wait for all; settling the chunk in use first leaves the next
// chunk's loads in flight while it is computed.  Per-lane (vector) loads
// complete in order and need no settling.
template <class Ptr, int N>
__device__ __forceinline__ void settle(const float (&c)[N]) {
  if constexpr (std::is_same<Ptr, ConstF *>::value) {
#pragma unroll
    for (int t = 0; t < N; ++t) asm volatile("" ::"s"(c[t]));
  }
}

// One group of U rows, swept column by column (group column s is matrix
// column j = i0 + s - R).  Column values are fetched one chunk of kColChunk
// columns ahead of their use, which bounds the registers that hold them.
constexpr int kColChunk = 16;

// first[] holds the group's first chunk of column values on entry.  With
// next_base set, the last chunk's step loads the next group's first chunk
// (whose base is next_base) into first[], so no group starts by waiting for
// its column values.
// WT: weighted DTW, cell cost wt[|d - R|] (column - row value)^2 (wt holds
// the weights of the band's phase differences 0..R).
template <int R, int U, bool WT = false, class Ptr>
__device__ __forceinline__ void sweep_group(float (&v)[2 * R + 1], const float (&rv)[U],
                                            Cols<Ptr> cs, float (&first)[kColChunk],
                                            Ptr next_base, const float *wt = nullptr) {
  constexpr int W = 2 * R + 1;
  constexpr int NS = W + U - 1;
  constexpr int CH = kColChunk;
  constexpr int NCH = (NS + CH - 1) / CH;
  const int64_t stride = cs.stride;
  float cur[CH];
#pragma unroll
  for (int t = 0; t < CH; ++t) cur[t] = first[t];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    float nxt[CH];
    settle<Ptr>(cur);
    if (c + 1 < NCH) {
      Ptr pn = opaque(cs.base + (int64_t)(c + 1) * CH * stride);
#pragma unroll
      for (int t = 0; t < CH; ++t)
        nxt[t] = ((c + 1) * CH + t < NS) ? pn[t * stride + cs.lane_off] : 0.0f;
    } else {
      Ptr pn = opaque(next_base);
#pragma unroll
      for (int t = 0; t < CH; ++t) first[t] = pn[t * stride + cs.lane_off];
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
        const float dw = WT ? diff * wt[d < R ? R - d : d - R] : diff;
        v[d] = __builtin_fmaf(dw, diff, fmin3(left, top, v[d]));
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

// Loads the first chunk of a group's column values (see sweep_group).
template <int U, class Ptr>
__device__ __forceinline__ void load_first(float (&first)[kColChunk], Cols<Ptr> cs) {
  Ptr p0 = opaque(cs.base);
#pragma unroll
  for (int t = 0; t < kColChunk; ++t) first[t] = p0[t * cs.stride + cs.lane_off];
}

// Without look-ahead: the group's first chunk is loaded on entry.
template <int R, int U, class Ptr>
__device__ __forceinline__ void sweep_group(float (&v)[2 * R + 1], const float (&rv)[U],
                                            Cols<Ptr> cs) {
  float first[kColChunk];
  load_first<U>(first, cs);
  sweep_group<R, U>(v, rv, cs, first, cs.base);
}

template <int R>
__device__ __forceinline__ float band_min(const float (&v)[2 * R + 1]) {
  float m = v[0];
#pragma unroll
  for (int d = 1; d < 2 * R + 1; ++d) m = fminf(m, v[d]);
  return m;
}

// ---------------------------------------------------------------------------
// Pruning borders kept per wave (Section 3: a cell above the bound can only
// feed cells above the bound, so a row only needs the cells between the
// first one reachable from the previous row's live cells and the last one
// whose left neighbour is live).  The band of the last swept row is cut into
// diagonal chunks of kBorderChunk cells; Border holds the first and last
// chunk that hold a cell at most the bound in some live lane.  Every register
// outside the swept range holds a value above the bound, and the recurrence
// keeps cells at most the bound exact whatever those values are, so the
// bordered sweep gives bit-identical results for every cell at most the bound.
constexpr int kBorderChunk = 8;
constexpr int kStageRows = 512;  // rows of the series staged in LDS per copy

// Copies src[min(t, lim)] to dst[t] for t < N: every lane's loads are issued
// before the first store, so the copy costs one memory round trip.
template <int N>
__device__ __forceinline__ void stage_copy(float *dst, const float *__restrict__ src, int64_t lim,
                                           int lane) {
  constexpr int NJ = (N + kWave - 1) / kWave;
  float tmp[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int t = lane + kWave * j;
    tmp[j] = src[t < lim ? t : lim];
  }
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int t = lane + kWave * j;
    if (t < N) dst[t] = tmp[j];
  }
}

struct Border {
  int lo, hi;  // diagonal chunks [kBorderChunk * lo, kBorderChunk * (hi + 1))
};

// One group of U rows swept over the group columns that can hold live cells.
// Group column s (row u computes diagonal s - u) starts at kBorderChunk * lo - 1,
// the column of the first diagonal a live cell of the previous row can reach;
// the columns up to the one where row U - 1 passes the previous row's last
// live chunk are always swept; after that the sweep stops at the first check
// point (every half chunk) where the last cell of every row is above the
// bound in every live lane.  Returns the last swept column.
// Calls f(std::integral_constant<int, i>) for i = 0 .. N-1, every index a
// compile-time constant (register arrays stay statically indexed).
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F &f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Bitwise OR over the wave (row shifts, then row broadcasts into lane 63).
__device__ __forceinline__ uint32_t wave_or(uint32_t x) {
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// One group of U rows swept over the group columns that can hold live cells.
// Columns are taken in units of kBorderChunk: unit k covers group columns
// [CH k - 1, CH k + CH - 1) (row u computes diagonal s - u at column s).  The
// first unit is b.lo: its first column reaches the diagonal just left of the
// previous row's first live chunk.  Units up to the one where row U - 1
// passes the previous row's last live chunk are always swept; after the last
// unit the sweep extends by one unit while the last cell of some row is at
// most the bound in some lane.  Returns the last swept column.
//
// qn / qn_unit: column values of unit qn_unit of this group, loaded during the
// previous group; on return, those of unit b.lo of the next group (whose
// columns start next_base), loaded while this group is swept.
template <int R, int U, bool WT = false, class Ptr>
__device__ __forceinline__ int sweep_group_border(float (&v)[2 * R + 1], const float (&rv)[U],
                                                  Cols<Ptr> cs, const Border &b, uint32_t ubits,
                                                  uint64_t amask, float (&qn)[kColChunk],
                                                  int &qn_unit, Ptr next_base,
                                                  const float *wt = nullptr) {
  static_assert(kBorderChunk <= kColChunk, "look-ahead buffer too small");
  constexpr int W = 2 * R + 1;
  constexpr int NS = W + U - 1;
  constexpr int CH = kBorderChunk;
  constexpr int NU = (NS + CH) / CH;
  const int u0 = b.lo;
  int uend = (CH * (b.hi + 1) + U - 1) / CH;  // unit holding column CH (hi + 1) + U - 2
  uend = uend < NU - 1 ? uend : NU - 1;
  // column values of even units in qa, odd units in qb
  float qa[CH], qb[CH];
  {
    const bool have = qn_unit == u0;
    Ptr p0 = opaque(cs.base + (int64_t)(CH * u0 - 1) * cs.stride);
    if (u0 & 1) {
#pragma unroll
      for (int t = 0; t < CH; ++t) qb[t] = have ? qn[t] : p0[t * cs.stride + cs.lane_off];
    } else {
#pragma unroll
      for (int t = 0; t < CH; ++t) qa[t] = have ? qn[t] : p0[t * cs.stride + cs.lane_off];
    }
  }
  static_for<NU>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if ((unsigned)(k - u0) > (unsigned)(uend - u0)) return;  // k outside [u0, uend]
    float(&cur)[CH] = (k & 1) ? qb : qa;
    float(&nxt)[CH] = (k & 1) ? qa : qb;
    settle<Ptr>(cur);
    if (k == u0) {
      // the next group most often starts at the same unit
      Ptr pq = opaque(next_base + (int64_t)(CH * k - 1) * cs.stride);
#pragma unroll
      for (int t = 0; t < CH; ++t) qn[t] = pq[t * cs.stride + cs.lane_off];
      qn_unit = k;
    }
    if constexpr (k + 1 < NU) {
      Ptr pn = opaque(cs.base + (int64_t)(CH * (k + 1) - 1) * cs.stride);
#pragma unroll
      for (int t = 0; t < CH; ++t) nxt[t] = pn[t * cs.stride + cs.lane_off];
      // keeps the loads here: they are not sunk into the next unit's block
      // (where their latency would be exposed)
      asm volatile("" ::: "memory");
    }
    __builtin_amdgcn_sched_barrier(0);
    constexpr int sb = CH * k - 1;
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int s = sb + t;
      if (s < 0 || s >= NS) continue;
      const float cvl = cur[t];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int d = s - u;
        if (d < 0 || d >= W) continue;
        const float left = (d > 0) ? v[d > 0 ? d - 1 : 0] : kInf;
        const float top = (d < W - 1) ? v[d < W - 1 ? d + 1 : 0] : kInf;
        const float diff = cvl - rv[u];
        const float dw = WT ? diff * wt[d < R ? R - d : d - R] : diff;
        v[d] = __builtin_fmaf(dw, diff, fmin3(left, top, v[d]));
      }
    }
    // volatile asm keeps its order, so the next unit's loads cannot be
    // hoisted above these cells
#pragma unroll
    for (int j = 0; j < CH + U - 1; ++j) {
      const int d = sb - (U - 1) + j;
      if (d >= 0 && d < W) asm volatile("" : "+v"(v[d >= 0 && d < W ? d : 0]));
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (k + 1 < NU) {
      if (k == uend) {
        // the last cells of the rows, at column sb + CH - 1
        uint32_t mn = cell_bits(kInf);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int d = sb + CH - 1 - u;
          if (d >= 0 && d < W) mn = min(mn, cell_bits(v[d >= 0 && d < W ? d : 0]));
        }
        if (__builtin_amdgcn_ballot_w64(mn <= ubits) & amask) uend = k + 1;
      }
    }
  });
  const int slast = CH * uend + CH - 2;
  return slast < NS - 1 ? slast : NS - 1;
}

// Minimum of diagonal chunk C of the band (bit patterns).
template <int R, int C>
__device__ __forceinline__ uint32_t chunk_min_bits(const float (&v)[2 * R + 1]) {
  constexpr int W = 2 * R + 1;
  constexpr int CH = kBorderChunk;
  uint32_t mn = cell_bits(v[CH * C < W ? CH * C : 0]);
#pragma unroll
  for (int t = 1; t < CH; t += 2) {
    const int d0 = CH * C + t, d1 = d0 + 1;
    if (d1 < W && t + 1 < CH)
      mn = umin3(mn, cell_bits(v[d0 < W ? d0 : 0]), cell_bits(v[d1 < W ? d1 : 0]));
    else if (d0 < W)
      mn = min(mn, cell_bits(v[d0 < W ? d0 : 0]));
  }
  return mn;
}

// Borders of the last swept row.  Registers outside the swept range hold
// values above the bound (or +inf, see clear_outside), so every chunk can be
// tested without a range check.  Returns whether this lane still has a live cell; hi < 0 when no
// lane has one.
template <int R>
__device__ __forceinline__ bool border_update(const float (&v)[2 * R + 1], Border &b,
                                              uint32_t ubits, bool alive) {
  constexpr int NCD = (2 * R + 1 + kBorderChunk - 1) / kBorderChunk;
  static_assert(NCD <= 32, "chunk mask is 32 bits");
  uint32_t mask = 0;
  static_for<NCD>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    mask |= (chunk_min_bits<R, c>(v) <= ubits) ? (1u << c) : 0u;
  });
  mask = alive ? mask : 0u;
  const uint32_t all = wave_or(mask);
  b.lo = all ? __builtin_ctz(all) : -1;
  b.hi = all ? 31 - __builtin_clz(all) : -1;
  return mask != 0u;
}

// Sets every register of the chunks outside [b.lo, b.hi] to +inf.  The
// bordered sweep leaves those registers holding values of older rows, which
// is harmless while the bound can only fall (they were above it when their
// chunk was dropped); a bound that can rise from row to row (the list mode's
// tightening) must not see them again.  Cells outside the borders lie on no
// path that ends at or below the bound, so +inf stands in for them.
template <int R>
__device__ __forceinline__ void clear_outside(float (&v)[2 * R + 1], const Border &b) {
  constexpr int W = 2 * R + 1;
  constexpr int NCD = (W + kBorderChunk - 1) / kBorderChunk;
  static_for<NCD>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    if (c < b.lo || c > b.hi) {
#pragma unroll
      for (int t = 0; t < kBorderChunk; ++t) {
        const int d = c * kBorderChunk + t;
        if (d < W) v[d < W ? d : 0] = kInf;
      }
    }
  });
}

// Cells of rows [i0, i0 + U) swept over group columns [s0, s1]: in the band,
// and in the matrix (lcol columns) for the evaluated count.
template <int U>
__device__ __forceinline__ void swept_cells(int i0, int s0, int s1, int lcol, int r, int &band,
                                            int &matrix) {
  const int w = 2 * r + 1;
  if (s0 >= U - 1 && s1 <= w - 1 && i0 >= r && i0 + U <= lcol - r) {
    band = matrix = U * (s1 - s0 + 1);  // every row inside band and matrix
    return;
  }
  band = matrix = 0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int i = i0 + u;
    int lo = s0 - u, hi = s1 - u;
    lo = lo > 0 ? lo : 0;
    hi = hi < w - 1 ? hi : w - 1;
    band += hi >= lo ? hi - lo + 1 : 0;
    const int mlo = lo > r - i ? lo : r - i;
    const int mhi = hi < r + lcol - 1 - i ? hi : r + lcol - 1 - i;
    matrix += mhi >= mlo ? mhi - mlo + 1 : 0;
  }
}

// In-matrix cells of rows [i0, i0+u) (scalar bookkeeping for the counters).
template <int U>
__device__ __forceinline__ int rows_cells(int i0, int lcol, int r) {
  int c = 0;
#pragma unroll
  for (int u = 0; u < U; ++u) c += row_cells(i0 + u, lcol, r);
  return c;
}

// Row groups between reads of the shared best-so-far when none is chosen:
// enough groups to cover an L2 round trip (about 2,400 cycles) with one
// wave's own cell work (about 12 cycles per cell row of a group).
template <int R, int U>
__host__ __device__ constexpr int auto_check_interval() {
  return (200 + U * (2 * R + U) - 1) / (U * (2 * R + U));
}

// Publishes the wave's best kept candidate: one atomic per wave instead of
// one per lane (same-address atomics serialise in the L2).
__device__ __forceinline__ void publish_best(unsigned long long *bsf, bool keep, float d,
                                             uint32_t id) {
  unsigned long long v = keep ? pack_best(d, id) : ~0ull;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const unsigned long long t = __shfl_xor(v, o, kWave);
    v = t < v ? t : v;
  }
  if (threadIdx.x % kWave == 0 && v != ~0ull) atomicMin(bsf, v);
}

// Ascending bitonic sort of one u64 per lane across the wave (lane l ends
// with the l-th smallest).
__device__ __forceinline__ unsigned long long wave_sort_u64(unsigned long long v) {
  const int lane = threadIdx.x % kWave;
#pragma unroll
  for (int size = 2; size <= kWave; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride >= 1; stride >>= 1) {
      const unsigned long long o = __shfl_xor(v, stride, kWave);
      const bool up = (lane & size) == 0;           // this block sorts ascending
      const bool low = (lane & stride) == 0;        // this lane holds the lower slot
      const unsigned long long lo = o < v ? o : v, hi = o < v ? v : o;
      v = (up == low) ? lo : hi;
    }
  }
  return v;
}

// k-nearest-neighbour publication of a wave.  Its kept candidates go to the
// buffer.  Two upper bounds of the search's k-th best distance are min-ed
// into the bound word:
//  * when the wave kept at least k candidates, its k-th smallest distance
//    (the k-th best of k actual candidates);
//  * k slots (with counters): candidate `id` lowers slot id mod k to its
//    distance, so the k slots hold distances of k distinct candidates once
//    all are filled, and their largest bounds the k-th best.  Neighbouring
//    offsets of a good match fill different slots, so this bound follows the
//    search's progress rather than waiting for one wave with k survivors.
//    Slots store 2^32 - 1 - (distance bits), 0 meaning empty, and take
//    atomicMax.
__device__ __forceinline__ void publish_knn(const KnnOut &a, bool keep, float d, uint32_t id) {
  const int lane = threadIdx.x % kWave;
  const unsigned long long mask = __builtin_amdgcn_ballot_w64(keep);
  if (!mask) return;
  const unsigned long long v = keep ? pack_best(d, id) : ~0ull;
  if (a.buf) {
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(a.n, (unsigned long long)__popcll(mask));
    base = __shfl(base, 0, kWave);
    if (keep) {
      const unsigned r = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
      a.buf[base + r] = v;
    }
  }
  if (__popcll(mask) >= a.k) {
    const unsigned long long s = wave_sort_u64(v);
    const unsigned long long kth = __shfl(s, a.k - 1, kWave);
    if (lane == 0) atomicMin(a.bound, pack_best(best_dist(kth), 0xffffffffu));
  }
  unsigned long long *slots = a.slots ? a.slots : (a.counters ? a.counters + kCntKnnSlot : nullptr);
  if (slots) {
    if (keep)
      atomicMax(&slots[(id % (uint32_t)a.k) * kCntStride],
                (unsigned long long)(0xffffffffu - __builtin_bit_cast(uint32_t, d)));
    unsigned long long sv = 1;  // lanes past k: no constraint
    if (lane < a.k)
      sv = __hip_atomic_load(&slots[lane * kCntStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!wave_any(sv == 0)) {
      uint32_t bits = lane < a.k ? 0xffffffffu - (uint32_t)sv : 0u;
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const uint32_t t = __shfl_xor(bits, o, kWave);
        bits = t > bits ? t : bits;
      }
      if (lane == 0) atomicMin(a.bound, pack_best(__builtin_bit_cast(float, bits), 0xffffffffu));
    }
  }
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
template <int R, int U, bool DISTS, bool BORDER = false, bool LIST = false, bool WT = false>
__device__ __forceinline__ void nn_band_body(const NNArgs &a, int64_t blk) {
  constexpr int W = 2 * R + 1;
  const int lane = threadIdx.x;
  const int m = a.m;
  int64_t kb = 0, k;
  bool active;
  float mu_hi, mu_lo, inv;
  // list mode: the candidate's series, its LB_Keogh (query envelope) total
  // lowered by the margin, and its largest lower bound
  const float *xk = nullptr;
  float lb_total = 0.0f, lb_max = 0.0f;
  if constexpr (LIST) {
    const int64_t nl = (int64_t)*a.list_n;
    const int64_t e0 = blk * kWave;
    if (e0 >= nl) return;
    active = e0 + lane < nl;
    const int64_t e = active ? e0 + lane : nl - 1;
    k = (int64_t)a.list_k[e];
    mu_hi = a.list_mh[e];
    mu_lo = a.list_ml[e];
    inv = a.list_inv[e];
    lb_total = a.list_lbq[e] * (1.0f - kLbMargin);
    lb_max = a.list_lbmax[e];
    xk = a.x + k;
  } else {
    int64_t kbeg = a.k_begin, kend = a.k_end;
    if (a.center) {
      // seed launch: the 64 offsets of the block holding the best offset of an
      // earlier pass
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
    kb = kbeg + blk * kWave * (a.block_stride > 1 ? a.block_stride : 1);
    if (kb >= kend) return;
    k = kb + lane;
    active = k < kend;
    double mean, sd;
    wave_window_stats(a.x, a.n, m, kb, lane, mean, sd);
    znorm_params(mean, sd, mu_hi, mu_lo, inv);
  }

  // The wave's 64 candidates read rows of one stretch of the series: it is
  // staged in LDS kStageRows rows at a time (one coalesced copy), so a row's
  // values come from LDS instead of a dependent global load.  (List mode:
  // the lanes' candidates lie anywhere, each lane reads its own rows.)
  __shared__ float stage[kWave + kStageRows - 1];
  int sbase = 0;  // first row held in stage
  auto refill = [&](int i0) {
    __syncthreads();
    const float *__restrict__ xs = a.x + kb + i0;
    const int64_t lim = a.n - 1 - (kb + i0);
#pragma unroll 1
    for (int t = lane; t < kWave + kStageRows - 1; t += kWave) stage[t] = xs[t < lim ? t : lim];
    __syncthreads();
  };
  if constexpr (!LIST) {
    stage_copy<kWave + kStageRows - 1>(stage, a.x + kb, a.n - 1 - kb, lane);
    __syncthreads();
  }
  auto row_value = [&](int i) -> float {
    if constexpr (LIST) return xk[i];
    else return stage[lane + i - sbase];
  };

  float v[W];
#pragma unroll
  for (int d = 0; d < W; ++d) v[d] = kInf;
  v[R] = 0.0f;  // M(0,0) lies on diagonal R of the row above the first row
  Border bd{R / kBorderChunk, R / kBorderChunk};

  // (+ 0 turns a bound of -0 into +0, which the bit-pattern comparisons of
  // the bordered sweep need)
  float ub = (DISTS ? a.fixed_ub : load_bsf_dist(a.bsf)) + 0.0f;
  if (!DISTS && a.bsf_init) ub = fminf(ub, best_dist(*a.bsf_init));
  bool alive = active && ub >= 0.0f;
  uint64_t rechecked = 0;  // list mode: entries whose bound now exceeds the best-so-far
  if constexpr (LIST) {
    alive = alive && !(lb_max * (1.0f - kLbMargin) > ub);
    rechecked = (uint64_t)__popcll(__builtin_amdgcn_ballot_w64(active && !alive));
  }
  // List mode tightens the bound row by row (the UCR Suite's use of LB_Keogh):
  // every path still has to pay, in each row t below the current one, at
  // least the squared distance from z(c_t) to the query envelope [L_t, U_t]
  // (the columns of row t lie within r of t), so a cell above
  // ub - (sum of those terms) cannot reach a result <= ub.  The remaining sum
  // is the lowered total minus the running prefix; the envelope is read one
  // group ahead with vector loads (all lanes, one address).
  float lb_prefix = 0.0f;
  const float *uqv = a.uq, *lqv = a.lq;
  if constexpr (LIST) {
    int vz;
    asm volatile("v_mov_b32 %0, 0" : "=v"(vz));
    uqv += vz;
    lqv += vz;
  }
  auto lb_term = [&](float z, float lo, float hi) {
    const float dd = z - __builtin_amdgcn_fmed3f(z, lo, hi);
    lb_prefix = __builtin_fmaf(dd, dd, lb_prefix);
  };
  // the bound for cells of rows up to the last one folded into lb_prefix
  auto row_bound = [&]() -> float {
    if constexpr (LIST) {
      const float rest = lb_total - lb_prefix;
      return ub - (rest > 0.0f ? rest : 0.0f);
    } else {
      return ub;
    }
  };
  // The shared best-so-far is read once every ci groups; each read is
  // issued ci groups before its value is applied, so its latency (an L2 round
  // trip) hides behind that many groups even when a group is short.
  const int ci = a.check_interval > 0 ? a.check_interval : auto_check_interval<R, U>();
  int since = 0;
  bool pending = false;
  unsigned long long bpend = 0;
  uint64_t evaluated = 0, computed = 0;
  const int mg = m - m % U;  // rows covered by full groups
  bool stopped = !wave_any(alive);
  // column values the next group starts with, loaded one group ahead
  float qfirst[kColChunk];
  int qfirst_unit = -1;  // bordered sweep: the unit they belong to (-1: none)
  if constexpr (!BORDER) load_first<U>(qfirst, Cols<ConstF *>{as_const(a.qpad + kColPad - R), 1, 0});

  float rv_next[U], uq_next[U], lq_next[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    rv_next[u] = (u < mg) ? row_value(u) : 0.0f;
    uq_next[u] = 0.0f;
    lq_next[u] = 0.0f;
    if constexpr (LIST) {
      if (u < mg) {
        uq_next[u] = uqv[u];
        lq_next[u] = lqv[u];
      }
    }
  }

  // One group of G rows starting at row i.
  auto group = [&](auto gtag, int i, const float *rvg, const float *uqg, const float *lqg) {
    constexpr int G = decltype(gtag)::value;
    float thr = ub;
    if constexpr (LIST) {
#pragma unroll
      for (int u = 0; u < G; ++u) lb_term(rvg[u], lqg[u], uqg[u]);
      thr = row_bound();
      alive = alive && thr >= 0.0f;
      thr = thr > 0.0f ? thr : 0.0f;
    }
    if (!DISTS && !pending) {
      bpend = __hip_atomic_load(a.bsf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      pending = true;
      since = 0;
    }
    const Cols<ConstF *> cols{as_const(a.qpad + kColPad + i - R), 1, 0};
    int band, mat;
    float rvl[G];
#pragma unroll
    for (int u = 0; u < G; ++u) rvl[u] = rvg[u];
    int slast = W + G - 2;
    if constexpr (BORDER) {
      slast = sweep_group_border<R, G, WT>(v, rvl, cols, bd, cell_bits(thr),
                                           __builtin_amdgcn_ballot_w64(alive), qfirst,
                                           qfirst_unit, as_const(a.qpad + kColPad + i + G - R),
                                           a.wgt);
      swept_cells<G>(i, kBorderChunk * bd.lo - 1, slast, m, R, band, mat);
    } else {
      sweep_group<R, G, WT>(v, rvl, cols, qfirst, as_const(a.qpad + kColPad + i + G - R), a.wgt);
      band = G * W;
      mat = rows_cells<G>(i, m, R);
    }
    evaluated += (uint64_t)mat * (uint64_t)__popcll(__builtin_amdgcn_ballot_w64(alive));
    computed += (uint64_t)band * kWave;
    if (!DISTS && ++since >= ci) {
      ub = fminf(ub, best_dist(bpend));
      pending = false;
      if constexpr (LIST) {
        thr = row_bound();
        alive = alive && thr >= 0.0f;
        thr = thr > 0.0f ? thr : 0.0f;
      } else {
        thr = ub;
      }
    }
    if constexpr (BORDER) {
      alive = border_update<R>(v, bd, cell_bits(thr), alive);
      if (bd.hi < 0) stopped = true;
      if constexpr (LIST) {
        if (!stopped) clear_outside<R>(v, bd);
      }
    } else {
      alive = alive && band_min<R>(v) <= thr;
      if (!wave_any(alive)) stopped = true;
    }
  };

  for (int i0 = 0; i0 < mg && !stopped; i0 += U) {
    float rv[U], uqg[U], lqg[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      rv[u] = znorm_value(rv_next[u], mu_hi, mu_lo, inv);
      uqg[u] = uq_next[u];
      lqg[u] = lq_next[u];
    }
    if (i0 + U < mg) {
      if constexpr (!LIST) {
        if (i0 + U - sbase >= kStageRows) {
          sbase = i0 + U;
          refill(sbase);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        rv_next[u] = row_value(i0 + U + u);
        if constexpr (LIST) {
          uq_next[u] = uqv[i0 + U + u];
          lq_next[u] = lqv[i0 + U + u];
        }
      }
    }
    group(std::integral_constant<int, U>{}, i0, rv, uqg, lqg);
  }
  // remaining rows, one at a time
  for (int i = mg; i < m && !stopped; ++i) {
    if constexpr (!LIST) {
      if (i - sbase >= kStageRows) {
        sbase = i;
        refill(sbase);
      }
    }
    const float rv1[1] = {znorm_value(row_value(i), mu_hi, mu_lo, inv)};
    float uq1[1] = {0.0f}, lq1[1] = {0.0f};
    if constexpr (LIST) {
      uq1[0] = uqv[i];
      lq1[0] = lqv[i];
    }
    group(std::integral_constant<int, 1>{}, i, rv1, uq1, lq1);
  }

  const float d = v[R];
  const bool keep = alive && !stopped && d <= ub;
  if (DISTS) {
    if (active) a.dists[k - a.k_begin] = keep ? d : kInf;
  } else if (a.knn > 0) {
    publish_knn(KnnOut{a.bsf, a.knn, a.knn_buf, a.knn_n, a.counters, a.knn_slots}, keep, d,
                (uint32_t)k);
  } else {
    publish_best(a.bsf, keep, d, a.bound_only ? 0xffffffffu : (uint32_t)k);
  }
  if (a.counters) {
    const uint64_t aband = (uint64_t)__popcll(__ballot(active && !keep));
    if (lane == 0) {
      unsigned long long *c = counter_stripe(a.counters, blockIdx.x);
      atomicAdd(&c[kCntEvaluated], (unsigned long long)evaluated);
      atomicAdd(&c[kCntComputed], (unsigned long long)computed);
      atomicAdd(&c[kCntAbandoned], (unsigned long long)aband);
      if (LIST) atomicAdd(&c[kCntLbRecheck], (unsigned long long)rechecked);
    }
  }
}

// At most 128 VGPRs where the band allows it, so that four waves share a SIMD
// (the bordered sweep's bookkeeping otherwise pushes a few windows just past).
template <int R, int U, bool DISTS, bool BORDER>
__global__ __launch_bounds__(64, (BORDER && R <= 52) ? 4 : 1) void nn_band_kernel(NNArgs a) {
  nn_band_body<R, U, DISTS, BORDER>(a, xcd_block(blockIdx.x, gridDim.x));
}

// Weighted DTW (cost w(|i-j|) (a-b)^2, weights in NNArgs::wgt): the same
// search with one more multiply per cell.
template <int R, int U, bool DISTS, bool BORDER>
__global__ __launch_bounds__(64, (BORDER && R <= 52) ? 4 : 1) void nn_wband_kernel(NNArgs a) {
  nn_band_body<R, U, DISTS, BORDER, false, true>(a, xcd_block(blockIdx.x, gridDim.x));
}

// The candidates that passed the lower bounds (list mode of the same sweep);
// its per-lane bound tightening fits four waves per SIMD up to window 40.
template <int R, int U, bool DISTS, bool BORDER>
__global__ __launch_bounds__(64, (BORDER && R <= 40) ? 4 : 1) void nn_list_kernel(NNArgs a) {
  nn_band_body<R, U, DISTS, BORDER, true>(a, xcd_block(blockIdx.x, gridDim.x));
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
  for (int i0 = 0; i0 < mg && !stopped; i0 += U) {
    float rv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) rv[u] = rows[(int64_t)(i0 + u) * ld];
    sweep_group<R, U>(v, rv, Cols<const float *>{colu + (int64_t)(i0 - R) * ld, ld, (int)pc});
    const int cells = rows_cells<U>(i0, lcol, R);
    evaluated += (uint64_t)cells * (uint64_t)__popcll(__ballot(alive));
    computed += (uint64_t)cells * kWave;
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
                          bool border, hipStream_t st);
template <int R>
hipError_t launch_nn_list(const NNArgs &a, int64_t nblocks, bool dists, bool border,
                          hipStream_t st);
template <int R>
hipError_t launch_nn_wband(const NNArgs &a, int64_t nblocks, bool dists, bool border,
                           hipStream_t st);
template <int R>
hipError_t launch_pair_band(const PairArgs &a, int64_t nblocks, int rows_per_group,
                            hipStream_t st);

}  // namespace eapdtw
