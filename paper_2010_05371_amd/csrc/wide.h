// wide.h -- tiled DTW kernels for windows wider than the register band
// (kBandRMax < r, including unconstrained DTW), gfx950.
//
// One SIMD lane owns one problem.  The matrix is cut into tiles of H rows;
// a tile is swept column by column (column j holds cells (i0+h, j), h < H, in
// H VGPRs), so every cell reads
//   left (i, j-1)   -> the same register before the column update,
//   top  (i-1, j)   -> the register of row h-1 just updated,
//   diag (i-1, j-1) -> the register of row h-1 before the update,
// and row 0 of a tile reads the last row of the tile above from a per-wave
// boundary row kept in global memory ([column][lane], coalesced).
// The Sakoe-Chiba band (Section 2.1) makes each tile a parallelogram: an
// entering triangle of H columns where rows join the band one per column, a
// middle stretch where all H rows are admissible and an exiting triangle where
// rows leave it.  The triangles are unrolled statically so that out-of-band
// cells are never computed and read as +inf.
//
// Pruning (Section 4 recast per tile and wave): the sweep of a tile starts at
// the first column where the row above had a live cell (<= ub) in any lane --
// columns to its left are dead in every later row (left border) -- and, past
// the last column where the row above was live, stops after the first column
// whose H cells are all dead in every lane (right border: from there on a
// cell can only depend on its dead left neighbour).  A lane whose tile ended
// without a live cell in its last row is dead; a wave whose lanes are all dead
// stops (early abandoning, Section 2.2).
#pragma once
#include "band.h"

namespace eapdtw {

// Kinds of problem a wide wave can own.
enum WideKind : int {
  kWideSearch = 0,   // rows: z-normalised candidate (per lane); columns: query (uniform)
  kWidePairwise = 1, // rows: X[i] (uniform); columns: X[j] (per lane), i < j
  kWidePairs = 2,    // rows and columns per lane from transposed copies
  kWideSearchW = 3,  // as kWideSearch, cell (i, j) costing w(|i - j|) (a - b)^2 (weighted DTW)
};

// Padding of the weighted search's weight table on each side: the rows a
// whole-matrix tile computes past the matrix's last row (values +inf) reach up
// to H - 1 diagonals beyond -r, and read a finite weight there.
constexpr int kWtPad = 64;

__host__ __device__ constexpr bool wide_is_search(int kind) {
  return kind == kWideSearch || kind == kWideSearchW;
}

struct WideArgs {
  int lrow, lcol, r;
  // search
  const float *x;
  int64_t n;
  const float *qpad;                 // z(query), kColPad +inf on each side
  unsigned long long *bsf;
  int64_t k_begin, k_end;
  float fixed_ub;                    // per-candidate-distance mode
  float *dists;
  int dists_mode;
  int bound_only;
  const float *wt_band;              // weighted search: w(|d|) at index d + r + kWtPad, d = -r..r,
                                     // kWtPad entries of 1 on each side
  // pairwise / pairs
  const float *X;                    // pairwise: rows X [N][len]
  const float *XT;                   // pairwise: X transposed [len][ldN]; pairs: columns [lcol][ld]
  const float *RT;                   // pairs: rows transposed [lrow][ld]
  int64_t N, ld;
  int64_t nblk_j;                    // pairwise: column blocks per row series
  int ub_mode;                       // pairs: 0 none, 1 array, 2 ED; pairwise: ED
  unsigned long long *nn1;           // pairwise: per-series nearest neighbour words (NN1 mode)
  int knn;                           // search: k nearest neighbours (bsf bounds the k-th best)
  unsigned long long *knn_buf, *knn_n;
  unsigned long long *knn_slots;     // the k slot words (nullptr: those of the counter array)
  // search over a survivor list (lower-bound cascade, wide_list_kernel):
  // entry e holds the offset list_k[e], its normalisation constants and its
  // largest lower bound; list_n counts the entries
  const unsigned long long *list_n;
  const uint32_t *list_k;
  const float *list_mh, *list_ml, *list_inv, *list_lbmax;
  const float *list_lbq;             // LB_Keogh with the query's envelope (full sum)
  const float *uq, *lq;              // envelope of z(query) [lrow]
  int64_t nq;                        // pairwise: > 0 = rows are the nq series of X, columns the
                                     // N series of XT, every (row, column) pair (NN1 of a test
                                     // set against a reference set); 0 = i < j within one set
  const float *ub;
  float ub_scalar;
  float *out;
  // common
  int64_t ntasks;
  float *bnd;                        // boundary rows: [gridDim.x][lcol + 1][64]
  int64_t bnd_stride;                // floats per wave
  unsigned long long *counters;
  int check_interval;
};

// Column value access per kind, for the lane's problem.
struct WideProblem {
  // rows
  const float *xk;      // search: candidate start (per lane)
  float mu_hi, mu_lo, inv;
  const float *rowp;    // pairwise: row series (uniform); pairs: rows transposed + p
  // columns
  const float *colp;    // pairwise/pairs: column series transposed + lane offset
  int64_t cstride;
  float ub;
  bool active;
  float ed;
  // pairwise NN1: the two series' nearest-neighbour words (row uniform)
  const unsigned long long *nn_i, *nn_j;
  // weighted search: the weights staged in LDS, w(|d|) at index d + r
  const float *wsh;
  // cascade list mode: the candidate's query-envelope LB_Keogh (lowered) and
  // the sum of its terms over the rows swept so far
  float lb_total, lb_prefix;
};

template <int KIND>
__device__ __forceinline__ float wide_row_value(const WideArgs &a, const WideProblem &p, int i) {
  if (i >= a.lrow) return kInf;  // rows past the end: every cell +inf
  if (wide_is_search(KIND)) return znorm_value(p.xk[i], p.mu_hi, p.mu_lo, p.inv);
  if (KIND == kWidePairwise) return p.rowp[i];  // uniform address; kept in VGPRs
  return p.rowp[(int64_t)i * a.ld];
}

template <int KIND>
__device__ __forceinline__ float wide_col_value(const WideArgs &a, const WideProblem &p, int j) {
  // the query value is wave-uniform; it is loaded into a VGPR (one cache line
  // per wave) so that the prefetch queue does not compete for SGPRs
  if (wide_is_search(KIND)) return (a.qpad + kColPad)[j];
  return p.colp[(int64_t)j * p.cstride];
}

// Computes column j of the tile for rows [h_lo, h_hi] (static); rows above
// h_lo read +inf as their top neighbour (out of band), rows below h_hi are not
// computed and are forced to +inf when FORCE_BELOW.
// wl (weighted search only): the weight of row h of the column is wl[H-1-h].
template <int H, int H_LO, int H_HI, bool FORCE_BELOW, bool WT = false>
__device__ __forceinline__ void wide_column(float (&col)[H], const float (&rv)[H], float cv,
                                            float top0, float diag0, const float *wl = nullptr) {
  float up = (H_LO == 0) ? top0 : kInf;
  float dg = (H_LO == 0) ? diag0 : col[H_LO > 0 ? H_LO - 1 : 0];
  if (H_LO > 0) dg = col[H_LO - 1];
#pragma unroll
  for (int h = H_LO; h <= H_HI; ++h) {
    const float left = col[h];
    const float diff = cv - rv[h];
    const float dw = WT ? diff * wl[H - 1 - h] : diff;
    const float nv = __builtin_fmaf(dw, diff, fmin3(left, up, dg));
    dg = left;
    up = nv;
    col[h] = nv;
  }
  if (FORCE_BELOW && H_HI + 1 < H) col[H_HI + 1 < H ? H_HI + 1 : 0] = kInf;
}

template <int H>
__device__ __forceinline__ float col_min(const float (&col)[H]) {
  float m = col[0];
#pragma unroll
  for (int h = 1; h < H; ++h) m = fminf(m, col[h]);
  return m;
}

}  // namespace eapdtw

namespace eapdtw {

// Per-column bookkeeping state of one tile sweep.  The boundary value from
// the tile above and the column value of the next PD columns are loaded ahead
// of their use (a small queue in registers) so that the memory latency of a
// column overlaps the cells of the columns before it.
template <int PD>
struct Sweep {
  int j;              // next column
  int jend;           // last column the tile may reach
  int jmand;          // columns up to here may still be reached from the tile above
  int first_live, last_live;
  unsigned long long lane_live;
  bool go;
  float diag0;        // (i0-1, j-1)
  int bv_lo, bv_hi;   // boundary columns valid from the tile above
  int t;              // tile index
  int64_t rows;       // admissible rows of the tile (<= H, last tile may be shorter)
  uint64_t evaluated, computed;
  unsigned long long alive_mask;
  float qtop[PD], qcv[PD];  // prefetched values of columns j .. j+PD-1
};

template <int KIND, int PD>
__device__ __forceinline__ void wide_fetch(const WideArgs &a, const WideProblem &p, const float *Bw,
                                           int lane, const Sweep<PD> &s, int c, float &top,
                                           float &cv) {
  const bool in = c <= s.jend;
  const bool have_top = in && s.t > 0 && c >= s.bv_lo && c <= s.bv_hi;
  top = have_top ? Bw[(int64_t)(c + 1) * kWave + lane] : kInf;
  cv = in ? wide_col_value<KIND>(a, p, c) : 0.0f;
}

// Unconditional form for the rotating queue: both loads are issued for every
// column (from a clamped, valid column) with no branch around them, and the
// boundary value's validity travels beside it as a wave-uniform flag applied
// when the column is used -- so the compiler waits only for the loads of the
// column about to be computed.  (A column past the tile's end is never used.)
template <int KIND, int PD>
__device__ __forceinline__ void wide_fetch_raw(const WideArgs &a, const WideProblem &p,
                                               const float *Bw, int lane, const Sweep<PD> &s,
                                               int c, float &top, float &cv, bool &have_top) {
  have_top = c <= s.jend && s.t > 0 && c >= s.bv_lo && c <= s.bv_hi;
  const int cc = c < 0 ? 0 : (c > a.lcol - 1 ? a.lcol - 1 : c);
  top = Bw[(int64_t)(cc + 1) * kWave + lane];
  cv = wide_col_value<KIND>(a, p, cc);
}

template <int H, int KIND, int H_LO, int H_HI, int PD>
__device__ __forceinline__ void wide_step_body(const WideArgs &a, float *Bw, int lane,
                                               float (&col)[H], const float (&rv)[H], Sweep<PD> &s,
                                               float ub, int tlast, int hans, float &ans,
                                               float top0, float cv, const float *wl);

// Weighted search: where column j's weights start in LDS (row h of the tile
// takes wl[H-1-h] = w(|j - (i0 + h)|)); nullptr for the other kinds.
template <int H, int KIND, int PD>
__device__ __forceinline__ const float *wide_weights(const WideArgs &a, const WideProblem &p,
                                                     const Sweep<PD> &s, int j) {
  if constexpr (KIND == kWideSearchW) return p.wsh + (j - s.t * H + a.r - (H - 1));
  return nullptr;
}

// One column: its prefetched values leave the front of the queue, whose
// entries shift down, and column j + PD enters at the back.
template <int H, int KIND, int H_LO, int H_HI, int PD>
__device__ __forceinline__ void wide_step(const WideArgs &a, const WideProblem &p, float *Bw,
                                          int lane, float (&col)[H], const float (&rv)[H],
                                          Sweep<PD> &s, float ub, int tlast, int hans, float &ans) {
  const int j = s.j;
  const float top0 = s.qtop[0];
  const float cv = s.qcv[0];
#pragma unroll
  for (int k = 0; k + 1 < PD; ++k) {
    s.qtop[k] = s.qtop[k + 1];
    s.qcv[k] = s.qcv[k + 1];
  }
  wide_fetch<KIND, PD>(a, p, Bw, lane, s, j + PD, s.qtop[PD - 1], s.qcv[PD - 1]);
  wide_step_body<H, KIND, H_LO, H_HI, PD>(a, Bw, lane, col, rv, s, ub, tlast, hans, ans, top0, cv,
                                          wide_weights<H, KIND, PD>(a, p, s, j));
}

// One column taking queue slot K (the column's index from the queue's start,
// mod PD) and refilling the same slot with column j + PD.  Slots rotate
// statically over PD unrolled steps, so no register is moved while its load
// is in flight: a move would have to wait for the load, and the queue's
// moves made every column wait for the loads issued just before it.
template <int H, int KIND, int PD, int K>
__device__ __forceinline__ void wide_step_slot(const WideArgs &a, const WideProblem &p, float *Bw,
                                               int lane, float (&col)[H], const float (&rv)[H],
                                               Sweep<PD> &s, bool (&qhave)[PD], float ub,
                                               int tlast, int hans, float &ans) {
  const int j = s.j;
  const float top0 = qhave[K] ? s.qtop[K] : kInf;
  const float cv = s.qcv[K];
  wide_fetch_raw<KIND, PD>(a, p, Bw, lane, s, j + PD, s.qtop[K], s.qcv[K], qhave[K]);
  wide_step_body<H, KIND, 0, H - 1, PD>(a, Bw, lane, col, rv, s, ub, tlast, hans, ans, top0, cv,
                                        wide_weights<H, KIND, PD>(a, p, s, j));
}

template <int H, int KIND, int H_LO, int H_HI, int PD>
__device__ __forceinline__ void wide_step_body(const WideArgs &a, float *Bw, int lane,
                                               float (&col)[H], const float (&rv)[H], Sweep<PD> &s,
                                               float ub, int tlast, int hans, float &ans,
                                               float top0, float cv, const float *wl) {
  const int j = s.j;
  wide_column<H, H_LO, H_HI, false, KIND == kWideSearchW>(col, rv, cv, top0, s.diag0, wl);
  s.diag0 = top0;
  Bw[(int64_t)(j + 1) * kWave + lane] = col[H - 1];
  const bool lane_alive = (s.alive_mask >> lane) & 1ull;
  const unsigned long long lm = __ballot(lane_alive && col[H - 1] <= ub);
  if (lm) {
    if (s.first_live > j) s.first_live = j;
    s.last_live = j;
    s.lane_live |= lm;
  }
  if (s.t == tlast && j == a.lcol - 1) {
#pragma unroll
    for (int h = 0; h < H; ++h)
      if (h == hans) ans = col[h];
  }
  // admissible cells of this column inside the matrix
  int hl = H_LO, hh = H_HI;
  if (hh > s.rows - 1) hh = (int)s.rows - 1;
  const int nc = hh >= hl ? hh - hl + 1 : 0;
  s.computed += (uint64_t)nc * kWave;
  s.evaluated += (uint64_t)nc * (uint64_t)__popcll(s.alive_mask);
  // right border: past the columns reachable from the tile above, stop after a
  // column whose cells are all dead in every lane
  if (j > s.jmand && ((j - s.jmand) & 3) == 0) {
    if (!wave_any(lane_alive && col_min<H>(col) <= ub)) s.go = false;
  }
  s.j = j + 1;
  if (s.j > s.jend) s.go = false;
}

// Two full columns j, j+1 in one step: the cells of column j+1 trail those of
// column j by one row, so the two dependency chains interleave.  Used where
// neither column needs the answer capture or a right-border check.
template <int H, int KIND, int PD>
__device__ __forceinline__ void wide_step2(const WideArgs &a, const WideProblem &p, float *Bw,
                                           int lane, float (&col)[H], const float (&rv)[H],
                                           Sweep<PD> &s, float ub) {
  const int j = s.j;
  const float topA = s.qtop[0], cvA = s.qcv[0];
  const float topB = s.qtop[1], cvB = s.qcv[1];
#pragma unroll
  for (int k = 0; k + 2 < PD; ++k) {
    s.qtop[k] = s.qtop[k + 2];
    s.qcv[k] = s.qcv[k + 2];
  }
  wide_fetch<KIND, PD>(a, p, Bw, lane, s, j + PD, s.qtop[PD - 2], s.qcv[PD - 2]);
  wide_fetch<KIND, PD>(a, p, Bw, lane, s, j + PD + 1, s.qtop[PD - 1], s.qcv[PD - 1]);
  // keep column j's last row for the boundary store before it is overwritten
  float lastA;
  const float *wlA = wide_weights<H, KIND, PD>(a, p, s, j);  // column j + 1: wlA + 1
  {
    float upA = topA, dgA = s.diag0;
    float prevA = 0.0f;
    float upB = topB, dgB = topA;
#pragma unroll
    for (int h = 0; h <= H; ++h) {
      float nA = 0.0f;
      if (h < H) {
        const float left = col[h];
        const float diff = cvA - rv[h];
        const float dw = KIND == kWideSearchW ? diff * wlA[H - 1 - h] : diff;
        nA = __builtin_fmaf(dw, diff, fmin3(left, upA, dgA));
        dgA = left;
        upA = nA;
      }
      if (h >= 1) {
        const int hb = h - 1;
        const float diff = cvB - rv[hb];
        const float dw = KIND == kWideSearchW ? diff * wlA[1 + H - 1 - hb] : diff;
        const float nB = __builtin_fmaf(dw, diff, fmin3(prevA, upB, dgB));
        dgB = prevA;
        upB = nB;
        col[hb] = nB;
      }
      prevA = nA;
    }
    lastA = upA;
  }
  s.diag0 = topB;
  Bw[(int64_t)(j + 1) * kWave + lane] = lastA;
  Bw[(int64_t)(j + 2) * kWave + lane] = col[H - 1];
  const bool lane_alive = (s.alive_mask >> lane) & 1ull;
  const unsigned long long lmA = __ballot(lane_alive && lastA <= ub);
  const unsigned long long lmB = __ballot(lane_alive && col[H - 1] <= ub);
  if (lmA) {
    if (s.first_live > j) s.first_live = j;
    s.last_live = j;
    s.lane_live |= lmA;
  }
  if (lmB) {
    if (s.first_live > j + 1) s.first_live = j + 1;
    s.last_live = j + 1;
    s.lane_live |= lmB;
  }
  int hh = H - 1;
  if (hh > s.rows - 1) hh = (int)s.rows - 1;
  const int nc = hh + 1;
  s.computed += (uint64_t)(2 * nc) * kWave;
  s.evaluated += (uint64_t)(2 * nc) * (uint64_t)__popcll(s.alive_mask);
  s.j = j + 2;
  if (s.j > s.jend) s.go = false;
}

// True when columns j and j+1 are both full columns of the middle stretch,
// neither holds the answer cell and neither is due for a right-border check.
template <int PD>
__device__ __forceinline__ bool wide_pair_ok(const Sweep<PD> &s, int jlast, int tlast, int lcol) {
  const int j = s.j;
  if (j + 1 > jlast || j + 1 > s.jend) return false;
  if (s.t == tlast && j + 1 >= lcol - 1) return false;
  if (j + 1 > s.jmand) return false;
  return true;
}

// entering triangle: column c = j - (i0 - r) has rows 0..c admissible
template <int H, int KIND, int C, int PD>
struct EnterPhase {
  __device__ __forceinline__ static void run(const WideArgs &a, const WideProblem &p, float *Bw,
                                             int lane, float (&col)[H], const float (&rv)[H],
                                             Sweep<PD> &s, float ub, int tlast, int hans, float &ans,
                                             int jbase) {
    if (s.go && s.j == jbase + C) wide_step<H, KIND, 0, C, PD>(a, p, Bw, lane, col, rv, s, ub, tlast, hans, ans);
    EnterPhase<H, KIND, C + 1, PD>::run(a, p, Bw, lane, col, rv, s, ub, tlast, hans, ans, jbase);
  }
};
template <int H, int KIND, int PD>
struct EnterPhase<H, KIND, H - 1, PD> {
  __device__ __forceinline__ static void run(const WideArgs &, const WideProblem &, float *, int,
                                             float (&)[H], const float (&)[H], Sweep<PD> &, float,
                                             int, int, float &, int) {}
};

// exiting triangle: column c = j - (i0 + r + 1) has rows c+1..H-1 admissible
template <int H, int KIND, int C, int PD>
struct ExitPhase {
  __device__ __forceinline__ static void run(const WideArgs &a, const WideProblem &p, float *Bw,
                                             int lane, float (&col)[H], const float (&rv)[H],
                                             Sweep<PD> &s, float ub, int tlast, int hans, float &ans,
                                             int jbase) {
    if (s.go && s.j == jbase + C) wide_step<H, KIND, C + 1, H - 1, PD>(a, p, Bw, lane, col, rv, s, ub, tlast, hans, ans);
    ExitPhase<H, KIND, C + 1, PD>::run(a, p, Bw, lane, col, rv, s, ub, tlast, hans, ans, jbase);
  }
};
template <int H, int KIND, int PD>
struct ExitPhase<H, KIND, H - 1, PD> {
  __device__ __forceinline__ static void run(const WideArgs &, const WideProblem &, float *, int,
                                             float (&)[H], const float (&)[H], Sweep<PD> &, float,
                                             int, int, float &, int) {}
};

// One problem per lane: all tiles.  Returns the lane's result (+inf if the
// distance exceeds the bound); accumulates the work counters.
template <int H, int KIND, bool BANDED, bool LIST = false>
__device__ __forceinline__ float wide_problem(const WideArgs &a, WideProblem &p, float *Bw, int lane,
                                              uint64_t &evaluated, uint64_t &computed) {
  const int r = a.r, lrow = a.lrow, lcol = a.lcol;
  const int ntiles = (lrow + H - 1) / H;
  const int tlast = ntiles - 1;
  const int hans = (lrow - 1) - tlast * H;
  float ub = p.ub;
  bool alive = p.active && ub >= 0.0f;
  bool stopped = !wave_any(alive);
  int lo = 0, hi = -1;       // live columns of the row above the tile (border row: origin)
  int bv_lo = 0, bv_hi = -1;
  float ans = kInf;
  int since = 0;
  for (int t = 0; t < ntiles && !stopped; ++t) {
    const int i0 = t * H;
    float rv[H], col[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
      rv[h] = wide_row_value<KIND>(a, p, i0 + h);
      col[h] = kInf;
    }
    // cascade list mode: every path through the tile still pays the
    // query-envelope LB_Keogh terms of the rows below it, so the tile's
    // liveness tests use the bound lowered by that rest (the cumulative-bound
    // tightening); the answer itself is compared with the bound
    float ubt = ub;
    if constexpr (LIST) {
#pragma unroll
      for (int h = 0; h < H; ++h) {
        if (i0 + h < lrow) {
          const float z = rv[h];
          const float dd = z - __builtin_amdgcn_fmed3f(z, a.lq[i0 + h], a.uq[i0 + h]);
          p.lb_prefix = __builtin_fmaf(dd, dd, p.lb_prefix);
        }
      }
      const float rest = p.lb_total - p.lb_prefix;
      ubt = ub - (rest > 0.0f ? rest : 0.0f);
    }
    const int jb_lo = i0 - r > 0 ? i0 - r : 0;
    const int jb_hi = i0 + H - 1 + r < lcol - 1 ? i0 + H - 1 + r : lcol - 1;
    constexpr int PD = H >= 64 ? 4 : 8;
    Sweep<PD> s;
    s.j = jb_lo > lo ? jb_lo : lo;
    s.jend = jb_hi;
    s.jmand = hi + 1;
    s.first_live = 0x7fffffff;
    s.last_live = -1;
    s.lane_live = 0ull;
    s.go = s.j <= s.jend;
    s.bv_lo = bv_lo;
    s.bv_hi = bv_hi;
    s.t = t;
    s.rows = lrow - i0 < H ? lrow - i0 : H;
    s.evaluated = 0;
    s.computed = 0;
    s.alive_mask = __ballot(alive);
    if (t == 0) s.diag0 = (s.j == 0) ? 0.0f : kInf;
    else s.diag0 = (s.j - 1 >= bv_lo && s.j - 1 <= bv_hi) ? Bw[(int64_t)s.j * kWave + lane] : kInf;
    const int jstart = s.j;
#pragma unroll
    for (int k = 0; k < PD; ++k) wide_fetch<KIND, PD>(a, p, Bw, lane, s, s.j + k, s.qtop[k], s.qcv[k]);
    // entering triangle [i0-r, i0-r+H-2], full columns up to i0+r, exiting triangle
    if (BANDED) {
      EnterPhase<H, KIND, 0, PD>::run(a, p, Bw, lane, col, rv, s, ubt, tlast, hans, ans, i0 - r);
      while (s.go && s.j <= i0 + r) {
        if (H <= 32 && wide_pair_ok(s, i0 + r, tlast, a.lcol)) wide_step2<H, KIND, PD>(a, p, Bw, lane, col, rv, s, ubt);
        else wide_step<H, KIND, 0, H - 1, PD>(a, p, Bw, lane, col, rv, s, ubt, tlast, hans, ans);
      }
      ExitPhase<H, KIND, 0, PD>::run(a, p, Bw, lane, col, rv, s, ubt, tlast, hans, ans, i0 + r + 1);
    } else {
      // the window covers the whole matrix: every column is a full column
      if constexpr (H > 32) {
        // PD columns per iteration, queue slots in static rotation
        static_assert(PD == 4, "four queue slots per rotation");
        bool qhave[PD];
#pragma unroll
        for (int k = 0; k < PD; ++k)
          wide_fetch_raw<KIND, PD>(a, p, Bw, lane, s, s.j + k, s.qtop[k], s.qcv[k], qhave[k]);
        while (s.go) {
          wide_step_slot<H, KIND, PD, 0>(a, p, Bw, lane, col, rv, s, qhave, ubt, tlast, hans, ans);
          if (s.go) wide_step_slot<H, KIND, PD, 1 % PD>(a, p, Bw, lane, col, rv, s, qhave, ubt, tlast, hans, ans);
          if (s.go) wide_step_slot<H, KIND, PD, 2 % PD>(a, p, Bw, lane, col, rv, s, qhave, ubt, tlast, hans, ans);
          if (s.go) wide_step_slot<H, KIND, PD, 3 % PD>(a, p, Bw, lane, col, rv, s, qhave, ubt, tlast, hans, ans);
        }
      } else {
        while (s.go) {
          // (two-column steps only pay off while the doubled state still fits
          // in registers at a useful occupancy)
          if (wide_pair_ok(s, s.jend, tlast, a.lcol)) wide_step2<H, KIND, PD>(a, p, Bw, lane, col, rv, s, ubt);
          else wide_step<H, KIND, 0, H - 1, PD>(a, p, Bw, lane, col, rv, s, ubt, tlast, hans, ans);
        }
      }
    }
    evaluated += s.evaluated;
    computed += s.computed;
    bv_lo = jstart;
    bv_hi = s.j - 1;
    if (t == tlast) break;  // the answer cell was captured during the sweep
    alive = alive && ((s.lane_live >> lane) & 1ull);
    if (s.last_live < 0 || !wave_any(alive)) {
      stopped = true;
      break;
    }
    lo = s.first_live;
    hi = s.last_live;
    if (wide_is_search(KIND) && !a.dists_mode && ++since >= a.check_interval) {
      since = 0;
      ub = fminf(ub, load_bsf_dist(a.bsf));
    } else if (KIND == kWidePairwise && a.nn1 && ++since >= a.check_interval) {
      since = 0;
      ub = fminf(ub, fmaxf(load_bsf_dist(p.nn_i), load_bsf_dist(p.nn_j)));
    }
  }
  return (alive && !stopped && ans <= ub) ? ans : kInf;
}

// One block of 64 consecutive candidate offsets of a search (task t covers
// offsets k_begin + 64 t + lane).
template <int H, bool BANDED, int KIND = kWideSearch>
__device__ __forceinline__ void wide_search_task(const WideArgs &a, int64_t task, float *Bw,
                                                 int lane, uint64_t &evaluated, uint64_t &computed,
                                                 uint64_t &abandoned, const float *wsh = nullptr) {
  WideProblem p{};
  p.wsh = wsh;
  const int64_t kb = a.k_begin + task * kWave;
  const int64_t k = kb + lane;
  p.active = k < a.k_end;
  const int64_t kc = p.active ? k : a.k_end - 1;
  double mean, sd;
  wave_window_stats(a.x, a.n, a.lrow, kb, lane, mean, sd);
  znorm_params(mean, sd, p.mu_hi, p.mu_lo, p.inv);
  p.xk = a.x + kc;
  p.ub = a.dists_mode ? a.fixed_ub : load_bsf_dist(a.bsf);
  const float d = wide_problem<H, KIND, BANDED>(a, p, Bw, lane, evaluated, computed);
  const bool keep = p.active && d <= p.ub && d < kInf;
  if (a.dists_mode) {
    if (p.active) a.dists[k - a.k_begin] = d;
  } else if (a.knn > 0) {
    publish_knn(KnnOut{a.bsf, a.knn, a.knn_buf, a.knn_n, a.counters, a.knn_slots}, keep, d,
                (uint32_t)k);
  } else {
    publish_best(a.bsf, keep, d, a.bound_only ? 0xffffffffu : (uint32_t)k);
  }
  abandoned += (uint64_t)__popcll(__ballot(p.active && !(d < kInf)));
}

// The search over a survivor list of the lower-bound cascade: lane l of task
// t takes list entry 64 t + l (tasks cover the longest possible list; entries
// past list_n are inactive) with the normalisation constants the bound pass
// stored; an entry whose largest lower bound (lowered by kLbMargin) is now
// above the bound in force is dropped before its sweep (counted as
// re-checked).  Otherwise the tiled sweep of wide_search_task, each tile's
// liveness tests taking the bound lowered by the rest of the entry's
// query-envelope LB_Keogh.
template <int H, bool BANDED>
__global__ __launch_bounds__(64) void wide_list_kernel(WideArgs a) {
  const int lane = threadIdx.x;
  float *Bw = a.bnd + (int64_t)blockIdx.x * a.bnd_stride;
  uint64_t evaluated = 0, computed = 0, abandoned = 0, rechecked = 0;
  const uint64_t nl = *a.list_n;
  for (int64_t task = blockIdx.x; task * kWave < (int64_t)nl; task += gridDim.x) {
    WideProblem p{};
    const int64_t e = task * kWave + lane;
    p.active = e < (int64_t)nl;
    const int64_t ec = p.active ? e : 0;
    const int64_t k = a.list_k[ec];
    p.mu_hi = a.list_mh[ec];
    p.mu_lo = a.list_ml[ec];
    p.inv = a.list_inv[ec];
    p.xk = a.x + k;
    p.ub = a.dists_mode ? a.fixed_ub : load_bsf_dist(a.bsf);
    p.lb_total = a.list_lbq[ec] * (1.0f - kLbMargin);
    p.lb_prefix = 0.0f;
    if (p.active && a.list_lbmax[ec] * (1.0f - kLbMargin) > p.ub) {
      p.ub = -1.0f;  // dead from the start: +inf, never kept
      ++rechecked;
    }
    const float d = wide_problem<H, kWideSearch, BANDED, true>(a, p, Bw, lane, evaluated, computed);
    const bool keep = p.active && d <= p.ub && d < kInf;
    if (a.dists_mode) {
      if (p.active) a.dists[k - a.k_begin] = d;
    } else if (a.knn > 0) {
      publish_knn(KnnOut{a.bsf, a.knn, a.knn_buf, a.knn_n, a.counters, a.knn_slots}, keep, d,
                  (uint32_t)k);
    } else {
      publish_best(a.bsf, keep, d, (uint32_t)k);
    }
    abandoned += (uint64_t)__popcll(__ballot(p.active && !(d < kInf)));
  }
  // (re-checked entries were counted per lane)
  for (int o = 32; o >= 1; o >>= 1) rechecked += (uint64_t)__shfl_xor((long long)rechecked, o, kWave);
  if (a.counters && lane == 0) {
    unsigned long long *c = counter_stripe(a.counters, blockIdx.x);
    atomicAdd(&c[kCntEvaluated], (unsigned long long)evaluated);
    atomicAdd(&c[kCntComputed], (unsigned long long)computed);
    atomicAdd(&c[kCntAbandoned], (unsigned long long)abandoned);
    atomicAdd(&c[kCntLbRecheck], (unsigned long long)rechecked);
  }
}

template <int H, int KIND, bool BANDED>
__global__ __launch_bounds__(64) void wide_kernel(WideArgs a) {
  const int lane = threadIdx.x;
  float *Bw = a.bnd + (int64_t)blockIdx.x * a.bnd_stride;
  uint64_t evaluated = 0, computed = 0, abandoned = 0;
  // weighted search: the 2r + 1 weights staged in LDS (launched with that
  // many floats of dynamic LDS; other kinds use none)
  extern __shared__ float wsh[];
  if constexpr (KIND == kWideSearchW) {
    for (int t = lane; t < 2 * a.r + 1 + 2 * kWtPad; t += kWave) wsh[t] = a.wt_band[t];
    __syncthreads();
  }
  for (int64_t task = blockIdx.x; task < a.ntasks; task += gridDim.x) {
    WideProblem p{};
    if (KIND == kWideSearch) {
      wide_search_task<H, BANDED>(a, task, Bw, lane, evaluated, computed, abandoned);
    } else if (KIND == kWideSearchW) {
      wide_search_task<H, BANDED, kWideSearchW>(a, task, Bw, lane, evaluated, computed, abandoned,
                                                wsh + kWtPad);
    } else if (KIND == kWidePairwise) {
      const int64_t i = task / a.nblk_j, jb = task % a.nblk_j;
      const bool cross = a.nq > 0;
      if (!cross && jb * kWave + kWave - 1 <= i) continue;  // block on or below the diagonal
      const int64_t j = jb * kWave + lane;
      p.active = (cross || j > i) && j < a.N;
      const int64_t jc = p.active ? j : a.N - 1;
      p.rowp = a.X + i * a.lrow;
      p.colp = a.XT + jc;
      p.cstride = a.ld;
      float acc = 0.0f;
      for (int t = 0; t < a.lrow; ++t) {
        const float diff = p.colp[(int64_t)t * p.cstride] - p.rowp[t];
        acc = __builtin_fmaf(diff, diff, acc);
      }
      p.ed = acc;
      p.ub = acc;
      if (a.nn1) {
        // NN1: the pair only matters if it beats the best of row i or of row j
        // so far, so it is abandoned above the larger of the two (re-read
        // during the sweep; never more than the squared ED, an admissible
        // path's cost)
        // (a reference-set column has no word: only row i's best counts)
        p.nn_i = a.nn1 + i;
        p.nn_j = cross ? p.nn_i : a.nn1 + jc;
        p.ub = fminf(acc, fmaxf(load_bsf_dist(p.nn_i), load_bsf_dist(p.nn_j)));
      }
      const float d = wide_problem<H, KIND, BANDED>(a, p, Bw, lane, evaluated, computed);
      if (a.nn1) {
        // the row learns the pair, and within one set so does the column:
        // (distance, other index) packed, min-ed
        const bool keep = p.active && d < kInf;
        publish_best(a.nn1 + i, keep, d, (uint32_t)j);
        if (!cross && keep) atomicMin(a.nn1 + j, pack_best(d, (uint32_t)i));
      } else if (p.active) {
        a.out[i * a.N - i * (i + 1) / 2 + (j - i - 1)] = d < kInf ? d : p.ed;
      }
      abandoned += (uint64_t)__popcll(__ballot(p.active && !(d < kInf)));
    } else {
      const int64_t pp = task * kWave + lane;
      p.active = pp < a.N;
      const int64_t pc = p.active ? pp : a.N - 1;
      p.rowp = a.RT + pc;
      p.colp = a.XT + pc;
      p.cstride = a.ld;
      if (a.ub_mode == 1) {
        p.ub = a.ub[pc];
      } else if (a.ub_mode == 2) {
        float acc = 0.0f;
        for (int t = 0; t < a.lrow; ++t) {
          const float diff = p.colp[(int64_t)t * p.cstride] - p.rowp[(int64_t)t * a.ld];
          acc = __builtin_fmaf(diff, diff, acc);
        }
        p.ed = acc;
        p.ub = acc;
      } else if (a.ub_mode == 3) {
        p.ub = a.ub_scalar;
      } else {
        p.ub = kInf;
      }
      const float d = wide_problem<H, KIND, BANDED>(a, p, Bw, lane, evaluated, computed);
      if (p.active) a.out[pp] = (d < kInf || a.ub_mode != 2) ? d : p.ed;
      abandoned += (uint64_t)__popcll(__ballot(p.active && !(d < kInf)));
    }
  }
  if (a.counters && lane == 0) {
    unsigned long long *c = counter_stripe(a.counters, blockIdx.x);
    atomicAdd(&c[kCntEvaluated], (unsigned long long)evaluated);
    atomicAdd(&c[kCntComputed], (unsigned long long)computed);
    atomicAdd(&c[kCntAbandoned], (unsigned long long)abandoned);
  }
}

}  // namespace eapdtw
