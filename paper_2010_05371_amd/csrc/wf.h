// wf.h -- wavefront pair kernels: one pair per group of G lanes, the DP swept
// along anti-diagonals with one matrix row per lane and cell slot.
//
// A pair (S, T) of lengths (ls, lt) under window r (Section 2 Eq. 1-5,
// Section 2.1) is computed by P = G * NC lane-slots: slot c of lane g owns the
// rows i = c G + g (mod P).  At step t every lane-slot computes the cell
// (i, t - i) of its current row; the cell's three predecessors are
//   (i-1, t-i)   -> the previous lane-slot's value of step t-1 (one rotation),
//   (i-1, t-i-1) -> the value the lane-slot received at step t-1,
//   (i,   t-i-1) -> its own value of step t-1,
// so one register rotation per step carries the whole recurrence.  At most
// min(r+1, ls, lt) rows are active at a step, and P exceeds that count, so a
// lane-slot never holds two active rows at once; it moves to row i + P after
// its row's last cell.  Out-of-band and out-of-matrix cells read +inf.
#pragma once
#include "common.h"

namespace eapdtw {

// One pair of a wavefront launch.  s_off / t_off index the S and T pools;
// rec_off is the first word of the pair's direction record (see below).
struct WfPair {
  int64_t s_off, t_off, rec_off;
  int32_t ls, lt, r, pad;
};

// Kernel classes: lanes per pair G and cell slots per lane NC, by lane-slots
// P = G NC.  A pair needs P >= min(r+1, ls, lt) + 1 (r clipped to
// max(ls, lt) - 1), and its two series must fit the class's LDS share
// (64 / G pairs per wave).
constexpr int kWfClasses = 9;
constexpr int kWfG[kWfClasses] = {16, 16, 32, 16, 32, 64, 64, 64, 64};
constexpr int kWfNC[kWfClasses] = {1, 2, 1, 4, 2, 1, 2, 4, 8};
constexpr int kWfMaxP = 512;
constexpr int kWfChunk = 16;               // steps per direction word (2 bits each)
constexpr int kWfLdsFloats = 16384;        // LDS of one wave (64 KB)
constexpr int kWfPad = 2 * kWfChunk + 1;   // guard cells on each side of a staged T (chunks of up to 32 steps)
constexpr int kWfMaxLen = 8191;            // longest series of a wavefront pair
constexpr int kDbaPairs = 64;              // pairs per partial sum of the DBA update
// Waves a launch should reach: two per SIMD lets the SIMDs issue VALU
// instructions of two waves in the same cycle.
constexpr int64_t kWfTargetWaves = 2048;

// Status word of a pair's record.
enum WfStatus : unsigned { kWfOk = 1u, kWfNoPath = 2u, kWfNonFinite = 3u };

__host__ __device__ inline int wf_active_rows(int ls, int lt, int r) {
  int a = r + 1;
  if (ls < a) a = ls;
  if (lt < a) a = lt;
  return a;
}

__host__ inline bool wf_plain_fits(int ls, int lt, int cls) {
  return (int64_t)(ls + lt + 2 * kWfPad) * (kWave / kWfG[cls]) <= kWfLdsFloats;
}

__host__ __device__ inline int64_t wf_steps(int ls, int lt) { return (int64_t)ls + lt - 1; }

// Chunks of kWfChunk steps of a pair (0 for an empty series).
__host__ __device__ inline int wf_chunks(int ls, int lt) {
  const int64_t ns = wf_steps(ls, lt);
  return ns > 0 ? (int)((ns + kWfChunk - 1) / kWfChunk) : 0;
}

// Code words of a pair's direction record in class c: one word per lane-slot
// and chunk of kWfChunk steps.
__host__ inline int64_t wf_rec_words(int ls, int lt, int cls) {
  const int64_t P = (int64_t)kWfG[cls] * kWfNC[cls];
  return (int64_t)wf_chunks(ls, lt) * P;
}

// LDS words of one group in a forward of mode 2 (series, guards, code words
// and path ranges) and whether a wave of class c holds them.
__host__ inline int64_t wf_fused_words(int ls, int lt, int cls) {
  return (int64_t)ls + lt + 2 * kWfPad + wf_rec_words(ls, lt, cls) + ls + lt;
}
// (a mode-2 wave keeps kWfScratchWords after its groups' regions: 9 words
// per lane)
constexpr int kWfScratchWords = 9 * kWave;
__host__ inline bool wf_fused_fits(int ls, int lt, int cls) {
  return wf_fused_words(ls, lt, cls) * (kWave / kWfG[cls]) <= kWfLdsFloats - kWfScratchWords;
}

// Class of a pair in a launch of about `npairs` pairs (0: many): the fewest
// lane-slots that hold the pair; among classes with as many, the most cell
// slots per lane (more independent work per lane) that still gives the
// launch kWfTargetWaves waves, else the one with the most waves.  `lanes`
// (16, 32, 64) restricts G; `fused` asks for a class whose codes fit in LDS.
// -1 when no class qualifies.
__host__ inline int wf_choose(int ls, int lt, int r, int64_t npairs, int lanes, bool fused) {
  const int need = wf_active_rows(ls, lt, r) + 1;
  int best = -1;
  for (int c = 0; c < kWfClasses; ++c) {
    const int P = kWfG[c] * kWfNC[c];
    if (P < need || (lanes && kWfG[c] != lanes) || !wf_plain_fits(ls, lt, c)) continue;
    if (fused && !wf_fused_fits(ls, lt, c)) continue;
    if (best < 0) {
      best = c;
      continue;
    }
    if (P > kWfG[best] * kWfNC[best]) break;  // classes are ordered by P
    const int64_t gb = kWave / kWfG[best], gc = kWave / kWfG[c];
    const int64_t wb = npairs > 0 ? (npairs + gb - 1) / gb : kWfTargetWaves;
    const int64_t wc = npairs > 0 ? (npairs + gc - 1) / gc : kWfTargetWaves;
    const bool ok_b = wb >= kWfTargetWaves, ok_c = wc >= kWfTargetWaves;
    if ((ok_c && !ok_b) || (ok_c && ok_b && kWfNC[c] > kWfNC[best]) ||
        (!ok_c && !ok_b && wc > wb))
      best = c;
  }
  return best;
}

// Class of a pair (r clipped) by size, or -1 when no class holds it.
__host__ inline int wf_class_for(int ls, int lt, int r) { return wf_choose(ls, lt, r, 0, 0, false); }

// Class of a pair whose path is wanted: the chosen class that keeps its codes
// in LDS (*fused = true), else the chosen class (codes in memory).  `lanes`
// (16, 32, 64; 0: any) picks the lanes per pair among the classes that keep
// the codes in LDS, so that the record's size does not depend on it.
__host__ inline int wf_path_class(int ls, int lt, int r, int64_t npairs, int lanes, bool *fused) {
  const int c = wf_choose(ls, lt, r, npairs, 0, true);
  *fused = c >= 0;
  if (c < 0) return wf_choose(ls, lt, r, npairs, 0, false);
  const int cl = lanes ? wf_choose(ls, lt, r, npairs, lanes, true) : -1;
  return cl >= 0 ? cl : c;
}

struct WfArgs {
  const float *S, *T;        // value pools
  const WfPair *pairs;       // descriptors (nullptr: uniform pairs, below)
  const int32_t *order;      // pair of launch item q (nullptr: q)
  int64_t nitems;            // pairs of this launch
  int ls, lt, r;             // uniform pairs: pair p = S[p ls ..], T[p lt ..]
  int64_t rec_words_u;       // uniform pairs: code words per pair
  float *out;                // distances [pair]
  unsigned *rec;             // mode 1: code words (pair p's at rec_off)
  unsigned *status;          // modes 1, 2: WfStatus [pair]
  unsigned *rowrng, *colrng; // mode 2: path ranges, pool-shaped (as the walk's)
  int lds_stride;            // floats of LDS per group (>= ls + lt + 2 kWfPad;
                             // mode 2: wf_fused_words)
  const float *ub;           // early-abandoning bound [pair] (nullptr: none; not with rec)
  unsigned long long *counters;  // kCntEvaluated / kCntComputed / kCntAbandoned (nullable)
};

// Forward sweep of one class: mode 0 distances, 1 also the 2-bit argmin
// codes, 2 also the path ranges (codes kept in LDS).
hipError_t launch_wf_fwd(int cls, int mode, const WfArgs &a, hipStream_t st);

// Backtrack of every pair from its record: per row i the column range of its
// path cells (jlo | jhi << 16 at rowrng[s_off + i]) and per column j the row
// range (colrng[t_off + j]).
struct WfWalkArgs {
  const WfPair *pairs;
  int64_t npairs;
  const int32_t *order;      // pair of launch item q (nullptr: q)
  int64_t nitems;            // pairs of this launch
  int ls, lt, r;             // uniform pairs (pairs == nullptr)
  int64_t rec_words_u;
  const unsigned *rec;       // code words
  const unsigned *status;    // WfStatus [pair]
  unsigned *rowrng, *colrng;
  int max_chunks;            // record chunks of the launch's longest pair
  int max_ranges;            // ls + lt of the launch's longest pair
  int win_words, lds_ranges; // set by the launcher
};
constexpr int kWalkWindow = 4096;          // record words an LDS window holds
constexpr int kWalkLds = 32768;            // LDS bytes of one walk
hipError_t launch_wf_walk(int P, const WfWalkArgs &a, hipStream_t st);

// Gradients from the path ranges: dS(i) = 2 g sum (S(i) - T(j)), dT(j) =
// -2 g sum (S(i) - T(j)) over the pair's path cells (zero without a path,
// NaN for a pair with a non-finite input).
struct WfGradArgs {
  const WfPair *pairs;
  int64_t npairs;
  int ls, lt;                // uniform pairs (pairs == nullptr)
  int max_ls, max_lt;        // pairs != nullptr: the longest series of the launch
  const unsigned *status;    // WfStatus [pair]
  const float *S, *T;
  const unsigned *rowrng, *colrng;
  const float *gout;
  float *gS, *gT;
};
hipError_t launch_wf_grad(const WfGradArgs &a, hipStream_t st);

// One DBA update of a barycentre B [lb] against n series of length len (the
// pairs (B, X[p]) of a uniform launch): per point i of B the sum and the count
// of the values X[p][j] its optimal paths align with it, per kDbaPairs pairs
// (partial [nchunk][lb], float64), then their totals in chunk order:
// out_B[i] = sum / count.
hipError_t launch_wf_dba(const float *X, int64_t n, int len, int lb, const unsigned *rowrng,
                         const unsigned *status, double *partial_sum, double *partial_cnt,
                         int64_t nchunk, float *out_B, float *out_count, hipStream_t st);

}  // namespace eapdtw
