// wf.hip -- wavefront pair kernels (gfx950): forward sweep with an optional
// record of the optimal predecessors, backtrack of the optimal warping path,
// and the path's gradient and DBA averages.
//
// DTW (Section 2, Eq. 1-5) is the cost of the optimal warping path; with the
// path fixed it is a sum of (S(i) - T(j))^2 over the path cells, so
//   dD/dS(i) =  2 sum over path cells (i, j) of (S(i) - T(j)),
//   dD/dT(j) = -2 sum over path cells (i, j) of (S(i) - T(j)).
// The forward records, per cell, which predecessor gave the minimum (2 bits;
// ties: diagonal, then (i-1, j), then (i, j-1)); the backtrack follows the
// record from (ls-1, lt-1) to (0, 0).  The ls x lt matrix is never stored.
#include "band.h"
#include "dispatch.h"
#include "wf.h"

namespace eapdtw {

namespace {

constexpr int kNever = 0x3fffffff;

// rotation by one lane inside groups of G lanes (lane g reads lane g-1, lane 0
// reads lane G-1): DPP row_ror:1 for G = 16, wave_ror:1 for G = 64.  For
// G = 32 the wave_ror:1 result is right except on lanes 0 and 32, which hold
// lanes 63 and 31; group_fix swaps them (below).
template <int G>
__device__ __forceinline__ float rot1(float x) {
  static_assert(G == 16 || G == 32 || G == 64, "groups of 16, 32 or 64 lanes");
  constexpr int ctrl = (G == 16) ? 0x121 : 0x13C;
  // every lane reads a lane of the wave: the old value is never used
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), ctrl, 0xf, 0xf, true));
}

// rotation by one lane the other way (lane g reads lane g+1, lane G-1 reads
// lane 0): row_ror:15 for G = 16, wave_rol:1 for G = 32 and 64 (G = 32: lanes
// 31 and 63 then need group_fix32 with the lanes G-1 taking the other half).
template <int G>
__device__ __forceinline__ uint32_t rot1_back(uint32_t x) {
  static_assert(G == 16 || G == 32 || G == 64, "groups of 16, 32 or 64 lanes");
  constexpr int ctrl = (G == 16) ? 0x12F : 0x134;
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, ctrl, 0xf, 0xf, true);
}

// G = 32: lanes 0 and 32 of a wave_ror:1 result y take each other's values.
// v_permlane32_swap of (y, y) gives lo = (y[0..31], y[0..31]) and
// hi = (y[32..63], y[32..63]); lanes 1..31 and 32 read lo, lanes 0 and
// 33..63 read hi (half_lo: all ones where lo is read).
__device__ __forceinline__ uint32_t group_fix32(uint32_t y, uint32_t half_lo) {
  const auto r = __builtin_amdgcn_permlane32_swap(y, y, false, false);
  return (half_lo & r[0]) | (~half_lo & r[1]);
}

struct PairView {
  int64_t s_off, t_off, rec_off;
  int ls, lt, r;
};

__device__ __forceinline__ PairView pair_view(const WfPair *pairs, int64_t p, int ls, int lt,
                                              int r, int64_t rec_words_u) {
  PairView v;
  if (pairs) {
    const WfPair d = pairs[p];
    v.s_off = d.s_off;
    v.t_off = d.t_off;
    v.rec_off = d.rec_off;
    v.ls = d.ls;
    v.lt = d.lt;
    v.r = d.r;
  } else {
    v.s_off = p * ls;
    v.t_off = p * lt;
    v.rec_off = p * rec_words_u;
    v.ls = ls;
    v.lt = lt;
    v.r = r;
  }
  return v;
}

__device__ __forceinline__ bool has_path(const PairView &v) {
  const int d = v.ls > v.lt ? v.ls - v.lt : v.lt - v.ls;
  return v.ls > 0 && v.lt > 0 && d <= v.r;
}

}  // namespace

// ---------------------------------------------------------------------------
// Forward sweep.  Group `grp` of the wave (G lanes) takes launch item
// blockIdx.x * (64 / G) + grp.  Its two series are staged in LDS, T between
// kWfPad guard cells on each side (0 on the left, +inf on the right).
// Lane g, slot c keeps its row's state in registers:
//   row, [ts, te]   current row and the steps of its in-band cells,
//   sv              S(row),
//   cur             value published at the last step (NaN when inactive),
//   up              value received at the last step (the diagonal predecessor).
// A NaN cell compares above +inf in the unsigned order of the minimum, so an
// inactive lane-slot acts as a border cell.
//
// Time.  The pair's steps are t = 0 .. ns-1 (ns = ls + lt - 1); the group
// starts at t = -e with e = (-ns) mod 16, so its last step closes a 16-step
// code word and the distance is read at the end of one.  Before t = 0,
// lane-slot P-1 holds a virtual row -1 whose cells cost (0 - 0)^2 = 0 (the
// left guard is 0) and carry the value 0 up to step -2: it is M(0,0) = 0, the
// diagonal predecessor of cell (0,0), and then leaves (+inf above row 0).
//
// Steps run in chunks of CH = 16 steps (32 when P >= 32 and NC <= 2).  A lane-slot's
// rows start at least P >= CH steps apart, so a chunk involves at most its
// current row a and the next row b = a + P: per chunk it prepares b's state,
// the steps that use b, and the mask of its active steps; a step then only
// selects between the two.
// MODE 0 computes distances only.  MODE 1 also writes every cell's argmin
// code to the record: word k = (t + e) / 16 of lane-slot l is
// rec[rec_off + k P + l], step t at bits 2 ((t + e) % 16).  MODE 2 keeps those
// words in the group's LDS and recovers the path in the same launch (the
// reverse sweep below), then writes the path ranges.

// (m & a) | (~m & b): with m all ones or all zeros, a or b (v_bfi_b32)
__device__ __forceinline__ uint32_t bit_select(uint32_t m, uint32_t a, uint32_t b) {
  return (m & a) | (~m & b);
}
__device__ __forceinline__ uint32_t umin2(uint32_t a, uint32_t b) { return a < b ? a : b; }
// bit s of m sign-extended to all ones / zeros (v_bfe_i32).  Written as asm so
// that the selections built on it stay v_bfi_b32 instead of becoming a
// compare and a v_cndmask each.
// The value of x, unknown to the optimiser (no instruction): keeps the
// selections and minimum below single VALU instructions instead of forms
// derived from known value ranges.
__device__ __forceinline__ uint32_t opaque(uint32_t x) {
  asm("" : "+v"(x));
  return x;
}
// Reverse sweep: 1 when a cell is named by a path cell (bit 2 of own, bit 1
// of rcv or bit 0 of rcvp; at most one of them is set), else 0.  One asm
// block: three VALU instructions.
__device__ __forceinline__ uint32_t path_named(uint32_t own, uint32_t rcv, uint32_t rcvp) {
  uint32_t r;
  asm("v_bfi_b32 %0, 2, %2, %3\n\t"
      "v_bfi_b32 %0, 4, %1, %0\n\t"
      "v_min_u32 %0, 1, %0"
      : "=&v"(r)
      : "v"(own), "v"(rcv), "v"(rcvp));
  return r;
}
__device__ __forceinline__ uint32_t mask_bit(uint32_t m, int s) {
  uint32_t r;
  asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(r) : "v"(m), "n"(s));
  return r;
}
// byte address of an LDS location and a load from one
__device__ __forceinline__ uint32_t lds_addr(const float *p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) float *)p;
}
__device__ __forceinline__ float lds_load(uint32_t a) {
  return *(const __attribute__((address_space(3))) float *)(uintptr_t)a;
}

// bits lo..hi of a CH-bit mask (empty when lo > hi), lo/hi clipped to 0..CH-1
template <int CH>
__device__ __forceinline__ unsigned bit_range(int lo, int hi) {
  lo = lo < 0 ? 0 : lo;
  hi = hi > CH - 1 ? CH - 1 : hi;
  if (lo > hi) return 0u;
  const unsigned top = hi == 31 ? ~0u : ((2u << hi) - 1u);
  return top & ~((1u << lo) - 1u);
}

// Copies src[0 .. n) (n >= 1) to LDS with the group's G lanes, eight loads per
// lane in flight before their stores (from clamped, always valid indexes, so
// no branch splits them): when the series come from HBM rather than the
// caches, a load-store-load chain would cost one memory latency per element.
// Notes a non-finite value in `bad`.
template <int G>
__device__ __forceinline__ void stage_series(const float *__restrict__ src, float *dst, int n,
                                             int g, bool &bad) {
  constexpr int B = 8;
  for (int k0 = g; k0 < n; k0 += B * G) {
    float x[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int k = k0 + u * G;
      x[u] = src[k < n ? k : n - 1];
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int k = k0 + u * G;
      if (k < n) {
        bad = bad || !__builtin_isfinite(x[u]);
        dst[k] = x[u];
      }
    }
  }
}

__device__ __forceinline__ int wf_lead(int ns) { return (kWfChunk - ns % kWfChunk) % kWfChunk; }

template <int G, int NC, int MODE>
__global__ __launch_bounds__(64) void wf_fwd_kernel(WfArgs a) {
  constexpr bool REC = MODE != 0;
  constexpr int P = G * NC;
  // steps per chunk: a chunk of at most P steps meets at most two rows of a
  // lane-slot (its rows start at least P steps apart), so classes with 32 or
  // more lane-slots and at most two cells per lane take 32 steps per chunk
  // (half the per-chunk work per step; with more cells per lane the longer
  // chunk's registers would not fit)
  constexpr int CH = (P >= 32 && NC <= 2) ? 32 : kWfChunk;
  constexpr int NW = CH / kWfChunk;  // code words per lane-slot and chunk
  constexpr int GPW = kWave / G;
  extern __shared__ float lds[];
  const int lane = threadIdx.x;
  const int grp = lane / G;
  const int g = lane & (G - 1);
  const int64_t q = (int64_t)blockIdx.x * GPW + grp;
  const bool valid = q < a.nitems;
  const int64_t p = valid ? (a.order ? (int64_t)a.order[q] : q) : 0;
  PairView v = pair_view(a.pairs, p, a.ls, a.lt, a.r, a.rec_words_u);
  if (!valid) v.ls = v.lt = 0;
  const int ls = v.ls, lt = v.lt, r = v.r;
  const bool path = valid && has_path(v);

  // stage S, then T with its guards; note non-finite inputs
  float *Sl = lds + grp * a.lds_stride;
  float *Tl = Sl + ls + kWfPad;  // Tl[j] for j in [-kWfPad, lt + kWfPad)
  bool bad = false;
  if (path) {
    stage_series<G>(a.S + v.s_off, Sl, ls, g, bad);
    stage_series<G>(a.T + v.t_off, Tl, lt, g, bad);
    for (int k = g; k < kWfPad; k += G) {
      Tl[-1 - k] = 0.0f;
      Tl[lt + k] = kInf;
    }
  }
  __syncthreads();
  const unsigned long long gmask = (G == 64) ? ~0ull : (((1ull << (G & 63)) - 1ull) << (grp * G));
  const bool pair_bad = (__builtin_amdgcn_ballot_w64(bad) & gmask) != 0ull;
  const bool run = path && !pair_bad;
  const int ns = run ? (int)wf_steps(ls, lt) : 0;
  const int e = wf_lead(ns);
  const int nsp = ns + e;  // steps of the group, a multiple of the chunk
  int nsw = nsp;           // steps of the wave: the longest of its groups
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const int t = __shfl_xor(nsw, o, kWave);
    nsw = t > nsw ? t : nsw;
  }

  // active steps [ts, te] of row i (row -1: the virtual row before step -1)
  auto span = [&](int i, int &ts, int &te) {
    if (i < 0) {
      ts = -kNever;
      te = -2;
      return;
    }
    if (!run || i >= ls) {
      ts = te = kNever;
      return;
    }
    const int jlo = i - r > 0 ? i - r : 0;
    const int jhi = i + r < lt - 1 ? i + r : lt - 1;
    ts = i + jlo;
    te = i + jhi;
  };
  const int lsm = ls > 0 ? ls - 1 : 0;
  auto s_of = [&](int i) -> float { return i < 0 ? 0.0f : Sl[i < lsm ? i : lsm]; };

  const float qnan = __builtin_nanf("");
  int row[NC], ts[NC], te[NC];
  float sv[NC], cur[NC], up[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int l = c * G + g;
    row[c] = (l == P - 1) ? -1 : l;
    span(row[c], ts[c], te[c]);
    sv[c] = s_of(row[c]);
    // the virtual row's 0 reaches cell (0,0) as its diagonal: through lane-slot
    // P-1 when the group starts before step 0, else directly
    cur[c] = (l == P - 1 && e >= 1) ? 0.0f : qnan;
    up[c] = (l == 0 && e == 0) ? 0.0f : qnan;
  }
  const int nch = run ? wf_chunks(ls, lt) : 0;
  // MODE 2: the group's code words and path ranges follow its series in LDS
  unsigned *codes_l = reinterpret_cast<unsigned *>(Tl + lt + kWfPad);
  unsigned *rr_l = codes_l + nch * P;
  unsigned *cr_l = rr_l + ls;
  unsigned *rec = MODE == 1 ? a.rec + v.rec_off : codes_l;
  const float *tbase = Tl;
  const uint32_t lane0 = g == 0 ? ~0u : 0u;
  const uint32_t half_lo = ((lane < 32) != (g == 0)) ? ~0u : 0u;  // G = 32 only
  // Early abandoning (Section 2.2): every warping path visits one of any two
  // consecutive anti-diagonals, and cell values never decrease along a path,
  // so once every cell of the chunk's last two anti-diagonals exceeds the
  // bound, so does the distance.
  const float ubv = (!REC && a.ub && valid) ? a.ub[p] : kInf;
  const bool check_ub = !REC && a.ub != nullptr;
  bool alive = run;
  float fin = kInf;  // the distance, read at the end of the group's last chunk
  const int le = run ? (ls - 1) % P : 0;
  uint64_t evaluated = 0, chunks = 0;

#pragma unroll 1
  for (int tau0 = 0; tau0 < nsw; tau0 += CH) {
    const int t0 = tau0 - e;  // the group's step at the chunk's start
    // per slot: row b's state, the steps of the chunk that use row b
    // (bsel), the inactive steps (idle), and the T reads of both rows
    int rowB[NC], tsB[NC], teB[NC];
    unsigned bsel[NC], idle[NC];
    uint32_t svA[NC], svBb[NC], pa[NC], pb[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      rowB[c] = row[c] + P;
      span(rowB[c], tsB[c], teB[c]);
      svA[c] = __float_as_uint(sv[c]);
      svBb[c] = __float_as_uint(s_of(rowB[c]));
      const int ea = te[c] - t0 + 1;  // row a is current for steps s < sw
      const int sw = ea > CH ? CH : ea;
      bsel[c] = bit_range<CH>(sw, CH - 1);
      idle[c] = ~(bit_range<CH>(ts[c] - t0, sw - 1) | bit_range<CH>(tsB[c] - t0, teB[c] - t0));
      int ja = t0 - row[c], jb = t0 - rowB[c];
      ja = ja < -kWfPad ? -kWfPad : (ja > lt ? lt : ja);
      jb = jb < -kWfPad ? -kWfPad : (jb > lt ? lt : jb);
      pa[c] = lds_addr(tbase + ja);
      pb[c] = lds_addr(tbase + jb);
    }
    unsigned cw[NC][NW];
    float c14[NC];  // values of the chunk's second-to-last step
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int h = 0; h < NW; ++h) cw[c][h] = 0u;
    // The cost differences of SUB steps, prepared ahead of their sweep so that
    // the LDS reads are in flight together: S(row) - T(t - row) on the
    // lane-slot's active steps, all-ones (a NaN) on the others.  Selections
    // use sign-extended mask bits (no compares).
    constexpr int SUB = NC >= 4 ? 4 : (NC == 2 ? 16 : CH);
#pragma unroll
    for (int s0 = 0; s0 < CH; s0 += SUB) {
      float dv[NC][SUB];
      // all reads first, then the arithmetic: one wait for the whole batch
      uint32_t bm[NC][SUB];
      float tv[NC][SUB];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
#pragma unroll
        for (int u = 0; u < SUB; ++u) {
          bm[c][u] = mask_bit(bsel[c], s0 + u);
          tv[c][u] = lds_load(bit_select(bm[c][u], pb[c], pa[c]) + 4u * (s0 + u));
        }
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
#pragma unroll
        for (int u = 0; u < SUB; ++u) {
          const float d = __uint_as_float(bit_select(bm[c][u], svBb[c], svA[c])) - tv[c][u];
          dv[c][u] = __uint_as_float(__float_as_uint(d) | mask_bit(idle[c], s0 + u));
        }
      }
#pragma unroll
      for (int u = 0; u < SUB; ++u) {
        const int s = s0 + u;
        if (s == CH - 1) {
#pragma unroll
          for (int c = 0; c < NC; ++c) c14[c] = cur[c];
        }
        if (s == kWfChunk && t0 + kWfChunk - 1 == ns - 1) {
          // the group's last step closed the chunk's first half: the cell
          // (ls-1, lt-1) of lane-slot (ls-1) mod P
#pragma unroll
          for (int c = 0; c < NC; ++c)
            if (le / G == c) fin = cur[c];
        }
        float rot[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) rot[c] = rot1<G>(cur[c]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          // the previous row: the previous lane of this slot, or for lane 0 the
          // last lane of the previous slot
          uint32_t topb =
              NC > 1 ? bit_select(lane0, cell_bits(rot[(c + NC - 1) % NC]), cell_bits(rot[c]))
                     : cell_bits(rot[c]);
          if constexpr (G == 32) topb = group_fix32(topb, half_lo);
          // cells are never negative (NaN: inactive): the unsigned order of
          // the bits is their order
          const uint32_t upb = cell_bits(up[c]);
          const uint32_t mb = umin3(topb, upb, cell_bits(cur[c]));
          if constexpr (REC) {
            // code 0: diagonal, 1: (i-1, j), 2: (i, j-1), ties in that order
            const uint32_t x = umin2(upb - mb, 1u);
            const uint32_t y = umin2(topb - mb, x);
            cw[c][s / kWfChunk] |= (x + y) << (2 * (s % kWfChunk));
          }
          up[c] = __uint_as_float(topb);
          cur[c] = __builtin_fmaf(dv[c][u], dv[c][u], __uint_as_float(mb));
        }
      }
    }
    if constexpr (REC) {
#pragma unroll
      for (int h = 0; h < NW; ++h) {
        if (tau0 + h * kWfChunk < nsp) {
          unsigned *w = rec + (tau0 / kWfChunk + h) * P + g;
#pragma unroll
          for (int c = 0; c < NC; ++c) w[c * G] = cw[c][h];
        }
      }
    }
    if (t0 + CH - 1 == ns - 1) {
      // the group's last step: the cell (ls-1, lt-1) of lane-slot (ls-1) mod P
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (le / G == c) fin = cur[c];
    }
    if (alive) {
      // matrix cells only (not the virtual row)
      const unsigned lim = bit_range<CH>(-t0, ns - 1 - t0);
#pragma unroll
      for (int c = 0; c < NC; ++c) evaluated += __builtin_popcount(~idle[c] & lim);
    }
    ++chunks;
    if (check_ub) {
      uint32_t m = ~0u;
#pragma unroll
      for (int c = 0; c < NC; ++c) m = umin3(m, cell_bits(c14[c]), cell_bits(cur[c]));
#pragma unroll
      for (int o = G / 2; o >= 1; o >>= 1) m = umin2(m, (uint32_t)__shfl_xor((int)m, o, kWave));
      // a bound of NaN never abandons
      if (alive && __uint_as_float(m) > ubv) alive = false;
    }
    if (!__builtin_amdgcn_ballot_w64(alive && tau0 + CH < nsp)) break;
    // the first row not ended by the chunk's last step: a, b or b + P
    const int tl = t0 + CH - 1;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (te[c] > tl) continue;
      if (teB[c] > tl) {
        row[c] = rowB[c];
        ts[c] = tsB[c];
        te[c] = teB[c];
        sv[c] = __uint_as_float(svBb[c]);
      } else {
        row[c] = rowB[c] + P;
        span(row[c], ts[c], te[c]);
        sv[c] = s_of(row[c]);
      }
    }
  }

  if (a.counters) {
    // one lane per wave adds the wave's counts into its counter stripe
    uint64_t ev = evaluated;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) ev += __shfl_xor(ev, o, kWave);
    const uint64_t ab = __popcll(__builtin_amdgcn_ballot_w64(run && !alive && g == 0));
    if (lane == 0) {
      unsigned long long *cs = counter_stripe(a.counters, blockIdx.x);
      atomicAdd(&cs[kCntEvaluated], (unsigned long long)ev);
      atomicAdd(&cs[kCntComputed], (unsigned long long)(chunks * CH * kWave * NC));
      if (ab) atomicAdd(&cs[kCntAbandoned], (unsigned long long)ab);
    }
  }
  if constexpr (MODE == 2) {
    // Reverse sweep.  The path is the chain of recorded predecessors from
    // (ls-1, lt-1) back to (0, 0); it holds at most one cell per
    // anti-diagonal.  Sweeping the steps backwards in the same lane layout,
    // a cell is on the path when a path cell names it: its own cell of step
    // t+1 (i, j+1) with code 2, the next lane-slot's cell of step t+1 (i+1, j)
    // with code 1, or that lane-slot's cell of step t+2 (i+1, j+1) with code
    // 0.  A path cell emits the bit of its code (bit 0 diagonal, 1 up, 2 left)
    // and the emissions rotate one lane-slot back per step, so the codes are
    // read from LDS once per chunk and the chain costs a few instructions per
    // step, with no memory access on it.  Each step's path cell leaves its
    // lane-slot at the step's halfword of `pslot` (in the series' LDS, no
    // longer read); a second pass turns each path cell and its neighbours on
    // the chain into the row and column ranges.
    constexpr unsigned kNoCell = 0xFFFFu;
    unsigned *pw = reinterpret_cast<unsigned *>(Sl);
    for (int k = g; k < (nsp + 1) / 2; k += G) pw[k] = 0xFFFFFFFFu;
    __syncthreads();
    const uint32_t pslot = lds_addr(Sl);
    // lanes off the path store to a word of their own (9-word stride: 64 banks)
    const uint32_t scratch = lds_addr(lds + GPW * a.lds_stride) + 36u * (uint32_t)lane;
    const uint32_t lane_last = g == G - 1 ? ~0u : 0u;
    const uint32_t half_lo_r = ((lane < 32) != (g == G - 1)) ? ~0u : 0u;  // G = 32 only
    uint32_t own[NC], rcv[NC], rcvp[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) own[c] = rcv[c] = rcvp[c] = 0u;
    const unsigned *cw_l = codes_l;
#pragma unroll 1
    for (int tau0 = nsw - kWfChunk; tau0 >= 0; tau0 -= kWfChunk) {
      const bool mine = tau0 < nsp;
      const int k = mine ? tau0 / kWfChunk : 0;
      uint32_t cw[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const uint32_t w = cw_l[k * P + c * G + g];
        cw[c] = mine ? w : 0u;
        // the path's last cell: named by a virtual cell (ls-1, lt)
        if (tau0 + kWfChunk == nsp && c * G + g == le) own[c] |= 4u;
      }
      // a path cell stores at base + 2 s, the others at scratch + 2 s
      const int32_t to_base = (int32_t)(pslot + 2u * (uint32_t)tau0) - (int32_t)scratch;
#pragma unroll
      for (int s = kWfChunk - 1; s >= 0; --s) {
        uint32_t emit[NC], on_any = 0u, slot = 0u;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          // bit 2 of own, bit 1 of rcv, bit 0 of rcvp (emissions use bits 0-2)
          const uint32_t on = path_named(own[c], rcv[c], rcvp[c]);
          emit[c] = on << ((cw[c] >> (2 * s)) & 3u);
          own[c] = emit[c];
          on_any |= on;
          if (NC > 1) slot = on ? (uint32_t)(c * G + g) : slot;
        }
        const uint32_t at =
            (uint32_t)__mul24((int)opaque(on_any), to_base) + scratch + 2u * (uint32_t)s;
        *(__attribute__((address_space(3))) uint16_t *)(uintptr_t)at =
            (uint16_t)(NC > 1 ? slot : (uint32_t)g);
        uint32_t r[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) r[c] = rot1_back<G>(emit[c]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          // from the next lane-slot: the next lane, or for lane G-1 lane 0 of
          // the next slot
          uint32_t x = NC > 1 ? bit_select(lane_last, r[(c + 1) % NC], r[c]) : r[c];
          if constexpr (G == 32) x = group_fix32(x, half_lo_r);
          rcvp[c] = rcv[c];
          rcv[c] = x;
        }
      }
    }
    __syncthreads();
    // Ranges.  A path cell (i, j) at step t opens its row's range unless the
    // path came from (i, j-1) (same lane-slot at t-1), closes it unless the
    // path goes on to (i, j+1) (same lane-slot at t+1); it opens its column's
    // range unless the path came from (i-1, j) (another lane-slot at t-1), and
    // closes it unless it goes on to (i+1, j).  (0, 0) opens both, the last
    // cell closes both.  The cell's row is the one active row of its
    // lane-slot at step t.
    if (run) {
      const uint16_t *ps = reinterpret_cast<const uint16_t *>(Sl);
      uint16_t *rr16 = reinterpret_cast<uint16_t *>(rr_l);
      uint16_t *cr16 = reinterpret_cast<uint16_t *>(cr_l);
      for (int tau = e + g; tau < nsp; tau += G) {
        const int t = tau - e;
        const unsigned v = ps[tau];
        if (v == kNoCell) continue;
        int lo = (t - r + 1) >> 1;  // first active row of step t
        lo = lo > t - (lt - 1) ? lo : t - (lt - 1);
        lo = lo > 0 ? lo : 0;
        const int i = lo + (((int)v - lo) & (P - 1));
        const int j = t - i;
        const unsigned vp = t >= 1 ? ps[tau - 1] : kNoCell;
        const unsigned vn = t + 1 < ns ? ps[tau + 1] : kNoCell;
        if (vp != v) rr16[2 * i] = (uint16_t)j;
        if (vn != v) rr16[2 * i + 1] = (uint16_t)j;
        if (vp == v || vp == kNoCell) cr16[2 * j] = (uint16_t)i;
        if (vn == v || vn == kNoCell) cr16[2 * j + 1] = (uint16_t)i;
      }
    }
    __syncthreads();
    if (run) {
      unsigned *grr = a.rowrng + v.s_off;
      unsigned *gcr = a.colrng + v.t_off;
      for (int k = g; k < ls; k += G) grr[k] = rr_l[k];
      for (int k = g; k < lt; k += G) gcr[k] = cr_l[k];
    }
  }
  if (!valid) return;
  if (g == le % G) {
    float d;
    if (run) {
      d = fin;
      if (!alive || d > ubv) d = kInf;  // strictly above the bound: abandoned
    } else if (pair_bad) {
      d = qnan;
    } else {
      d = (ls == 0 && lt == 0) ? 0.0f : kInf;
    }
    a.out[p] = d;
    if constexpr (REC) a.status[p] = run ? kWfOk : (pair_bad ? kWfNonFinite : kWfNoPath);
  }
}

// ---------------------------------------------------------------------------
// Backtrack: one pair per wave, from (ls-1, lt-1) to (0, 0), one path cell
// per iteration with the whole wave in lockstep on wave-uniform (scalar)
// state.  The pair's record is copied to LDS in windows of a.win_words words
// (every lane keeps eight loads in flight); when the path enters a chunk, its
// P words are read into registers (lane l holds lane-slot l's word; P above
// 64 reads the word from LDS per cell) and each cell's code is taken with one
// readlane.  Leaving row i closes its column range, leaving column j its row
// range; the ranges are kept in LDS (a.lds_ranges) or stored to memory as
// they close, and copied out coalesced at the end.  The path never leaves the
// matrix: at i = 0 only the left move, at j = 0 only the upward move remains,
// so even a record of non-finite values terminates.
template <int P>
__global__ __launch_bounds__(64) void wf_walk_kernel(WfWalkArgs a) {
  extern __shared__ unsigned wsh[];
  const int WCH = a.win_words / P;  // chunks per window
  const int lane = threadIdx.x;
  const int64_t q = blockIdx.x;
  if (q >= a.nitems) return;
  const int64_t p = a.order ? (int64_t)a.order[q] : q;
  const PairView v = pair_view(a.pairs, p, a.ls, a.lt, a.r, a.rec_words_u);
  if (a.status[p] != kWfOk) return;  // no path or non-finite input: the gradient kernel handles it
  unsigned *win = wsh;
  const bool in_lds = a.lds_ranges != 0;
  unsigned *rr = in_lds ? wsh + a.win_words : a.rowrng + v.s_off;
  unsigned *cr = in_lds ? rr + v.ls : a.colrng + v.t_off;
  const unsigned *chunks = a.rec + v.rec_off;
  const int lead = wf_lead((int)wf_steps(v.ls, v.lt));
  int i = v.ls - 1, j = v.lt - 1;
  int row_hi = j, col_hi = i;
  int w0 = 1 << 30;   // first chunk held in the window
  int held = -1;      // chunk whose words are in `word_l`
  unsigned word_l = 0;
  for (;;) {
    const int t = i + j + lead;  // the step in the record's time (see the forward)
    const int ch = t / kWfChunk;
    if (ch < w0) {
      w0 = ch + 1 - WCH > 0 ? ch + 1 - WCH : 0;
      __syncthreads();
      const unsigned *src = chunks + (int64_t)w0 * P;
      const int nw = (ch + 1 - w0) * P;
      for (int b = 0; b < nw; b += 8 * kWave) {
        unsigned tmp[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int k = b + u * kWave + lane;
          tmp[u] = src[k < nw ? k : 0];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int k = b + u * kWave + lane;
          if (k < nw) win[k] = tmp[u];
        }
      }
      __syncthreads();
      held = -1;
    }
    if (i == 0 && j == 0) break;
    unsigned word;
    if constexpr (P <= kWave) {
      if (ch != held) {
        word_l = win[(ch - w0) * P + (lane < P ? lane : 0)];
        held = ch;
      }
      word = (unsigned)__builtin_amdgcn_readlane((int)word_l, i % P);
    } else {
      word = __builtin_amdgcn_readfirstlane(win[(ch - w0) * P + i % P]);
    }
    unsigned code = (word >> (2 * (t % kWfChunk))) & 3u;
    code = i == 0 ? 2u : (j == 0 ? 1u : code);
    // code 0: diagonal (i-1, j-1), 1: (i-1, j), 2: (i, j-1)
    if (lane == 0) {
      if (code != 2u) rr[i] = (unsigned)j | ((unsigned)row_hi << 16);
      if (code != 1u) cr[j] = (unsigned)i | ((unsigned)col_hi << 16);
    }
    const int ni = code != 2u ? i - 1 : i;
    const int nj = code != 1u ? j - 1 : j;
    if (code != 2u) row_hi = nj;
    if (code != 1u) col_hi = ni;
    i = ni;
    j = nj;
  }
  if (lane == 0) {
    rr[0] = (unsigned)row_hi << 16;
    cr[0] = (unsigned)col_hi << 16;
  }
  if (in_lds) {
    __syncthreads();
    unsigned *grr = a.rowrng + v.s_off;
    unsigned *gcr = a.colrng + v.t_off;
    for (int k = lane; k < v.ls; k += kWave) grr[k] = rr[k];
    for (int k = lane; k < v.lt; k += kWave) gcr[k] = cr[k];
  }
}

// ---------------------------------------------------------------------------
// Gradients: one workgroup per pair; thread k handles S positions k, k+256, ...
// and T positions likewise.  Ranges are clamped to the matrix.
__global__ __launch_bounds__(256) void wf_grad_kernel(WfGradArgs a) {
  const int64_t p = blockIdx.x;
  if (p >= a.npairs) return;
  const PairView v = pair_view(a.pairs, p, a.ls, a.lt, 0, 0);
  const unsigned st = a.status[p];
  const float *Sp = a.S + v.s_off;
  const float *Tp = a.T + v.t_off;
  float *gS = a.gS + v.s_off;
  float *gT = a.gT + v.t_off;
  const float fill = st == kWfNonFinite ? __builtin_nanf("") : 0.0f;
  if (st != kWfOk) {
    for (int k = threadIdx.x; k < v.ls; k += blockDim.x) gS[k] = fill;
    for (int k = threadIdx.x; k < v.lt; k += blockDim.x) gT[k] = fill;
    return;
  }
  // both series staged in LDS (coalesced), then every range sum reads LDS
  extern __shared__ float gsh[];
  float *Sl = gsh, *Tl = gsh + v.ls;
  bool unused = false;
  stage_series<256>(Sp, Sl, v.ls, threadIdx.x, unused);
  stage_series<256>(Tp, Tl, v.lt, threadIdx.x, unused);
  __syncthreads();
  const float g2 = 2.0f * a.gout[p];
  const unsigned *rr = a.rowrng + v.s_off;
  const unsigned *cr = a.colrng + v.t_off;
  for (int i = threadIdx.x; i < v.ls; i += blockDim.x) {
    const unsigned w = rr[i];
    const int lo = (int)(w & 0xffffu);
    int hi = (int)(w >> 16);
    hi = hi < v.lt - 1 ? hi : v.lt - 1;
    const float s = Sl[i];
    float acc = 0.0f;
    for (int jj = lo; jj <= hi; ++jj) acc += s - Tl[jj];
    gS[i] = g2 * acc;
  }
  for (int j = threadIdx.x; j < v.lt; j += blockDim.x) {
    const unsigned w = cr[j];
    const int lo = (int)(w & 0xffffu);
    int hi = (int)(w >> 16);
    hi = hi < v.ls - 1 ? hi : v.ls - 1;
    const float tv = Tl[j];
    float acc = 0.0f;
    for (int ii = lo; ii <= hi; ++ii) acc += Sl[ii] - tv;
    gT[j] = -g2 * acc;
  }
}

// ---------------------------------------------------------------------------
// DBA: chunk k of 64 pairs, point i of the barycentre: the sum (float64) and
// the count of the values X[p][j], j in the path range of row i of pair p.

__global__ __launch_bounds__(256) void wf_dba_partial_kernel(const float *X, int64_t n, int len,
                                                             int lb, const unsigned *rowrng,
                                                             const unsigned *status, double *psum,
                                                             double *pcnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = blockIdx.y;
  if (i >= lb) return;
  double s = 0.0, c = 0.0;
  const int64_t p1 = (k + 1) * kDbaPairs < n ? (k + 1) * kDbaPairs : n;
  for (int64_t p = k * kDbaPairs; p < p1; ++p) {
    if (status[p] != kWfOk) continue;
    const unsigned w = rowrng[p * lb + i];
    const int lo = (int)(w & 0xffffu);
    int hi = (int)(w >> 16);
    hi = hi < len - 1 ? hi : len - 1;
    const float *x = X + p * len;
    for (int j = lo; j <= hi; ++j) s += (double)x[j];
    c += (double)(hi - lo + 1);
  }
  psum[k * lb + i] = s;
  pcnt[k * lb + i] = c;
}

__global__ __launch_bounds__(256) void wf_dba_total_kernel(const double *psum, const double *pcnt,
                                                           int64_t nchunk, int lb, float *out_B,
                                                           float *out_count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= lb) return;
  double s = 0.0, c = 0.0;
  for (int64_t k = 0; k < nchunk; ++k) {
    s += psum[k * lb + i];
    c += pcnt[k * lb + i];
  }
  out_B[i] = c > 0.0 ? (float)(s / c) : __builtin_nanf("");
  if (out_count) out_count[i] = (float)c;
}

// ---------------------------------------------------------------------------
// launchers

template <int G, int NC, int MODE>
static hipError_t launch_fwd_t(const WfArgs &a, hipStream_t st) {
  constexpr int GPW = kWave / G;
  const int64_t nb = (a.nitems + GPW - 1) / GPW;
  if (nb <= 0) return hipSuccess;
  // mode 2: kWfScratchWords after the groups' regions
  const size_t lds = sizeof(float) * ((size_t)a.lds_stride * GPW + (MODE == 2 ? kWfScratchWords : 0));
  hipLaunchKernelGGL((wf_fwd_kernel<G, NC, MODE>), dim3((unsigned)nb), dim3(kWave), lds, st, a);
  return hipGetLastError();
}

typedef hipError_t (*WfFwdFn)(const WfArgs &, hipStream_t);
#define EAPDTW_WF_MODE(M)                                                            \
  {&launch_fwd_t<16, 1, M>, &launch_fwd_t<16, 2, M>, &launch_fwd_t<32, 1, M>,      \
   &launch_fwd_t<16, 4, M>, &launch_fwd_t<32, 2, M>, &launch_fwd_t<64, 1, M>,      \
   &launch_fwd_t<64, 2, M>, &launch_fwd_t<64, 4, M>, &launch_fwd_t<64, 8, M>}
static const WfFwdFn kWfFwd[3][kWfClasses] = {EAPDTW_WF_MODE(0), EAPDTW_WF_MODE(1),
                                              EAPDTW_WF_MODE(2)};
#undef EAPDTW_WF_MODE

hipError_t launch_wf_fwd(int cls, int mode, const WfArgs &a, hipStream_t st) {
  if (cls < 0 || cls >= kWfClasses || mode < 0 || mode > 2) return hipErrorInvalidValue;
  if (a.lds_stride * (kWave / kWfG[cls]) > kWfLdsFloats) return hipErrorInvalidValue;
  return kWfFwd[mode][cls](a, st);
}

template <int P>
static hipError_t launch_walk_t(WfWalkArgs a, hipStream_t st) {
  if (a.nitems <= 0) return hipSuccess;
  // window: the longest record of the launch, at most kWalkWindow words
  int64_t win = (int64_t)a.max_chunks * P;
  if (win > kWalkWindow) win = kWalkWindow / P * P;
  a.win_words = (int)win;
  // ranges in LDS when they fit beside the window
  a.lds_ranges = (win + a.max_ranges) * (int64_t)sizeof(unsigned) <= kWalkLds ? 1 : 0;
  const size_t lds = sizeof(unsigned) * (size_t)(win + (a.lds_ranges ? a.max_ranges : 0));
  hipLaunchKernelGGL((wf_walk_kernel<P>), dim3((unsigned)a.nitems), dim3(kWave), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_wf_walk(int P, const WfWalkArgs &a, hipStream_t st) {
  if (a.max_chunks <= 0) return hipSuccess;
  switch (P) {
    case 16: return launch_walk_t<16>(a, st);
    case 32: return launch_walk_t<32>(a, st);
    case 64: return launch_walk_t<64>(a, st);
    case 128: return launch_walk_t<128>(a, st);
    case 256: return launch_walk_t<256>(a, st);
    case 512: return launch_walk_t<512>(a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_wf_grad(const WfGradArgs &a, hipStream_t st) {
  if (a.npairs <= 0) return hipSuccess;
  const int mls = a.pairs ? a.max_ls : a.ls, mlt = a.pairs ? a.max_lt : a.lt;
  if (mls < 0 || mlt < 0 || mls > kWfMaxLen || mlt > kWfMaxLen) return hipErrorInvalidValue;
  const size_t lds = sizeof(float) * (size_t)(mls + mlt);
  hipLaunchKernelGGL(wf_grad_kernel, dim3((unsigned)a.npairs), dim3(256), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_wf_dba(const float *X, int64_t n, int len, int lb, const unsigned *rowrng,
                         const unsigned *status, double *partial_sum, double *partial_cnt,
                         int64_t nchunk, float *out_B, float *out_count, hipStream_t st) {
  if (n <= 0 || lb <= 0) return hipSuccess;
  const unsigned bx = (unsigned)((lb + 255) / 256);
  hipLaunchKernelGGL(wf_dba_partial_kernel, dim3(bx, (unsigned)nchunk), dim3(256), 0, st, X, n,
                     len, lb, rowrng, status, partial_sum, partial_cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(wf_dba_total_kernel, dim3(bx), dim3(256), 0, st, partial_sum, partial_cnt,
                     nchunk, lb, out_B, out_count);
  return hipGetLastError();
}

}  // namespace eapdtw
