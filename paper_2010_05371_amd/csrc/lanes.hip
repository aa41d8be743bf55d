// lanes.hip -- band search with lane refill.
//
// The wave-synchronous band kernel keeps a lane whose candidate was abandoned
// idle until every lane of its wave is done, so about half of its lanes'
// cells are wasted on C2.  Here a wave owns a range of kLaneBlocks x 64
// consecutive candidates: the series stretch they read, their window
// statistics and the padded query are staged in LDS once, and a lane whose
// candidate is abandoned (Section 2.2) or finished takes the next candidate
// of the range at row 0.  Lanes therefore sit at different rows: each lane
// reads its query columns from LDS (two 16-byte reads per 8 columns; rows
// advance in groups of 4, so a lane's column index stays a multiple of 4)
// and its row values from the staged stretch.  The cells are the band
// kernel's (same operations, same bits); only the scheduling differs.
#include "band.h"
#include "dispatch.h"

namespace eapdtw {

namespace {

constexpr int kLaneBlocks = 8;
constexpr int kLaneCands = kLaneBlocks * kWave;
constexpr int kLaneU = 4;
constexpr int kLaneCH = 8;

// The staged stretch seen as the series: position p of the series is
// base[p - k0].
struct StagedSeries {
  const float *base;
  int64_t k0;
  __device__ float operator[](int64_t p) const { return base[p - k0]; }
};

__device__ __forceinline__ int round4(int v) { return (v + 3) & ~3; }

template <int R>
struct LaneLayout {
  static constexpr int W = 2 * R + 1;
  static constexpr int NS = W + kLaneU - 1;
  static constexpr int NCH = (NS + kLaneCH - 1) / kLaneCH;
  // floats of the padded query: columns i + s for i <= m - 4, s < NCH * 8
  __host__ __device__ static int lq(int m) { return (m + NCH * kLaneCH + 7) & ~3; }
  __host__ __device__ static int lx(int m) { return (kLaneCands + m + 3) & ~3; }
  __host__ __device__ static int floats(int m) { return lq(m) + lx(m) + 3 * kLaneCands; }
};

template <int R>
__global__ __launch_bounds__(64) void nn_lane_kernel(NNArgs a) {
  using L = LaneLayout<R>;
  constexpr int W = L::W;
  constexpr int U = kLaneU;
  constexpr int NS = L::NS;
  constexpr int CH = kLaneCH;
  constexpr int NCH = L::NCH;
  extern __shared__ __attribute__((aligned(16))) float lds[];
  const int lane = threadIdx.x;
  const int m = a.m;
  const int64_t K = a.k_end;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t k0 = blk * kLaneCands;
  if (k0 >= K) return;
  const int range_n = (int)(K - k0 < kLaneCands ? K - k0 : kLaneCands);
  float *lq = lds;                     // lq[i + s] = z(query)[i + s - R], +inf outside
  float *lx = lds + L::lq(m);          // lx[t] = series[k0 + t]
  float *lmh = lx + L::lx(m);          // per candidate: mean (hi, lo), inverse deviation
  float *lml = lmh + kLaneCands;
  float *linv = lml + kLaneCands;

  // staging: query and series stretch (loads batched eight per lane)
  {
    const float *qz = a.qpad + kColPad - R;
    const int nq = L::lq(m), nx = L::lx(m);
    const int64_t lim = a.n - 1 - k0;
    for (int t0 = 0; t0 < nq + nx; t0 += 8 * kWave) {
      float tmp[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int t = t0 + j * kWave + lane;
        if (t < nq) tmp[j] = qz[t];
        else tmp[j] = a.x[k0 + (t - nq < lim ? t - nq : lim)];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int t = t0 + j * kWave + lane;
        if (t < nq + nx) lds[t] = tmp[j];
      }
    }
  }
  __syncthreads();
  // window statistics of the range's candidates, from the staged stretch
  for (int j = 0; j < kLaneBlocks && j * kWave < range_n; ++j) {
    double mean, sd;
    wave_window_stats(StagedSeries{lx, k0}, a.n, m, k0 + j * kWave, lane, mean, sd);
    float mh, ml, iv;
    znorm_params(mean, sd, mh, ml, iv);
    lmh[j * kWave + lane] = mh;
    lml[j * kWave + lane] = ml;
    linv[j * kWave + lane] = iv;
  }
  __syncthreads();

  float ub = load_bsf_dist(a.bsf) + 0.0f;
  if (a.bsf_init) ub = fminf(ub, best_dist(*a.bsf_init));
  const int ci = a.check_interval > 0 ? a.check_interval : auto_check_interval<R, U>();
  int since = 0;
  bool pending = false;
  unsigned long long bpend = 0;

  float v[W];
#pragma unroll
  for (int d = 0; d < W; ++d) v[d] = kInf;
  int c = 0, i = 0;           // the lane's candidate (range index) and next row
  bool busy = false;
  float mu_hi = 0.f, mu_lo = 0.f, inv = 0.f;
  float rv_next[U];
#pragma unroll
  for (int u = 0; u < U; ++u) rv_next[u] = 0.f;
  int next_c = 0;             // next candidate of the range to hand out
  uint32_t eval = 0;          // in-matrix cells of this lane's live groups
  uint64_t computed = 0, aband = 0;

  for (;;) {
    // hand the range's next candidates to idle lanes
    const uint64_t idle = __builtin_amdgcn_ballot_w64(!busy);
    if (idle && next_c < range_n) {
      const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
      const int avail = range_n - next_c;
      const bool fresh = !busy && rank < avail;
      if (fresh) {
        c = next_c + rank;
        i = 0;
        busy = ub >= 0.0f;
        mu_hi = lmh[c];
        mu_lo = lml[c];
        inv = linv[c];
#pragma unroll
        for (int u = 0; u < U; ++u) rv_next[u] = lx[c + u];
      }
#pragma unroll
      for (int d = 0; d < W; ++d) v[d] = fresh ? (d == R ? 0.0f : kInf) : v[d];
      const int n_idle = __popcll(idle);
      next_c += n_idle < avail ? n_idle : avail;
    }
    // no busy lane after the hand-out: the range is done (a negative bound,
    // which abandons every candidate, also ends here)
    if (!__builtin_amdgcn_ballot_w64(busy)) break;
    if (!pending) {
      bpend = __hip_atomic_load(a.bsf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      pending = true;
      since = 0;
    }
    // one group of U rows for every busy lane
    float rv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) rv[u] = znorm_value(rv_next[u], mu_hi, mu_lo, inv);
    if (i + U < m) {
#pragma unroll
      for (int u = 0; u < U; ++u) rv_next[u] = lx[c + i + U + u];
    }
    {
      const float4 *qc = reinterpret_cast<const float4 *>(lq + i);
      float4 cur0 = qc[0], cur1 = qc[1];
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        float4 nx0, nx1;
        if (ch + 1 < NCH) {
          // an opaque address keeps these loads one chunk ahead, not hoisted
          const float4 *qn = qc + 2 * (ch + 1);
          asm volatile("" : "+v"(qn));
          nx0 = qn[0];
          nx1 = qn[1];
        }
        __builtin_amdgcn_sched_barrier(0);
        const float col[CH] = {cur0.x, cur0.y, cur0.z, cur0.w, cur1.x, cur1.y, cur1.z, cur1.w};
#pragma unroll
        for (int t = 0; t < CH; ++t) {
          const int s = ch * CH + t;
          if (s >= NS) continue;
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int d = s - u;
            if (d < 0 || d >= W) continue;
            const float left = (d > 0) ? v[d > 0 ? d - 1 : 0] : kInf;
            const float top = (d < W - 1) ? v[d < W - 1 ? d + 1 : 0] : kInf;
            const float diff = col[t] - rv[u];
            v[d] = __builtin_fmaf(diff, diff, fmin3(left, top, v[d]));
          }
        }
        // pin this chunk's cells before the next chunk's loads are issued
#pragma unroll
        for (int d = 0; d < W; ++d) {
          if (d + U - 1 < ch * CH || d > ch * CH + CH - 1) continue;
          asm volatile("" : "+v"(v[d]));
        }
        __builtin_amdgcn_sched_barrier(0);
        if (ch + 1 < NCH) {
          cur0 = nx0;
          cur1 = nx1;
        }
      }
    }
    if (busy) eval += (uint32_t)rows_cells<U>(i, m, R);
    computed += (uint64_t)U * W * kWave;
    i += U;
    if (++since >= ci) {
      ub = fminf(ub, best_dist(bpend));
      pending = false;
    }
    // abandon (Section 2.2): no cell of the last row within the bound
    uint32_t mn = cell_bits(v[0]);
#pragma unroll
    for (int d = 1; d < W; d += 2) {
      if (d + 1 < W) mn = umin3(mn, cell_bits(v[d]), cell_bits(v[d + 1 < W ? d + 1 : 0]));
      else mn = min(mn, cell_bits(v[d]));
    }
    const bool live = busy && mn <= cell_bits(ub);
    const bool done = live && i >= m;
    if (busy && !live) ++aband;
    if (done) {
      const float dist = v[R];
      if (dist <= ub) {
        atomicMin(a.bsf, pack_best(dist, (uint32_t)(k0 + c)));
        ub = dist;
      } else {
        ++aband;
      }
    }
    busy = live && !done;
  }

  if (a.counters) {
    uint64_t ev = eval;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) ev += __shfl_xor(ev, o, kWave);
    uint64_t ab = aband;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) ab += __shfl_xor(ab, o, kWave);
    if (lane == 0) {
      unsigned long long *cc = counter_stripe(a.counters, blockIdx.x);
      atomicAdd(&cc[kCntEvaluated], (unsigned long long)ev);
      atomicAdd(&cc[kCntComputed], (unsigned long long)computed);
      atomicAdd(&cc[kCntAbandoned], (unsigned long long)ab);
    }
  }
}

template <int R>
hipError_t launch_lane(const NNArgs &a, hipStream_t st) {
  const int64_t K = a.k_end;
  const int64_t nwaves = (K + kLaneCands - 1) / kLaneCands;
  const size_t sh = sizeof(float) * LaneLayout<R>::floats(a.m);
  hipLaunchKernelGGL(nn_lane_kernel<R>, dim3((unsigned)nwaves), dim3(kWave), sh, st, a);
  return hipGetLastError();
}

template <int... Rs>
hipError_t lane_dispatch(int r, const NNArgs &a, hipStream_t st, std::integer_sequence<int, Rs...>) {
  hipError_t e = hipErrorInvalidValue;
  ((r == Rs + 1 ? (e = launch_lane<Rs + 1>(a, st), 0) : 0), ...);
  return e;
}

}  // namespace

bool lane_search_supported(int r, int m) {
  return r >= 1 && r <= kBandRMax && m >= 4 && m % kLaneU == 0 && m <= kLaneMaxM;
}

hipError_t launch_lane_search(int r, const NNArgs &a, hipStream_t st) {
  if (!lane_search_supported(r, a.m) || a.k_begin != 0) return hipErrorInvalidValue;
  if (a.k_end <= 0) return hipSuccess;
  return lane_dispatch(r, a, st, std::make_integer_sequence<int, kBandRMax>{});
}

}  // namespace eapdtw
