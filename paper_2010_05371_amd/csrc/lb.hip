// lb.hip -- lower bounds in front of the search's DTW (Section 2.2: a cheap
// lower bound strictly above the bound skips the candidate; Section 5: the
// search experiments keep the UCR Suite's LB_Kim and LB_Keogh with the
// query's and with the candidate's envelope).
//
//  * envelope_kernel: running max / min under window r of the raw series and
//    of z(query) (the window clipped to the series);
//  * lb_pass_kernel: per candidate, LB_Kim, then LB_Keogh against the query
//    envelope, then LB_Keogh of z(query) against the candidate's envelope
//    (the series envelope z-normalised with the candidate's mean and sigma:
//    normalisation is increasing, so it maps the max / min of the raw values to
//    those of the normalised ones; optional in a search).  Each bound, lowered
//    by kLbMargin, is compared with the bound in force; candidates that pass go
//    to a list (offset, normalisation constants, bounds) in the order of their
//    waves' arrival, for the list mode of the band kernel.
#include "band.h"
#include "dispatch.h"

namespace eapdtw {

namespace {

constexpr int kEnvTile = 1024;   // outputs per envelope workgroup
constexpr int kEnvThreads = 256;
constexpr int kLbBlock = 16;     // rows between abandon checks of the LB_Keogh sums

// Block b < nbx: series positions [b kEnvTile, ...); the rest: z(query).
// Positions outside the array are replaced by the nearest end value, which
// leaves the max / min over the clipped window unchanged.
__global__ __launch_bounds__(kEnvThreads) void envelope_kernel(const float *__restrict__ x,
                                                               int64_t n,
                                                               const float *__restrict__ qz, int m,
                                                               int r, float *ux, float *lx,
                                                               float *uq, float *lq, int64_t nbx) {
  extern __shared__ float tile[];  // kEnvTile + 2 r values
  const bool isq = (int64_t)blockIdx.x >= nbx;
  const float *__restrict__ src = isq ? qz : x;
  const int64_t len = isq ? (int64_t)m : n;
  float *U = isq ? uq : ux;
  float *L = isq ? lq : lx;
  const int64_t t0 = (isq ? (int64_t)blockIdx.x - nbx : (int64_t)blockIdx.x) * kEnvTile;
  for (int i = threadIdx.x; i < kEnvTile + 2 * r; i += kEnvThreads) {
    int64_t g = t0 - r + i;
    g = g < 0 ? 0 : (g > len - 1 ? len - 1 : g);
    tile[i] = src[g];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kEnvTile; i += kEnvThreads) {
    const int64_t g = t0 + i;
    if (g >= len) break;
    float u = tile[i], l = tile[i];
    for (int s = 1; s <= 2 * r; ++s) {
      u = fmaxf(u, tile[i + s]);
      l = fminf(l, tile[i + s]);
    }
    U[g] = u;
    L[g] = l;
  }
}

__device__ __forceinline__ float sq(float a, float b) {
  const float d = a - b;
  return d * d;
}

// Lane l of the workgroup owns candidate kb + l (kb = k_begin + 64 b).
template <int MODE>
__global__ __launch_bounds__(64) void lb_pass_kernel(LBArgs a) {
  const int lane = threadIdx.x;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t kb = a.k_begin + blk * kWave;
  if (kb >= a.k_end) return;
  const int64_t k = kb + lane;
  const bool active = k < a.k_end;
  const int64_t kc = active ? k : a.k_end - 1;
  const int m = a.m;

  double mean, sd;
  wave_window_stats(a.x, a.n, m, kb, lane, mean, sd);
  float mu_hi, mu_lo, inv;
  znorm_params(mean, sd, mu_hi, mu_lo, inv);

  float ub = kInf;
  if (MODE == 0) {
    ub = load_bsf_dist(a.bsf);
    if (a.bsf_init) ub = fminf(ub, best_dist(*a.bsf_init));
  } else if (MODE == 1) {
    ub = a.fixed_ub;
  }
  ub += 0.0f;
  // a bound b skips the candidate when b (1 - margin) > ub
  auto passes = [&](float b) { return MODE == 2 || !(b * (1.0f - kLbMargin) > ub); };

  // LB_Kim: levels 1..L from each end, L = min(3, m / 2); level a takes the
  // cheapest cell with max(i, j) = a - 1 (front) and with min(i, j) = m - a
  // (back); i over the query, j over the candidate.
  float kim = 0.0f;
  {
    const float *__restrict__ xc = a.x + kc;
    const int L = m / 2 < 3 ? m / 2 : 3;
    float cf[3], cb[3], qf[3], qb[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int f = j < m ? j : m - 1, b = m - 1 - j >= 0 ? m - 1 - j : 0;
      cf[j] = znorm_value(xc[f], mu_hi, mu_lo, inv);
      cb[j] = znorm_value(xc[b], mu_hi, mu_lo, inv);
      qf[j] = a.qz[f];
      qb[j] = a.qz[b];
    }
    if (L >= 1) kim = sq(qf[0], cf[0]) + sq(qb[0], cb[0]);
    if (L >= 2) {
      kim += fminf(fminf(sq(qf[0], cf[1]), sq(qf[1], cf[0])), sq(qf[1], cf[1]));
      kim += fminf(fminf(sq(qb[0], cb[1]), sq(qb[1], cb[0])), sq(qb[1], cb[1]));
    }
    if (L >= 3) {
      kim += fminf(fminf(fminf(sq(qf[0], cf[2]), sq(qf[1], cf[2])), fminf(sq(qf[2], cf[2]),
                   sq(qf[2], cf[1]))), sq(qf[2], cf[0]));
      kim += fminf(fminf(fminf(sq(qb[0], cb[2]), sq(qb[1], cb[2])), fminf(sq(qb[2], cb[2]),
                   sq(qb[2], cb[1]))), sq(qb[2], cb[0]));
    }
  }
  bool alive = active && ub >= 0.0f && passes(kim);
  const bool after_kim = alive;

  // One LDS-staged sweep over the candidate's m positions per bound: the
  // 64 + rows - 1 series values of the wave and the rows' per-position
  // values (envelope or query) are copied once per stretch of kStageRows;
  // the per-position values are read four at a time (one ds_read_b128).
  __shared__ float s0[kWave + kStageRows - 1];
  __shared__ float s1[kWave + kStageRows - 1];
  __shared__ __attribute__((aligned(16))) float s2[kStageRows];
  __shared__ __attribute__((aligned(16))) float s3[kStageRows];

  // LB_Keogh of z(c) against the query envelope
  float eq = 0.0f;
  bool run = wave_any(MODE == 2 ? active : alive);
  for (int base = 0; base < m && run; base += kStageRows) {
    const int rows = m - base < kStageRows ? m - base : kStageRows;
    __syncthreads();
    stage_copy<kWave + kStageRows - 1>(s0, a.x + kb + base, a.n - 1 - (kb + base), lane);
    stage_copy<kStageRows>(s2, a.uq + base, m - 1 - base, lane);
    stage_copy<kStageRows>(s3, a.lq + base, m - 1 - base, lane);
    __syncthreads();
    for (int i = 0; i < rows && run; i += kLbBlock) {
      const int nr = rows - i < kLbBlock ? rows - i : kLbBlock;
      if (nr == kLbBlock) {
#pragma unroll
        for (int t = 0; t < kLbBlock; t += 4) {
          const float4 u4 = *reinterpret_cast<const float4 *>(&s2[i + t]);
          const float4 l4 = *reinterpret_cast<const float4 *>(&s3[i + t]);
          const float uv[4] = {u4.x, u4.y, u4.z, u4.w}, lv[4] = {l4.x, l4.y, l4.z, l4.w};
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float z = znorm_value(s0[lane + i + t + j], mu_hi, mu_lo, inv);
            const float d = z - __builtin_amdgcn_fmed3f(z, lv[j], uv[j]);
            eq = __builtin_fmaf(d, d, eq);
          }
        }
      } else {
        for (int t = 0; t < nr; ++t) {
          const float z = znorm_value(s0[lane + i + t], mu_hi, mu_lo, inv);
          const float d = z - __builtin_amdgcn_fmed3f(z, s3[i + t], s2[i + t]);
          eq = __builtin_fmaf(d, d, eq);
        }
      }
      if (MODE != 2) {
        alive = alive && passes(eq);
        run = wave_any(alive);
      }
    }
  }
  const bool after_eq = alive;

  // LB_Keogh of z(query) against the candidate's envelope (always for the
  // bounds-only mode, on request otherwise: a wave runs it whenever one of
  // its 64 lanes is still alive, which costs about as much as the first
  // LB_Keogh for the few candidates it removes)
  float ec = 0.0f;
  run = (MODE == 2 || a.use_ec) && wave_any(MODE == 2 ? active : alive);
  for (int base = 0; base < m && run; base += kStageRows) {
    const int rows = m - base < kStageRows ? m - base : kStageRows;
    __syncthreads();
    stage_copy<kWave + kStageRows - 1>(s0, a.ux + kb + base, a.n - 1 - (kb + base), lane);
    stage_copy<kWave + kStageRows - 1>(s1, a.lx + kb + base, a.n - 1 - (kb + base), lane);
    stage_copy<kStageRows>(s2, a.qz + base, m - 1 - base, lane);
    __syncthreads();
    for (int i = 0; i < rows && run; i += kLbBlock) {
      const int nr = rows - i < kLbBlock ? rows - i : kLbBlock;
      for (int t = 0; t < nr; ++t) {
        const float hi = znorm_value(s0[lane + i + t], mu_hi, mu_lo, inv);
        const float lo = znorm_value(s1[lane + i + t], mu_hi, mu_lo, inv);
        const float q = s2[i + t];
        const float d = q - __builtin_amdgcn_fmed3f(q, lo, hi);
        ec = __builtin_fmaf(d, d, ec);
      }
      if (MODE != 2) {
        alive = alive && passes(ec);
        run = wave_any(alive);
      }
    }
  }

  if (MODE == 2) {
    if (active) {
      a.out_kim[k - a.k_begin] = kim;
      a.out_eq[k - a.k_begin] = eq;
      a.out_ec[k - a.k_begin] = ec;
    }
    return;
  }
  if (MODE == 1 && active && !alive) a.dists[k - a.k_begin] = kInf;
  // append the survivors: one atomic per wave reserves their slots
  const unsigned long long mask = __builtin_amdgcn_ballot_w64(alive);
  if (mask) {
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(a.list_n, (unsigned long long)__popcll(mask));
    base = __shfl(base, 0, kWave);
    if (alive) {
      const unsigned pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
      const int64_t e = (int64_t)base + pos;
      a.list_k[e] = (uint32_t)k;
      a.list_mh[e] = mu_hi;
      a.list_ml[e] = mu_lo;
      a.list_inv[e] = inv;
      a.list_lbq[e] = eq;
      a.list_lbmax[e] = fmaxf(fmaxf(kim, eq), ec);
    }
  }
  if (a.counters) {
    const uint64_t nk = (uint64_t)__popcll(__builtin_amdgcn_ballot_w64(active && !after_kim));
    const uint64_t ne = (uint64_t)__popcll(__builtin_amdgcn_ballot_w64(after_kim && !after_eq));
    const uint64_t nc = (uint64_t)__popcll(__builtin_amdgcn_ballot_w64(after_eq && !alive));
    if (lane == 0) {
      unsigned long long *c = counter_stripe(a.counters, blockIdx.x);
      atomicAdd(&c[kCntLbKim], (unsigned long long)nk);
      atomicAdd(&c[kCntLbEq], (unsigned long long)ne);
      atomicAdd(&c[kCntLbEc], (unsigned long long)nc);
    }
  }
}

}  // namespace

hipError_t launch_envelopes(const float *x, int64_t n, const float *qz, int m, int r, float *ux,
                            float *lx, float *uq, float *lq, hipStream_t st) {
  if (r < 0 || r > kEnvMaxR) return hipErrorInvalidValue;
  const int64_t nbx = (n + kEnvTile - 1) / kEnvTile;
  const int64_t nbq = ((int64_t)m + kEnvTile - 1) / kEnvTile;
  const size_t lds = sizeof(float) * (size_t)(kEnvTile + 2 * r);
  hipLaunchKernelGGL(envelope_kernel, dim3((unsigned)(nbx + nbq)), dim3(kEnvThreads), lds, st, x,
                     n, qz, m, r, ux, lx, uq, lq, nbx);
  return hipGetLastError();
}

hipError_t launch_lb_pass(const LBArgs &a, hipStream_t st) {
  const int64_t nblk = (a.k_end - a.k_begin + kWave - 1) / kWave;
  if (nblk <= 0) return hipSuccess;
  const dim3 grid((unsigned)nblk), block(kWave);
  switch (a.mode) {
    case 0: hipLaunchKernelGGL(lb_pass_kernel<0>, grid, block, 0, st, a); break;
    case 1: hipLaunchKernelGGL(lb_pass_kernel<1>, grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL(lb_pass_kernel<2>, grid, block, 0, st, a); break;
  }
  return hipGetLastError();
}

}  // namespace eapdtw
