// bwd.hip -- backward of the differentiable DTW batch (gfx950).
//
// DTW is the cost of the optimal warping path (Section 2), a sum of
// (S(i)-T(j))^2 over the path cells, so with the path fixed
//   dD/dS(i) =  sum over path cells (i,j) of 2 (S(i) - T(j)),
//   dD/dT(j) = -sum over path cells (i,j) of 2 (S(i) - T(j)).
//
// The forward (pair_band_kernel with checkpoints) keeps the band state every
// kBwdBlock rows.  Here one lane per pair walks the blocks from the last to
// the first: it restores the block's starting band from the checkpoint,
// recomputes the block's rows recording for every cell which predecessor gave
// the minimum (2 bits in LDS; ties: diagonal, then (i-1,j), then (i,j-1)), and
// backtracks the optimal path through the block.  Because the path is
// monotone, its cells in one row (column) form one contiguous column (row)
// range; the backtrack records those ranges and a second, fully coalesced
// kernel turns them into the two gradients.  The l_S x l_T matrix is never
// stored.
#include "band.h"
#include "bwd.h"
#include "dispatch.h"

namespace eapdtw {

// Recomputes one group of U rows (block rows u0..u0+U-1) exactly like
// sweep_group (same operations, so the values equal the forward's bit for
// bit) and records the argmin code of every cell into the lane's LDS words.
template <int R, int U>
__device__ __forceinline__ void sweep_group_dirs(float (&v)[2 * R + 1], const float (&rv)[U],
                                                 Cols<const float *> cs, unsigned *lds_row) {
  constexpr int W = 2 * R + 1;
  constexpr int WPR = (W + 15) / 16;  // words per block row
  constexpr int NS = W + U - 1;
  constexpr int CH = kColChunk;
  constexpr int NCH = (NS + CH - 1) / CH;
  const int64_t stride = cs.stride;
  unsigned words[U][WPR];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int w = 0; w < WPR; ++w) words[u][w] = 0u;
  float cur[CH];
  {
    const float *p0 = opaque(cs.base);
#pragma unroll
    for (int t = 0; t < CH; ++t) cur[t] = (t < NS) ? p0[t * stride + cs.lane_off] : 0.0f;
  }
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    float nxt[CH];
    if (c + 1 < NCH) {
      const float *pn = opaque(cs.base + (int64_t)(c + 1) * CH * stride);
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
        const float diag = v[d];
        const float diff = cv - rv[u];
        v[d] = __builtin_fmaf(diff, diff, fmin3(left, top, diag));
        // 0: diagonal, 1: top (i-1,j), 2: left (i,j-1); ties in that order
        const unsigned code = (diag <= fminf(top, left)) ? 0u : ((top <= left) ? 1u : 2u);
        words[u][d / 16] |= code << (2 * (d % 16));
      }
    }
#pragma unroll
    for (int d = 0; d < W; ++d) {
      if (d + U - 1 < c * CH || d > c * CH + CH - 1) continue;
      asm volatile("" : "+v"(v[d]));
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int w = 0; w < WPR; ++w) asm volatile("" : "+v"(words[u][w]));
    __builtin_amdgcn_sched_barrier(0);
    if (c + 1 < NCH) {
#pragma unroll
      for (int t = 0; t < CH; ++t) cur[t] = nxt[t];
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int w = 0; w < WPR; ++w) lds_row[(u * WPR + w) * kWave] = words[u][w];
}

template <int R>
__global__ __launch_bounds__(64) void dtw_bwd_kernel(BwdArgs a) {
  constexpr int W = 2 * R + 1;
  constexpr int WPR = (W + 15) / 16;
  constexpr int K = kBwdBlock;
  constexpr int U = 4;
  static_assert(K % U == 0, "block must hold whole row groups");
  extern __shared__ unsigned lds[];
  const int lane = threadIdx.x;
  unsigned *lds_lane = lds + lane;  // word w of the lane at lds_lane[w * 64]
  const int64_t p = (int64_t)blockIdx.x * kWave + lane;
  const bool active = p < a.npairs;
  const int64_t pc = active ? p : a.npairs - 1;
  const int64_t ld = a.ld;
  const int L = a.len;
  const float *rows = a.rowsT + pc;
  const float *cols = a.colsT + (int64_t)kColPad * ld + pc;
  const float *colu = a.colsT + (int64_t)kColPad * ld;  // wave-uniform column base
  unsigned *rowrng = a.rowrng + pc * L;
  unsigned *colrng = a.colrng + pc * L;

  // equal lengths always admit a path; a distance array (if given) can mark
  // pairs to skip
  const float dist = a.dist ? a.dist[pc] : 0.0f;
  bool done = !active || !(dist < kInf);
  // path position (0-based) and the open row/column ranges
  int i = L - 1, j = L - 1;
  int row_hi = j, col_hi = i;
  const int nb = (L + K - 1) / K;
  for (int b = nb - 1; b >= 0; --b) {
    if (!wave_any(!done)) break;
    const int r0 = b * K;
    const int r1 = (r0 + K < L) ? r0 + K : L;
    float v[W];
    if (b == 0) {
#pragma unroll
      for (int d = 0; d < W; ++d) v[d] = kInf;
      v[R] = 0.0f;
    } else {
      const float *cp = a.ckpt + (int64_t)(b - 1) * W * ld + pc;
#pragma unroll
      for (int d = 0; d < W; ++d) v[d] = cp[(int64_t)d * ld];
    }
    // recompute the block's rows, recording argmin codes
    const int full = (r1 - r0) / U * U;
    for (int g = 0; g < full; g += U) {
      float rv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) rv[u] = rows[(int64_t)(r0 + g + u) * ld];
      sweep_group_dirs<R, U>(v, rv, Cols<const float *>{colu + (int64_t)(r0 + g - R) * ld, ld, (int)pc},
                             lds_lane + g * WPR * kWave);
    }
    for (int ii = r0 + full; ii < r1; ++ii) {
      // ragged tail of the last block, one row at a time
      const float rvi = rows[(int64_t)ii * ld];
      const float *cb = cols + (int64_t)(ii - R) * ld;
      unsigned words[WPR];
#pragma unroll
      for (int w = 0; w < WPR; ++w) words[w] = 0u;
#pragma unroll
      for (int d = 0; d < W; ++d) {
        const float cv = cb[(int64_t)d * ld];
        const float left = (d > 0) ? v[d > 0 ? d - 1 : 0] : kInf;
        const float top = (d < W - 1) ? v[d < W - 1 ? d + 1 : 0] : kInf;
        const float diag = v[d];
        const float diff = cv - rvi;
        v[d] = __builtin_fmaf(diff, diff, fmin3(left, top, diag));
        const unsigned code = (diag <= fminf(top, left)) ? 0u : ((top <= left) ? 1u : 2u);
        words[d / 16] |= code << (2 * (d % 16));
      }
      const int u0 = ii - r0;
#pragma unroll
      for (int w = 0; w < WPR; ++w) lds_lane[(u0 * WPR + w) * kWave] = words[w];
    }
    // backtrack through the block (each lane reads only its own LDS words).
    // row_hi / col_hi: column (row) at which the path entered the current row
    // (column); leaving a row or column closes its range.
    while (!done && i >= r0) {
      if (i == 0 && j == 0) {
        rowrng[0] = (unsigned)row_hi << 16;
        colrng[0] = (unsigned)col_hi << 16;
        done = true;
        break;
      }
      const int d = j - i + R;
      const int u = i - r0;
      const unsigned word = lds_lane[(u * WPR + d / 16) * kWave];
      const unsigned code = (word >> (2 * (d % 16))) & 3u;
      if (code == 0u) {         // diagonal
        rowrng[i] = (unsigned)j | ((unsigned)row_hi << 16);
        colrng[j] = (unsigned)i | ((unsigned)col_hi << 16);
        --i;
        --j;
        row_hi = j;
        col_hi = i;
      } else if (code == 1u) {  // top: (i-1, j)
        rowrng[i] = (unsigned)j | ((unsigned)row_hi << 16);
        --i;
        row_hi = j;
      } else {                  // left: (i, j-1)
        colrng[j] = (unsigned)i | ((unsigned)col_hi << 16);
        --j;
        col_hi = i;
      }
    }
  }
}

// Gradients from the recorded path ranges: thread (p, t) computes dS(t) over
// the path cells of row t and dT(t) over those of column t.
__global__ void dtw_grad_kernel(const float *__restrict__ S, const float *__restrict__ T,
                                int64_t npairs, int L, const unsigned *__restrict__ rowrng,
                                const unsigned *__restrict__ colrng, const float *__restrict__ dist,
                                const float *__restrict__ gout, float *__restrict__ gS,
                                float *__restrict__ gT) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= npairs * L) return;
  const int64_t p = id / L;
  const int t = (int)(id % L);
  const float *Sp = S + p * L;
  const float *Tp = T + p * L;
  if (dist && !(dist[p] < kInf)) {
    gS[id] = 0.0f;
    gT[id] = 0.0f;
    return;
  }
  const float g2 = 2.0f * gout[p];
  const unsigned rr = rowrng[id], cr = colrng[id];
  const int jlo = (int)(rr & 0xffffu), jhi = (int)(rr >> 16);
  const int ilo = (int)(cr & 0xffffu), ihi = (int)(cr >> 16);
  const float s = Sp[t];
  float accS = 0.0f;
  for (int jj = jlo; jj <= jhi; ++jj) accS += s - Tp[jj];
  const float tv = Tp[t];
  float accT = 0.0f;
  for (int ii = ilo; ii <= ihi; ++ii) accT += Sp[ii] - tv;
  gS[id] = g2 * accS;
  gT[id] = -g2 * accT;
}

template <int R>
static hipError_t launch_bwd_r(const BwdArgs &a, hipStream_t st) {
  constexpr int W = 2 * R + 1;
  constexpr int WPR = (W + 15) / 16;
  const size_t lds = sizeof(unsigned) * (size_t)kBwdBlock * WPR * kWave;
  hipLaunchKernelGGL((dtw_bwd_kernel<R>), dim3((unsigned)(a.ld / kWave)), dim3(kWave), lds, st, a);
  return hipGetLastError();
}

typedef hipError_t (*BwdFn)(const BwdArgs &, hipStream_t);

#define EAPDTW_B(R) &launch_bwd_r<R>
#define EAPDTW_B8(a) EAPDTW_B(a), EAPDTW_B(a + 1), EAPDTW_B(a + 2), EAPDTW_B(a + 3), \
  EAPDTW_B(a + 4), EAPDTW_B(a + 5), EAPDTW_B(a + 6), EAPDTW_B(a + 7)
static const BwdFn kBwd[kBandRMax + 1] = {EAPDTW_B8(0),  EAPDTW_B8(8),  EAPDTW_B8(16),
                                          EAPDTW_B8(24), EAPDTW_B8(32), EAPDTW_B8(40),
                                          EAPDTW_B8(48), EAPDTW_B8(56), EAPDTW_B(64)};

hipError_t launch_dtw_bwd(int r, const BwdArgs &a, hipStream_t st) {
  if (r < 0 || r > kBandRMax) return hipErrorInvalidValue;
  return kBwd[r](a, st);
}

hipError_t launch_dtw_grad(const float *S, const float *T, int64_t npairs, int L,
                           const unsigned *rowrng, const unsigned *colrng, const float *dist,
                           const float *gout, float *gS, float *gT, hipStream_t st) {
  const int64_t n = npairs * L;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dtw_grad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, S, T,
                     npairs, L, rowrng, colrng, dist, gout, gS, gT);
  return hipGetLastError();
}

}  // namespace eapdtw
