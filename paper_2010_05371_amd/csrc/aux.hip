// aux.hip -- small kernels around the DTW sweeps: query normalisation, input
// checks, transposition into the coalesced pair layout, counters.
#include "band.h"
#include "dispatch.h"
#include "znorm.h"

namespace eapdtw {

__global__ void fill_u64_kernel(unsigned long long *p, unsigned long long v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

// z-normalisation of one short series by one workgroup; counts non-finite
// inputs into the counters.
__global__ void znorm_kernel(const float *__restrict__ q, int m, float *__restrict__ out, int pad,
                             unsigned long long *counters) {
  __shared__ double sh[16];
  const int bad = znorm_block(q, m, out, pad, sh);
  if (counters && bad && threadIdx.x == 0) atomicAdd(&counters[kCntNonFinite], (unsigned long long)bad);
}

hipError_t launch_znorm(const float *x, int m, float *out, hipStream_t st) {
  hipLaunchKernelGGL(znorm_kernel, dim3(1), dim3(256), 0, st, x, m, out, 0,
                     (unsigned long long *)nullptr);
  return hipGetLastError();
}

// Everything a search needs before its first pass, in one launch: workgroup 0
// clears the counters, sets the best-so-far words to +inf and z-normalises
// the query into its padded buffer; every workgroup checks a share of the
// series.  A non-finite input stores this call's epoch into *flag (a racy
// store of one value; the word needs no clearing between calls).
__global__ void search_prep_kernel(const float *__restrict__ q, int m, float *__restrict__ qpad,
                                   const float *__restrict__ x, int64_t n,
                                   unsigned long long *cnt, unsigned long long *bsf, int nbsf,
                                   unsigned *flag, unsigned epoch) {
  __shared__ double sh[16];
  bool bad = false;
  if (blockIdx.x == 0) {
    for (int t = threadIdx.x; t < kCntWords; t += blockDim.x) cnt[t] = 0ull;
    if ((int)threadIdx.x < nbsf) bsf[threadIdx.x] = pack_best(kInf, 0xffffffffu);
    bad = znorm_block(q, m, qpad, kColPad, sh) != 0;
  }
  if (x) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
      bad = bad || not_finite(x[i]);
  }
  if (bad) *flag = epoch;
}

hipError_t launch_search_prep(const float *q, int m, float *qpad, const float *x, int64_t n,
                              unsigned long long *cnt, unsigned long long *bsf, int nbsf,
                              unsigned *flag, unsigned epoch, hipStream_t st) {
  int64_t blocks = x ? (n + 255) / 256 : 1;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(search_prep_kernel, dim3((unsigned)blocks), dim3(256), 0, st, q, m, qpad, x,
                     n, cnt, bsf, nbsf, flag, epoch);
  return hipGetLastError();
}

__global__ void check_finite_kernel(const float *__restrict__ x, int64_t n,
                                    unsigned long long *counters) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    bad += not_finite(x[i]);
  if (bad) atomicAdd(&counter_stripe(counters, blockIdx.x)[kCntNonFinite], (unsigned long long)bad);
}

__global__ void fill_f32_kernel(float *p, float v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

// dst[p][i] = src[i] for p < n, i < len
__global__ void broadcast_rows_kernel(const float *__restrict__ src, int64_t len, int64_t n,
                                      float *__restrict__ dst) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n * len) dst[k] = src[k % len];
}

hipError_t launch_broadcast_rows(const float *src, int64_t len, int64_t n, float *dst,
                                 hipStream_t st) {
  const int64_t total = n * len;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(broadcast_rows_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     st, src, len, n, dst);
  return hipGetLastError();
}

hipError_t launch_check_finite(const float *x, int64_t n, unsigned long long *counters,
                               hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x, n,
                     counters);
  return hipGetLastError();
}

// src [npairs][len] row-major  ->  dst [(len + 2 pad)][ld], element t of pair p
// at dst[(t + pad) * ld + p]; padding rows and the columns p >= npairs hold
// padval.  32x32 tiles through LDS keep both sides coalesced.
__global__ void transpose_pad_kernel(const float *__restrict__ src, int64_t npairs, int len,
                                     int64_t ld, int pad, float padval, float *__restrict__ dst) {
  __shared__ float tile[32][33];
  const int64_t p0 = (int64_t)blockIdx.x * 32;
  const int64_t t0 = (int64_t)blockIdx.y * 32 - pad;  // padded row index start (in t units)
  const int tx = threadIdx.x, ty = threadIdx.y;       // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int64_t p = p0 + r, t = t0 + tx;
    float v = padval;
    if (p < npairs && t >= 0 && t < len) v = src[p * len + t];
    tile[r][tx] = v;
  }
  __syncthreads();
  const int64_t rows = (int64_t)len + 2 * pad;
  for (int r = ty; r < 32; r += 8) {
    const int64_t trow = t0 + r + pad, p = p0 + tx;
    if (trow >= 0 && trow < rows && p < ld) dst[trow * ld + p] = tile[tx][r];
  }
}

hipError_t launch_transpose_pad(const float *src, int64_t npairs, int len, int64_t ld, int pad,
                                float padval, float *dst, hipStream_t st) {
  const int64_t rows = (int64_t)len + 2 * pad;
  dim3 grid((unsigned)((ld + 31) / 32), (unsigned)((rows + 31) / 32));
  hipLaunchKernelGGL(transpose_pad_kernel, grid, dim3(32, 8), 0, st, src, npairs, len, ld, pad,
                     padval, dst);
  return hipGetLastError();
}

// Window statistics exactly as the search kernels compute them (one wave per
// 64 consecutive offsets).
__global__ __launch_bounds__(64) void window_stats_kernel(const float *__restrict__ x, int64_t n,
                                                          int m, double *mean, double *sd) {
  const int64_t K = n - m + 1;
  const int64_t kb = (int64_t)blockIdx.x * kWave;
  const int lane = threadIdx.x;
  double mu, s;
  wave_window_stats(x, n, m, kb, lane, mu, s);
  if (kb + lane < K) {
    mean[kb + lane] = mu;
    sd[kb + lane] = s;
  }
}

hipError_t launch_window_stats(const float *x, int64_t n, int m, double *mean, double *sd,
                               hipStream_t st) {
  const int64_t K = n - m + 1;
  hipLaunchKernelGGL(window_stats_kernel, dim3((unsigned)((K + 63) / 64)), dim3(64), 0, st, x, n,
                     m, mean, sd);
  return hipGetLastError();
}

}  // namespace eapdtw
