// znorm.h -- workgroup-wide z-normalisation of one short series.
#pragma once
#include "band.h"

namespace eapdtw {

__device__ __forceinline__ bool not_finite(float v) { return !(fabsf(v) <= 3.402823466e38f); }

// Workgroup-wide float64 sum (blockDim.x a multiple of 64, at most 1024).
__device__ __forceinline__ double block_sum_f64(double v, double *sh) {
  v = wave_sum_f64(v);
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x / kWave); ++i) t += sh[i];
  return t;
}

// Two passes in float64, population sigma; a flat series normalises to zeros.
// Writes out[pad + j] for j < m and +inf into the `pad` entries on each side.
// Returns (in every thread) the number of non-finite inputs.
__device__ __forceinline__ int znorm_block(const float *__restrict__ q, int m,
                                           float *__restrict__ out, int pad, double *sh) {
  double s = 0.0;
  int bad = 0;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    const float v = q[j];
    bad += not_finite(v);
    s += (double)v;
  }
  const double mean = block_sum_f64(s, sh) / (double)m;
  double ss = 0.0;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    const double dv = (double)q[j] - mean;
    ss += dv * dv;
  }
  const double var = block_sum_f64(ss, sh) / (double)m;
  // flat (variance at most kFlatRel of the mean square): zeros
  const double sd = (var > kFlatRel * (var + mean * mean)) ? sqrt(var) : 0.0;
  for (int j = threadIdx.x; j < m; j += blockDim.x)
    out[pad + j] = sd > 0.0 ? (float)(((double)q[j] - mean) / sd) : 0.0f;
  for (int j = threadIdx.x; j < pad; j += blockDim.x) {
    out[j] = kInf;
    out[pad + m + j] = kInf;
  }
  return (int)block_sum_f64((double)bad, sh);
}

}  // namespace eapdtw
