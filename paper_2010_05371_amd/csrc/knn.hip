// knn.hip -- selection of the k nearest neighbours of a search from the
// candidates its waves kept (packed (distance, offset) words, appended in
// any order).  Every kept word whose distance is above the final bound (an
// upper bound of the k-th best) can be dropped; at least k words remain at or
// below it (the k candidates that set the bound were kept and appended, or,
// for a bound from the seeding workgroup, were kept by the search with a
// bound never below it).
//
//  * knn_filter_kernel: grid-stride compaction of the words at or below the
//    bound (one atomic per wave);
//  * knn_topk_kernel:   one workgroup: tiles of the survivors are sorted in
//    LDS (bitonic) together with the current k best, which are carried to the
//    next tile; the k smallest words in (distance, offset) order are written
//    out.
#include "common.h"
#include "dispatch.h"

namespace eapdtw {

namespace {

constexpr int kSelThreads = 1024;
constexpr int kSelTile = 4096;  // words sorted per step (32 KB of LDS)

__global__ __launch_bounds__(256) void knn_filter_kernel(const unsigned long long *__restrict__ buf,
                                                         const unsigned long long *n_in,
                                                         const unsigned long long *bound,
                                                         unsigned long long *out,
                                                         unsigned long long *n_out) {
  const uint64_t n = *n_in;
  const uint32_t bd = (uint32_t)(*bound >> 32);  // float32 bits of the bound distance
  const int lane = threadIdx.x % kWave;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  // every lane of a wave runs the same number of iterations (the wave-level
  // ballot and shuffle below need all 64 lanes)
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x - lane); base < n;
       base += stride) {
    const uint64_t i = base + lane;
    unsigned long long v = ~0ull;
    if (i < n) v = buf[i];
    const bool take = i < n && (uint32_t)(v >> 32) <= bd;
    const unsigned long long mask = __builtin_amdgcn_ballot_w64(take);
    if (!mask) continue;
    unsigned long long o = 0;
    if (lane == 0) o = atomicAdd(n_out, (unsigned long long)__popcll(mask));
    o = __shfl(o, 0, kWave);
    if (take) {
      const unsigned r = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
      out[o + r] = v;
    }
  }
}

__global__ __launch_bounds__(kSelThreads) void knn_topk_kernel(const unsigned long long *__restrict__ in,
                                                               const unsigned long long *n_in, int k,
                                                               unsigned long long *out) {
  __shared__ unsigned long long t[kSelTile];
  const uint64_t n = *n_in;
  const int tid = threadIdx.x;
  // slots [0, k) carry the best words so far (all ones = none yet)
  for (int i = tid; i < kSelTile; i += kSelThreads) t[i] = ~0ull;
  __syncthreads();
  const uint64_t per = (uint64_t)(kSelTile - k);
  for (uint64_t base = 0; base < n || base == 0; base += per) {
    for (int i = tid; i < kSelTile - k; i += kSelThreads) {
      const uint64_t g = base + (uint64_t)i;
      t[k + i] = g < n ? in[g] : ~0ull;
    }
    __syncthreads();
    for (int size = 2; size <= kSelTile; size <<= 1) {
      for (int stride = size >> 1; stride >= 1; stride >>= 1) {
        for (int i = tid; i < kSelTile / 2; i += kSelThreads) {
          // pair (lo, lo + stride) with lo's stride bit clear
          const int lo = 2 * i - (i & (stride - 1));
          const int hi = lo + stride;
          const bool up = (lo & size) == 0;
          const unsigned long long a = t[lo], b = t[hi];
          if ((a > b) == up) {
            t[lo] = b;
            t[hi] = a;
          }
        }
        __syncthreads();
      }
    }
    if (base + per >= n) break;
  }
  for (int i = tid; i < k; i += kSelThreads) out[i] = t[i];
}

}  // namespace

hipError_t launch_knn_select(const unsigned long long *buf, const unsigned long long *n_buf,
                             const unsigned long long *bound, unsigned long long *tmp,
                             unsigned long long *n_tmp, int k, unsigned long long *out,
                             hipStream_t st) {
  if (k < 1 || k > kKnnMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(knn_filter_kernel, dim3(1024), dim3(256), 0, st, buf, n_buf, bound, tmp,
                     n_tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(knn_topk_kernel, dim3(1), dim3(kSelThreads), 0, st, tmp, n_tmp, k, out);
  return hipGetLastError();
}

}  // namespace eapdtw
