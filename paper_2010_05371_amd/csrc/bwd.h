// bwd.h -- arguments of the backward kernels of the differentiable batch.
#pragma once
#include "common.h"

namespace eapdtw {

// Rows between two band checkpoints of the forward; the backward recomputes
// one such block at a time.
constexpr int kBwdBlock = 16;

struct BwdArgs {
  const float *rowsT;    // S transposed [len][ld]
  const float *colsT;    // T transposed and padded [len + 2 kColPad][ld]
  const float *ckpt;     // [nck][2r+1][ld] band after rows 15, 31, ...
  const float *dist;     // [npairs] forward distances
  unsigned *rowrng;      // [ld][len]  jlo | jhi << 16 of the path cells in row i
  unsigned *colrng;      // [ld][len]  ilo | ihi << 16 of the path cells in column j
  int64_t npairs, ld;
  int len;
};

hipError_t launch_dtw_bwd(int r, const BwdArgs &a, hipStream_t st);
hipError_t launch_dtw_grad(const float *S, const float *T, int64_t npairs, int L,
                           const unsigned *rowrng, const unsigned *colrng, const float *dist,
                           const float *gout, float *gS, float *gT, hipStream_t st);

// Checkpoints kept by the forward: one after every kBwdBlock rows except the last.
inline int64_t bwd_num_ckpt(int64_t len) { return len > 0 ? (len - 1) / kBwdBlock : 0; }

}  // namespace eapdtw
