// wide_inst.hip -- launchers of the wide-window kernels.
#include "dispatch.h"
#include "wide.h"

namespace eapdtw {

template <int H, bool BANDED>
static hipError_t launch_wide_h(int kind, const WideArgs &a, int grid, hipStream_t st) {
  switch (kind) {
    case kWideSearch:
      hipLaunchKernelGGL((wide_kernel<H, kWideSearch, BANDED>), dim3(grid), dim3(kWave), 0, st, a);
      break;
    case kWidePairwise:
      hipLaunchKernelGGL((wide_kernel<H, kWidePairwise, BANDED>), dim3(grid), dim3(kWave), 0, st, a);
      break;
    case kWideSearchW:
      // weighted search: windows above the band kernels' (tall banded tiles
      // or whole-matrix tiles), the 2r + 1 weights in dynamic LDS
      if constexpr ((BANDED && H == kWideBandRowsTall) || (!BANDED && (H == 32 || H == 64))) {
        hipLaunchKernelGGL((wide_kernel<H, kWideSearchW, BANDED>), dim3(grid), dim3(kWave),
                           sizeof(float) * (size_t)(2 * a.r + 1 + 2 * kWtPad), st, a);
        break;
      } else {
        return hipErrorInvalidValue;
      }
    default:
      hipLaunchKernelGGL((wide_kernel<H, kWidePairs, BANDED>), dim3(grid), dim3(kWave), 0, st, a);
      break;
  }
  return hipGetLastError();
}

// NN1 seeding: for every pair i < j the squared Euclidean distance, with the
// operations of the pairwise kernel's (so it is never below the pair's DTW),
// lowers both series' words to (ED, other index): each word then starts
// from an admissible path's cost to an actual neighbour.  Task t = (i, block
// of 64 j); one wave per workgroup.
__global__ __launch_bounds__(64) void nn1_seed_kernel(WideArgs a) {
  const int lane = threadIdx.x;
  for (int64_t task = blockIdx.x; task < a.ntasks; task += gridDim.x) {
    const int64_t i = task / a.nblk_j, jb = task % a.nblk_j;
    const bool cross = a.nq > 0;  // test set against a reference set: every pair
    if (!cross && jb * kWave + kWave - 1 <= i) continue;
    const int64_t j = jb * kWave + lane;
    const bool active = (cross || j > i) && j < a.N;
    const int64_t jc = active ? j : a.N - 1;
    const float *rowp = a.X + i * a.lrow;
    const float *colp = a.XT + jc;
    float acc = 0.0f;
    for (int t = 0; t < a.lrow; ++t) {
      const float diff = colp[(int64_t)t * a.ld] - rowp[t];
      acc = __builtin_fmaf(diff, diff, acc);
    }
    publish_best(a.nn1 + i, active, acc, (uint32_t)j);
    if (!cross && active) atomicMin(a.nn1 + j, pack_best(acc, (uint32_t)i));
  }
}

hipError_t launch_nn1_seed(const WideArgs &a, int grid, hipStream_t st) {
  if (grid <= 0 || a.ntasks <= 0) return hipSuccess;
  hipLaunchKernelGGL(nn1_seed_kernel, dim3(grid), dim3(kWave), 0, st, a);
  return hipGetLastError();
}

int wide_rows_for(int r, int lrow, int lcol) {
  const int lmax = lrow > lcol ? lrow : lcol;
  if (r >= lmax - 1) return kWideFullRows;
  // a banded tile of H rows needs 2r + 2 >= H (its entering and exiting
  // triangles must not overlap)
  if (2 * r + 2 >= kWideBandRowsTall) return kWideBandRowsTall;
  if (2 * r + 2 >= kWideBandRows) return kWideBandRows;
  if (2 * r + 2 >= 4) return 4;
  return 2;
}

// Windows covering the whole matrix use tiles of kWideFullRows rows with full
// columns only; banded windows use the triangle-unrolled tiles.
hipError_t launch_wide(int kind, int rows, const WideArgs &a, int grid, hipStream_t st) {
  if (grid <= 0 || a.ntasks <= 0) return hipSuccess;
  switch (wide_rows_for(a.r, a.lrow, a.lcol)) {
    case kWideFullRows:
      // whole-matrix windows: 32- or 64-row tiles (rows option, default 64)
      if (rows == 32) return launch_wide_h<32, false>(kind, a, grid, st);
      return launch_wide_h<64, false>(kind, a, grid, st);
    case kWideBandRowsTall: return launch_wide_h<kWideBandRowsTall, true>(kind, a, grid, st);
    case kWideBandRows: return launch_wide_h<kWideBandRows, true>(kind, a, grid, st);
    case 4: return launch_wide_h<4, true>(kind, a, grid, st);
    default: return launch_wide_h<2, true>(kind, a, grid, st);
  }
}

// The cascade's search over a survivor list (windows above the band
// kernels': banded 32-row tiles or whole-matrix tiles).
hipError_t launch_wide_list(int rows, const WideArgs &a, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  const dim3 g((unsigned)grid), b(kWave);
  switch (wide_rows_for(a.r, a.lrow, a.lcol)) {
    case kWideFullRows:
      if (rows == 32)
        hipLaunchKernelGGL((wide_list_kernel<32, false>), g, b, 0, st, a);
      else
        hipLaunchKernelGGL((wide_list_kernel<64, false>), g, b, 0, st, a);
      break;
    case kWideBandRowsTall: hipLaunchKernelGGL((wide_list_kernel<kWideBandRowsTall, true>), g, b, 0, st, a); break;
    default: return hipErrorInvalidValue;  // narrower windows: the band kernels' list mode
  }
  return hipGetLastError();
}

}  // namespace eapdtw
