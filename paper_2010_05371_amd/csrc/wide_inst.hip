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
    default:
      hipLaunchKernelGGL((wide_kernel<H, kWidePairs, BANDED>), dim3(grid), dim3(kWave), 0, st, a);
      break;
  }
  return hipGetLastError();
}

int wide_rows_for(int r, int lrow, int lcol) {
  const int lmax = lrow > lcol ? lrow : lcol;
  if (r >= lmax - 1) return kWideFullRows;
  // a banded tile of H rows needs 2r + 2 >= H (its entering and exiting
  // triangles must not overlap)
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
    case kWideBandRows: return launch_wide_h<kWideBandRows, true>(kind, a, grid, st);
    case 4: return launch_wide_h<4, true>(kind, a, grid, st);
    default: return launch_wide_h<2, true>(kind, a, grid, st);
  }
}

}  // namespace eapdtw
