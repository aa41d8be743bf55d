// band_inst.hip -- explicit instantiations of the band kernels for the windows
// EAPDTW_R_LO..EAPDTW_R_HI.  The build compiles this file once per window range
// so that the instantiations compile in parallel.
#include "band.h"

#ifndef EAPDTW_R_LO
#define EAPDTW_R_LO 0
#define EAPDTW_R_HI 64
#endif

namespace eapdtw {

template <int R>
hipError_t launch_nn_band(const NNArgs &a, int64_t nblocks, int rows_per_group, bool dists,
                          bool border, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  const dim3 grid((unsigned)nblocks), block(kWave);
  constexpr bool kB = R >= kBorderMinR;  // bordered variants exist from this window on
  if (kB && border) {
    if (dists)
      hipLaunchKernelGGL((nn_band_kernel<R, 4, true, kB>), grid, block, 0, st, a);
    else
      hipLaunchKernelGGL((nn_band_kernel<R, 4, false, kB>), grid, block, 0, st, a);
  } else if (dists) {
    hipLaunchKernelGGL((nn_band_kernel<R, 4, true, false>), grid, block, 0, st, a);
  } else {
    switch (rows_per_group) {
      case 2: hipLaunchKernelGGL((nn_band_kernel<R, 2, false, false>), grid, block, 0, st, a); break;
      case 8: hipLaunchKernelGGL((nn_band_kernel<R, 8, false, false>), grid, block, 0, st, a); break;
      default: hipLaunchKernelGGL((nn_band_kernel<R, 4, false, false>), grid, block, 0, st, a); break;
    }
  }
  return hipGetLastError();
}

template <int R>
hipError_t launch_nn_list(const NNArgs &a, int64_t nblocks, bool dists, bool border,
                          hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  const dim3 grid((unsigned)nblocks), block(kWave);
  constexpr bool kB = R >= kBorderMinR;
  if (kB && border) {
    if (dists)
      hipLaunchKernelGGL((nn_list_kernel<R, 4, true, kB>), grid, block, 0, st, a);
    else
      hipLaunchKernelGGL((nn_list_kernel<R, 4, false, kB>), grid, block, 0, st, a);
  } else if (dists) {
    hipLaunchKernelGGL((nn_list_kernel<R, 4, true, false>), grid, block, 0, st, a);
  } else {
    hipLaunchKernelGGL((nn_list_kernel<R, 4, false, false>), grid, block, 0, st, a);
  }
  return hipGetLastError();
}

template <int R>
hipError_t launch_nn_wband(const NNArgs &a, int64_t nblocks, bool dists, bool border,
                           hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  const dim3 grid((unsigned)nblocks), block(kWave);
  constexpr bool kB = R >= kBorderMinR;
  if (kB && border) {
    if (dists)
      hipLaunchKernelGGL((nn_wband_kernel<R, 4, true, kB>), grid, block, 0, st, a);
    else
      hipLaunchKernelGGL((nn_wband_kernel<R, 4, false, kB>), grid, block, 0, st, a);
  } else if (dists) {
    hipLaunchKernelGGL((nn_wband_kernel<R, 4, true, false>), grid, block, 0, st, a);
  } else {
    hipLaunchKernelGGL((nn_wband_kernel<R, 4, false, false>), grid, block, 0, st, a);
  }
  return hipGetLastError();
}

template <int R>
hipError_t launch_pair_band(const PairArgs &a, int64_t nblocks, int rows_per_group,
                            hipStream_t st) {
  (void)rows_per_group;
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((pair_band_kernel<R, 4>), dim3((unsigned)nblocks), dim3(kWave), 0, st, a);
  return hipGetLastError();
}

#define EAPDTW_INST(R)                                                                       \
  template hipError_t launch_nn_band<R>(const NNArgs &, int64_t, int, bool, bool, hipStream_t); \
  template hipError_t launch_nn_list<R>(const NNArgs &, int64_t, bool, bool, hipStream_t);     \
  template hipError_t launch_nn_wband<R>(const NNArgs &, int64_t, bool, bool, hipStream_t);    \
  template hipError_t launch_pair_band<R>(const PairArgs &, int64_t, int, hipStream_t);

#if EAPDTW_R_LO <= 0 && 0 <= EAPDTW_R_HI
EAPDTW_INST(0)
#endif
#if EAPDTW_R_LO <= 1 && 1 <= EAPDTW_R_HI
EAPDTW_INST(1)
#endif
#if EAPDTW_R_LO <= 2 && 2 <= EAPDTW_R_HI
EAPDTW_INST(2)
#endif
#if EAPDTW_R_LO <= 3 && 3 <= EAPDTW_R_HI
EAPDTW_INST(3)
#endif
#if EAPDTW_R_LO <= 4 && 4 <= EAPDTW_R_HI
EAPDTW_INST(4)
#endif
#if EAPDTW_R_LO <= 5 && 5 <= EAPDTW_R_HI
EAPDTW_INST(5)
#endif
#if EAPDTW_R_LO <= 6 && 6 <= EAPDTW_R_HI
EAPDTW_INST(6)
#endif
#if EAPDTW_R_LO <= 7 && 7 <= EAPDTW_R_HI
EAPDTW_INST(7)
#endif
#if EAPDTW_R_LO <= 8 && 8 <= EAPDTW_R_HI
EAPDTW_INST(8)
#endif
#if EAPDTW_R_LO <= 9 && 9 <= EAPDTW_R_HI
EAPDTW_INST(9)
#endif
#if EAPDTW_R_LO <= 10 && 10 <= EAPDTW_R_HI
EAPDTW_INST(10)
#endif
#if EAPDTW_R_LO <= 11 && 11 <= EAPDTW_R_HI
EAPDTW_INST(11)
#endif
#if EAPDTW_R_LO <= 12 && 12 <= EAPDTW_R_HI
EAPDTW_INST(12)
#endif
#if EAPDTW_R_LO <= 13 && 13 <= EAPDTW_R_HI
EAPDTW_INST(13)
#endif
#if EAPDTW_R_LO <= 14 && 14 <= EAPDTW_R_HI
EAPDTW_INST(14)
#endif
#if EAPDTW_R_LO <= 15 && 15 <= EAPDTW_R_HI
EAPDTW_INST(15)
#endif
#if EAPDTW_R_LO <= 16 && 16 <= EAPDTW_R_HI
EAPDTW_INST(16)
#endif
#if EAPDTW_R_LO <= 17 && 17 <= EAPDTW_R_HI
EAPDTW_INST(17)
#endif
#if EAPDTW_R_LO <= 18 && 18 <= EAPDTW_R_HI
EAPDTW_INST(18)
#endif
#if EAPDTW_R_LO <= 19 && 19 <= EAPDTW_R_HI
EAPDTW_INST(19)
#endif
#if EAPDTW_R_LO <= 20 && 20 <= EAPDTW_R_HI
EAPDTW_INST(20)
#endif
#if EAPDTW_R_LO <= 21 && 21 <= EAPDTW_R_HI
EAPDTW_INST(21)
#endif
#if EAPDTW_R_LO <= 22 && 22 <= EAPDTW_R_HI
EAPDTW_INST(22)
#endif
#if EAPDTW_R_LO <= 23 && 23 <= EAPDTW_R_HI
EAPDTW_INST(23)
#endif
#if EAPDTW_R_LO <= 24 && 24 <= EAPDTW_R_HI
EAPDTW_INST(24)
#endif
#if EAPDTW_R_LO <= 25 && 25 <= EAPDTW_R_HI
EAPDTW_INST(25)
#endif
#if EAPDTW_R_LO <= 26 && 26 <= EAPDTW_R_HI
EAPDTW_INST(26)
#endif
#if EAPDTW_R_LO <= 27 && 27 <= EAPDTW_R_HI
EAPDTW_INST(27)
#endif
#if EAPDTW_R_LO <= 28 && 28 <= EAPDTW_R_HI
EAPDTW_INST(28)
#endif
#if EAPDTW_R_LO <= 29 && 29 <= EAPDTW_R_HI
EAPDTW_INST(29)
#endif
#if EAPDTW_R_LO <= 30 && 30 <= EAPDTW_R_HI
EAPDTW_INST(30)
#endif
#if EAPDTW_R_LO <= 31 && 31 <= EAPDTW_R_HI
EAPDTW_INST(31)
#endif
#if EAPDTW_R_LO <= 32 && 32 <= EAPDTW_R_HI
EAPDTW_INST(32)
#endif
#if EAPDTW_R_LO <= 33 && 33 <= EAPDTW_R_HI
EAPDTW_INST(33)
#endif
#if EAPDTW_R_LO <= 34 && 34 <= EAPDTW_R_HI
EAPDTW_INST(34)
#endif
#if EAPDTW_R_LO <= 35 && 35 <= EAPDTW_R_HI
EAPDTW_INST(35)
#endif
#if EAPDTW_R_LO <= 36 && 36 <= EAPDTW_R_HI
EAPDTW_INST(36)
#endif
#if EAPDTW_R_LO <= 37 && 37 <= EAPDTW_R_HI
EAPDTW_INST(37)
#endif
#if EAPDTW_R_LO <= 38 && 38 <= EAPDTW_R_HI
EAPDTW_INST(38)
#endif
#if EAPDTW_R_LO <= 39 && 39 <= EAPDTW_R_HI
EAPDTW_INST(39)
#endif
#if EAPDTW_R_LO <= 40 && 40 <= EAPDTW_R_HI
EAPDTW_INST(40)
#endif
#if EAPDTW_R_LO <= 41 && 41 <= EAPDTW_R_HI
EAPDTW_INST(41)
#endif
#if EAPDTW_R_LO <= 42 && 42 <= EAPDTW_R_HI
EAPDTW_INST(42)
#endif
#if EAPDTW_R_LO <= 43 && 43 <= EAPDTW_R_HI
EAPDTW_INST(43)
#endif
#if EAPDTW_R_LO <= 44 && 44 <= EAPDTW_R_HI
EAPDTW_INST(44)
#endif
#if EAPDTW_R_LO <= 45 && 45 <= EAPDTW_R_HI
EAPDTW_INST(45)
#endif
#if EAPDTW_R_LO <= 46 && 46 <= EAPDTW_R_HI
EAPDTW_INST(46)
#endif
#if EAPDTW_R_LO <= 47 && 47 <= EAPDTW_R_HI
EAPDTW_INST(47)
#endif
#if EAPDTW_R_LO <= 48 && 48 <= EAPDTW_R_HI
EAPDTW_INST(48)
#endif
#if EAPDTW_R_LO <= 49 && 49 <= EAPDTW_R_HI
EAPDTW_INST(49)
#endif
#if EAPDTW_R_LO <= 50 && 50 <= EAPDTW_R_HI
EAPDTW_INST(50)
#endif
#if EAPDTW_R_LO <= 51 && 51 <= EAPDTW_R_HI
EAPDTW_INST(51)
#endif
#if EAPDTW_R_LO <= 52 && 52 <= EAPDTW_R_HI
EAPDTW_INST(52)
#endif
#if EAPDTW_R_LO <= 53 && 53 <= EAPDTW_R_HI
EAPDTW_INST(53)
#endif
#if EAPDTW_R_LO <= 54 && 54 <= EAPDTW_R_HI
EAPDTW_INST(54)
#endif
#if EAPDTW_R_LO <= 55 && 55 <= EAPDTW_R_HI
EAPDTW_INST(55)
#endif
#if EAPDTW_R_LO <= 56 && 56 <= EAPDTW_R_HI
EAPDTW_INST(56)
#endif
#if EAPDTW_R_LO <= 57 && 57 <= EAPDTW_R_HI
EAPDTW_INST(57)
#endif
#if EAPDTW_R_LO <= 58 && 58 <= EAPDTW_R_HI
EAPDTW_INST(58)
#endif
#if EAPDTW_R_LO <= 59 && 59 <= EAPDTW_R_HI
EAPDTW_INST(59)
#endif
#if EAPDTW_R_LO <= 60 && 60 <= EAPDTW_R_HI
EAPDTW_INST(60)
#endif
#if EAPDTW_R_LO <= 61 && 61 <= EAPDTW_R_HI
EAPDTW_INST(61)
#endif
#if EAPDTW_R_LO <= 62 && 62 <= EAPDTW_R_HI
EAPDTW_INST(62)
#endif
#if EAPDTW_R_LO <= 63 && 63 <= EAPDTW_R_HI
EAPDTW_INST(63)
#endif
#if EAPDTW_R_LO <= 64 && 64 <= EAPDTW_R_HI
EAPDTW_INST(64)
#endif

}  // namespace eapdtw
