// dispatch.cpp -- run-time window -> compiled band kernel tables.
#include "band.h"
#include "dispatch.h"

namespace eapdtw {

#define EAPDTW_DECL(R)                                                                          \
  extern template hipError_t launch_nn_band<R>(const NNArgs &, int64_t, int, bool, bool, hipStream_t); \
  extern template hipError_t launch_nn_list<R>(const NNArgs &, int64_t, bool, bool, hipStream_t); \
  extern template hipError_t launch_nn_wband<R>(const NNArgs &, int64_t, bool, bool, hipStream_t); \
  extern template hipError_t launch_pair_band<R>(const PairArgs &, int64_t, int, hipStream_t);
#define EAPDTW_ROW8(a) EAPDTW_DECL(a) EAPDTW_DECL(a + 1) EAPDTW_DECL(a + 2) EAPDTW_DECL(a + 3) \
  EAPDTW_DECL(a + 4) EAPDTW_DECL(a + 5) EAPDTW_DECL(a + 6) EAPDTW_DECL(a + 7)
EAPDTW_ROW8(0)
EAPDTW_ROW8(8)
EAPDTW_ROW8(16)
EAPDTW_ROW8(24)
EAPDTW_ROW8(32)
EAPDTW_ROW8(40)
EAPDTW_ROW8(48)
EAPDTW_ROW8(56)
EAPDTW_DECL(64)

#define EAPDTW_NN(R) &launch_nn_band<R>
#define EAPDTW_NN8(a) EAPDTW_NN(a), EAPDTW_NN(a + 1), EAPDTW_NN(a + 2), EAPDTW_NN(a + 3), \
  EAPDTW_NN(a + 4), EAPDTW_NN(a + 5), EAPDTW_NN(a + 6), EAPDTW_NN(a + 7)
#define EAPDTW_NL(R) &launch_nn_list<R>
#define EAPDTW_NL8(a) EAPDTW_NL(a), EAPDTW_NL(a + 1), EAPDTW_NL(a + 2), EAPDTW_NL(a + 3), \
  EAPDTW_NL(a + 4), EAPDTW_NL(a + 5), EAPDTW_NL(a + 6), EAPDTW_NL(a + 7)
#define EAPDTW_NW(R) &launch_nn_wband<R>
#define EAPDTW_NW8(a) EAPDTW_NW(a), EAPDTW_NW(a + 1), EAPDTW_NW(a + 2), EAPDTW_NW(a + 3), \
  EAPDTW_NW(a + 4), EAPDTW_NW(a + 5), EAPDTW_NW(a + 6), EAPDTW_NW(a + 7)
#define EAPDTW_PB(R) &launch_pair_band<R>
#define EAPDTW_PB8(a) EAPDTW_PB(a), EAPDTW_PB(a + 1), EAPDTW_PB(a + 2), EAPDTW_PB(a + 3), \
  EAPDTW_PB(a + 4), EAPDTW_PB(a + 5), EAPDTW_PB(a + 6), EAPDTW_PB(a + 7)

static const NNLaunchFn kNN[kBandRMax + 1] = {
    EAPDTW_NN8(0),  EAPDTW_NN8(8),  EAPDTW_NN8(16), EAPDTW_NN8(24), EAPDTW_NN8(32),
    EAPDTW_NN8(40), EAPDTW_NN8(48), EAPDTW_NN8(56), EAPDTW_NN(64)};
static const NNListLaunchFn kList[kBandRMax + 1] = {
    EAPDTW_NL8(0),  EAPDTW_NL8(8),  EAPDTW_NL8(16), EAPDTW_NL8(24), EAPDTW_NL8(32),
    EAPDTW_NL8(40), EAPDTW_NL8(48), EAPDTW_NL8(56), EAPDTW_NL(64)};
static const NNListLaunchFn kWBand[kBandRMax + 1] = {
    EAPDTW_NW8(0),  EAPDTW_NW8(8),  EAPDTW_NW8(16), EAPDTW_NW8(24), EAPDTW_NW8(32),
    EAPDTW_NW8(40), EAPDTW_NW8(48), EAPDTW_NW8(56), EAPDTW_NW(64)};
static const PairLaunchFn kPair[kBandRMax + 1] = {
    EAPDTW_PB8(0),  EAPDTW_PB8(8),  EAPDTW_PB8(16), EAPDTW_PB8(24), EAPDTW_PB8(32),
    EAPDTW_PB8(40), EAPDTW_PB8(48), EAPDTW_PB8(56), EAPDTW_PB(64)};

NNLaunchFn nn_band_launcher(int r) { return (r >= 0 && r <= kBandRMax) ? kNN[r] : nullptr; }
NNListLaunchFn nn_list_launcher(int r) { return (r >= 0 && r <= kBandRMax) ? kList[r] : nullptr; }
NNListLaunchFn nn_wband_launcher(int r) { return (r >= 0 && r <= kBandRMax) ? kWBand[r] : nullptr; }
PairLaunchFn pair_band_launcher(int r) { return (r >= 0 && r <= kBandRMax) ? kPair[r] : nullptr; }

}  // namespace eapdtw
