// wp_pass_c128.hip -- line-pass kernels: FP64 state and arithmetic, default shapes.
#include "wp_pass.hpp"

namespace wp {

hipError_t dispatch_pass_c128_0(int lgN, const PassArgs &a, hipStream_t s) {
  return dispatch_pass<double, double, 0>(lgN, a, s);
}
hipError_t dispatch_batch_c128_0(const BatchLaunch &b, hipStream_t s) {
  return dispatch_batch<double, double, 0>(b, s);
}
int pass_tile_c128_0(int lgN, bool strided, int kind) { return pass_tile_t<double, double, 0>(lgN, strided, kind); }

}  // namespace wp
