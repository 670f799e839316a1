// wp_pass_c64x.hip -- line-pass kernels: FP32 state, FP64 arithmetic.
#include "wp_pass.hpp"

namespace wp {

hipError_t dispatch_pass_c64x_0(int lgN, const PassArgs &a, hipStream_t s) {
  return dispatch_pass<float, double, 0>(lgN, a, s);
}
hipError_t dispatch_batch_c64x_0(const BatchLaunch &b, hipStream_t s) {
  return dispatch_batch<float, double, 0>(b, s);
}
int pass_tile_c64x_0(int lgN, bool strided, int kind) { return pass_tile_t<float, double, 0>(lgN, strided, kind); }

}  // namespace wp
