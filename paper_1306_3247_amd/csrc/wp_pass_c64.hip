// wp_pass_c64.hip -- line-pass kernels: FP32 state, FP32 arithmetic with FP64 factors, default shapes.
#include "wp_pass.hpp"

namespace wp {

hipError_t dispatch_pass_c64_0(int lgN, const PassArgs &a, hipStream_t s) {
  return dispatch_pass<float, float, 0>(lgN, a, s);
}
hipError_t dispatch_batch_c64_0(const BatchLaunch &b, hipStream_t s) {
  return dispatch_batch<float, float, 0>(b, s);
}
int pass_tile_c64_0(int lgN, bool strided, int kind) { return pass_tile_t<float, float, 0>(lgN, strided, kind); }

}  // namespace wp
