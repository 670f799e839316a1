// wp_pass_c64_t2.hip -- line-pass kernels: FP32 state, tuning variant 2 (256-thread workgroups).
#include "wp_pass.hpp"

namespace wp {

hipError_t dispatch_pass_c64_2(int lgN, const PassArgs &a, hipStream_t s) {
  return dispatch_pass<float, float, 2>(lgN, a, s);
}
hipError_t dispatch_batch_c64_2(const BatchLaunch &b, hipStream_t s) {
  return dispatch_batch<float, float, 2>(b, s);
}
int pass_tile_c64_2(int lgN, bool strided, int kind) { return pass_tile_t<float, float, 2>(lgN, strided, kind); }

}  // namespace wp
