// wp_pass_c64_t3.hip -- line-pass kernels: FP32 state, tuning variant 3 (8 values per thread, 256-thread workgroups).
#include "wp_pass.hpp"

namespace wp {

hipError_t dispatch_pass_c64_3(int lgN, const PassArgs &a, hipStream_t s) {
  return dispatch_pass<float, float, 3>(lgN, a, s);
}
hipError_t dispatch_batch_c64_3(const BatchLaunch &b, hipStream_t s) {
  return dispatch_batch<float, float, 3>(b, s);
}
int pass_tile_c64_3(int lgN, bool strided, int kind) { return pass_tile_t<float, float, 3>(lgN, strided, kind); }

}  // namespace wp
