// wp_pass_c64_t1.hip -- line-pass kernels: FP32 state, tuning variant 1 (8 values per thread).
#include "wp_pass.hpp"

namespace wp {

hipError_t dispatch_pass_c64_1(int lgN, const PassArgs &a, hipStream_t s) {
  return dispatch_pass<float, float, 1>(lgN, a, s);
}
hipError_t dispatch_batch_c64_1(const BatchLaunch &b, hipStream_t s) {
  return dispatch_batch<float, float, 1>(b, s);
}
int pass_tile_c64_1(int lgN, bool strided, int kind) { return pass_tile_t<float, float, 1>(lgN, strided, kind); }

}  // namespace wp
