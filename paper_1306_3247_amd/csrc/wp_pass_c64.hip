// wp_pass_c64.hip -- line-pass kernels for the FP32 state, FP32 arithmetic with FP64 factors.
#include "wp_pass.hpp"

namespace wp {

hipError_t dispatch_pass_c64(int lgN, const PassArgs &a, hipStream_t s) { return dispatch_pass<float, float>(lgN, a, s); }
hipError_t dispatch_batch_c64(const BatchLaunch &b, hipStream_t s) { return dispatch_batch<float, float>(b, s); }
int pass_tile_c64(int lgN, bool strided, int kind) { return pass_tile_t<float, float>(lgN, strided, kind); }

}  // namespace wp
