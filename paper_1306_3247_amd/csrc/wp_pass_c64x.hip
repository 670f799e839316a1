// wp_pass_c64x.hip -- line-pass kernels for the FP32 state, FP64 arithmetic.
#include "wp_pass.hpp"

namespace wp {

hipError_t dispatch_pass_c64x(int lgN, const PassArgs &a, hipStream_t s) { return dispatch_pass<float, double>(lgN, a, s); }
hipError_t dispatch_batch_c64x(const BatchLaunch &b, hipStream_t s) { return dispatch_batch<float, double>(b, s); }
int pass_tile_c64x(int lgN, bool strided, int kind) { return pass_tile_t<float, double>(lgN, strided, kind); }

}  // namespace wp
