// wp_pass_c128.hip -- line-pass kernels for the FP64 state.
#include "wp_pass.hpp"

namespace wp {

hipError_t dispatch_pass_c128(int lgN, const PassArgs &a, hipStream_t s) { return dispatch_pass<double, double>(lgN, a, s); }
hipError_t dispatch_batch_c128(const BatchLaunch &b, hipStream_t s) { return dispatch_batch<double, double>(b, s); }
int pass_tile_c128(int lgN, bool strided, int kind) { return pass_tile_t<double, double>(lgN, strided, kind); }

}  // namespace wp
