// wp_pass_c64x.hip -- line-pass kernels for the FP32 state, FP64 arithmetic.
#include "wp_pass.hpp"

namespace wp {

hipError_t dispatch_pass_c64x(int lgN, const PassArgs &a, hipStream_t s) { return dispatch_pass<float, double>(lgN, a, s); }

}  // namespace wp
