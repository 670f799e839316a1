// wp_pass_c64.hip -- line-pass kernels for the FP32 state, FP32 arithmetic with FP64 factors.
#include "wp_pass.hpp"

namespace wp {

hipError_t dispatch_pass_c64(int lgN, const PassArgs &a, hipStream_t s) { return dispatch_pass<float, float>(lgN, a, s); }

}  // namespace wp
