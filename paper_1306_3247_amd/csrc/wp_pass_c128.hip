// wp_pass_c128.hip -- line-pass kernels for the FP64 state.
#include "wp_pass.hpp"

namespace wp {

hipError_t dispatch_pass_c128(int lgN, const PassArgs &a, hipStream_t s) { return dispatch_pass<double, double>(lgN, a, s); }

}  // namespace wp
