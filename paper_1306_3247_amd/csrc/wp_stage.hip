// wp_stage.hip -- conversions between a host-order staging run of points and
// the stored state, for state transfers that change the precision
// (wp_set_state into an FP32 state, wp_get_state in the other precision).
// The conversion runs on the device, so a transfer moves each point over
// PCIe once, in the host's precision, and the host does no per-point work.
#include "wp_stage.hpp"

namespace wp {

namespace {

// Points first .. first+count-1 (logical row-major order) between the
// contiguous staging run `run` (complex of H) and the stored state (complex
// of S, planes laid out as GridDev describes).
template <class S, class H>
__global__ void stage_in_kernel(void *psi, GridDev g, const typename storage<H>::type *run, int64_t first,
                                int64_t count) {
  using T = typename storage<S>::type;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    store_from((T *)psi + phys_index(g, first + i), load_as<S>(run + i));
}

template <class S, class H>
__global__ void stage_out_kernel(const void *psi, GridDev g, typename storage<H>::type *run, int64_t first,
                                 int64_t count) {
  using T = typename storage<S>::type;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    store_from(run + i, load_as<H>((const T *)psi + phys_index(g, first + i)));
}

unsigned stage_blocks(int64_t count) {
  const int64_t b = (count + 255) / 256;
  return (unsigned)(b > 16384 ? 16384 : (b < 1 ? 1 : b));
}

}  // namespace

hipError_t launch_stage_in(int store_prec, void *psi, const GridDev &g, int host_prec, const void *run, int64_t first,
                           int64_t count, hipStream_t s) {
  const dim3 grid(stage_blocks(count)), block(256);
  if (store_prec == 1 && host_prec == 2)
    return launch_kernel(stage_in_kernel<float, double>, grid, block, s, psi, g, (const double2 *)run, first, count);
  if (store_prec == 2 && host_prec == 1)
    return launch_kernel(stage_in_kernel<double, float>, grid, block, s, psi, g, (const float2 *)run, first, count);
  return hipErrorInvalidValue;
}

hipError_t launch_stage_out(int store_prec, const void *psi, const GridDev &g, int host_prec, void *run, int64_t first,
                            int64_t count, hipStream_t s) {
  const dim3 grid(stage_blocks(count)), block(256);
  if (store_prec == 1 && host_prec == 2)
    return launch_kernel(stage_out_kernel<float, double>, grid, block, s, psi, g, (double2 *)run, first, count);
  if (store_prec == 2 && host_prec == 1)
    return launch_kernel(stage_out_kernel<double, float>, grid, block, s, psi, g, (float2 *)run, first, count);
  return hipErrorInvalidValue;
}

}  // namespace wp
