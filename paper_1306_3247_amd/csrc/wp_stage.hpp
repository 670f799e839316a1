// wp_stage.hpp -- launchers of the precision-changing state transfers
// (wp_stage.hip).  Precisions: 1 = complex64, 2 = complex128.
#pragma once
#include "wp_internal.hpp"

namespace wp {

// Stored state <- staging run: points first .. first+count-1 (logical
// order) read from `run` (host_prec, contiguous) and stored converted to
// store_prec.
hipError_t launch_stage_in(int store_prec, void *psi, const GridDev &g, int host_prec, const void *run, int64_t first,
                           int64_t count, hipStream_t s);
// Staging run <- stored state, the other way.
hipError_t launch_stage_out(int store_prec, const void *psi, const GridDev &g, int host_prec, void *run, int64_t first,
                            int64_t count, hipStream_t s);

}  // namespace wp
