// Internal interface of the conservative front update (lbm_front_heat.hip),
// used by the host context (lbm_capi.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.h"

namespace lbmk {

// Heat carried into the interface of every column by the streaming from the
// state (g, s, cnt) (post-collision g, fronts and liquid counts before the
// step): over each link that crosses the front, what the cell sent toward
// it minus what the interpolated anti-bounce-back gave back.  Links along
// the melt axis count for their column, a lateral link for the column of its
// solid cell.  heat: n^2 FP64 values, column layout of s.
hipError_t launch_front_heat(int kind, const KParams& P, const void* g, const double* s,
                             const int* cnt, double* heat, hipStream_t st);

}  // namespace lbmk
