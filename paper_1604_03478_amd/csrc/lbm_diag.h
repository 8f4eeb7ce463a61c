// Internal interface of the diagnostics kernels (lbm_diag.hip), used by the
// host context (lbm_capi.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.h"

namespace lbmk {

// Local Nusselt number of every column on the heated wall (n^2 FP64 values,
// column layout of s): -n dT/da at a = 0 over (t_h - t_m), dT/da from the
// quadratic through the wall point and the first two cell centres when both
// are liquid, else the chord to the front point (s, t_m); 0 without liquid.
hipError_t launch_wall_nusselt(int kind, const KParams& P, const void* g, const double* s,
                               const double* th, double* nu, hipStream_t st);

}  // namespace lbmk
