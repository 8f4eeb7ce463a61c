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

// FP64 reductions of the state in two deterministic passes over
// diag_blocks(n) workgroups.  part must hold diag_scratch_doubles(n) values;
// on return part[5 * diag_blocks(n) + k] holds, for k = 0..4: the liquid mass
// (sum of rho over liquid cells), the sum of T - t_m over all cells, the
// sum of the fronts, and the melted and frozen cell counts.  Every value of
// part is overwritten; nothing needs clearing.  f may be null when P.flow == 0.
constexpr int kDiagBlocks = 1024;
inline int diag_blocks(int n) { return n * n < kDiagBlocks ? n * n : kDiagBlocks; }
inline size_t diag_scratch_doubles(int n) { return 5 * (size_t)diag_blocks(n) + 5; }
hipError_t launch_diag_sums(int kind, const KParams& P, const void* f, const void* g,
                            const int* cnt, const double* s, const int* melted,
                            const int* frozen, double* part, hipStream_t st);

}  // namespace lbmk
