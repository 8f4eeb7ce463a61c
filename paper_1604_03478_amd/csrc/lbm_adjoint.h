// Internal interface of the reverse sweep (lbm_adjoint.hip), used by the
// host context (lbm_capi.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.h"

namespace lbmk {

// One reverse step from the state t+1 to the state t (FP64 adjoints, dense
// [q][n^3] and [n^2] arrays).  lg1 receives the front contributions; lf0/lg0
// are written where they are live (f: cells liquid at t), ls0 is
// overwritten, lth is incremented.
struct AdjointStep {
  const void* f0;
  const void* g0;
  const double* s0;  // state t
  const void* g1;
  const double* s1;  // state t+1 (post-collision g and front)
  const double* th;
  const int* cnt;    // liquid counts of state t
  const int* cmin2;  // their min / max over the 5x5 columns around each column
  const int* cmax2;
  double* lf1;
  double* lg1;
  const double* ls1;
  double* lf0;
  double* lg0;
  double* ls0;
  double* lfh;
  double* lgh;       // per-cell adjoint of the pulled populations
  double* out5;
  double* own;       // per-column scratch of the front adjoint
  double* lth;
};
hipError_t launch_adjoint_step(int kind, const KParams& P, const AdjointStep& A, hipStream_t st);
hipError_t launch_fill(double* v, size_t count, double value, hipStream_t st);

}  // namespace lbmk
