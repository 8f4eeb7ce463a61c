// Internal interface of the reverse sweep (lbm_adjoint.hip), used by the
// host context (lbm_capi.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.h"

namespace lbmk {

// One reverse step from the state t+1 to the state t.  Per-cell adjoints
// (lf*, lg*: dense [q][n^3] arrays) are stored in the type lambda_bytes
// gives (FP64 for FP64 storage, FP32 otherwise); the per-column ones (ls*,
// lth, out5, own: [n^2]) are FP64.  lg1 receives the front contributions; lf0/lg0
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
  const int* rowb;   // one int: the largest liquid count of state t
  void* lf1;
  void* lg1;
  const double* ls1;
  void* lf0;
  void* lg0;
  double* ls0;
  void* lfh;
  void* lgh;         // per-cell adjoint of the pulled populations
  // Pairing of the bulk-solid rows (lattices above the shared-launch size):
  // rowb_prev is state t+1's largest liquid count when the step after this
  // one in time (reversed just before) left the transposed streaming of the
  // paired rows to this step, whose reverse collision then gathers from
  // lgh_prev, that step's lgh; rowb_next is state t-1's when the step reversed
  // next pairs with this one (this step then skips the paired rows'
  // streaming).  NULL when there is no such pairing.
  const int* rowb_prev;
  const int* rowb_next;
  const void* lgh_prev;
  double* out5;
  double* own;       // per-column scratch of the front adjoint
  double* lth;
  // conservative front update (front scheme 1) only, else NULL: the interface
  // heat of state t per column, and the per-column weight d(J)/d(heat)
  const double* heat;
  double* wq;
};
// Largest lattice whose reverse step uses the two shared launches; above it
// the bulk-solid rows of consecutive reverse steps are paired.
constexpr int kAdjFuseMaxN = 128;
hipError_t launch_adjoint_step(int kind, const KParams& P, const AdjointStep& A, hipStream_t st);
// For each of `count` states (device array `states` of their fronts, n^2
// values each): the liquid counts (cnt), their min / max over the 5x5 columns
// around each column (cmin2, cmax2) and the largest count, merged into
// rmax[t], which must be zero.  The outputs of state t start at t n^2 and at
// rmax[t].
hipError_t launch_adj_partition(const KParams& P, const double* const* states, int count,
                                int* cnt, int* cmin2, int* cmax2, int* rmax, hipStream_t st);
hipError_t launch_fill(double* v, size_t count, double value, hipStream_t st);

// Bytes of one per-cell adjoint value for a storage kind, and a fill of such
// an array.
size_t lambda_bytes(int kind);
hipError_t launch_fill_lambda(int kind, void* v, size_t count, double value, hipStream_t st);

}  // namespace lbmk
