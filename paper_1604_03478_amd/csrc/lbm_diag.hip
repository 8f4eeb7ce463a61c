// Diagnostics of the melting state on gfx950.
//
// Heated-wall Nusselt number: the paper shows its distribution over the hot
// wall (section 3.2, Fig. 4(b) for case 1, Fig. 5(b) for case 2) without
// defining it.  Here Nu = -H (dT/da)(a = 0) / (t_h - t_m) with H = n and a the
// melt-axis coordinate: the temperature gradient at the wall, in units of the
// conduction gradient across the cavity.  With the wall at a = 0 and cell
// centres at 1/2 and 3/2, the quadratic through (0, T_w), (1/2, T_0),
// (3/2, T_1) has slope (9 T_0 - T_1 - 8 T_w) / 3 at the wall.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.h"
#include "lbm_diag.h"
#include "lbm_internal.h"

namespace lbmk {
namespace {

// temperature of cell (x, y, z) from the stored (shifted) energy distribution
template <typename Ts>
__device__ __forceinline__ double temp_at(const Ts* g, const KParams& P, int x, int y, int z) {
  const Ts* row = row_ptr<7>(g, P, y, z);
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < 7; ++q) acc += (double)load(row, q * P.pitch + x);
  return acc + P.tref;
}

// one thread per column (x, o); a = melt-axis coordinate
template <typename Ts, bool MZ>
__global__ void k_wall_nusselt(const Ts* __restrict__ g, const double* __restrict__ s,
                               const double* __restrict__ th, double* __restrict__ nu,
                               KParams P) {
  const int n = P.n;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, o = blockIdx.y;
  if (x >= n) return;
  const int col = o * n + x;
  const double sc = s[col], Tw = th[col];
  double slope = 0.0;
  if (sc > 1.5) {  // both first centres liquid (liquid iff centre < s)
    const double T0 = MZ ? temp_at(g, P, x, o, 0) : temp_at(g, P, x, 0, o);
    const double T1 = MZ ? temp_at(g, P, x, o, 1) : temp_at(g, P, x, 1, o);
    slope = (9.0 * T0 - T1 - 8.0 * Tw) / 3.0;
  } else if (sc > 0.0) {
    slope = (P.t_m - Tw) / sc;
  }
  nu[col] = -(double)n * slope / P.dT;
}

template <typename Ts>
hipError_t nusselt_dispatch(const KParams& P, const void* g, const double* s, const double* th,
                            double* nu, hipStream_t st) {
  const dim3 block(64, 1, 1), grid((P.n + 63) / 64, P.n, 1);
  const Ts* G = static_cast<const Ts*>(g);
  if (P.melt_z)
    hipLaunchKernelGGL((k_wall_nusselt<Ts, true>), grid, block, 0, st, G, s, th, nu, P);
  else
    hipLaunchKernelGGL((k_wall_nusselt<Ts, false>), grid, block, 0, st, G, s, th, nu, P);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_wall_nusselt(int kind, const KParams& P, const void* g, const double* s,
                               const double* th, double* nu, hipStream_t st) {
  if (!g || !s || !th || !nu) return hipErrorInvalidValue;
  switch (kind) {
    case kF64: return nusselt_dispatch<double>(P, g, s, th, nu, st);
    case kF32: return nusselt_dispatch<float>(P, g, s, th, nu, st);
    case kF16S: return nusselt_dispatch<_Float16>(P, g, s, th, nu, st);
    case kBF16S: return nusselt_dispatch<__bf16>(P, g, s, th, nu, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lbmk
