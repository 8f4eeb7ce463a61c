// Conservative front update on gfx950: the energy balance at the interface
// (the one Eq. (6) expresses with temperature gradients) taken from the
// lattice's own heat flow.  The streaming moves every energy population to a
// neighbour, except across a link that crosses the front: there the
// population a cell sends toward the front is lost and the one it receives
// is set by the interpolated anti-bounce-back (wall value t_m).  The
// difference, summed over the links of a column's front, is the heat that
// column's front absorbed in the step; moving the front by heat / L with
// L = (t_h - t_m) / Ste keeps sum(T) + L sum(s) equal to the heat let in
// through the walls, to round-off.
//
// One thread per column gathers every link it is charged with (no atomics:
// the sums are deterministic): the link along the melt axis between its last
// liquid and first solid cell, and the lateral links of its solid cells that
// face a liquid cell of a neighbouring column (both sides of each).  All
// arithmetic is FP64 on the stored (shifted) populations; the shift cancels
// in sent - received because opposite directions share a weight.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.h"
#include "lbm_front_heat.h"
#include "lbm_internal.h"

namespace lbmk {
namespace {

template <typename Ts, bool MZ>
struct Cells {
  const Ts* g;
  const double* s;
  const int* cnt;
  const KParams& P;
  __device__ int col(int x, int y, int z) const { return (MZ ? y : z) * P.n + x; }
  __device__ int melt(int y, int z) const { return MZ ? z : y; }
  __device__ bool in(int x, int y, int z) const {
    const unsigned n = (unsigned)P.n;
    return (unsigned)x < n && (unsigned)y < n && (unsigned)z < n;
  }
  __device__ bool liquid(int x, int y, int z) const { return melt(y, z) < cnt[col(x, y, z)]; }
  __device__ double gv(int q, int x, int y, int z) const {
    return (double)load(row_ptr<7>(g, P, y, z), q * P.pitch + x);
  }
  // sent - received over the link of cell (x, y, z) whose incoming
  // direction q has its source across the front
  __device__ double link_heat(int x, int y, int z, int q) const {
    const int p = opp7(q);
    const int ex = ex7(q), ey = ey7(q), ez = ez7(q);
    const bool L = liquid(x, y, z);
    const double a = melt(y, z) + 0.5;
    const double sself = s[col(x, y, z)];
    const bool along = MZ ? (ez != 0) : (ey != 0);
    const double d = along ? fabs(sself - a)
                           : (a - sself) / (s[col(x - ex, y - ey, z - ez)] - sself);
    const double wTm = kW7Axis * (P.t_m - P.tref);
    const double gp = gv(p, x, y, z);
    double recv;
    if (d < 0.5) {
      const int bx = x + ex, by = y + ey, bz = z + ez;
      if (in(bx, by, bz) && liquid(bx, by, bz) == L)
        recv = -(2.0 * d * gp + (1.0 - 2.0 * d) * gv(p, bx, by, bz)) + 2.0 * wTm;
      else
        recv = -gp + 2.0 * wTm;
    } else {
      recv = -gp / (2.0 * d) + (2.0 * d - 1.0) / (2.0 * d) * gv(q, x, y, z) + wTm / d;
    }
    return gp - recv;
  }
};

template <typename Ts, bool MZ>
__global__ void k_front_heat(const Ts* __restrict__ g, const double* __restrict__ s,
                             const int* __restrict__ cnt, double* __restrict__ heat, KParams P) {
  const int n = P.n;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, o = blockIdx.y;
  if (x >= n) return;
  const Cells<Ts, MZ> C{g, s, cnt, P};
  const int c = o * n + x;
  const int cc = cnt[c];
  // cell of this column at height a
  auto Y = [&](int a) { return MZ ? o : a; };
  auto Z = [&](int a) { return MZ ? a : o; };
  // incoming directions along the melt axis: from above (source a + 1) and
  // from below (source a - 1)
  const int q_from_above = MZ ? 6 : 4, q_from_below = MZ ? 5 : 3;
  double Q = 0.0;
  if (cc >= 1 && cc <= n - 1) {
    Q += C.link_heat(x, Y(cc - 1), Z(cc - 1), q_from_above);  // last liquid cell
    Q += C.link_heat(x, Y(cc), Z(cc), q_from_below);          // first solid cell
  }
  // lateral neighbours: dx along x, or along the other lateral axis
  for (int j = 0; j < 4; ++j) {
    const int dx = j == 0 ? 1 : (j == 1 ? -1 : 0);
    const int dob = j == 2 ? 1 : (j == 3 ? -1 : 0);
    const int xn = x + dx, on = o + dob;
    if (xn < 0 || xn >= n || on < 0 || on >= n) continue;
    const int cn = cnt[on * n + xn];
    // the D3Q7 direction pointing from the neighbour to this column
    const int q_in = dx == 1 ? 2 : (dx == -1 ? 1 : (MZ ? (dob == 1 ? 4 : 3) : (dob == 1 ? 6 : 5)));
    for (int a = cc; a < cn; ++a) {  // solid here, liquid in the neighbour
      Q += C.link_heat(x, Y(a), Z(a), q_in);
      Q += C.link_heat(xn, MZ ? on : a, MZ ? a : on, opp7(q_in));
    }
  }
  heat[c] = Q;
}

template <typename Ts>
hipError_t heat_dispatch(const KParams& P, const void* g, const double* s, const int* cnt,
                         double* heat, hipStream_t st) {
  const dim3 block(64, 1, 1), grid((P.n + 63) / 64, P.n, 1);
  const Ts* G = static_cast<const Ts*>(g);
  if (P.melt_z)
    hipLaunchKernelGGL((k_front_heat<Ts, true>), grid, block, 0, st, G, s, cnt, heat, P);
  else
    hipLaunchKernelGGL((k_front_heat<Ts, false>), grid, block, 0, st, G, s, cnt, heat, P);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_front_heat(int kind, const KParams& P, const void* g, const double* s,
                             const int* cnt, double* heat, hipStream_t st) {
  if (!g || !s || !cnt || !heat) return hipErrorInvalidValue;
  switch (kind) {
    case kF64: return heat_dispatch<double>(P, g, s, cnt, heat, st);
    case kF32: return heat_dispatch<float>(P, g, s, cnt, heat, st);
    case kF16S: return heat_dispatch<_Float16>(P, g, s, cnt, heat, st);
    case kBF16S: return heat_dispatch<__bf16>(P, g, s, cnt, heat, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lbmk
