// Diagnostics of the melting state on gfx950: the heated-wall Nusselt number
// and the FP64 reductions (mass, energy, fronts, phase switches).
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

// ---------------------------------------------------------------- reductions
// The FP64 diagnostics of the state in two deterministic passes.  Pass one:
// kDiagBlocks workgroups take the lattice rows r = b, b + B, ... (each
// thread the cells x = t, t + 256, ... of a row) and the columns
// c = 256 b + t, + 256 B, ...; each reduces its five sums (liquid mass,
// sum of T - t_m, sum of s, melted and frozen counts) in a fixed tree and
// writes them to part[k * B + b].  Pass two: one workgroup sums the B
// partials of each quantity in a fixed order into part[5 B + k].  No atomics:
// the result is the same bit for bit on every run.
constexpr int kDiagThreads = 256;

__device__ __forceinline__ double diag_block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();  // sh may still be read by the previous call
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kDiagThreads / 64; ++w) t += sh[w];
  return t;  // valid in thread 0
}

template <typename Ts, bool MZ>
__global__ __launch_bounds__(kDiagThreads) void k_diag_partial(
    const Ts* __restrict__ f, const Ts* __restrict__ g, const int* __restrict__ cnt,
    const double* __restrict__ s, const int* __restrict__ melted, const int* __restrict__ frozen,
    double* __restrict__ part, KParams P) {
  __shared__ double sh[kDiagThreads / 64];
  const int n = P.n, B = gridDim.x, b = blockIdx.x, t = threadIdx.x;
  const int rows = n * n;
  double mass = 0.0, energy = 0.0, fsum = 0.0, mel = 0.0, fro = 0.0;
  for (int r = b; r < rows; r += B) {
    const int y = r % n, z = r / n;
    const int a = MZ ? z : y, o = MZ ? y : z;
    const Ts* gr = row_ptr<7>(g, P, y, z);
    const Ts* fr = P.flow ? row_ptr<19>(f, P, y, z) : nullptr;
    for (int x = t; x < n; x += kDiagThreads) {
      double tt = 0.0;
#pragma unroll
      for (int q = 0; q < 7; ++q) tt += (double)load(gr, q * P.pitch + x);
      energy += tt + (P.tref - P.t_m);
      if (P.flow && a < cnt[o * n + x]) {
        double d = 0.0;
#pragma unroll
        for (int q = 0; q < 19; ++q) d += (double)load(fr, q * P.pitch + x);
        mass += 1.0 + d;
      }
    }
  }
  for (int c = b * kDiagThreads + t; c < rows; c += B * kDiagThreads) {
    fsum += s[c];
    mel += (double)melted[c];
    fro += (double)frozen[c];
  }
  const double v[5] = {mass, energy, fsum, mel, fro};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double tot = diag_block_sum(v[k], sh);
    if (t == 0) part[k * B + b] = tot;
  }
}

__global__ __launch_bounds__(kDiagThreads) void k_diag_final(double* __restrict__ part,
                                                             int nblocks) {
  __shared__ double sh[kDiagThreads / 64];
  for (int k = 0; k < 5; ++k) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += kDiagThreads) acc += part[k * nblocks + i];
    const double tot = diag_block_sum(acc, sh);
    if (threadIdx.x == 0) part[5 * nblocks + k] = tot;
  }
}

template <typename Ts>
hipError_t diag_dispatch(const KParams& P, const void* f, const void* g, const int* cnt,
                         const double* s, const int* melted, const int* frozen, double* part,
                         hipStream_t st) {
  const int nb = diag_blocks(P.n);
  const Ts* F = static_cast<const Ts*>(f);
  const Ts* G = static_cast<const Ts*>(g);
  if (P.melt_z)
    hipLaunchKernelGGL((k_diag_partial<Ts, true>), dim3(nb), dim3(kDiagThreads), 0, st, F, G, cnt,
                       s, melted, frozen, part, P);
  else
    hipLaunchKernelGGL((k_diag_partial<Ts, false>), dim3(nb), dim3(kDiagThreads), 0, st, F, G,
                       cnt, s, melted, frozen, part, P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kDiagThreads), 0, st, part, nb);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_diag_sums(int kind, const KParams& P, const void* f, const void* g,
                            const int* cnt, const double* s, const int* melted,
                            const int* frozen, double* part, hipStream_t st) {
  if (!g || !cnt || !s || !melted || !frozen || !part || (P.flow && !f))
    return hipErrorInvalidValue;
  switch (kind) {
    case kF64: return diag_dispatch<double>(P, f, g, cnt, s, melted, frozen, part, st);
    case kF32: return diag_dispatch<float>(P, f, g, cnt, s, melted, frozen, part, st);
    case kF16S: return diag_dispatch<_Float16>(P, f, g, cnt, s, melted, frozen, part, st);
    case kBF16S: return diag_dispatch<__bf16>(P, f, g, cnt, s, melted, frozen, part, st);
    default: return hipErrorInvalidValue;
  }
}

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
