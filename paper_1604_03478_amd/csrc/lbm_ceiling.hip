// Bandwidth ceilings for the measurement of the step kernel (not part of the
// method): two data-movement kernels the benchmark times beside it.
//
//  * a float4 copy of one buffer into another, the simplest HBM-bound kernel
//    (one 16-byte load and one 16-byte store per lane);
//  * the bare access pattern of the fused step in the all-liquid state: for
//    every cell the 19 + 7 pulled loads of the row-interleaved layout (the
//    same source rows, x shifts and wall bounce-back address selects, and
//    off the y and z walls the fast path's uniform-base addressing) and the
//    19 + 7 non-temporal stores, with the step kernel's launch shape and the
//    row order it takes in that state, and no arithmetic at all.
//
// Both move exactly the bytes they are credited with; the step kernel's
// fraction of each tells how much of the gap to peak belongs to its access
// pattern rather than to its arithmetic.
#include <hip/hip_runtime.h>

#include "lbm_ceiling.h"
#include "lbm_device.h"

namespace lbmk {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy4(const f32x4* __restrict__ src,
                                               f32x4* __restrict__ dst, uint64_t count) {
  const uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  if (i < count) __builtin_nontemporal_store(src[i], &dst[i]);
}

// The pulled loads of one distribution with Q directions of cell (x, y, z):
// the source row (y - e_y, z - e_z) at x - e_x, or, where the source lies
// outside the box, the cell's own opposite direction (bounce-back).  Values
// go straight to the destination rows.
template <int Q, typename Ts>
__device__ __forceinline__ void move_pulled(const Ts* __restrict__ src, Ts* __restrict__ dst,
                                            const KParams& P, int x, int y, int z) {
  const int n = P.n;
  const uint32_t pitch = P.pitch;
  Ts v[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int ex = Q == 19 ? ex19(q) : ex7(q), ey = Q == 19 ? ey19(q) : ey7(q),
              ez = Q == 19 ? ez19(q) : ez7(q), p = Q == 19 ? opp19(q) : opp7(q);
    const int sy = y - ey, sz = z - ez, sx = x - ex;
    const bool row_in = (unsigned)sy < (unsigned)n && (unsigned)sz < (unsigned)n;  // uniform
    const bool in = row_in && (unsigned)sx < (unsigned)n;
    const Ts* row = row_in ? row_ptr<Q>(src, P, sy, sz) : row_ptr<Q>(src, P, y, z);
    const uint32_t i = in ? q * pitch + (uint32_t)sx : p * pitch + (uint32_t)x;
    const Ts* base = in ? row : row_ptr<Q>(src, P, y, z);
    v[q] = load_stream<Ts>(base, i);
  }
  Ts* out = row_ptr<Q>(dst, P, y, z);
#pragma unroll
  for (int q = 0; q < Q; ++q) __builtin_nontemporal_store(v[q], out + q * pitch + x);
}

// The same for a row off the y and z walls, addressed as the step kernel's
// fast path does: one uniform base (the row block's first row, y - 1, z - 1)
// and a 32-bit offset per lane and direction, the x-wall bounce-back an
// offset select.
template <int Q, typename Ts>
__device__ __forceinline__ void move_pulled_interior(const Ts* __restrict__ src,
                                                     Ts* __restrict__ dst, const KParams& P,
                                                     int x, int y, int z) {
  const int n = P.n;
  const uint32_t pitch = P.pitch, un = (uint32_t)n;
  const Ts* b = row_ptr<Q>(src, P, y - 1, z - 1);
  auto row_ofs = [&](int dy, int dz) {  // row (y + dy, z + dz)
    return ((uint32_t)(1 + dz) * un + (uint32_t)(1 + dy)) * ((uint32_t)Q * pitch);
  };
  Ts v[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int ex = Q == 19 ? ex19(q) : ex7(q), ey = Q == 19 ? ey19(q) : ey7(q),
              ez = Q == 19 ? ez19(q) : ez7(q), p = Q == 19 ? opp19(q) : opp7(q);
    uint32_t i = row_ofs(-ey, -ez) + q * pitch + (uint32_t)(x - ex);
    if (ex != 0) {
      const bool wall = ex > 0 ? (x == 0) : (x == n - 1);
      i = wall ? row_ofs(0, 0) + p * pitch + x : i;
    }
    v[q] = load_stream<Ts>(b, i);
  }
  Ts* out = row_ptr<Q>(dst, P, y, z);
#pragma unroll
  for (int q = 0; q < Q; ++q) __builtin_nontemporal_store(v[q], out + q * pitch + x);
}

template <typename Ts, bool PAIR>
__global__ __launch_bounds__(512) void k_pull_pattern(const Ts* __restrict__ fs,
                                                      Ts* __restrict__ fd,
                                                      const Ts* __restrict__ gs,
                                                      Ts* __restrict__ gd, KParams P) {
  int y, z, xb;
  step_row<row_run<Ts>(), PAIR>(P, y, z, xb);
  const int x = xb * blockDim.x + threadIdx.x;
  if (x >= P.n) return;
  if (y >= 1 && y <= P.n - 2 && z >= 1 && z <= P.n - 2) {  // uniform
    move_pulled_interior<7>(gs, gd, P, x, y, z);
    if (P.flow) move_pulled_interior<19>(fs, fd, P, x, y, z);
    return;
  }
  move_pulled<7>(gs, gd, P, x, y, z);
  if (P.flow) move_pulled<19>(fs, fd, P, x, y, z);
}

template <typename Ts>
hipError_t pattern_dispatch(const KParams& P, const void* fs, void* fd, const void* gs, void* gd,
                            hipStream_t st) {
  // the step kernel's launch: one x row per workgroup, split as the step
  // kernel splits it, and for 16-bit storage at two workgroups per row the
  // order the host picks for a mostly liquid lattice (both halves of a row
  // on one XCD)
  const int bmax = step_block_max(sizeof(Ts));
  const int bx = P.n >= bmax ? bmax : ((P.n + 63) / 64) * 64;
  const dim3 grid((P.n + bx - 1) / bx, P.n, P.n);
  const bool pair = sizeof(Ts) == 2 && grid.x == 2 && (P.n & 7) == 0;
  if (pair)
    hipLaunchKernelGGL((k_pull_pattern<Ts, true>), grid, dim3(bx), 0, st, static_cast<const Ts*>(fs),
                       static_cast<Ts*>(fd), static_cast<const Ts*>(gs), static_cast<Ts*>(gd), P);
  else
    hipLaunchKernelGGL((k_pull_pattern<Ts, false>), grid, dim3(bx), 0, st,
                       static_cast<const Ts*>(fs), static_cast<Ts*>(fd),
                       static_cast<const Ts*>(gs), static_cast<Ts*>(gd), P);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_copy4(const void* src, void* dst, uint64_t bytes, hipStream_t st) {
  const uint64_t count = bytes / 16;
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy4, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                     static_cast<const f32x4*>(src), static_cast<f32x4*>(dst), count);
  return hipGetLastError();
}

hipError_t launch_pull_pattern(int kind, const KParams& P, const void* fs, void* fd,
                               const void* gs, void* gd, hipStream_t st) {
  switch (kind) {
    case kF64: return pattern_dispatch<double>(P, fs, fd, gs, gd, st);
    case kF32: return pattern_dispatch<float>(P, fs, fd, gs, gd, st);
    case kF16S: return pattern_dispatch<_Float16>(P, fs, fd, gs, gd, st);
    case kBF16S: return pattern_dispatch<__bf16>(P, fs, fd, gs, gd, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lbmk
