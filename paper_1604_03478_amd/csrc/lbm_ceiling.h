// Internal interface of the bandwidth-ceiling kernels (lbm_ceiling.hip), used
// by the host context (lbm_capi.hip) for measurement.  Not part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.h"

namespace lbmk {

// float4 copy of `bytes` (a multiple of 16) from src to dst.
hipError_t launch_copy4(const void* src, void* dst, uint64_t bytes, hipStream_t st);

// The bare access pattern of the all-liquid step (pulled loads and stores of
// every population, no arithmetic), in the step kernel's layout, launch shape
// and row order: (fs, gs) -> (fd, gd).  fs/fd are not touched when P.flow == 0.
hipError_t launch_pull_pattern(int kind, const KParams& P, const void* fs, void* fd,
                               const void* gs, void* gd, hipStream_t st);

}  // namespace lbmk
