// Host-side declarations of the kernel launchers (one translation unit per
// kernel family) used by the plan and API code.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"

namespace enufft {

template <typename T>
hipError_t launch_fwd(const FwdArgs<T> &a, int W, int blocks, int threads, size_t lds, hipStream_t s);
template <typename T>
hipError_t fwd_occupancy(int W, int threads, size_t lds, int *blocks_per_cu);

template <typename T>
hipError_t launch_adj(const AdjArgs<T> &a, int W, int blocks, int threads, size_t lds, hipStream_t s);
template <typename T>
hipError_t adj_occupancy(int W, int threads, size_t lds, int *blocks_per_cu);

// LDS bytes of the forward kernel: the FP64 spread grid with W wrap rows
// (a merged run of points spans up to W + 1 rows).
inline size_t fwd_lds_bytes(const Geom &g, int W) {
  return (size_t)(g.n2 + W) * g.pitch * sizeof(double);
}

}  // namespace enufft
