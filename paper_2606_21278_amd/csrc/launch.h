// Host-side declarations of the kernel launchers (one translation unit per
// kernel family) used by the plan and API code.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"

namespace enufft {

template <typename T>
hipError_t launch_fwd(const FwdArgs<T> &a, int W, int blocks, int threads, size_t lds, hipStream_t s);
template <typename T>
hipError_t fwd_occupancy(int W, int threads, int pitch, int acc, size_t lds, int *blocks_per_cu);

template <typename T>
hipError_t launch_adj(const AdjArgs<T> &a, int W, int blocks, int threads, size_t lds, hipStream_t s);
template <typename T>
hipError_t adj_occupancy(int W, int threads, size_t lds, int *blocks_per_cu);

// Per-wave queue of deferred point groups in the forward kernel (entries).
constexpr int FWD_QCAP = 128;
// Row pitch of the 128-wide fine grid (64-mode boxes at sigma 2), for which
// the FP32 forward kernel is compiled with the pitch as a constant.
constexpr int FWD_PITCH128 = 130;

// Pitch argument that selects the forward build: FWD_PITCH128 for the
// constant-pitch polynomial build, FWD_POLY_ANY for the polynomial build with
// the pitch read at run time, 0 for the general one (exact kernel or
// polynomial, chosen at run time).
constexpr int FWD_POLY_ANY = -1;
inline int fwd_variant_pitch(const Geom &g, const EsPoly &es) {
  if (!es.on) return 0;
  return g.pitch == FWD_PITCH128 ? FWD_PITCH128 : FWD_POLY_ANY;
}

// LDS bytes of the forward kernel: the spread grid (acc = 8 or 4 bytes per
// cell) with W wrap rows (a merged run of points spans up to W + 1 rows), then
// one deferred-group queue per wave.
__host__ __device__ inline size_t fwd_grid_bytes(const Geom &g, int W, size_t acc) {
  return ((size_t)(g.n2 + W) * g.pitch * acc + 15) / 16 * 16;
}
inline size_t fwd_lds_bytes(const Geom &g, int W, int threads, size_t acc) {
  return fwd_grid_bytes(g, W, acc) + (size_t)(threads / 64) * FWD_QCAP * sizeof(int);
}

}  // namespace enufft
