// Internal plan state of the ENUFFT library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/enufft.h"
#include "device_common.h"

namespace enufft {

struct Timing {
  std::vector<hipEvent_t> start, stop;
  std::vector<int> kind;           // 0 type-1, 1 EMS, 2 adjoint
};

struct UnitTable {                 // EMS units for one (use_pairs, exclude_dc) choice
  bool built = false;
  int32_t J = 0;                   // number of units
  int32_t Jpad = 0;                // power of two >= J used by the in-LDS sort
  int2 *d_units = nullptr;         // (rep, partner or -1), ascending unit id
};

}  // namespace enufft

struct enufft_plan_s {
  // configuration
  int64_t n_cells = 0, n_points = 0;
  int N1 = 0, N2 = 0, n1 = 0, n2 = 0, W = 0;
  double beta = 0.0, sigma = 2.0, eps = 1e-5, scale = 1.0;
  int prec = ENUFFT_F32, window_kind = ENUFFT_WIN_HANN_RADIAL;
  size_t elem = 4;
  hipStream_t stream = nullptr;
  int device = 0, n_cu = 0;
  enufft::Geom geom{};
  std::vector<int64_t> offsets;

  // forward schedule
  std::vector<enufft::FwdItem> fwd_items;        // descending size (batched launch)
  std::vector<enufft::FwdItem> fwd_items_cell;   // grouped by cell (per-cell loop)
  std::vector<int64_t> fwd_cell_first;           // per cell: first index in fwd_items_cell (+ n_cells sentinel)
  int64_t n_slots = 0, n_split = 0;
  int fwd_threads = 512, fwd_blocks = 0;
  size_t fwd_lds = 0;

  // adjoint schedule
  std::vector<enufft::AdjItem> adj_items;
  int adj_bands = 1, adj_band_rows = 0;
  int adj_threads = 512, adj_blocks = 0;
  size_t adj_lds = 0;

  // device memory
  void *d_windows = nullptr;
  void *d_fwd_items = nullptr, *d_fwd_items_cell = nullptr, *d_adj_items = nullptr;
  int *d_counters = nullptr;       // [0] fwd work, [1] fwd done, [2] adj work, [3] adj done
  int *d_cell_counters = nullptr;
  void *d_partial = nullptr;
  void *d_decon_x = nullptr, *d_decon_y = nullptr, *d_tw1 = nullptr, *d_tw2 = nullptr;
  enufft::EsPoly es{};             // FP32 plans: kernel polynomial coefficients (es.on = 0: exact)
  double es_poly_err = 0.0;        // max |poly - psi| over the fit interval
  enufft::UnitTable units[2][2];
  int64_t workspace_bytes = 0;
  std::vector<void *> allocations;

  // state
  bool faulted = false;
  std::string last_error;
  bool timing = false;
  enufft::Timing tim;
};
