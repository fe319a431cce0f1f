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
  int32_t Jpad = 0;                // power of two >= max(J, 64): the in-register sort size
  int2 *d_units = nullptr;         // (rep, partner or -1), ascending unit id
  int4 *d_mode_unit = nullptr;     // [M]: (rep, partner, unit id, 0) of each mode's unit, rep -1: none
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
  enufft_opts opts{};              // as given to enufft_plan
  std::vector<enufft_window> windows_host;

  // launch-shape parameters (defaults, or chosen by the autotuner)
  int64_t fwd_chunk_min = 16384;   // smallest forward work item (points)
  int fwd_items_per_slot = 2;      // target forward items per resident workgroup
  int adj_items_per_slot = 2;      // same for the adjoint
  int adj_band_mult = 1;           // adjoint bands = mult x the fewest that fit LDS
  int fwd_acc = 8;                 // bytes per forward LDS grid cell: 8 (FP64 sums) or 4 (FP32 sums)
  bool tuned = false, tune_cache_hit = false;
  double tune_fwd_ms = 0.0, tune_adj_ms = 0.0;   // best trial times (ms)

  // forward schedule
  std::vector<enufft::FwdItem> fwd_items;        // descending size (batched launch)
  std::vector<enufft::FwdItem> fwd_items_cell;   // per-cell loop: each cell split over the resident workgroups
  std::vector<int64_t> fwd_cell_first;           // per cell: first index in fwd_items_cell (+ n_cells sentinel)
  int64_t n_slots = 0, n_split = 0;              // batched schedule: partial slots, split cells
  int64_t n_partial = 0;                         // partial grids held: max(batched slots, per-cell chunks)
  int fwd_threads = 512, fwd_blocks = 0, fwd_slots = 0;
  size_t fwd_lds = 0;

  // single-grid adjoint (FP32 plans, kernel width W + 2 <= 8): one LDS grid of the cell with
  // value and derivative taps of its own, wider kernel (adj1_W, adj1_beta) and tables
  bool adj1 = false;                 // in use (the autotuner may choose the banded adjoint instead)
  bool adj1_avail = false;           // its kernel and tables are set up
  int adj1_W = 0;
  double adj1_beta = 0.0;
  enufft::EsPoly adj1_es{};        // taps (their derivatives d/dt come from the same polynomials)
  double adj1_poly_err = 0.0, adj1_dpoly_err = 0.0;
  void *d_adj1_decon_x = nullptr, *d_adj1_decon_y = nullptr;
  std::vector<enufft::AdjItem> adj1_items;
  void *d_adj1_items = nullptr;
  int adj1_threads = 512, adj1_blocks = 0;
  size_t adj1_lds = 0;

  // adjoint schedule (also used by the reconstruction diagnostics)
  std::vector<enufft::AdjItem> adj_items;
  void *d_rec_part = nullptr;        // [items][3] doubles: per-item reconstruction sums
  void *d_cell_items = nullptr;      // int32 item indices grouped by cell (ascending)
  void *d_cell_item_off = nullptr;   // int64 [n_cells + 1] offsets into d_cell_items
  void *d_cell_off = nullptr;        // int64 [n_cells + 1] the plan's cell offsets
  int32_t *d_sort_perm = nullptr;    // [n_points] enufft_sort_points' permutation when the caller asks for none
  void *d_sort_rec = nullptr;        // [n_points] enufft_sort_points' interleaved (x, y, h, w) records
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
  void *d_decon_x1 = nullptr;      // 1 / p_x(|k|) without the plan's scale (reconstruction)
  enufft::EsPoly es{};             // FP32 plans: kernel polynomial coefficients (es.on = 0: exact)
  enufft::EsPoly64 es64{};         // FP64 large-cell plans: the same in FP64 (es64.on = 0: exact)
  double es_poly_err = 0.0;        // max |poly - psi| over the fit interval
  enufft::UnitTable units[2][2];
  int64_t workspace_bytes = 0;
  std::vector<void *> allocations;

  // large-cell path: fine grid in HBM, points sorted by tile (mode boxes above 64 per axis)
  bool big = false;
  int big_ntx = 0, big_nty = 0;              // tiles per axis
  int *big_chunk_hist = nullptr;             // [chunks][tiles] counts, then chunk starts in each tile
  int *big_group_sum = nullptr;              // [chunk groups][tiles]
  int64_t *big_offsets = nullptr;            // [tiles + 1] tile ranges of the sorted order
  int *big_unit_base = nullptr;              // [tiles + 1] first work unit of each tile
  int *big_inv = nullptr;                    // [largest cell] sorted position of each input point
  int *big_chunk_fl = nullptr;               // [chunks][4] first and last key, descent flags of each sort chunk
  int *big_flags = nullptr;                  // [0]: the current cell's input is in tile order, [1]: and by cell
  // enufft_bind_points: coordinate arrays bound in tile order (large cells) and,
  // per cell, their tile ranges, unit offsets and order flags
  const void *bound_x = nullptr, *bound_y = nullptr;
  int64_t *bound_offsets = nullptr;          // [cells][tiles + 1]
  int *bound_unit_base = nullptr;            // [cells][tiles + 1]
  int *bound_flags = nullptr;                // [cells][4]
  int64_t bound_cap = 0;                     // cells the bound arrays hold
  void *big_xs = nullptr, *big_ys = nullptr, *big_hs = nullptr, *big_ws = nullptr;
  double *big_partial = nullptr;             // [units][S x S] FP64 sub-grids of the spreading units
  int64_t big_units_max = 0;
  void *big_gout = nullptr;                  // [largest cell] gradients in sorted order (4-vectors)
  double *big_grid = nullptr;                // n2 x n1 FP64 spreading grid
  void *big_cb = nullptr, *big_cby = nullptr;   // column buffers [K1 + 1][n2] complex
  void *big_gu = nullptr;                    // adjoint grids: n2 x n1 cells of (u, du/dx, du/dy, 0)
  int *big_work = nullptr;                   // persistent-loop counters
  double *big_sort = nullptr;                // EMS sort buffer, partials, cut record, tie flags
  int64_t big_sort_jpad = 0, big_ems_parts = 0;

  // cell geometry (Voronoi weights): sorted sample copy (double2) and index + slot (2 x int32)
  void *geo_ws = nullptr, *geo_ws_i = nullptr;
  int64_t geo_ws_points = 0;
  void *cell_order = nullptr;      // int32 cells, largest first (geometry)

  // captured forward (type-1 + EMS) graph and the arguments it was captured with
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<uint8_t> graph_key;
  int64_t graph_launches = 0, graph_captures = 0;

  // state
  bool faulted = false;
  std::string last_error;
  bool timing = false;
  enufft::Timing tim;
};

namespace enufft {
// Kernel arguments of the batched forward for plan p (defined with the plan).
template <typename T>
FwdArgs<T> make_fwd_args(enufft_plan_t p, const void *x, const void *y, const void *h, const void *w, void *f);
enufft_status check_plan(enufft_plan_t p, const char *fn);
// Workspace helpers shared by the translation units (defined with the plan).
void dev_release(enufft_plan_t p, void **ptr, size_t bytes);
enufft_status install_fwd_schedule(enufft_plan_t p);
enufft_status set_fwd_threads(enufft_plan_t p, int threads, size_t lds_limit);
void adj_reset(enufft_plan_t p);
enufft_status autotune(enufft_plan_t p);
// Device array of the cells ordered by point count, largest first (built once).
enufft_status cells_largest_first(enufft_plan_t p, const int32_t **order);
enufft_status ems_units(enufft_plan_t p, const enufft_ems_params *prm, UnitTable **ut);
// Large-cell path (fine grid in HBM).
enufft_status big_prepare(enufft_plan_t p);
enufft_status big_type1(enufft_plan_t p, const void *x, const void *y, const void *h, const void *w, void *f,
                        int64_t c0, int64_t c1);
enufft_status big_adjoint(enufft_plan_t p, const void *x, const void *y, const void *h, const void *w,
                          const void *fin, const uint8_t *keep, const double *lam, void *gh, void *gx, void *gy);
enufft_status big_bind_points(enufft_plan_t p, const void *x, const void *y);
enufft_status big_sort_points(enufft_plan_t p, const void *x, const void *y, const void *h, const void *w, void *xs,
                              void *ys, void *hs, void *ws, int32_t *perm);
enufft_status big_ems(enufft_plan_t p, const void *f, const enufft_ems_params *prm, const double *mode_weight,
                      uint8_t *keep, int32_t *k_star, double *stats, const UnitTable *ut, int64_t cell_begin,
                      int64_t cell_count);
}  // namespace enufft
