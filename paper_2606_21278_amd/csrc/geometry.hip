// Per-cell geometry of a triangular mesh (enufft_cell_geometry): local frames
// and the square spectral box of Appendix A1, the square / triangle / circle
// support masks, uniform or raster-Voronoi quadrature weights (Appendix A2,
// eqs. uniform_weights, raster_grid .. voronoi_weights) and deplaning by the
// weighted cell mean (Appendix A6, eq. alps_deplaning).
//
// One workgroup per cell.  Phases, separated by workgroup barriers:
//   0  thread 0: centroid, rotation, rotated vertices, H and the mask area;
//   1  every sample: local and box coordinates, the mask flag; with Voronoi
//      weights also its bin in an nb x nb grid over the box (LDS counters) and
//      its slot in that bin;
//   2  exclusive scan of the bin counters (LDS);
//   3  inside samples scattered by bin into a workspace copy (u_x, u_y, index);
//   4  every raster cell centre inside the mask finds its nearest inside
//      sample by rings of bins around its own, stopping once no farther bin
//      can hold a sample as near; the sample's count is incremented;
//   5  weights, their FP64 sum and the weighted mean; deplaned heights.
// Decisions that yield integers (mask flags, nearest samples) use FP64 with
// contraction off, so they are exact functions of the FP64 inputs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "plan.h"

namespace enufft {
namespace {

constexpr int kGeoThreads = 512;
constexpr int kGeoMaxBins = 128;                 // bins per axis

struct GeoParams {
  int frame, mask, weights, raster, deplane;
  double eta, floor_frac;
};

struct GeoFrame {
  double cx, cy, cs, sn, H, area;
  double ut[6];                                   // rotated vertices
};

// Sutherland-Hodgman: the rotated triangle cut by the four half-planes of the
// box [-H, H]^2, then the shoelace area of what is left.
__device__ double tri_box_area(const double *ut, double H) {
#pragma clang fp contract(off)
  double ax[10], ay[10], bx[10], by[10];
  int n = 3;
  for (int i = 0; i < 3; ++i) { ax[i] = ut[2 * i]; ay[i] = ut[2 * i + 1]; }
  for (int side = 0; side < 4; ++side) {
    const bool on_y = side >= 2;
    const double s = (side & 1) ? -1.0 : 1.0;
    int m = 0;
    for (int i = 0; i < n; ++i) {
      const int k = (i + 1 == n) ? 0 : i + 1;
      const double pa = s * (on_y ? ay[i] : ax[i]) - H;
      const double pb = s * (on_y ? ay[k] : ax[k]) - H;
      if (pa <= 0.0) { bx[m] = ax[i]; by[m] = ay[i]; ++m; }
      if ((pa < 0.0 && pb > 0.0) || (pa > 0.0 && pb < 0.0)) {
        const double t = pa / (pa - pb);
        bx[m] = ax[i] + t * (ax[k] - ax[i]);
        by[m] = ay[i] + t * (ay[k] - ay[i]);
        ++m;
      }
    }
    n = m;
    for (int i = 0; i < n; ++i) { ax[i] = bx[i]; ay[i] = by[i]; }
  }
  double s2 = 0.0;
  for (int i = 0; i < n; ++i) {
    const int k = (i + 1 == n) ? 0 : i + 1;
    s2 += ax[i] * ay[k] - ax[k] * ay[i];
  }
  return 0.5 * fabs(s2);
}

__device__ void make_frame(const double *v, const GeoParams &g, GeoFrame &F) {
#pragma clang fp contract(off)
  F.cx = (v[0] + v[2] + v[4]) / 3.0;
  F.cy = (v[1] + v[3] + v[5]) / 3.0;
  double cs = 1.0, sn = 0.0;
  if (g.frame == ENUFFT_FRAME_EDGE) {
    // edges v2 - v1, v3 - v2, v1 - v3; the first of the longest
    double best = -1.0, ex = 0.0, ey = 0.0;
    for (int i = 0; i < 3; ++i) {
      const int k = (i + 1) % 3;
      const double dx = v[2 * k] - v[2 * i], dy = v[2 * k + 1] - v[2 * i + 1];
      const double len = sqrt(dx * dx + dy * dy);
      if (len > best) { best = len; ex = dx; ey = dy; }
    }
    cs = ex / best;
    sn = ey / best;
  }
  F.cs = cs;
  F.sn = sn;
  double lo_x = 0.0, hi_x = 0.0, lo_y = 0.0, hi_y = 0.0;
  for (int i = 0; i < 3; ++i) {
    const double dx = v[2 * i] - F.cx, dy = v[2 * i + 1] - F.cy;
    const double ux = cs * dx + sn * dy, uy = -sn * dx + cs * dy;
    F.ut[2 * i] = ux;
    F.ut[2 * i + 1] = uy;
    lo_x = i ? fmin(lo_x, ux) : ux;
    hi_x = i ? fmax(hi_x, ux) : ux;
    lo_y = i ? fmin(lo_y, uy) : uy;
    hi_y = i ? fmax(hi_y, uy) : uy;
  }
  F.H = 0.5 * g.eta * fmax(hi_x - lo_x, hi_y - lo_y);
  if (g.mask == ENUFFT_MASK_SQUARE) F.area = 4.0 * F.H * F.H;
  else if (g.mask == ENUFFT_MASK_CIRCLE) F.area = M_PI * F.H * F.H;
  else F.area = tri_box_area(F.ut, F.H);
}

// Mask membership of a local point.  The triangle test takes the orientation
// of the point against each edge traversed v2 -> v1, v3 -> v2, v1 -> v3 (base
// at the edge's start); on the triangle when no two orientations have opposite
// signs.
__device__ bool in_support(const GeoFrame &F, int mask, double ux, double uy) {
#pragma clang fp contract(off)
  const double H = F.H;
  if (mask == ENUFFT_MASK_CIRCLE) return ux * ux + uy * uy <= H * H;
  if (!(fabs(ux) <= H && fabs(uy) <= H)) return false;
  if (mask == ENUFFT_MASK_SQUARE) return true;
  const double *t = F.ut;
  bool neg = false, pos = false;
  for (int e = 0; e < 3; ++e) {
    const int s = (e + 1) % 3, d = e;          // start vertex s, end vertex d
    const double o = (ux - t[2 * s]) * (t[2 * d + 1] - t[2 * s + 1]) - (t[2 * d] - t[2 * s]) * (uy - t[2 * s + 1]);
    neg = neg || (o < 0.0);
    pos = pos || (o > 0.0);
  }
  return !(neg && pos);
}

__device__ inline void to_local(const GeoFrame &F, double x, double y, double &ux, double &uy) {
#pragma clang fp contract(off)
  const double dx = x - F.cx, dy = y - F.cy;
  ux = F.cs * dx + F.sn * dy;
  uy = -F.sn * dx + F.cs * dy;
}

__device__ inline int bin_of(double u, double H, double inv_bw, int nb) {
  const int b = (int)floor((u + H) * inv_bw);
  return b < 0 ? 0 : (b >= nb ? nb - 1 : b);
}

// Workgroup sum of one double per thread (tree in LDS; fixed order).
__device__ double wg_sum(double v, double *red) {
  const int t = threadIdx.x;
  __syncthreads();
  red[t] = v;
  __syncthreads();
  for (int s = kGeoThreads / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  return red[0];
}

// Persistent workgroups take cells from a counter, largest cells first (the order
// array), so the largest cells do not end the launch alone; each workgroup keeps
// its Voronoi workspace in its own slice (the size of the largest cell).
template <typename T>
__global__ void __launch_bounds__(kGeoThreads) geometry_kernel(
    GeoParams g, const int32_t *__restrict__ order, int64_t n_cells, int *counter, int *done, int64_t slice,
    const int64_t *__restrict__ off, const double *__restrict__ tri,
    const T *__restrict__ x, const T *__restrict__ y, const T *__restrict__ h, T *__restrict__ xb,
    T *__restrict__ yb, T *__restrict__ hb, T *__restrict__ wb, uint8_t *__restrict__ inside,
    double *__restrict__ info, int32_t *__restrict__ counts, double2 *__restrict__ ws_u,
    int32_t *__restrict__ ws_idx, int32_t *__restrict__ ws_slot) {
#pragma clang fp contract(off)
  extern __shared__ __align__(16) unsigned char geo_lds[];
  __shared__ GeoFrame F;
  __shared__ double red[kGeoThreads];
  __shared__ int part[kGeoThreads];
  __shared__ int qin_s, ng_s, s_idx;
  int *bins = reinterpret_cast<int *>(geo_lds);   // [nb * nb + 1] (Voronoi only)

  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * slice;   // this workgroup's workspace slice
  for (;;) {
  if (t == 0) s_idx = atomicAdd(counter, 1);
  __syncthreads();
  const int64_t idx = s_idx;
  __syncthreads();
  if (idx >= n_cells) break;
  const int64_t c = order[idx];
  const int64_t a = off[c], b = off[c + 1];
  const int64_t Q = b - a;
  const bool vor = g.weights == ENUFFT_WEIGHTS_VORONOI;
  const int nb = vor ? (int)min<int64_t>(kGeoMaxBins, max<int64_t>(1, (int64_t)sqrt((double)Q / 3.0))) : 1;
  const int nbin = nb * nb;

  if (t == 0) {
    make_frame(tri + 6 * c, g, F);
    qin_s = 0;
    ng_s = 0;
  }
  if (vor)
    for (int i = t; i <= nbin; i += kGeoThreads) bins[i] = 0;
  __syncthreads();
  const double H = F.H;
  const double inv_bw = (double)nb / (2.0 * H);

  // phase 1: coordinates, mask flags, bin slots
  int my_in = 0;
  for (int64_t j = a + t; j < b; j += kGeoThreads) {
    double ux, uy;
    to_local(F, (double)x[j], (double)y[j], ux, uy);
    const bool in = in_support(F, g.mask, ux, uy);
    xb[j] = (T)(ux * M_PI / H);
    yb[j] = (T)(uy * M_PI / H);
    if (inside) inside[j] = in ? 1 : 0;
    if (counts) counts[j] = 0;
    my_in += in ? 1 : 0;
    if (vor && in) {
      const int bi = bin_of(uy, H, inv_bw, nb) * nb + bin_of(ux, H, inv_bw, nb);
      ws_slot[base + (j - a)] = atomicAdd(&bins[bi], 1);
    }
  }
  if (my_in) atomicAdd(&qin_s, my_in);
  __syncthreads();
  const int64_t qin = qin_s;

  if (vor && qin > 0) {
    // phase 2: exclusive scan of the bin counters
    const int per = (nbin + kGeoThreads - 1) / kGeoThreads;
    const int lo = min(nbin, t * per), hi = min(nbin, lo + per);
    int s = 0;
    for (int i = lo; i < hi; ++i) s += bins[i];
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < kGeoThreads; o <<= 1) {
      const int v = t >= o ? part[t - o] : 0;
      __syncthreads();
      part[t] += v;
      __syncthreads();
    }
    int run = part[t] - s;
    for (int i = lo; i < hi; ++i) {
      const int cnt = bins[i];
      bins[i] = run;
      run += cnt;
    }
    if (t == kGeoThreads - 1) bins[nbin] = part[t];
    __syncthreads();

    // phase 3: scatter the inside samples by bin
    for (int64_t j = a + t; j < b; j += kGeoThreads) {
      double ux, uy;
      to_local(F, (double)x[j], (double)y[j], ux, uy);
      if (!in_support(F, g.mask, ux, uy)) continue;
      const int bi = bin_of(uy, H, inv_bw, nb) * nb + bin_of(ux, H, inv_bw, nb);
      const int64_t pos = base + bins[bi] + ws_slot[base + (j - a)];
      ws_u[pos] = make_double2(ux, uy);
      ws_idx[pos] = (int32_t)(j - a);
    }
    __syncthreads();

    // phase 4: nearest inside sample of every raster cell centre in the mask
    int32_t *cnt = counts ? counts + a : ws_slot + base;   // ws_slot is free again after phase 3
    if (!counts) {
      __syncthreads();
      for (int64_t j = t; j < Q; j += kGeoThreads) cnt[j] = 0;
    }
    __syncthreads();
    const int Ng = g.raster;
    const double step = 2.0 * H / Ng;
    const double bw = 2.0 * H / nb;
    int my_ng = 0;
    for (int64_t r = t; r < (int64_t)Ng * Ng; r += kGeoThreads) {
      const int ia = (int)(r % Ng), ib = (int)(r / Ng);
      const double gx = -H + step * (ia + 0.5);
      const double gy = -H + step * (ib + 0.5);
      if (!in_support(F, g.mask, gx, gy)) continue;
      ++my_ng;
      const int bx = bin_of(gx, H, inv_bw, nb), by = bin_of(gy, H, inv_bw, nb);
      int arg = -1;
      double bd = 0.0;
      for (int ring = 0; ring < nb; ++ring) {
        const int y0 = by - ring, y1 = by + ring;
        for (int yy = max(0, y0); yy <= min(nb - 1, y1); ++yy) {
          const bool edge_row = (yy == y0 || yy == y1);
          const int xstep = edge_row ? 1 : 2 * ring;
          for (int xx = bx - ring; xx <= bx + ring; xx += (xstep > 0 ? xstep : 1)) {
            if (xx < 0 || xx >= nb) continue;
            const int bi = yy * nb + xx;
            for (int p = bins[bi]; p < bins[bi + 1]; ++p) {
              const double2 u = ws_u[base + p];
              const double d = (u.x - gx) * (u.x - gx) + (u.y - gy) * (u.y - gy);
              const int id = ws_idx[base + p];
              if (arg < 0 || d < bd || (d == bd && id < arg)) {
                bd = d;
                arg = id;
              }
            }
          }
        }
        // every bin beyond this ring is more than ring * bw away (less a margin
        // for the rounding of the bin index)
        if (arg >= 0) {
          const double lim = (double)ring * bw * (1.0 - 1e-9);
          if (bd < lim * lim) break;
        }
      }
      atomicAdd(&cnt[arg], 1);
    }
    if (my_ng) atomicAdd(&ng_s, my_ng);
    __syncthreads();
    const int64_t ng = ng_s;

    // phase 5: areas, their sum, the normalised weights
    double my_tot = 0.0;
    for (int64_t j = a + t; j < b; j += kGeoThreads) {
      double ux, uy;
      to_local(F, (double)x[j], (double)y[j], ux, uy);
      double A = 0.0;
      if (in_support(F, g.mask, ux, uy) && ng > 0) {
        const int n = cnt[j - a];
        A = F.area * (n > 0 ? (double)n : g.floor_frac) / (double)ng;
      }
      my_tot += A;
      ws_u[base + (j - a)].x = A;   // the areas reuse the (now consumed) sorted copy
    }
    const double tot = wg_sum(my_tot, red);
    for (int64_t j = a + t; j < b; j += kGeoThreads) {
      const double A = ws_u[base + (j - a)].x;
      wb[j] = (T)(tot > 0.0 ? A / tot : 0.0);
      ws_u[base + (j - a)].y = tot > 0.0 ? A / tot : 0.0;
    }
  } else {
    for (int64_t j = a + t; j < b; j += kGeoThreads) {
      double ux, uy;
      to_local(F, (double)x[j], (double)y[j], ux, uy);
      const bool in = in_support(F, g.mask, ux, uy);
      const double wq = (!vor && in) ? 1.0 / (double)qin : 0.0;
      wb[j] = (T)wq;
      if (vor) ws_u[base + (j - a)].y = 0.0;
    }
  }

  // phase 6: weighted mean and deplaning
  double my_h = 0.0;
  for (int64_t j = a + t; j < b; j += kGeoThreads) {
    double wq;
    if (vor) {
      wq = ws_u[base + (j - a)].y;
    } else {
      double ux, uy;
      to_local(F, (double)x[j], (double)y[j], ux, uy);
      wq = in_support(F, g.mask, ux, uy) ? 1.0 / (double)qin : 0.0;
    }
    my_h += wq * (double)h[j];
  }
  const double hbar = wg_sum(my_h, red);
  for (int64_t j = a + t; j < b; j += kGeoThreads) hb[j] = (T)(g.deplane ? (double)h[j] - hbar : (double)h[j]);
  if (t == 0 && info) {
    double *ci = info + 8 * c;
    ci[0] = F.cx; ci[1] = F.cy; ci[2] = F.cs; ci[3] = F.sn;
    ci[4] = F.H; ci[5] = F.area; ci[6] = (double)qin; ci[7] = g.deplane ? hbar : 0.0;
  }
  __syncthreads();   // the frame, bins and sums are the next cell's
  }
  if (t == 0) {
    __threadfence();
    if (atomicAdd(done, 1) == (int)gridDim.x - 1) {   // the last workgroup resets the counters
      *counter = 0;
      *done = 0;
    }
  }
}

}  // namespace
}  // namespace enufft

namespace enufft {
namespace {

// Bins per axis of a cell of Q samples (the kernel's rule).
int geo_bins(int64_t Q) {
  return (int)std::min<int64_t>(kGeoMaxBins, std::max<int64_t>(1, (int64_t)std::sqrt((double)Q / 3.0)));
}

// Workspace allocation recorded in the plan (released with the plan or by dev_release).
enufft_status geo_alloc(enufft_plan_t p, void **d, size_t bytes, const char *what) {
  hipError_t e = hipMalloc(d, std::max<size_t>(16, bytes));
  if (e != hipSuccess) {
    *d = nullptr;
    p->last_error = std::string("enufft_cell_geometry: ") + what + " allocation failed";
    return ENUFFT_ENOMEM;
  }
  p->allocations.push_back(*d);
  p->workspace_bytes += (int64_t)std::max<size_t>(16, bytes);
  return ENUFFT_OK;
}

enufft_status geo_fail(enufft_plan_t p, enufft_status st, const std::string &msg) {
  p->last_error = "enufft_cell_geometry: " + msg;
  return st;
}

template <typename T>
hipError_t geo_launch(enufft_plan_t p, const GeoParams &g, const int32_t *order, int blocks, int64_t slice, size_t lds, const double *tri,
                      const void *x, const void *y, const void *h, void *xb, void *yb, void *hb, void *wb,
                      uint8_t *inside, double *info, int32_t *counts, double2 *ws_u, int32_t *ws_idx,
                      int32_t *ws_slot) {
  auto fn = geometry_kernel<T>;
  hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(kGeoThreads), lds, p->stream, g, order,
                     p->n_cells, p->d_counters + 6, p->d_counters + 7, slice, (const int64_t *)p->d_cell_off, tri,
                     (const T *)x, (const T *)y, (const T *)h, (T *)xb, (T *)yb, (T *)hb, (T *)wb, inside, info,
                     counts, ws_u, ws_idx, ws_slot);
  return hipGetLastError();
}

template <typename T>
hipError_t geo_occupancy(size_t lds, int *per_cu) {
  hipError_t e = hipFuncSetAttribute((const void *)geometry_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, (const void *)geometry_kernel<T>, kGeoThreads, lds);
}

}  // namespace

enufft_status adj_prepare(enufft_plan_t p);

}  // namespace enufft

extern "C" enufft_status enufft_cell_geometry(enufft_plan_t p, const double *tri, const void *x, const void *y,
                                              const void *h, const enufft_geometry_opts *opts, void *xb, void *yb,
                                              void *hb, void *wb, uint8_t *inside, double *info,
                                              int32_t *counts) {
  using namespace enufft;
  enufft_status st = check_plan(p, "enufft_cell_geometry");
  if (st != ENUFFT_OK) return st;
  if (!opts) return geo_fail(p, ENUFFT_EINVAL, "null options");
  const enufft_geometry_opts &o = *opts;
  if (o.frame < 0 || o.frame > 1 || o.mask < 0 || o.mask > 2 || o.weights < 0 || o.weights > 1)
    return geo_fail(p, ENUFFT_EINVAL, "unknown frame, mask or weights kind");
  if (!(o.eta >= 1.0) || !std::isfinite(o.eta) || !(o.floor_frac >= 0.0) || !std::isfinite(o.floor_frac))
    return geo_fail(p, ENUFFT_EINVAL, "eta must be finite and >= 1, floor_frac finite and >= 0");
  if (o.weights == ENUFFT_WEIGHTS_VORONOI && (o.raster < 1 || o.raster > 4096))
    return geo_fail(p, ENUFFT_EINVAL, "raster must be in [1, 4096] for Voronoi weights");
  if (p->n_cells == 0) return ENUFFT_OK;
  if (!tri) return geo_fail(p, ENUFFT_EINVAL, "null triangle array");
  if (p->n_points > 0 && (!x || !y || !h || !xb || !yb || !hb || !wb))
    return geo_fail(p, ENUFFT_EINVAL, "null point or output array");
  // device copy of the cell offsets (shared with the adjoint's schedule)
  st = adj_prepare(p);
  if (st != ENUFFT_OK) return st;
  const bool vor = o.weights == ENUFFT_WEIGHTS_VORONOI;
  GeoParams g{o.frame, o.mask, o.weights, o.raster, o.deplane ? 1 : 0, o.eta, o.floor_frac};

  // cells largest first (computed once per plan)
  int64_t largest = 0;
  for (int64_t c = 0; c < p->n_cells; ++c) largest = std::max(largest, p->offsets[c + 1] - p->offsets[c]);
  if (largest >= (int64_t(1) << 31)) return geo_fail(p, ENUFFT_EUNSUPPORTED, "cells of 2^31 points or more");
  const int32_t *order = nullptr;
  st = cells_largest_first(p, &order);
  if (st != ENUFFT_OK) return st;
  // persistent workgroups: as many as are resident (the Voronoi bins take the LDS
  // of the largest cell's bin grid)
  const int nbl = vor ? std::min(kGeoMaxBins, geo_bins(largest) + 1) : 0;
  const size_t lds = vor ? (size_t)(nbl * nbl + 1) * sizeof(int) : 16;
  int per_cu = 0;
  hipError_t e = p->prec == ENUFFT_F64 ? geo_occupancy<double>(lds, &per_cu) : geo_occupancy<float>(lds, &per_cu);
  if (e != hipSuccess || per_cu < 1) return geo_fail(p, ENUFFT_EDEVICE, "geometry kernel cannot be resident");
  const int blocks = (int)std::min<int64_t>(p->n_cells, (int64_t)p->n_cu * per_cu);
  const int64_t slice = vor ? largest : 0;
  const int64_t need = (int64_t)blocks * slice;
  if (vor && need > p->geo_ws_points) {
    dev_release(p, &p->geo_ws, (size_t)p->geo_ws_points * 16);
    dev_release(p, &p->geo_ws_i, (size_t)p->geo_ws_points * 8);
    p->geo_ws_points = 0;
    st = geo_alloc(p, &p->geo_ws, (size_t)std::max<int64_t>(1, need) * 16, "geometry sample copy");
    if (st == ENUFFT_OK)
      st = geo_alloc(p, &p->geo_ws_i, (size_t)std::max<int64_t>(1, need) * 8, "geometry sample index");
    if (st != ENUFFT_OK) return st;
    p->geo_ws_points = need;
  }
  double2 *ws_u = vor ? (double2 *)p->geo_ws : nullptr;
  int32_t *ws_idx = vor ? (int32_t *)p->geo_ws_i : nullptr;
  int32_t *ws_slot = vor ? ws_idx + p->geo_ws_points : nullptr;
  if (p->prec == ENUFFT_F64)
    e = geo_launch<double>(p, g, order, blocks, slice, lds, tri, x, y, h, xb, yb, hb, wb, inside, info, counts, ws_u, ws_idx,
                           ws_slot);
  else
    e = geo_launch<float>(p, g, order, blocks, slice, lds, tri, x, y, h, xb, yb, hb, wb, inside, info, counts, ws_u, ws_idx,
                          ws_slot);
  if (e != hipSuccess) {
    p->last_error = std::string("enufft_cell_geometry launch: ") + hipGetErrorString(e);
    p->faulted = true;
    return ENUFFT_EDEVICE;
  }
  return ENUFFT_OK;
}
