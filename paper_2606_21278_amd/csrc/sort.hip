// Point sort (enufft_sort_points): a device counting sort of every cell's
// samples by the fine-grid cell where their kernel footprint starts, row-major
// (Section 2.1.2 Step 1: the spreading of eq. spreading adds a sample's
// contributions around that cell).  In that order consecutive samples have
// nearby footprints, which the batched type-1 needs for its merged runs;
// samples stored in any other order (shuffled, or grouped by something other
// than position) otherwise take its one-point-at-a-time path.  The sort is a
// one-time preparation: it writes sorted copies of the caller's arrays and the
// permutation, and the caller works on the sorted arrays from then on.
//
// One workgroup per cell: an LDS histogram over the n1 x n2 fine cells, its
// exclusive scan, and a scatter with LDS cursors (the order inside one fine cell
// is that of the cursor increments, which is immaterial to the sum).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "device_common.h"
#include "plan.h"

namespace enufft {

template <typename T>
void split_scale(int n, T *hi, T *lo);

namespace {

constexpr int kSortThreads = 1024;

template <typename T>
struct SortKey {
  T s1_hi, s1_lo, s2_hi, s2_lo, halfw;
  int n1, n2, log_n1;
  __device__ __forceinline__ int operator()(T x, T y) const {
    const FineCoord<T> fx = fine_coord<T>(x, s1_hi, s1_lo, halfw);
    const FineCoord<T> fy = fine_coord<T>(y, s2_hi, s2_lo, halfw);
    return ((fy.i0 & (n2 - 1)) << log_n1) | (fx.i0 & (n1 - 1));
  }
};

template <typename T>
__global__ __launch_bounds__(kSortThreads) void sort_kernel(const int64_t *__restrict__ off,
                                                                const T *__restrict__ x, const T *__restrict__ y,
                                                                const T *__restrict__ h, const T *__restrict__ w,
                                                                SortKey<T> key, int32_t *__restrict__ perm,
                                                                T *__restrict__ xs, T *__restrict__ ys,
                                                                T *__restrict__ hs, T *__restrict__ ws) {
  extern __shared__ int hist[];   // [n1 n2] counts, then starts, then cursors
  __shared__ int part[kSortThreads];
  const int t = threadIdx.x;
  const int64_t c = blockIdx.x;
  const int64_t a = off[c], b = off[c + 1];
  if (a == b) return;
  const int nk = key.n1 * key.n2;
  for (int i = t; i < nk; i += kSortThreads) hist[i] = 0;
  __syncthreads();
  for (int64_t j = a + t; j < b; j += kSortThreads) atomicAdd(&hist[key(x[j], y[j])], 1);
  __syncthreads();
  // exclusive scan: per-thread segments, then a scan of the segment sums
  const int per = (nk + kSortThreads - 1) / kSortThreads;
  const int lo = min(nk, t * per), hi = min(nk, lo + per);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += hist[i];
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < kSortThreads; o <<= 1) {
    const int v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;
  for (int i = lo; i < hi; ++i) {
    const int n = hist[i];
    hist[i] = run;
    run += n;
  }
  __syncthreads();
  for (int64_t j = a + t; j < b; j += kSortThreads) {
    const T xj = x[j], yj = y[j];
    const int64_t pos = a + atomicAdd(&hist[key(xj, yj)], 1);
    if (perm) perm[pos] = (int32_t)j;
    xs[pos] = xj;
    ys[pos] = yj;
    if (hs) hs[pos] = h[j];
    if (ws) ws[pos] = w[j];
  }
}

int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

template <typename T>
hipError_t launch_sort(enufft_plan_t p, const void *x, const void *y, const void *h, const void *w, void *xs,
                       void *ys, void *hs, void *ws, int32_t *perm) {
  SortKey<T> k;
  split_scale<T>(p->n1, &k.s1_hi, &k.s1_lo);
  split_scale<T>(p->n2, &k.s2_hi, &k.s2_lo);
  k.halfw = T(p->W) / T(2);
  k.n1 = p->n1;
  k.n2 = p->n2;
  k.log_n1 = log2i(p->n1);
  const size_t lds = (size_t)p->n1 * p->n2 * sizeof(int);
  hipError_t e = hipFuncSetAttribute((const void *)sort_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sort_kernel<T>, dim3((unsigned)p->n_cells), dim3(kSortThreads), lds, p->stream,
                     (const int64_t *)p->d_cell_off, (const T *)x, (const T *)y, (const T *)h, (const T *)w, k,
                     perm, (T *)xs, (T *)ys, (T *)hs, (T *)ws);
  return hipGetLastError();
}

}  // namespace

enufft_status adj_prepare(enufft_plan_t p);

}  // namespace enufft

extern "C" enufft_status enufft_sort_points(enufft_plan_t p, const void *x, const void *y, const void *h,
                                            const void *w, void *xs, void *ys, void *hs, void *ws, int32_t *perm) {
  using namespace enufft;
  enufft_status st = check_plan(p, "enufft_sort_points");
  if (st != ENUFFT_OK) return st;
  if (p->n_points >= (int64_t(1) << 31)) {
    p->last_error = "enufft_sort_points: batches of 2^31 points or more are not supported";
    return ENUFFT_EUNSUPPORTED;
  }
  if (p->n_points > 0 && (!x || !y || !xs || !ys || (hs && !h) || (ws && !w))) {
    p->last_error = "enufft_sort_points: null coordinate or output array";
    return ENUFFT_EINVAL;
  }
  if (p->n_cells == 0 || p->n_points == 0) return ENUFFT_OK;
  // large cells: the order their tiled spreading uses (by 32 x 32 tile); calls on
  // input in that order skip the per-call scatter
  if (p->big) return big_sort_points(p, x, y, h, w, xs, ys, hs, ws, perm);
  st = adj_prepare(p);   // device copy of the cell offsets
  if (st != ENUFFT_OK) return st;
  // cells in their own order: largest first was slower (92.7 against 70 ms for 8e8 shuffled points in
  // 20,480 cells), more large cells' output ranges being written at once
  hipError_t e = p->prec == ENUFFT_F64 ? launch_sort<double>(p, x, y, h, w, xs, ys, hs, ws, perm)
                                       : launch_sort<float>(p, x, y, h, w, xs, ys, hs, ws, perm);
  if (e != hipSuccess) {
    p->last_error = std::string("enufft_sort_points launch: ") + hipGetErrorString(e);
    p->faulted = true;
    return ENUFFT_EDEVICE;
  }
  return ENUFFT_OK;
}

extern "C" enufft_status enufft_bind_points(enufft_plan_t p, const void *x, const void *y) {
  using namespace enufft;
  enufft_status st = check_plan(p, "enufft_bind_points");
  if (st != ENUFFT_OK) return st;
  if ((x == nullptr) != (y == nullptr)) {
    p->last_error = "enufft_bind_points: x and y are both given (bind) or both NULL (unbind)";
    return ENUFFT_EINVAL;
  }
  // cells that fit LDS sort nothing per call: there is nothing to keep
  if (!p->big || p->n_points == 0) return ENUFFT_OK;
  return big_bind_points(p, x, y);
}
