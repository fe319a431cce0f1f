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
// Two passes.  The ranking pass takes one workgroup per cell: an LDS histogram
// over the n1 x n2 fine cells, its exclusive scan, and a scatter of the input
// indices with LDS cursors (the order inside one fine cell is that of the cursor
// increments, which is immaterial to the sum); it also writes each sample as one
// interleaved (x, y, h, w) record at its input index, in order.  The gather pass
// then walks the sorted positions in order and copies each sample's record from
// its input index: one 16-byte read (32 in FP64) per sample, and the four output
// arrays written with coalesced stores.  (Scattering the four arrays themselves
// wrote 4-byte values at random positions of every resident cell's output
// ranges, far more than L2 holds, so nearly every store left as a partial-line
// write to HBM; gathering them from the four separate arrays fetched four cache
// lines per sample.)
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
__global__ __launch_bounds__(kSortThreads) void sort_rank_kernel(const int64_t *__restrict__ off,
                                                                     const T *__restrict__ x, const T *__restrict__ y,
                                                                     const T *__restrict__ h, const T *__restrict__ w,
                                                                     SortKey<T> key, int32_t *__restrict__ perm,
                                                                     typename vec4<T>::type *__restrict__ rec) {
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
    typename vec4<T>::type r;
    r.x = xj;
    r.y = yj;
    r.z = h ? h[j] : T(0);
    r.w = w ? w[j] : T(0);
    rec[j] = r;
    perm[a + atomicAdd(&hist[key(xj, yj)], 1)] = (int32_t)j;
  }
}

// Sorted copies: position i takes the record at input index perm[i] (inside the
// same cell, so the reads stay within the ranges of the few cells in flight).
template <typename T>
__global__ __launch_bounds__(256) void sort_gather_kernel(int64_t n, const int32_t *__restrict__ perm,
                                                          const typename vec4<T>::type *__restrict__ rec,
                                                          T *__restrict__ xs, T *__restrict__ ys,
                                                          T *__restrict__ hs, T *__restrict__ ws) {
  using V = typename vec4<T>::type;
  constexpr int U = 4;   // positions per thread and round, their loads issued together
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < n; i0 += U * stride) {
    int32_t j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * stride;
      j[u] = i < n ? perm[i] : 0;
    }
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = rec[j[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * stride;
      if (i < n) {
        xs[i] = v[u].x;
        ys[i] = v[u].y;
        if (hs) hs[i] = v[u].z;
        if (ws) ws[i] = v[u].w;
      }
    }
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
  hipError_t e = hipFuncSetAttribute((const void *)sort_rank_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  using V = typename vec4<T>::type;
  const int64_t n = p->n_points;
  V *rec = (V *)p->d_sort_rec;
  hipLaunchKernelGGL(sort_rank_kernel<T>, dim3((unsigned)p->n_cells), dim3(kSortThreads), lds, p->stream,
                     (const int64_t *)p->d_cell_off, (const T *)x, (const T *)y, (const T *)(hs ? h : nullptr),
                     (const T *)(ws ? w : nullptr), k, perm, rec);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int blocks = (int)std::min<int64_t>((int64_t)p->n_cu * 16, (n + 255) / 256);
  hipLaunchKernelGGL(sort_gather_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, p->stream, n,
                     (const int32_t *)perm, (const V *)rec, (T *)xs, (T *)ys, (T *)hs, (T *)ws);
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
  // plan-owned workspace, allocated on first use and kept for later calls (freed by
  // enufft_destroy): the interleaved records, and the permutation when the caller
  // asks for none (the gather pass reads it)
  auto keep_alloc = [&](void **d, size_t bytes, const char *what) -> enufft_status {
    if (*d) return ENUFFT_OK;
    if (hipMalloc(d, bytes) != hipSuccess) {
      *d = nullptr;
      p->last_error = std::string("enufft_sort_points: ") + what + " allocation failed";
      return ENUFFT_ENOMEM;
    }
    p->allocations.push_back(*d);
    p->workspace_bytes += (int64_t)bytes;
    return ENUFFT_OK;
  };
  st = keep_alloc(&p->d_sort_rec, (size_t)p->n_points * 4 * p->elem, "interleaved sample records");
  if (st != ENUFFT_OK) return st;
  if (!perm) {
    st = keep_alloc((void **)&p->d_sort_perm, (size_t)p->n_points * sizeof(int32_t), "sort permutation");
    if (st != ENUFFT_OK) return st;
    perm = p->d_sort_perm;
  }
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
