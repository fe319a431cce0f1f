// Cells whose fine grid does not fit one workgroup's LDS (mode boxes above 64
// per axis, e.g. 512 x 512 modes on a 1024^2 grid): the same type-1, EMS and
// adjoint, with the grid in HBM and the work tiled.
//
// Type-1 (Section 2.1.2):
//   1. a device counting sort of the cell's points by the fine-grid tile of
//      their footprint origin (BIG_TS x BIG_TS cells per tile): per-chunk LDS
//      histograms, a scan, and a scatter that copies the points into tile order
//      together with their original index;
//   2. spreading (Step 1) by persistent workgroups over fixed-size chunks of the
//      sorted points: each run of one tile accumulates in an FP64 LDS sub-grid
//      (the tile, the kernel's reach and a one-cell margin) that is then added
//      to the FP64 grid in HBM, so a crowded tile is shared by several
//      workgroups and no work unit is heavier than one chunk;
//   3. the FFT (Step 3): length-n1 transforms of row pairs (two real rows as one
//      complex row, split into the kept kx >= 0 bins) into a column buffer,
//      then the column transforms, each radix-2 Stockham in LDS;
//   4. deconvolution and crop (Step 4, eq. deconv) fused into the column pass,
//      the kx < 0 half of the box from Hermitian symmetry.
// EMS (Section 2.2): unit energies, a bitonic sort of the values (LDS-resident
// blocks plus global passes), the scores from one workgroup, the keep mask;
// units tied at the cut energy are ranked by unit id.
// Adjoint: the grids u, du/dx and du/dy built in HBM by the inverse column and
// row passes, then a tiled gather over the sorted points (each run stages its
// tile of the three grids in LDS) that writes the gradients at the original
// point indices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <string>
#include <type_traits>
#include <vector>

#include "device_common.h"
#include "launch.h"
#include "plan.h"

namespace enufft {

constexpr int BIG_TS = 32;            // tile side in fine-grid cells
constexpr int BIG_SORT_BLOCK = 4096;  // elements of one LDS-resident EMS sort block
constexpr int BIG_SPREAD_THREADS = 256;

template <typename T>
void split_scale(int n, T *hi, T *lo);

// ------------------------------------------------------------------ helpers

template <typename T>
__global__ void fill_kernel(T *p, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename T>
static hipError_t fill(T *p, int64_t n, T v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL((fill_kernel<T>), dim3(blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// Footprint origin of a point on the (wrapped) fine grid.
template <typename T>
__device__ __forceinline__ int big_origin(T x, T s_hi, T s_lo, int W, int n) {
  return fine_coord<T>(x, s_hi, s_lo, T(W) / T(2)).i0 & (n - 1);
}

// Local footprint origin inside the staged sub-grid of a tile whose cells start
// at t0: one cell of margin before the tile, so an origin that lands one cell
// off the tile the sort gave it still has its whole footprint inside the
// sub-grid; anything further off is clamped (it cannot occur: both sides
// compute the origin with the same code).
__device__ __forceinline__ int big_local(int i0, int t0, int n) {
  const int l = ((i0 - t0 + 1) & (n - 1));
  return l < BIG_TS + 1 ? l : BIG_TS + 1;
}

// FP64 per-tap polynomials (EsPoly64): u = 2 v - 1 with v = i0 - t + W/2 clamped
// to [0, 1]; tap d < W/2 is P_d(u), its mirror W - 1 - d is P_d(-u) (psi is even).
__device__ __forceinline__ double tap_u64(const FineCoord<double> &c, double halfw) {
  const double v = ((double(c.i0) - c.hi) - c.lo) + halfw;
  return 2.0 * fmin(fmax(v, 0.0), 1.0) - 1.0;
}

// The coefficients of mirror pair d, read where they are used: the offset is
// opaque to the compiler, so the loads are not hoisted out of the caller's point
// loop (all W/2 pairs at once would need more scalar registers than there are,
// and the spills cost a lane move per use).
__device__ __forceinline__ const double *poly64_pair(const EsPoly64 &cf, int d) {
  int z = 0;
  asm volatile("" : "+s"(z));
  return cf.c + d * (ES64_DEG + 1) + z;
}

// Mirror pair d at u: P_d(+-u) = E(u^2) +- u O(u^2).
__device__ __forceinline__ void poly64_pair_eval(const double *cd, double u, double s, double &t0, double &t1) {
  double e = cd[ES64_DEG - 1], o = cd[ES64_DEG];
#pragma unroll
  for (int k = ES64_DEG - 3; k >= 0; k -= 2) {
    e = fma(e, s, cd[k]);
    o = fma(o, s, cd[k + 1]);
  }
  t0 = fma(u, o, e);
  t1 = fma(-u, o, e);
}

// All W taps along both axes, pair by pair (one pair's coefficients live at a time).
template <int W>
__device__ __forceinline__ void es_taps_poly64_xy(double ux, double uy, const EsPoly64 &cf, double (&kx)[W],
                                                  double (&ky)[W]) {
  static_assert(W % 2 == 0 && ES64_DEG % 2 == 1 && W <= ES64_MAXW, "mirror pairs of an odd-degree fit");
  const double sx = ux * ux, sy = uy * uy;
#pragma unroll
  for (int d = 0; d < W / 2; ++d) {
    const double *cd = poly64_pair(cf, d);
    poly64_pair_eval(cd, ux, sx, kx[d], kx[W - 1 - d]);
    poly64_pair_eval(cd, uy, sy, ky[d], ky[W - 1 - d]);
  }
}

// The x taps alone.
template <int W>
__device__ __forceinline__ void es_taps_poly64(double u, const EsPoly64 &cf, double (&out)[W]) {
  static_assert(W % 2 == 0 && ES64_DEG % 2 == 1 && W <= ES64_MAXW, "mirror pairs of an odd-degree fit");
  const double s = u * u;
#pragma unroll
  for (int d = 0; d < W / 2; ++d) poly64_pair_eval(poly64_pair(cf, d), u, s, out[d], out[W - 1 - d]);
}

// One tap, dd in [0, W): Horner on its pair's coefficients at +-u (dd uniform
// across the wave, so the coefficient loads stay scalar).
template <int W>
__device__ __forceinline__ double es_tap_poly64(double u, const EsPoly64 &cf, int dd) {
  const bool m = dd >= W / 2;
  const double *cd = cf.c + (m ? W - 1 - dd : dd) * (ES64_DEG + 1);
  const double x = m ? -u : u;
  double acc = cd[ES64_DEG];
#pragma unroll
  for (int k = ES64_DEG - 1; k >= 0; --k) acc = fma(acc, x, cd[k]);
  return acc;
}

// Kernel-argument form of EsPoly64 per precision (FP32 kernels carry only the flag).
struct NoPoly64 {
  int on;
};
template <typename T>
using Poly64Of = typename std::conditional<sizeof(T) == 8, EsPoly64, NoPoly64>::type;

// The W kernel values of one point along one axis: the plan's per-tap
// polynomials (FP32, W <= ES_MAXW) when POLY; for FP64 plans their FP64 ones
// when the plan carries them; else psi itself.
template <typename T, int W, bool POLY>
__device__ __forceinline__ void big_taps(const FineCoord<T> &c, T beta, const EsPoly &cf, const Poly64Of<T> &c64,
                                         T (&out)[W]) {
  if constexpr (POLY) {
    es_taps_poly<W>(c, float(W) * 0.5f, cf, out);
  } else {
    if constexpr (sizeof(T) == 8 && W % 2 == 0 && W <= ES64_MAXW) {
      if (c64.on) {
        es_taps_poly64<W>(tap_u64(c, double(W) * 0.5), c64, out);
        return;
      }
    }
    const T zsc = T(2) / T(W);
#pragma unroll
    for (int d = 0; d < W; ++d) out[d] = ker_eval(c.offset(d) * zsc, beta);
  }
}

// Radix-2 Stockham transform of length n (a power of two) in LDS: a holds the
// input, b is the ping-pong buffer, natural order in and out.  Forward uses
// tw[j] = exp(-2 pi i j / n), INV the conjugates; unnormalised.  Returns the
// buffer holding the result.  Every thread of the block must call it.
template <bool INV, typename T>
__device__ T *stockham(T *a, T *b, int n, const T *tw) {
  T *x = a, *y = b;
  for (int ns = 1; ns < n; ns <<= 1) {
    for (int j = threadIdx.x; j < n / 2; j += blockDim.x) {
      const int k = j & (ns - 1);
      const T v0r = x[2 * j], v0i = x[2 * j + 1];
      const T ur = x[2 * (j + n / 2)], ui = x[2 * (j + n / 2) + 1];
      const int t = k * (n / (2 * ns));
      const T c = tw[2 * t], s = INV ? -tw[2 * t + 1] : tw[2 * t + 1];
      const T v1r = ur * c - ui * s, v1i = ur * s + ui * c;
      const int d = (j - k) * 2 + k;   // (j / ns) * 2 ns + k
      y[2 * d] = v0r + v1r;
      y[2 * d + 1] = v0i + v1i;
      y[2 * (d + ns)] = v0r - v1r;
      y[2 * (d + ns) + 1] = v0i - v1i;
    }
    __syncthreads();
    T *tmp = x;
    x = y;
    y = tmp;
  }
  return x;
}

// ------------------------------------------------------------------ device sort by tile

// The cell's input points are taken in chunks of BIG_SORT_CHUNK.  Each chunk's
// tile histogram goes to memory; scans over chunks and tiles give every chunk
// its start in every tile's range, so no pass uses atomics in global memory.
// (Device-scope atomics that many workgroups aim at the same few addresses
// serialise far from the CUs; a thousand tile cursors hit by every chunk cost
// milliseconds.)
constexpr int BIG_SORT_CHUNK = 16384;
constexpr int BIG_SORT_THREADS = 512;
constexpr int BIG_SCAN_GROUP = 64;     // chunks per group in the chunk scans
constexpr int BIG_UNIT_CHUNK = 16384;  // sorted points per spreading / gather work unit

template <typename T>
struct BigSortArgs {
  const T *x, *y, *h, *w;   // the cell's points (h may be NULL: copied as 0)
  int64_t n;
  T s1h, s1l, s2h, s2l;
  int W, n1, n2, ntx, ntiles;
  int nchunks, ngroups;
  int *chunk_hist;          // [nchunks][ntiles]: counts, then each chunk's start in each tile
  int *group_sum;           // [ngroups][ntiles]
  int64_t *offsets;         // [ntiles + 1] tile ranges of the sorted order
  int *unit_base;           // [ntiles + 1] first work unit of each tile; [ntiles] = units in all
  int *inv;                 // [n] sorted position of each input point
  T *xs, *ys, *hs, *ws;     // [n] points in tile order
  int *chunk_fl;            // [nchunks][4] first key, last key, tiles descend inside, keys descend inside
  int *presorted;           // [0]: input in tile order, [1]: also by fine cell inside each tile (NULL: always scatter)
};

template <typename T>
__device__ __forceinline__ int big_tile(const BigSortArgs<T> &a, T x, T y) {
  const int ix = big_origin<T>(x, a.s1h, a.s1l, a.W, a.n1);
  const int iy = big_origin<T>(y, a.s2h, a.s2l, a.W, a.n2);
  return (iy / BIG_TS) * a.ntx + ix / BIG_TS;
}

// Tile and fine cell of the footprint origin as one key: the tile times
// BIG_TS^2 plus the cell's row-major index inside the tile (tiles start at
// multiples of BIG_TS, so the in-tile index is the origin modulo BIG_TS).
constexpr int BIG_TS2 = BIG_TS * BIG_TS;
template <typename T>
__device__ __forceinline__ int big_key(const BigSortArgs<T> &a, T x, T y) {
  const int ix = big_origin<T>(x, a.s1h, a.s1l, a.W, a.n1);
  const int iy = big_origin<T>(y, a.s2h, a.s2l, a.W, a.n2);
  return ((iy / BIG_TS) * a.ntx + ix / BIG_TS) * BIG_TS2 + (iy % BIG_TS) * BIG_TS + ix % BIG_TS;
}

__device__ __forceinline__ int big_wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Exclusive scan of cnt[0 .. n) into out[0 .. n) by a workgroup of NT threads,
// each owning a contiguous run of entries; returns the total.  cnt and out may
// be the same array.
template <int NT, typename O>
__device__ int big_block_scan(const int *cnt, O *out, int n, int *wsum) {
  constexpr int NW = NT / 64;
  const int per = (n + NT - 1) / NT;
  const int t0 = min(n, (int)threadIdx.x * per), t1 = min(n, t0 + per);
  int v = 0;
  for (int t = t0; t < t1; ++t) v += cnt[t];
  const int inc = big_wave_incl_scan(v);
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 63) wsum[wave] = inc;
  __syncthreads();
  int run = inc - v, total = 0;
  for (int w = 0; w < NW; ++w) {
    if (w < wave) run += wsum[w];
    total += wsum[w];
  }
  for (int t = t0; t < t1; ++t) {
    const int c = cnt[t];
    out[t] = (O)run;
    run += c;
  }
  __syncthreads();
  return total;
}

// Tile histogram of each chunk, written in full, and the chunk's order: its
// first and last key (tile and fine cell, big_key) and whether tiles, or keys,
// descend inside it.  The tile scan concludes from these whether the whole input
// is in tile order, and whether it is also in fine-cell order inside each tile.
template <typename T>
__global__ __launch_bounds__(BIG_SORT_THREADS) void big_count_kernel(BigSortArgs<T> a) {
  extern __shared__ int hist[];            // [ntiles], then the chunk's keys [BIG_SORT_CHUNK]
  int *keys = hist + a.ntiles;
  __shared__ int s_desc[2];
  for (int i = threadIdx.x; i < a.ntiles; i += blockDim.x) hist[i] = 0;
  if (threadIdx.x < 2) s_desc[threadIdx.x] = 0;
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * BIG_SORT_CHUNK, e = min(a.n, s + BIG_SORT_CHUNK);
  const int cnt = (int)(e - s);
  // CB points per thread and round, every load of a round issued before the
  // first is used (one memory latency per round, not per point)
  constexpr int CB = 8;
  for (int64_t j0 = s + threadIdx.x; j0 < e; j0 += (int64_t)CB * blockDim.x) {
    T xv[CB], yv[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int64_t j = min(j0 + (int64_t)c * blockDim.x, e - 1);
      xv[c] = a.x[j];
      yv[c] = a.y[j];
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int64_t j = j0 + (int64_t)c * blockDim.x;
      if (j >= e) break;
      const int k = big_key<T>(a, xv[c], yv[c]);
      keys[j - s] = k;
      // a wave whose points all lie in one tile (input in tile order) adds its
      // count once: 64 adds to one LDS counter are served one after another
      const int t = k / BIG_TS2;
      const int t0 = __builtin_amdgcn_readfirstlane(t);
      const uint64_t act = __ballot(1), same = __ballot(t == t0);
      if (same == act) {
        if ((int)(threadIdx.x & 63) == __ffsll((unsigned long long)act) - 1) atomicAdd(&hist[t0], __popcll(act));
      } else {
        atomicAdd(&hist[t], 1);
      }
    }
  }
  __syncthreads();
  int tdesc = 0, kdesc = 0;
  for (int i = threadIdx.x; i + 1 < cnt; i += blockDim.x) {
    tdesc |= keys[i] / BIG_TS2 > keys[i + 1] / BIG_TS2;
    kdesc |= keys[i] > keys[i + 1];
  }
  if (tdesc) s_desc[0] = 1;
  if (kdesc) s_desc[1] = 1;
  int *row = a.chunk_hist + (int64_t)blockIdx.x * a.ntiles;
  for (int i = threadIdx.x; i < a.ntiles; i += blockDim.x) row[i] = hist[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    int *fl = a.chunk_fl + 4 * (int64_t)blockIdx.x;
    fl[0] = keys[0];
    fl[1] = keys[cnt - 1];
    fl[2] = s_desc[0];
    fl[3] = s_desc[1];
  }
}

// Per tile, the sum over each group of BIG_SCAN_GROUP chunks.
__global__ __launch_bounds__(256) void big_group_sum_kernel(const int *chunk_hist, int nchunks, int ntiles,
                                                            int *group_sum) {
  const int t = blockIdx.x * 256 + threadIdx.x, g = blockIdx.y;
  if (t >= ntiles) return;
  const int b0 = g * BIG_SCAN_GROUP, b1 = min(nchunks, b0 + BIG_SCAN_GROUP);
  int s = 0;
  for (int b = b0; b < b1; ++b) s += chunk_hist[(int64_t)b * ntiles + t];
  group_sum[(int64_t)g * ntiles + t] = s;
}

// One workgroup: per tile, the exclusive scan of its group sums (in place) and
// its total; the tile offsets (exclusive scan of the totals); the number of
// work units of each tile (the unit chunks its range touches) and their scan.
__global__ __launch_bounds__(1024) void big_tile_scan_kernel(int *group_sum, int ngroups, int ntiles,
                                                             int64_t *offsets, int *unit_base, const int *chunk_fl,
                                                             int nchunks, int *presorted) {
  extern __shared__ int tot[];   // [ntiles]
  __shared__ int wsum[16];
  // the input is in tile order when no chunk's tiles descend inside and each
  // chunk's last tile is at most the next chunk's first; in key order (tile,
  // then fine cell) likewise with the keys
  int tbad = 0, kbad = 0;
  for (int b = threadIdx.x; b < nchunks; b += blockDim.x) {
    const int *fl = chunk_fl + 4 * (int64_t)b;
    const bool more = b + 1 < nchunks;
    tbad |= fl[2] || (more && fl[1] / BIG_TS2 > fl[4] / BIG_TS2);
    kbad |= fl[3] || (more && fl[1] > fl[4]);
  }
  tbad = __syncthreads_or(tbad);
  kbad = __syncthreads_or(kbad);
  if (threadIdx.x == 0 && presorted) {
    presorted[0] = tbad ? 0 : 1;
    presorted[1] = (tbad || kbad) ? 0 : 1;
  }
  for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
    int run = 0;
    for (int g = 0; g < ngroups; ++g) {
      int *p = group_sum + (int64_t)g * ntiles + t;
      const int v = *p;
      *p = run;
      run += v;
    }
    tot[t] = run;
  }
  __syncthreads();
  const int n = big_block_scan<1024, int64_t>(tot, offsets, ntiles, wsum);
  if (threadIdx.x == 0) offsets[ntiles] = n;
  __syncthreads();
  for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
    const int64_t t0 = offsets[t], t1 = t0 + tot[t];
    tot[t] = t1 > t0 ? (int)((t1 - 1) / BIG_UNIT_CHUNK - t0 / BIG_UNIT_CHUNK + 1) : 0;
  }
  __syncthreads();
  const int units = big_block_scan<1024, int>(tot, unit_base, ntiles, wsum);
  if (threadIdx.x == 0) unit_base[ntiles] = units;
}

// Each chunk's start in each tile: the tile offset, the chunk group's prefix
// and the counts of the earlier chunks of the group.
__global__ __launch_bounds__(256) void big_chunk_base_kernel(int *chunk_hist, const int *group_sum,
                                                             const int64_t *offsets, int nchunks, int ntiles) {
  const int t = blockIdx.x * 256 + threadIdx.x, g = blockIdx.y;
  if (t >= ntiles) return;
  const int b0 = g * BIG_SCAN_GROUP, b1 = min(nchunks, b0 + BIG_SCAN_GROUP);
  int run = (int)offsets[t] + group_sum[(int64_t)g * ntiles + t];
  for (int b = b0; b < b1; ++b) {
    int *p = chunk_hist + (int64_t)b * ntiles + t;
    const int v = *p;
    *p = run;
    run += v;
  }
}

// Scatter, one chunk per workgroup, in sub-chunks that fit LDS: each
// sub-chunk's points loaded once (coalesced, into registers, every load of a
// thread issued before the first is used), its tile histogram and scan, the
// points ranked and staged in LDS in tile order, then copied out with
// consecutive threads on consecutive positions of each tile's segment, so the
// stores coalesce.  The chunk's start in every tile advances by each
// sub-chunk's count.  The inverse permutation is written in input order.
// (Ranking in LDS but reading the points back from memory in tile order would
// fetch a whole cache line for every 4-byte value.)
template <typename T>
constexpr int big_scatter_sub() { return sizeof(T) == 4 ? 4096 : 2048; }

template <typename T>
__global__ __launch_bounds__(BIG_SORT_THREADS) void big_scatter_kernel(BigSortArgs<T> a) {
  if (a.presorted && *a.presorted) return;   // the tile ranges are the input's own: nothing to move
  using V4 = typename vec4<T>::type;
  constexpr int SUB = big_scatter_sub<T>();
  extern __shared__ __align__(32) unsigned char sm_raw[];
  V4 *staged = reinterpret_cast<V4 *>(sm_raw);              // [SUB] (x, y, h, w) in tile order
  int *hist = reinterpret_cast<int *>(staged + SUB);        // [ntiles] counts, then the fill cursors
  int *lstart = hist + a.ntiles;                            // [ntiles] sub-chunk start of each tile
  int *gbase = lstart + a.ntiles;                           // [ntiles] global start of the next points of each tile
  __shared__ int wsum[BIG_SORT_THREADS / 64];
  const int64_t s0 = (int64_t)blockIdx.x * BIG_SORT_CHUNK;
  const int64_t e0 = min(a.n, s0 + BIG_SORT_CHUNK);
  const int *base_row = a.chunk_hist + (int64_t)blockIdx.x * a.ntiles;
  for (int i = threadIdx.x; i < a.ntiles; i += blockDim.x) gbase[i] = base_row[i];
  // each thread holds PER points of a sub-chunk in registers (all loads issued
  // before the first is used), counts them and then ranks them
  constexpr int PER = SUB / BIG_SORT_THREADS;
  static_assert(SUB % BIG_SORT_THREADS == 0, "sub-chunks are whole rounds of the workgroup");
  for (int64_t s = s0; s < e0; s += SUB) {
    const int cnt = (int)(min(e0, s + SUB) - s);
    V4 v[PER];
    int tile[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int64_t j = s + min(k * BIG_SORT_THREADS + (int)threadIdx.x, cnt - 1);
      v[k].x = a.x[j];
      v[k].y = a.y[j];
      v[k].z = a.h ? a.h[j] : T(0);
      v[k].w = a.w[j];
    }
    for (int i = threadIdx.x; i < a.ntiles; i += blockDim.x) hist[i] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      tile[k] = big_tile<T>(a, v[k].x, v[k].y);
      if (k * BIG_SORT_THREADS + (int)threadIdx.x < cnt) atomicAdd(&hist[tile[k]], 1);
    }
    __syncthreads();
    big_block_scan<BIG_SORT_THREADS, int>(hist, lstart, a.ntiles, wsum);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int li = k * BIG_SORT_THREADS + threadIdx.x;
      if (li >= cnt) continue;
      const int t = tile[k];
      // the histogram pass counted this point in tile t: hist[t] - 1 - (rank so far) is free
      const int slot = lstart[t] + atomicSub(&hist[t], 1) - 1;
      const int64_t pos = (int64_t)gbase[t] + (slot - lstart[t]);
      if (slot >= 0 && slot < cnt) staged[slot] = v[k];   // always true: both passes use tile[k]
      a.inv[s + li] = (pos >= 0 && pos < a.n) ? (int)pos : -1;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
      const V4 v = staged[i];
      const int t = big_tile<T>(a, v.x, v.y);
      const int64_t pos = (int64_t)gbase[t] + (i - lstart[t]);
      if (pos < 0 || pos >= a.n) continue;   // only if the passes disagreed on a tile; never out of bounds
      a.xs[pos] = v.x;
      a.ys[pos] = v.y;
      a.hs[pos] = v.z;
      a.ws[pos] = v.w;
    }
    __syncthreads();
    // advance each tile's start by this sub-chunk's count (the slots of tile t
    // are [lstart[t], lstart[t + 1]))
    for (int i = threadIdx.x; i < a.ntiles; i += blockDim.x) {
      const int end = i + 1 < a.ntiles ? lstart[i + 1] : cnt;
      gbase[i] += end - lstart[i];
    }
    __syncthreads();
  }
}

// Common arguments of the tiled spreading and gather passes.  Their work units
// are the pieces of each tile's range that fall in one BIG_UNIT_CHUNK of the
// sorted order, so no unit holds more than one chunk of points.
template <typename T>
struct BigTileArgs {
  const T *xs, *ys, *hs, *ws;
  const T *xi, *yi, *hi, *wi;   // the input points (read instead when *presorted)
  const int *presorted;
  const int64_t *offsets;    // [ntiles + 1]
  const int *unit_base;      // [ntiles + 1]; [ntiles] = number of units
  int ntiles, ntx;
  int64_t n;
  int *work_counter, *done_counter;
  const double *windows;     // per cell (cx, cy, R)
  int64_t cell;
  int window_kind;
  Geom g;
  T s1h, s1l, s2h, s2l, beta;
  EsPoly es;
  Poly64Of<T> es64;
  double *partial;           // spreading: [units][S * S] FP64 sub-grids
  const typename vec4<T>::type *G4;   // gather: n2 x n1 cells of (u, du/dx, du/dy, 0)
  typename vec4<T>::type *gout;       // gather: [n] (dL/dh, dL/dx, dL/dy, 0) in sorted order
  T *gh, *gx, *gy;                    // gather, input in tile order: the cell's gradients (each may be NULL)
};

// Persistent loop over the work units; body(t, lo, hi, u) runs unit u, the
// sorted positions [lo, hi) of tile t.  The last workgroup to finish resets the
// counters for the next launch.
template <typename T, typename Body>
__device__ __forceinline__ void big_units(const BigTileArgs<T> &a, int *s_unit, const Body &body) {
  const int nunits = a.unit_base[a.ntiles];
  for (;;) {
    if (threadIdx.x == 0) *s_unit = atomicAdd(a.work_counter, 1);
    __syncthreads();
    const int u = *s_unit;
    __syncthreads();
    if (u >= nunits) break;
    int lo = 0, hi = a.ntiles - 1;   // the tile of unit u: the largest t with unit_base[t] <= u
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.unit_base[mid] <= u) lo = mid;
      else hi = mid - 1;
    }
    const int t = lo;
    const int64_t t0 = a.offsets[t], t1 = a.offsets[t + 1];
    const int64_t c = t0 / BIG_UNIT_CHUNK + (u - a.unit_base[t]);
    const int64_t k0 = max(t0, c * BIG_UNIT_CHUNK), k1 = min(t1, (c + 1) * BIG_UNIT_CHUNK);
    if (k0 < k1) body(t, k0, k1, u);
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(a.done_counter, 1) == (int)gridDim.x - 1) {
      *a.work_counter = 0;
      *a.done_counter = 0;
    }
  }
}

// ------------------------------------------------------------------ spreading into the HBM grid

// Each unit accumulates in an FP64 LDS sub-grid and writes it out whole; the
// assemble pass adds the sub-grids up.
template <typename T, int W, bool POLY>
__global__ __launch_bounds__(BIG_SPREAD_THREADS) void big_spread_kernel(BigTileArgs<T> a) {
  constexpr int S = BIG_TS + W + 1;   // margin cell, tile, reach of the last origin
  __shared__ double sub[S * S];
  __shared__ int s_unit;
  const Geom &g = a.g;
  const T halfw = T(W) / T(2);
  const double *wn = a.windows + 3 * a.cell;
  const T cx = T(wn[0]), cy = T(wn[1]), R = T(wn[2]);
  const T pr = R > T(0) ? T(M_PI) / R : T(0);
  const bool pre = a.presorted[0];
  // points in fine-cell order inside each tile go to big_spread_run_kernel
  if constexpr (sizeof(T) == 4 && POLY) {
    if (a.presorted[1]) return;
  }
  const T *X = pre ? a.xi : a.xs, *Y = pre ? a.yi : a.ys, *Hh = pre ? a.hi : a.hs, *Wq = pre ? a.wi : a.ws;
  big_units<T>(a, &s_unit, [&](int t, int64_t lo, int64_t hi, int u) {
    for (int i = threadIdx.x; i < S * S; i += blockDim.x) sub[i] = 0.0;
    __syncthreads();
    const int tx0 = (t % a.ntx) * BIG_TS, ty0 = (t / a.ntx) * BIG_TS;
    for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) {
      const T xj = X[k], yj = Y[k];
      const T cj = Wq[k] * Hh[k] * hann_w(a.window_kind, xj, yj, cx, cy, R, pr);
      const FineCoord<T> fx = fine_coord<T>(xj, a.s1h, a.s1l, halfw);
      const FineCoord<T> fy = fine_coord<T>(yj, a.s2h, a.s2l, halfw);
      const int lx = big_local(fx.i0 & (g.n1 - 1), tx0, g.n1);
      const int ly = big_local(fy.i0 & (g.n2 - 1), ty0, g.n2);
      T kx[W], ky[W];
      bool both = false;
      if constexpr (sizeof(T) == 8 && !POLY && W % 2 == 0 && W <= ES64_MAXW) {
        if (a.es64.on) {
          es_taps_poly64_xy<W>(tap_u64(fx, double(W) * 0.5), tap_u64(fy, double(W) * 0.5), a.es64, kx, ky);
          both = true;
        }
      }
      if (!both) {
        big_taps<T, W, POLY>(fx, a.beta, a.es, a.es64, kx);
        big_taps<T, W, POLY>(fy, a.beta, a.es, a.es64, ky);
      }
#pragma unroll
      for (int dy = 0; dy < W; ++dy) {
        const double vy = (double)(cj * ky[dy]);
        double *row = sub + (ly + dy) * S + lx;
#pragma unroll
        for (int dx = 0; dx < W; ++dx)
          __hip_atomic_fetch_add(row + dx, vy * (double)kx[dx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
    __syncthreads();
    double *dst = a.partial + (int64_t)u * (S * S);
    for (int i = threadIdx.x; i < S * S; i += blockDim.x) dst[i] = sub[i];
    __syncthreads();
  });
}

// FP32 spreading of points that arrive in fine-cell order inside each tile (the
// order enufft_sort_points leaves): runs of points with one footprint origin
// add their W x W contributions in FP32 registers, and each run goes to the
// FP64 sub-grid once, W^2 adds for the run instead of W^2 per point.  Each unit
// is staged through LDS in pieces of BIG_RUN_P points per thread (coalesced
// loads); thread t walks its own BIG_RUN_P consecutive points of each piece, the
// lanes of a wave a few segments apart.  A run is flushed when the origin
// changes and at the end of the segment, where lanes whose runs share an origin
// are summed across the wave first (big_run_flush_wave).
constexpr int BIG_RUN_P = 8;
constexpr int BIG_RUN_NP = BIG_RUN_P * BIG_SPREAD_THREADS;

template <int W>
__device__ __forceinline__ void big_run_flush(double *sub, int key, float (&acc)[W][W]) {
  constexpr int S = BIG_TS + W + 1;
  double *base = sub + key;
#pragma unroll
  for (int dy = 0; dy < W; ++dy)
#pragma unroll
    for (int dx = 0; dx < W; ++dx) {
      __hip_atomic_fetch_add(base + dy * S + dx, (double)acc[dy][dx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      acc[dy][dx] = 0.0f;
    }
}

// Sum of v over the 64 lanes of the wave, in lane 63 (row shifts inside each row
// of 16 lanes, then the row broadcasts); every lane must be active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float big_dpp_add(float v) {
  const int t = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf, false);
  return v + __builtin_bit_cast(float, t);
}
__device__ __forceinline__ float big_wave_total(float v) {
  v = big_dpp_add<0x111, 0xf>(v);   // row_shr:1
  v = big_dpp_add<0x112, 0xf>(v);   // row_shr:2
  v = big_dpp_add<0x114, 0xf>(v);   // row_shr:4
  v = big_dpp_add<0x118, 0xf>(v);   // row_shr:8
  v = big_dpp_add<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v = big_dpp_add<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}

// End-of-segment flush, called by every lane of the wave: lanes whose runs share
// an origin with many others (a dense fine cell can hold every lane's run) are
// first summed across the wave, one group of equal origins at a time, and lane 63
// adds each sum once; the rest add their own values.  Without this, 64 lanes
// adding to one address are served one after another.
template <int W>
__device__ __forceinline__ void big_run_flush_wave(double *sub, int &cur, float (&acc)[W][W]) {
  constexpr int S = BIG_TS + W + 1;
  const int lane = threadIdx.x & 63;
  for (int grp = 0; grp < 4; ++grp) {
    const uint64_t pend = __ballot(cur >= 0);
    if (pend == 0) return;
    const int lead = __ffsll((unsigned long long)pend) - 1;
    const int k = __builtin_amdgcn_readlane(cur, lead);
    const bool mine = cur == k;
    if (__popcll(__ballot(mine)) < 8) break;   // a small group: its own adds are cheap
#pragma unroll
    for (int dy = 0; dy < W; ++dy)
#pragma unroll
      for (int dx = 0; dx < W; ++dx) {
        const float tot = big_wave_total(mine ? acc[dy][dx] : 0.0f);
        if (lane == 63)
          __hip_atomic_fetch_add(sub + k + dy * S + dx, (double)tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (mine) acc[dy][dx] = 0.0f;
      }
    if (mine) cur = -1;
  }
  if (cur >= 0) big_run_flush<W>(sub, cur, acc);
  cur = -1;
}

template <int W>
__global__ __launch_bounds__(BIG_SPREAD_THREADS) void big_spread_run_kernel(BigTileArgs<float> a) {
  constexpr int S = BIG_TS + W + 1;   // as big_spread_kernel
  constexpr int NW = BIG_SPREAD_THREADS / 64;
  // staged segment s starts at s * PP + s / NW (one spare slot per segment and
  // per NW segments, so the lanes of a wave, NW segments apart, read distinct banks)
  constexpr int PP = BIG_RUN_P + 1;
  __shared__ double sub[S * S];
  __shared__ float4 piece[BIG_SPREAD_THREADS * PP + BIG_SPREAD_THREADS / NW];
  __shared__ int s_unit;
  if (!a.presorted[1]) return;        // not in cell order: big_spread_kernel spreads this cell
  const Geom &g = a.g;
  const float halfw = float(W) / 2.0f;
  const double *wn = a.windows + 3 * a.cell;
  const float cx = float(wn[0]), cy = float(wn[1]), R = float(wn[2]);
  const float pr = R > 0.0f ? float(M_PI) / R : 0.0f;
  // cell order implies tile order: the input arrays are the tile-sorted points
  const float *X = a.xi, *Y = a.yi, *Hh = a.hi, *Wq = a.wi;
  const int seg = (threadIdx.x & 63) * NW + (threadIdx.x >> 6);   // this thread's segment of a piece
  big_units<float>(a, &s_unit, [&](int t, int64_t lo, int64_t hi, int u) {
    for (int i = threadIdx.x; i < S * S; i += blockDim.x) sub[i] = 0.0;
    const int tx0 = (t % a.ntx) * BIG_TS, ty0 = (t / a.ntx) * BIG_TS;
    for (int64_t p0 = lo; p0 < hi; p0 += BIG_RUN_NP) {
      const int np = (int)min<int64_t>(BIG_RUN_NP, hi - p0);
      __syncthreads();   // the previous piece is consumed (and the sub-grid zeroed)
      for (int q = threadIdx.x; q < np; q += BIG_SPREAD_THREADS) {
        float4 v;
        v.x = X[p0 + q];
        v.y = Y[p0 + q];
        v.z = Hh[p0 + q];
        v.w = Wq[p0 + q];
        const int sq = q / BIG_RUN_P;
        piece[sq * PP + sq / NW + q % BIG_RUN_P] = v;
      }
      __syncthreads();
      const int q0 = seg * BIG_RUN_P, q1 = min(np, q0 + BIG_RUN_P);
      float acc[W][W];
#pragma unroll
      for (int dy = 0; dy < W; ++dy)
#pragma unroll
        for (int dx = 0; dx < W; ++dx) acc[dy][dx] = 0.0f;
      int cur = -1;   // sub-grid offset of the run's origin; -1: no run yet
      for (int q = q0; q < q1; ++q) {
        const float4 v = piece[seg * PP + seg / NW + (q - q0)];
        const float cj = v.w * v.z * hann_w(a.window_kind, v.x, v.y, cx, cy, R, pr);
        const FineCoord<float> fx = fine_coord<float>(v.x, a.s1h, a.s1l, halfw);
        const FineCoord<float> fy = fine_coord<float>(v.y, a.s2h, a.s2l, halfw);
        const int lx = big_local(fx.i0 & (g.n1 - 1), tx0, g.n1);
        const int ly = big_local(fy.i0 & (g.n2 - 1), ty0, g.n2);
        const int key = ly * S + lx;
        if (key != cur) {
          if (cur >= 0) big_run_flush<W>(sub, cur, acc);
          cur = key;
        }
        float kx[W], ky[W];
        big_taps<float, W, true>(fx, a.beta, a.es, a.es64, kx);
        big_taps<float, W, true>(fy, a.beta, a.es, a.es64, ky);
#pragma unroll
        for (int dy = 0; dy < W; ++dy) {
          const float vy = cj * ky[dy];
#pragma unroll
          for (int dx = 0; dx < W; ++dx) acc[dy][dx] = fmaf(vy, kx[dx], acc[dy][dx]);
        }
      }
      // (carrying runs over to the next piece was slower: the lanes whose origin
      // then changed at the piece's first point all flushed at once, unsummed)
      big_run_flush_wave<W>(sub, cur, acc);
    }
    __syncthreads();
    double *dst = a.partial + (int64_t)u * (S * S);
    for (int i = threadIdx.x; i < S * S; i += blockDim.x) dst[i] = sub[i];
    __syncthreads();
  });
}

// Every fine-grid cell: the sum of the sub-grids that cover it, over all units
// of its own tile and of the neighbouring tiles whose sub-grids reach it (the
// tile above / left through their kernel reach, the tile below / right through
// their margin cell).  Replaces clearing the grid and adding with atomics.
__global__ __launch_bounds__(256) void big_assemble_kernel(const double *partial, const int *unit_base, Geom g,
                                                           int ntx, int nty, int S, double *grid) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)g.n1 * g.n2) return;
  const int gy = (int)(i / g.n1), gx = (int)(i - (int64_t)gy * g.n1);
  const int tx = gx / BIG_TS, ty = gy / BIG_TS;
  const int px = gx - tx * BIG_TS, py = gy - ty * BIG_TS;
  double s = 0.0;
  for (int dyt = -1; dyt <= 1; ++dyt) {
    const int ly = py + 1 - dyt * BIG_TS;
    if (ly < 0 || ly >= S) continue;
    const int tyy = (ty + dyt + nty) % nty;
    for (int dxt = -1; dxt <= 1; ++dxt) {
      const int lx = px + 1 - dxt * BIG_TS;
      if (lx < 0 || lx >= S) continue;
      const int t = tyy * ntx + (tx + dxt + ntx) % ntx;
      const int64_t off = (int64_t)ly * S + lx, stride = (int64_t)S * S;
      const int u0 = unit_base[t], u1 = unit_base[t + 1];
      int u = u0;
      // crowded tiles have hundreds of units: keep eight loads in flight
      for (; u + 8 <= u1; u += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = partial[(int64_t)(u + q) * stride + off];
#pragma unroll
        for (int q = 0; q < 8; ++q) s += v[q];
      }
      for (; u < u1; ++u) s += partial[(int64_t)u * stride + off];
    }
  }
  grid[i] = s;
}

// ------------------------------------------------------------------ FFT passes

// Row pass: rows 2p and 2p + 1 of the FP64 grid as one complex row, forward
// transform, then the bins kx = 0..K1 of each real row into the column buffer
// cb[kx][row] (complex, n2 rows per column).
template <typename T>
__global__ __launch_bounds__(512) void big_rows_kernel(const double *grid, Geom g, const T *tw1, T *cb) {
  extern __shared__ __align__(16) unsigned char sm_raw[];
  const int n1 = g.n1;
  T *A = reinterpret_cast<T *>(sm_raw), *B = A + 2 * n1;
  const int p = blockIdx.x;
  const double *r0 = grid + (int64_t)(2 * p) * n1, *r1 = r0 + n1;
  for (int i = threadIdx.x; i < n1; i += blockDim.x) {
    A[2 * i] = (T)r0[i];
    A[2 * i + 1] = (T)r1[i];
  }
  __syncthreads();
  const T *Z = stockham<false, T>(A, B, n1, tw1);
  for (int k = threadIdx.x; k <= g.K1; k += blockDim.x) {
    const int m = (n1 - k) & (n1 - 1);
    const T zr = Z[2 * k], zi = Z[2 * k + 1], mr = Z[2 * m], mi = Z[2 * m + 1];
    // row 2p: (Z(k) + conj Z(-k)) / 2; row 2p + 1: (Z(k) - conj Z(-k)) / 2i
    T *c = cb + (int64_t)k * g.n2 * 2 + 4 * p;
    c[0] = T(0.5) * (zr + mr);
    c[1] = T(0.5) * (zi - mi);
    c[2] = T(0.5) * (zi + mi);
    c[3] = T(-0.5) * (zr - mr);
  }
}

// Column pass: transform of column kx over the n2 rows, deconvolution and crop
// into the mode box, the (-kx, -ky) entry as the conjugate.
template <typename T>
__global__ __launch_bounds__(512) void big_cols_kernel(const T *cb, Geom g, const T *tw2, const T *decon_x,
                                                       const T *decon_y, T *f) {
  extern __shared__ __align__(16) unsigned char sm_raw[];
  const int n2 = g.n2;
  T *A = reinterpret_cast<T *>(sm_raw), *B = A + 2 * n2;
  const int kx = blockIdx.x;
  const T *c = cb + (int64_t)kx * n2 * 2;
  for (int i = threadIdx.x; i < 2 * n2; i += blockDim.x) A[i] = c[i];
  __syncthreads();
  const T *Z = stockham<false, T>(A, B, n2, tw2);
  const int hi1 = g.lo1 + g.N1 - 1, hi2 = g.lo2 + g.N2 - 1;
  for (int ky = -g.K2 + (int)threadIdx.x; ky <= g.K2; ky += blockDim.x) {
    const int bin = ky & (n2 - 1);
    const T s = decon_x[kx] * decon_y[ky < 0 ? -ky : ky];
    const T vr = Z[2 * bin] * s, vi = Z[2 * bin + 1] * s;
    if (kx <= hi1 && ky >= g.lo2 && ky <= hi2) {
      T *o = f + 2 * ((int64_t)(ky - g.lo2) * g.N1 + (kx - g.lo1));
      o[0] = vr;
      o[1] = vi;
    }
    if (kx >= 1 && -kx >= g.lo1 && -ky >= g.lo2 && -ky <= hi2) {
      T *o = f + 2 * ((int64_t)(-ky - g.lo2) * g.N1 + (-kx - g.lo1));
      o[0] = vr;
      o[1] = -vi;
    }
  }
}

// ------------------------------------------------------------------ EMS for one large cell

struct BigCut {   // written by the scores pass
  double T1, T2, neff, sdel, Cs, alphaC, th, eth;
  int kstar, need, split, J;
};

template <typename C>
__device__ __forceinline__ double big_pair_energy(const C *f, const double *mw, int rep, int partner) {
#pragma clang fp contract(off)
  const int pq = partner >= 0 ? partner : rep;
  const C fr = f[rep], fp = f[pq];
  // each product and sum rounded on its own (no fused multiply-add), as the
  // in-register EMS path does
  double e = (double)fr.x * (double)fr.x + (double)fr.y * (double)fr.y;
  double ep = (double)fp.x * (double)fp.x + (double)fp.y * (double)fp.y;
  if (mw) {
    e = e * mw[rep];
    ep = ep * mw[pq];
  }
  return partner >= 0 ? e + ep : e;
}

// eq. (energy) / (weighted_e) of every unit into the sort buffer (padding +0
// sorts last), with per-workgroup partial sums of E and E^2.
template <typename T>
__global__ __launch_bounds__(256) void big_ems_energy_kernel(const T *f, const double *mw, const int2 *units, int J,
                                                             int Jpad, double *S, double *partial) {
  using C = typename vec2<T>::type;
  const C *fc = reinterpret_cast<const C *>(f);
  __shared__ double r1[256], r2[256];
  double s1 = 0.0, s2 = 0.0;
  const int u = blockIdx.x * 256 + threadIdx.x;
  if (u < Jpad) {
    double e = 0.0;
    if (u < J) {
      const int2 un = units[u];
      e = big_pair_energy<C>(fc, mw, un.x, un.y);
      s1 = e;
      s2 = e * e;
    }
    S[u] = e;
  }
  r1[threadIdx.x] = s1;
  r2[threadIdx.x] = s2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      r1[threadIdx.x] += r1[threadIdx.x + o];
      r2[threadIdx.x] += r2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = r1[0];
    partial[2 * blockIdx.x + 1] = r2[0];
  }
}

// Bitonic network, descending overall (eq. sorted_energy): the pair (i, i ^ j)
// with i < i ^ j keeps the larger value at i when (i & k) == 0, at i ^ j
// otherwise.  Equal values are interchangeable, so only values are sorted.
__device__ __forceinline__ void bitonic_ce(double &lo_v, double &hi_v, bool desc) {
  const double a = lo_v, b = hi_v;
  if (desc ? (a < b) : (a > b)) {
    lo_v = b;
    hi_v = a;
  }
}

// The stages j <= jmax of block sizes k = kfirst, 2 kfirst, .., klast inside
// one LDS-resident block of BIG_SORT_BLOCK values.
__global__ __launch_bounds__(512) void big_sort_block_kernel(double *S, int kfirst, int klast, int jmax) {
  __shared__ double b[BIG_SORT_BLOCK];
  const int64_t base = (int64_t)blockIdx.x * BIG_SORT_BLOCK;
  for (int i = threadIdx.x; i < BIG_SORT_BLOCK; i += blockDim.x) b[i] = S[base + i];
  __syncthreads();
  for (int k = kfirst; k <= klast; k <<= 1) {
    for (int j = min(k >> 1, jmax); j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < BIG_SORT_BLOCK; i += blockDim.x) {
        const int l = i ^ j;
        if (l > i) bitonic_ce(b[i], b[l], ((base + i) & k) == 0);
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < BIG_SORT_BLOCK; i += blockDim.x) S[base + i] = b[i];
}

// One stage (k, j) with j >= BIG_SORT_BLOCK over the whole buffer.
__global__ __launch_bounds__(256) void big_sort_global_kernel(double *S, int64_t n, int64_t k, int64_t j) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = i ^ j;
    if (l > i) {
      double a = S[i], b = S[l];
      bitonic_ce(a, b, (i & k) == 0);
      S[i] = a;
      S[l] = b;
    }
  }
}

// Workgroup reductions and scans in a fixed order: within each wave by
// shuffles, then over the waves' totals (wred holds one value per wave).
template <typename V>
__device__ V big_block_sum(V v, V *wred) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) wred[threadIdx.x >> 6] = v;
  __syncthreads();
  V s = V(0);
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += wred[w];
  return s;
}

template <typename V>
__device__ V big_block_excl_scan(V v, V *wred) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  V inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const V t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  __syncthreads();
  if (lane == 63) wred[wave] = inc;
  __syncthreads();
  V base = V(0);
  for (int w = 0; w < wave; ++w) base += wred[w];
  return base + inc - v;
}

// Term j of eq. (s_delta): the exponential of the relative gap between sorted
// energies j and j + 1 (1 for two zeros, 0 before a zero).
__device__ __forceinline__ double big_sdelta_term(double ea, double eb, double delta) {
  if (eb == 0.0 && ea == 0.0) return 1.0;
  if (eb == 0.0) return 0.0;
  return exp(-(ea / eb - 1.0) / delta);
}

// The sum of eq. (s_delta)'s terms over the first J_max - 1 gaps, in parts: block b
// sums the terms of its range of sorted positions into tpart[b] (all CUs share
// the exponentials; one workgroup had spent most of the scores pass on them).
constexpr int BIG_TERM_BLOCKS = 256;
__global__ __launch_bounds__(256) void big_ems_terms_kernel(const double *S, int J, enufft_ems_params prm,
                                                            double *tpart) {
  __shared__ double wred[4];
  const int Jmax = J < prm.k_max ? J : prm.k_max;
  const int n = max(0, Jmax - 1);
  const int chunk = (n + BIG_TERM_BLOCKS - 1) / BIG_TERM_BLOCKS;
  const int lo = min(n, (int)blockIdx.x * chunk), hi = min(n, lo + chunk);
  double sd = 0.0;
  for (int j = lo + threadIdx.x; j < hi; j += blockDim.x) sd += big_sdelta_term(S[j], S[j + 1], prm.delta);
  sd = big_block_sum(sd, wred);
  if (threadIdx.x == 0) tpart[blockIdx.x] = sd;
}

// Scores over the sorted energies (one workgroup of 1024 threads, each owning
// a contiguous run of sorted positions, read eight at a time with the loads of
// a batch issued together): eqs. (n_eff), (c_score), (alpha_c), (f_cum) and
// (k_elastic), as in the per-cell kernel, with eq. (s_delta) from the parts.
constexpr int BIG_SCORE_BATCH = 8;
__global__ __launch_bounds__(1024) void big_ems_scores_kernel(const double *S, const double *partial, int nparts,
                                                              const double *tpart, int J, enufft_ems_params prm,
                                                              BigCut *cut) {
  __shared__ double wred[16];
  __shared__ int wredi[16];
  __shared__ int s_kc;
  constexpr int B = BIG_SCORE_BATCH;
  const int t = threadIdx.x;
  if (t == 0) s_kc = INT_MAX;
  double pa = 0.0, pb = 0.0;
  for (int i = t; i < nparts; i += blockDim.x) {
    pa += partial[2 * i];
    pb += partial[2 * i + 1];
  }
  const double T1 = big_block_sum(pa, wred);
  const double T2 = big_block_sum(pb, wred);
  const int Jmax = J < prm.k_max ? J : prm.k_max;
  const double neff = T2 > 0.0 ? T1 * T1 / T2 : 0.0;
  const double nclip = neff < (double)Jmax ? neff : (double)Jmax;
  const double sdsum = big_block_sum(t < BIG_TERM_BLOCKS ? tpart[t] : 0.0, wred);
  const double sdel = Jmax < 2 ? 1.0 : sdsum / (double)(Jmax - 1);
  const double Cs = (Jmax > 0 ? prm.w1 * nclip / (double)Jmax : 0.0) + prm.w2 * sdel;
  const double alphaC = prm.alpha_min + (prm.alpha_max - prm.alpha_min) * Cs;
  const int per = (J + 1023) / 1024;
  const int j0 = min(J, t * per), j1 = min(J, j0 + per);
  auto batch = [&](int jb, double (&v)[B]) {
#pragma unroll
    for (int q = 0; q < B; ++q) v[q] = S[min(jb + q, j1 - 1)];   // j1 > jb >= j0 here
  };
  // running sum: per-thread totals, an exclusive scan in thread order, then the threshold
  double loc = 0.0;
  for (int jb = j0; jb < j1; jb += B) {
    double v[B];
    batch(jb, v);
#pragma unroll
    for (int q = 0; q < B; ++q)
      if (jb + q < j1) loc += v[q];
  }
  double run = big_block_excl_scan(loc, wred);
  if (T1 > 0.0) {
    bool found = false;
    for (int jb = j0; jb < j1 && !found; jb += B) {
      double v[B];
      batch(jb, v);
#pragma unroll
      for (int q = 0; q < B; ++q) {
        if (found || jb + q >= j1) continue;
        run += v[q];
        if (run / T1 >= alphaC) {
          atomicMin(&s_kc, jb + q + 1);
          found = true;
        }
      }
    }
  }
  __syncthreads();
  int kstar;
  if (!(T1 > 0.0)) {
    kstar = prm.k_min < J ? prm.k_min : J;
  } else {
    const int kc = s_kc == INT_MAX ? J : s_kc;
    const int k = kc > prm.k_min ? kc : prm.k_min;
    kstar = k < Jmax ? k : Jmax;
  }
  const double eth = kstar > 0 ? S[kstar - 1] : 0.0;
  double part = 0.0;
  int cgt = 0, ceq = 0;
  for (int jb = j0; jb < j1; jb += B) {
    double v[B];
    batch(jb, v);
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int j = jb + q;
      if (j >= j1) continue;
      if (j < kstar) part += v[q];
      cgt += v[q] > eth;
      ceq += v[q] == eth;
    }
  }
  const double th = big_block_sum(part, wred);
  const int ngt = big_block_sum(cgt, wredi);
  const int neq = big_block_sum(ceq, wredi);
  if (t == 0) {
    cut->T1 = T1; cut->T2 = T2; cut->neff = neff; cut->sdel = sdel; cut->Cs = Cs; cut->alphaC = alphaC;
    cut->th = th; cut->eth = eth; cut->kstar = kstar; cut->need = kstar - ngt;
    cut->split = kstar > 0 && neq > kstar - ngt;
    cut->J = J;
  }
}

// Units tied at the cut energy when not all of them are kept: the `need` tied
// units of lowest id are kept (one workgroup, units in id order).
template <typename T>
__global__ __launch_bounds__(1024) void big_ems_ties_kernel(const T *f, const double *mw, const int2 *units, int J,
                                                            const BigCut *cut, uint8_t *tie_kept) {
  if (!cut->split) return;
  using C = typename vec2<T>::type;
  const C *fc = reinterpret_cast<const C *>(f);
  __shared__ int cnt[1024];
  const double eth = cut->eth;
  const int need = cut->need;
  const int per = (J + 1023) / 1024;
  const int u0 = min(J, (int)threadIdx.x * per), u1 = min(J, u0 + per);
  int c = 0;
  for (int u = u0; u < u1; ++u) {
    const int2 un = units[u];
    c += big_pair_energy<C>(fc, mw, un.x, un.y) == eth;
  }
  cnt[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int i = 0; i < 1024; ++i) {
      const int v = cnt[i];
      cnt[i] = run;
      run += v;
    }
  }
  __syncthreads();
  int rank = cnt[threadIdx.x];
  for (int u = u0; u < u1; ++u) {
    const int2 un = units[u];
    const bool tie = big_pair_energy<C>(fc, mw, un.x, un.y) == eth;
    tie_kept[u] = tie && rank < need;
    rank += tie;
  }
}

// Keep mask over the modes and per-workgroup partials of the retained power.
template <typename T>
__global__ __launch_bounds__(256) void big_ems_keep_kernel(const T *f, const double *mw, const int4 *mode_unit, int M,
                                                           const BigCut *cut, const uint8_t *tie_kept, uint8_t *keep,
                                                           double *partial) {
  using C = typename vec2<T>::type;
  const C *fc = reinterpret_cast<const C *>(f);
  __shared__ double red[256];
  const int m = blockIdx.x * 256 + threadIdx.x;
  double pw = 0.0;
  if (m < M) {
    const int4 mu = mode_unit[m];
    uint8_t v = 0;
    if (cut->kstar > 0 && mu.x >= 0) {
      const double eu = big_pair_energy<C>(fc, mw, mu.x, mu.y);
      v = eu > cut->eth || (eu == cut->eth && (!cut->split || tie_kept[mu.z]));
    }
    keep[m] = v;
    if (v) {
      const C fr = fc[m];
      pw = (double)fr.x * (double)fr.x + (double)fr.y * (double)fr.y;
    }
  }
  red[threadIdx.x] = pw;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void big_ems_finish_kernel(const BigCut *cut, const double *partial, int nparts,
                                                             int32_t *k_star, double *stats) {
  __shared__ double wred[4];
  double v = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) v += partial[i];
  const double P = big_block_sum(v, wred);
  if (threadIdx.x != 0) return;
  *k_star = cut->kstar;
  stats[0] = cut->T1;
  stats[1] = P;
  stats[2] = cut->neff;
  stats[3] = cut->sdel;
  stats[4] = cut->Cs;
  stats[5] = cut->alphaC;
  stats[6] = cut->T1 > 0.0 ? cut->th / cut->T1 : 0.0;
  stats[7] = (double)cut->J;
}

// ------------------------------------------------------------------ adjoint for one large cell

// Column pass of the adjoint.  The cotangent gbar (2 lam_c f keep for the
// retained-power loss) times the deconvolution factors, made Hermitian
// (H(k) = (G(k) + conj G(-k)) / 2, so the grids are real), and the same times
// i ky, each inverse transformed along y into cb / cby (columns kx = 0..K1).
template <typename T>
__global__ __launch_bounds__(512) void big_adj_cols_kernel(const T *fin, const uint8_t *keep, const double *lam,
                                                           int64_t cell, Geom g, const T *tw2, const T *decon_x,
                                                           const T *decon_y, T *cb, T *cby) {
  extern __shared__ __align__(16) unsigned char sm_raw[];
  const int n2 = g.n2;
  T *A = reinterpret_cast<T *>(sm_raw), *B = A + 2 * n2;
  const int kx = blockIdx.x;
  const int hi1 = g.lo1 + g.N1 - 1, hi2 = g.lo2 + g.N2 - 1;
  const T sc_keep = keep ? T(2.0 * (lam ? lam[cell] : 1.0)) : T(1);
  for (int pass = 0; pass < 2; ++pass) {
    for (int bin = threadIdx.x; bin < n2; bin += blockDim.x) {
      const int ky = bin <= n2 / 2 ? bin : bin - n2;
      T hr = 0, hi = 0;
      if (ky >= -g.K2 && ky <= g.K2) {
        if (kx <= hi1 && ky >= g.lo2 && ky <= hi2) {
          const int64_t m = (int64_t)(ky - g.lo2) * g.N1 + (kx - g.lo1);
          const T sc = keep ? (keep[m] ? sc_keep : T(0)) : T(1);
          hr += sc * fin[2 * m];
          hi += sc * fin[2 * m + 1];
        }
        if (-kx >= g.lo1 && -ky >= g.lo2 && -ky <= hi2) {
          const int64_t m = (int64_t)(-ky - g.lo2) * g.N1 + (-kx - g.lo1);
          const T sc = keep ? (keep[m] ? sc_keep : T(0)) : T(1);
          hr += sc * fin[2 * m];
          hi -= sc * fin[2 * m + 1];
        }
        const T s = T(0.5) * decon_x[kx] * decon_y[ky < 0 ? -ky : ky];
        hr *= s;
        hi *= s;
      }
      if (pass == 0) {
        A[2 * bin] = hr;
        A[2 * bin + 1] = hi;
      } else {   // times i ky
        A[2 * bin] = -T(ky) * hi;
        A[2 * bin + 1] = T(ky) * hr;
      }
    }
    __syncthreads();
    const T *Z = stockham<true, T>(A, B, n2, tw2);
    T *c = (pass == 0 ? cb : cby) + (int64_t)kx * n2 * 2;
    for (int i = threadIdx.x; i < 2 * n2; i += blockDim.x) c[i] = Z[i];
    __syncthreads();
  }
}

// Row pass of the adjoint for rows 2p and 2p + 1, three inverse transforms of
// length n1: u + i du/dx of row 2p (spectrum D + i (i kx D) = (1 - kx) D), the
// same for row 2p + 1, and du/dy of row 2p + i du/dy of row 2p + 1.  Bins
// kx < 0 are the conjugates of column -kx (the grids are real).
template <typename T>
__global__ __launch_bounds__(512) void big_adj_rows_kernel(const T *cb, const T *cby, Geom g, const T *tw1,
                                                           typename vec4<T>::type *G4) {
  extern __shared__ __align__(16) unsigned char sm_raw[];
  const int n1 = g.n1, n2 = g.n2;
  T *A = reinterpret_cast<T *>(sm_raw), *B = A + 2 * n1;
  const int p = blockIdx.x;
  const int64_t r0 = (int64_t)(2 * p) * n1, r1 = r0 + n1;
  for (int pass = 0; pass < 3; ++pass) {
    for (int k = threadIdx.x; k < n1; k += blockDim.x) {
      const int kk = k <= n1 / 2 ? k : n1 - k;
      const bool neg = k != kk;
      T zr = 0, zi = 0;
      if (kk <= g.K1) {
        const T *src = (pass == 2 ? cby : cb) + (int64_t)kk * n2 * 2 + 4 * p;
        T a0r = src[0], a0i = src[1], a1r = src[2], a1i = src[3];
        if (neg) {
          a0i = -a0i;
          a1i = -a1i;
        }
        if (pass < 2) {
          const T kf = neg ? -T(kk) : T(kk);
          const T dr = pass == 0 ? a0r : a1r, di = pass == 0 ? a0i : a1i;
          zr = dr - kf * dr;
          zi = di - kf * di;
        } else {
          zr = a0r - a1i;
          zi = a0i + a1r;
        }
      }
      A[2 * k] = zr;
      A[2 * k + 1] = zi;
    }
    __syncthreads();
    const T *Z = stockham<true, T>(A, B, n1, tw1);
    for (int i = threadIdx.x; i < n1; i += blockDim.x) {
      if (pass == 0) {
        G4[r0 + i].x = Z[2 * i];
        G4[r0 + i].y = Z[2 * i + 1];
      } else if (pass == 1) {
        G4[r1 + i].x = Z[2 * i];
        G4[r1 + i].y = Z[2 * i + 1];
      } else {
        G4[r0 + i].z = Z[2 * i];
        G4[r0 + i].w = T(0);
        G4[r1 + i].z = Z[2 * i + 1];
        G4[r1 + i].w = T(0);
      }
    }
    __syncthreads();
  }
}

// Gather (the type-2 interpolation back to the points) from the three grids,
// each tile run staging its sub-grid of u, du/dx and du/dy in LDS.
// FP32 stages (u, du/dx, du/dy, 0) as one 16-byte vector per cell (one read per
// tap); FP64 as three planes of doubles: 24 instead of 32 bytes per cell, so three
// 256-thread workgroups share a CU instead of two at W = 12.
template <typename T, int W>
constexpr size_t big_gather_lds() {
  constexpr size_t n = (size_t)(BIG_TS + W + 1) * (BIG_TS + W + 1);
  return sizeof(T) == 8 ? 3 * n * sizeof(double) : n * sizeof(typename vec4<T>::type);
}

template <typename T, int W, bool POLY>
__global__ __launch_bounds__(256) void big_gather_kernel(BigTileArgs<T> a) {
  constexpr int S = BIG_TS + W + 1;
  using V4 = typename vec4<T>::type;
  extern __shared__ __align__(32) unsigned char sm_raw[];
  V4 *sg = reinterpret_cast<V4 *>(sm_raw);   // FP32: [S * S] staged (u, du/dx, du/dy, 0)
  T *su = reinterpret_cast<T *>(sm_raw);     // FP64: [S * S] u, then du/dx, then du/dy
  T *sx = su + S * S, *sy = sx + S * S;
  __shared__ int s_unit;
  const Geom &g = a.g;
  const T halfw = T(W) / T(2);
  const double *wn = a.windows + 3 * a.cell;
  const T cx = T(wn[0]), cy = T(wn[1]), R = T(wn[2]);
  const T pr = R > T(0) ? T(M_PI) / R : T(0);
  const bool pre = *a.presorted;
  const T *X = pre ? a.xi : a.xs, *Y = pre ? a.yi : a.ys, *Hh = pre ? a.hi : a.hs, *Wq = pre ? a.wi : a.ws;
  big_units<T>(a, &s_unit, [&](int t, int64_t lo, int64_t hi, int) {
    const int tx0 = (t % a.ntx) * BIG_TS, ty0 = (t / a.ntx) * BIG_TS;
    for (int i = threadIdx.x; i < S * S; i += blockDim.x) {
      const int r = i / S, q = i - r * S;
      const V4 v = a.G4[(int64_t)((ty0 - 1 + r) & (g.n2 - 1)) * g.n1 + ((tx0 - 1 + q) & (g.n1 - 1))];
      if constexpr (sizeof(T) == 8) {
        su[i] = v.x;
        sx[i] = v.y;
        sy[i] = v.z;
      } else {
        sg[i] = v;
      }
    }
    __syncthreads();
    for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) {
      const T xj = X[k], yj = Y[k];
      const FineCoord<T> fx = fine_coord<T>(xj, a.s1h, a.s1l, halfw);
      const FineCoord<T> fy = fine_coord<T>(yj, a.s2h, a.s2l, halfw);
      const int lx = big_local(fx.i0 & (g.n1 - 1), tx0, g.n1);
      const int ly = big_local(fy.i0 & (g.n2 - 1), ty0, g.n2);
      T kx[W];
      big_taps<T, W, POLY>(fx, a.beta, a.es, a.es64, kx);
      T u = 0, ux = 0, uy = 0;
      auto row = [&](int dy, T kyv) {
        const int rb = (ly + dy) * S + lx;
        T au = 0, ax = 0, ay = 0;
#pragma unroll
        for (int dx = 0; dx < W; ++dx) {
          if constexpr (sizeof(T) == 8) {
            au += kx[dx] * su[rb + dx];
            ax += kx[dx] * sx[rb + dx];
            ay += kx[dx] * sy[rb + dx];
          } else {
            const V4 v = sg[rb + dx];
            au += kx[dx] * v.x;
            ax += kx[dx] * v.y;
            ay += kx[dx] * v.z;
          }
        }
        u += kyv * au;
        ux += kyv * ax;
        uy += kyv * ay;
      };
      // one row at a time keeps the loads of W rows from being hoisted together
      if constexpr (POLY) {
        T ky[W];
        big_taps<T, W, POLY>(fy, a.beta, a.es, a.es64, ky);
#pragma unroll 1
        for (int dy = 0; dy < W; ++dy) {
          T kyv = ky[0];
#pragma unroll
          for (int q = 1; q < W; ++q) kyv = dy == q ? ky[q] : kyv;   // register select, no indexed access
          row(dy, kyv);
        }
      } else {
        bool done = false;
        if constexpr (sizeof(T) == 8 && W % 2 == 0 && W <= ES64_MAXW) {
          if (a.es64.on) {
            const double uy64 = tap_u64(fy, double(W) * 0.5);
#pragma unroll 1
            for (int dy = 0; dy < W; ++dy) row(dy, es_tap_poly64<W>(uy64, a.es64, dy));
            done = true;
          }
        }
        if (!done) {
          const T zsc = T(2) / T(W);
#pragma unroll 1
          for (int dy = 0; dy < W; ++dy) row(dy, ker_eval(fy.offset(dy) * zsc, a.beta));
        }
      }
      T dWx, dWy;
      const T Wv = hann_wg(a.window_kind, xj, yj, cx, cy, R, pr, dWx, dWy);
      const T wj = Wq[k], wh = wj * Hh[k];
      V4 o;
      o.x = wj * Wv * u;
      o.y = wh * (dWx * u + Wv * ux);
      o.z = wh * (dWy * u + Wv * uy);
      o.w = T(0);
      if (pre) {   // the sorted position is the input position: the gradients go straight out
        if (a.gh) a.gh[k] = o.x;
        if (a.gx) a.gx[k] = o.y;
        if (a.gy) a.gy[k] = o.z;
      } else {
        a.gout[k] = o;   // sorted order, coalesced; the unpermute pass puts it at the input index
      }
    }
    __syncthreads();
  });
}

// Gradients back to input order: one read of the sorted-order record per point
// (at its sorted position) and coalesced writes of the three outputs.  Input
// already in tile order needs none: the gather wrote the gradients itself.
template <typename T>
__global__ __launch_bounds__(256) void big_unpermute_kernel(const typename vec4<T>::type *gout, const int *inv,
                                                            const int *presorted, int64_t n, T *gh, T *gx, T *gy) {
  if (*presorted) return;   // sorted order is the input order: the gather wrote the gradients
  // U points per thread and round, all loads of a round before its stores (the
  // stores could alias the records as far as the compiler knows, so a store
  // between loads would serialise them)
  constexpr int U = 4;
  using V4 = typename vec4<T>::type;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j0 < n; j0 += U * stride) {
    int k[U];
    V4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + u * stride;
      k[u] = j < n ? inv[j] : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = k[u] >= 0 && k[u] < n;   // false only past the end (or if the sort's passes disagreed)
      v[u] = gout[ok ? k[u] : 0];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + u * stride;
      if (j >= n || k[u] < 0 || k[u] >= n) continue;
      if (gh) gh[j] = v[u].x;
      if (gx) gx[j] = v[u].y;
      if (gy) gy[j] = v[u].z;
    }
  }
}

// Second pass of the one-time point sort (enufft_sort_points): inside each
// tile, by the fine cell of the footprint origin (big_key).  The work units of
// the tile order (pieces of at most BIG_UNIT_CHUNK points, one tile each) share
// the tiles' points out, so a crowded tile is spread over many workgroups:
//   1. per unit, its cell histogram (LDS) written to uh[unit][cell];
//   2. per tile, the cells' starts (a scan over the cells of the units' totals)
//      and each unit's start in every cell, in place in uh;
//   3. per unit, every point moved to its cell's next slot, with its input index
//      when pin is given, through LDS in cell order (below).
// The order inside a cell is not fixed (LDS atomics rank the points).
constexpr int BIG_CS_THREADS = 1024;
constexpr int BIG_CS_PER = BIG_UNIT_CHUNK / BIG_CS_THREADS;   // points per thread and unit

// The sorted range [k0, k1) of unit u and its tile; false past the last unit.
template <typename T>
__device__ __forceinline__ bool big_unit_range(const BigSortArgs<T> &a, int u, int &t, int64_t &k0, int64_t &k1) {
  if (u >= a.unit_base[a.ntiles]) return false;
  int lo = 0, hi = a.ntiles - 1;   // the largest t with unit_base[t] <= u
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.unit_base[mid] <= u) lo = mid;
    else hi = mid - 1;
  }
  t = lo;
  const int64_t t0 = a.offsets[t], t1 = a.offsets[t + 1];
  const int64_t c = t0 / BIG_UNIT_CHUNK + (u - a.unit_base[t]);
  k0 = max(t0, c * BIG_UNIT_CHUNK);
  k1 = min(t1, (c + 1) * BIG_UNIT_CHUNK);
  return k0 < k1;
}

template <typename T>
__global__ __launch_bounds__(BIG_CS_THREADS) void big_cell_count_kernel(BigSortArgs<T> a, const T *xt, const T *yt,
                                                                        int *uh) {
  __shared__ int cnt[BIG_TS2];
  int t;
  int64_t k0, k1;
  if (!big_unit_range<T>(a, blockIdx.x, t, k0, k1)) return;   // the whole workgroup
  for (int i = threadIdx.x; i < BIG_TS2; i += BIG_CS_THREADS) cnt[i] = 0;
  __syncthreads();
  int key[BIG_CS_PER];
#pragma unroll
  for (int j = 0; j < BIG_CS_PER; ++j) {   // every load issued before the first add
    const int64_t k = k0 + threadIdx.x + (int64_t)j * BIG_CS_THREADS;
    key[j] = k < k1 ? big_key<T>(a, xt[k], yt[k]) % BIG_TS2 : -1;
  }
#pragma unroll
  for (int j = 0; j < BIG_CS_PER; ++j)
    if (key[j] >= 0) atomicAdd(&cnt[key[j]], 1);
  __syncthreads();
  for (int i = threadIdx.x; i < BIG_TS2; i += BIG_CS_THREADS) uh[(int64_t)blockIdx.x * BIG_TS2 + i] = cnt[i];
}

__global__ __launch_bounds__(BIG_CS_THREADS) void big_cell_scan_kernel(const int64_t *offsets, const int *unit_base,
                                                                       int *uh) {
  __shared__ int tot[BIG_TS2];
  __shared__ int wsum[16];
  const int t = blockIdx.x, c = threadIdx.x;   // one thread per cell of tile t
  const int u0 = unit_base[t], u1 = unit_base[t + 1];
  int n = 0;
  for (int u = u0; u < u1; ++u) n += uh[(int64_t)u * BIG_TS2 + c];
  tot[c] = n;
  __syncthreads();
  big_block_scan<BIG_CS_THREADS, int>(tot, tot, BIG_TS2, wsum);
  int run = (int)offsets[t] + tot[c];
  for (int u = u0; u < u1; ++u) {
    int *p = uh + (int64_t)u * BIG_TS2 + c;
    const int v = *p;
    *p = run;
    run += v;
  }
}

// Step 3, staged: the unit in sub-chunks of SUB points, each loaded once
// (coalesced), ranked inside its cells (LDS counts, their scan), placed in LDS in
// cell order, and written out with consecutive threads on consecutive slots of
// each cell's range, so a cell's points leave as contiguous stores.
template <typename T>
__global__ __launch_bounds__(BIG_CS_THREADS) void big_cell_scatter_kernel(BigSortArgs<T> a, const T *xt, const T *yt,
                                                                          const T *ht, const T *wt,
                                                                          const int32_t *pin, const int *uh, T *xo,
                                                                          T *yo, T *ho, T *wo, int32_t *pout) {
  constexpr int SUB = sizeof(T) == 4 ? 2048 : 1024;
  constexpr int PT = SUB / BIG_CS_THREADS;
  static_assert(BIG_TS2 == BIG_CS_THREADS && PT >= 1, "one thread per cell of a tile");
  using V4 = typename vec4<T>::type;
  __shared__ int cur[BIG_TS2];   // this unit's next global slot in each cell
  __shared__ int lh[BIG_TS2];    // the sub-chunk's count per cell, then its start in the staged order
  __shared__ int wsum[16];
  __shared__ V4 st[SUB];         // the sub-chunk in cell order
  __shared__ int sk[SUB], sp[SUB];
  int t;
  int64_t k0, k1;
  if (!big_unit_range<T>(a, blockIdx.x, t, k0, k1)) return;   // the whole workgroup
  const int c = threadIdx.x;   // the cell this thread keeps the counts of
  cur[c] = uh[(int64_t)blockIdx.x * BIG_TS2 + c];
  const int64_t e0 = a.offsets[t], e1 = a.offsets[t + 1];
  for (int64_t p0 = k0; p0 < k1; p0 += SUB) {
    const int m = (int)min<int64_t>(SUB, k1 - p0);
    lh[c] = 0;
    __syncthreads();
    V4 v[PT];
    int key[PT], rk[PT], pi[PT];
#pragma unroll
    for (int j = 0; j < PT; ++j) {   // every load issued before the first is used
      const int q = min(c + j * BIG_CS_THREADS, m - 1);
      v[j].x = xt[p0 + q];
      v[j].y = yt[p0 + q];
      v[j].z = ht[p0 + q];
      v[j].w = wt[p0 + q];
      pi[j] = pin ? pin[p0 + q] : 0;
    }
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      const bool on = c + j * BIG_CS_THREADS < m;
      key[j] = big_key<T>(a, v[j].x, v[j].y) % BIG_TS2;
      rk[j] = on ? atomicAdd(&lh[key[j]], 1) : 0;
    }
    __syncthreads();
    const int mine = lh[c];
    big_block_scan<BIG_CS_THREADS, int>(lh, lh, BIG_TS2, wsum);
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      if (c + j * BIG_CS_THREADS >= m) continue;
      const int slot = lh[key[j]] + rk[j];   // < m: the rank is below the cell's count
      st[slot] = v[j];
      sk[slot] = key[j];
      sp[slot] = pi[j];
    }
    __syncthreads();
    for (int i = c; i < m; i += BIG_CS_THREADS) {
      const int ki = sk[i];
      const int64_t pos = (int64_t)cur[ki] + (i - lh[ki]);
      if (pos < e0 || pos >= e1) continue;   // only if the passes disagreed on a key; never out of the tile's range
      const V4 w4 = st[i];
      xo[pos] = w4.x;
      yo[pos] = w4.y;
      if (ho) ho[pos] = w4.z;
      if (wo) wo[pos] = w4.w;
      if (pout) pout[pos] = sp[i];
    }
    __syncthreads();
    cur[c] += mine;
  }
}

// perm[inv[j]] = base + j: the input index of each sorted position.
__global__ __launch_bounds__(256) void big_perm_kernel(const int *inv, int64_t n, int32_t base, int32_t *perm) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    const int k = inv[j];
    if (k >= 0 && k < n) perm[k] = base + (int32_t)j;
  }
}

// ------------------------------------------------------------------ host side

namespace {

enufft_status big_fail(enufft_plan_t p, hipError_t e, const char *what) {
  if (e == hipSuccess) return ENUFFT_OK;
  p->last_error = std::string(what) + ": " + hipGetErrorString(e);
  if (e == hipErrorMemoryAllocation || e == hipErrorOutOfMemory) return ENUFFT_ENOMEM;
  if (e != hipErrorInvalidValue) p->faulted = true;
  return ENUFFT_EDEVICE;
}

int stock_threads(int n) { return std::min(512, std::max(64, n / 2)); }

template <typename T>
size_t sort_lds(int ntiles) {
  return (size_t)big_scatter_sub<T>() * sizeof(typename vec4<T>::type) + (size_t)3 * ntiles * sizeof(int);
}

size_t count_lds(int ntiles) { return ((size_t)ntiles + BIG_SORT_CHUNK) * sizeof(int); }

template <typename T>
hipError_t set_attrs_t(int n1, int n2, int ntiles) {
  const size_t el = sizeof(T);
  auto set = [](const void *fn, size_t bytes) {
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  };
  hipError_t e = set((const void *)&big_count_kernel<T>, count_lds(ntiles));
  if (e == hipSuccess) e = set((const void *)&big_scatter_kernel<T>, sort_lds<T>(ntiles));
  if (e == hipSuccess) e = set((const void *)&big_tile_scan_kernel, (size_t)ntiles * sizeof(int));
  if (e == hipSuccess) e = set((const void *)&big_rows_kernel<T>, 4 * (size_t)n1 * el);
  if (e == hipSuccess) e = set((const void *)&big_cols_kernel<T>, 4 * (size_t)n2 * el);
  if (e == hipSuccess) e = set((const void *)&big_adj_cols_kernel<T>, 4 * (size_t)n2 * el);
  if (e == hipSuccess) e = set((const void *)&big_adj_rows_kernel<T>, 4 * (size_t)n1 * el);
  return e;
}

template <typename T>
BigSortArgs<T> sort_args(enufft_plan_t p, int64_t c, const T *x, const T *y, const T *h, const T *w) {
  const int64_t a0 = p->offsets[c];
  BigSortArgs<T> a{};
  a.x = x + a0; a.y = y + a0; a.h = h ? h + a0 : nullptr; a.w = w + a0;
  a.n = p->offsets[c + 1] - a0;
  split_scale<T>(p->n1, &a.s1h, &a.s1l);
  split_scale<T>(p->n2, &a.s2h, &a.s2l);
  a.W = p->W; a.n1 = p->n1; a.n2 = p->n2;
  a.ntx = p->big_ntx; a.ntiles = p->big_ntx * p->big_nty;
  a.nchunks = (int)((a.n + BIG_SORT_CHUNK - 1) / BIG_SORT_CHUNK);
  a.ngroups = (a.nchunks + BIG_SCAN_GROUP - 1) / BIG_SCAN_GROUP;
  a.chunk_hist = p->big_chunk_hist; a.group_sum = p->big_group_sum;
  a.offsets = p->big_offsets; a.unit_base = p->big_unit_base; a.inv = p->big_inv;
  a.xs = (T *)p->big_xs; a.ys = (T *)p->big_ys; a.hs = (T *)p->big_hs; a.ws = (T *)p->big_ws;
  a.chunk_fl = p->big_chunk_fl;
  a.presorted = p->big_flags;
  return a;
}

// Sort the points of cell c (n > 0) by tile into the plan's buffers: chunk
// histograms, group sums, the tile scan, chunk starts, scatter.
template <typename T>
hipError_t sort_launch(enufft_plan_t p, const BigSortArgs<T> &a) {
  const dim3 tg((a.ntiles + 255) / 256, a.ngroups);
  hipLaunchKernelGGL((big_count_kernel<T>), dim3(a.nchunks), dim3(BIG_SORT_THREADS), count_lds(a.ntiles),
                     p->stream, a);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(big_group_sum_kernel, tg, dim3(256), 0, p->stream, (const int *)a.chunk_hist, a.nchunks,
                       a.ntiles, a.group_sum);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(big_tile_scan_kernel, dim3(1), dim3(1024), (size_t)a.ntiles * sizeof(int), p->stream,
                       a.group_sum, a.ngroups, a.ntiles, a.offsets, a.unit_base, (const int *)a.chunk_fl, a.nchunks,
                       a.presorted);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(big_chunk_base_kernel, tg, dim3(256), 0, p->stream, a.chunk_hist,
                       (const int *)a.group_sum, (const int64_t *)a.offsets, a.nchunks, a.ntiles);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL((big_scatter_kernel<T>), dim3(a.nchunks), dim3(BIG_SORT_THREADS), sort_lds<T>(a.ntiles),
                       p->stream, a);
    e = hipGetLastError();
  }
  return e;
}

template <typename T>
hipError_t sort_cell(enufft_plan_t p, int64_t c, const T *x, const T *y, const T *h, const T *w) {
  return sort_launch<T>(p, sort_args<T>(p, c, x, y, h, w));
}

// The tile ranges, unit offsets and order flags a call uses for cell c: those
// that enufft_bind_points stored when x and y are the bound arrays (the call
// then sorts nothing), else the plan's, which the call's own sort fills.
struct CellMeta {
  int64_t *offsets;
  int *unit_base;
  int *flags;
  bool bound;
};
CellMeta cell_meta(enufft_plan_t p, int64_t c, const void *x, const void *y) {
  const int64_t nt1 = (int64_t)p->big_ntx * p->big_nty + 1;
  if (p->bound_x && x == p->bound_x && y == p->bound_y)
    return CellMeta{p->bound_offsets + c * nt1, p->bound_unit_base + c * nt1, p->bound_flags + 4 * c, true};
  return CellMeta{p->big_offsets, p->big_unit_base, p->big_flags, false};
}

template <typename T>
BigTileArgs<T> tile_args(enufft_plan_t p, int64_t c, const T *x, const T *y, const T *h, const T *w,
                         const CellMeta &m) {
  BigTileArgs<T> a{};
  a.xs = (const T *)p->big_xs; a.ys = (const T *)p->big_ys; a.hs = (const T *)p->big_hs; a.ws = (const T *)p->big_ws;
  const int64_t a0 = p->offsets[c];
  a.xi = x + a0; a.yi = y + a0; a.hi = h + a0; a.wi = w + a0;
  a.presorted = m.flags;
  a.offsets = m.offsets;
  a.unit_base = m.unit_base;
  a.ntiles = p->big_ntx * p->big_nty;
  a.ntx = p->big_ntx;
  a.n = p->offsets[c + 1] - p->offsets[c];
  a.windows = (const double *)p->d_windows;
  a.cell = c;
  a.window_kind = p->window_kind;
  a.g = p->geom;
  split_scale<T>(p->n1, &a.s1h, &a.s1l);
  split_scale<T>(p->n2, &a.s2h, &a.s2l);
  a.beta = (T)p->beta;
  a.es = p->es;
  if constexpr (sizeof(T) == 8) a.es64 = p->es64;
  else a.es64.on = 0;
  return a;
}

// Persistent workgroups for the unit passes (the unit count is known only on
// the device; idle workgroups exit at once).
int tile_blocks(enufft_plan_t p, int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)p->n_cu * 8, p->big_units_max));
}

template <typename T, int W, bool POLY>
struct SpreadW {
  static hipError_t run(const BigTileArgs<T> &a, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((big_spread_kernel<T, W, POLY>), dim3(blocks), dim3(BIG_SPREAD_THREADS), 0, s, a);
    return hipGetLastError();
  }
};
template <typename T, int W, bool POLY>
struct GatherW {
  static hipError_t run(const BigTileArgs<T> &a, int blocks, hipStream_t s) {
    const size_t lds = big_gather_lds<T, W>();
    hipLaunchKernelGGL((big_gather_kernel<T, W, POLY>), dim3(blocks), dim3(256), lds, s, a);
    return hipGetLastError();
  }
  static hipError_t attr() {
    return hipFuncSetAttribute((const void *)&big_gather_kernel<T, W, POLY>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)big_gather_lds<T, W>());
  }
};

// Launch of the run kernel for FP32 plans with the kernel polynomial.
hipError_t spread_runs(int W, const BigTileArgs<float> &a, int blocks, hipStream_t s) {
  switch (W) {
    case 4: hipLaunchKernelGGL((big_spread_run_kernel<4>), dim3(blocks), dim3(BIG_SPREAD_THREADS), 0, s, a); break;
    case 6: hipLaunchKernelGGL((big_spread_run_kernel<6>), dim3(blocks), dim3(BIG_SPREAD_THREADS), 0, s, a); break;
    case 8: hipLaunchKernelGGL((big_spread_run_kernel<8>), dim3(blocks), dim3(BIG_SPREAD_THREADS), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Width dispatch; the polynomial taps exist for FP32 plans with W <= ES_MAXW.
template <typename T, template <typename, int, bool> class Fn>
hipError_t by_width(int W, const BigTileArgs<T> &a, int blocks, hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    if (a.es.on) {
      switch (W) {
        case 4: return Fn<T, 4, true>::run(a, blocks, s);
        case 6: return Fn<T, 6, true>::run(a, blocks, s);
        case 8: return Fn<T, 8, true>::run(a, blocks, s);
        default: return hipErrorInvalidValue;
      }
    }
  }
  switch (W) {
    case 4: return Fn<T, 4, false>::run(a, blocks, s);
    case 6: return Fn<T, 6, false>::run(a, blocks, s);
    case 8: return Fn<T, 8, false>::run(a, blocks, s);
    case 10: return Fn<T, 10, false>::run(a, blocks, s);
    case 12: return Fn<T, 12, false>::run(a, blocks, s);
    case 14: return Fn<T, 14, false>::run(a, blocks, s);
    case 16: return Fn<T, 16, false>::run(a, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

// Dynamic LDS limits of every gather variant (the FP64 wide ones exceed 64 KB).
template <typename T>
hipError_t gather_attrs() {
  hipError_t e = hipSuccess;
  if constexpr (sizeof(T) == 4) {
    if (e == hipSuccess) e = GatherW<T, 4, true>::attr();
    if (e == hipSuccess) e = GatherW<T, 6, true>::attr();
    if (e == hipSuccess) e = GatherW<T, 8, true>::attr();
  }
  if (e == hipSuccess) e = GatherW<T, 4, false>::attr();
  if (e == hipSuccess) e = GatherW<T, 6, false>::attr();
  if (e == hipSuccess) e = GatherW<T, 8, false>::attr();
  if (e == hipSuccess) e = GatherW<T, 10, false>::attr();
  if (e == hipSuccess) e = GatherW<T, 12, false>::attr();
  if (e == hipSuccess) e = GatherW<T, 14, false>::attr();
  if (e == hipSuccess) e = GatherW<T, 16, false>::attr();
  return e;
}

template <typename T>
enufft_status type1_t(enufft_plan_t p, const T *x, const T *y, const T *h, const T *w, T *f, int64_t c0,
                      int64_t c1) {
  const Geom &g = p->geom;
  const size_t el = sizeof(T);
  const int64_t n12 = (int64_t)g.n1 * g.n2;
  for (int64_t c = c0; c < c1; ++c) {
    const int64_t n = p->offsets[c + 1] - p->offsets[c];
    hipError_t e = hipSuccess;
    if (n == 0) {
      e = fill<double>(p->big_grid, n12, 0.0, p->stream);
    } else {
      const CellMeta m = cell_meta(p, c, x, y);
      if (!m.bound) e = sort_cell<T>(p, c, x, y, h, w);
      if (e == hipSuccess) {
        BigTileArgs<T> a = tile_args<T>(p, c, x, y, h, w, m);
        a.partial = p->big_partial;
        a.work_counter = p->big_work;
        a.done_counter = p->big_work + 1;
        e = by_width<T, SpreadW>(p->W, a, tile_blocks(p, n), p->stream);
        // cells whose points are in fine-cell order: the run kernel (the kernel
        // above returned at once for them; the flag is known on the device only)
        if constexpr (sizeof(T) == 4) {
          if (e == hipSuccess && a.es.on) e = spread_runs(p->W, a, tile_blocks(p, n), p->stream);
        }
      }
      if (e == hipSuccess) {
        hipLaunchKernelGGL(big_assemble_kernel, dim3((unsigned)((n12 + 255) / 256)), dim3(256), 0, p->stream,
                           (const double *)p->big_partial, (const int *)m.unit_base, g, p->big_ntx, p->big_nty,
                           BIG_TS + p->W + 1, p->big_grid);
        e = hipGetLastError();
      }
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL((big_rows_kernel<T>), dim3(g.n2 / 2), dim3(stock_threads(g.n1)), 4 * (size_t)g.n1 * el,
                         p->stream, (const double *)p->big_grid, g, (const T *)p->d_tw1, (T *)p->big_cb);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL((big_cols_kernel<T>), dim3(g.K1 + 1), dim3(stock_threads(g.n2)), 4 * (size_t)g.n2 * el,
                         p->stream, (const T *)p->big_cb, g, (const T *)p->d_tw2, (const T *)p->d_decon_x,
                         (const T *)p->d_decon_y, f + c * (int64_t)g.N1 * g.N2 * 2);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return big_fail(p, e, "large-cell type-1");
  }
  return ENUFFT_OK;
}

template <typename T>
enufft_status adjoint_t(enufft_plan_t p, const T *x, const T *y, const T *h, const T *w, const T *fin,
                        const uint8_t *keep, const double *lam, T *gh, T *gx, T *gy) {
  const Geom &g = p->geom;
  const int64_t M = (int64_t)g.N1 * g.N2;
  const size_t el = sizeof(T);
  using V4 = typename vec4<T>::type;
  for (int64_t c = 0; c < p->n_cells; ++c) {
    const int64_t a0 = p->offsets[c], n = p->offsets[c + 1] - a0;
    if (n == 0) continue;
    const CellMeta m = cell_meta(p, c, x, y);
    hipError_t e = m.bound ? hipSuccess : sort_cell<T>(p, c, x, y, h, w);
    if (e == hipSuccess) {
      hipLaunchKernelGGL((big_adj_cols_kernel<T>), dim3(g.K1 + 1), dim3(stock_threads(g.n2)), 4 * (size_t)g.n2 * el,
                         p->stream, fin + c * M * 2, keep ? keep + c * M : nullptr, lam, c, g, (const T *)p->d_tw2,
                         (const T *)p->d_decon_x, (const T *)p->d_decon_y, (T *)p->big_cb, (T *)p->big_cby);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL((big_adj_rows_kernel<T>), dim3(g.n2 / 2), dim3(stock_threads(g.n1)), 4 * (size_t)g.n1 * el,
                         p->stream, (const T *)p->big_cb, (const T *)p->big_cby, g, (const T *)p->d_tw1,
                         (V4 *)p->big_gu);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      BigTileArgs<T> a = tile_args<T>(p, c, x, y, h, w, m);
      a.G4 = (const V4 *)p->big_gu;
      a.gout = (V4 *)p->big_gout;
      a.gh = gh ? gh + a0 : nullptr;
      a.gx = gx ? gx + a0 : nullptr;
      a.gy = gy ? gy + a0 : nullptr;
      a.work_counter = p->big_work + 2;
      a.done_counter = p->big_work + 3;
      e = by_width<T, GatherW>(p->W, a, tile_blocks(p, n), p->stream);
    }
    if (e == hipSuccess) {
      const int blocks = (int)std::min<int64_t>(8192, (n + 255) / 256);
      hipLaunchKernelGGL((big_unpermute_kernel<T>), dim3(blocks), dim3(256), 0, p->stream, (const V4 *)p->big_gout,
                         (const int *)p->big_inv, (const int *)m.flags, n, gh ? gh + a0 : nullptr, gx ? gx + a0 : nullptr,
                         gy ? gy + a0 : nullptr);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return big_fail(p, e, "large-cell adjoint");
  }
  return ENUFFT_OK;
}

}  // namespace

// Workspace of a large-cell plan, sized for the largest cell: the sort's chunk
// histograms, tile and unit offsets, the inverse permutation and the points in
// tile order; the unit sub-grids and the FP64 spreading grid; the column
// buffers and the interleaved adjoint grids; the sorted-order gradients; the
// EMS sort buffer (when a unit table can exceed the per-cell kernel's 4096) and
// the work counters.
enufft_status big_prepare(enufft_plan_t p) {
  const Geom &g = p->geom;
  p->big_ntx = g.n1 / BIG_TS;
  p->big_nty = g.n2 / BIG_TS;
  const int ntiles = p->big_ntx * p->big_nty;
  int64_t qmax = 0;
  for (int64_t c = 0; c < p->n_cells; ++c) qmax = std::max(qmax, p->offsets[c + 1] - p->offsets[c]);
  if (qmax > (int64_t)INT32_MAX) {
    p->last_error = "enufft_plan: a large cell holds more than 2^31 - 1 points";
    return ENUFFT_EUNSUPPORTED;
  }
  const size_t el = p->elem;
  const int64_t M = (int64_t)g.N1 * g.N2;
  int64_t jpad = 64;
  while (jpad < M) jpad <<= 1;
  p->big_sort_jpad = jpad > BIG_SORT_BLOCK ? jpad : 0;
  p->big_ems_parts = std::max<int64_t>(2 * ((jpad + 255) / 256), (M + 255) / 256);
  const size_t n12 = (size_t)g.n1 * g.n2;
  const size_t cols = (size_t)(g.K1 + 1) * g.n2 * 2 * el;
  // sort buffer, partial sums, cut record (256 bytes reserved), tie flags
  const size_t ems_bytes =
      p->big_sort_jpad ? (size_t)p->big_sort_jpad * 8 + (size_t)p->big_ems_parts * 8 + 256 + (size_t)p->big_sort_jpad
                       : 0;
  struct A {
    void **ptr;
    size_t bytes;
    const char *what;
  };
  const int64_t q1 = std::max<int64_t>(qmax, 1);
  const int64_t nchunks = (q1 + BIG_SORT_CHUNK - 1) / BIG_SORT_CHUNK;
  const int64_t ngroups = (nchunks + BIG_SCAN_GROUP - 1) / BIG_SCAN_GROUP;
  // a tile's range touches at most (its length / chunk) + 2 unit chunks
  p->big_units_max = (q1 + BIG_UNIT_CHUNK - 1) / BIG_UNIT_CHUNK + 2 * (int64_t)ntiles;
  const int64_t S = BIG_TS + p->W + 1;
  const A list[] = {
      {(void **)&p->big_chunk_hist, (size_t)(nchunks * ntiles) * sizeof(int), "chunk tile histograms"},
      {(void **)&p->big_group_sum, (size_t)(ngroups * ntiles) * sizeof(int), "chunk group sums"},
      {(void **)&p->big_offsets, (size_t)(ntiles + 1) * sizeof(int64_t), "tile offsets"},
      {(void **)&p->big_unit_base, (size_t)(ntiles + 1) * sizeof(int), "tile unit offsets"},
      {(void **)&p->big_inv, (size_t)q1 * sizeof(int), "inverse permutation"},
      {(void **)&p->big_chunk_fl, (size_t)(nchunks * 4) * sizeof(int), "chunk key bounds"},
      {(void **)&p->big_flags, 4 * sizeof(int), "input order flag"},
      {(void **)&p->big_partial, (size_t)(p->big_units_max * S * S) * sizeof(double), "unit sub-grids"},
      {&p->big_gout, (size_t)q1 * 4 * el, "sorted-order gradients"},
      {&p->big_xs, (size_t)q1 * el, "sorted x"},
      {&p->big_ys, (size_t)q1 * el, "sorted y"},
      {&p->big_hs, (size_t)q1 * el, "sorted h"},
      {&p->big_ws, (size_t)q1 * el, "sorted w"},
      {(void **)&p->big_grid, n12 * sizeof(double), "fine grid"},
      {&p->big_cb, cols, "column buffer"},
      {&p->big_cby, cols, "column buffer (y)"},
      {&p->big_gu, 4 * n12 * el, "adjoint grids (u, du/dx, du/dy) interleaved"},
      {(void **)&p->big_work, 4 * sizeof(int), "work counters"},
      {(void **)&p->big_sort, ems_bytes, "EMS sort buffer"},
  };
  for (const A &it : list) {
    if (it.bytes == 0) continue;
    hipError_t e = hipMalloc(it.ptr, it.bytes);
    if (e != hipSuccess) {
      *it.ptr = nullptr;
      p->last_error = std::string("hipMalloc failed for ") + it.what + ": " + hipGetErrorString(e);
      return ENUFFT_ENOMEM;
    }
    p->allocations.push_back(*it.ptr);
    p->workspace_bytes += (int64_t)it.bytes;
  }
  hipError_t e = hipMemset(p->big_work, 0, 4 * sizeof(int));
  if (e == hipSuccess)
    e = p->prec == ENUFFT_F64 ? set_attrs_t<double>(g.n1, g.n2, ntiles) : set_attrs_t<float>(g.n1, g.n2, ntiles);
  if (e == hipSuccess) e = p->prec == ENUFFT_F64 ? gather_attrs<double>() : gather_attrs<float>();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  return big_fail(p, e, "large-cell workspace");
}

namespace {
template <typename T>
enufft_status sort_points_t(enufft_plan_t p, const T *x, const T *y, const T *h, const T *w, T *xs, T *ys, T *hs,
                            T *ws, int32_t *perm) {
  static_assert(BIG_TS2 == BIG_CS_THREADS, "the cell scan runs one thread per cell of a tile");
  static_assert(BIG_CS_PER * BIG_CS_THREADS == BIG_UNIT_CHUNK, "a unit is at most one pass of the workgroup");
  // the units' cell histograms and starts borrow the spreading sub-grids
  int *uh = reinterpret_cast<int *>(p->big_partial);
  if ((size_t)(BIG_TS + p->W + 1) * (BIG_TS + p->W + 1) * sizeof(double) < BIG_TS2 * sizeof(int)) {
    p->last_error = "enufft_sort_points: unit histograms do not fit the sub-grid buffer";
    return ENUFFT_EUNSUPPORTED;
  }
  const unsigned ublocks = (unsigned)std::max<int64_t>(1, p->big_units_max);
  // the cell order inside tiles only where the run kernel spreads it: spread
  // point by point, samples that share a fine cell would add to one address from
  // every lane of a wave (FP64 C4 type-1 took 71 ms in cell order, 13 in tile order)
  const bool by_cell = sizeof(T) == 4 && p->es.on && (p->W == 4 || p->W == 6 || p->W == 8);
  for (int64_t c = 0; c < p->n_cells; ++c) {
    const int64_t a0 = p->offsets[c], n = p->offsets[c + 1] - a0;
    if (n == 0) continue;
    // by tile, always scattering (sorted input or not): straight into the
    // caller's arrays, or into the plan's buffers and then by fine cell inside
    // each tile into the caller's arrays
    BigSortArgs<T> a = sort_args<T>(p, c, x, y, h, w ? w : x);
    a.presorted = nullptr;
    if (!by_cell) {
      a.xs = xs + a0; a.ys = ys + a0;
      a.hs = hs ? hs + a0 : (T *)p->big_hs;
      a.ws = ws ? ws + a0 : (T *)p->big_ws;
    }
    hipError_t e = sort_launch<T>(p, a);
    if (!by_cell) {
      if (e == hipSuccess && perm) {
        hipLaunchKernelGGL(big_perm_kernel, dim3((unsigned)std::min<int64_t>(8192, (n + 255) / 256)), dim3(256), 0,
                           p->stream, (const int *)p->big_inv, n, (int32_t)a0, perm + a0);
        e = hipGetLastError();
      }
      if (e != hipSuccess) return big_fail(p, e, "large-cell point sort");
      continue;
    }
    int32_t *ptile = perm ? (int32_t *)p->big_gout : nullptr;   // input index of each tile-order position
    if (e == hipSuccess && perm) {
      hipLaunchKernelGGL(big_perm_kernel, dim3((unsigned)std::min<int64_t>(8192, (n + 255) / 256)), dim3(256), 0,
                         p->stream, (const int *)p->big_inv, n, (int32_t)a0, ptile);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL((big_cell_count_kernel<T>), dim3(ublocks), dim3(BIG_CS_THREADS), 0, p->stream, a,
                         (const T *)a.xs, (const T *)a.ys, uh);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL(big_cell_scan_kernel, dim3((unsigned)a.ntiles), dim3(BIG_CS_THREADS), 0, p->stream,
                         (const int64_t *)a.offsets, (const int *)a.unit_base, uh);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL((big_cell_scatter_kernel<T>), dim3(ublocks), dim3(BIG_CS_THREADS), 0, p->stream, a,
                         (const T *)a.xs, (const T *)a.ys, (const T *)a.hs, (const T *)a.ws, (const int32_t *)ptile,
                         (const int *)uh, xs + a0, ys + a0, hs ? hs + a0 : nullptr, ws ? ws + a0 : nullptr,
                         perm ? perm + a0 : nullptr);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return big_fail(p, e, "large-cell point sort");
  }
  return ENUFFT_OK;
}
}  // namespace

enufft_status big_sort_points(enufft_plan_t p, const void *x, const void *y, const void *h, const void *w, void *xs,
                              void *ys, void *hs, void *ws, int32_t *perm) {
  if (p->prec == ENUFFT_F64)
    return sort_points_t<double>(p, (const double *)x, (const double *)y, (const double *)h, (const double *)w,
                                 (double *)xs, (double *)ys, (double *)hs, (double *)ws, perm);
  return sort_points_t<float>(p, (const float *)x, (const float *)y, (const float *)h, (const float *)w, (float *)xs,
                              (float *)ys, (float *)hs, (float *)ws, perm);
}

namespace {
// The counting pass, group sums and tile scan of cell c (no scatter): tile
// ranges, unit offsets and order flags into m.
template <typename T>
hipError_t bind_cell(enufft_plan_t p, int64_t c, const T *x, const T *y, const CellMeta &m) {
  BigSortArgs<T> a = sort_args<T>(p, c, x, y, nullptr, x);
  a.offsets = m.offsets;
  a.unit_base = m.unit_base;
  a.presorted = m.flags;
  const dim3 tg((a.ntiles + 255) / 256, a.ngroups);
  hipLaunchKernelGGL((big_count_kernel<T>), dim3(a.nchunks), dim3(BIG_SORT_THREADS), count_lds(a.ntiles),
                     p->stream, a);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(big_group_sum_kernel, tg, dim3(256), 0, p->stream, (const int *)a.chunk_hist, a.nchunks,
                       a.ntiles, a.group_sum);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(big_tile_scan_kernel, dim3(1), dim3(1024), (size_t)a.ntiles * sizeof(int), p->stream,
                       a.group_sum, a.ngroups, a.ntiles, a.offsets, a.unit_base, (const int *)a.chunk_fl, a.nchunks,
                       a.presorted);
    e = hipGetLastError();
  }
  return e;
}
}  // namespace

enufft_status big_bind_points(enufft_plan_t p, const void *x, const void *y) {
  p->bound_x = p->bound_y = nullptr;   // unbound while (re)binding, and for good if it fails
  p->graph_key.clear();                // a captured forward graph holds the sort as it was: capture again
  if (!x) return ENUFFT_OK;
  const int64_t nt1 = (int64_t)p->big_ntx * p->big_nty + 1;
  if (p->bound_cap < p->n_cells) {
    const size_t bytes[3] = {(size_t)(p->n_cells * nt1) * sizeof(int64_t), (size_t)(p->n_cells * nt1) * sizeof(int),
                             (size_t)(p->n_cells * 4) * sizeof(int)};
    void **ptrs[3] = {(void **)&p->bound_offsets, (void **)&p->bound_unit_base, (void **)&p->bound_flags};
    for (int i = 0; i < 3; ++i) {
      void *q = nullptr;
      const hipError_t e = hipMalloc(&q, bytes[i]);
      if (e != hipSuccess) {
        p->last_error = std::string("enufft_bind_points: hipMalloc: ") + hipGetErrorString(e);
        return ENUFFT_ENOMEM;
      }
      p->allocations.push_back(q);   // freed with the plan (a smaller earlier set stays until then)
      p->workspace_bytes += (int64_t)bytes[i];
      *ptrs[i] = q;
    }
    p->bound_cap = p->n_cells;
  }
  std::vector<int> flags((size_t)p->n_cells * 4, 1);
  hipError_t e = hipSuccess;
  for (int64_t c = 0; c < p->n_cells && e == hipSuccess; ++c) {
    if (p->offsets[c + 1] == p->offsets[c]) {   // empty: no spreading, nothing to bind
      e = hipMemcpyAsync(p->bound_flags + 4 * c, flags.data(), 4 * sizeof(int), hipMemcpyHostToDevice, p->stream);
      continue;
    }
    const CellMeta m{p->bound_offsets + c * nt1, p->bound_unit_base + c * nt1, p->bound_flags + 4 * c, true};
    e = p->prec == ENUFFT_F64 ? bind_cell<double>(p, c, (const double *)x, (const double *)y, m)
                              : bind_cell<float>(p, c, (const float *)x, (const float *)y, m);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(flags.data(), p->bound_flags, flags.size() * sizeof(int), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return big_fail(p, e, "enufft_bind_points");
  for (int64_t c = 0; c < p->n_cells; ++c)
    if (!flags[(size_t)4 * c]) {
      p->last_error = "enufft_bind_points: the samples of cell " + std::to_string(c) +
                      " are not in tile order (sort them once with enufft_sort_points)";
      return ENUFFT_EINVAL;
    }
  p->bound_x = x;
  p->bound_y = y;
  return ENUFFT_OK;
}

enufft_status big_type1(enufft_plan_t p, const void *x, const void *y, const void *h, const void *w, void *f,
                        int64_t c0, int64_t c1) {
  if (p->prec == ENUFFT_F64)
    return type1_t<double>(p, (const double *)x, (const double *)y, (const double *)h, (const double *)w,
                           (double *)f, c0, c1);
  return type1_t<float>(p, (const float *)x, (const float *)y, (const float *)h, (const float *)w, (float *)f, c0,
                        c1);
}

enufft_status big_adjoint(enufft_plan_t p, const void *x, const void *y, const void *h, const void *w,
                          const void *fin, const uint8_t *keep, const double *lam, void *gh, void *gx, void *gy) {
  if (p->prec == ENUFFT_F64)
    return adjoint_t<double>(p, (const double *)x, (const double *)y, (const double *)h, (const double *)w,
                             (const double *)fin, keep, lam, (double *)gh, (double *)gx, (double *)gy);
  return adjoint_t<float>(p, (const float *)x, (const float *)y, (const float *)h, (const float *)w,
                          (const float *)fin, keep, lam, (float *)gh, (float *)gx, (float *)gy);
}

// EMS of cells [cell_begin, cell_begin + cell_count) when the unit table is
// larger than the per-cell kernel's register sort: energies, device sort,
// scores, ties, keep, finish; one cell after the other.
enufft_status big_ems(enufft_plan_t p, const void *f, const enufft_ems_params *prm, const double *mode_weight,
                      uint8_t *keep, int32_t *k_star, double *stats, const UnitTable *ut, int64_t cell_begin,
                      int64_t cell_count) {
  const int J = ut->J, M = p->N1 * p->N2;
  const int64_t Jpad = ut->Jpad;
  if (!p->big_sort || Jpad > p->big_sort_jpad || Jpad < 2 * BIG_SORT_BLOCK) {
    p->last_error = "EMS: unit table size not supported by the large-cell sort";
    return ENUFFT_EUNSUPPORTED;
  }
  const int nb = (int)((Jpad + 255) / 256), mb = (M + 255) / 256;
  double *S = p->big_sort;
  double *partial = S + p->big_sort_jpad;
  BigCut *cut = reinterpret_cast<BigCut *>(partial + p->big_ems_parts);
  uint8_t *tie = reinterpret_cast<uint8_t *>(cut) + 256;
  static_assert(sizeof(BigCut) <= 256, "cut record must fit its reserved bytes");
  const size_t el = p->elem;
  const int nblk = (int)(Jpad / BIG_SORT_BLOCK);
  hipError_t e = hipSuccess;
  for (int64_t c = cell_begin; c < cell_begin + cell_count && e == hipSuccess; ++c) {
    const void *fc = (const char *)f + (size_t)c * M * 2 * el;
    if (p->prec == ENUFFT_F64)
      hipLaunchKernelGGL((big_ems_energy_kernel<double>), dim3(nb), dim3(256), 0, p->stream, (const double *)fc,
                         mode_weight, ut->d_units, J, (int)Jpad, S, partial);
    else
      hipLaunchKernelGGL((big_ems_energy_kernel<float>), dim3(nb), dim3(256), 0, p->stream, (const float *)fc,
                         mode_weight, ut->d_units, J, (int)Jpad, S, partial);
    e = hipGetLastError();
    if (e == hipSuccess) {
      hipLaunchKernelGGL(big_sort_block_kernel, dim3(nblk), dim3(512), 0, p->stream, S, 2, BIG_SORT_BLOCK,
                         BIG_SORT_BLOCK / 2);
      e = hipGetLastError();
    }
    for (int64_t k = 2 * BIG_SORT_BLOCK; k <= Jpad && e == hipSuccess; k <<= 1) {
      for (int64_t j = k >> 1; j >= BIG_SORT_BLOCK && e == hipSuccess; j >>= 1) {
        hipLaunchKernelGGL(big_sort_global_kernel, dim3((int)std::min<int64_t>(4096, Jpad / 256)), dim3(256), 0,
                           p->stream, S, Jpad, k, j);
        e = hipGetLastError();
      }
      if (e == hipSuccess) {
        hipLaunchKernelGGL(big_sort_block_kernel, dim3(nblk), dim3(512), 0, p->stream, S, (int)k, (int)k,
                           BIG_SORT_BLOCK / 2);
        e = hipGetLastError();
      }
    }
    // the parts of eq. (s_delta) go where the tie flags go later (Jpad >= 8,192 bytes there)
    double *tpart = reinterpret_cast<double *>(tie);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(big_ems_terms_kernel, dim3(BIG_TERM_BLOCKS), dim3(256), 0, p->stream, (const double *)S, J,
                         *prm, tpart);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL(big_ems_scores_kernel, dim3(1), dim3(1024), 0, p->stream, (const double *)S,
                         (const double *)partial, nb, (const double *)tpart, J, *prm, cut);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      if (p->prec == ENUFFT_F64)
        hipLaunchKernelGGL((big_ems_ties_kernel<double>), dim3(1), dim3(1024), 0, p->stream, (const double *)fc,
                           mode_weight, ut->d_units, J, (const BigCut *)cut, tie);
      else
        hipLaunchKernelGGL((big_ems_ties_kernel<float>), dim3(1), dim3(1024), 0, p->stream, (const float *)fc,
                           mode_weight, ut->d_units, J, (const BigCut *)cut, tie);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      if (p->prec == ENUFFT_F64)
        hipLaunchKernelGGL((big_ems_keep_kernel<double>), dim3(mb), dim3(256), 0, p->stream, (const double *)fc,
                           mode_weight, ut->d_mode_unit, M, (const BigCut *)cut, (const uint8_t *)tie, keep + c * M,
                           partial);
      else
        hipLaunchKernelGGL((big_ems_keep_kernel<float>), dim3(mb), dim3(256), 0, p->stream, (const float *)fc,
                           mode_weight, ut->d_mode_unit, M, (const BigCut *)cut, (const uint8_t *)tie, keep + c * M,
                           partial);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL(big_ems_finish_kernel, dim3(1), dim3(256), 0, p->stream, (const BigCut *)cut,
                         (const double *)partial, mb, k_star + c, stats + c * 8);
      e = hipGetLastError();
    }
  }
  return big_fail(p, e, "large-cell EMS");
}

}  // namespace enufft
