// Adjoint of the batched type-1 map on gfx950: a type-2 NUFFT (the +i sign of
// the series, eq. series) followed by the chain rule through the per-point
// strength c_j = w_j W(x_j) h_j.
//
// For a cotangent g on the coefficients, u_j = scale Re sum_k g_k exp(+i k.x_j)
// and its coordinate derivatives come from three fine grids: the pre-corrected
// spectrum (g_k divided by the kernel factors p(kx) p(ky), the inverse of
// Step 4) made Hermitian, and the same times i kx and i ky, each brought to the
// grid by an inverse FFT; the points then gather W x W taps from each grid with
// the same spreading kernel.  The three grids of a whole cell do not fit in
// LDS, so each work item rebuilds one row band (plus the kernel's halo) and
// serves the points whose footprint starts in that band.  Nothing of the
// forward pass is stored.
#include <algorithm>
#include <string>

#include "device_common.h"
#include "launch.h"
#include "plan.h"

namespace enufft {

struct AdjLayout {
  int rows;       // band rows including halo = band_rows + W
  int apitch;     // grid row pitch (elements) = n1 + W - 1, rounded up to even: the first W - 1
                  // columns are repeated after the last, so a footprint's W columns are contiguous
  int cpitch;     // column-workspace pitch (elements) = 2 (K1 + 1) + 2
  size_t g_off, gx_off, gy_off, db0_off, db1_off, ws_off;   // element offsets
  size_t st_off;  // staged cell spectrum, deconvolution factors and keep bytes
  size_t tw_off;  // twiddles of the row (n1) and column (n2) transforms, interleaved complex
  size_t total;   // elements
};

// Elements of the staging area: the cell's N1 N2 complex coefficients, the
// K1 + 1 and K2 + 1 deconvolution factors, then N1 N2 keep bytes.
__host__ __device__ inline size_t adj_stage_elems(const Geom &g, size_t elem) {
  const size_t M = (size_t)g.N1 * g.N2;
  return 2 * M + (g.K1 + 1) + (g.K2 + 1) + (M + elem - 1) / elem;
}

__host__ __device__ inline AdjLayout adj_layout(const Geom &g, int W, int band_rows, size_t elem) {
  AdjLayout L;
  L.rows = band_rows + W;   // R + W - 1 rows are used; one more keeps the uy rows paired
  L.apitch = (g.n1 + W - 1 + 1) & ~1;
  L.cpitch = 2 * (g.K1 + 1) + 2;
  const size_t gsz = (size_t)L.rows * L.apitch;
  L.g_off = 0;
  L.gx_off = gsz;
  L.gy_off = 2 * gsz;
  // the column workspace and the staging area behind it alias the grids (they
  // are dead before the grids are written) but never the band spectra, which
  // are filled while they are live
  const size_t ws = (size_t)g.n2 * L.cpitch;
  L.ws_off = 0;
  L.st_off = ws;
  L.db0_off = std::max(3 * gsz, ws + adj_stage_elems(g, elem));
  L.db1_off = L.db0_off + (size_t)L.rows * (g.K1 + 1) * 2;
  L.tw_off = L.db1_off + (size_t)L.rows * (g.K1 + 1) * 2;
  L.total = L.tw_off + 2 * (size_t)(g.n1 + g.n2);
  return L;
}

// Copy the cell's cotangent spectrum, its keep bytes and the deconvolution
// factors into the staging area.  Every thread issues all of its global loads
// before it stores any (the loads are unconditional, clamped to the last
// element), so the copy costs about one memory latency instead of one per
// element.
template <typename T, int NT>
__device__ void stage_spectrum(const AdjArgs<T> &a, const T *gc, int cell, T *st) {
  const Geom &g = a.g;
  const int M = g.N1 * g.N2, n = 2 * M;
  constexpr int U = 16;
  for (int base = 0; base < n; base += U * NT) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = gc[min(base + u * NT + (int)threadIdx.x, n - 1)];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * NT + threadIdx.x;
      if (i < n) st[i] = v[u];
    }
  }
  T *sdx = st + n, *sdy = sdx + g.K1 + 1;
  for (int i = threadIdx.x; i <= g.K1; i += NT) sdx[i] = a.decon_x[i];
  for (int i = threadIdx.x; i <= g.K2; i += NT) sdy[i] = a.decon_y[i];
  if (a.keep) {
    const uint8_t *kp = a.keep + (int64_t)cell * M;
    uint8_t *sk = reinterpret_cast<uint8_t *>(sdy + g.K2 + 1);
    for (int base = 0; base < M; base += U * NT) {
      uint8_t v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = kp[min(base + u * NT + (int)threadIdx.x, M - 1)];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = base + u * NT + threadIdx.x;
        if (i < M) sk[i] = v[u];
      }
    }
  }
  __syncthreads();
}

// First-step accessor of the column transforms: load(i) forms bin i (fine
// row, natural order) of column kx of the Hermitian, pre-corrected spectrum
// from the staged copy: (G(kx, ky) + conj G(-kx, -ky)) / 2 divided by the
// kernel transform, each term zero outside the mode box, with the
// retained-power factor two_lam on kept modes (1 without a keep mask); with
// yderiv, times i ky.  store() writes the column workspace.
template <typename T>
struct ColSpecAcc {
  const T *sf, *sdx, *sdy;
  const uint8_t *kp;
  T two_lam;
  T *col;   // column kx of the workspace (interleaved complex, row pitch cpitch)
  int cpitch, kx, n2, K2, N1, lo1, lo2, hi1, hi2;
  bool yderiv;
  __device__ void load(int bin, T &re, T &im) const {
    const int ky = bin <= n2 / 2 ? bin : bin - n2;   // signed frequency of this bin
    T hr = 0, hi = 0;
    if (ky >= -K2 && ky <= K2) {
      const T s = sdx[kx] * sdy[ky < 0 ? -ky : ky];
      if (kx <= hi1 && ky >= lo2 && ky <= hi2) {
        const int m = (ky - lo2) * N1 + (kx - lo1);
        const T sc = kp ? (kp[m] ? two_lam : T(0)) : T(1);
        hr += sc * sf[2 * m];
        hi += sc * sf[2 * m + 1];
      }
      if (-kx >= lo1 && -ky >= lo2 && -ky <= hi2) {
        const int m = (-ky - lo2) * N1 + (-kx - lo1);
        const T sc = kp ? (kp[m] ? two_lam : T(0)) : T(1);
        hr += sc * sf[2 * m];
        hi -= sc * sf[2 * m + 1];
      }
      hr *= T(0.5) * s;
      hi *= T(0.5) * s;
      if (yderiv) {
        const T t = hr;
        hr = -T(ky) * hi;
        hi = T(ky) * t;
      }
    }
    re = hr;
    im = hi;
  }
  __device__ void store(int i, T re, T im) const {
    col[i * cpitch] = re;
    col[i * cpitch + 1] = im;
  }
};

// Second step of the column transforms, out of place: item k1 of column kx
// computes fine rows y = k1 + A k2 and writes those of the band (band row r
// holds fine row (y0 + r) mod n2, r < rows) to the band spectra db
// ([row][kx] complex).
template <int A, int B, typename T>
__device__ __forceinline__ void col_step2_band(const T *col, int cpitch, int k1, int n2, T *db, int per, int kx,
                                               int rows, int y0) {
  T re[B], im[B];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    re[b] = col[(k1 * B + b) * cpitch];
    im[b] = col[(k1 * B + b) * cpitch + 1];
  }
  dft_reg<B, true, T>(re, im);
#pragma unroll
  for (int k2 = 0; k2 < B; ++k2) {
    // band row r, and r + n2 too when the band's halo wraps onto its own
    // first rows (one band per cell: rows = n2 + W)
    const int r = (k1 + A * k2 - y0) & (n2 - 1);
    if (r < rows) {
      db[2 * (r * per + kx)] = re[k2];
      db[2 * (r * per + kx) + 1] = im[k2];
    }
    if (r + n2 < rows) {
      db[2 * ((r + n2) * per + kx)] = re[k2];
      db[2 * ((r + n2) * per + kx) + 1] = im[k2];
    }
  }
}

// One column pass: the inverse transforms along y of columns kx = 0..K1 of the
// spectrum (times i ky with yderiv), formed from the staged copy in the first
// step and written to the band spectra db by the second.
template <typename T, int NT>
__device__ void column_pass(const AdjArgs<T> &a, const T *st, const T *tw2, T two_lam, T *ws, int cpitch,
                            bool yderiv, T *db, int rows, int y0) {
  const Geom &g = a.g;
  const int per = g.K1 + 1, n2 = g.n2, M = g.N1 * g.N2;
  const int A = fft_A(n2), B = fft_B(n2);
  ColSpecAcc<T> acc;
  acc.sf = st;
  acc.sdx = st + 2 * M;
  acc.sdy = acc.sdx + per;
  acc.kp = a.keep ? reinterpret_cast<const uint8_t *>(acc.sdy + g.K2 + 1) : nullptr;
  acc.two_lam = two_lam;
  acc.cpitch = cpitch;
  acc.n2 = n2; acc.K2 = g.K2; acc.N1 = g.N1; acc.lo1 = g.lo1; acc.lo2 = g.lo2;
  acc.hi1 = g.lo1 + g.N1 - 1; acc.hi2 = g.lo2 + g.N2 - 1;
  acc.yderiv = yderiv;
  // Consecutive lanes take consecutive columns (the column is the fast index of
  // both steps), so their LDS words are adjacent: the staged coefficients of
  // consecutive kx, the workspace elements 2 kx apart, the band spectra of
  // consecutive kx.  (With the transform position as the fast index, lanes
  // were a row of the staged box, or 8 or 16 workspace rows, apart: 8- and
  // 16-way bank conflicts.)
  for (int it = threadIdx.x; it < per * B; it += NT) {
    const int b = it / per, q = it - b * per;
    ColSpecAcc<T> c = acc;
    c.kx = q;
    c.col = ws + 2 * q;
    fft4_dispatch<true, 1, T>(n2, c, b, tw2);
  }
  __syncthreads();
  for (int it = threadIdx.x; it < per * A; it += NT) {
    const int k1 = it / per, q = it - k1 * per;
    const T *col = ws + 2 * q;
    switch (n2) {
      case 16: col_step2_band<4, 4, T>(col, cpitch, k1, n2, db, per, q, rows, y0); break;
      case 32: col_step2_band<8, 4, T>(col, cpitch, k1, n2, db, per, q, rows, y0); break;
      case 64: col_step2_band<8, 8, T>(col, cpitch, k1, n2, db, per, q, rows, y0); break;
      default: col_step2_band<16, 8, T>(col, cpitch, k1, n2, db, per, q, rows, y0); break;
    }
  }
  __syncthreads();
}

// Second step of the row transforms, writing natural column order.  Item k1
// of a row computes bins k1 + A k2 (k2 = 0 .. B - 1) from positions k1 B + b
// and stores bin k at column k, and again at n1 + k for k < W - 1 (the first
// W - 1 columns repeated after the last, so a footprint's W taps in a row are
// W consecutive elements).  The store lands on positions other items of the
// same row still read, so the A items of a row must be one wave's lanes: a
// wave's LDS accesses complete in issue order and every item loads before it
// stores.  With A | 64 and 64 | NT, the items q A .. q A + A - 1 of the
// batched loop below always share a wave.  The first step stores with
// fft4_step1_swz (the inputs of item k1 sit at k1 B + (b ^ fft_swz(k1, B))).
template <int A, int B, typename T, typename Acc>
__device__ __forceinline__ void row_step2_natural(const Acc &acc, int k1, int n, int wrap) {
  T re[B], im[B];
  const int sw = fft_swz(k1, B);
#pragma unroll
  for (int b = 0; b < B; ++b) acc.load(k1 * B + (b ^ sw), re[b], im[b]);
  dft_reg<B, true, T>(re, im);
#pragma unroll
  for (int k2 = 0; k2 < B; ++k2) {
    const int k = k1 + A * k2;
    acc.store(k, re[k2], im[k2]);
    if (k < wrap) acc.store(n + k, re[k2], im[k2]);
  }
}

// The batched inverse row transforms: step 1 through make1(q) (forming the
// spectra), step 2 in place through make2(q) into natural column order.
template <int NT, typename T, typename Make1, typename Make2>
__device__ __forceinline__ void row_ifft_natural(int n, int count, const T *tw, int wrap, const Make1 &make1,
                                                 const Make2 &make2) {
  static_assert(NT % 64 == 0, "whole waves");
  const int A = fft_A(n), B = fft_B(n), la = fft_logA(n), lb = fft_logB(n);
  for (int it = threadIdx.x; it < count * B; it += NT) {
    const int q = it >> lb, b = it & (B - 1);
    fft4_step1_swz_dispatch<true, T>(n, make1(q), b, tw);
  }
  __syncthreads();
  for (int it = threadIdx.x; it < count * A; it += NT) {
    const int q = it >> la, k1 = it & (A - 1);
    switch (n) {
      case 16: row_step2_natural<4, 4, T>(make2(q), k1, n, wrap); break;
      case 32: row_step2_natural<8, 4, T>(make2(q), k1, n, wrap); break;
      case 64: row_step2_natural<8, 8, T>(make2(q), k1, n, wrap); break;
      default: row_step2_natural<16, 8, T>(make2(q), k1, n, wrap); break;
    }
  }
  __syncthreads();
}

// First-step accessor of the row transforms: load(k) forms bin k of the row's
// spectrum from the band's column data db ([row][kx] complex, kx = 0..K1):
// for a (u, du/dx) row, (1 - k) D(k); for a du/dy pair (rows row, row + 1),
// D_row(k) + i D_row+1(k); D(-k) = conj D(k), zero beyond K1.  store() writes
// the grid row like StridedPairAcc.
template <typename T>
struct RowSpecAcc {
  const T *db;
  T *r0, *r1;
  int stride, row, per, n1, K1;
  bool pair;
  __device__ void load(int k, T &re, T &im) const {
    const int kk = k <= n1 / 2 ? k : n1 - k;
    re = T(0);
    im = T(0);
    if (kk > K1) return;
    const bool neg = k != kk;
    const T *d = db + 2 * (row * per + kk);
    T dr = d[0], di = d[1];
    if (neg) di = -di;
    if (!pair) {
      const T kf = neg ? -T(kk) : T(kk);
      re = dr - kf * dr;
      im = di - kf * di;
    } else {
      T br = d[2 * per], bi = d[2 * per + 1];
      if (neg) bi = -bi;
      re = dr - bi;
      im = di + br;
    }
  }
  __device__ void store(int i, T re, T im) const {
    r0[i * stride] = re;
    r1[i * stride] = im;
  }
};

// Gradients at one point from the band's three grids (W x W taps each), if the
// point's footprint starts in this band; the chain rule through the strength
// c_j = w_j W(x_j) h_j turns the interpolated u, du/dx, du/dy into dL/dh,
// dL/dx, dL/dy.
//
// RECON: the reconstruction mode.  Only u is interpolated (from the u half of
// Guv); it is the truncated series h_rec(x_j) (the plan's scale is not applied in
// this mode), stored to grad_h when given, and the point adds (t - h_rec)^2, t^2
// and w t^2 to acc, with t = W(x_j) h_j the windowed height.
template <typename T, int W, bool POLY, bool RECON>
__device__ __forceinline__ void gather_point(const AdjArgs<T> &a, const T *Guv, const T *Gy, int apitch,
                                             int band_lo, int64_t j, T xj, T yj, T hj, T wj, T cx, T cy, T R,
                                             T pr, double (&acc)[3]) {
  const Geom &g = a.g;
  const T halfw = T(W) / T(2);
  const FineCoord<T> fy = fine_coord<T>(yj, a.s2_hi, a.s2_lo, halfw);
  const int r0 = (fy.i0 & (g.n2 - 1)) - band_lo;    // first footprint row, band-local
  if (r0 < 0 || r0 >= a.band_rows) return;
  const FineCoord<T> fx = fine_coord<T>(xj, a.s1_hi, a.s1_lo, halfw);
  T kx[W];
  T u = 0, ux = 0, uy = 0;
  // rows in natural column order with the wrap-around columns repeated: the
  // W taps of a row are W consecutive elements from one base address
  using V2 = typename vec2<T>::type;
  const int e0 = r0 * apitch + (fx.i0 & (g.n1 - 1));
  const V2 *puv = reinterpret_cast<const V2 *>(Guv) + e0;
  const T *py = Gy + e0;
  auto row = [&](T kyv) {
    T su = 0, sx = 0, sy = 0;
#pragma unroll
    for (int dx = 0; dx < W; ++dx) {
      const V2 v = puv[dx];
      su += kx[dx] * v.x;
      if constexpr (!RECON) {
        sx += kx[dx] * v.y;
        sy += kx[dx] * py[dx];
      }
    }
    u += kyv * su;
    if constexpr (!RECON) {
      ux += kyv * sx;
      uy += kyv * sy;
    }
    puv += apitch;
    py += apitch;
  };
  // kernel values: the plan's per-tap polynomials (FP32, W <= ES_MAXW) or psi
  // itself, chosen at compile time (a run-time choice makes the compiler keep
  // the taps in scratch); the exact kernel goes one row at a time, so the
  // loads of all W rows are not hoisted into registers together
  if constexpr (POLY) {
    T ky[W];
    es_taps_poly<W>(fx, float(W) * 0.5f, a.es, kx);
    es_taps_poly<W>(fy, float(W) * 0.5f, a.es, ky);
#pragma unroll
    for (int dy = 0; dy < W; ++dy) row(ky[dy]);
  } else {
    const T zsc = T(2) / T(W);
#pragma unroll
    for (int d = 0; d < W; ++d) kx[d] = ker_eval(fx.offset(d) * zsc, a.beta);
#pragma unroll 1
    for (int dy = 0; dy < W; ++dy) row(ker_eval(fy.offset(dy) * zsc, a.beta));
  }
  if constexpr (RECON) {
    const double t = (double)(hj * hann_w(a.window_kind, xj, yj, cx, cy, R, pr));
    const double d = t - (double)u;
    acc[0] += d * d;
    acc[1] += t * t;
    acc[2] += (double)wj * t * t;
    if (a.grad_h) a.grad_h[j] = u;
    return;
  }
  T dWx, dWy;
  const T Wv = hann_wg(a.window_kind, xj, yj, cx, cy, R, pr, dWx, dWy);
  if (a.grad_h) a.grad_h[j] = wj * Wv * u;
  if (a.grad_x || a.grad_y) {
    const T wh = wj * hj;
    if (a.grad_x) a.grad_x[j] = wh * (dWx * u + Wv * ux);
    if (a.grad_y) a.grad_y[j] = wh * (dWy * u + Wv * uy);
  }
}

// All points of one item; every point is read (its band decides whether it is
// served).  Wave w takes blocks of 256 consecutive points and lane l gathers
// points l, l + 64, l + 128 and l + 192 of a block, so at every step the 64
// lanes work on 64 consecutive points: for points stored in raster order their
// footprints overlap, many lanes read the same LDS words (one broadcast) and
// the others fall on neighbouring banks.  (Runs of 4 consecutive points per
// lane put the lanes 4 points apart, and about half of the LDS time went to
// bank conflicts.)  The loads run two blocks ahead in three register buffers,
// so the gather is not serialised behind point loads; each wave load reads 256
// contiguous bytes of an array.  FP64 and the wider kernels (register budget)
// take one point per thread and step.
template <typename T, int W, int NT, bool POLY, bool RECON>
__device__ __forceinline__ void gather_item(const AdjArgs<T> &a, const T *Guv, const T *Gy, int apitch,
                                            int band_lo, int64_t begin, int64_t end, T cx, T cy, T R,
                                            double (&acc)[3]) {
  const T pr = R > T(0) ? T(M_PI) / R : T(0);
  constexpr bool kBlocks = sizeof(T) == 4 && W <= 6;
  if constexpr (kBlocks) {
    constexpr int U = 4, BLK = 64 * U, NWV = NT / 64;
    struct Pts {
      T x[U], y[U], h[U], w[U];
    };
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)NWV * BLK;
    auto load = [&](Pts &b, int64_t pb) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = pb + u * 64 + lane;
        const int64_t ic = i < end ? i : end - 1;   // past the end: re-read the last point (unused)
        b.x[u] = a.x[ic]; b.y[u] = a.y[ic]; b.h[u] = a.h[ic]; b.w[u] = a.w[ic];
      }
    };
    auto step = [&](const Pts &b, int64_t pb) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = pb + u * 64 + lane;
        if (i < end)
          gather_point<T, W, POLY, RECON>(a, Guv, Gy, apitch, band_lo, i, b.x[u], b.y[u], b.h[u], b.w[u], cx, cy,
                                          R, pr, acc);
      }
    };
    if (begin < end) {
      int64_t p = begin + (int64_t)(threadIdx.x >> 6) * BLK;
      Pts b0, b1, b2;
      load(b0, p);
      load(b1, p + stride);
      for (; p < end; p += 3 * stride) {
        load(b2, p + 2 * stride);
        step(b0, p);
        load(b0, p + 3 * stride);
        step(b1, p + stride);
        load(b1, p + 4 * stride);
        step(b2, p + 2 * stride);
      }
    }
  } else {
    for (int64_t j = begin + threadIdx.x; j < end; j += NT)
      gather_point<T, W, POLY, RECON>(a, Guv, Gy, apitch, band_lo, j, a.x[j], a.y[j], a.h[j], a.w[j], cx, cy, R,
                                      pr, acc);
  }
}

template <typename T, int W, int NT, bool POLY, bool RECON>
__global__ __launch_bounds__(NT) void adj_kernel(AdjArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *sm = reinterpret_cast<T *>(smem_raw);
  __shared__ int s_item;
  const Geom &g = a.g;
  const AdjLayout L = adj_layout(g, W, a.band_rows, sizeof(T));
  const int pitch = L.apitch;
  // Guv: rows of (u, du/dx) pairs (the real and imaginary parts of one complex
  // row transform, kept interleaved); Gy: rows of du/dy
  T *Guv = sm + L.g_off, *Gy = sm + L.gy_off;
  T *db0 = sm + L.db0_off, *db1 = sm + L.db1_off, *ws = sm + L.ws_off;
  const int per = g.K1 + 1;
  const bool persistent = a.work_counter != nullptr;
  int64_t idx = a.item_base + blockIdx.x;
  if (!persistent && idx >= a.n_items) return;
  // the transforms' twiddles stay in LDS for all items of this workgroup (the
  // barrier at the top of the item loop orders them before first use)
  T *tw1 = sm + L.tw_off, *tw2 = tw1 + 2 * g.n1;
  for (int i = threadIdx.x; i < 2 * g.n1; i += NT) tw1[i] = a.tw1[i];
  for (int i = threadIdx.x; i < 2 * g.n2; i += NT) tw2[i] = a.tw2[i];
  if (!persistent) __syncthreads();
  for (;;) {
    if (persistent) {
      if (threadIdx.x == 0) s_item = atomicAdd(a.work_counter, 1);
      __syncthreads();
      idx = s_item;
      __syncthreads();
      if (idx >= a.n_items) break;
    }
    const AdjItem it = a.items[idx];
    const T *gc = a.fbar + (int64_t)it.cell * g.N1 * g.N2 * 2;
    const int y0 = it.band * a.band_rows;   // fine row of band-local row 0

    // columns of H and of i ky H, inverse transformed along y; keep the band rows
    T *st = sm + L.st_off;
    const T two_lam = RECON ? T(1) : a.keep ? T(2.0 * (a.lam ? a.lam[it.cell] : 1.0)) : T(1);
    stage_spectrum<T, NT>(a, gc, it.cell, st);
    for (int pass = 0; pass < (RECON ? 1 : 2); ++pass)
      column_pass<T, NT>(a, st, tw2, two_lam, ws, L.cpitch, pass == 1, pass == 0 ? db0 : db1, L.rows, y0);

    // Row stage, one batch of inverse transforms: the (u, du/dx) rows, spectrum
    // Z(k) = D(k) + i (i k D(k)) = (1 - k) D(k), stored interleaved in Guv, and
    // the du/dy row pairs, Z(k) = Dy_r(k) + i Dy_r+1(k), in Gy; the bins k < 0
    // are the conjugates of column -k.  The first step of the transform reads
    // the spectra straight from the band's column data (no separate pass
    // writing them into the grids), the second writes natural column order with
    // the wrap-around columns; band rows = band_rows + W is even, so the du/dy
    // rows pair up exactly.
    const int n1 = g.n1;
    const int ny_pairs = L.rows / 2;
    const int K1 = g.K1;
    row_ifft_natural<NT, T>(
        n1, RECON ? L.rows : L.rows + ny_pairs, tw1, W - 1,
        [&](int q) {
          RowSpecAcc<T> acc;
          acc.db = q < L.rows ? db0 : db1;
          acc.row = q < L.rows ? q : 2 * (q - L.rows);
          acc.pair = q >= L.rows;
          acc.per = per;
          acc.n1 = n1;
          acc.K1 = K1;
          if (q < L.rows) {
            acc.r0 = Guv + 2 * q * pitch;
            acc.r1 = acc.r0 + 1;
            acc.stride = 2;
          } else {
            acc.r0 = Gy + 2 * (q - L.rows) * pitch;
            acc.r1 = acc.r0 + pitch;
            acc.stride = 1;
          }
          return acc;
        },
        [&](int q) {
          StridedPairAcc<T> acc;
          if (q < L.rows) {
            acc.r0 = Guv + 2 * q * pitch;
            acc.r1 = acc.r0 + 1;
            acc.stride = 2;
          } else {
            acc.r0 = Gy + 2 * (q - L.rows) * pitch;
            acc.r1 = acc.r0 + pitch;
            acc.stride = 1;
          }
          return acc;
        });

    // Gather at the points of this band.
    const double *wn = a.windows + 3 * (int64_t)it.cell;
    double acc[3] = {0.0, 0.0, 0.0};
    gather_item<T, W, NT, POLY, RECON>(a, Guv, Gy, L.apitch, it.band * a.band_rows, it.begin, it.end, T(wn[0]),
                                       T(wn[1]), T(wn[2]), acc);
    if constexpr (RECON) {
      // the item's three sums, reduced in a fixed order (waves, then lanes)
      __syncthreads();
      double *red = reinterpret_cast<double *>(sm);
      for (int k = 0; k < 3; ++k) {
        double v = acc[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if ((threadIdx.x & 63) == 0) red[k * (NT / 64) + (threadIdx.x >> 6)] = v;
      }
      __syncthreads();
      if (threadIdx.x < 3) {
        double v = 0.0;
        for (int q = 0; q < NT / 64; ++q) v += red[threadIdx.x * (NT / 64) + q];
        a.rec_part[3 * idx + threadIdx.x] = v;
      }
    }
    __syncthreads();
    if (!persistent) break;
  }
  if (persistent && threadIdx.x == 0) {
    __threadfence();
    const int old = atomicAdd(a.done_counter, 1);
    if (old == (int)gridDim.x - 1) {
      *a.work_counter = 0;
      *a.done_counter = 0;
    }
  }
}

// Compiled with the polynomial taps for FP32 plans that carry them (W <= ES_MAXW).
template <typename T, int W>
constexpr bool adj_has_poly() { return sizeof(T) == 4 && W <= ES_MAXW; }

template <typename T, int W>
static const void *adj_fn(int threads, bool poly) {
  if constexpr (adj_has_poly<T, W>()) {
    if (poly)
      return threads == 256 ? (const void *)&adj_kernel<T, W, 256, true, false>
                            : (const void *)&adj_kernel<T, W, 512, true, false>;
  }
  return threads == 256 ? (const void *)&adj_kernel<T, W, 256, false, false>
                        : (const void *)&adj_kernel<T, W, 512, false, false>;
}

template <typename T, int W, bool RECON>
static hipError_t launch_adj_w(const AdjArgs<T> &a, int blocks, int threads, size_t lds, hipStream_t s) {
  if constexpr (adj_has_poly<T, W>()) {
    if (a.es.on) {
      if (threads == 256) hipLaunchKernelGGL((adj_kernel<T, W, 256, true, RECON>), dim3(blocks), dim3(256), lds, s, a);
      else hipLaunchKernelGGL((adj_kernel<T, W, 512, true, RECON>), dim3(blocks), dim3(512), lds, s, a);
      return hipGetLastError();
    }
  }
  if (threads == 256) hipLaunchKernelGGL((adj_kernel<T, W, 256, false, RECON>), dim3(blocks), dim3(256), lds, s, a);
  else hipLaunchKernelGGL((adj_kernel<T, W, 512, false, RECON>), dim3(blocks), dim3(512), lds, s, a);
  return hipGetLastError();
}

template <typename T, bool RECON>
static hipError_t launch_adj_mode(const AdjArgs<T> &a, int W, int blocks, int threads, size_t lds, hipStream_t s) {
  switch (W) {
    case 4: return launch_adj_w<T, 4, RECON>(a, blocks, threads, lds, s);
    case 6: return launch_adj_w<T, 6, RECON>(a, blocks, threads, lds, s);
    case 8: return launch_adj_w<T, 8, RECON>(a, blocks, threads, lds, s);
    case 10: return launch_adj_w<T, 10, RECON>(a, blocks, threads, lds, s);
    case 12: return launch_adj_w<T, 12, RECON>(a, blocks, threads, lds, s);
    case 14: return launch_adj_w<T, 14, RECON>(a, blocks, threads, lds, s);
    case 16: return launch_adj_w<T, 16, RECON>(a, blocks, threads, lds, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_adj(const AdjArgs<T> &a, int W, int blocks, int threads, size_t lds, hipStream_t s) {
  return a.rec_part ? launch_adj_mode<T, true>(a, W, blocks, threads, lds, s)
                    : launch_adj_mode<T, false>(a, W, blocks, threads, lds, s);
}

template hipError_t launch_adj<float>(const AdjArgs<float> &, int, int, int, size_t, hipStream_t);
template hipError_t launch_adj<double>(const AdjArgs<double> &, int, int, int, size_t, hipStream_t);

// ------------------------------------------------------------------ single-grid adjoint
//
// FP32 plans whose kernel takes the polynomial path: the cell's whole real grid
// of u (the inverse transform of the pre-corrected, Hermitian spectrum) fits
// LDS, and du/dx, du/dy come from the same grid through the derivatives of the
// kernel taps: u(t) = sum_m G_m psi_x psi_y, du/dt_x = sum_m G_m psi_x' psi_y.
// The interpolant's derivative converges more slowly than the interpolant, so
// this path uses its own kernel two cells wider than the forward's (with its
// own deconvolution factors).  One pass per cell: one column transform pass,
// half as many row transforms as rows (real rows in pairs), then the gather.

struct Adj1Layout {
  int rows;      // grid rows stored: n2 + W (the first W - 1 repeated after the last)
  int apitch;    // row pitch: n1 + W - 1 rounded up to even (first W - 1 columns repeated)
  int cpitch;    // column-workspace pitch
  int rsplit;    // compact layout: rows [rsplit, n2) are transformed in the staged batch; 0: not compact
  size_t g_off, ws_off, st_off, db_off, tw_off, total;   // element offsets
};

// The column output db ([n2][K1 + 1] complex) must not overlap the column
// workspace while the column pass writes it.  Compact layout: db ends where the
// grid does, so it shares the grid's last rows; the row transforms then run in
// two batches, rows [0, rsplit) (which lie below db) and rows [rsplit, n2), whose
// first step loads every input before any store (at most one item per thread of
// the NT-thread workgroup).  Otherwise db follows the grid.
__host__ __device__ inline Adj1Layout adj1_layout(const Geom &g, int W, size_t elem, int NT) {
  Adj1Layout L;
  L.rows = g.n2 + W;
  L.apitch = (g.n1 + W - 1 + 1) & ~1;
  L.cpitch = 2 * (g.K1 + 1) + 2;
  L.g_off = 0;
  // the column workspace and the staged spectrum alias the grid (both are dead
  // before the row transforms write it)
  L.ws_off = 0;
  const size_t ws = (size_t)g.n2 * L.cpitch;
  L.st_off = ws;
  const size_t gsz = (size_t)L.rows * L.apitch, wst = ws + adj_stage_elems(g, elem);
  const size_t dbsz = (size_t)g.n2 * (g.K1 + 1) * 2;
  L.rsplit = 0;
  size_t db = gsz > wst ? gsz : wst;
  if (gsz >= dbsz && gsz - dbsz >= ws) {
    const size_t dc = gsz - dbsz;
    int rs = (int)(dc / L.apitch) & ~1;                 // rows [0, rs) end at or below db
    const int items = (g.n2 - rs) / 2 * fft_B(g.n1);    // first-step items of the staged batch
    if (rs >= 2 && rs < g.n2 && items <= NT) {
      L.rsplit = rs;
      db = dc;
    }
  }
  L.db_off = db;
  const size_t end = db + dbsz;
  const size_t top = end > gsz ? end : gsz;
  L.tw_off = top > wst ? top : wst;
  L.total = L.tw_off + 2 * (size_t)(g.n1 + g.n2);
  return L;
}

// First step of the row-pair inverse transforms for pairs [q0, q0 + count) whose
// spectra are read from LDS that the step's own stores overwrite: every item
// loads its A inputs, the workgroup waits, then every item transforms and
// stores (one item per thread, count * B <= NT).  The same arithmetic as
// fft4_step1_swz.
template <int A, int B, int NT, typename Make>
__device__ __forceinline__ void row_step1_staged(int q0, int count, const float *tw, const Make &make1) {
  const int it = threadIdx.x;
  const bool on = it < count * B;
  const int q = q0 + (on ? it / B : 0), b = on ? it % B : 0;
  const auto acc = make1(q);
  float re[A], im[A];
#pragma unroll
  for (int a = 0; a < A; ++a) {
    re[a] = 0.0f;
    im[a] = 0.0f;
    if (on) acc.load(a * B + b, re[a], im[a]);
  }
  __syncthreads();
  if (on) {
    dft_reg<A, true, float>(re, im);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      float r = re[k1], i = im[k1];
      if (k1 > 0) {
        const int j = b * k1;
        const float c = tw[2 * j], sn = -tw[2 * j + 1];
        const float nr = r * c - i * sn;
        i = r * sn + i * c;
        r = nr;
      }
      acc.store(k1 * B + (b ^ fft_swz(k1, B)), r, i);
    }
  }
  __syncthreads();
}

// Taps and their derivatives from the mirror-pair polynomials of the taps alone
// (no second set of coefficients, so the kernel's scalar registers hold one
// table).  With P_d(u) = E(s) + u O(s) and s = u^2: dP_d/du = O + 2 u (E' + u O'),
// and the mirror tap W - 1 - d, E - u O, has -O + 2 u (E' - u O'); E' and O'
// (d/ds) come out of the same Horner steps.
// Mirror pair d of the taps and of their u-derivatives: tap d, tap W - 1 - d and
// the two derivatives dP/du, from the pair's coefficients cd at u and s = u^2.
// (With u = 2 (i0 - t + W/2) - 1, d/dt = -2 d/du: the caller's scale carries the
// factor -2, so it is not multiplied into every tap.)
__device__ __forceinline__ void es_pair_dtaps(float u, float s, const float *cd, float &t0, float &t1, float &d0,
                                              float &d1) {
  float e = cd[ES_DEG - 1], o = cd[ES_DEG], de = 0.0f, dO = 0.0f;
#pragma unroll
  for (int k = ES_DEG - 3; k >= 0; k -= 2) {
    de = fmaf(de, s, e);
    dO = fmaf(dO, s, o);
    e = fmaf(e, s, cd[k]);
    o = fmaf(o, s, cd[k + 1]);
  }
  t0 = fmaf(u, o, e);
  t1 = fmaf(-u, o, e);
  const float u2 = 2.0f * u;
  d0 = fmaf(u2, fmaf(u, dO, de), o);
  d1 = fmaf(u2, fmaf(-u, dO, de), -o);
}

template <int W>
__device__ __forceinline__ void es_taps_dtaps_poly_v(float v, const EsPoly &cf, float (&out)[W],
                                                     float (&dout)[W]) {
  const float u = 2.0f * v - 1.0f;
  const float s = u * u;
#pragma unroll
  for (int d = 0; d < W / 2; ++d)
    es_pair_dtaps(u, s, cf.c + d * (ES_DEG + 1), out[d], out[W - 1 - d], dout[d], dout[W - 1 - d]);
}

// Holds the two rows' grid values until every read of the pair has returned,
// so the reads are issued together and waited for once (left to itself the
// compiler waited after each read, one LDS round trip per two values).
template <int W>
__device__ __forceinline__ void hold_rows(float (&ra)[W], float (&rb)[W]) {
  if constexpr (W == 8) {
    asm volatile("" : "+v"(ra[0]), "+v"(ra[1]), "+v"(ra[2]), "+v"(ra[3]), "+v"(ra[4]), "+v"(ra[5]), "+v"(ra[6]),
                      "+v"(ra[7]), "+v"(rb[0]), "+v"(rb[1]), "+v"(rb[2]), "+v"(rb[3]), "+v"(rb[4]), "+v"(rb[5]),
                      "+v"(rb[6]), "+v"(rb[7]));
  } else if constexpr (W == 6) {
    asm volatile("" : "+v"(ra[0]), "+v"(ra[1]), "+v"(ra[2]), "+v"(ra[3]), "+v"(ra[4]), "+v"(ra[5]), "+v"(rb[0]),
                      "+v"(rb[1]), "+v"(rb[2]), "+v"(rb[3]), "+v"(rb[4]), "+v"(rb[5]));
  }
}

// Gradients at one point: W x W taps of the grid with value and derivative
// weights (row sums with psi_x and psi_x', then combined with psi_y, psi_y'),
// then the chain rule through the strength as in gather_point.
template <int W>
__device__ __forceinline__ void gather1_point(const AdjArgs<float> &a, const float *G, int apitch, int64_t j, float xj,
                                              float yj, float hj, float wj, float cx, float cy, float R, float pr) {
  const Geom &g = a.g;
  const float halfw = float(W) * 0.5f;
  const FineCoord<float> fx = fine_coord<float>(xj, a.s1_hi, a.s1_lo, halfw);
  const FineCoord<float> fy = fine_coord<float>(yj, a.s2_hi, a.s2_lo, halfw);
  const float vx = tap_v(fx, halfw), vy = tap_v(fy, halfw);
  float kx[W], kxd[W];
  es_taps_dtaps_poly_v<W>(vx, a.es, kx, kxd);
  const float uyv = 2.0f * vy - 1.0f, syv = uyv * uyv;
  const float *p = G + (fy.i0 & (g.n2 - 1)) * apitch + (fx.i0 & (g.n1 - 1));
  float u = 0.0f, ux = 0.0f, uy = 0.0f;
  // rows in mirror pairs (d, W - 1 - d), whose y taps come from one polynomial pair
#pragma unroll
  for (int d = 0; d < W / 2; ++d) {
    const float *pa = p + d * apitch, *pb = p + (W - 1 - d) * apitch;
    float ra[W], rb[W];
#pragma unroll
    for (int dx = 0; dx < W; ++dx) {
      ra[dx] = pa[dx];
      rb[dx] = pb[dx];
    }
    float ta, tb, da, db;
    es_pair_dtaps(uyv, syv, a.es.c + d * (ES_DEG + 1), ta, tb, da, db);
    hold_rows<W>(ra, rb);
    float sa = 0.0f, sda = 0.0f, sb = 0.0f, sdb = 0.0f;
#pragma unroll
    for (int dx = 0; dx < W; ++dx) {
      sa = fmaf(kx[dx], ra[dx], sa);
      sda = fmaf(kxd[dx], ra[dx], sda);
      sb = fmaf(kx[dx], rb[dx], sb);
      sdb = fmaf(kxd[dx], rb[dx], sdb);
    }
    u = fmaf(ta, sa, u);
    ux = fmaf(ta, sda, ux);
    uy = fmaf(da, sa, uy);
    u = fmaf(tb, sb, u);
    ux = fmaf(tb, sdb, ux);
    uy = fmaf(db, sb, uy);
  }
  // the derivative sums are formed here, in the row loop, not sunk into the
  // branch that stores them (which kept all W x W grid values live)
  asm volatile("" : "+v"(ux), "+v"(uy));
  ux *= a.dsx;   // -2 n1 / (2 pi): d/dt of the fine coordinate, d/du = -2 d/dt
  uy *= a.dsy;
  float dWx, dWy;
  const float Wv = hann_wg(a.window_kind, xj, yj, cx, cy, R, pr, dWx, dWy);
  if (a.grad_h) a.grad_h[j] = wj * Wv * u;
  if (a.grad_x || a.grad_y) {
    const float wh = wj * hj;
    if (a.grad_x) a.grad_x[j] = wh * (dWx * u + Wv * ux);
    if (a.grad_y) a.grad_y[j] = wh * (dWy * u + Wv * uy);
  }
}

// All points of one item: wave w takes blocks of 64 consecutive points, one per
// lane (so the 64 lanes of a step read overlapping footprints of raster-ordered
// points); each lane's next point is loaded while the current one is gathered.
// (Four points per lane and block, picked by a run-time index, had put the
// buffers in scratch memory: 16 bytes per point written and read back.)
template <int W, int NT>
__device__ __forceinline__ void gather1_item(const AdjArgs<float> &a, const float *G, int apitch, int64_t begin,
                                             int64_t end, float cx, float cy, float R) {
  const float pr = R > 0.0f ? float(M_PI) / R : 0.0f;
  constexpr int NWV = NT / 64;
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)NWV * 64;
  struct Pt {
    float x, y, h, w;
  };
  auto load = [&](Pt &b, int64_t i) {
    const int64_t ic = i < end ? i : end - 1;   // past the end: re-read the last point (unused)
    b.x = a.x[ic]; b.y = a.y[ic]; b.h = a.h[ic]; b.w = a.w[ic];
  };
  if (begin >= end) return;
  int64_t i = begin + (int64_t)(threadIdx.x >> 6) * 64 + lane;
  Pt b0, b1;
  load(b0, i);
  for (; i - lane < end; i += 2 * stride) {
    load(b1, i + stride);
    if (i < end) gather1_point<W>(a, G, apitch, i, b0.x, b0.y, b0.h, b0.w, cx, cy, R, pr);
    load(b0, i + 2 * stride);
    if (i + stride < end) gather1_point<W>(a, G, apitch, i + stride, b1.x, b1.y, b1.h, b1.w, cx, cy, R, pr);
  }
}

// Four waves per SIMD: two 512-thread workgroups per CU with the compact layout
// (each thread then within 128 VGPRs).
template <int W, int NT>
__global__ __launch_bounds__(NT, (NT == 512 ? 4 : 1)) void adj1_kernel(AdjArgs<float> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float *sm = reinterpret_cast<float *>(smem_raw);
  __shared__ int s_item;
  const Geom &g = a.g;
  const Adj1Layout L = adj1_layout(g, W, sizeof(float), NT);
  float *G = sm + L.g_off, *ws = sm + L.ws_off, *st = sm + L.st_off, *db = sm + L.db_off;
  float *tw1 = sm + L.tw_off, *tw2 = tw1 + 2 * g.n1;
  const int per = g.K1 + 1, pitch = L.apitch;
  const bool persistent = a.work_counter != nullptr;
  int64_t idx = a.item_base + blockIdx.x;
  if (!persistent && idx >= a.n_items) return;
  for (int i = threadIdx.x; i < 2 * g.n1; i += NT) tw1[i] = a.tw1[i];
  for (int i = threadIdx.x; i < 2 * g.n2; i += NT) tw2[i] = a.tw2[i];
  if (!persistent) __syncthreads();
  for (;;) {
    if (persistent) {
      if (threadIdx.x == 0) s_item = atomicAdd(a.work_counter, 1);
      __syncthreads();
      idx = s_item;
      __syncthreads();
      if (idx >= a.n_items) break;
    }
    const AdjItem it = a.items[idx];
    const float *gc = a.fbar + (int64_t)it.cell * g.N1 * g.N2 * 2;
    const float two_lam = a.keep ? float(2.0 * (a.lam ? a.lam[it.cell] : 1.0)) : 1.0f;
    stage_spectrum<float, NT>(a, gc, it.cell, st);
    // columns kx = 0 .. K1 of the pre-corrected spectrum, inverse transformed along y
    column_pass<float, NT>(a, st, tw2, two_lam, ws, L.cpitch, false, db, g.n2, 0);
    // rows in pairs: Z(k) = D_2q(k) + i D_2q+1(k) gives rows 2q and 2q + 1 as its real
    // and imaginary parts (both rows' spectra are Hermitian)
    const int n1 = g.n1, K1 = g.K1;
    auto make1 = [&](int q) {
      RowSpecAcc<float> acc;
      acc.db = db;
      acc.row = 2 * q;
      acc.pair = true;
      acc.per = per;
      acc.n1 = n1;
      acc.K1 = K1;
      acc.r0 = G + 2 * q * pitch;
      acc.r1 = acc.r0 + pitch;
      acc.stride = 1;
      return acc;
    };
    auto make2 = [&](int q) {
      StridedPairAcc<float> acc;
      acc.r0 = G + 2 * q * pitch;
      acc.r1 = acc.r0 + pitch;
      acc.stride = 1;
      return acc;
    };
    if (L.rsplit == 0) {
      row_ifft_natural<NT, float>(n1, g.n2 / 2, tw1, W - 1, make1, make2);
    } else {
      // rows below db first, then the rows that share its space
      const int qs = L.rsplit / 2, qn = g.n2 / 2 - qs;
      row_ifft_natural<NT, float>(n1, qs, tw1, W - 1, make1, make2);
      switch (n1) {
        case 16: row_step1_staged<4, 4, NT>(qs, qn, tw1, make1); break;
        case 32: row_step1_staged<8, 4, NT>(qs, qn, tw1, make1); break;
        case 64: row_step1_staged<8, 8, NT>(qs, qn, tw1, make1); break;
        default: row_step1_staged<16, 8, NT>(qs, qn, tw1, make1); break;
      }
      const int A2 = fft_A(n1), la = fft_logA(n1);
      for (int it = threadIdx.x; it < qn * A2; it += NT) {
        const int q = qs + (it >> la), k1 = it & (A2 - 1);
        switch (n1) {
          case 16: row_step2_natural<4, 4, float>(make2(q), k1, n1, W - 1); break;
          case 32: row_step2_natural<8, 4, float>(make2(q), k1, n1, W - 1); break;
          case 64: row_step2_natural<8, 8, float>(make2(q), k1, n1, W - 1); break;
          default: row_step2_natural<16, 8, float>(make2(q), k1, n1, W - 1); break;
        }
      }
      __syncthreads();
    }
    // the first W - 1 rows again after the last (with their repeated columns)
    for (int i = threadIdx.x; i < (W - 1) * pitch; i += NT) G[g.n2 * pitch + i] = G[i];
    __syncthreads();
    const double *wn = a.windows + 3 * (int64_t)it.cell;
    gather1_item<W, NT>(a, G, pitch, it.begin, it.end, float(wn[0]), float(wn[1]), float(wn[2]));
    __syncthreads();
    if (!persistent) break;
  }
  if (persistent && threadIdx.x == 0) {
    __threadfence();
    const int old = atomicAdd(a.done_counter, 1);
    if (old == (int)gridDim.x - 1) {
      *a.work_counter = 0;
      *a.done_counter = 0;
    }
  }
}

static const void *adj1_fn(int W, int threads) {
  if (W == 6) return threads == 512 ? (const void *)&adj1_kernel<6, 512> : (const void *)&adj1_kernel<6, 1024>;
  if (W == 8) return threads == 512 ? (const void *)&adj1_kernel<8, 512> : (const void *)&adj1_kernel<8, 1024>;
  return nullptr;
}

static hipError_t launch_adj1(const AdjArgs<float> &a, int W, int blocks, int threads, size_t lds, hipStream_t s) {
  const void *fn = adj1_fn(W, threads);
  if (!fn) return hipErrorInvalidValue;
  void *args[] = {const_cast<AdjArgs<float> *>(&a)};
  return hipLaunchKernel(fn, dim3(blocks), dim3(threads), args, lds, s);
}

// ------------------------------------------------------------------ host side

enufft_status record_start(enufft_plan_t p, int kind, hipEvent_t *ev);
enufft_status record_stop(enufft_plan_t p, int kind, hipEvent_t start);
template <typename T>
void split_scale(int n, T *hi, T *lo);

// Bands per cell: the fewest row bands whose three grids, band spectra and
// column workspace fit one workgroup's LDS.
int choose_bands(const Geom &g, int W, size_t elem, size_t lds_max, int *band_rows, size_t *lds) {
  if (W & 1) return 0;   // uy rows are transformed in pairs: band rows must be even
  for (int B = 1; B <= g.n2 / 2; B <<= 1) {
    const int R = g.n2 / B;
    if (R < 2) break;
    const AdjLayout L = adj_layout(g, W, R, elem);
    const size_t bytes = L.total * elem;
    if (bytes <= lds_max) {
      *band_rows = R;
      *lds = bytes;
      return B;
    }
  }
  return 0;
}

// Adjoint work list: every (cell, band) pair, cells above the chunk target cut
// into point chunks (gathers need no merge), longest first.
void build_adj_schedule(enufft_plan_t p, int slots, int B, std::vector<AdjItem> &items) {
  const int64_t Q = p->n_points;
  const int64_t per = (int64_t)p->adj_items_per_slot * std::max(1, slots);
  const int64_t T = std::max<int64_t>(16384, (Q * B + per - 1) / per);
  items.clear();
  for (int64_t c = 0; c < p->n_cells; ++c) {
    const int64_t a = p->offsets[c], b = p->offsets[c + 1];
    const int64_t q = b - a;
    if (q == 0) continue;
    const int64_t nch = std::max<int64_t>(1, (q + T - 1) / T);
    for (int band = 0; band < B; ++band)
      for (int64_t i = 0; i < nch; ++i)
        items.push_back(AdjItem{a + q * i / nch, a + q * (i + 1) / nch, (int32_t)c, band, 0, 0});
  }
  std::stable_sort(items.begin(), items.end(), [](const AdjItem &x, const AdjItem &y) {
    return (x.end - x.begin) > (y.end - y.begin);
  });
}

template <typename T>
hipError_t adj_occ(int W, int threads, bool poly, size_t lds, int *per_cu) {
  const void *fn = nullptr;
#define ENUFFT_PICK(WW) \
  case WW: fn = adj_fn<T, WW>(threads, poly); break;
  switch (W) {
    ENUFFT_PICK(4) ENUFFT_PICK(6) ENUFFT_PICK(8) ENUFFT_PICK(10) ENUFFT_PICK(12) ENUFFT_PICK(14) ENUFFT_PICK(16)
    default: return hipErrorInvalidValue;
  }
#undef ENUFFT_PICK
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, fn, threads, lds);
}

// Release the adjoint schedule so the next call rebuilds it (autotuner).
void adj_reset(enufft_plan_t p) {
  if (!p->d_adj_items) return;
  const size_t n = std::max<size_t>(1, p->adj_items.size());
  dev_release(p, &p->d_adj_items, n * sizeof(AdjItem));
  dev_release(p, &p->d_rec_part, n * 3 * sizeof(double));
  dev_release(p, &p->d_cell_items, n * sizeof(int32_t));
  dev_release(p, &p->d_cell_item_off, (size_t)(p->n_cells + 1) * sizeof(int64_t));
  dev_release(p, &p->d_cell_off, (size_t)(p->n_cells + 1) * sizeof(int64_t));
  p->adj_items.clear();
  dev_release(p, &p->d_adj1_items, std::max<size_t>(1, p->adj1_items.size()) * sizeof(AdjItem));
  p->adj1_items.clear();
}

// Device allocation recorded in the plan's workspace (released with the plan).
static enufft_status adj_alloc(enufft_plan_t p, void **d, size_t bytes, const char *what) {
  hipError_t e = hipMalloc(d, std::max<size_t>(16, bytes));
  if (e != hipSuccess) {
    *d = nullptr;
    p->last_error = std::string(what) + " allocation failed";
    return ENUFFT_ENOMEM;
  }
  p->allocations.push_back(*d);
  p->workspace_bytes += (int64_t)std::max<size_t>(16, bytes);
  return ENUFFT_OK;
}

// Lazily set up the adjoint schedule on first use.
enufft_status adj_prepare(enufft_plan_t p) {
  if (p->d_adj_items) return ENUFFT_OK;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, p->device);
  if (e != hipSuccess) {
    p->last_error = std::string("hipGetDeviceProperties: ") + hipGetErrorString(e);
    return ENUFFT_EDEVICE;
  }
  p->adj_threads = p->prec == ENUFFT_F64 ? 256 : 512;
  int B = choose_bands(p->geom, p->W, p->elem, (size_t)prop.sharedMemPerBlock, &p->adj_band_rows, &p->adj_lds);
  if (B == 0) {
    p->last_error = "adjoint: fine-grid bands do not fit in LDS";
    return ENUFFT_EUNSUPPORTED;
  }
  // more bands than the minimum (autotuner choice): smaller LDS footprint per item
  for (int m = p->adj_band_mult; m > 1 && p->geom.n2 / (B * 2) >= 2; m >>= 1) {
    B *= 2;
    p->adj_band_rows = p->geom.n2 / B;
    p->adj_lds = adj_layout(p->geom, p->W, p->adj_band_rows, p->elem).total * p->elem;
  }
  p->adj_bands = B;
  int per_cu = 0;
  e = p->prec == ENUFFT_F64 ? adj_occ<double>(p->W, p->adj_threads, p->es.on != 0, p->adj_lds, &per_cu)
                            : adj_occ<float>(p->W, p->adj_threads, p->es.on != 0, p->adj_lds, &per_cu);
  if (e != hipSuccess || per_cu < 1) {
    p->last_error = "adjoint kernel cannot be resident";
    return ENUFFT_EDEVICE;
  }
  const int slots = p->n_cu * per_cu;
  build_adj_schedule(p, slots, p->adj_bands, p->adj_items);
  p->adj_blocks = (int)std::min<int64_t>(slots, std::max<int64_t>(1, (int64_t)p->adj_items.size()));
  const size_t n_items = std::max<size_t>(1, p->adj_items.size());
  // the items of each cell, ascending (the reconstruction sums a cell's item
  // partials in this fixed order)
  std::vector<int64_t> coff(p->n_cells + 1, 0);
  for (const AdjItem &it : p->adj_items) ++coff[it.cell + 1];
  for (int64_t c = 0; c < p->n_cells; ++c) coff[c + 1] += coff[c];
  std::vector<int32_t> citems(n_items, 0);
  {
    std::vector<int64_t> pos(coff.begin(), coff.end() - 1);
    for (size_t i = 0; i < p->adj_items.size(); ++i) citems[pos[p->adj_items[i].cell]++] = (int32_t)i;
  }
  void *d = nullptr;
  enufft_status st = adj_alloc(p, &d, n_items * sizeof(AdjItem), "adjoint item");
  if (st == ENUFFT_OK) st = adj_alloc(p, &p->d_rec_part, n_items * 3 * sizeof(double), "reconstruction partials");
  if (st == ENUFFT_OK) st = adj_alloc(p, &p->d_cell_items, n_items * sizeof(int32_t), "cell item list");
  if (st == ENUFFT_OK)
    st = adj_alloc(p, &p->d_cell_item_off, (size_t)(p->n_cells + 1) * sizeof(int64_t), "cell item offsets");
  if (st == ENUFFT_OK) st = adj_alloc(p, &p->d_cell_off, (size_t)(p->n_cells + 1) * sizeof(int64_t), "cell offsets");
  if (st != ENUFFT_OK) return st;
  if (!p->adj_items.empty())
    e = hipMemcpy(d, p->adj_items.data(), p->adj_items.size() * sizeof(AdjItem), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_cell_items, citems.data(), n_items * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_cell_item_off, coff.data(), coff.size() * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_cell_off, p->offsets.data(), p->offsets.size() * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    p->last_error = std::string("adjoint item upload: ") + hipGetErrorString(e);
    p->faulted = true;
    return ENUFFT_EDEVICE;
  }
  if (p->adj1) {
    // single-grid adjoint: one item per cell (or chunk of a large cell), no bands;
    // 512 threads, so two workgroups fit a CU with the compact layout
    if (const char *ev = std::getenv("ENUFFT_ADJ1_THREADS")) p->adj1_threads = std::atoi(ev) == 1024 ? 1024 : 512;
    p->adj1_lds = adj1_layout(p->geom, p->adj1_W, sizeof(float), p->adj1_threads).total * sizeof(float);
    const void *fn = adj1_fn(p->adj1_W, p->adj1_threads);
    int per1 = 0;
    e = fn ? hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p->adj1_lds)
           : hipErrorInvalidValue;
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per1, fn, p->adj1_threads, p->adj1_lds);
    if (e != hipSuccess || per1 < 1) {
      p->last_error = "single-grid adjoint kernel cannot be resident";
      return ENUFFT_EDEVICE;
    }
    const int slots1 = p->n_cu * per1;
    build_adj_schedule(p, slots1, 1, p->adj1_items);
    p->adj1_blocks = (int)std::min<int64_t>(slots1, std::max<int64_t>(1, (int64_t)p->adj1_items.size()));
    void *d1 = nullptr;
    st = adj_alloc(p, &d1, std::max<size_t>(1, p->adj1_items.size()) * sizeof(AdjItem), "adjoint item");
    if (st != ENUFFT_OK) return st;
    if (!p->adj1_items.empty())
      e = hipMemcpy(d1, p->adj1_items.data(), p->adj1_items.size() * sizeof(AdjItem), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      p->last_error = std::string("adjoint item upload: ") + hipGetErrorString(e);
      p->faulted = true;
      return ENUFFT_EDEVICE;
    }
    p->d_adj1_items = d1;
  }
  p->d_adj_items = d;
  return ENUFFT_OK;
}

template <typename T>
AdjArgs<T> make_adj_args(enufft_plan_t p, const void *x, const void *y, const void *h, const void *w,
                         const void *fbar, void *gh, void *gx, void *gy) {
  AdjArgs<T> a{};
  a.x = (const T *)x; a.y = (const T *)y; a.h = (const T *)h; a.w = (const T *)w;
  {
    const size_t al = 4 * sizeof(T);
    a.vec4 = ((uintptr_t)x % al == 0 && (uintptr_t)y % al == 0 && (uintptr_t)h % al == 0 &&
              (uintptr_t)w % al == 0) ? 1 : 0;
  }
  a.fbar = (const T *)fbar;
  a.keep = nullptr;
  a.lam = nullptr;
  a.grad_h = (T *)gh; a.grad_x = (T *)gx; a.grad_y = (T *)gy;
  a.items = (const AdjItem *)p->d_adj_items;
  a.n_items = (int64_t)p->adj_items.size();
  a.item_base = 0;
  a.work_counter = p->d_counters + 2;
  a.done_counter = p->d_counters + 3;
  a.windows = (const double *)p->d_windows;
  a.window_kind = p->window_kind;
  a.decon_x = (const T *)p->d_decon_x; a.decon_y = (const T *)p->d_decon_y;
  a.tw1 = (const T *)p->d_tw1; a.tw2 = (const T *)p->d_tw2;
  a.beta = (T)p->beta;
  split_scale<T>(p->n1, &a.s1_hi, &a.s1_lo);
  split_scale<T>(p->n2, &a.s2_hi, &a.s2_lo);
  a.es = p->es;
  a.bands = p->adj_bands;
  a.band_rows = p->adj_band_rows;
  a.g = p->geom;
  return a;
}

}  // namespace enufft

namespace enufft {
enufft_status adjoint_common(enufft_plan_t p, const char *fn, const void *x, const void *y, const void *h,
                             const void *w, const void *fin, const uint8_t *keep, const double *lam, void *grad_h,
                             void *grad_x, void *grad_y) {
  if (!p) return ENUFFT_EINVAL;
  if (p->faulted) {
    p->last_error = std::string(fn) + ": plan unusable after a device fault";
    return ENUFFT_ESTATE;
  }
  if (p->n_cells == 0 || p->n_points == 0) return ENUFFT_OK;
  if (!fin) {
    p->last_error = std::string(fn) + ": null coefficient input";
    return ENUFFT_EINVAL;
  }
  if (!x || !y || !h || !w) {   // every kernel reads all four arrays
    p->last_error = std::string(fn) + ": null point array";
    return ENUFFT_EINVAL;
  }
  if (!grad_h && !grad_x && !grad_y) return ENUFFT_OK;
  hipEvent_t ev;
  if (p->big) {
    enufft_status st = record_start(p, 2, &ev);
    if (st != ENUFFT_OK) return st;
    st = big_adjoint(p, x, y, h, w, fin, keep, lam, grad_h, grad_x, grad_y);
    if (st != ENUFFT_OK) return st;
    return record_stop(p, 2, ev);
  }
  enufft_status st = adj_prepare(p);
  if (st != ENUFFT_OK) return st;
  st = record_start(p, 2, &ev);
  if (st != ENUFFT_OK) return st;
  hipError_t e;
  if (p->prec == ENUFFT_F64) {
    auto a = make_adj_args<double>(p, x, y, h, w, fin, grad_h, grad_x, grad_y);
    a.keep = keep;
    a.lam = lam;
    e = launch_adj<double>(a, p->W, p->adj_blocks, p->adj_threads, p->adj_lds, p->stream);
  } else if (p->adj1) {
    auto a = make_adj_args<float>(p, x, y, h, w, fin, grad_h, grad_x, grad_y);
    a.keep = keep;
    a.lam = lam;
    a.items = (const AdjItem *)p->d_adj1_items;
    a.n_items = (int64_t)p->adj1_items.size();
    a.decon_x = (const float *)p->d_adj1_decon_x;
    a.decon_y = (const float *)p->d_adj1_decon_y;
    a.es = p->adj1_es;
    a.dsx = (float)(-2.0 * p->n1 / (2.0 * M_PI));   // dt/dx times du/dt of the tap polynomials
    a.dsy = (float)(-2.0 * p->n2 / (2.0 * M_PI));
    a.bands = 1;
    a.band_rows = p->n2;
    e = launch_adj1(a, p->adj1_W, p->adj1_blocks, p->adj1_threads, p->adj1_lds, p->stream);
  } else {
    auto a = make_adj_args<float>(p, x, y, h, w, fin, grad_h, grad_x, grad_y);
    a.keep = keep;
    a.lam = lam;
    e = launch_adj<float>(a, p->W, p->adj_blocks, p->adj_threads, p->adj_lds, p->stream);
  }
  if (e != hipSuccess) {
    p->last_error = std::string(fn) + " launch: " + hipGetErrorString(e);
    p->faulted = true;
    return ENUFFT_EDEVICE;
  }
  return record_stop(p, 2, ev);
}
}  // namespace enufft

extern "C" enufft_status enufft_type1_adjoint(enufft_plan_t p, const void *x, const void *y, const void *h,
                                              const void *w, const void *fbar, void *grad_h, void *grad_x,
                                              void *grad_y) {
  return enufft::adjoint_common(p, "enufft_type1_adjoint", x, y, h, w, fbar, nullptr, nullptr, grad_h, grad_x,
                                grad_y);
}

extern "C" enufft_status enufft_retained_power_adjoint(enufft_plan_t p, const void *x, const void *y,
                                                       const void *h, const void *w, const void *f,
                                                       const uint8_t *keep, const double *lam, void *grad_h,
                                                       void *grad_x, void *grad_y) {
  if (p && !keep) {
    p->last_error = "enufft_retained_power_adjoint: null keep";
    return ENUFFT_EINVAL;
  }
  return enufft::adjoint_common(p, "enufft_retained_power_adjoint", x, y, h, w, f, keep, lam, grad_h, grad_x,
                                grad_y);
}

// ------------------------------------------------------------------ reconstruction

namespace enufft {

// Per cell: the sums over its items' partials (fixed order) and the spectral
// sums of Parseval's identity over the modes k != 0, all of them and the kept
// ones (a fixed-order tree over 256 threads), then the diagnostics.
template <typename T>
__global__ __launch_bounds__(256) void rec_finalize_kernel(const T *coef, const uint8_t *keep, const double *area,
                                                           const double *part, const int32_t *cell_items,
                                                           const int64_t *cell_item_off, const int64_t *cell_off,
                                                           Geom g, double *diag) {
  __shared__ double s_all[256], s_kept[256];
  const int64_t c = blockIdx.x;
  const int M = g.N1 * g.N2;
  const T *cc = coef + 2 * (int64_t)M * c;
  const uint8_t *kc = keep ? keep + (int64_t)M * c : nullptr;
  double sa = 0.0, sk = 0.0;
  for (int m = threadIdx.x; m < M; m += 256) {
    const int r = m / g.N1, i = m - r * g.N1;
    if (g.lo1 + i == 0 && g.lo2 + r == 0) continue;
    const double re = (double)cc[2 * m], im = (double)cc[2 * m + 1];
    const double p2 = re * re + im * im;
    sa += p2;
    if (!kc || kc[m]) sk += p2;
  }
  s_all[threadIdx.x] = sa;
  s_kept[threadIdx.x] = sk;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s_all[threadIdx.x] += s_all[threadIdx.x + o];
      s_kept[threadIdx.x] += s_kept[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double e2 = 0.0, t2 = 0.0, wt2 = 0.0;
    for (int64_t q = cell_item_off[c]; q < cell_item_off[c + 1]; ++q) {
      const int64_t it = cell_items[q];
      e2 += part[3 * it];
      t2 += part[3 * it + 1];
      wt2 += part[3 * it + 2];
    }
    const double A = area ? area[c] : 1.0;
    double *d = diag + 8 * c;
    d[0] = (double)(cell_off[c + 1] - cell_off[c]);
    d[1] = e2;
    d[2] = t2;
    d[3] = wt2 / A;
    d[4] = s_all[0];
    d[5] = s_kept[0];
    d[6] = t2 > 0.0 ? sqrt(e2 / t2) : 0.0;
    d[7] = d[3] > 0.0 ? d[4] / d[3] : 0.0;
  }
}

}  // namespace enufft

extern "C" enufft_status enufft_reconstruct(enufft_plan_t p, const void *x, const void *y, const void *h,
                                            const void *w, const void *coef, const uint8_t *keep,
                                            const double *area, void *h_rec, double *diag) {
  using namespace enufft;
  if (!p) return ENUFFT_EINVAL;
  if (p->faulted) {
    p->last_error = "enufft_reconstruct: plan unusable after a device fault";
    return ENUFFT_ESTATE;
  }
  if (p->big) {
    p->last_error = "enufft_reconstruct: not implemented for large-cell plans (mode boxes above 64 per axis)";
    return ENUFFT_EUNSUPPORTED;
  }
  if (p->n_cells == 0) return ENUFFT_OK;
  if (!coef || !diag) {
    p->last_error = "enufft_reconstruct: null coefficients or diagnostics";
    return ENUFFT_EINVAL;
  }
  if (p->n_points > 0 && (!x || !y || !h || !w)) {
    p->last_error = "enufft_reconstruct: null point array";
    return ENUFFT_EINVAL;
  }
  enufft_status st = adj_prepare(p);
  if (st != ENUFFT_OK) return st;
  hipError_t e = hipSuccess;
  if (p->n_points > 0) {
    if (p->prec == ENUFFT_F64) {
      auto a = make_adj_args<double>(p, x, y, h, w, coef, h_rec, nullptr, nullptr);
      a.keep = keep;
      a.decon_x = (const double *)p->d_decon_x1;
      a.rec_part = (double *)p->d_rec_part;
      e = launch_adj<double>(a, p->W, p->adj_blocks, p->adj_threads, p->adj_lds, p->stream);
    } else {
      auto a = make_adj_args<float>(p, x, y, h, w, coef, h_rec, nullptr, nullptr);
      a.keep = keep;
      a.decon_x = (const float *)p->d_decon_x1;
      a.rec_part = (double *)p->d_rec_part;
      e = launch_adj<float>(a, p->W, p->adj_blocks, p->adj_threads, p->adj_lds, p->stream);
    }
  }
  if (e == hipSuccess) {
    if (p->prec == ENUFFT_F64)
      hipLaunchKernelGGL(rec_finalize_kernel<double>, dim3((unsigned)p->n_cells), dim3(256), 0, p->stream,
                         (const double *)coef, keep, area, (const double *)p->d_rec_part,
                         (const int32_t *)p->d_cell_items, (const int64_t *)p->d_cell_item_off,
                         (const int64_t *)p->d_cell_off, p->geom, diag);
    else
      hipLaunchKernelGGL(rec_finalize_kernel<float>, dim3((unsigned)p->n_cells), dim3(256), 0, p->stream,
                         (const float *)coef, keep, area, (const double *)p->d_rec_part,
                         (const int32_t *)p->d_cell_items, (const int64_t *)p->d_cell_item_off,
                         (const int64_t *)p->d_cell_off, p->geom, diag);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    p->last_error = std::string("enufft_reconstruct launch: ") + hipGetErrorString(e);
    p->faulted = true;
    return ENUFFT_EDEVICE;
  }
  return ENUFFT_OK;
}
