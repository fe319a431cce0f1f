// Device building blocks shared by the gfx950 kernels: work-item records,
// kernel-argument blocks, the exponential-of-semicircle (ES) spreading kernel,
// and an in-LDS four-step FFT with small in-register DFTs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace enufft {

// ------------------------------------------------------------------ records

// One forward work item: points [begin, end) of `cell`.  A cell with more
// points than one item holds is split into `nchunks` items; chunk partial
// grids go to slots [slot0, slot0 + nchunks) and the last chunk to finish
// merges them.  `slot` is this chunk's slot (-1 for an unsplit cell).
struct FwdItem {
  int64_t begin, end;
  int32_t cell, nchunks, slot, slot0;
};

// One adjoint work item: points [begin, end) of `cell`, row band `band`.
struct AdjItem {
  int64_t begin, end;
  int32_t cell, band, pad0, pad1;
};

// Degree of the per-tap kernel polynomials (FP32 plans) and the largest width
// they are fitted for; the coefficients travel by value in the kernel arguments
// so every lane reads them from scalar registers.
constexpr int ES_DEG = 7;
constexpr int ES_MAXW = 8;
struct EsPoly {
  int on;
  float c[(ES_MAXW / 2) * (ES_DEG + 1)];   // taps 0 .. W/2 - 1, tap-major, ascending powers of u = 2 v - 1
};

// The same per-tap form in FP64 for the large-cell kernels of FP64 plans: degree
// 13 reproduces the taps of the widths those plans use (W = 10 .. 16, eps 1e-9 ..
// 1e-14) to about 5e-13 at W = 12 (the outer tap's square-root branch point at the
// edge of the support limits the fit, not the degree).  Also by value in the
// kernel arguments: its loads are scalar, the same address for every lane.
constexpr int ES64_DEG = 13;
constexpr int ES64_MAXW = 16;
struct EsPoly64 {
  int on;
  double c[(ES64_MAXW / 2) * (ES64_DEG + 1)];   // as EsPoly
};

// Fine-grid and mode-box geometry.
struct Geom {
  int n1, n2;       // fine grid (powers of two: 16..128 in LDS, 64..4096 for large cells)
  int N1, N2;       // modes per axis
  int lo1, lo2;     // -floor(N/2)
  int K1, K2;       // floor(N/2): largest |k| needed per axis
  int pitch;        // LDS row pitch (elements) = n1 + 2
};

template <typename T>
struct FwdArgs {
  const T *x, *y, *h, *w;
  T *f;                      // interleaved complex, n_cells * N2 * N1
  const FwdItem *items;
  int64_t n_items;
  int64_t item_base;         // static mode: block b runs item item_base + b
  int *work_counter;         // persistent mode (NULL: static mode)
  int *done_counter;
  int *cell_counters;        // per cell, for merging split cells
  T *partial;                // partial grids, n1 * n2 reals per slot
  const double *windows;     // per cell (cx, cy, R)
  int window_kind;
  const T *decon_x;          // [K1 + 1]: scale / p_x(|k|)
  const T *decon_y;          // [K2 + 1]: 1 / p_y(|k|)
  const T *tw1, *tw2;        // forward twiddles exp(-2 pi i j / n), interleaved, n entries
  T beta;                    // kernel shape: ES beta (> 0) or -gamma of the Kaiser-Bessel kernel
  T s1_hi, s1_lo, s2_hi, s2_lo;   // n1 / (2 pi) and n2 / (2 pi) as hi + lo
  int vec4;                  // x, y, h, w are 16-byte aligned: load runs of 4 points
  int acc;                   // bytes per LDS grid cell: 8 (FP64 sums) or 4 (FP32 sums)
  EsPoly es;                 // FP32 plans: per-tap kernel polynomials (es.on = 0: exact kernel)
  Geom g;
};

template <typename T>
struct AdjArgs {
  const T *x, *y, *h, *w;
  const T *fbar;             // interleaved complex cotangent (or f when keep != NULL)
  const uint8_t *keep;       // non-NULL: cotangent is 2 lam_c f keep (retained-power loss)
  const double *lam;         // per-cell loss weights lam_c (NULL: 1)
  T *grad_h, *grad_x, *grad_y;
  const AdjItem *items;
  int64_t n_items;
  int64_t item_base;
  int *work_counter;
  int *done_counter;
  const double *windows;
  int window_kind;
  const T *decon_x, *decon_y;  // as the forward (decon_x carries scale)
  const T *tw1, *tw2;          // forward twiddles (the inverse uses their conjugates)
  T beta;
  T s1_hi, s1_lo, s2_hi, s2_lo;
  EsPoly es;                   // as in FwdArgs (the single-grid adjoint: its own kernel's taps)
  T dsx, dsy;                  // single-grid adjoint: -2 n1 / (2 pi), -2 n2 / (2 pi)
  int vec4;                    // x, y, h, w are 16-byte aligned: load runs of 4 points
  int bands, band_rows;        // row bands per cell and rows per band
  double *rec_part;            // reconstruction mode: per item (sum (t - h_rec)^2, sum t^2, sum w t^2)
  Geom g;
};

// ------------------------------------------------------------------ ES kernel

// psi(z) = exp(beta (sqrt(1 - z^2) - 1)) on |z| <= 1, evaluated as
// exp(-beta z^2 / (1 + sqrt(1 - z^2))) so the exponent has no cancellation.
// Rounding can push |z| a hair past 1; those taps take the edge value.
__device__ __forceinline__ float es_eval(float z, float beta) {
  const float z2 = z * z;
  const float s = __builtin_sqrtf(fmaxf(1.0f - z2, 0.0f));
  return __expf(-beta * z2 * __builtin_amdgcn_rcpf(1.0f + s));
}
__device__ __forceinline__ double es_eval(double z, double beta) {
  const double z2 = z * z;
  const double s = sqrt(fmax(1.0 - z2, 0.0));
  return exp(-beta * z2 / (1.0 + s));
}

// Modified Bessel function I0 by its power series sum_k ((x/2)^2)^k / (k!)^2, summed
// until a term no longer changes the sum (at most 120 terms: enough for x <= 60).
template <typename T>
__device__ __forceinline__ T bessel_i0(T x) {
  const T t = T(0.25) * x * x;
  T term = T(1), sum = T(1);
  for (int k = 1; k < 120; ++k) {
    term *= t / T(k * k);
    const T next = sum + term;
    if (next == sum) break;
    sum = next;
  }
  return sum;
}

// The Kaiser-Bessel kernel of eq. (kb_compact) on z = x / a in [-1, 1], normalised to
// 1 at z = 0: I0(gamma sqrt(1 - z^2)) / I0(gamma).
template <typename T>
__device__ __forceinline__ T kb_eval(T z, T gamma) {
  const T s = sqrt(fmax(T(1) - z * z, T(0)));
  return bessel_i0<T>(gamma * s) / bessel_i0<T>(gamma);
}

// The plan's spreading kernel at z in [-1, 1]: shape > 0 is the exponential of a
// semicircle with beta = shape, shape < 0 the Kaiser-Bessel kernel with gamma = -shape.
__device__ __forceinline__ float ker_eval(float z, float shape) {
  return shape > 0.0f ? es_eval(z, shape) : kb_eval<float>(z, -shape);
}
__device__ __forceinline__ double ker_eval(double z, double shape) {
  return shape > 0.0 ? es_eval(z, shape) : kb_eval<double>(z, -shape);
}

// Fine-grid coordinate t = x n / (2 pi), kept as t_hi + t_lo with the scale
// n / (2 pi) split the same way, so the tap offsets (i0 + d) - t are exact to a
// few units in the last place whatever the size of t.  The footprint starts at
// i0 = ceil(t - W/2); indices are wrapped with the grid mask by the caller, so
// no folding rounds t.  Non-finite or huge coordinates (|t| >= 2^22) are
// placed at t = 0 so every index stays in range.
template <typename T>
struct FineCoord {
  int i0;
  T hi, lo;
  __device__ __forceinline__ T offset(int d) const { return (T(i0 + d) - hi) - lo; }
};

template <typename T>
__device__ __forceinline__ FineCoord<T> fine_coord(T x, T s_hi, T s_lo, T halfw) {
  FineCoord<T> c;
  c.hi = x * s_hi;
  c.lo = fma(x, s_hi, -c.hi) + x * s_lo;
  const T t = c.hi + c.lo;
  if (!(fabs(t) < T(4194304))) { c.hi = T(0); c.lo = T(0); }
  c.i0 = (int)ceil((c.hi + c.lo) - halfw);
  return c;
}

// Radial Hann window W = (1 + cos(pi r / R)) / 2 for r < R, else 0, and its
// gradient -(pi^2 / (2 R^2)) sinc(pi r / R) (x - cx, y - cy).  kind 0 is no
// window.  pr = pi / R is precomputed per cell.  FP32 uses the hardware
// sqrt / reciprocal / sin / cos instructions (errors ~1e-6 absolute on W, far
// inside the FP32 tolerance; the correctly rounded square root costs about ten
// more instructions per point); FP64 uses the accurate library functions.
__device__ __forceinline__ float hann_w(int kind, float x, float y, float cx, float cy, float R, float pr) {
  if (kind == 0) return 1.0f;
  const float dx = x - cx, dy = y - cy;
  const float r = __builtin_amdgcn_sqrtf(dx * dx + dy * dy);
  if (!(r < R)) return 0.0f;
  return 0.5f + 0.5f * __cosf(pr * r);
}
__device__ __forceinline__ double hann_w(int kind, double x, double y, double cx, double cy, double R, double pr) {
  if (kind == 0) return 1.0;
  const double dx = x - cx, dy = y - cy;
  const double r = sqrt(dx * dx + dy * dy);
  if (!(r < R)) return 0.0;
  return 0.5 + 0.5 * cos(pr * r);
}
__device__ __forceinline__ float hann_wg(int kind, float x, float y, float cx, float cy, float R, float pr,
                                         float &gx, float &gy) {
  gx = 0.0f; gy = 0.0f;
  if (kind == 0) return 1.0f;
  const float dx = x - cx, dy = y - cy;
  const float r = __builtin_amdgcn_sqrtf(dx * dx + dy * dy);
  if (!(r < R)) return 0.0f;
  const float u = pr * r;
  const float s = __sinf(u), c = __cosf(u);
  const float sinc = (u > 1e-4f) ? s * __builtin_amdgcn_rcpf(u) : 1.0f - u * u * (1.0f / 6.0f);
  const float k = -0.5f * pr * pr * sinc;
  gx = k * dx;
  gy = k * dy;
  return 0.5f + 0.5f * c;
}
__device__ __forceinline__ double hann_wg(int kind, double x, double y, double cx, double cy, double R, double pr,
                                          double &gx, double &gy) {
  gx = 0.0; gy = 0.0;
  if (kind == 0) return 1.0;
  const double dx = x - cx, dy = y - cy;
  const double r = sqrt(dx * dx + dy * dy);
  if (!(r < R)) return 0.0;
  const double u = pr * r;
  double s, c;
  sincos(u, &s, &c);
  const double sinc = (u > 1e-8) ? s / u : 1.0 - u * u / 6.0;
  const double k = -0.5 * pr * pr * sinc;
  gx = k * dx;
  gy = k * dy;
  return 0.5 + 0.5 * c;
}

// Polynomial form of the spreading kernel.  With v = i0 - t + W/2 in [0, 1),
// tap d sits at z = (v + d - W/2) 2 / W, a smooth function of v on the whole
// interval; psi there is fitted (plan time, FP64 Chebyshev interpolation) by a
// degree-ES_DEG polynomial in u = 2 v - 1.  Horner on these coefficients
// replaces the square root, reciprocal and exponential of every tap by ES_DEG
// fused multiply-adds.
//
// psi is even, so tap W - 1 - d at u equals tap d at -u.  Splitting tap d's
// polynomial into even and odd parts, P_d(u) = E(u^2) + u O(u^2), gives both
// mirror taps from one pair of half-degree Horner chains: E + u O and E - u O.
//
// tap_v gives v = i0 - t + W/2 clamped to [0, 1]; es_taps_poly_v the W taps from it.
__device__ __forceinline__ float tap_v(const FineCoord<float> &c, float halfw) {
  const float v = ((float(c.i0) - c.hi) - c.lo) + halfw;
  return fminf(fmaxf(v, 0.0f), 1.0f);
}

template <int W>
__device__ __forceinline__ void es_taps_poly_v(float v, const EsPoly &cf, float (&out)[W]) {
  static_assert(W % 2 == 0 && ES_DEG % 2 == 1, "mirror-pair evaluation needs even W and odd degree");
  const float u = 2.0f * v - 1.0f;
  const float s = u * u;
#pragma unroll
  for (int d = 0; d < W / 2; ++d) {
    const float *cd = cf.c + d * (ES_DEG + 1);
    float e = cd[ES_DEG - 1], o = cd[ES_DEG];
#pragma unroll
    for (int k = ES_DEG - 3; k >= 0; k -= 2) {
      e = fmaf(e, s, cd[k]);
      o = fmaf(o, s, cd[k + 1]);
    }
    out[d] = fmaf(u, o, e);
    out[W - 1 - d] = fmaf(-u, o, e);
  }
}

template <int W>
__device__ __forceinline__ void es_taps_poly(const FineCoord<float> &c, float halfw, const EsPoly &cf,
                                             float (&out)[W]) {
  es_taps_poly_v<W>(tap_v(c, halfw), cf, out);
}

// Exact FP32 taps from v (tap d at z = (v + d - W/2) 2 / W).
template <int W>
__device__ __forceinline__ void es_taps_exact_v(float v, float beta, float (&out)[W]) {
  const float zsc = 2.0f / float(W);
#pragma unroll
  for (int d = 0; d < W; ++d) out[d] = ker_eval((v + float(d - W / 2)) * zsc, beta);
}

// The W kernel values of one point along one axis: polynomial form when the
// plan provides it (FP32, W <= ES_MAXW), else the exponential of the semicircle.
template <typename T, int W>
__device__ __forceinline__ void es_taps(const FineCoord<T> &c, T beta, const EsPoly &cf, T (&out)[W]) {
  if constexpr (sizeof(T) == 4 && W <= ES_MAXW) {
    if (cf.on) {
      es_taps_poly<W>(c, float(W) * 0.5f, cf, out);
      return;
    }
  }
  const T zsc = T(2) / T(W);
#pragma unroll
  for (int d = 0; d < W; ++d) out[d] = ker_eval(c.offset(d) * zsc, beta);
}

// ------------------------------------------------------------------ small DFTs

// cos(2 pi k / 16) and sin(2 pi k / 16).  Used with compile-time k only, so
// every twiddle below folds to an immediate.
__host__ __device__ constexpr double cos16(int k) {
  switch (k & 15) {
    case 0: return 1.0;
    case 1: return 0.92387953251128673848;
    case 2: return 0.70710678118654752440;
    case 3: return 0.38268343236508977173;
    case 4: return 0.0;
    case 5: return -0.38268343236508977173;
    case 6: return -0.70710678118654752440;
    case 7: return -0.92387953251128673848;
    case 8: return -1.0;
    case 9: return -0.92387953251128673848;
    case 10: return -0.70710678118654752440;
    case 11: return -0.38268343236508977173;
    case 12: return 0.0;
    case 13: return 0.38268343236508977173;
    case 14: return 0.70710678118654752440;
    default: return 0.92387953251128673848;
  }
}
__host__ __device__ constexpr double sin16(int k) { return cos16(k - 4); }

// In-register DFT of length R (R | 16): X[k] = sum_m x[m] exp(-+ 2 pi i m k / R),
// minus sign for the forward transform, plus for INV.  Radix-2 decimation in
// time by recursion; natural order in and out.
template <int R, bool INV, typename T>
__device__ __forceinline__ void dft_reg(T *re, T *im) {
  if constexpr (R == 2) {
    T ar = re[0], ai = im[0];
    re[0] = ar + re[1]; im[0] = ai + im[1];
    re[1] = ar - re[1]; im[1] = ai - im[1];
  } else if constexpr (R > 2) {
    constexpr int H = R / 2;
    T er[H], ei[H], orr[H], oi[H];
#pragma unroll
    for (int k = 0; k < H; ++k) {
      er[k] = re[2 * k]; ei[k] = im[2 * k];
      orr[k] = re[2 * k + 1]; oi[k] = im[2 * k + 1];
    }
    dft_reg<H, INV, T>(er, ei);
    dft_reg<H, INV, T>(orr, oi);
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const T c = T(cos16(k * (16 / R)));
      const T s = INV ? T(sin16(k * (16 / R))) : T(-sin16(k * (16 / R)));
      const T tr = c * orr[k] - s * oi[k];
      const T ti = c * oi[k] + s * orr[k];
      re[k] = er[k] + tr; im[k] = ei[k] + ti;
      re[k + H] = er[k] - tr; im[k + H] = ei[k] - ti;
    }
  }
}

// Four-step FFT of length N = A * B held in LDS (any element accessor).
// Index x = a B + b, k = k1 + A k2:
//   Z[k1 + A k2] = sum_b W_B^{b k2} ( W_N^{b k1} sum_a z[a B + b] W_A^{a k1} ).
// Step 1 (one call per column b) transforms over a, applies W_N^{b k1} and stores
// back in place at k1 B + b.  Step 2 (one call per k1) transforms over b and
// stores Z[k1 + A k2] in place at k1 B + k2.  Output: Z[k] at (k % A) B + k / A.
template <int A, int B, bool INV, typename T, typename Acc>
__device__ __forceinline__ void fft4_step1(const Acc &acc, int b, const T *tw) {
  T re[A], im[A];
#pragma unroll
  for (int a = 0; a < A; ++a) acc.load(a * B + b, re[a], im[a]);
  dft_reg<A, INV, T>(re, im);
#pragma unroll
  for (int k1 = 0; k1 < A; ++k1) {
    T r = re[k1], i = im[k1];
    if (k1 > 0) {
      const int j = b * k1;
      const T c = tw[2 * j];
      const T s = INV ? -tw[2 * j + 1] : tw[2 * j + 1];
      const T nr = r * c - i * s;
      i = r * s + i * c;
      r = nr;
    }
    acc.store(k1 * B + b, r, i);
  }
}
template <int A, int B, bool INV, typename T, typename Acc>
__device__ __forceinline__ void fft4_step2(const Acc &acc, int k1) {
  T re[B], im[B];
#pragma unroll
  for (int b = 0; b < B; ++b) acc.load(k1 * B + b, re[b], im[b]);
  dft_reg<B, INV, T>(re, im);
#pragma unroll
  for (int k2 = 0; k2 < B; ++k2) acc.store(k1 * B + k2, re[k2], im[k2]);
}

// The same first step storing position k1 B + b at k1 B + (b ^ fft_swz(k1, B)).
// A second step whose items of one transform are consecutive lanes (k1 fast)
// reads its B inputs at k1 B + (b ^ fft_swz(k1, B)): without the swizzle the
// lanes' words are 8 or 16 apart in the same instruction and land on a few
// of the 32 LDS banks.
__device__ __forceinline__ int fft_swz(int k1, int B) { return (k1 >> 1) & (B - 1); }

template <int A, int B, bool INV, typename T, typename Acc>
__device__ __forceinline__ void fft4_step1_swz(const Acc &acc, int b, const T *tw) {
  T re[A], im[A];
#pragma unroll
  for (int a = 0; a < A; ++a) acc.load(a * B + b, re[a], im[a]);
  dft_reg<A, INV, T>(re, im);
#pragma unroll
  for (int k1 = 0; k1 < A; ++k1) {
    T r = re[k1], i = im[k1];
    if (k1 > 0) {
      const int j = b * k1;
      const T c = tw[2 * j];
      const T s = INV ? -tw[2 * j + 1] : tw[2 * j + 1];
      const T nr = r * c - i * s;
      i = r * s + i * c;
      r = nr;
    }
    acc.store(k1 * B + (b ^ fft_swz(k1, B)), r, i);
  }
}

// Factorisation used for each supported length (both factors powers of two;
// the index arithmetic below uses their logarithms, since a division by a
// factor known only at run time would compile to a full integer division).
__host__ __device__ constexpr int fft_A(int n) { return n == 16 ? 4 : n == 32 ? 8 : n == 64 ? 8 : 16; }
__host__ __device__ constexpr int fft_B(int n) { return n == 16 ? 4 : n == 32 ? 4 : n == 64 ? 8 : 8; }
__host__ __device__ constexpr int fft_logA(int n) { return n == 16 ? 2 : n == 32 ? 3 : n == 64 ? 3 : 4; }
__host__ __device__ constexpr int fft_logB(int n) { return n == 16 ? 2 : n == 32 ? 2 : n == 64 ? 3 : 3; }
// Position of output bin k (>= 0) after the four-step transform: (k mod A) B + k / A.
__device__ __forceinline__ int fft_pos(int k, int n) {
  const int la = fft_logA(n), lb = fft_logB(n);
  return ((k & ((1 << la) - 1)) << lb) + (k >> la);
}

// First step with the swizzled store, for one (instance, column) item.
template <bool INV, typename T, typename Acc>
__device__ __forceinline__ void fft4_step1_swz_dispatch(int n, const Acc &acc, int idx, const T *tw) {
  switch (n) {
    case 16: fft4_step1_swz<4, 4, INV, T>(acc, idx, tw); break;
    case 32: fft4_step1_swz<8, 4, INV, T>(acc, idx, tw); break;
    case 64: fft4_step1_swz<8, 8, INV, T>(acc, idx, tw); break;
    default: fft4_step1_swz<16, 8, INV, T>(acc, idx, tw); break;
  }
}

// Run step 1 or 2 of a length-n transform for one (instance, column) item.
template <bool INV, int STEP, typename T, typename Acc>
__device__ __forceinline__ void fft4_dispatch(int n, const Acc &acc, int idx, const T *tw) {
  switch (n) {
    case 16: if (STEP == 1) fft4_step1<4, 4, INV, T>(acc, idx, tw); else fft4_step2<4, 4, INV, T>(acc, idx); break;
    case 32: if (STEP == 1) fft4_step1<8, 4, INV, T>(acc, idx, tw); else fft4_step2<8, 4, INV, T>(acc, idx); break;
    case 64: if (STEP == 1) fft4_step1<8, 8, INV, T>(acc, idx, tw); else fft4_step2<8, 8, INV, T>(acc, idx); break;
    default: if (STEP == 1) fft4_step1<16, 8, INV, T>(acc, idx, tw); else fft4_step2<16, 8, INV, T>(acc, idx); break;
  }
}

// Accessors.  Pair of real rows viewed as one complex row (re in r0, im in r1).
template <typename T>
struct RowPairAcc {
  T *r0, *r1;
  __device__ void load(int i, T &re, T &im) const { re = r0[i]; im = r1[i]; }
  __device__ void store(int i, T re, T im) const { r0[i] = re; r1[i] = im; }
};
// Complex sequence with re and im in two strided arrays: element i is
// (r0[i * stride], r1[i * stride]) -- a pair of real rows (r1 = r0 + pitch,
// stride 1) or an interleaved complex row (r1 = r0 + 1, stride 2).
template <typename T>
struct StridedPairAcc {
  T *r0, *r1;
  int stride;
  __device__ void load(int i, T &re, T &im) const { re = r0[i * stride]; im = r1[i * stride]; }
  __device__ void store(int i, T re, T im) const { r0[i * stride] = re; r1[i * stride] = im; }
};
// Complex column: element i at base[i * stride], interleaved (re, im).
template <typename T>
struct ColAcc {
  T *base;
  int stride;
  __device__ void load(int i, T &re, T &im) const { re = base[i * stride]; im = base[i * stride + 1]; }
  __device__ void store(int i, T re, T im) const { base[i * stride] = re; base[i * stride + 1] = im; }
};

// As fft_batch, with separate accessors for the two steps: step 1 reads
// instance q through make1(q) and stores through it, step 2 reads and writes
// through make2(q).  make1 may read its inputs from elsewhere (the first step
// then runs out of place), as long as its stores land where make2 reads.
template <bool INV, int NT, typename T, typename Make1, typename Make2>
__device__ __forceinline__ void fft_batch2(int n, int count, const T *tw, const Make1 &make1, const Make2 &make2) {
  const int A = fft_A(n), B = fft_B(n), la = fft_logA(n), lb = fft_logB(n);
  for (int it = threadIdx.x; it < count * B; it += NT) {
    const int q = it >> lb, b = it & (B - 1);
    fft4_dispatch<INV, 1, T>(n, make1(q), b, tw);
  }
  __syncthreads();
  for (int it = threadIdx.x; it < count * A; it += NT) {
    const int q = it >> la, k1 = it & (A - 1);
    fft4_dispatch<INV, 2, T>(n, make2(q), k1, tw);
  }
  __syncthreads();
}

// Batched four-step transform over `count` instances of length n; instance q is
// addressed through make(q).  All threads of the block take part.
template <bool INV, int NT, typename T, typename Make>
__device__ __forceinline__ void fft_batch(int n, int count, const T *tw, const Make &make) {
  const int A = fft_A(n), B = fft_B(n), la = fft_logA(n), lb = fft_logB(n);
  for (int it = threadIdx.x; it < count * B; it += NT) {
    const int q = it >> lb, b = it & (B - 1);
    fft4_dispatch<INV, 1, T>(n, make(q), b, tw);
  }
  __syncthreads();
  for (int it = threadIdx.x; it < count * A; it += NT) {
    const int q = it >> la, k1 = it & (A - 1);
    fft4_dispatch<INV, 2, T>(n, make(q), k1, tw);
  }
  __syncthreads();
}

// As fft_batch, with the instance as the fast item index of both steps:
// consecutive lanes take consecutive instances, which suits instances stored
// side by side (the columns of a row-major grid: their elements are adjacent
// words, where a transform's own positions are a whole row apart).
template <bool INV, int NT, typename T, typename Make>
__device__ __forceinline__ void fft_batch_instfast(int n, int count, const T *tw, const Make &make) {
  const int A = fft_A(n), B = fft_B(n);
  for (int it = threadIdx.x; it < count * B; it += NT) {
    const int b = it / count, q = it - b * count;
    fft4_dispatch<INV, 1, T>(n, make(q), b, tw);
  }
  __syncthreads();
  for (int it = threadIdx.x; it < count * A; it += NT) {
    const int k1 = it / count, q = it - k1 * count;
    fft4_dispatch<INV, 2, T>(n, make(q), k1, tw);
  }
  __syncthreads();
}

template <typename T> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };
template <typename T> struct vec4;
template <> struct vec4<float> { using type = float4; };
template <> struct vec4<double> { using type = double4; };

}  // namespace enufft
