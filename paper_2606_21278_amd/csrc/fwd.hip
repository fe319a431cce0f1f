// Batched type-1 NUFFT on gfx950: spread -> fold -> FFT -> deconvolve -> crop,
// one fine grid per workgroup, resident in LDS from the first atomic add to
// the last coefficient written.
//
// Section 2.1.2 of the paper: Step 1 spreads every sample onto an oversampled
// periodic grid with a compact kernel (eq. spreading, here the exponential of a
// semicircle); Step 2's quadrature weight is folded into the per-point
// strength c_j = w_j W(x_j) h_j; Step 3 is the 2D FFT; Step 4 divides by the
// kernel's Fourier transform (eq. deconv) and the result is truncated to the
// mode box.
#include <climits>

#include "device_common.h"
#include "launch.h"

namespace enufft {

// Row pitch of the LDS grid: P > 0 is known at compile time (immediate LDS
// offsets for the rows of a footprint), P <= 0 reads it from the geometry.
// P != 0 builds evaluate the kernel polynomial without a run-time switch (the
// switch made the compiler keep the taps in scratch memory).
template <int P>
__device__ __forceinline__ int grid_pitch(const Geom &g) {
  return P > 0 ? P : g.pitch;
}

// Waves per SIMD the register allocation must allow: an FP32 grid of the
// 128-wide fine grid takes about 70 KB, so two 512-thread workgroups share a
// CU when each wave stays within 128 VGPRs.
template <typename A, int NT>
constexpr int fwd_min_waves() {
  return (sizeof(A) == 4 && NT == 512) ? 4 : 1;
}

// Kernel values along one axis.  The P != 0 builds are launched only when the
// plan carries the kernel polynomial, so they evaluate it directly.
template <typename T, int W, int P>
__device__ __forceinline__ void taps(const FwdArgs<T> &a, const FineCoord<T> &c, T (&out)[W]) {
  if constexpr (P != 0 && sizeof(T) == 4 && W <= ES_MAXW)
    es_taps_poly<W>(c, float(W) * 0.5f, a.es, out);
  else
    es_taps<T, W>(c, a.beta, a.es, out);
}

// Add one point's W x W contributions to the grid, whose cells accumulate in A
// (FP32 or FP64; FP64 plans always use FP64).  Stored row r holds fine row
// r mod n2 (rows n2 .. n2 + W - 1 are folded back afterwards); columns wrap
// with the grid mask.
template <typename T, typename A, int W, int P>
__device__ __forceinline__ void spread_point(const FwdArgs<T> &a, A *grid, T c, const FineCoord<T> &fx,
                                             const FineCoord<T> &fy) {
  const Geom &g = a.g;
  const int pitch = grid_pitch<P>(g);
  T tx[W], ty[W];
  taps<T, W, P>(a, fx, tx);
  taps<T, W, P>(a, fy, ty);
  A kx[W], ky[W];
#pragma unroll
  for (int d = 0; d < W; ++d) {
    kx[d] = (A)tx[d];
    ky[d] = (A)(c * ty[d]);
  }
  int col[W];
#pragma unroll
  for (int d = 0; d < W; ++d) col[d] = (fx.i0 + d) & (g.n1 - 1);
  A *rowp = grid + (fy.i0 & (g.n2 - 1)) * pitch;
#pragma unroll
  for (int dy = 0; dy < W; ++dy) {
#pragma unroll
    for (int dx = 0; dx < W; ++dx) {
      __hip_atomic_fetch_add(rowp + dy * pitch + col[dx], ky[dy] * kx[dx], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
}

// Runs of consecutive points.  Each thread takes K = 4 consecutive points (one
// 16-byte load per array).  When their footprints start within two rows and
// three columns of each other -- the usual case for points stored in raster
// order, several per fine-grid cell -- their contributions are summed over a
// (W + 1) x (W + 2) window in registers and each window cell is added to the
// grid once, which cuts the LDS atomics per point and spreads neighbouring
// lanes apart.
// Groups that do not fit one window are deferred by the caller.
constexpr int RUN_K = 4, RUN_SX = 2, RUN_SY = 1;

// Geometry of one group: the in-cell offsets v = i0 - t + W/2 (all the taps
// need), each point's shift against the window origin and the window origin.
//
// A lane with rev set walks its window's columns from the last to the first
// (see spread_item).  It takes the x taps mirrored, which for the even kernel
// is the same as evaluating them at 1 - v, and counts its column shifts from
// the window's far edge, so the column loop below is the same for every lane.
struct RunGeom {
  int sx[RUN_K], sy[RUN_K];
  float vx[RUN_K], vy[RUN_K];
  int cmin, rmin;
  int cspan, rspan;   // spread of the footprint origins (columns, rows)
  bool fits, any;
};

template <typename T, int W>
__device__ __forceinline__ RunGeom run_geom(const FwdArgs<T> &a, const float (&xs)[RUN_K], const float (&ys)[RUN_K],
                                            const float (&cs)[RUN_K], bool rev) {
  const float halfw = float(W) / 2.0f;
  RunGeom rg;
  int ix[RUN_K], iy[RUN_K];
  int cmax = INT_MIN, rmax = INT_MIN;
  rg.cmin = INT_MAX; rg.rmin = INT_MAX;
#pragma unroll
  for (int k = 0; k < RUN_K; ++k) {
    const FineCoord<float> fx = fine_coord<float>(xs[k], a.s1_hi, a.s1_lo, halfw);
    const FineCoord<float> fy = fine_coord<float>(ys[k], a.s2_hi, a.s2_lo, halfw);
    ix[k] = fx.i0; iy[k] = fy.i0;
    const float vx = tap_v(fx, halfw);
    rg.vx[k] = rev ? 1.0f - vx : vx;
    rg.vy[k] = tap_v(fy, halfw);
    if (cs[k] != 0.0f) {
      rg.cmin = min(rg.cmin, ix[k]); cmax = max(cmax, ix[k]);
      rg.rmin = min(rg.rmin, iy[k]); rmax = max(rmax, iy[k]);
    }
  }
  rg.any = rg.rmin != INT_MAX;   // some point inside the cell window
  rg.fits = !rg.any || (cmax - rg.cmin <= RUN_SX && rmax - rg.rmin <= RUN_SY);
  rg.cspan = cmax - rg.cmin;
  rg.rspan = rmax - rg.rmin;
#pragma unroll
  for (int k = 0; k < RUN_K; ++k) {
    // points with c = 0 may lie anywhere: their shifts then match no column
    // and they add nothing
    const int d = ix[k] - rg.cmin;
    rg.sx[k] = rev ? RUN_SX - d : d;
    rg.sy[k] = iy[k] - rg.rmin;
  }
  return rg;
}

// Spread one fitting group: the (W + RUN_SY) x (W + RUN_SX) window of the
// summed footprints goes to the grid one column at a time.  Each column is
// formed in registers from the four points' taps (every point enters,
// branch-free: one with c = 0 contributes exact zeros, and its taps stay finite
// because the offsets are clamped to the kernel's interval) and added with
// one LDS atomic per row, so the adds of a column overlap the arithmetic of
// the next.  With rev the columns go out from the last to the first, so two
// lanes whose windows start at the same cell never add to one address in the
// same instruction.
template <typename T, typename A, int W, int P>
__device__ __forceinline__ void run_spread(const FwdArgs<T> &a, A *grid, const RunGeom &rg,
                                           const float (&cs)[RUN_K], bool rev) {
  constexpr int WC = W + RUN_SX, WR = W + RUN_SY;
  const Geom &g = a.g;
  float kx[RUN_K][W], KY[RUN_K][WR];
#pragma unroll
  for (int k = 0; k < RUN_K; ++k) {
    float ky[W];
    if constexpr (P != 0) {
      es_taps_poly_v<W>(rg.vx[k], a.es, kx[k]);
      es_taps_poly_v<W>(rg.vy[k], a.es, ky);
    } else if (a.es.on) {
      es_taps_poly_v<W>(rg.vx[k], a.es, kx[k]);
      es_taps_poly_v<W>(rg.vy[k], a.es, ky);
    } else {
      es_taps_exact_v<W>(rg.vx[k], a.beta, kx[k]);
      es_taps_exact_v<W>(rg.vy[k], a.beta, ky);
    }
#pragma unroll
    for (int r = 0; r < WR; ++r) {
      float v = 0.0f;
#pragma unroll
      for (int s = 0; s <= RUN_SY; ++s)
        if (r - s >= 0 && r - s < W) v = (rg.sy[k] == s) ? ky[r - s] : v;
      KY[k][r] = v * cs[k];
    }
  }
  const int pitch = grid_pitch<P>(g);
  A *rowp = grid + (rg.rmin & (g.n2 - 1)) * pitch;
  const int c0 = rev ? rg.cmin + WC - 1 : rg.cmin;
  // The column step, tied to this group's origin by an empty asm statement so
  // the compiler forms dc j per group instead of holding the products live
  // across the point loop (where they had been spilled, and each reload waited
  // for the next block's loads).
  int dc = rev ? -1 : 1;
  asm("" : "+v"(dc) : "v"(rg.cmin));
#pragma unroll
  for (int j = 0; j < WC; ++j) {
    float col[WR];
#pragma unroll
    for (int k = 0; k < RUN_K; ++k) {
      float xv = 0.0f;
#pragma unroll
      for (int s = 0; s <= RUN_SX; ++s)
        if (j - s >= 0 && j - s < W) xv = (rg.sx[k] == s) ? kx[k][j - s] : xv;
#pragma unroll
      for (int r = 0; r < WR; ++r) col[r] = (k == 0) ? KY[k][r] * xv : fmaf(KY[k][r], xv, col[r]);
    }
    A *cp = rowp + ((c0 + dc * j) & (g.n1 - 1));
    // window cells outside the footprints' bounding box hold exact zeros: their
    // lanes skip the add (fewer lanes per LDS atomic)
    const bool cact = rev ? (j >= RUN_SX - rg.cspan) : (j < W + rg.cspan);
    if (cact) {
#pragma unroll
      for (int r = 0; r < W; ++r)
        __hip_atomic_fetch_add(cp + r * pitch, (A)col[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
      for (int r = W; r < WR; ++r)
        if (r < W + rg.rspan)
          __hip_atomic_fetch_add(cp + r * pitch, (A)col[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
}

// Orders this wave's LDS accesses around the deferred-group queue (LDS
// operations of one wave complete in issue order; this keeps the compiler
// from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Spread the deferred groups queue[0 .. n) of this wave, one group per lane,
// point by point.  Entries are group offsets from g0 (groups of RUN_K points).
template <typename T, typename A, int W, int P>
__device__ __forceinline__ void drain_groups(const FwdArgs<T> &a, A *grid, const int *queue, int n,
                                             int64_t g0, T cx, T cy, T R, T pr) {
  using V = typename vec4<T>::type;
  const int lane = threadIdx.x & 63;
  if (lane >= n) return;
  const int64_t q = g0 + queue[lane];
  const V xv = reinterpret_cast<const V *>(a.x)[q], yv = reinterpret_cast<const V *>(a.y)[q];
  const V hv = reinterpret_cast<const V *>(a.h)[q], wv = reinterpret_cast<const V *>(a.w)[q];
  const T xs[RUN_K] = {xv.x, xv.y, xv.z, xv.w}, ys[RUN_K] = {yv.x, yv.y, yv.z, yv.w};
  const T hs[RUN_K] = {hv.x, hv.y, hv.z, hv.w}, ws[RUN_K] = {wv.x, wv.y, wv.z, wv.w};
  const T halfw = T(W) / T(2);
  // one copy of the per-point code (instruction-cache footprint of the loop)
#pragma unroll 1
  for (int k = 0; k < RUN_K; ++k) {
    const T xk = k == 0 ? xs[0] : k == 1 ? xs[1] : k == 2 ? xs[2] : xs[3];
    const T yk = k == 0 ? ys[0] : k == 1 ? ys[1] : k == 2 ? ys[2] : ys[3];
    const T hk = k == 0 ? hs[0] : k == 1 ? hs[1] : k == 2 ? hs[2] : hs[3];
    const T wk = k == 0 ? ws[0] : k == 1 ? ws[1] : k == 2 ? ws[2] : ws[3];
    const T c = wk * hk * hann_w(a.window_kind, xk, yk, cx, cy, R, pr);
    if (c != T(0))
      spread_point<T, A, W, P>(a, grid, c, fine_coord<T>(xk, a.s1_hi, a.s1_lo, halfw),
                               fine_coord<T>(yk, a.s2_hi, a.s2_lo, halfw));
  }
}

// Spread the points [begin, end) of one item into the LDS grid.
template <typename T, typename A, int W, int NT, int P>
__device__ __forceinline__ void spread_item(const FwdArgs<T> &a, A *grid, int *queue, int64_t begin,
                                            int64_t end, T cx, T cy, T R) {
  const T halfw = T(W) / T(2);
  const T pr = R > T(0) ? T(M_PI) / R : T(0);
  int64_t body0 = end, body1 = end;
  // runs need 16-byte aligned arrays; the register window is sized for FP32 and W <= 6
  constexpr bool kRuns = sizeof(T) == 4 && W <= 6;
  if (kRuns && a.vec4) {
    body0 = min(end, (begin + RUN_K - 1) / RUN_K * RUN_K);
    body1 = max(body0, end / RUN_K * RUN_K);
  }
  using V = typename vec4<T>::type;
  const V *x4 = reinterpret_cast<const V *>(a.x), *y4 = reinterpret_cast<const V *>(a.y);
  const V *h4 = reinterpret_cast<const V *>(a.h), *w4 = reinterpret_cast<const V *>(a.w);
  if constexpr (kRuns) {
    // Group-to-lane map: in each block of NT consecutive groups, wave w takes
    // the 64 groups w 64 .. w 64 + 63 and lane l the group 2 (l mod 32) + l / 32.
    // Each wave load reads 1 KiB contiguous (whole cache lines, no re-fetch).
    // Lanes l and l + 1 hold groups 2 runs apart: for raster-ordered points
    // their windows start a few cells apart, at different grid cells (LDS
    // atomics on one address serialise) but on nearby banks, and the
    // neighbouring groups of lanes l and l + 32 flush in opposite orders.
    // (Measured on C3 against lanes 1, 4, 8 and 16 groups apart: 2 was
    // fastest, 8.9 ms against 9.3, 9.2, 9.7 and 9.8.)
    //
    // Groups that do not fit one window (a raster row ends inside the group,
    // or the points are unordered) are queued per wave and spread point by
    // point 64 at a time, so the rare misfit does not stall the other 63 lanes.
    const int lane = threadIdx.x & 63;
    const int lane_off = (threadIdx.x >> 6) * 64 + ((lane & 31) << 1) + (lane >> 5);
    const bool rev = (lane >> 5) & 1;
    const int64_t g0 = body0 / RUN_K, q1 = body1 / RUN_K;
    int64_t q = g0 + lane_off;
    int nq = 0;   // queued groups (the same in every lane)
    // With 512 threads, loads run two blocks ahead in three register buffers
    // (the loop is unrolled by three so no buffer is copied and the compiler
    // waits only for the block about to be used): with one workgroup per CU,
    // this is what keeps enough HBM requests in flight.
    // Loads are unconditional (control flow around them makes the compiler
    // wait for every load in flight); past the end they re-read the last group.
    auto load = [&](V &xb, V &yb, V &hb, V &wb, int64_t qq) {
      const int64_t qc = qq < q1 ? qq : q1 - 1;
      xb = x4[qc]; yb = y4[qc]; hb = h4[qc]; wb = w4[qc];
    };
    auto step = [&](const V &xv, const V &yv, const V &hv, const V &wv, int64_t qq) {
      const bool live = qq < q1;
      const float xs[RUN_K] = {xv.x, xv.y, xv.z, xv.w}, ys[RUN_K] = {yv.x, yv.y, yv.z, yv.w};
      float cs[RUN_K];
#pragma unroll
      for (int k = 0; k < RUN_K; ++k)
        cs[k] = live ? (&wv.x)[k] * (&hv.x)[k] * hann_w(a.window_kind, xs[k], ys[k], cx, cy, R, pr) : 0.0f;
      const RunGeom rg = run_geom<T, W>(a, xs, ys, cs, rev);
      const bool defer = live && !rg.fits;
      if (live && rg.any && rg.fits) run_spread<T, A, W, P>(a, grid, rg, cs, rev);
      const uint64_t m = __ballot(defer);
      if (m != 0) {
        if (defer) {
          const int pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
          queue[nq + pos] = (int)(qq - g0);   // nq < 64 here, so nq + pos < FWD_QCAP
        }
        nq += __popcll(m);
        if (nq >= 64) {
          wave_lds_sync();
          drain_groups<T, A, W, P>(a, grid, queue, 64, g0, cx, cy, R, pr);
          nq -= 64;
          const int rest = lane < nq ? queue[64 + lane] : 0;
          wave_lds_sync();
          if (lane < nq) queue[lane] = rest;
          wave_lds_sync();
        }
      }
    };
    V x0{}, y0{}, h0{}, w0{}, x1{}, y1{}, h1{}, w1{};
    if constexpr (NT * fwd_min_waves<A, NT>() >= 1024 || NT >= 1024) {
      // four waves per SIMD hide the load latency with one block in flight
      if (q1 > g0) load(x0, y0, h0, w0, q);
      for (int64_t qb = g0; qb < q1; qb += 2 * NT, q += 2 * NT) {
        load(x1, y1, h1, w1, q + NT);
        step(x0, y0, h0, w0, q);
        load(x0, y0, h0, w0, q + 2 * NT);
        step(x1, y1, h1, w1, q + NT);
      }
    } else {
      V x2{}, y2{}, h2{}, w2{};
      if (q1 > g0) {
        load(x0, y0, h0, w0, q);
        load(x1, y1, h1, w1, q + NT);
      }
      for (int64_t qb = g0; qb < q1; qb += 3 * NT, q += 3 * NT) {
        load(x2, y2, h2, w2, q + 2 * NT);
        step(x0, y0, h0, w0, q);
        load(x0, y0, h0, w0, q + 3 * NT);
        step(x1, y1, h1, w1, q + NT);
        load(x1, y1, h1, w1, q + 4 * NT);
        step(x2, y2, h2, w2, q + 2 * NT);
      }
    }
    if (nq > 0) {
      wave_lds_sync();
      drain_groups<T, A, W, P>(a, grid, queue, nq, g0, cx, cy, R, pr);
    }
  }
  // points outside the aligned body, one per thread
  const int64_t nhead = body0 - begin, ntail = end - body1;
  for (int64_t i = threadIdx.x; i < nhead + ntail; i += NT) {
    const int64_t j = i < nhead ? begin + i : body1 + (i - nhead);
    const T xj = a.x[j], yj = a.y[j];
    const T c = a.w[j] * a.h[j] * hann_w(a.window_kind, xj, yj, cx, cy, R, pr);
    if (c == T(0)) continue;
    spread_point<T, A, W, P>(a, grid, c, fine_coord<T>(xj, a.s1_hi, a.s1_lo, halfw),
                             fine_coord<T>(yj, a.s2_hi, a.s2_lo, halfw));
  }
}

// Fold stored rows n2 .. n2 + W - 1 onto rows 0 .. W - 1.
template <typename A, int W, int NT>
__device__ __forceinline__ void fold_rows(A *grid, const Geom &g) {
  const int pitch = g.pitch;
  for (int i = threadIdx.x; i < W * g.n1; i += NT) {
    const int r = i / g.n1, c = i - r * g.n1;
    grid[r * pitch + c] += grid[(r + g.n2) * pitch + c];
  }
  __syncthreads();
}

// Round the FP64 grid (n2 rows of `pitch`) to T in place: element i moves from
// byte 8 i to byte sizeof(T) i.  Each round reads a block before any thread
// writes it, and a write of round k lands on bytes read in rounds <= k.
// Nothing to do when the grid already accumulates in T.
template <typename T, typename A, int NT>
__device__ __forceinline__ void grid_to_t(A *grid, const Geom &g) {
  if constexpr (sizeof(T) == sizeof(A)) {
    return;
  } else {
    constexpr int PER = 8;
    const int total = g.n2 * g.pitch;
    T *out = reinterpret_cast<T *>(grid);
    for (int base = 0; base < total; base += PER * NT) {
      double v[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int i = base + q * NT + threadIdx.x;
        v[q] = i < total ? grid[i] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int i = base + q * NT + threadIdx.x;
        if (i < total) out[i] = (T)v[q];
      }
      __syncthreads();
    }
  }
}

// Second step of the row-pair transforms with the unpacking of the two real
// rows' spectra fused in.  Z = FFT(row 2p + i row 2p+1); A(k) = (Z(k) + conj
// Z(-k)) / 2 is row 2p's spectrum and B(k) = (Z(k) - conj Z(-k)) / 2i is row
// 2p+1's.  Item k1 computes Z(k1 + A k2) and (1) stores it in transform order,
// (2) reads the partners Z(-k) of its bins k <= K1, (3) writes A(k) and B(k)
// to elements 2k, 2k+1 of the two rows.  Steps (2) and (3) touch positions of
// other items of the same row pair, so those items must be one wave's lanes:
// a wave's LDS accesses complete in issue order, and every lane finishes each
// step before any lane starts the next.  With A | 64 and 64 | NT, the items
// q A .. q A + A - 1 of the loop below always share a wave.
template <int A, int B, typename T>
__device__ __forceinline__ void row_step2_unpack(const RowPairAcc<T> &acc, int k1, int n, int K1) {
  T re[B], im[B];
  const int sw = fft_swz(k1, B);   // the first step stored with fft4_step1_swz
#pragma unroll
  for (int b = 0; b < B; ++b) acc.load(k1 * B + (b ^ sw), re[b], im[b]);
  dft_reg<B, false, T>(re, im);
#pragma unroll
  for (int k2 = 0; k2 < B; ++k2) acc.store(k1 * B + k2, re[k2], im[k2]);
  T mr[B], mi[B];
#pragma unroll
  for (int k2 = 0; k2 < B; ++k2) {
    const int k = k1 + A * k2;
    mr[k2] = T(0);
    mi[k2] = T(0);
    if (k <= K1) acc.load(fft_pos((n - k) & (n - 1), n), mr[k2], mi[k2]);
  }
#pragma unroll
  for (int k2 = 0; k2 < B; ++k2) {
    const int k = k1 + A * k2;
    if (k <= K1) {
      acc.r0[2 * k] = T(0.5) * (re[k2] + mr[k2]);
      acc.r0[2 * k + 1] = T(0.5) * (im[k2] - mi[k2]);
      acc.r1[2 * k] = T(0.5) * (im[k2] + mi[k2]);
      acc.r1[2 * k + 1] = T(-0.5) * (re[k2] - mr[k2]);
    }
  }
}

// The row stage: forward transforms of the row pairs, unpacked in their
// second step (see above).
template <int NT, typename T, typename Make>
__device__ __forceinline__ void row_fft_unpack(int n, int count, const T *tw, int K1, const Make &make) {
  static_assert(NT % 64 == 0, "whole waves");
  const int A = fft_A(n), B = fft_B(n), la = fft_logA(n), lb = fft_logB(n);
  for (int it = threadIdx.x; it < count * B; it += NT) {
    const int q = it >> lb, b = it & (B - 1);
    fft4_step1_swz_dispatch<false, T>(n, make(q), b, tw);
  }
  __syncthreads();
  for (int it = threadIdx.x; it < count * A; it += NT) {
    const int q = it >> la, k1 = it & (A - 1);
    switch (n) {
      case 16: row_step2_unpack<4, 4, T>(make(q), k1, n, K1); break;
      case 32: row_step2_unpack<8, 4, T>(make(q), k1, n, K1); break;
      case 64: row_step2_unpack<8, 8, T>(make(q), k1, n, K1); break;
      default: row_step2_unpack<16, 8, T>(make(q), k1, n, K1); break;
    }
  }
  __syncthreads();
}

// FFT of the folded real grid G (logical row 0 at G), deconvolution and crop.
// Row stage: rows are transformed two at a time as one complex row; the
// needed bins kx = 0..K1 of each real row are unpacked in place into the
// first 2 (K1 + 1) elements of that row.  Column stage: complex transforms
// along y of those columns.  Output: bins (kx, ky), kx in [0, K1], |ky| <= K2;
// the box's negative-kx modes come from Hermitian symmetry of the real grid.
template <typename T, int NT>
__device__ void fft_deconv_store(const FwdArgs<T> &a, T *G, int cell) {
  const Geom &g = a.g;
  const int pitch = g.pitch;
  const int n1 = g.n1, n2 = g.n2;
  const int npairs = n2 / 2;
  row_fft_unpack<NT, T>(n1, npairs, a.tw1, g.K1, [&](int q) {
    RowPairAcc<T> acc;
    acc.r0 = G + (2 * q) * pitch;
    acc.r1 = acc.r0 + pitch;
    return acc;
  });
  const int per = g.K1 + 1;
  fft_batch_instfast<false, NT, T>(n2, per, a.tw2, [&](int q) {
    ColAcc<T> acc;
    acc.base = G + 2 * q;
    acc.stride = pitch;
    return acc;
  });
  // Deconvolve (real, even factor) and write the mode box.
  using C = typename vec2<T>::type;
  C *fout = reinterpret_cast<C *>(a.f) + (int64_t)cell * g.N1 * g.N2;
  const int hi1 = g.lo1 + g.N1 - 1, hi2 = g.lo2 + g.N2 - 1;
  // Items in rounds of U per thread, with the factors' loads of a round issued
  // before its stores (the stores could alias the factor tables as far as the
  // compiler knows, so a store between loads would serialise them).
  const int nky = 2 * g.K2 + 1, nit = nky * per;
  constexpr int U = 4;
  for (int it0 = threadIdx.x; it0 < nit; it0 += U * NT) {
    int kx[U], ky[U];
    T s[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int it = min(it0 + u * NT, nit - 1);
      const int kyi = it / per;
      kx[u] = it - kyi * per;
      ky[u] = kyi - g.K2;
      s[u] = a.decon_x[kx[u]] * a.decon_y[ky[u] < 0 ? -ky[u] : ky[u]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (it0 + u * NT >= nit) break;
      const int pos = fft_pos(ky[u] & (n2 - 1), n2);
      const T vr = G[pos * pitch + 2 * kx[u]] * s[u], vi = G[pos * pitch + 2 * kx[u] + 1] * s[u];
      if (kx[u] <= hi1 && ky[u] >= g.lo2 && ky[u] <= hi2) {
        C v; v.x = vr; v.y = vi;
        fout[(ky[u] - g.lo2) * g.N1 + (kx[u] - g.lo1)] = v;
      }
      if (kx[u] >= 1 && -kx[u] >= g.lo1 && -ky[u] >= g.lo2 && -ky[u] <= hi2) {
        C v; v.x = vr; v.y = -vi;
        fout[(-ky[u] - g.lo2) * g.N1 + (-kx[u] - g.lo1)] = v;
      }
    }
  }
}

template <typename T, typename A, int W, int NT, int P>
__global__ __launch_bounds__(NT, (fwd_min_waves<A, NT>())) void fwd_kernel(FwdArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  A *grid = reinterpret_cast<A *>(smem_raw);
  int *queue = reinterpret_cast<int *>(smem_raw + fwd_grid_bytes(a.g, W, sizeof(A))) + (threadIdx.x >> 6) * FWD_QCAP;
  T *G = reinterpret_cast<T *>(smem_raw);   // the same grid after rounding to T
  __shared__ int s_item, s_last;
  const Geom &g = a.g;
  const int pitch = g.pitch;
  const int total = (g.n2 + W) * pitch;
  const bool persistent = a.work_counter != nullptr;
  int64_t idx = a.item_base + blockIdx.x;
  if (!persistent && idx >= a.n_items) return;
  for (;;) {
    if (persistent) {
      if (threadIdx.x == 0) s_item = atomicAdd(a.work_counter, 1);
      __syncthreads();
      idx = s_item;
      __syncthreads();
      if (idx >= a.n_items) break;
    }
    const FwdItem it = a.items[idx];
    for (int i = threadIdx.x; i < total; i += NT) grid[i] = A(0);
    __syncthreads();
    const double *wn = a.windows + 3 * (int64_t)it.cell;
    spread_item<T, A, W, NT, P>(a, grid, queue, it.begin, it.end, T(wn[0]), T(wn[1]), T(wn[2]));
    __syncthreads();
    fold_rows<A, W, NT>(grid, g);
    grid_to_t<T, A, NT>(grid, g);
    bool run_fft = true;
    if (it.nchunks > 1) {
      const int nn = g.n1 * g.n2;
      T *slot = a.partial + (int64_t)it.slot * nn;
      for (int i = threadIdx.x; i < nn; i += NT) {
        const int r = i / g.n1, c = i - r * g.n1;
        slot[i] = G[r * pitch + c];
      }
      __threadfence();
      __syncthreads();
      if (threadIdx.x == 0) {
        const int old = atomicAdd(a.cell_counters + it.cell, 1);
        s_last = (old == it.nchunks - 1);
        if (s_last) a.cell_counters[it.cell] = 0;   // ready for the next call
      }
      __syncthreads();
      run_fft = s_last != 0;
      if (run_fft) {
        __threadfence();
        // the chunks' grids summed in chunk order (the same order whichever chunk
        // finishes last); this chunk's own grid is still in LDS.  Each thread
        // takes MV cells at a time with two chunks' loads in flight (one load at
        // a time had cost a memory latency per cell and chunk on the critical
        // path of every split cell).
        constexpr int MV = 8;
        const T *p0 = a.partial + (int64_t)it.slot0 * nn;
        const int own = it.slot - it.slot0;
        // (each thread reads and then writes only its own cells of G)
        for (int i0 = threadIdx.x; i0 < nn; i0 += MV * NT) {
          int li[MV];
          bool in[MV];
          T sum[MV];
#pragma unroll
          for (int v = 0; v < MV; ++v) {
            in[v] = i0 + v * NT < nn;
            const int i = in[v] ? i0 + v * NT : i0;
            const int r = i / g.n1, c = i - r * g.n1;
            li[v] = r * pitch + c;
            sum[v] = T(0);
          }
          for (int q = 0; q < it.nchunks; q += 2) {
            const bool two = q + 1 < it.nchunks;
            T t0[MV], t1[MV];
#pragma unroll
            for (int v = 0; v < MV; ++v) {
              const int i = in[v] ? i0 + v * NT : i0;
              t0[v] = q == own ? G[li[v]] : p0[(int64_t)q * nn + i];
              t1[v] = !two ? T(0) : (q + 1 == own ? G[li[v]] : p0[(int64_t)(q + 1) * nn + i]);
            }
#pragma unroll
            for (int v = 0; v < MV; ++v) {
              sum[v] += t0[v];
              if (two) sum[v] += t1[v];
            }
          }
#pragma unroll
          for (int v = 0; v < MV; ++v)
            if (in[v]) G[li[v]] = sum[v];
        }
        __syncthreads();
      }
    }
    if (run_fft) fft_deconv_store<T, NT>(a, G, it.cell);
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

// The compiled variants: FP32 with the kernel polynomial (W <= 8) also has
// polynomial builds, one with the constant pitch of the 128-wide grid and one
// for any pitch, used when the plan carries the polynomial; those builds come
// with an FP64 and an FP32 LDS grid (acc = 8 or 4 bytes per cell).
template <typename T, int W>
constexpr bool has_pitch128() {
  return sizeof(T) == 4 && W <= ES_MAXW;
}

template <typename T, typename A, int W, int P>
static const void *fwd_fn_threads(int threads) {
  if (threads == 256) return (const void *)&fwd_kernel<T, A, W, 256, P>;
  if (threads == 512) return (const void *)&fwd_kernel<T, A, W, 512, P>;
  return (const void *)&fwd_kernel<T, A, W, 1024, P>;
}

template <typename T, int W>
static const void *fwd_fn(int threads, int pitch, int acc) {
  if constexpr (has_pitch128<T, W>()) {
    if (pitch == FWD_PITCH128)
      return acc == 4 ? fwd_fn_threads<T, float, W, FWD_PITCH128>(threads)
                      : fwd_fn_threads<T, double, W, FWD_PITCH128>(threads);
    if (pitch == FWD_POLY_ANY)
      return acc == 4 ? fwd_fn_threads<T, float, W, FWD_POLY_ANY>(threads)
                      : fwd_fn_threads<T, double, W, FWD_POLY_ANY>(threads);
  }
  if (acc != 8) return nullptr;
  return fwd_fn_threads<T, double, W, 0>(threads);
}

template <typename T>
static const void *fwd_fn_w(int W, int threads, int pitch, int acc) {
  switch (W) {
    case 4: return fwd_fn<T, 4>(threads, pitch, acc);
    case 6: return fwd_fn<T, 6>(threads, pitch, acc);
    case 8: return fwd_fn<T, 8>(threads, pitch, acc);
    case 10: return fwd_fn<T, 10>(threads, pitch, acc);
    case 12: return fwd_fn<T, 12>(threads, pitch, acc);
    case 14: return fwd_fn<T, 14>(threads, pitch, acc);
    case 16: return fwd_fn<T, 16>(threads, pitch, acc);
    default: return nullptr;
  }
}

template <typename T>
hipError_t launch_fwd(const FwdArgs<T> &a, int W, int blocks, int threads, size_t lds, hipStream_t s) {
  if (threads != 256 && threads != 512 && threads != 1024) return hipErrorInvalidValue;
  const void *fn = fwd_fn_w<T>(W, threads, fwd_variant_pitch(a.g, a.es), a.acc);
  if (!fn) return hipErrorInvalidValue;
  void *args[] = {const_cast<FwdArgs<T> *>(&a)};
  return hipLaunchKernel(fn, dim3(blocks), dim3(threads), args, lds, s);
}

template <typename T>
hipError_t fwd_occupancy(int W, int threads, int pitch, int acc, size_t lds, int *blocks_per_cu) {
  if (threads != 256 && threads != 512 && threads != 1024) return hipErrorInvalidValue;
  const void *fn = fwd_fn_w<T>(W, threads, pitch, acc);
  if (!fn) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, threads, lds);
}

template hipError_t launch_fwd<float>(const FwdArgs<float> &, int, int, int, size_t, hipStream_t);
template hipError_t launch_fwd<double>(const FwdArgs<double> &, int, int, int, size_t, hipStream_t);
template hipError_t fwd_occupancy<float>(int, int, int, int, size_t, int *);
template hipError_t fwd_occupancy<double>(int, int, int, int, size_t, int *);

}  // namespace enufft
