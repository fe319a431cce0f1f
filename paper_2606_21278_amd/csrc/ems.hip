// Elastic Mode Selection on gfx950: one workgroup per cell; the unit energies
// are sorted in registers per wave and merged through LDS.
//
// Section 2.2 of the paper, in its order: unit energies (eq. energy, with the
// optional weight of eq. weighted_e), the descending order of eq.
// sorted_energy, the participation ratio (eq. n_eff), the gap-ratio score
// (eq. s_delta), the combined measure and target fraction (eqs. c_score,
// alpha_c), the retained fraction (eq. f_cum) and the elastic count
// (eq. k_elastic).  Energies, sums, the running sum and the threshold test are
// FP64 so the ordering and the cut do not depend on FP32 rounding of the sums.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <string>
#include <vector>

#include "device_common.h"
#include "launch.h"
#include "plan.h"

namespace enufft {

struct EmsArgs {
  const void *f;
  const double *mode_weight;
  const double *flow;         // flow mode: [n_steps * n_cells_f][6] records (ux, uy, N, fc, rho, kscale)
  int64_t n_cells_f;          // flow mode: cells per step (the coefficients of cell v mod n_cells_f)
  uint8_t *keep;
  int32_t *k_star;
  double *stats;
  const int2 *units;          // (rep, partner | -1), ascending unit id
  const int4 *mode_unit;      // [M]: (rep, partner | -1, unit id, 0) of each mode's unit; rep -1: no unit
  int J;
  int M;                      // modes per cell = N1 * N2
  int N1, N2;                 // mode box (row-major, N1 modes per row)
  int64_t cell_begin, cell_end;
  int k_min, k_max;
  double alpha_min, alpha_max, delta, w1, w2;
};

// One wave per cell.  Wave-wide helpers: every lane returns the same value.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
// Exclusive prefix over lanes (Hillis-Steele on the wave).
template <typename V>
__device__ __forceinline__ V wave_exclusive_scan(V v, int lane) {
  V inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const V t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  return inc - v;
}

// max / min of two energies.  The values are finite and never signalling
// NaNs, so the plain instructions do (the generic fmax would first quiet both
// operands).
__device__ __forceinline__ double dmax(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double dmin(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Descending bitonic sort of the wave's JP = 64 R values held blocked (lane l
// holds positions l R .. l R + R - 1), in the flip form: for each block size
// k a flip comparator (i against i ^ (k - 1)) then half-cleaners j = k/4 .. 1;
// the lower index of every pair takes the larger value, so no direction bits.
// Pairs inside a lane are register compare-exchanges; pairs across lanes
// exchange through cross-lane shuffles.  Stages are template-expanded so every
// register index is a constant.
template <int R, int K>
__device__ __forceinline__ void flip_stage(double (&e)[R], int lane) {
  if constexpr (K <= R) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = r ^ (K - 1);
      if (r < q) {
        const double hi = dmax(e[r], e[q]), lo = dmin(e[r], e[q]);
        e[r] = hi; e[q] = lo;
      }
    }
  } else {
    constexpr int lm = K / R - 1;
    const bool lower = (lane & (K / (2 * R))) == 0;
#pragma unroll
    for (int r = 0; r < (R + 1) / 2; ++r) {
      const int q = R - 1 - r;
      const double o1 = __shfl_xor(e[q], lm, 64);   // partner of my r is the partner lane's q
      if (q != r) {
        const double o2 = __shfl_xor(e[r], lm, 64);
        const double h2 = dmax(e[q], o2), l2 = dmin(e[q], o2);
        e[q] = lower ? h2 : l2;
      }
      const double h1 = dmax(e[r], o1), l1 = dmin(e[r], o1);
      e[r] = lower ? h1 : l1;
      if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);   // bound the shuffles in flight
    }
  }
}

template <int R, int J>
__device__ __forceinline__ void half_stages(double (&e)[R], int lane) {
  if constexpr (J >= 1) {
    if constexpr (J < R) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int q = r ^ J;
        if (r < q) {
          const double hi = dmax(e[r], e[q]), lo = dmin(e[r], e[q]);
          e[r] = hi; e[q] = lo;
        }
      }
    } else {
      constexpr int lm = J / R;
      const bool lower = (lane & lm) == 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double o = __shfl_xor(e[r], lm, 64);
        const double hi = dmax(e[r], o), lo = dmin(e[r], o);
        e[r] = lower ? hi : lo;
        if ((r & 15) == 15) __builtin_amdgcn_sched_barrier(0);
      }
    }
    half_stages<R, J / 2>(e, lane);
  }
}

template <int R, int K = 2>
__device__ __forceinline__ void wave_sort_desc(double (&e)[R], int lane) {
  if constexpr (K <= 64 * R) {
    flip_stage<R, K>(e, lane);
    half_stages<R, K / 4>(e, lane);
    wave_sort_desc<R, 2 * K>(e, lane);
  }
}

// Energy of unit u (FP64; products of FP32 values are exact in FP64) from its
// loaded coefficients and mode weights (1 without weights: the product by 1
// is exact).  The same arithmetic serves the sort (unit order), the tie
// ranking and the keep pass (mode order), so a unit's energy is bit-identical
// in all three.  Loads are unconditional (a missing partner reads the
// representative and is masked).
//
// Every product and sum is rounded on its own (contraction into fused
// multiply-adds is off here): the keep pass forms a pair's energy from either
// member first, and only separately rounded member terms make
// w_a |f_a|^2 + w_b |f_b|^2 the same bits in both orders when the weights are
// not 1.
__device__ __forceinline__ double member_energy(double re, double im, double w) {
#pragma clang fp contract(off)
  return (re * re + im * im) * w;
}

template <typename C>
__device__ __forceinline__ double pair_energy_v(const C fr, const C fp, double wr, double wp, bool partner) {
#pragma clang fp contract(off)
  const double e = member_energy((double)fr.x, (double)fr.y, wr);
  const double ep = member_energy((double)fp.x, (double)fp.y, wp);
  return partner ? e + ep : e;
}

// Flow mode: the weight of eq. (weighted_e) is the launch weight of an
// orographic gravity wave (Appendix A7) under the cell's flow record, in the
// paper's order: intrinsic frequency omega = -k . u (eq. mountain_omega), the
// vertical wave number from the dispersion relation (eq. mw_dispersion), the
// wave action of eq. (mw_action) per unit modal power, taken in magnitude (the
// action and omega share their signed branch, so the wave energy is positive).
// Modes outside the propagating band fc < |omega| < N, and k = 0, weigh 0.
// k = kscale (kx, ky) is the physical wave vector.
struct FlowRec {
  double ux, uy, N, fc, rho, ks;
  bool on;
};

__device__ __forceinline__ double flow_weight(const FlowRec &fl, int kx, int ky) {
#pragma clang fp contract(off)
  const double k1 = fl.ks * (double)kx, k2 = fl.ks * (double)ky;
  const double kk = k1 * k1 + k2 * k2;
  if (!(kk > 0.0)) return 0.0;
  const double omega = -(k1 * fl.ux + k2 * fl.uy);
  const double aw = fabs(omega);
  if (!(aw > fabs(fl.fc) && aw < fl.N)) return 0.0;
  const double m2 = kk * (fl.N * fl.N - omega * omega) / (omega * omega - fl.fc * fl.fc);
  const double act = -(fl.rho / 2.0) * (k1 * fl.ux + k2 * fl.uy) * (kk + m2) / kk;
  return fabs(act);
}

// Weight of mode m (row-major, N1 per row): the flow weight, the caller's
// mode_weight, or 1.
__device__ __forceinline__ double mode_w(const EmsArgs &a, const FlowRec &fl, int m) {
  if (fl.on) {
    const int r = m / a.N1, i = m - r * a.N1;
    return flow_weight(fl, i - (a.N1 >> 1), r - (a.N2 >> 1));
  }
  return a.mode_weight ? a.mode_weight[m] : 1.0;
}

template <typename C>
__device__ __forceinline__ double pair_energy(const EmsArgs &a, const FlowRec &fl, const C *f, int rep, int partner) {
  const int pq = partner >= 0 ? partner : rep;
  const bool wt = a.mode_weight || fl.on;
  const double wr = wt ? mode_w(a, fl, rep) : 1.0, wp = wt ? mode_w(a, fl, pq) : 1.0;
  return pair_energy_v<C>(f[rep], f[pq], wr, wp, partner >= 0);
}

// The energies of n units (or of the units of n modes) with all loads of the
// batch issued before any is used: member indices first, then coefficients,
// then (with mode weights) the weights.  reps[i] < 0 marks an entry with no
// unit (its energy is returned as 0).
template <typename C, int N>
__device__ __forceinline__ void batch_energy(const EmsArgs &a, const FlowRec &fl, const C *f, const int (&reps)[N],
                                             const int (&partners)[N], double (&e)[N]) {
  C fr[N], fp[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int rep = reps[i] >= 0 ? reps[i] : 0;
    fr[i] = f[rep];
    fp[i] = f[partners[i] >= 0 ? partners[i] : rep];
  }
  if (a.mode_weight || fl.on) {
    double wr[N], wp[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int rep = reps[i] >= 0 ? reps[i] : 0;
      wr[i] = mode_w(a, fl, rep);
      wp[i] = mode_w(a, fl, partners[i] >= 0 ? partners[i] : rep);
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
      e[i] = reps[i] >= 0 ? pair_energy_v<C>(fr[i], fp[i], wr[i], wp[i], partners[i] >= 0) : 0.0;
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i)
      e[i] = reps[i] >= 0 ? pair_energy_v<C>(fr[i], fp[i], 1.0, 1.0, partners[i] >= 0) : 0.0;
  }
}

// Workgroup-wide sum / integer sum / integer min / exclusive scan for NW
// waves (NW = 1: the wave operations alone, no barrier).  Every thread gets
// the result; the summation order is fixed.
template <int NW>
__device__ __forceinline__ double block_sum(double v, double *red, int wave) {
  v = wave_sum(v);
  if constexpr (NW == 1) {
    return v;
  } else {
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[w];
    return s;
  }
}
template <int NW>
__device__ __forceinline__ int block_sum_i(int v, int *red, int wave) {
  v = wave_sum_i(v);
  if constexpr (NW == 1) {
    return v;
  } else {
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    int s = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[w];
    return s;
  }
}
template <int NW>
__device__ __forceinline__ int block_min_i(int v, int *red, int wave) {
  v = wave_min_i(v);
  if constexpr (NW == 1) {
    return v;
  } else {
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    int s = INT_MAX;
#pragma unroll
    for (int w = 0; w < NW; ++w) s = min(s, red[w]);
    return s;
  }
}
template <int NW, typename V>
__device__ __forceinline__ V block_exclusive_scan(V v, V *red, int wave, int lane) {
  V x = wave_exclusive_scan<V>(v, lane);
  if constexpr (NW == 1) {
    return x;
  } else {
    const V tot = __shfl(x + v, 63, 64);
    __syncthreads();
    if (lane == 0) red[wave] = tot;
    __syncthreads();
    V base = V(0);
#pragma unroll
    for (int w = 0; w < NW; ++w)
      if (w < wave) base += red[w];
    return base + x;
  }
}

// five waves per SIMD (96 VGPRs) for up to three waves per cell; the four-wave
// form's sort does not fit that and keeps four; the wide forms (below) need one
// workgroup per CU
template <int NW>
constexpr int ems_min_waves() {
  return NW <= 3 ? 5 : NW == 4 ? 4 : (NW + 3) / 4;
}

// One workgroup of NW waves per cell; thread t holds sort positions
// t R .. t R + R - 1.  Each wave sorts its 64 R energies in registers, the
// sorted runs are merged pairwise through LDS (merge path: every thread finds
// where its R outputs start by binary search and merges them sequentially),
// and the scores are read from the sorted array.
//
// The order of eq. (sorted_energy) is by energy, ties by ascending unit id.
// Every quantity before the cut depends only on the sorted energy values, so
// the sort carries values only; which of several units tied at the cut energy
// are kept is settled afterwards by ascending id (a prefix count of the ties).
template <typename T, int R, int NW>
__global__ __launch_bounds__(64 * NW, (ems_min_waves<NW>())) void ems_kernel(EmsArgs a) {
  constexpr int NT = 64 * NW, JW = 64 * R, JP = JW * NW;
  __shared__ double sorted[JP];
  // the tie flags reuse the sorted values' storage: they are written only after
  // every read of the sorted values (see the tie ranking below)
  uint8_t *tie_kept = reinterpret_cast<uint8_t *>(sorted);
  __shared__ double redd[NW];
  __shared__ int redi[NW];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, t = threadIdx.x;
  // cell: the output index; in flow mode step s of cell c is v = s n_cells_f + c
  // and reads the coefficients of cell c
  const int64_t cell = a.cell_begin + blockIdx.x;
  const int64_t fcell = a.flow ? cell % a.n_cells_f : cell;
  using C = typename vec2<T>::type;
  const C *f = reinterpret_cast<const C *>(a.f) + fcell * a.M;
  FlowRec fl{};
  fl.on = a.flow != nullptr;
  if (fl.on) {
    const double *fr = a.flow + 6 * cell;
    fl.ux = fr[0]; fl.uy = fr[1]; fl.N = fr[2]; fl.fc = fr[3]; fl.rho = fr[4]; fl.ks = fr[5];
  }
  const int J = a.J;

  // eq. (energy) / (weighted_e), unit u = position t R + r.  Padding is +0,
  // which sorts among real zero energies; positions >= J are excluded from
  // every sum below, and equal values are interchangeable.
  double e[R];
  double t1 = 0.0, t2 = 0.0;
  // batches of EB units: few memory latencies per thread, few live registers
  // (the kernel's register peak sets how many workgroups share a CU)
  constexpr int EB = R < 4 ? R : 4;
  static_assert(R % EB == 0, "energy batches must divide R");
#pragma unroll
  for (int r0 = 0; r0 < R; r0 += EB) {
    int reps[EB], partners[EB];
#pragma unroll
    for (int i = 0; i < EB; ++i) {
      const int u = t * R + r0 + i;
      const int2 un = a.units[u < J ? u : max(J - 1, 0)];
      reps[i] = u < J ? un.x : -1;
      partners[i] = un.y;
    }
    double eb[EB];
    batch_energy<C, EB>(a, fl, f, reps, partners, eb);
#pragma unroll
    for (int i = 0; i < EB; ++i) e[r0 + i] = eb[i];
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    t1 += e[r];
    t2 += e[r] * e[r];
  }
  const double T1 = block_sum<NW>(t1, redd, wave);
  const double T2 = block_sum<NW>(t2, redd, wave);

  // eq. (sorted_energy): runs of JW per wave, then merges
  wave_sort_desc<R>(e, lane);
#pragma unroll
  for (int r = 0; r < R; ++r) sorted[t * R + r] = e[r];
#pragma unroll
  for (int width = JW; width < JP; width *= 2) {
    __syncthreads();
    const int o0 = t * R;                       // first output position
    const int base = o0 / (2 * width) * (2 * width);
    // runs A = [base, base + width) and B = the rest of the pair (shorter, or
    // empty, at the end when NW is not a power of two)
    const int lb = min(width, max(0, JP - base - width));
    const double *A = sorted + base, *B = A + width;
    const int d = o0 - base;                    // outputs before mine in this merged run
    double out[R];
    if (lb > 0) {
      int lo = d > lb ? d - lb : 0, hi = d < width ? d : width;
      while (lo < hi) {                         // first d outputs take lo from A
        const int mid = (lo + hi) >> 1;
        if (A[mid] >= B[d - 1 - mid]) lo = mid + 1;
        else hi = mid;
      }
      int ia = lo, ib = d - lo;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double va = A[min(ia, width - 1)], vb = B[min(ib, lb - 1)];   // in bounds; guarded below
        const bool take_a = ib >= lb || (ia < width && va >= vb);
        out[r] = take_a ? va : vb;
        ia += take_a;
        ib += !take_a;
      }
    } else {                                    // unpaired run: already in place
#pragma unroll
      for (int r = 0; r < R; ++r) out[r] = sorted[o0 + r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) sorted[o0 + r] = out[r];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) e[r] = sorted[t * R + r];   // this thread's sorted positions
  const double enext = (t * R + R < JP) ? sorted[t * R + R] : 0.0;

  const int Jmax = J < a.k_max ? J : a.k_max;
  // eq. (n_eff) over all J units, clipped by the budget
  const double neff = T2 > 0.0 ? T1 * T1 / T2 : 0.0;
  const double nclip = neff < (double)Jmax ? neff : (double)Jmax;
  // eq. (s_delta) over the first J_max - 1 gaps
  double sd = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = t * R + r;
    if (j < Jmax - 1) {
      const double ea = e[r], eb = (r + 1 < R) ? e[r + 1 < R ? r + 1 : r] : enext;
      double term;
      if (eb == 0.0 && ea == 0.0) term = 1.0;
      else if (eb == 0.0) term = 0.0;
      else term = exp(-(ea / eb - 1.0) / a.delta);
      sd += term;
    }
  }
  const double sdsum = block_sum<NW>(sd, redd, wave);
  const double sdel = Jmax < 2 ? 1.0 : sdsum / (double)(Jmax - 1);
  // eqs. (c_score), (alpha_c)
  const double Cs = (Jmax > 0 ? a.w1 * nclip / (double)Jmax : 0.0) + a.w2 * sdel;
  const double alphaC = a.alpha_min + (a.alpha_max - a.alpha_min) * Cs;

  // eq. (f_cum): running sum in sorted order; the first K with theta(K) >= alpha_C
  double loc = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (t * R + r < J) loc += e[r];
  double run = block_exclusive_scan<NW, double>(loc, redd, wave, lane);
  int kc = INT_MAX;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = t * R + r;
    if (j < J) {
      run += e[r];
      if (T1 > 0.0 && kc == INT_MAX && run / T1 >= alphaC) kc = j + 1;
    }
  }
  kc = block_min_i<NW>(kc, redi, wave);
  // eq. (k_elastic)
  int kstar;
  if (!(T1 > 0.0)) {
    kstar = a.k_min < J ? a.k_min : J;
  } else {
    const int kcc = kc == INT_MAX ? J : kc;
    const int k = kcc > a.k_min ? kcc : a.k_min;
    kstar = k < Jmax ? k : Jmax;
  }
  // cut energy E_(K*), the retained sum of the first K* sorted energies, and
  // how many units lie strictly above the cut or at it
  const double eth = kstar > 0 ? sorted[kstar - 1] : 0.0;
  double part = 0.0;
  int cgt = 0, ceq = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = t * R + r;
    if (j < kstar) part += e[r];
    if (j < J) {
      cgt += e[r] > eth;
      ceq += e[r] == eth;
    }
  }
  const double th = block_sum<NW>(part, redd, wave);
  const int ngt = block_sum_i<NW>(cgt, redi, wave);
  const int neq = block_sum_i<NW>(ceq, redi, wave);
  const int need = kstar - ngt;   // units kept at the cut energy, lowest ids first

  // Ties straddling the cut (more units at the cut energy than kept there):
  // rank the tied units by id.  Otherwise every unit at the cut is kept.
  const bool split_ties = kstar > 0 && neq > need;
  if (split_ties) {   // the same in every thread
    __syncthreads();   // every thread has read the sorted values (tie_kept overwrites them)
    int ties = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int u = t * R + r;
      const int2 un = a.units[u < J ? u : max(J - 1, 0)];
      ties += (u < J && pair_energy<C>(a, fl, f, un.x, un.y) == eth);
    }
    int rank = block_exclusive_scan<NW, int>(ties, redi, wave, lane);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int u = t * R + r;
      const int2 un = a.units[u < J ? u : max(J - 1, 0)];
      const bool tie = u < J && pair_energy<C>(a, fl, f, un.x, un.y) == eth;
      tie_kept[u] = tie && rank < need;
      rank += tie;
    }
    __syncthreads();
  }

  // modes (coalesced): keep flags and the retained power.  Batches of UK modes
  // per thread: all loads of a batch come before its stores (the byte stores
  // may alias the coefficients as far as the compiler knows, so a store
  // between loads would serialise them).  A paired mode's other member is its
  // mirror -k, whose index follows from the mode's own, so the coefficient
  // loads need not wait for the mode's unit record and a batch costs about
  // one memory latency.  The energy e(m) + e(mirror) equals the unit's
  // e(rep) + e(partner) bit for bit (the same member terms; FP64 addition
  // commutes).
  double pw = 0.0;
  uint8_t *kout = a.keep ? a.keep + cell * a.M : nullptr;   // flow mode may skip the masks
  constexpr int UK = 2;
  const int N1 = a.N1, hm1 = 2 * (a.N1 >> 1), hm2 = 2 * (a.N2 >> 1);
  const float inv_n1 = 1.0f / (float)N1;
  for (int m0 = t; m0 < a.M; m0 += UK * NT) {
    uint8_t v[UK];
    int4 mu[UK];
    C fm[UK], fo[UK];
    int mm[UK], mo[UK];
#pragma unroll
    for (int u = 0; u < UK; ++u) {
      const int m = min(m0 + u * NT, a.M - 1);
      // row and column of m (the float quotient is within one of the true one)
      int r = (int)((float)m * inv_n1);
      r -= r * N1 > m;
      r += (r + 1) * N1 <= m;
      const int ri = hm2 - r, ii = hm1 - (m - r * N1);   // the mirror's row and column
      mm[u] = m;
      mo[u] = (ri < a.N2 && ii < N1) ? ri * N1 + ii : m;
      mu[u] = a.mode_unit[m];
      fm[u] = f[m];
      fo[u] = f[mo[u]];
    }
    double eu[UK];
    if (a.mode_weight || fl.on) {
      double wm[UK], wo[UK];
#pragma unroll
      for (int u = 0; u < UK; ++u) {
        wm[u] = mode_w(a, fl, mm[u]);
        wo[u] = mode_w(a, fl, mo[u]);
      }
#pragma unroll
      for (int u = 0; u < UK; ++u) eu[u] = pair_energy_v<C>(fm[u], fo[u], wm[u], wo[u], mu[u].y >= 0);
    } else {
#pragma unroll
      for (int u = 0; u < UK; ++u) eu[u] = pair_energy_v<C>(fm[u], fo[u], 1.0, 1.0, mu[u].y >= 0);
    }
#pragma unroll
    for (int u = 0; u < UK; ++u) {
      const bool keep = m0 + u * NT < a.M && mu[u].x >= 0 && kstar > 0 &&
                        (eu[u] > eth || (eu[u] == eth && (!split_ties || tie_kept[mu[u].z])));
      v[u] = keep;
      if (keep) pw += (double)fm[u].x * (double)fm[u].x + (double)fm[u].y * (double)fm[u].y;
    }
#pragma unroll
    for (int u = 0; u < UK; ++u) {
      const int m = m0 + u * NT;
      if (m < a.M && kout) kout[m] = v[u];
    }
  }
  const double P = block_sum<NW>(pw, redd, wave);
  if (t == 0) {
    a.k_star[cell] = kstar;
    double *st = a.stats + cell * 8;
    st[0] = T1; st[1] = P; st[2] = neff; st[3] = sdel;
    st[4] = Cs; st[5] = alphaC; st[6] = T1 > 0.0 ? th / T1 : 0.0; st[7] = (double)J;
  }
}

// Units on the host: +-k pairs (representative k_y > 0, or k_y = 0 and k_x > 0)
// when both members lie in the box, otherwise single modes; ascending id.
static void build_units(int N1, int N2, bool pairs, bool exclude_dc, std::vector<int2> &out) {
  out.clear();
  const int lo1 = -(N1 / 2), lo2 = -(N2 / 2), hi1 = lo1 + N1 - 1, hi2 = lo2 + N2 - 1;
  for (int r = 0; r < N2; ++r) {
    for (int i = 0; i < N1; ++i) {
      const int kx = lo1 + i, ky = lo2 + r, idx = r * N1 + i;
      const bool dc = kx == 0 && ky == 0;
      if (dc && exclude_dc) continue;
      int partner = -1;
      if (pairs && !dc) {
        const int mx = -kx, my = -ky;
        if (mx >= lo1 && mx <= hi1 && my >= lo2 && my <= hi2) partner = (my - lo2) * N1 + (mx - lo1);
      }
      if (partner >= 0 && !(ky > 0 || (ky == 0 && kx > 0))) continue;
      out.push_back(make_int2(idx, partner));
    }
  }
}


enufft_status ems_units(enufft_plan_t p, const enufft_ems_params *prm, UnitTable **ut) {
  UnitTable &u = p->units[prm->use_pairs ? 1 : 0][prm->exclude_dc ? 1 : 0];
  if (!u.built) {
    std::vector<int2> v;
    build_units(p->N1, p->N2, prm->use_pairs != 0, prm->exclude_dc != 0, v);
    const int M = p->N1 * p->N2;
    u.J = (int)v.size();
    // the kernel's branch-free loads read unit max(J - 1, 0): give an empty set
    // one harmless entry (mode 0, no partner) that is never counted
    if (v.empty()) v.push_back(make_int2(0, -1));
    std::vector<int4> of_mode(M, make_int4(-1, -1, -1, 0));
    for (int i = 0; i < u.J; ++i) {
      of_mode[v[i].x] = make_int4(v[i].x, v[i].y, i, 0);
      if (v[i].y >= 0) of_mode[v[i].y] = make_int4(v[i].x, v[i].y, i, 0);
    }
    u.Jpad = 64;
    while (u.Jpad < u.J) u.Jpad <<= 1;
    void *d = nullptr, *dm = nullptr;
    hipError_t e = hipMalloc(&d, std::max<size_t>(1, v.size()) * sizeof(int2));
    if (e == hipSuccess) p->allocations.push_back(d);
    if (e == hipSuccess) e = hipMalloc(&dm, (size_t)M * sizeof(int4));
    if (e == hipSuccess) p->allocations.push_back(dm);
    if (e != hipSuccess) {
      p->last_error = "EMS unit table allocation failed";
      return ENUFFT_ENOMEM;
    }
    if (!v.empty()) e = hipMemcpy(d, v.data(), v.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dm, of_mode.data(), (size_t)M * sizeof(int4), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      p->last_error = std::string("EMS unit table upload: ") + hipGetErrorString(e);
      p->faulted = true;
      return ENUFFT_EDEVICE;
    }
    u.d_units = (int2 *)d;
    u.d_mode_unit = (int4 *)dm;
    u.built = true;
  }
  *ut = &u;
  return ENUFFT_OK;
}

enufft_status ems_validate(enufft_plan_t p, const void *f, const enufft_ems_params *prm, uint8_t *keep,
                           int32_t *k_star, double *stats) {
  auto bad = [&](const char *m) {
    p->last_error = std::string("enufft_ems: ") + m;
    return ENUFFT_EINVAL;
  };
  if (!prm) return bad("null params");
  if (!f || !keep || !k_star || !stats) return bad("null output or input pointer");
  if (prm->k_min < 0 || prm->k_max < 1 || prm->k_min > prm->k_max) return bad("need 0 <= k_min <= k_max, k_max >= 1");
  if (!(prm->alpha_min >= 0.0 && prm->alpha_min <= 1.0 && prm->alpha_max >= 0.0 && prm->alpha_max <= 1.0))
    return bad("alpha_min and alpha_max must be in [0, 1]");
  if (!(prm->delta > 0.0) || !std::isfinite(prm->delta)) return bad("delta must be > 0");
  if (!(prm->w1 >= 0.0 && prm->w1 <= 1.0 && prm->w2 >= 0.0 && prm->w2 <= 1.0)) return bad("w1, w2 must be in [0, 1]");
  if ((prm->use_pairs != 0 && prm->use_pairs != 1) || (prm->exclude_dc != 0 && prm->exclude_dc != 1))
    return bad("use_pairs and exclude_dc must be 0 or 1");
  return ENUFFT_OK;
}

// Sort size per cell: the smallest 64 R NW >= J (R a power of two up to 16,
// then 1 to 4 waves of 1,024).
// Whether a launch of `blocks` cells leaves the CUs mostly idle with the narrow
// forms (fewer than eight of their waves per CU): then the wide forms.
// ENUFFT_EMS_WIDE=0 or 1 forces the choice.
bool ems_wide(const enufft_plan_t p, int J, int64_t blocks) {
  if (const char *ev = std::getenv("ENUFFT_EMS_WIDE")) return std::atoi(ev) != 0;
  const int64_t waves = blocks * ((J + 1023) / 1024);
  return waves < (int64_t)p->n_cu * 8;
}

template <typename T>
hipError_t launch_ems_t(const EmsArgs &a, int J, int blocks, hipStream_t s, bool wide) {
  const dim3 g(blocks);
  if (wide && J > 256) {
    // few cells: each cell's latency is the launch's, so more waves per cell, four
    // values per lane (a shorter register sort, more merge rounds through LDS)
    if (J <= 512) hipLaunchKernelGGL((ems_kernel<T, 4, 2>), g, dim3(128), 0, s, a);
    else if (J <= 768) hipLaunchKernelGGL((ems_kernel<T, 4, 3>), g, dim3(192), 0, s, a);
    else if (J <= 1024) hipLaunchKernelGGL((ems_kernel<T, 4, 4>), g, dim3(256), 0, s, a);
    else if (J <= 1536) hipLaunchKernelGGL((ems_kernel<T, 4, 6>), g, dim3(384), 0, s, a);
    else if (J <= 2048) hipLaunchKernelGGL((ems_kernel<T, 4, 8>), g, dim3(512), 0, s, a);
    else if (J <= 3072) hipLaunchKernelGGL((ems_kernel<T, 4, 12>), g, dim3(768), 0, s, a);
    else if (J <= 4096) hipLaunchKernelGGL((ems_kernel<T, 4, 16>), g, dim3(1024), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (J <= 64) hipLaunchKernelGGL((ems_kernel<T, 1, 1>), g, dim3(64), 0, s, a);
  else if (J <= 128) hipLaunchKernelGGL((ems_kernel<T, 2, 1>), g, dim3(64), 0, s, a);
  else if (J <= 256) hipLaunchKernelGGL((ems_kernel<T, 4, 1>), g, dim3(64), 0, s, a);
  else if (J <= 512) hipLaunchKernelGGL((ems_kernel<T, 8, 1>), g, dim3(64), 0, s, a);
  else if (J <= 1024) hipLaunchKernelGGL((ems_kernel<T, 16, 1>), g, dim3(64), 0, s, a);
  else if (J <= 2048) hipLaunchKernelGGL((ems_kernel<T, 16, 2>), g, dim3(128), 0, s, a);
  else if (J <= 3072) hipLaunchKernelGGL((ems_kernel<T, 16, 3>), g, dim3(192), 0, s, a);
  else if (J <= 4096) hipLaunchKernelGGL((ems_kernel<T, 16, 4>), g, dim3(256), 0, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

enufft_status record_start(enufft_plan_t p, int kind, hipEvent_t *ev);
enufft_status record_stop(enufft_plan_t p, int kind, hipEvent_t start);

enufft_status ems_launch(enufft_plan_t p, const void *f, const enufft_ems_params *prm, const double *mode_weight,
                         uint8_t *keep, int32_t *k_star, double *stats, int64_t cell_begin, int64_t cell_count) {
  UnitTable *ut = nullptr;
  enufft_status st = ems_units(p, prm, &ut);
  if (st != ENUFFT_OK) return st;
  if (ut->Jpad > 4096)   // beyond the per-cell register sort: device sort per cell
    return big_ems(p, f, prm, mode_weight, keep, k_star, stats, ut, cell_begin, cell_count);
  EmsArgs a{};
  a.f = f; a.mode_weight = mode_weight; a.keep = keep; a.k_star = k_star; a.stats = stats;
  a.units = ut->d_units; a.mode_unit = ut->d_mode_unit; a.J = ut->J; a.M = p->N1 * p->N2;
  a.N1 = p->N1; a.N2 = p->N2;
  a.cell_begin = cell_begin;
  a.cell_end = cell_begin + cell_count;
  a.k_min = prm->k_min; a.k_max = prm->k_max;
  a.alpha_min = prm->alpha_min; a.alpha_max = prm->alpha_max; a.delta = prm->delta;
  a.w1 = prm->w1; a.w2 = prm->w2;
  const int blocks = (int)cell_count;
  const bool wide = ems_wide(p, ut->J, blocks);
  hipError_t e = p->prec == ENUFFT_F64 ? launch_ems_t<double>(a, ut->J, blocks, p->stream, wide)
                                       : launch_ems_t<float>(a, ut->J, blocks, p->stream, wide);
  if (e != hipSuccess) {
    p->last_error = std::string("EMS launch: ") + hipGetErrorString(e);
    p->faulted = true;
    return ENUFFT_EDEVICE;
  }
  return ENUFFT_OK;
}

}  // namespace enufft

extern "C" enufft_status enufft_ems(enufft_plan_t p, const void *f, const enufft_ems_params *prm,
                                    const double *mode_weight, uint8_t *keep, int32_t *k_star, double *stats) {
  if (!p) return ENUFFT_EINVAL;
  if (p->faulted) {
    p->last_error = "enufft_ems: plan unusable after a device fault";
    return ENUFFT_ESTATE;
  }
  enufft_status st = enufft::ems_validate(p, f, prm, keep, k_star, stats);
  if (st != ENUFFT_OK) return st;
  if (p->n_cells == 0) return ENUFFT_OK;
  hipEvent_t ev;
  st = enufft::record_start(p, 1, &ev);
  if (st != ENUFFT_OK) return st;
  st = enufft::ems_launch(p, f, prm, mode_weight, keep, k_star, stats, 0, p->n_cells);
  if (st != ENUFFT_OK) return st;
  return enufft::record_stop(p, 1, ev);
}

extern "C" enufft_status enufft_ems_flow(enufft_plan_t p, const void *f, const enufft_ems_params *prm,
                                         int32_t n_steps, const double *flow, uint8_t *keep, int32_t *k_star,
                                         double *stats) {
  if (!p) return ENUFFT_EINVAL;
  if (p->faulted) {
    p->last_error = "enufft_ems_flow: plan unusable after a device fault";
    return ENUFFT_ESTATE;
  }
  uint8_t dummy = 0;
  // the masks are optional here: validate with a stand-in pointer
  enufft_status st = enufft::ems_validate(p, f, prm, keep ? keep : &dummy, k_star, stats);
  if (st != ENUFFT_OK) return st;
  if (n_steps < 1 || !flow) {
    p->last_error = "enufft_ems_flow: need n_steps >= 1 and flow records";
    return ENUFFT_EINVAL;
  }
  if (p->n_cells == 0) return ENUFFT_OK;
  if ((int64_t)n_steps * p->n_cells > (int64_t)INT32_MAX) {
    p->last_error = "enufft_ems_flow: n_steps * n_cells above 2^31 - 1";
    return ENUFFT_EINVAL;
  }
  enufft::UnitTable *ut = nullptr;
  st = enufft::ems_units(p, prm, &ut);
  if (st != ENUFFT_OK) return st;
  if (ut->Jpad > 4096) {
    p->last_error = "enufft_ems_flow: more than 4096 units per cell is not supported";
    return ENUFFT_EUNSUPPORTED;
  }
  enufft::EmsArgs a{};
  a.f = f; a.mode_weight = nullptr; a.flow = flow; a.n_cells_f = p->n_cells;
  a.keep = keep; a.k_star = k_star; a.stats = stats;
  a.units = ut->d_units; a.mode_unit = ut->d_mode_unit; a.J = ut->J; a.M = p->N1 * p->N2;
  a.N1 = p->N1; a.N2 = p->N2;
  a.cell_begin = 0;
  a.cell_end = (int64_t)n_steps * p->n_cells;
  a.k_min = prm->k_min; a.k_max = prm->k_max;
  a.alpha_min = prm->alpha_min; a.alpha_max = prm->alpha_max; a.delta = prm->delta;
  a.w1 = prm->w1; a.w2 = prm->w2;
  hipEvent_t ev;
  st = enufft::record_start(p, 1, &ev);
  if (st != ENUFFT_OK) return st;
  const int blocks = (int)a.cell_end;
  const bool wide = enufft::ems_wide(p, ut->J, blocks);
  hipError_t e = p->prec == ENUFFT_F64 ? enufft::launch_ems_t<double>(a, ut->J, blocks, p->stream, wide)
                                       : enufft::launch_ems_t<float>(a, ut->J, blocks, p->stream, wide);
  if (e != hipSuccess) {
    p->last_error = std::string("enufft_ems_flow launch: ") + hipGetErrorString(e);
    p->faulted = true;
    return ENUFFT_EDEVICE;
  }
  return enufft::record_stop(p, 1, ev);
}
