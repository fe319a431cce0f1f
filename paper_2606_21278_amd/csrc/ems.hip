// Elastic Mode Selection on gfx950: one workgroup per cell.
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
#include <string>
#include <vector>

#include "device_common.h"
#include "launch.h"
#include "plan.h"

namespace enufft {

struct EmsArgs {
  const void *f;
  const double *mode_weight;
  uint8_t *keep;
  int32_t *k_star;
  double *stats;
  const int2 *units;          // (rep, partner | -1), ascending unit id
  int J, Jpad;
  int M;                      // modes per cell = N1 * N2
  int64_t cell_begin;
  int k_min, k_max;
  double alpha_min, alpha_max, delta, w1, w2;
};

template <int NT>
__device__ double block_sum(double v, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < NT / 64; ++i) s += red[i];
    red[NT / 64] = s;
  }
  __syncthreads();
  s = red[NT / 64];
  __syncthreads();
  return s;
}

// "a precedes b" in the order of eq. (sorted_energy): larger energy first, ties
// by smaller unit id.
__device__ __forceinline__ bool precedes(double ea, int ia, double eb, int ib) {
  return ea > eb || (ea == eb && ia < ib);
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void ems_kernel(EmsArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *E = reinterpret_cast<double *>(smem_raw);
  int *id = reinterpret_cast<int *>(E + a.Jpad);
  uint8_t *kp = reinterpret_cast<uint8_t *>(id + a.Jpad);
  __shared__ double red[NT / 64 + 1];
  __shared__ double scan_tot[NT];
  __shared__ int s_kc;

  const int64_t cell = a.cell_begin + blockIdx.x;
  using C = typename vec2<T>::type;
  const C *f = reinterpret_cast<const C *>(a.f) + cell * a.M;
  const int J = a.J, Jpad = a.Jpad;

  // unit energies in FP64 (products of FP32 values are exact in FP64)
  double t1 = 0.0, t2 = 0.0;
  for (int u = threadIdx.x; u < Jpad; u += NT) {
    if (u < J) {
      const int2 un = a.units[u];
      const C fr = f[un.x];
      double e = (double)fr.x * (double)fr.x + (double)fr.y * (double)fr.y;
      if (a.mode_weight) e *= a.mode_weight[un.x];
      if (un.y >= 0) {
        const C fp = f[un.y];
        double ep = (double)fp.x * (double)fp.x + (double)fp.y * (double)fp.y;
        if (a.mode_weight) ep *= a.mode_weight[un.y];
        e += ep;
      }
      E[u] = e;
      id[u] = u;
      t1 += e;
      t2 += e * e;
    } else {
      E[u] = -1.0;
      id[u] = INT_MAX;
    }
  }
  const double T1 = block_sum<NT>(t1, red);
  const double T2 = block_sum<NT>(t2, red);

  // bitonic sort of (E, id) into the order of eq. (sorted_energy)
  for (int k = 2; k <= Jpad; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < Jpad; i += NT) {
        const int l = i ^ j;
        if (l > i) {
          const double ei = E[i], el = E[l];
          const int ii = id[i], il = id[l];
          const bool up = (i & k) == 0;
          const bool sw = up ? precedes(el, il, ei, ii) : precedes(ei, ii, el, il);
          if (sw) { E[i] = el; E[l] = ei; id[i] = il; id[l] = ii; }
        }
      }
      __syncthreads();
    }
  }

  const int Jmax = J < a.k_max ? J : a.k_max;
  // eq. (n_eff) over all J* units, clipped by the budget
  const double neff = T2 > 0.0 ? T1 * T1 / T2 : 0.0;
  const double nclip = neff < (double)Jmax ? neff : (double)Jmax;
  // eq. (s_delta) over the first J_max - 1 gaps
  double sd = 0.0;
  for (int j = threadIdx.x; j < Jmax - 1; j += NT) {
    const double ea = E[j], eb = E[j + 1];
    double term;
    if (eb == 0.0 && ea == 0.0) term = 1.0;
    else if (eb == 0.0) term = 0.0;
    else term = exp(-(ea / eb - 1.0) / a.delta);
    sd += term;
  }
  const double sdsum = block_sum<NT>(sd, red);
  const double sdel = Jmax < 2 ? 1.0 : sdsum / (double)(Jmax - 1);
  const double Cs = (Jmax > 0 ? a.w1 * nclip / (double)Jmax : 0.0) + a.w2 * sdel;
  const double alphaC = a.alpha_min + (a.alpha_max - a.alpha_min) * Cs;

  // running sum of the sorted energies (eq. f_cum): contiguous segments per
  // thread, then a scan of the segment totals
  const int seg = (J + NT - 1) / NT;
  const int s0 = threadIdx.x * seg;
  const int s1 = min(J, s0 + seg);
  double loc = 0.0;
  for (int j = s0; j < s1; ++j) loc += E[j];
  scan_tot[threadIdx.x] = loc;
  if (threadIdx.x == 0) s_kc = INT_MAX;
  __syncthreads();
  for (int o = 1; o < NT; o <<= 1) {
    const double v = threadIdx.x >= o ? scan_tot[threadIdx.x - o] : 0.0;
    __syncthreads();
    scan_tot[threadIdx.x] += v;
    __syncthreads();
  }
  double run = threadIdx.x > 0 ? scan_tot[threadIdx.x - 1] : 0.0;
  if (T1 > 0.0) {
    for (int j = s0; j < s1; ++j) {
      run += E[j];
      if (run / T1 >= alphaC) { atomicMin(&s_kc, j + 1); break; }
    }
  }
  // zero the keep staging area
  for (int m = threadIdx.x; m < a.M; m += NT) kp[m] = 0;
  __syncthreads();
  int kstar;
  if (!(T1 > 0.0)) {
    kstar = a.k_min < J ? a.k_min : J;
  } else {
    const int kc = s_kc == INT_MAX ? J : s_kc;
    const int k = kc > a.k_min ? kc : a.k_min;
    kstar = k < Jmax ? k : Jmax;
  }
  // eq. (k_elastic): keep every mode of the first K* units
  for (int j = threadIdx.x; j < kstar; j += NT) {
    const int2 un = a.units[id[j]];
    kp[un.x] = 1;
    if (un.y >= 0) kp[un.y] = 1;
  }
  __syncthreads();
  double pw = 0.0, th = 0.0;
  for (int m = threadIdx.x; m < a.M; m += NT) {
    const uint8_t v = kp[m];
    a.keep[cell * a.M + m] = v;
    if (v) {
      const C fr = f[m];
      pw += (double)fr.x * (double)fr.x + (double)fr.y * (double)fr.y;
    }
  }
  for (int j = threadIdx.x; j < kstar; j += NT) th += E[j];
  const double P = block_sum<NT>(pw, red);
  const double TH = block_sum<NT>(th, red);
  if (threadIdx.x == 0) {
    a.k_star[cell] = kstar;
    double *st = a.stats + cell * 8;
    st[0] = T1; st[1] = P; st[2] = neff; st[3] = sdel;
    st[4] = Cs; st[5] = alphaC; st[6] = T1 > 0.0 ? TH / T1 : 0.0; st[7] = (double)J;
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

static int ems_threads() { return 512; }

static size_t ems_lds(int Jpad, int M) { return (size_t)Jpad * (8 + 4) + (size_t)M + 16; }

enufft_status ems_units(enufft_plan_t p, const enufft_ems_params *prm, UnitTable **ut) {
  UnitTable &u = p->units[prm->use_pairs ? 1 : 0][prm->exclude_dc ? 1 : 0];
  if (!u.built) {
    std::vector<int2> v;
    build_units(p->N1, p->N2, prm->use_pairs != 0, prm->exclude_dc != 0, v);
    u.J = (int)v.size();
    u.Jpad = 1;
    while (u.Jpad < std::max(1, u.J)) u.Jpad <<= 1;
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, std::max<size_t>(1, v.size()) * sizeof(int2));
    if (e != hipSuccess) {
      p->last_error = "EMS unit table allocation failed";
      return ENUFFT_ENOMEM;
    }
    p->allocations.push_back(d);
    if (!v.empty()) {
      e = hipMemcpy(d, v.data(), v.size() * sizeof(int2), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        p->last_error = std::string("EMS unit table upload: ") + hipGetErrorString(e);
        p->faulted = true;
        return ENUFFT_EDEVICE;
      }
    }
    u.d_units = (int2 *)d;
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

template <typename T>
hipError_t launch_ems_t(const EmsArgs &a, int blocks, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL((ems_kernel<T, 512>), dim3(blocks), dim3(512), lds, s, a);
  return hipGetLastError();
}

enufft_status record_start(enufft_plan_t p, int kind, hipEvent_t *ev);
enufft_status record_stop(enufft_plan_t p, int kind, hipEvent_t start);

enufft_status ems_launch(enufft_plan_t p, const void *f, const enufft_ems_params *prm, const double *mode_weight,
                         uint8_t *keep, int32_t *k_star, double *stats, int64_t cell_begin, int64_t cell_count) {
  UnitTable *ut = nullptr;
  enufft_status st = ems_units(p, prm, &ut);
  if (st != ENUFFT_OK) return st;
  EmsArgs a{};
  a.f = f; a.mode_weight = mode_weight; a.keep = keep; a.k_star = k_star; a.stats = stats;
  a.units = ut->d_units; a.J = ut->J; a.Jpad = ut->Jpad; a.M = p->N1 * p->N2;
  a.cell_begin = cell_begin;
  a.k_min = prm->k_min; a.k_max = prm->k_max;
  a.alpha_min = prm->alpha_min; a.alpha_max = prm->alpha_max; a.delta = prm->delta;
  a.w1 = prm->w1; a.w2 = prm->w2;
  const size_t lds = ems_lds(a.Jpad, a.M);
  hipError_t e = p->prec == ENUFFT_F64 ? launch_ems_t<double>(a, (int)cell_count, lds, p->stream)
                                       : launch_ems_t<float>(a, (int)cell_count, lds, p->stream);
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
