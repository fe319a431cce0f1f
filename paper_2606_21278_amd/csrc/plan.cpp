// Host side of the ENUFFT library: argument validation, kernel parameters,
// FP64 deconvolution tables, the work schedule, workspace and the C ABI.
#include "plan.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "launch.h"

using enufft::AdjItem;
using enufft::FwdItem;
using enufft::Geom;

namespace {

thread_local std::string g_thread_error;

enufft_status fail(enufft_plan_t p, enufft_status s, const std::string &msg) {
  if (p) p->last_error = msg;
  g_thread_error = msg;
  return s;
}

enufft_status hip_fail(enufft_plan_t p, hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  if (p && e != hipErrorInvalidValue && e != hipErrorMemoryAllocation && e != hipErrorOutOfMemory)
    p->faulted = true;
  return fail(p, (e == hipErrorMemoryAllocation || e == hipErrorOutOfMemory) ? ENUFFT_ENOMEM : ENUFFT_EDEVICE, m);
}

#define HIP_TRY(p, expr, what)                      \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) return hip_fail(p, e_, what); \
  } while (0)

int next_pow2(int v) {
  int n = 1;
  while (n < v) n <<= 1;
  return n;
}

// Widths with compiled kernels; a requested width is rounded up to one of these.
const int kWidths[] = {4, 6, 8, 10, 12, 14, 16};

// Spreading-kernel width for a requested accuracy and effective oversampling:
// the exponential-of-semicircle kernel at upsampling 2 reaches about
// 10^-(W-1) with W grid points and shape beta = 2.30 W; for smaller upsampling
// the width grows as -ln(eps) / (pi sqrt(1 - 1/sigma)) with
// beta = 0.97 pi (1 - 1/(2 sigma)) W.
void kernel_params(double eps, double sigma_eff, int min_w, int *W_out, double *beta_out) {
  int w;
  if (sigma_eff >= 2.0 - 1e-12) {
    w = (int)std::ceil(-std::log10(eps / 10.0));
  } else {
    w = (int)std::ceil(-std::log(eps) / (M_PI * std::sqrt(1.0 - 1.0 / sigma_eff)));
  }
  w = std::max(w, min_w);
  w = std::max(w, 2);
  int W = 16;
  for (int c : kWidths)
    if (c >= w) { W = c; break; }
  double beta;
  if (sigma_eff >= 2.0 - 1e-12) beta = 2.30 * W;
  else beta = 0.97 * M_PI * (1.0 - 1.0 / (2.0 * sigma_eff)) * W;
  *W_out = W;
  *beta_out = beta;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on the Legendre recurrence).
void gauss_legendre(int M, std::vector<double> &x, std::vector<double> &w) {
  x.resize(M);
  w.resize(M);
  for (int i = 0; i < M; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (M + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= M; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double dp = M * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= M; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double dp = M * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Kernel Fourier factor p(k) = (1/Delta) int phi(x) exp(-i k x) dx for the grid
// spacing Delta = 2 pi / n and phi(x) = psi(x / alpha), alpha = W Delta / 2:
//   p(k) = (W / 2) int_{-1}^{1} psi(z) cos(k pi W z / n) dz.
// With z = sin(theta) the integrand is smooth:
//   int_{-pi/2}^{pi/2} exp(beta (cos theta - 1)) cos(a sin theta) cos theta dtheta.
// This is the factor divided out in Step 4 (eq. deconv).
std::vector<double> kernel_ft(int W, double beta, int n, int kmax) {
  static std::vector<double> gx, gw;
  if (gx.empty()) gauss_legendre(200, gx, gw);
  std::vector<double> p(kmax + 1);
  for (int k = 0; k <= kmax; ++k) {
    const double a = k * M_PI * W / n;
    double s = 0.0;
    for (size_t i = 0; i < gx.size(); ++i) {
      const double th = 0.5 * M_PI * gx[i];
      s += gw[i] * std::exp(beta * (std::cos(th) - 1.0)) * std::cos(a * std::sin(th)) * std::cos(th);
    }
    p[k] = 0.5 * W * s * 0.5 * M_PI;
  }
  return p;
}

// psi(z) = exp(beta (sqrt(1 - z^2) - 1)), zero for |z| > 1.
double es_host(double z, double beta) {
  if (std::fabs(z) > 1.0) return 0.0;
  return std::exp(-beta * z * z / (1.0 + std::sqrt(1.0 - z * z)));
}

// I0 by its power series (x <= 60 needs at most about 100 terms).
double bessel_i0_host(double x) {
  const double t = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 200; ++k) {
    term *= t / ((double)k * k);
    const double next = sum + term;
    if (next == sum) break;
    sum = next;
  }
  return sum;
}

// Kaiser-Bessel shape gamma of eq. (kaisal_bessel_coeffs) (MIRT form, beta = 2.34) or
// eq. (kb_type_2) (gamma = 2.34), for half-width a = W / 2 grid cells.
double kb_gamma(int kind, int W) {
  const double a = 0.5 * W, b = 2.34;
  if (kind == ENUFFT_KERNEL_KB_FESSLER) return b;
  const double r = 2.0 * a * b / M_PI;
  return M_PI * std::sqrt(r * r - 0.8);
}

// The plan's kernel at z in [-1, 1] (shape > 0: ES beta; shape < 0: KB with gamma = -shape,
// normalised to 1 at 0).
double kernel_host(double z, double shape) {
  if (std::fabs(z) > 1.0) return 0.0;
  if (shape > 0.0) return es_host(z, shape);
  const double g = -shape;
  return bessel_i0_host(g * std::sqrt(std::max(0.0, 1.0 - z * z))) / bessel_i0_host(g);
}

// Deconvolution factor of the normalised Kaiser-Bessel kernel, the closed form of
// eq. (kb_fourier) divided by I0(gamma) / I0(beta): at kappa = 2 pi k / n radians per
// grid cell, p(k) = (2 a / I0(gamma)) sinh(r) / r with r = sqrt(gamma^2 - (a kappa)^2),
// continued as sin(r') / r' with r' = sqrt((a kappa)^2 - gamma^2) beyond gamma.
std::vector<double> kb_ft(int W, double gamma, int n, int kmax) {
  std::vector<double> p(kmax + 1);
  const double a = 0.5 * W, i0 = bessel_i0_host(gamma);
  for (int k = 0; k <= kmax; ++k) {
    const double ak = a * 2.0 * M_PI * k / n;
    const double d = gamma * gamma - ak * ak;
    double f;
    if (d > 0.0) {
      const double r = std::sqrt(d);
      f = std::sinh(r) / r;
    } else if (d < 0.0) {
      const double r = std::sqrt(-d);
      f = std::sin(r) / r;
    } else {
      f = 1.0;
    }
    p[k] = 2.0 * a * f / i0;
  }
  return p;
}

// d psi / dz of the plan's kernel on |z| < 1 (ES: psi beta (-z / sqrt(1 - z^2)); KB:
// -gamma z I1(gamma s) / (s I0(gamma)), s = sqrt(1 - z^2)), zero outside.
double bessel_i1_host(double x) {
  const double t = 0.25 * x * x;
  double term = 0.5 * x, sum = term;
  for (int k = 1; k < 200; ++k) {
    term *= t / ((double)k * (k + 1));
    const double next = sum + term;
    if (next == sum) break;
    sum = next;
  }
  return sum;
}

double kernel_deriv_host(double z, double shape) {
  if (!(std::fabs(z) < 1.0)) return 0.0;
  const double s = std::sqrt(1.0 - z * z);
  if (shape > 0.0) return es_host(z, shape) * shape * (-z / s);
  const double g = -shape;
  const double gs = g * s;
  // I1(g s) / s = g (I1(g s) / (g s)), finite as s -> 0
  const double i1_over = gs > 1e-8 ? bessel_i1_host(gs) / gs : 0.5;
  return -g * g * z * i1_over / bessel_i0_host(g);
}

// Per-tap polynomials in u = 2 v - 1, v = i0 - t + W/2 in [0, 1) (tap d sits at
// z = (v + d - W/2) 2 / W): Chebyshev interpolation of f(d, z) at deg + 1 nodes,
// converted to monomial coefficients (ascending).  Returns the largest deviation on
// a fine sample.
template <typename F>
double fit_tap_poly(int W, int deg, const F &f, std::vector<double> &coef) {
  coef.assign((size_t)W * (deg + 1), 0.0);
  double maxerr = 0.0;
  const int n = deg + 1;
  for (int d = 0; d < W; ++d) {
    std::vector<double> cheb(n, 0.0), yn(n), un(n);
    for (int i = 0; i < n; ++i) {
      un[i] = std::cos(M_PI * (i + 0.5) / n);
      yn[i] = f(d, ((0.5 * (un[i] + 1.0)) + d - 0.5 * W) * 2.0 / W);
    }
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += yn[i] * std::cos(j * M_PI * (i + 0.5) / n);
      cheb[j] = (j == 0 ? 1.0 : 2.0) * s / n;
    }
    // Chebyshev -> monomial: T_0 = 1, T_1 = u, T_{j+1} = 2 u T_j - T_{j-1}
    std::vector<std::vector<double>> Tm(n, std::vector<double>(n, 0.0));
    Tm[0][0] = 1.0;
    if (n > 1) Tm[1][1] = 1.0;
    for (int j = 1; j + 1 < n; ++j)
      for (int k = 0; k < n; ++k) {
        double v = -Tm[j - 1][k];
        if (k > 0) v += 2.0 * Tm[j][k - 1];
        Tm[j + 1][k] = v;
      }
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) coef[(size_t)d * n + k] += cheb[j] * Tm[j][k];
    for (int i = 0; i <= 2000; ++i) {
      const double v = i / 2000.0, u = 2.0 * v - 1.0;
      double acc = coef[(size_t)d * n + deg];
      for (int k = deg - 1; k >= 0; --k) acc = acc * u + coef[(size_t)d * n + k];
      maxerr = std::max(maxerr, std::fabs(acc - f(d, (v + d - 0.5 * W) * 2.0 / W)));
    }
  }
  return maxerr;
}

// The kernel's taps as polynomials (the forward and both adjoints).
double fit_es_poly(int W, double beta, int deg, std::vector<double> &coef) {
  return fit_tap_poly(W, deg, [&](int, double z) { return kernel_host(z, beta); }, coef);
}

// Largest deviation of the fitted taps' derivatives with respect to the fine coordinate t,
// -2 dP_d/du (u = 2 v - 1, v = i0 - t + W/2), from d/dt psi((i0 + d - t) 2 / W) = -(2 / W) psi'(z).
double tap_deriv_error(int W, double beta, int deg, const std::vector<double> &coef) {
  double maxerr = 0.0;
  for (int d = 0; d < W; ++d) {
    const double *c = coef.data() + (size_t)d * (deg + 1);
    for (int i = 0; i <= 2000; ++i) {
      const double v = i / 2000.0, u = 2.0 * v - 1.0;
      double dp = deg * c[deg];
      for (int k = deg - 1; k >= 1; --k) dp = dp * u + k * c[k];
      const double want = -(2.0 / W) * kernel_deriv_host((v + d - 0.5 * W) * 2.0 / W, beta);
      maxerr = std::max(maxerr, std::fabs(-2.0 * dp - want));
    }
  }
  return maxerr;
}

int64_t alloc_cap_bytes() {
  const char *s = std::getenv("ENUFFT_ALLOC_CAP_MB");
  if (!s || !*s) return -1;
  return (int64_t)(std::atof(s) * 1048576.0);
}

enufft_status dev_alloc(enufft_plan_t p, void **ptr, size_t bytes, const char *what) {
  *ptr = nullptr;
  if (bytes == 0) bytes = 16;
  const int64_t cap = alloc_cap_bytes();
  if (cap >= 0 && p->workspace_bytes + (int64_t)bytes > cap)
    return fail(p, ENUFFT_ENOMEM, std::string("workspace over ENUFFT_ALLOC_CAP_MB while allocating ") + what);
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    return fail(p, ENUFFT_ENOMEM, std::string("hipMalloc failed for ") + what + ": " + hipGetErrorString(e));
  }
  p->allocations.push_back(*ptr);
  p->workspace_bytes += (int64_t)bytes;
  return ENUFFT_OK;
}

template <typename T>
std::vector<T> cast_vec(const std::vector<double> &v) {
  return std::vector<T>(v.begin(), v.end());
}

void free_plan(enufft_plan_t p) {
  if (!p) return;
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  for (void *a : p->allocations) (void)hipFree(a);
  for (size_t i = 0; i < p->tim.start.size(); ++i) {
    (void)hipEventDestroy(p->tim.start[i]);
    (void)hipEventDestroy(p->tim.stop[i]);
  }
  delete p;
}

bool check_gfx950(std::string *name) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
  *name = prop.gcnArchName;
  return std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
}

}  // namespace

// ---------------------------------------------------------------------- scheduling

namespace enufft {

enufft_status autotune(enufft_plan_t p);

// Free one workspace allocation made by dev_alloc (no-op for NULL).
void dev_release(enufft_plan_t p, void **ptr, size_t bytes) {
  if (!*ptr) return;
  for (auto it = p->allocations.begin(); it != p->allocations.end(); ++it)
    if (*it == *ptr) { p->allocations.erase(it); break; }
  (void)hipFree(*ptr);
  *ptr = nullptr;
  p->workspace_bytes -= (int64_t)(bytes == 0 ? 16 : bytes);
}

// Forward work lists.  Batched: target chunk size T keeps roughly two items per
// resident workgroup so the largest cells do not leave CUs idle; cells above T
// are cut into near-equal chunks whose partial grids are merged; ordered by
// decreasing size (longest first).  Per-cell loop: one launch per cell, the
// cell cut into chunks of at least kPercellChunkMin points so that a cell's
// launch occupies up to every resident workgroup (below that size a chunk's
// fixed costs, zeroing, folding and writing a whole grid, outweigh its points).
constexpr int64_t kPercellChunkMin = 4096;

void build_fwd_schedule(enufft_plan_t p, int slots) {
  const int64_t Q = p->n_points;
  const int64_t per = (int64_t)p->fwd_items_per_slot * std::max(1, slots);
  const int64_t T = std::max<int64_t>(p->fwd_chunk_min, (Q + per - 1) / per);
  p->fwd_items.clear();
  p->fwd_items_cell.clear();
  p->fwd_cell_first.assign(p->n_cells + 1, 0);
  int64_t slot = 0, nsplit = 0, pc_slots = 1;
  for (int64_t c = 0; c < p->n_cells; ++c) {
    const int64_t a = p->offsets[c], b = p->offsets[c + 1];
    const int64_t q = b - a;
    // batched schedule: chunks of about T points, every split cell its own partial slots
    const int64_t nch = std::max<int64_t>(1, (q + T - 1) / T);
    if (nch == 1) {
      p->fwd_items.push_back(FwdItem{a, b, (int32_t)c, 1, -1, -1});
    } else {
      ++nsplit;
      for (int64_t i = 0; i < nch; ++i) {
        const int64_t s = a + q * i / nch, e = a + q * (i + 1) / nch;
        p->fwd_items.push_back(FwdItem{s, e, (int32_t)c, (int32_t)nch, (int32_t)(slot + i), (int32_t)slot});
      }
      slot += nch;
    }
    // per-cell loop: a launch holds one cell, so the cell alone is split over the
    // resident workgroups (chunks of at least kPercellChunkMin points); launches
    // follow one another on the stream, so every cell reuses partial slots 0..n-1
    const int64_t tc = std::max<int64_t>(kPercellChunkMin, (q + slots - 1) / std::max(1, slots));
    const int64_t ncc = std::max<int64_t>(1, (q + tc - 1) / tc);
    p->fwd_cell_first[c] = (int64_t)p->fwd_items_cell.size();
    for (int64_t i = 0; i < ncc; ++i) {
      const int64_t s = a + q * i / ncc, e = a + q * (i + 1) / ncc;
      p->fwd_items_cell.push_back(ncc == 1 ? FwdItem{s, e, (int32_t)c, 1, -1, -1}
                                           : FwdItem{s, e, (int32_t)c, (int32_t)ncc, (int32_t)i, 0});
    }
    pc_slots = std::max(pc_slots, ncc);
  }
  p->fwd_cell_first[p->n_cells] = (int64_t)p->fwd_items_cell.size();
  std::stable_sort(p->fwd_items.begin(), p->fwd_items.end(), [](const FwdItem &x, const FwdItem &y) {
    return (x.end - x.begin) > (y.end - y.begin);
  });
  p->n_slots = slot;
  p->n_split = nsplit;
  p->n_partial = std::max(slot, pc_slots);
}

// Forward workgroup size (256, 512 or 1024 threads): LDS footprint and the
// resident workgroups per CU that size the schedule.
enufft_status set_fwd_threads(enufft_plan_t p, int threads, size_t lds_limit) {
  if (threads != 256 && threads != 512 && threads != 1024)
    return fail(p, ENUFFT_EINVAL, "forward threads must be 256, 512 or 1024");
  const int vp = fwd_variant_pitch(p->geom, p->es);
  // FP32 sums in LDS exist only for the FP32 polynomial builds
  if (p->prec == ENUFFT_F64 || vp == 0) p->fwd_acc = 8;
  const size_t lds = fwd_lds_bytes(p->geom, p->W, threads, (size_t)p->fwd_acc);
  if (lds > lds_limit) return fail(p, ENUFFT_EUNSUPPORTED, "enufft_plan: fine grid does not fit in LDS at this precision");
  int per_cu = 0;
  hipError_t e = (p->prec == ENUFFT_F64) ? fwd_occupancy<double>(p->W, threads, vp, p->fwd_acc, lds, &per_cu)
                                         : fwd_occupancy<float>(p->W, threads, vp, p->fwd_acc, lds, &per_cu);
  if (e != hipSuccess) return hip_fail(p, e, "occupancy query");
  if (per_cu < 1) return fail(p, ENUFFT_EDEVICE, "forward kernel cannot be resident");
  p->fwd_threads = threads;
  p->fwd_lds = lds;
  p->fwd_slots = p->n_cu * per_cu;
  return ENUFFT_OK;
}

// (Re)build the forward schedule for the plan's launch-shape parameters and
// replace its device copies (item lists and the partial grids of split cells).
enufft_status install_fwd_schedule(enufft_plan_t p) {
  dev_release(p, &p->d_fwd_items, std::max<size_t>(1, p->fwd_items.size()) * sizeof(FwdItem));
  dev_release(p, &p->d_fwd_items_cell, std::max<size_t>(1, p->fwd_items_cell.size()) * sizeof(FwdItem));
  dev_release(p, &p->d_partial, std::max<int64_t>(1, p->n_partial) * (size_t)p->n1 * p->n2 * p->elem);
  build_fwd_schedule(p, p->fwd_slots);
  p->fwd_blocks = (int)std::min<int64_t>((int64_t)p->fwd_slots, std::max<int64_t>(1, (int64_t)p->fwd_items.size()));
  enufft_status st = dev_alloc(p, &p->d_fwd_items, std::max<size_t>(1, p->fwd_items.size()) * sizeof(FwdItem),
                               "forward items");
  if (st == ENUFFT_OK)
    st = dev_alloc(p, &p->d_fwd_items_cell, std::max<size_t>(1, p->fwd_items_cell.size()) * sizeof(FwdItem),
                   "forward items by cell");
  if (st == ENUFFT_OK)
    st = dev_alloc(p, &p->d_partial, std::max<int64_t>(1, p->n_partial) * (size_t)p->n1 * p->n2 * p->elem,
                   "partial grids");
  if (st != ENUFFT_OK) return st;
  hipError_t e = hipSuccess;
  if (!p->fwd_items.empty())
    e = hipMemcpy(p->d_fwd_items, p->fwd_items.data(), p->fwd_items.size() * sizeof(FwdItem), hipMemcpyHostToDevice);
  if (e == hipSuccess && !p->fwd_items_cell.empty())
    e = hipMemcpy(p->d_fwd_items_cell, p->fwd_items_cell.data(), p->fwd_items_cell.size() * sizeof(FwdItem),
                  hipMemcpyHostToDevice);
  return e == hipSuccess ? ENUFFT_OK : hip_fail(p, e, "upload forward items");
}

}  // namespace enufft

// ---------------------------------------------------------------------- C ABI

extern "C" {

const char *enufft_version(void) { return "enufft-gfx950 0.1"; }

const char *enufft_last_error(enufft_plan_t p) {
  return p ? p->last_error.c_str() : g_thread_error.c_str();
}

enufft_status enufft_default_opts(enufft_opts *o) {
  if (!o) return fail(nullptr, ENUFFT_EINVAL, "enufft_default_opts: null opts");
  o->n_modes[0] = 64;
  o->n_modes[1] = 64;
  o->sigma = 2.0;
  o->eps = 1e-5;
  o->precision = ENUFFT_F32;
  o->window_kind = ENUFFT_WIN_HANN_RADIAL;
  o->scale = 1.0;
  o->autotune = 0;
  o->kernel_width = 0;
  o->kernel_kind = ENUFFT_KERNEL_ES;
  return ENUFFT_OK;
}

enufft_status enufft_plan(enufft_plan_t *out, int64_t n_cells, const int64_t *cell_offsets,
                          const enufft_window *windows, const enufft_opts *opts, void *hip_stream) {
  if (!out) return fail(nullptr, ENUFFT_EINVAL, "enufft_plan: null output pointer");
  *out = nullptr;
  if (!opts) return fail(nullptr, ENUFFT_EINVAL, "enufft_plan: null opts");
  if (n_cells < 0 || n_cells > (int64_t)INT32_MAX)
    return fail(nullptr, ENUFFT_EINVAL, "enufft_plan: n_cells out of range");
  if (!cell_offsets) return fail(nullptr, ENUFFT_EINVAL, "enufft_plan: null cell_offsets");
  if (cell_offsets[0] != 0) return fail(nullptr, ENUFFT_EINVAL, "enufft_plan: cell_offsets[0] must be 0");
  for (int64_t c = 0; c < n_cells; ++c)
    if (cell_offsets[c + 1] < cell_offsets[c])
      return fail(nullptr, ENUFFT_EINVAL, "enufft_plan: cell_offsets must be non-decreasing");
  const int N1 = opts->n_modes[0], N2 = opts->n_modes[1];
  if (N1 < 1 || N2 < 1) return fail(nullptr, ENUFFT_EINVAL, "enufft_plan: n_modes must be >= 1");
  if (opts->precision != ENUFFT_F32 && opts->precision != ENUFFT_F64)
    return fail(nullptr, ENUFFT_EINVAL, "enufft_plan: unknown precision");
  if (opts->window_kind != ENUFFT_WIN_NONE && opts->window_kind != ENUFFT_WIN_HANN_RADIAL)
    return fail(nullptr, ENUFFT_EINVAL, "enufft_plan: unknown window kind");
  if (opts->autotune < 0 || opts->autotune > 2)
    return fail(nullptr, ENUFFT_EINVAL, "enufft_plan: autotune must be 0, 1 or 2");
  if (!(opts->sigma >= 1.25) || !(opts->sigma <= 16.0))
    return fail(nullptr, ENUFFT_EINVAL, "enufft_plan: sigma must be in [1.25, 16]");
  if (!(opts->eps > 0.0) || !(opts->eps < 1.0))
    return fail(nullptr, ENUFFT_EINVAL, "enufft_plan: eps must be in (0, 1)");
  if (opts->precision == ENUFFT_F32 && opts->eps < 1e-6)
    return fail(nullptr, ENUFFT_EEPS, "enufft_plan: eps below 1e-6 is not attainable in FP32");
  if (opts->precision == ENUFFT_F64 && opts->eps < 1e-13)
    return fail(nullptr, ENUFFT_EEPS, "enufft_plan: eps below 1e-13 is not attainable in FP64");
  if (!std::isfinite(opts->scale)) return fail(nullptr, ENUFFT_EINVAL, "enufft_plan: scale must be finite");
  if (opts->kernel_width < 0 || opts->kernel_width > 16)
    return fail(nullptr, ENUFFT_EINVAL, "enufft_plan: kernel_width must be in [0, 16]");
  if (opts->kernel_kind != ENUFFT_KERNEL_ES && opts->kernel_kind != ENUFFT_KERNEL_KB_MIRT &&
      opts->kernel_kind != ENUFFT_KERNEL_KB_FESSLER)
    return fail(nullptr, ENUFFT_EINVAL, "enufft_plan: unknown kernel kind");
  if (opts->window_kind == ENUFFT_WIN_HANN_RADIAL && n_cells > 0) {
    if (!windows) return fail(nullptr, ENUFFT_EINVAL, "enufft_plan: Hann window needs windows");
    for (int64_t c = 0; c < n_cells; ++c)
      if (!(windows[c].radius > 0.0) || !std::isfinite(windows[c].cx) || !std::isfinite(windows[c].cy) ||
          !std::isfinite(windows[c].radius))
        return fail(nullptr, ENUFFT_EINVAL, "enufft_plan: window radius must be > 0 and finite");
  }
  // Fine grid: the smallest power of two >= sigma N (and >= 16); the kernel
  // parameters follow the effective oversampling, and a grid narrower than two
  // kernel widths is widened (which only raises the oversampling).
  int n1 = std::max(16, next_pow2((int)std::ceil(opts->sigma * N1 - 1e-9)));
  int n2 = std::max(16, next_pow2((int)std::ceil(opts->sigma * N2 - 1e-9)));
  const double sigma_eff = std::min((double)n1 / N1, (double)n2 / N2);
  int W;
  double beta;
  kernel_params(opts->eps, sigma_eff, opts->kernel_width, &W, &beta);
  // Kaiser-Bessel: the given width (or the eps-derived one) and its shape gamma, stored
  // negated so the kernels can tell the two kernels apart by the sign
  const bool kb = opts->kernel_kind != ENUFFT_KERNEL_ES;
  if (kb && opts->kernel_width > 0) {
    W = 16;
    for (int c : kWidths)
      if (c >= opts->kernel_width) { W = c; break; }
  }
  if (kb) beta = -kb_gamma(opts->kernel_kind, W);
  n1 = std::max(n1, next_pow2(2 * W));
  n2 = std::max(n2, next_pow2(2 * W));
  // Mode boxes above 64 per axis (or grids above 128) take the large-cell path:
  // the grid lives in HBM and is tiled, each axis at least two tiles wide.
  const bool big = N1 > 64 || N2 > 64 || n1 > 128 || n2 > 128;
  if (big) {
    n1 = std::max(n1, 64);
    n2 = std::max(n2, 64);
    if (n1 > 4096 || n2 > 4096 || (int64_t)n1 * n2 > (int64_t)1 << 22)
      return fail(nullptr, ENUFFT_EUNSUPPORTED,
                  "enufft_plan: fine grid above 4096 per axis or 2^22 cells is not supported");
  }

  // ---- device
  std::string arch;
  if (!check_gfx950(&arch))
    return fail(nullptr, ENUFFT_EDEVICE, "enufft_plan: no gfx950 device (found '" + arch + "')");

  enufft_plan_t p = new enufft_plan_s();
  p->n_cells = n_cells;
  p->n_points = cell_offsets[n_cells];
  p->offsets.assign(cell_offsets, cell_offsets + n_cells + 1);
  p->N1 = N1; p->N2 = N2; p->n1 = n1; p->n2 = n2; p->W = W; p->beta = beta;
  p->sigma = opts->sigma; p->eps = opts->eps; p->scale = opts->scale;
  p->prec = opts->precision; p->window_kind = opts->window_kind;
  p->elem = p->prec == ENUFFT_F64 ? 8 : 4;
  p->stream = (hipStream_t)hip_stream;
  p->opts = *opts;
  p->big = big;
  if (windows) p->windows_host.assign(windows, windows + n_cells);
  Geom &g = p->geom;
  g.n1 = n1; g.n2 = n2; g.N1 = N1; g.N2 = N2;
  g.lo1 = -(N1 / 2); g.lo2 = -(N2 / 2);
  g.K1 = N1 / 2; g.K2 = N2 / 2;
  g.pitch = n1 + 2;

  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) { enufft_status s = hip_fail(p, e, "hipGetDevice"); free_plan(p); return s; }
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, p->device);
  if (e != hipSuccess) { enufft_status s = hip_fail(p, e, "hipGetDeviceProperties"); free_plan(p); return s; }
  p->n_cu = prop.multiProcessorCount;

  // FP32 plans evaluate the kernel as per-tap polynomials when the fit is far
  // below the requested accuracy (it is for the compiled widths 4..8).
  if (p->prec == ENUFFT_F32 && W <= enufft::ES_MAXW) {
    std::vector<double> cf;
    const double err = fit_es_poly(W, beta, enufft::ES_DEG, cf);
    if (err <= std::max(0.1 * opts->eps, 1e-6)) {
      p->es_poly_err = err;
      p->es.on = 1;
      // the mirror taps W/2 .. W - 1 are evaluated from these (psi is even)
      for (size_t i = 0; i < (size_t)(W / 2) * (enufft::ES_DEG + 1); ++i) p->es.c[i] = (float)cf[i];
    }
  }

  // FP64 large-cell plans: the same per-tap form in FP64 (even widths), kept when its fit
  // is at least ten times below the requested accuracy
  if (p->prec == ENUFFT_F64 && big && W % 2 == 0 && W <= enufft::ES64_MAXW) {
    const char *ev = std::getenv("ENUFFT_POLY64");
    if (!(ev && std::atoi(ev) == 0)) {
      std::vector<double> cf;
      const double err = fit_es_poly(W, beta, enufft::ES64_DEG, cf);
      if (err <= 0.1 * opts->eps) {
        p->es_poly_err = err;
        p->es64.on = 1;
        for (size_t i = 0; i < (size_t)(W / 2) * (enufft::ES64_DEG + 1); ++i) p->es64.c[i] = cf[i];
      }
    }
  }

  // Single-grid adjoint: FP32 plans whose kernel takes the polynomial path use one LDS
  // grid per cell with value and derivative taps of a kernel two cells wider (the
  // derivative of the interpolant converges more slowly than the interpolant itself).
  if (p->prec == ENUFFT_F32 && !big && p->es.on && W + 2 <= enufft::ES_MAXW) {
    const char *ev = std::getenv("ENUFFT_ADJ_SINGLE");
    if (!(ev && std::atoi(ev) == 0)) {
      const int Wa = W + 2;
      double ba = 0.0;
      if (kb) {
        ba = -kb_gamma(opts->kernel_kind, Wa);
      } else {
        int Wt = 0;
        kernel_params(opts->eps, sigma_eff, Wa, &Wt, &ba);
        if (Wt != Wa) ba = 0.0;
      }
      std::vector<double> cf;
      const double e0 = ba != 0.0 ? fit_es_poly(Wa, ba, enufft::ES_DEG, cf) : 1.0;
      // the kernel takes the derivative taps from the same polynomials
      const double e1 = ba != 0.0 ? tap_deriv_error(Wa, ba, enufft::ES_DEG, cf) : 1.0;
      if (e0 <= std::max(0.1 * opts->eps, 1e-6) && e1 <= std::max(opts->eps, 1e-5)) {
        p->adj1 = true;
        p->adj1_avail = true;
        p->adj1_W = Wa;
        p->adj1_beta = ba;
        p->adj1_poly_err = e0;
        p->adj1_dpoly_err = e1;
        p->adj1_es.on = 1;
        for (size_t i = 0; i < (size_t)(Wa / 2) * (enufft::ES_DEG + 1); ++i) p->adj1_es.c[i] = (float)cf[i];
      }
    }
  }

  // ---- forward launch shape (threads per workgroup: ENUFFT_FWD_THREADS, or the autotuner)
  enufft_status st = ENUFFT_OK;
  if (!big) {
    int threads = 512;
    if (const char *ev = std::getenv("ENUFFT_FWD_THREADS")) threads = std::atoi(ev);
    if (const char *ev = std::getenv("ENUFFT_FWD_ACC")) p->fwd_acc = std::atoi(ev) == 4 ? 4 : 8;
    if (const char *ev = std::getenv("ENUFFT_FWD_CHUNK_MIN")) p->fwd_chunk_min = std::max(1024LL, std::atoll(ev));
    if (const char *ev = std::getenv("ENUFFT_FWD_ITEMS_PER_SLOT")) p->fwd_items_per_slot = std::max(1, std::atoi(ev));
    st = enufft::set_fwd_threads(p, threads, (size_t)prop.sharedMemPerBlock);
    if (st != ENUFFT_OK) { std::string m = p->last_error; free_plan(p); return fail(nullptr, st, m); }
  }

  // ---- tables (FP64 on the host, rounded to the compute precision)
  const int Kx = g.K1, Ky = g.K2;
  std::vector<double> px = kb ? kb_ft(W, -beta, n1, Kx) : kernel_ft(W, beta, n1, Kx);
  std::vector<double> py = kb ? kb_ft(W, -beta, n2, Ky) : kernel_ft(W, beta, n2, Ky);
  std::vector<double> dx(Kx + 1), dy(Ky + 1), dx1(Kx + 1);
  for (int k = 0; k <= Kx; ++k) dx[k] = opts->scale / px[k];
  for (int k = 0; k <= Kx; ++k) dx1[k] = 1.0 / px[k];
  for (int k = 0; k <= Ky; ++k) dy[k] = 1.0 / py[k];
  std::vector<double> adx, ady;
  if (p->adj1) {
    const int Wa = p->adj1_W;
    const double ba = p->adj1_beta;
    std::vector<double> qx = kb ? kb_ft(Wa, -ba, n1, Kx) : kernel_ft(Wa, ba, n1, Kx);
    std::vector<double> qy = kb ? kb_ft(Wa, -ba, n2, Ky) : kernel_ft(Wa, ba, n2, Ky);
    for (int k = 0; k <= Kx; ++k) adx.push_back(opts->scale / qx[k]);
    for (int k = 0; k <= Ky; ++k) ady.push_back(1.0 / qy[k]);
  }
  std::vector<double> tw1(2 * n1), tw2(2 * n2);
  for (int j = 0; j < n1; ++j) { tw1[2 * j] = std::cos(2 * M_PI * j / n1); tw1[2 * j + 1] = -std::sin(2 * M_PI * j / n1); }
  for (int j = 0; j < n2; ++j) { tw2[2 * j] = std::cos(2 * M_PI * j / n2); tw2[2 * j + 1] = -std::sin(2 * M_PI * j / n2); }

#define ALLOC(ptr, bytes, what)                                              \
  do {                                                                       \
    st = dev_alloc(p, (void **)&(ptr), (bytes), what);                       \
    if (st != ENUFFT_OK) { std::string m_ = p->last_error; free_plan(p); return fail(nullptr, st, m_); } \
  } while (0)
#define UPLOAD(dst, src, bytes, what)                                        \
  do {                                                                       \
    hipError_t e_ = hipMemcpy((dst), (src), (bytes), hipMemcpyHostToDevice); \
    if (e_ != hipSuccess) { st = hip_fail(p, e_, what); std::string m_ = p->last_error; free_plan(p); return fail(nullptr, st, m_); } \
  } while (0)

  auto upload_table = [&](void **dst, const std::vector<double> &v, const char *what) -> enufft_status {
    enufft_status s2 = dev_alloc(p, dst, v.size() * p->elem, what);
    if (s2 != ENUFFT_OK) return s2;
    hipError_t e2;
    if (p->prec == ENUFFT_F64) {
      e2 = hipMemcpy(*dst, v.data(), v.size() * 8, hipMemcpyHostToDevice);
    } else {
      std::vector<float> f = cast_vec<float>(v);
      e2 = hipMemcpy(*dst, f.data(), f.size() * 4, hipMemcpyHostToDevice);
    }
    return e2 == hipSuccess ? ENUFFT_OK : hip_fail(p, e2, what);
  };
  for (auto &tb : {std::make_pair(&p->d_decon_x, &dx), std::make_pair(&p->d_decon_y, &dy),
                   std::make_pair(&p->d_decon_x1, &dx1),
                   std::make_pair(&p->d_tw1, &tw1), std::make_pair(&p->d_tw2, &tw2)}) {
    st = upload_table(tb.first, *tb.second, "tables");
    if (st != ENUFFT_OK) { std::string m = p->last_error; free_plan(p); return fail(nullptr, st, m); }
  }
  if (p->adj1) {
    st = upload_table(&p->d_adj1_decon_x, adx, "adjoint tables");
    if (st == ENUFFT_OK) st = upload_table(&p->d_adj1_decon_y, ady, "adjoint tables");
    if (st != ENUFFT_OK) { std::string m = p->last_error; free_plan(p); return fail(nullptr, st, m); }
  }

  std::vector<double> win(3 * std::max<int64_t>(1, n_cells), 0.0);
  for (int64_t c = 0; c < n_cells; ++c) {
    if (windows) { win[3 * c] = windows[c].cx; win[3 * c + 1] = windows[c].cy; win[3 * c + 2] = windows[c].radius; }
  }
  ALLOC(p->d_windows, win.size() * sizeof(double), "windows");
  UPLOAD(p->d_windows, win.data(), win.size() * sizeof(double), "upload windows");
  st = big ? enufft::big_prepare(p) : enufft::install_fwd_schedule(p);
  if (st != ENUFFT_OK) { std::string m = p->last_error; free_plan(p); return fail(nullptr, st, m); }
  ALLOC(p->d_counters, 16 * sizeof(int), "counters");
  ALLOC(p->d_cell_counters, std::max<int64_t>(1, n_cells) * sizeof(int), "cell counters");
  e = hipMemset(p->d_counters, 0, 16 * sizeof(int));
  if (e == hipSuccess) e = hipMemset(p->d_cell_counters, 0, std::max<int64_t>(1, n_cells) * sizeof(int));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) { st = hip_fail(p, e, "zero counters"); std::string m = p->last_error; free_plan(p); return fail(nullptr, st, m); }
#undef ALLOC
#undef UPLOAD
  if (opts->autotune && !big) {
    st = enufft::autotune(p);
    if (st != ENUFFT_OK) { std::string m = p->last_error; free_plan(p); return fail(nullptr, st, m); }
  }
  *out = p;
  return ENUFFT_OK;
}

enufft_status enufft_set_stream(enufft_plan_t p, void *hip_stream) {
  if (!p) return fail(nullptr, ENUFFT_EINVAL, "enufft_set_stream: null plan");
  p->stream = (hipStream_t)hip_stream;
  return ENUFFT_OK;
}

enufft_status enufft_destroy(enufft_plan_t p) {
  if (!p) return ENUFFT_OK;
  if (p->stream || true) (void)hipStreamSynchronize(p->stream);
  free_plan(p);
  return ENUFFT_OK;
}

enufft_status enufft_get_info(enufft_plan_t p, enufft_plan_info *info) {
  if (!p || !info) return fail(p, ENUFFT_EINVAL, "enufft_get_info: null argument");
  std::memset(info, 0, sizeof(*info));
  info->n_modes[0] = p->N1; info->n_modes[1] = p->N2;
  info->grid[0] = p->n1; info->grid[1] = p->n2;
  info->kernel_width = p->W;
  info->beta = std::fabs(p->beta);
  info->kernel_kind = p->opts.kernel_kind;
  info->adj_kernel_width = p->adj1 ? p->adj1_W : 0;
  info->n_cells = p->n_cells;
  info->n_points = p->n_points;
  info->n_items_fwd = (int64_t)p->fwd_items.size();
  info->n_split_cells = p->n_split;
  info->n_items_adj = (int64_t)p->adj_items.size();
  info->adj_bands = p->adj_bands;
  info->fwd_threads = p->fwd_threads; info->fwd_blocks = p->fwd_blocks;
  info->adj_threads = p->adj_threads; info->adj_blocks = p->adj_blocks;
  info->workspace_bytes = p->workspace_bytes;
  info->kernel_poly_err = p->es_poly_err;
  info->tuned = p->tuned;
  info->tune_cache_hit = p->tune_cache_hit;
  info->fwd_chunk_min = p->fwd_chunk_min;
  info->fwd_items_per_slot = p->fwd_items_per_slot;
  info->adj_items_per_slot = p->adj_items_per_slot;
  info->adj_band_mult = p->adj_band_mult;
  info->fwd_acc = p->big ? 8 : p->fwd_acc;
  info->tune_fwd_ms = p->tune_fwd_ms;
  info->tune_adj_ms = p->tune_adj_ms;
  return ENUFFT_OK;
}

enufft_status enufft_set_timing(enufft_plan_t p, int32_t enable) {
  if (!p) return fail(nullptr, ENUFFT_EINVAL, "enufft_set_timing: null plan");
  p->timing = enable != 0;
  return ENUFFT_OK;
}

enufft_status enufft_get_timing(enufft_plan_t p, double *out8) {
  if (!p || !out8) return fail(p, ENUFFT_EINVAL, "enufft_get_timing: null argument");
  for (int i = 0; i < 8; ++i) out8[i] = 0.0;
  enufft_status st = ENUFFT_OK;
  for (size_t i = 0; i < p->tim.start.size(); ++i) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(p->tim.stop[i]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p->tim.start[i], p->tim.stop[i]);
    if (e != hipSuccess && st == ENUFFT_OK) st = hip_fail(p, e, "event timing");
    out8[p->tim.kind[i]] += ms;
    out8[4 + p->tim.kind[i]] += 1.0;
    (void)hipEventDestroy(p->tim.start[i]);
    (void)hipEventDestroy(p->tim.stop[i]);
  }
  p->tim.start.clear(); p->tim.stop.clear(); p->tim.kind.clear();
  return st;
}

}  // extern "C"

// ---------------------------------------------------------------------- launches

namespace enufft {

enufft_status record_start(enufft_plan_t p, int kind, hipEvent_t *ev) {
  *ev = nullptr;
  if (!p->timing) return ENUFFT_OK;
  HIP_TRY(p, hipEventCreate(ev), "hipEventCreate");
  HIP_TRY(p, hipEventRecord(*ev, p->stream), "hipEventRecord");
  (void)kind;
  return ENUFFT_OK;
}
enufft_status record_stop(enufft_plan_t p, int kind, hipEvent_t start) {
  if (!p->timing || !start) return ENUFFT_OK;
  hipEvent_t ev;
  HIP_TRY(p, hipEventCreate(&ev), "hipEventCreate");
  HIP_TRY(p, hipEventRecord(ev, p->stream), "hipEventRecord");
  p->tim.start.push_back(start);
  p->tim.stop.push_back(ev);
  p->tim.kind.push_back(kind);
  return ENUFFT_OK;
}

// n / (2 pi) as hi + lo in T (from extended precision on the host).
template <typename T>
void split_scale(int n, T *hi, T *lo) {
  const long double s = (long double)n / (2.0L * 3.141592653589793238462643383279502884L);
  *hi = (T)s;
  *lo = (T)(s - (long double)*hi);
}
template void split_scale<float>(int, float *, float *);
template void split_scale<double>(int, double *, double *);

template <typename T>
FwdArgs<T> make_fwd_args(enufft_plan_t p, const void *x, const void *y, const void *h, const void *w, void *f) {
  FwdArgs<T> a{};
  a.x = (const T *)x; a.y = (const T *)y; a.h = (const T *)h; a.w = (const T *)w;
  a.f = (T *)f;
  {
    const size_t al = 4 * sizeof(T);
    a.vec4 = ((uintptr_t)x % al == 0 && (uintptr_t)y % al == 0 && (uintptr_t)h % al == 0 &&
              (uintptr_t)w % al == 0) ? 1 : 0;
  }
  a.items = (const FwdItem *)p->d_fwd_items;
  a.n_items = (int64_t)p->fwd_items.size();
  a.item_base = 0;
  a.work_counter = p->d_counters + 0;
  a.done_counter = p->d_counters + 1;
  a.cell_counters = p->d_cell_counters;
  a.partial = (T *)p->d_partial;
  a.windows = (const double *)p->d_windows;
  a.window_kind = p->window_kind;
  a.decon_x = (const T *)p->d_decon_x; a.decon_y = (const T *)p->d_decon_y;
  a.tw1 = (const T *)p->d_tw1; a.tw2 = (const T *)p->d_tw2;
  a.beta = (T)p->beta;
  split_scale<T>(p->n1, &a.s1_hi, &a.s1_lo);
  split_scale<T>(p->n2, &a.s2_hi, &a.s2_lo);
  a.acc = p->fwd_acc;
  a.es = p->es;
  a.g = p->geom;
  return a;
}

template FwdArgs<float> make_fwd_args<float>(enufft_plan_t, const void *, const void *, const void *, const void *,
                                             void *);
template FwdArgs<double> make_fwd_args<double>(enufft_plan_t, const void *, const void *, const void *, const void *,
                                               void *);

enufft_status cells_largest_first(enufft_plan_t p, const int32_t **order) {
  if (!p->cell_order) {
    std::vector<int32_t> o((size_t)std::max<int64_t>(1, p->n_cells), 0);
    for (int64_t c = 0; c < p->n_cells; ++c) o[c] = (int32_t)c;
    std::stable_sort(o.begin(), o.begin() + p->n_cells, [&](int32_t u, int32_t v) {
      return p->offsets[u + 1] - p->offsets[u] > p->offsets[v + 1] - p->offsets[v];
    });
    void *d = nullptr;
    enufft_status st = dev_alloc(p, &d, o.size() * sizeof(int32_t), "cell order");
    if (st != ENUFFT_OK) return st;
    hipError_t e = hipMemcpy(d, o.data(), o.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      dev_release(p, &d, o.size() * sizeof(int32_t));
      return hip_fail(p, e, "cell order upload");
    }
    p->cell_order = d;
  }
  *order = (const int32_t *)p->cell_order;
  return ENUFFT_OK;
}

enufft_status check_plan(enufft_plan_t p, const char *fn) {
  if (!p) return fail(nullptr, ENUFFT_EINVAL, std::string(fn) + ": null plan");
  if (p->faulted) return fail(p, ENUFFT_ESTATE, std::string(fn) + ": plan unusable after a device fault");
  return ENUFFT_OK;
}

}  // namespace enufft

extern "C" enufft_status enufft_type1_batched(enufft_plan_t p, const void *x, const void *y, const void *h,
                                              const void *w, void *f) {
  enufft_status st = enufft::check_plan(p, "enufft_type1_batched");
  if (st != ENUFFT_OK) return st;
  if (p->n_cells == 0) return ENUFFT_OK;
  if (!f) return fail(p, ENUFFT_EINVAL, "enufft_type1_batched: null f");
  if (p->n_points > 0 && (!x || !y || !h || !w))
    return fail(p, ENUFFT_EINVAL, "enufft_type1_batched: null point array");
  hipEvent_t ev;
  st = enufft::record_start(p, 0, &ev);
  if (st != ENUFFT_OK) return st;
  if (p->big) {
    st = enufft::big_type1(p, x, y, h, w, f, 0, p->n_cells);
    if (st != ENUFFT_OK) return st;
    return enufft::record_stop(p, 0, ev);
  }
  hipError_t e;
  if (p->prec == ENUFFT_F64) {
    auto a = enufft::make_fwd_args<double>(p, x, y, h, w, f);
    e = enufft::launch_fwd<double>(a, p->W, p->fwd_blocks, p->fwd_threads, p->fwd_lds, p->stream);
  } else {
    auto a = enufft::make_fwd_args<float>(p, x, y, h, w, f);
    e = enufft::launch_fwd<float>(a, p->W, p->fwd_blocks, p->fwd_threads, p->fwd_lds, p->stream);
  }
  if (e != hipSuccess) return hip_fail(p, e, "forward launch");
  return enufft::record_stop(p, 0, ev);
}

namespace enufft {
enufft_status percell_fwd(enufft_plan_t p, int64_t c, const void *x, const void *y, const void *h, const void *w,
                          void *f) {
  if (p->big) return big_type1(p, x, y, h, w, f, c, c + 1);
  const int64_t first = p->fwd_cell_first[c], cnt = p->fwd_cell_first[c + 1] - first;
  if (cnt == 0) return ENUFFT_OK;
  hipError_t e;
  if (p->prec == ENUFFT_F64) {
    auto a = make_fwd_args<double>(p, x, y, h, w, f);
    a.items = (const FwdItem *)p->d_fwd_items_cell;
    a.n_items = (int64_t)p->fwd_items_cell.size();
    a.item_base = first;
    a.work_counter = nullptr; a.done_counter = nullptr;
    e = launch_fwd<double>(a, p->W, (int)cnt, p->fwd_threads, p->fwd_lds, p->stream);
  } else {
    auto a = make_fwd_args<float>(p, x, y, h, w, f);
    a.items = (const FwdItem *)p->d_fwd_items_cell;
    a.n_items = (int64_t)p->fwd_items_cell.size();
    a.item_base = first;
    a.work_counter = nullptr; a.done_counter = nullptr;
    e = launch_fwd<float>(a, p->W, (int)cnt, p->fwd_threads, p->fwd_lds, p->stream);
  }
  if (e != hipSuccess) return hip_fail(p, e, "per-cell forward launch");
  return ENUFFT_OK;
}
}  // namespace enufft

// Defined with the EMS kernel.
namespace enufft {
enufft_status ems_launch(enufft_plan_t p, const void *f, const enufft_ems_params *prm, const double *mode_weight,
                         uint8_t *keep, int32_t *k_star, double *stats, int64_t cell_begin, int64_t cell_count);
enufft_status ems_validate(enufft_plan_t p, const void *f, const enufft_ems_params *prm, uint8_t *keep,
                           int32_t *k_star, double *stats);
}  // namespace enufft

extern "C" enufft_status enufft_percell_loop(enufft_plan_t p, const void *x, const void *y, const void *h,
                                             const void *w, void *f, const enufft_ems_params *prm,
                                             const double *mode_weight, uint8_t *keep, int32_t *k_star,
                                             double *stats) {
  enufft_status st = enufft::check_plan(p, "enufft_percell_loop");
  if (st != ENUFFT_OK) return st;
  if (p->n_cells == 0) return ENUFFT_OK;
  if (!f) return fail(p, ENUFFT_EINVAL, "enufft_percell_loop: null f");
  if (p->n_points > 0 && (!x || !y || !h || !w)) return fail(p, ENUFFT_EINVAL, "enufft_percell_loop: null point array");
  const bool with_ems = prm != nullptr;
  if (with_ems) {
    st = enufft::ems_validate(p, f, prm, keep, k_star, stats);
    if (st != ENUFFT_OK) return st;
  }
  for (int64_t c = 0; c < p->n_cells; ++c) {
    st = enufft::percell_fwd(p, c, x, y, h, w, f);
    if (st != ENUFFT_OK) return st;
    if (with_ems) {
      st = enufft::ems_launch(p, f, prm, mode_weight, keep, k_star, stats, c, 1);
      if (st != ENUFFT_OK) return st;
    }
  }
  return ENUFFT_OK;
}

// ---------------------------------------------------------------------- graph

namespace {
void key_append(std::vector<uint8_t> &k, const void *ptr, size_t n) {
  const uint8_t *b = (const uint8_t *)ptr;
  k.insert(k.end(), b, b + n);
}
}  // namespace

// Type-1 + EMS as one captured graph.  The two launches (the persistent
// forward kernel and the per-cell EMS kernel) are recorded once on a private
// stream and replayed on the plan's stream; nothing in them needs a memset
// (the forward's work counters reset themselves), so replays are independent.
// A call with different pointers or EMS parameters re-captures.
extern "C" enufft_status enufft_forward_graph(enufft_plan_t p, const void *x, const void *y, const void *h,
                                              const void *w, void *f, const enufft_ems_params *prm,
                                              const double *mode_weight, uint8_t *keep, int32_t *k_star,
                                              double *stats) {
  enufft_status st = enufft::check_plan(p, "enufft_forward_graph");
  if (st != ENUFFT_OK) return st;
  if (p->n_cells == 0) return ENUFFT_OK;
  if (!f) return fail(p, ENUFFT_EINVAL, "enufft_forward_graph: null f");
  if (p->n_points > 0 && (!x || !y || !h || !w)) return fail(p, ENUFFT_EINVAL, "enufft_forward_graph: null point array");
  st = enufft::ems_validate(p, f, prm, keep, k_star, stats);
  if (st != ENUFFT_OK) return st;
  {   // unit tables are built (allocated, uploaded) outside the capture
    enufft::UnitTable *ut = nullptr;
    st = enufft::ems_units(p, prm, &ut);
    if (st != ENUFFT_OK) return st;
  }
  std::vector<uint8_t> key;
  const void *ptrs[] = {x, y, h, w, f, mode_weight, keep, k_star, stats};
  key_append(key, ptrs, sizeof(ptrs));
  key_append(key, prm, sizeof(*prm));
  if (!p->graph_exec || key != p->graph_key) {
    if (!p->capture_stream) HIP_TRY(p, hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking), "capture stream");
    if (p->graph_exec) { (void)hipGraphExecDestroy(p->graph_exec); p->graph_exec = nullptr; }
    if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
    HIP_TRY(p, hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    hipStream_t user = p->stream;
    const bool timing = p->timing;
    p->stream = p->capture_stream;
    p->timing = false;
    enufft_status s1 = enufft_type1_batched(p, x, y, h, w, f);
    enufft_status s2 = s1 == ENUFFT_OK ? enufft::ems_launch(p, f, prm, mode_weight, keep, k_star, stats, 0, p->n_cells)
                                       : s1;
    p->stream = user;
    p->timing = timing;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->capture_stream, &g);
    if (s2 != ENUFFT_OK) { if (g) (void)hipGraphDestroy(g); return s2; }
    if (e != hipSuccess) return hip_fail(p, e, "end capture");
    p->graph = g;
    HIP_TRY(p, hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0), "graph instantiate");
    p->graph_key = key;
    ++p->graph_captures;
  }
  hipEvent_t ev;
  st = enufft::record_start(p, 3, &ev);
  if (st != ENUFFT_OK) return st;
  HIP_TRY(p, hipGraphLaunch(p->graph_exec, p->stream), "graph launch");
  ++p->graph_launches;
  return enufft::record_stop(p, 3, ev);
}
