// Plan-time autotuner: timed trials of the launch-shape parameters on
// synthetic points with the plan's own cell sizes, and an on-disk cache of the
// choice keyed by device, transform shape and batch layout.
//
// Tuned: the forward workgroup size, the smallest forward work item and the
// number of work items per resident workgroup (how finely the batched launch
// cuts large cells), and the adjoint's items per workgroup and row-band count.
// The kernel width is not tuned: it is the narrowest that meets eps, and a
// wider one only adds work.
#include <hip/hip_runtime.h>

#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "device_common.h"
#include "launch.h"
#include "plan.h"

namespace enufft {
namespace {

__device__ __forceinline__ uint32_t mix32(uint64_t v) {
  v ^= v >> 33;
  v *= 0xff51afd7ed558ccdULL;
  v ^= v >> 33;
  v *= 0xc4ceb9fe1a85ec53ULL;
  v ^= v >> 33;
  return (uint32_t)v;
}

// One workgroup per cell: a jittered square lattice over the cell's window
// square, smooth heights and equal weights.  In raster order (the point order
// of gridded terrain samples), or with unordered set: stored point i takes
// lattice site (i P) mod q for a prime P that does not divide q, a bijection
// that scatters consecutive points across the cell (scattered samples).
// Every thread stays inside [off[c], off[c+1]).
template <typename T>
__global__ void tune_points_kernel(const int64_t *off, const double *win, int use_win, int unordered, T *x, T *y,
                                   T *h, T *w) {
  const int64_t c = blockIdx.x;
  const int64_t a = off[c], b = off[c + 1];
  const int64_t q = b - a;
  if (q <= 0) return;
  // q < 2^31 cannot be a multiple of both primes; i P < 2^61
  const int64_t P = (q % 1000003 == 0) ? 998244353 : 1000003;
  const int64_t m = (int64_t)ceil(sqrt((double)q));
  double cx = 0.0, cy = 0.0, R = 3.0;
  if (use_win) { cx = win[3 * c]; cy = win[3 * c + 1]; R = win[3 * c + 2]; }
  const double d = 2.0 * R / (double)m;
  for (int64_t i = threadIdx.x; i < q; i += blockDim.x) {
    const int64_t site = unordered ? (i * P) % q : i;
    const int64_t r = site / m, s = site - r * m;
    const uint32_t hs = mix32((uint64_t)(a + i) * 0x9e3779b97f4a7c15ULL + 12345u);
    const double jx = ((hs & 0xffffu) * (1.0 / 65536.0) - 0.5) * 0.6;
    const double jy = ((hs >> 16) * (1.0 / 65536.0) - 0.5) * 0.6;
    const double px = cx - R + ((double)s + 0.5 + jx) * d;
    const double py = cy - R + ((double)r + 0.5 + jy) * d;
    x[a + i] = (T)px;
    y[a + i] = (T)py;
    h[a + i] = (T)(sin(1.7 * px) * cos(2.3 * py) + 0.25 * sin(5.0 * (px + py)));
    w[a + i] = (T)(d * d);
  }
}

struct Choice {
  int64_t chunk_min = 16384;
  int fwd_ips = 2, adj_ips = 2, band_mult = 1, fwd_threads = 512, fwd_acc = 8;
  double fwd_ms = 0.0, adj_ms = 0.0;
};

uint64_t fnv1a(const void *data, size_t n, uint64_t h = 1469598103934665603ULL) {
  const unsigned char *b = (const unsigned char *)data;
  for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ULL; }
  return h;
}

std::string cache_key(enufft_plan_t p, const char *arch) {
  uint64_t hsh = fnv1a(p->offsets.data(), p->offsets.size() * sizeof(int64_t));
  char buf[320];
  std::snprintf(buf, sizeof(buf), "v4_%s_cu%d_p%d_m%dx%d_g%dx%d_w%d_k%d_win%d_o%d_c%lld_q%lld_h%016llx", arch,
                p->n_cu, p->prec, p->N1, p->N2, p->n1, p->n2, p->W, p->opts.kernel_kind, p->window_kind,
                p->opts.autotune == 2 ? 1 : 0,
                (long long)p->n_cells, (long long)p->n_points, (unsigned long long)hsh);
  std::string k(buf);
  for (char &ch : k)
    if (ch == ' ' || ch == ':') ch = '-';
  return k;
}

// ENUFFT_TUNE_CACHE: a file path, or "off"; unset: $HOME/.cache/enufft/tune_cache.txt.
std::string cache_path() {
  const char *e = std::getenv("ENUFFT_TUNE_CACHE");
  if (e && std::strcmp(e, "off") == 0) return "";
  if (e && *e) return e;
  const char *home = std::getenv("HOME");
  if (!home || !*home) return "";
  std::string dir = std::string(home) + "/.cache";
  (void)mkdir(dir.c_str(), 0755);
  dir += "/enufft";
  (void)mkdir(dir.c_str(), 0755);
  return dir + "/tune_cache.txt";
}

bool valid(const Choice &c) {
  // band_mult 0: the single-grid adjoint
  const bool pow2 = c.fwd_ips > 0 && c.adj_ips > 0 && c.band_mult >= 0;
  const bool thr = c.fwd_threads == 256 || c.fwd_threads == 512 || c.fwd_threads == 1024;
  const bool acc = c.fwd_acc == 4 || c.fwd_acc == 8;
  return pow2 && thr && acc && c.chunk_min >= 1024 && c.chunk_min <= (1LL << 24) && c.fwd_ips <= 64 && c.adj_ips <= 64 &&
         c.band_mult <= 8;
}

bool cache_lookup(const std::string &path, const std::string &key, Choice *out) {
  if (path.empty()) return false;
  FILE *f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  bool found = false;
  char line[512];
  while (std::fgets(line, sizeof(line), f)) {
    char k[400];
    long long cm = 0;
    Choice c;
    if (std::sscanf(line, "%399s %lld %d %d %d %d %d %lf %lf", k, &cm, &c.fwd_ips, &c.adj_ips, &c.band_mult,
                    &c.fwd_threads, &c.fwd_acc, &c.fwd_ms, &c.adj_ms) == 9 &&
        key == k) {
      c.chunk_min = cm;
      if (valid(c)) { *out = c; found = true; }   // the last valid entry wins
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const std::string &path, const std::string &key, const Choice &c) {
  if (path.empty()) return;
  FILE *f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%s %lld %d %d %d %d %d %.6f %.6f\n", key.c_str(), (long long)c.chunk_min, c.fwd_ips, c.adj_ips,
               c.band_mult, c.fwd_threads, c.fwd_acc, c.fwd_ms, c.adj_ms);
  std::fclose(f);
}

// Device buffers of one trial set; released by the destructor.
struct TrialBuffers {
  std::vector<void *> ptrs;
  ~TrialBuffers() {
    for (void *q : ptrs) (void)hipFree(q);
  }
  hipError_t alloc(void **q, size_t bytes) {
    hipError_t e = hipMalloc(q, std::max<size_t>(bytes, 16));
    if (e == hipSuccess) ptrs.push_back(*q);
    return e;
  }
};

enufft_status tune_err(enufft_plan_t p, enufft_status s, const std::string &m) {
  p->last_error = "autotune: " + m;
  return s;
}

// Mean time of `reps` calls of fn after one untimed call, in ms.
template <typename F>
enufft_status time_calls(enufft_plan_t t, F fn, int reps, hipEvent_t e0, hipEvent_t e1, double *ms) {
  enufft_status st = fn();
  if (st != ENUFFT_OK) return st;
  if (hipEventRecord(e0, t->stream) != hipSuccess) return ENUFFT_EDEVICE;
  for (int i = 0; i < reps && st == ENUFFT_OK; ++i) st = fn();
  if (st != ENUFFT_OK) return st;
  if (hipEventRecord(e1, t->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return ENUFFT_EDEVICE;
  float f = 0.f;
  if (hipEventElapsedTime(&f, e0, e1) != hipSuccess) return ENUFFT_EDEVICE;
  *ms = f / reps;
  return ENUFFT_OK;
}

// Timed trials on plan t (the plan itself or a plan over a prefix of its cells),
// on raster-ordered or unordered synthetic points.
enufft_status run_trials(enufft_plan_t t, size_t lds_limit, int unordered, Choice *best) {
  const int64_t Q = t->n_points;
  const size_t el = t->elem;
  const int64_t M = (int64_t)t->N1 * t->N2;
  TrialBuffers buf;
  void *x, *y, *h, *w, *f, *keep, *gh, *gx, *gy, *off;
  hipError_t e = buf.alloc(&x, Q * el);
  if (e == hipSuccess) e = buf.alloc(&y, Q * el);
  if (e == hipSuccess) e = buf.alloc(&h, Q * el);
  if (e == hipSuccess) e = buf.alloc(&w, Q * el);
  if (e == hipSuccess) e = buf.alloc(&gh, Q * el);
  if (e == hipSuccess) e = buf.alloc(&gx, Q * el);
  if (e == hipSuccess) e = buf.alloc(&gy, Q * el);
  if (e == hipSuccess) e = buf.alloc(&f, t->n_cells * M * 2 * el);
  if (e == hipSuccess) e = buf.alloc(&keep, t->n_cells * M);
  if (e == hipSuccess) e = buf.alloc(&off, t->offsets.size() * sizeof(int64_t));
  if (e != hipSuccess) return tune_err(t, ENUFFT_ENOMEM, std::string("trial buffers: ") + hipGetErrorString(e));
  e = hipMemcpy(off, t->offsets.data(), t->offsets.size() * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemsetAsync(keep, 1, t->n_cells * M, t->stream);
  if (e == hipSuccess && t->n_cells > 0) {
    const int use_win = t->window_kind == ENUFFT_WIN_HANN_RADIAL;
    if (t->prec == ENUFFT_F64)
      hipLaunchKernelGGL(tune_points_kernel<double>, dim3((unsigned)t->n_cells), dim3(256), 0, t->stream,
                         (const int64_t *)off, (const double *)t->d_windows, use_win, unordered, (double *)x, (double *)y,
                         (double *)h, (double *)w);
    else
      hipLaunchKernelGGL(tune_points_kernel<float>, dim3((unsigned)t->n_cells), dim3(256), 0, t->stream,
                         (const int64_t *)off, (const double *)t->d_windows, use_win, unordered, (float *)x, (float *)y,
                         (float *)h, (float *)w);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(t->stream);
  if (e != hipSuccess) return tune_err(t, ENUFFT_EDEVICE, std::string("synthetic points: ") + hipGetErrorString(e));

  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return tune_err(t, ENUFFT_EDEVICE, "event");
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return tune_err(t, ENUFFT_EDEVICE, "event"); }
  const bool timing = t->timing;
  t->timing = false;
  enufft_status st = ENUFFT_OK;
  const int reps = 3;

  // forward: workgroup size x chunk floor x items per resident workgroup.  The
  // grid sums stay FP64: the FP32-sum build (half the LDS, two workgroups per
  // CU) measured about six times slower on the 20,480-cell batch, its LDS adds
  // being far slower per instruction, so it is not a candidate.
  double fbest = 1e300;
  Choice c = *best;
  const int acc = 8;
  t->fwd_acc = acc;
  for (int thr : {512, 1024}) {
    if (set_fwd_threads(t, thr, lds_limit) != ENUFFT_OK) continue;   // does not fit: not a candidate
    for (int64_t cm : {4096LL, 16384LL, 65536LL}) {
      for (int ips : {1, 2, 4}) {
        t->fwd_chunk_min = cm;
        t->fwd_items_per_slot = ips;
        st = install_fwd_schedule(t);
        if (st != ENUFFT_OK) break;
        double ms = 0.0;
        st = time_calls(t, [&] { return enufft_type1_batched(t, x, y, h, w, f); }, reps, e0, e1, &ms);
        if (st != ENUFFT_OK) break;
        if (ms < fbest) { fbest = ms; c.chunk_min = cm; c.fwd_ips = ips; c.fwd_threads = thr; c.fwd_acc = acc; }
      }
      if (st != ENUFFT_OK) break;
    }
    if (st != ENUFFT_OK) break;
  }
  if (fbest == 1e300 && st == ENUFFT_OK) st = tune_err(t, ENUFFT_EDEVICE, "no forward launch shape fits");
  // adjoint: items per resident workgroup x row bands (the forward output above
  // stands in for the cotangent source; keep is all ones)
  double abest = 1e300;
  t->fwd_acc = c.fwd_acc;
  if (st == ENUFFT_OK) st = set_fwd_threads(t, c.fwd_threads, lds_limit);
  if (st == ENUFFT_OK) {
    t->fwd_chunk_min = c.chunk_min;
    t->fwd_items_per_slot = c.fwd_ips;
    st = install_fwd_schedule(t);
  }
  if (st == ENUFFT_OK) st = enufft_type1_batched(t, x, y, h, w, f);
  for (int bm : {0, 1, 2}) {
    if (st != ENUFFT_OK) break;
    if (bm == 0 && !t->adj1_avail) continue;
    for (int ips : {1, 2, 4}) {
      t->adj1 = bm == 0;
      t->adj_band_mult = bm == 0 ? 1 : bm;
      t->adj_items_per_slot = ips;
      adj_reset(t);
      double ms = 0.0;
      st = time_calls(t, [&] {
        return enufft_retained_power_adjoint(t, x, y, h, w, f, (const uint8_t *)keep, nullptr, gh, gx, gy);
      }, reps, e0, e1, &ms);
      if (st != ENUFFT_OK) break;
      if (ms < abest) { abest = ms; c.adj_ips = ips; c.band_mult = bm; }
    }
  }
  adj_reset(t);
  t->adj1 = t->adj1_avail;
  t->adj_band_mult = 1;
  t->timing = timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != ENUFFT_OK) return st;
  c.fwd_ms = fbest;
  c.adj_ms = abest;
  *best = c;
  return ENUFFT_OK;
}

}  // namespace

enufft_status autotune(enufft_plan_t p) {
  if (p->n_cells == 0 || p->n_points == 0) return ENUFFT_OK;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, p->device) != hipSuccess) return tune_err(p, ENUFFT_EDEVICE, "device query");
  const int unordered = p->opts.autotune == 2;
  const std::string key = cache_key(p, prop.gcnArchName);
  const std::string path = cache_path();
  Choice c;
  bool hit = cache_lookup(path, key, &c);
  if (!hit) {
    // Trials run on the plan itself, or on a plan over the longest prefix of
    // cells that stays under the point cap (ENUFFT_TUNE_MAX_POINTS).
    int64_t cap = 1LL << 27;
    if (const char *s = std::getenv("ENUFFT_TUNE_MAX_POINTS")) cap = std::max<int64_t>(1 << 16, std::atoll(s));
    enufft_status st;
    if (p->n_points <= cap) {
      st = run_trials(p, (size_t)prop.sharedMemPerBlock, unordered, &c);
    } else {
      int64_t nc = 0;
      while (nc < p->n_cells && p->offsets[nc + 1] <= cap) ++nc;
      nc = std::max<int64_t>(nc, 1);
      enufft_opts o = p->opts;
      o.autotune = 0;
      enufft_plan_t sub = nullptr;
      st = enufft_plan(&sub, nc, p->offsets.data(), p->windows_host.empty() ? nullptr : p->windows_host.data(), &o,
                       p->stream);
      if (st != ENUFFT_OK) return tune_err(p, st, std::string("prefix plan: ") + enufft_last_error(nullptr));
      st = run_trials(sub, (size_t)prop.sharedMemPerBlock, unordered, &c);
      if (st != ENUFFT_OK) p->last_error = sub->last_error;
      (void)enufft_destroy(sub);
    }
    if (st != ENUFFT_OK) return st;
    cache_store(path, key, c);
  }
  p->fwd_acc = c.fwd_acc;
  enufft_status st = set_fwd_threads(p, c.fwd_threads, (size_t)prop.sharedMemPerBlock);
  if (st != ENUFFT_OK) return st;
  p->fwd_chunk_min = c.chunk_min;
  p->fwd_items_per_slot = c.fwd_ips;
  p->adj_items_per_slot = c.adj_ips;
  p->adj1 = p->adj1_avail && c.band_mult == 0;
  p->adj_band_mult = c.band_mult == 0 ? 1 : c.band_mult;
  p->tuned = true;
  p->tune_cache_hit = hit;
  p->tune_fwd_ms = c.fwd_ms;
  p->tune_adj_ms = c.adj_ms;
  adj_reset(p);
  return install_fwd_schedule(p);
}

}  // namespace enufft
