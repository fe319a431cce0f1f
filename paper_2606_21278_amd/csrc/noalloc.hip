// Allocation-free batched type-1 (enufft_type1_batched_noalloc): the forward
// kernel with its scratch memory -- the persistent loop's work counters, the
// per-cell merge counters of split cells and the split cells' partial grids --
// taken from one fixed device array instead of the plan's workspace.  For
// callers that cannot allocate device memory while they run (code under HIP
// graph capture, tight serving loops): the call itself makes no allocation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "device_common.h"
#include "launch.h"
#include "plan.h"

namespace enufft {
namespace {

// The scratch array: one copy per GPU, held until the process ends.  In host
// code its name stands for the device symbol, not an address; the address of
// each device's copy comes from hipGetSymbolAddress and is kept per device.
constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Address of this device's scratch copy: looked up once per device, with that
// device current.
enufft_status scratch_address(enufft_plan_t p, void **out) {
  *out = nullptr;
  if (p->device < 0 || p->device >= kMaxDevices) {
    p->last_error = "enufft_type1_batched_noalloc: device index beyond the supported count";
    return ENUFFT_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[p->device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != p->device) e = hipSetDevice(p->device);
    void *ptr = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != p->device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) {
      p->last_error = std::string("enufft_type1_batched_noalloc: scratch address: ") + hipGetErrorString(e);
      return ENUFFT_EDEVICE;
    }
    g_scratch_ptr[p->device] = ptr;
  }
  *out = g_scratch_ptr[p->device];
  return ENUFFT_OK;
}

// Zero n words (a kernel rather than a memset, so the call can be captured).
__global__ void zero_words_kernel(int *w, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    w[i] = 0;
}

size_t round256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

// Scratch layout for a plan: counters (16 ints), per-cell merge counters, then
// the partial grids of the split cells.
size_t noalloc_scratch_bytes(enufft_plan_t p, size_t *cell_off, size_t *part_off) {
  *cell_off = 256;
  *part_off = round256(*cell_off + (size_t)p->n_cells * sizeof(int));
  return *part_off + (size_t)p->n_slots * p->n1 * p->n2 * p->elem;
}

}  // namespace enufft

extern "C" enufft_status enufft_type1_batched_noalloc(enufft_plan_t p, const void *x, const void *y, const void *h,
                                                      const void *w, void *f) {
  using namespace enufft;
  enufft_status st = check_plan(p, "enufft_type1_batched_noalloc");
  if (st != ENUFFT_OK) return st;
  if (p->big) {
    p->last_error = "enufft_type1_batched_noalloc: large-cell plans (mode boxes above 64 per axis) are not supported";
    return ENUFFT_EUNSUPPORTED;
  }
  if (p->n_cells == 0) return ENUFFT_OK;
  if (!f) {
    p->last_error = "enufft_type1_batched_noalloc: null f";
    return ENUFFT_EINVAL;
  }
  if (p->n_points > 0 && (!x || !y || !h || !w)) {
    p->last_error = "enufft_type1_batched_noalloc: null point array";
    return ENUFFT_EINVAL;
  }
  size_t cell_off = 0, part_off = 0;
  const size_t need = noalloc_scratch_bytes(p, &cell_off, &part_off);
  if (need > kScratchBytes) {
    p->last_error = "enufft_type1_batched_noalloc: the plan needs " + std::to_string(need) +
                    " bytes of scratch (counters and split-cell partial grids), above the fixed " +
                    std::to_string(kScratchBytes) + "; use enufft_type1_batched or fewer split cells";
    return ENUFFT_EINVAL;
  }
  void *base = nullptr;
  st = scratch_address(p, &base);
  if (st != ENUFFT_OK) return st;
  unsigned char *b = static_cast<unsigned char *>(base);
  int *counters = reinterpret_cast<int *>(b);
  // the counters and merge counters start at zero on every call (the kernels
  // leave them at zero, but a call that did not finish may not have)
  const int64_t nz = (int64_t)(part_off / sizeof(int));
  hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)std::min<int64_t>(1024, (nz + 255) / 256)), dim3(256), 0,
                     p->stream, counters, nz);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    if (p->prec == ENUFFT_F64) {
      auto a = make_fwd_args<double>(p, x, y, h, w, f);
      a.work_counter = counters;
      a.done_counter = counters + 1;
      a.cell_counters = reinterpret_cast<int *>(b + cell_off);
      a.partial = reinterpret_cast<double *>(b + part_off);
      e = launch_fwd<double>(a, p->W, p->fwd_blocks, p->fwd_threads, p->fwd_lds, p->stream);
    } else {
      auto a = make_fwd_args<float>(p, x, y, h, w, f);
      a.work_counter = counters;
      a.done_counter = counters + 1;
      a.cell_counters = reinterpret_cast<int *>(b + cell_off);
      a.partial = reinterpret_cast<float *>(b + part_off);
      e = launch_fwd<float>(a, p->W, p->fwd_blocks, p->fwd_threads, p->fwd_lds, p->stream);
    }
  }
  if (e != hipSuccess) {
    p->last_error = std::string("enufft_type1_batched_noalloc launch: ") + hipGetErrorString(e);
    p->faulted = true;
    return ENUFFT_EDEVICE;
  }
  return ENUFFT_OK;
}
