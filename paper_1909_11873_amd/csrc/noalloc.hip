// gwl_logl_batch_noalloc: the forward evaluation with its workspace in a fixed, file-scope device
// array instead of the event's per-stream workspace, for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops that must not call the allocator).
//
// The array is a __device__ variable: every GPU that runs the library holds its own copy, at its
// own address, for the life of the process. Host code must not pass the variable's name to a
// kernel (in host code it is a host-side stand-in); its device address is looked up once per
// device with hipGetSymbolAddress and kept here.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/gwlike.h"
#include "gwl_common.h"
#include "gwl_launch.h"
#include "gwl_runtime.h"

using namespace gwl;

namespace {

constexpr size_t kScratchBytes = (size_t)GWL_NOALLOC_SCRATCH_BYTES;
constexpr size_t kScratchCounters = 16384;
static_assert(kScratchBytes % 256 == 0, "scratch size");

// the workspace (set-up rows, partial sums) and the evaluation kernel's completion counters
__device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];
__device__ __align__(256) unsigned int scratch_cnt[kScratchCounters];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};
void* g_scratch_cnt[kMaxDevices] = {};

// The device addresses of this device's copies of the arrays (looked up on the first call per
// device, with that device current).
gwl_status scratch_address(int dev, double** ws, unsigned int** cnt) {
  if (dev < 0 || dev >= kMaxDevices) return fail(GWL_E_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev] || !g_scratch_cnt[dev]) {
    void *p = nullptr, *q = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch_cnt));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch_cnt)");
    if (!p || !q) return fail(GWL_E_DEVICE, "hipGetSymbolAddress returned a null address");
    g_scratch[dev] = p;
    g_scratch_cnt[dev] = q;
  }
  *ws = (double*)g_scratch[dev];
  *cnt = (unsigned int*)g_scratch_cnt[dev];
  return GWL_OK;
}

// The counters must be zero when the evaluation starts; every call clears the ones it uses (a fill
// kernel, so that the call can also be captured in a graph).
__global__ void k_zero_counters(unsigned int* __restrict__ c, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = 0u;
}

}  // namespace

extern "C" {

gwl_status gwl_logl_batch_noalloc(gwl_event ev, const double* theta, int64_t B, gwl_precision prec, double* logl,
                                  void* stream) {
  clear_error();
  if (!ev) return fail(GWL_E_INVALID, "event is null");
  if (prec != GWL_FP64 && prec != GWL_MIXED) return fail(GWL_E_INVALID, "unknown precision %d", (int)prec);
  if (B < 0 || B > kMaxBatch) return fail(GWL_E_SHAPE, "B=%lld outside [0, %lld]", (long long)B, (long long)kMaxBatch);
  if (B == 0) return GWL_OK;
  if (!theta || !logl) return fail(GWL_E_INVALID, "theta and logl must be device pointers");
  if (ev->ncal > 0) return fail(GWL_E_UNSUPPORTED, "calibrated events are not supported by the no-allocation call");
  gwl_status st = check_device(ev->device);
  if (st != GWL_OK) return st;
  double* ws = nullptr;
  unsigned int* cnt = nullptr;
  st = scratch_address(ev->device, &ws, &cnt);
  if (st != GWL_OK) return st;
  const int64_t Bp = (B + WAVE - 1) / WAVE * WAVE;
  const int nd = ev->ndet;
  const bool mixed = use_mixed(ev, prec);
  // the tuned shape, with fewer workgroups per point group while its workspace would not fit,
  // and the set-up in the kernel (which needs no workspace) as the last resort
  LoopShape sh = choose_shape(ev, B, mixed, false);
  while (sh.G > 1 && (workspace_bytes(Bp, sh, nd, false) > kScratchBytes || workspace_counters(sh, false) > kScratchCounters))
    sh = make_shape(B, ev->M, sh.W, sh.G / 2, sh.setup, sh.sepepi);
  if (workspace_bytes(Bp, sh, nd, false) > kScratchBytes) sh = make_shape(B, ev->M, sh.W, 1, 1);
  if (workspace_bytes(Bp, sh, nd, false) > kScratchBytes || workspace_counters(sh, false) > kScratchCounters)
    return fail(GWL_E_INTERNAL, "no launch shape fits the static scratch");
  hipStream_t s = (hipStream_t)stream;
  const int nc = (int)workspace_counters(sh, false);
  if (nc > 0) {
    hipLaunchKernelGGL(k_zero_counters, dim3((nc + 255) / 256), dim3(256), 0, s, cnt, nc);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "launch");
  }
  const hipError_t e = enqueue_logl(ev, theta, B, mixed, false, sh, ws, cnt, logl, nullptr, s);
  if (e != hipSuccess) return hip_fail(e, "launch");
  return GWL_OK;
}

}  // extern "C"
