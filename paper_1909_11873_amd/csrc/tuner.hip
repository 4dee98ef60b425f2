// Tile choice for the bin loop: a cache of measured choices keyed by launch shape, a
// heuristic when nothing is cached, and the timing search behind gwl_autotune.
//
// The one free shape parameter of a single-event launch is the number of bin chunks: more
// chunks give the chip more wavefronts (latency hiding, fewer idle SIMDs at the tail), fewer
// chunks give each wavefront a longer run per coefficient load and fewer partial sums.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "gwl_runtime.h"

using namespace gwl;

namespace {

struct Key {
  int nd, mixed, grad;
  int64_t M;
  int npg_bucket;  // point groups rounded up to a power of two
  bool operator<(const Key& o) const {
    return std::tie(nd, mixed, grad, M, npg_bucket) < std::tie(o.nd, o.mixed, o.grad, o.M, o.npg_bucket);
  }
};
struct Entry {
  int nchunk;
  double ms;
};

std::mutex g_mu;
std::map<Key, Entry> g_cache;

int pow2_ceil(int64_t x) {
  int b = 1;
  while (b < x && b < (1 << 30)) b <<= 1;
  return b;
}

Key make_key(int nd, bool mixed, bool grad, int64_t M, int64_t B) {
  return Key{nd, mixed ? 1 : 0, grad ? 1 : 0, M, pow2_ceil((B + WAVE - 1) / WAVE)};
}

// Read every "{...}" entry line of a cache file written by save_cache().
bool load_cache(const char* path) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[512];
  std::lock_guard<std::mutex> lk(g_mu);
  while (fgets(line, sizeof line, f)) {
    Key k;
    Entry e;
    long long M;
    if (sscanf(line, " {\"ndet\": %d, \"mixed\": %d, \"grad\": %d, \"M\": %lld, \"npg_bucket\": %d, \"nchunk\": %d, \"ms\": %lf}",
               &k.nd, &k.mixed, &k.grad, &M, &k.npg_bucket, &e.nchunk, &e.ms) == 7) {
      k.M = M;
      g_cache[k] = e;
    }
  }
  fclose(f);
  return true;
}

bool save_cache(const char* path) {
  FILE* f = fopen(path, "w");
  if (!f) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  fprintf(f, "{\"arch\": \"gfx950\", \"entries\": [\n");
  size_t i = 0;
  for (const auto& kv : g_cache) {
    const Key& k = kv.first;
    fprintf(f, "  {\"ndet\": %d, \"mixed\": %d, \"grad\": %d, \"M\": %lld, \"npg_bucket\": %d, \"nchunk\": %d, \"ms\": %.6f}%s\n",
            k.nd, k.mixed, k.grad, (long long)k.M, k.npg_bucket, kv.second.nchunk, kv.second.ms,
            ++i < g_cache.size() ? "," : "");
  }
  fprintf(f, "]}\n");
  fclose(f);
  return true;
}

__global__ void k_fill_theta(double* theta, int64_t B) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= B) return;
  // a fixed, valid parameter point with a small per-point variation; the cost of the
  // evaluation does not depend on the values
  const double row[NPARAM] = {30.0, 0.8, 0.1, -0.2, 400.0, 2.0, -0.5, 0.6, 1.0, 0.7, 0.0};
  for (int i = 0; i < NPARAM; ++i) theta[p * NPARAM + i] = row[i];
  theta[p * NPARAM + 0] += 1e-6 * (double)(p % 1024);
}

}  // namespace

namespace gwl {

int heuristic_nchunk(int64_t B, int64_t M) {
  // aim for ~8 wavefronts per SIMD (1024 SIMDs) with chunks of at least 512 bins
  const int64_t npg = (B + WAVE - 1) / WAVE;
  int64_t want = (8192 + npg - 1) / npg;
  const int64_t maxc = (M + 511) / 512;
  if (want > maxc) want = maxc;
  if (want < 1) want = 1;
  return (int)want;
}

int choose_nchunk(const gwl_event_s* ev, int64_t B, bool mixed, bool grad) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(make_key(ev->ndet, mixed, grad, ev->M, B));
    if (it != g_cache.end()) return it->second.nchunk;
  }
  return heuristic_nchunk(B, ev->M);
}

}  // namespace gwl

extern "C" {

gwl_status gwl_autotune_load(const char* cache_path) {
  clear_error();
  if (!cache_path) return fail(GWL_E_INVALID, "cache_path is null");
  if (!load_cache(cache_path)) return fail(GWL_E_INVALID, "cannot read %s", cache_path);
  return GWL_OK;
}

gwl_status gwl_autotune(const char* cache_path, gwl_event ev, int64_t B, gwl_precision prec, int with_grad) {
  clear_error();
  if (!ev) return fail(GWL_E_INVALID, "event is null");
  if (B < 1 || B > kMaxBatch) return fail(GWL_E_SHAPE, "B=%lld outside [1, %lld]", (long long)B, (long long)kMaxBatch);
  if (prec != GWL_FP64 && prec != GWL_MIXED) return fail(GWL_E_INVALID, "unknown precision %d", (int)prec);
  gwl_status st = check_device(ev->device);
  if (st != GWL_OK) return st;
  if (cache_path) load_cache(cache_path);  // keep entries of other shapes
  const bool mixed = prec == GWL_MIXED, grad = with_grad != 0;

  // candidate chunk counts around the heuristic, each distinct after rounding
  const int h = heuristic_nchunk(B, ev->M);
  std::vector<int> cand;
  const int mult[] = {1, 2, 4, 8, 16};
  for (int m : mult) {
    cand.push_back(h / m);
    cand.push_back(h * m);
  }
  // distinct launch shapes (the chunk count a shape really uses can differ from the request)
  std::vector<LoopShape> shapes;
  for (int c : cand) {
    if (c < 1 || (int64_t)c > ev->M) continue;
    const LoopShape sh = make_shape(B, ev->M, c);
    bool seen = false;
    for (const LoopShape& u : shapes) seen |= (u.nchunk == sh.nchunk);
    if (!seen) shapes.push_back(sh);
  }

  const int64_t Bp = (B + WAVE - 1) / WAVE * WAVE;
  int maxc = 1;
  for (const LoopShape& u : shapes) maxc = u.nchunk > maxc ? u.nchunk : maxc;
  double *theta = nullptr, *logl = nullptr, *grad_out = nullptr, *ws = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc((void**)&theta, sizeof(double) * NPARAM * (size_t)B);
  if (e == hipSuccess) e = hipMalloc((void**)&logl, sizeof(double) * (size_t)B);
  if (e == hipSuccess && grad) e = hipMalloc((void**)&grad_out, sizeof(double) * NPARAM * (size_t)B);
  if (e == hipSuccess) e = hipMalloc((void**)&ws, workspace_bytes(Bp, maxc, ev->ndet, grad));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_fill_theta, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, 0, theta, B);
    e = hipGetLastError();
  }
  int best = h;
  double best_ms = 1e300;
  for (size_t i = 0; e == hipSuccess && i < shapes.size(); ++i) {
    const LoopShape& sh = shapes[i];
    double* coef = ws;
    double* part = ws + (size_t)NCOEF * Bp;
    float ms_min = 1e30f;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
      e = hipEventRecord(e0, 0);
      if (e == hipSuccess) e = enqueue_logl(ev, theta, B, mixed, grad, sh, coef, part, logl, grad_out, 0);
      if (e == hipSuccess) e = hipEventRecord(e1, 0);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0 && ms < ms_min) ms_min = ms;  // first run is a warm-up
    }
    if (e == hipSuccess && ms_min < best_ms) {
      best_ms = ms_min;
      best = sh.nchunk;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (theta) (void)hipFree(theta);
  if (logl) (void)hipFree(logl);
  if (grad_out) (void)hipFree(grad_out);
  if (ws) (void)hipFree(ws);
  if (e != hipSuccess) return hip_fail(e, "autotune");
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[make_key(ev->ndet, mixed, grad, ev->M, B)] = Entry{best, best_ms};
  }
  if (cache_path && !save_cache(cache_path)) return fail(GWL_E_INVALID, "cannot write %s", cache_path);
  return GWL_OK;
}

}  // extern "C"
