// Slice-sampling bookkeeping for a sampler above the likelihood (stepping out and shrinkage
// along a line, Neal 2003, "Slice sampling", sections 4.1 and 4.2): one thread per chain, the
// chain's point and direction in d float64 coordinates. The likelihood itself is evaluated by
// the caller between these launches, at the points they write.
//
// Every product and sum is rounded on its own, in the order the C ABI documents, so a chain's
// interval, draws and points are the ones the same steps give when taken one array operation at
// a time; contraction into fused multiply-adds is switched off for this file.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include "gwl_runtime.h"

namespace gwl {

constexpr int SLICE_BLOCK = 256;

// p in the unit cube and ln L(p) >= lmin (false for a NaN ln L)
__device__ __forceinline__ bool in_region(const double* __restrict__ p, int d, double l, double lmin) {
  bool ok = l >= lmin;
  for (int j = 0; j < d; ++j) ok = ok && p[j] >= 0.0 && p[j] <= 1.0;
  return ok;
}

__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_ends(int64_t n, int d, int m, const double* __restrict__ x,
                                                            const double* __restrict__ dirn,
                                                            const double* __restrict__ u0,
                                                            const double* __restrict__ u1, double* __restrict__ pts,
                                                            double* __restrict__ lo, double* __restrict__ hi,
                                                            double* __restrict__ jl, double* __restrict__ jr) {
  const int64_t i = (int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x;
  if (i >= n) return;
  const double l0 = -u0[i], h0 = 1.0 - u0[i];
  const double sl = floor((double)m * u1[i]);
  lo[i] = l0;
  hi[i] = h0;
  jl[i] = sl;
  jr[i] = (double)(m - 1) - sl;
  const double* xi = x + i * d;
  const double* di = dirn + i * d;
  for (int j = 0; j < m; ++j) {
    const double el = l0 - (double)j, er = h0 + (double)j;
    double* pl = pts + ((int64_t)j * n + i) * d;
    double* pr = pts + ((int64_t)(m + j) * n + i) * d;
    for (int c = 0; c < d; ++c) {
      pl[c] = xi[c] + el * di[c];
      pr[c] = xi[c] + er * di[c];
    }
  }
}

__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_ends_select(int64_t n, int d, int m,
                                                                   const double* __restrict__ pts,
                                                                   const double* __restrict__ logl,
                                                                   const double* __restrict__ lmin,
                                                                   double* __restrict__ lo, double* __restrict__ hi,
                                                                   const double* __restrict__ jl,
                                                                   const double* __restrict__ jr) {
  const int64_t i = (int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x;
  if (i >= n) return;
  const double lm = *lmin;
  int out_l = m, out_r = m;
  for (int j = m - 1; j >= 0; --j) {   // the first end outside on each side
    const int64_t kl = (int64_t)j * n + i, kr = (int64_t)(m + j) * n + i;
    if (!in_region(pts + kl * d, d, logl[kl], lm)) out_l = j;
    if (!in_region(pts + kr * d, d, logl[kr], lm)) out_r = j;
  }
  lo[i] = lo[i] - fmin((double)out_l, jl[i]);
  hi[i] = hi[i] + fmin((double)out_r, jr[i]);
}

__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_draws(int64_t n, int d, int G, const double* __restrict__ x,
                                                             const double* __restrict__ dirn,
                                                             const double* __restrict__ lo,
                                                             const double* __restrict__ hi,
                                                             const double* __restrict__ u, double* __restrict__ t,
                                                             double* __restrict__ pts, double* __restrict__ a,
                                                             double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x;
  if (i >= n) return;
  double ai = lo[i], bi = hi[i];
  const double* xi = x + i * d;
  const double* di = dirn + i * d;
  for (int k = 0; k < G; ++k) {
    const int64_t r = (int64_t)k * n + i;
    const double tk = ai + u[r] * (bi - ai);
    t[r] = tk;
    double* p = pts + r * d;
    for (int c = 0; c < d; ++c) p[c] = xi[c] + tk * di[c];
    if (tk < 0.0)
      ai = tk;
    else
      bi = tk;
  }
  a[i] = ai;
  b[i] = bi;
}

__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_select(int64_t n, int d, int G, const double* __restrict__ pts,
                                                              const double* __restrict__ logl,
                                                              const double* __restrict__ lmin,
                                                              const double* __restrict__ a,
                                                              const double* __restrict__ b, double* __restrict__ xn,
                                                              unsigned char* __restrict__ done,
                                                              double* __restrict__ lo, double* __restrict__ hi) {
  const int64_t i = (int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x;
  if (i >= n) return;
  if (done[i]) return;
  const double lm = *lmin;
  for (int k = 0; k < G; ++k) {
    const int64_t r = (int64_t)k * n + i;
    if (in_region(pts + r * d, d, logl[r], lm)) {
      for (int c = 0; c < d; ++c) xn[i * d + c] = pts[r * d + c];
      done[i] = 1;
      return;
    }
  }
  lo[i] = a[i];
  hi[i] = b[i];
}

static unsigned grid_of(int64_t n) { return (unsigned)((n + SLICE_BLOCK - 1) / SLICE_BLOCK); }

static gwl_status check_shape(int64_t n, int d, int k) {
  if (n < 1 || n > kMaxBatch || d < 1 || d > 4096 || k < 1 || k > 4096)
    return fail(GWL_E_SHAPE, "n=%lld, d=%d, m or G=%d outside [1, 2^30] x [1, 4096] x [1, 4096]", (long long)n, d, k);
  if ((int64_t)2 * k * n > kMaxBatch) return fail(GWL_E_SHAPE, "2 * %d * %lld points exceed 2^30", k, (long long)n);
  return GWL_OK;
}

static gwl_status launched(const char* what) {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? GWL_OK : hip_fail(e, what);
}

}  // namespace gwl

using namespace gwl;

extern "C" {

gwl_status gwl_slice_ends(int64_t n, int d, int m, const double* x, const double* dirn, const double* u0,
                          const double* u1, double* pts, double* lo, double* hi, double* jl, double* jr,
                          void* stream) {
  clear_error();
  gwl_status st = check_shape(n, d, m);
  if (st != GWL_OK) return st;
  if (!x || !dirn || !u0 || !u1 || !pts || !lo || !hi || !jl || !jr)
    return fail(GWL_E_INVALID, "gwl_slice_ends: null pointer");
  hipLaunchKernelGGL(k_slice_ends, dim3(grid_of(n)), dim3(SLICE_BLOCK), 0, (hipStream_t)stream, n, d, m, x, dirn,
                     u0, u1, pts, lo, hi, jl, jr);
  return launched("gwl_slice_ends");
}

gwl_status gwl_slice_ends_select(int64_t n, int d, int m, const double* pts, const double* logl, const double* lmin,
                                 double* lo, double* hi, const double* jl, const double* jr, void* stream) {
  clear_error();
  gwl_status st = check_shape(n, d, m);
  if (st != GWL_OK) return st;
  if (!pts || !logl || !lmin || !lo || !hi || !jl || !jr)
    return fail(GWL_E_INVALID, "gwl_slice_ends_select: null pointer");
  hipLaunchKernelGGL(k_slice_ends_select, dim3(grid_of(n)), dim3(SLICE_BLOCK), 0, (hipStream_t)stream, n, d, m, pts,
                     logl, lmin, lo, hi, jl, jr);
  return launched("gwl_slice_ends_select");
}

gwl_status gwl_slice_draws(int64_t n, int d, int G, const double* x, const double* dirn, const double* lo,
                           const double* hi, const double* u, double* t, double* pts, double* a, double* b,
                           void* stream) {
  clear_error();
  gwl_status st = check_shape(n, d, G);
  if (st != GWL_OK) return st;
  if (!x || !dirn || !lo || !hi || !u || !t || !pts || !a || !b)
    return fail(GWL_E_INVALID, "gwl_slice_draws: null pointer");
  hipLaunchKernelGGL(k_slice_draws, dim3(grid_of(n)), dim3(SLICE_BLOCK), 0, (hipStream_t)stream, n, d, G, x, dirn,
                     lo, hi, u, t, pts, a, b);
  return launched("gwl_slice_draws");
}

gwl_status gwl_slice_select(int64_t n, int d, int G, const double* x, const double* dirn, const double* t,
                            const double* pts, const double* logl, const double* lmin, const double* a,
                            const double* b, double* xn, unsigned char* done, double* lo, double* hi, void* stream) {
  clear_error();
  gwl_status st = check_shape(n, d, G);
  if (st != GWL_OK) return st;
  if (!x || !dirn || !t || !pts || !logl || !lmin || !a || !b || !xn || !done || !lo || !hi)
    return fail(GWL_E_INVALID, "gwl_slice_select: null pointer");
  hipLaunchKernelGGL(k_slice_select, dim3(grid_of(n)), dim3(SLICE_BLOCK), 0, (hipStream_t)stream, n, d, G, pts, logl,
                     lmin, a, b, xn, done, lo, hi);
  return launched("gwl_slice_select");
}

}  // extern "C"
