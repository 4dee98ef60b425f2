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

__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_ends(int64_t n, int m, const double* __restrict__ u0,
                                                            const double* __restrict__ u1, double* __restrict__ lo,
                                                            double* __restrict__ hi, double* __restrict__ jl,
                                                            double* __restrict__ jr) {
  const int64_t i = (int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x;
  if (i >= n) return;
  const double sl = floor((double)m * u1[i]);
  lo[i] = -u0[i];
  hi[i] = 1.0 - u0[i];
  jl[i] = sl;
  jr[i] = (double)(m - 1) - sl;
}

// One thread per coordinate of a candidate end: row r = j n + i is chain i's left end j
// (lo - j) for j < m and its right end j - m (hi + j - m) above.
__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_end_points(int64_t n, int d, int m,
                                                                  const double* __restrict__ x,
                                                                  const double* __restrict__ dirn,
                                                                  const double* __restrict__ lo,
                                                                  const double* __restrict__ hi,
                                                                  double* __restrict__ pts) {
  const int64_t e = (int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x;
  if (e >= 2 * (int64_t)m * n * d) return;
  const int64_t r = e / d, c = e - r * d;
  const int j = (int)(r / n);
  const int64_t i = r - (int64_t)j * n;
  const double t = j < m ? lo[i] - (double)j : hi[i] + (double)(j - m);
  pts[e] = x[i * d + c] + t * dirn[i * d + c];
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

__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_draws(int64_t n, int G, const double* __restrict__ lo,
                                                             const double* __restrict__ hi,
                                                             const double* __restrict__ u, double* __restrict__ t,
                                                             double* __restrict__ a, double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x;
  if (i >= n) return;
  double ai = lo[i], bi = hi[i];
  for (int k = 0; k < G; ++k) {
    const int64_t r = (int64_t)k * n + i;
    const double tk = ai + u[r] * (bi - ai);
    t[r] = tk;
    if (tk < 0.0)
      ai = tk;
    else
      bi = tk;
  }
  a[i] = ai;
  b[i] = bi;
}

// One thread per coordinate of a draw: pts[r d + c] = x_i + t_r dirn_i, r = k n + i.
__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_draw_points(int64_t n, int d, int G,
                                                                   const double* __restrict__ x,
                                                                   const double* __restrict__ dirn,
                                                                   const double* __restrict__ t,
                                                                   double* __restrict__ pts) {
  const int64_t e = (int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x;
  if (e >= (int64_t)G * n * d) return;
  const int64_t r = e / d, c = e - r * d;
  const int64_t i = r % n;
  pts[e] = x[i * d + c] + t[r] * dirn[i * d + c];
}

// The cube test recomputes the draw's coordinates (the same products and sums as the points
// the likelihood saw), so the chain reads its own x and direction instead of G point rows. The
// draws are judged without an early exit (the first one inside wins), which leaves their loads
// independent of one another.
__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_select(int64_t n, int d, int G, const double* __restrict__ x,
                                                              const double* __restrict__ dirn,
                                                              const double* __restrict__ t,
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
  const double* xi = x + i * d;
  const double* di = dirn + i * d;
  int first = G;
  double tf = 0.0;
  for (int k = G - 1; k >= 0; --k) {
    const int64_t r = (int64_t)k * n + i;
    const double tk = t[r];
    bool ok = logl[r] >= lm;
    for (int c = 0; c < d; ++c) {
      const double p = xi[c] + tk * di[c];
      ok = ok && p >= 0.0 && p <= 1.0;
    }
    if (ok) {
      first = k;
      tf = tk;
    }
  }
  if (first < G) {
    for (int c = 0; c < d; ++c) xn[i * d + c] = xi[c] + tf * di[c];
    done[i] = 1;
  } else {
    lo[i] = a[i];
    hi[i] = b[i];
  }
}

// Lane-parallel forms for groups of at most one wavefront: a chain's L candidates sit on L
// consecutive lanes of one wavefront (64 / L chains per wavefront, spare lanes idle), each lane
// judges its own candidate with loads independent of the others, and a ballot gives each chain
// the index of its first candidate inside (or outside). Same decisions, same arithmetic.
__device__ __forceinline__ uint64_t group_bits(uint64_t mask, int c, int L) {
  const uint64_t gm = L == 64 ? ~0ull : ((1ull << L) - 1);
  return (mask >> (c * L)) & gm;
}

__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_ends_select_lanes(int64_t n, int d, int m,
                                                                         const double* __restrict__ pts,
                                                                         const double* __restrict__ logl,
                                                                         const double* __restrict__ lmin,
                                                                         double* __restrict__ lo,
                                                                         double* __restrict__ hi,
                                                                         const double* __restrict__ jl,
                                                                         const double* __restrict__ jr) {
  const int L = 2 * m, cpw = WAVE / L;
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t wave = ((int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x) / WAVE;
  const int c = lane / L, j = lane - c * L;
  const int64_t i = wave * cpw + c;
  const bool active = c < cpw && i < n;
  bool in = false;
  if (active) {
    const int64_t r = (int64_t)j * n + i;   // left end j for j < m, right end j - m above
    in = in_region(pts + r * d, d, logl[r], *lmin);
  }
  const uint64_t mask = __ballot(in);
  if (!active || j != 0) return;
  const uint64_t bits = group_bits(mask, c, L), side = (1ull << m) - 1;
  const uint64_t out_l = ~bits & side, out_r = ~(bits >> m) & side;
  const int sl = out_l ? __builtin_ctzll(out_l) : m;
  const int sr = out_r ? __builtin_ctzll(out_r) : m;
  lo[i] = lo[i] - fmin((double)sl, jl[i]);
  hi[i] = hi[i] + fmin((double)sr, jr[i]);
}

__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_select_lanes(int64_t n, int d, int G,
                                                                    const double* __restrict__ x,
                                                                    const double* __restrict__ dirn,
                                                                    const double* __restrict__ t,
                                                                    const double* __restrict__ logl,
                                                                    const double* __restrict__ lmin,
                                                                    const double* __restrict__ a,
                                                                    const double* __restrict__ b,
                                                                    double* __restrict__ xn,
                                                                    unsigned char* __restrict__ done,
                                                                    double* __restrict__ lo, double* __restrict__ hi) {
  const int cpw = WAVE / G;
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t wave = ((int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x) / WAVE;
  const int c = lane / G, k = lane - c * G;
  const int64_t i = wave * cpw + c;
  const bool active = c < cpw && i < n;
  const bool was_done = active && done[i] != 0;
  bool ok = false;
  if (active && !was_done) {
    const int64_t r = (int64_t)k * n + i;
    const double tk = t[r];
    ok = logl[r] >= *lmin;
    for (int q = 0; q < d; ++q) {
      const double p = x[i * d + q] + tk * dirn[i * d + q];
      ok = ok && p >= 0.0 && p <= 1.0;
    }
  }
  const uint64_t mask = __ballot(ok);
  if (!active || was_done) return;
  const uint64_t bits = group_bits(mask, c, G);
  if (bits == 0) {
    if (k == 0) {
      lo[i] = a[i];
      hi[i] = b[i];
    }
    return;
  }
  // the first draw inside: the chain's lanes write its coordinates together
  const double tf = t[(int64_t)__builtin_ctzll(bits) * n + i];
  for (int q = k; q < d; q += G) xn[i * d + q] = x[i * d + q] + tf * dirn[i * d + q];
  if (k == 0) done[i] = 1;
}

static unsigned lane_grid(int64_t n, int L) {
  const int64_t waves = (n + WAVE / L - 1) / (WAVE / L);
  return (unsigned)((waves * WAVE + SLICE_BLOCK - 1) / SLICE_BLOCK);
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
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_slice_ends, dim3(grid_of(n)), dim3(SLICE_BLOCK), 0, s, n, m, u0, u1, lo, hi, jl, jr);
  hipLaunchKernelGGL(k_slice_end_points, dim3(grid_of(2 * (int64_t)m * n * d)), dim3(SLICE_BLOCK), 0, s, n, d, m, x,
                     dirn, (const double*)lo, (const double*)hi, pts);
  return launched("gwl_slice_ends");
}

gwl_status gwl_slice_ends_select(int64_t n, int d, int m, const double* pts, const double* logl, const double* lmin,
                                 double* lo, double* hi, const double* jl, const double* jr, void* stream) {
  clear_error();
  gwl_status st = check_shape(n, d, m);
  if (st != GWL_OK) return st;
  if (!pts || !logl || !lmin || !lo || !hi || !jl || !jr)
    return fail(GWL_E_INVALID, "gwl_slice_ends_select: null pointer");
  if (2 * m <= WAVE)
    hipLaunchKernelGGL(k_slice_ends_select_lanes, dim3(lane_grid(n, 2 * m)), dim3(SLICE_BLOCK), 0, (hipStream_t)stream,
                       n, d, m, pts, logl, lmin, lo, hi, jl, jr);
  else
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
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_slice_draws, dim3(grid_of(n)), dim3(SLICE_BLOCK), 0, s, n, G, lo, hi, u, t, a, b);
  hipLaunchKernelGGL(k_slice_draw_points, dim3(grid_of((int64_t)G * n * d)), dim3(SLICE_BLOCK), 0, s, n, d, G, x,
                     dirn, (const double*)t, pts);
  return launched("gwl_slice_draws");
}

gwl_status gwl_slice_select(int64_t n, int d, int G, const double* x, const double* dirn, const double* t,
                            const double* logl, const double* lmin, const double* a, const double* b, double* xn,
                            unsigned char* done, double* lo, double* hi, void* stream) {
  clear_error();
  gwl_status st = check_shape(n, d, G);
  if (st != GWL_OK) return st;
  if (!x || !dirn || !t || !logl || !lmin || !a || !b || !xn || !done || !lo || !hi)
    return fail(GWL_E_INVALID, "gwl_slice_select: null pointer");
  if (G <= WAVE)
    hipLaunchKernelGGL(k_slice_select_lanes, dim3(lane_grid(n, G)), dim3(SLICE_BLOCK), 0, (hipStream_t)stream, n, d, G,
                       x, dirn, t, logl, lmin, a, b, xn, done, lo, hi);
  else
    hipLaunchKernelGGL(k_slice_select, dim3(grid_of(n)), dim3(SLICE_BLOCK), 0, (hipStream_t)stream, n, d, G, x, dirn,
                       t, logl, lmin, a, b, xn, done, lo, hi);
  return launched("gwl_slice_select");
}

}  // extern "C"
