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

// The stepping out of a chain examines at most m - 1 ends: its left ends lo - s for s < jl
// (stopping at the first outside) and its right ends hi + s for s < jr, jl + jr = m - 1. Slot s
// of chain i (row s n + i) is its left end s for s < jl and its right end s - jl from there on,
// so every chain has exactly m - 1 slots and no end that cannot matter is evaluated.
// One thread per coordinate of a slot's point.
__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_end_points(int64_t n, int d, int m,
                                                                  const double* __restrict__ x,
                                                                  const double* __restrict__ dirn,
                                                                  const double* __restrict__ u0,
                                                                  const double* __restrict__ u1,
                                                                  double* __restrict__ pts, double* __restrict__ lo,
                                                                  double* __restrict__ hi, double* __restrict__ jl,
                                                                  double* __restrict__ jr) {
  const int64_t e = (int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x;
  if (e >= (int64_t)(m - 1) * n * d) return;
  const int64_t r = e / d, c = e - r * d;
  const int64_t s = r / n;
  const int64_t i = r - s * n;
  // the interval as k_slice_ends writes it, recomputed by every thread of the chain
  const double l0 = -u0[i], h0 = 1.0 - u0[i], nl = floor((double)m * u1[i]);
  if (s == 0 && c == 0) {
    lo[i] = l0;
    hi[i] = h0;
    jl[i] = nl;
    jr[i] = (double)(m - 1) - nl;
  }
  const double sd = (double)s;
  const double t = sd < nl ? l0 - sd : h0 + (sd - nl);
  pts[e] = x[i * d + c] + t * dirn[i * d + c];
}

// The start of a move: xn = x, done = 0, and the list of all n chains (one thread per
// coordinate). The end of a move: moved |= done, x = xn.
__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_move_begin(int64_t n, int d, const double* __restrict__ x,
                                                                  double* __restrict__ xn,
                                                                  unsigned char* __restrict__ done,
                                                                  int* __restrict__ list,
                                                                  int64_t* __restrict__ nact) {
  const int64_t e = (int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x;
  if (e >= n * d) return;
  xn[e] = x[e];
  if (e == 0) *nact = n;
  if (e % d == 0) {
    const int64_t i = e / d;
    done[i] = 0;
    list[i] = (int)i;
  }
}

__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_move_end(int64_t n, int d, const unsigned char* __restrict__ done,
                                                                unsigned char* __restrict__ moved,
                                                                const double* __restrict__ xn,
                                                                double* __restrict__ x) {
  const int64_t e = (int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x;
  if (e >= n * d) return;
  x[e] = xn[e];
  if (e % d == 0) {
    const int64_t i = e / d;
    moved[i] = (unsigned char)(moved[i] | done[i]);
  }
}

// lo -= the number of left ends inside before the first outside (jl if none), hi += the same on
// the right (jr if none).
__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_ends_select(int64_t n, int d, int m,
                                                                   const double* __restrict__ pts,
                                                                   const double* __restrict__ logl,
                                                                   const double* __restrict__ lmin,
                                                                   double* __restrict__ lo, double* __restrict__ hi,
                                                                   const double* __restrict__ jl) {
  const int64_t i = (int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x;
  if (i >= n) return;
  const double lm = *lmin;
  const int L = m - 1, nl = (int)jl[i];
  int sl = nl, sr = L - nl;
  for (int s = L - 1; s >= 0; --s) {   // the first slot outside on each side
    const int64_t r = (int64_t)s * n + i;
    if (!in_region(pts + r * d, d, logl[r], lm)) {
      if (s < nl)
        sl = s;
      else
        sr = s - nl;
    }
  }
  lo[i] = lo[i] - (double)sl;
  hi[i] = hi[i] + (double)sr;
}

// Shrinkage groups work on a list of the chains still moving: list[0 .. *nact). A group's draws
// and points are written compactly, draw k of list entry j at row j G + k, so its live points
// are the first *nact G rows; the group's selection writes the list of the chains that are still
// moving after it (in an order that depends on scheduling; every chain's own steps do not).

// Draws and their points, one thread per coordinate of a listed chain: each thread repeats its
// chain's G draws (a few operations each) and writes its coordinate of every draw, so the stores
// of a draw are spread over d threads; the chain's coordinate-0 thread writes t, a and b. Thread
// 0 also publishes the group's live point count (*live = *nact G), adds it to *calls (if not
// null), and clears the next list's length for the selection that follows.
__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_draws(int64_t n, int d, int G, const int* __restrict__ list,
                                                             const int64_t* __restrict__ nact,
                                                             const double* __restrict__ x,
                                                             const double* __restrict__ dirn,
                                                             const double* __restrict__ lo,
                                                             const double* __restrict__ hi,
                                                             const double* __restrict__ u, double* __restrict__ t,
                                                             double* __restrict__ pts, double* __restrict__ a,
                                                             double* __restrict__ b, int64_t* __restrict__ live,
                                                             int64_t* __restrict__ nact_next,
                                                             int64_t* __restrict__ calls) {
  const int64_t e = (int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x;
  const int64_t na = min(max(*nact, (int64_t)0), n);
  if (e == 0) {
    *live = na * G;
    *nact_next = 0;
    if (calls) *calls += na * G;
  }
  const int64_t j = e / d, c = e - j * d;
  if (j >= na) return;
  const int64_t i = list[j];
  if (i < 0 || i >= n) return;                   // not a chain index
  const double xc = x[i * d + c], dc = dirn[i * d + c];
  double ai = lo[i], bi = hi[i];
  for (int k = 0; k < G; ++k) {
    const int64_t r = j * G + k;
    const double tk = ai + u[(int64_t)k * n + i] * (bi - ai);
    pts[r * d + c] = xc + tk * dc;
    if (c == 0) t[r] = tk;
    if (tk < 0.0)
      ai = tk;
    else
      bi = tk;
  }
  if (c == 0) {
    a[i] = ai;
    b[i] = bi;
  }
}

// One listed chain that stays (no draw inside) joins the next list: the wavefront's stayers take
// consecutive slots from one atomic add, in lane order.
__device__ __forceinline__ void append_stayers(bool stay, int lane, int i, int64_t n, int* __restrict__ list_next,
                                               int64_t* __restrict__ nact_next) {
  const uint64_t stays = __ballot(stay);
  if (!stays) return;
  const int leader = __builtin_ctzll(stays);
  long long base = 0;
  if (lane == leader)
    base = (long long)atomicAdd((unsigned long long*)nact_next, (unsigned long long)__popcll(stays));
  base = __shfl(base, leader);
  const long long slot = base + __popcll(stays & ((1ull << lane) - 1));
  if (stay && slot < n) list_next[slot] = i;     // at most n stay once *nact_next started at 0
}

// The cube test recomputes the draw's coordinates (the same products and sums as the points
// the likelihood saw), so the chain reads its own x and direction instead of G point rows. The
// draws are judged without an early exit (the first one inside wins), which leaves their loads
// independent of one another. One thread per listed chain (groups of more than 64 draws).
__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_select(int64_t n, int d, int G, const int* __restrict__ list,
                                                              const int64_t* __restrict__ nact,
                                                              const double* __restrict__ x,
                                                              const double* __restrict__ dirn,
                                                              const double* __restrict__ t,
                                                              const double* __restrict__ logl,
                                                              const double* __restrict__ lmin,
                                                              const double* __restrict__ a,
                                                              const double* __restrict__ b, double* __restrict__ xn,
                                                              unsigned char* __restrict__ done,
                                                              double* __restrict__ lo, double* __restrict__ hi,
                                                              int* __restrict__ list_next,
                                                              int64_t* __restrict__ nact_next) {
  const int64_t j = (int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x;
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t na = min(max(*nact, (int64_t)0), n);
  const int li = j < na ? list[j] : -1;
  const bool active = li >= 0 && li < n;
  const int i = active ? li : 0;
  const bool was_done = active && done[i] != 0;
  int first = G;
  double tf = 0.0;
  if (active && !was_done) {
    const double lm = *lmin;
    const double* xi = x + (int64_t)i * d;
    const double* di = dirn + (int64_t)i * d;
    for (int k = G - 1; k >= 0; --k) {
      const int64_t r = j * G + k;
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
      for (int c = 0; c < d; ++c) xn[(int64_t)i * d + c] = xi[c] + tf * di[c];
      done[i] = 1;
    } else {
      lo[i] = a[i];
      hi[i] = b[i];
    }
  }
  append_stayers(active && !was_done && first == G, lane, i, n, list_next, nact_next);
}

// Lane-parallel forms for groups of at most one wavefront: a chain's L candidates sit on L
// consecutive lanes of one wavefront (64 / L chains per wavefront, spare lanes idle), each lane
// judges its own candidate with loads independent of the others, and a ballot gives each chain
// the index of its first candidate inside (or outside). Same decisions, same arithmetic.
__device__ __forceinline__ uint64_t low_bits(int k) { return k >= 64 ? ~0ull : ((1ull << k) - 1); }
__device__ __forceinline__ uint64_t group_bits(uint64_t mask, int c, int L) { return (mask >> (c * L)) & low_bits(L); }

__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_ends_select_lanes(int64_t n, int d, int m,
                                                                         const double* __restrict__ pts,
                                                                         const double* __restrict__ logl,
                                                                         const double* __restrict__ lmin,
                                                                         double* __restrict__ lo,
                                                                         double* __restrict__ hi,
                                                                         const double* __restrict__ jl) {
  const int L = m - 1, cpw = WAVE / L;
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t wave = ((int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x) / WAVE;
  const int c = lane / L, s = lane - c * L;
  const int64_t i = wave * cpw + c;
  const bool active = c < cpw && i < n;
  bool in = false;
  if (active) {
    const int64_t r = (int64_t)s * n + i;
    in = in_region(pts + r * d, d, logl[r], *lmin);
  }
  const uint64_t mask = __ballot(in);
  if (!active || s != 0) return;
  const uint64_t bits = group_bits(mask, c, L);
  const int nl = (int)jl[i], nr = L - nl;
  const uint64_t out_l = ~bits & low_bits(nl);
  const uint64_t out_r = ~(nl >= 64 ? 0ull : bits >> nl) & low_bits(nr);
  const int sl = out_l ? __builtin_ctzll(out_l) : nl;
  const int sr = out_r ? __builtin_ctzll(out_r) : nr;
  lo[i] = lo[i] - (double)sl;
  hi[i] = hi[i] + (double)sr;
}

__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_select_lanes(int64_t n, int d, int G,
                                                                    const int* __restrict__ list,
                                                                    const int64_t* __restrict__ nact,
                                                                    const double* __restrict__ x,
                                                                    const double* __restrict__ dirn,
                                                                    const double* __restrict__ t,
                                                                    const double* __restrict__ logl,
                                                                    const double* __restrict__ lmin,
                                                                    const double* __restrict__ a,
                                                                    const double* __restrict__ b,
                                                                    double* __restrict__ xn,
                                                                    unsigned char* __restrict__ done,
                                                                    double* __restrict__ lo, double* __restrict__ hi,
                                                                    int* __restrict__ list_next,
                                                                    int64_t* __restrict__ nact_next) {
  const int cpw = WAVE / G;
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t wave = ((int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x) / WAVE;
  const int c = lane / G, k = lane - c * G;
  const int64_t j = wave * cpw + c;
  const int64_t na = min(max(*nact, (int64_t)0), n);
  const int li = c < cpw && j < na ? list[j] : -1;
  const bool active = li >= 0 && li < n;
  const int i = active ? li : 0;
  const bool was_done = active && done[i] != 0;
  bool ok = false;
  if (active && !was_done) {
    const int64_t r = j * G + k;
    const double tk = t[r];
    ok = logl[r] >= *lmin;
    for (int q = 0; q < d; ++q) {
      const double p = x[(int64_t)i * d + q] + tk * dirn[(int64_t)i * d + q];
      ok = ok && p >= 0.0 && p <= 1.0;
    }
  }
  const uint64_t mask = __ballot(ok);
  const bool live = active && !was_done;
  const uint64_t bits = live ? group_bits(mask, c, G) : 0ull;
  append_stayers(live && k == 0 && bits == 0, lane, i, n, list_next, nact_next);
  if (!live) return;
  if (bits == 0) {
    if (k == 0) {
      lo[i] = a[i];
      hi[i] = b[i];
    }
    return;
  }
  // the first draw inside: the chain's lanes write its coordinates together
  const double tf = t[j * G + __builtin_ctzll(bits)];
  for (int q = k; q < d; q += G) xn[(int64_t)i * d + q] = x[(int64_t)i * d + q] + tf * dirn[(int64_t)i * d + q];
  if (k == 0) done[i] = 1;
}

// The list of all n chains, for the first group of a move.
__global__ __launch_bounds__(SLICE_BLOCK) void k_slice_list_init(int64_t n, int* __restrict__ list,
                                                                 int64_t* __restrict__ nact) {
  const int64_t j = (int64_t)blockIdx.x * SLICE_BLOCK + threadIdx.x;
  if (j == 0) *nact = n;
  if (j < n) list[j] = (int)j;
}

static unsigned lane_grid(int64_t n, int L) {
  const int64_t waves = (n + WAVE / L - 1) / (WAVE / L);
  return (unsigned)((waves * WAVE + SLICE_BLOCK - 1) / SLICE_BLOCK);
}

static unsigned grid_of(int64_t n) { return (unsigned)((n + SLICE_BLOCK - 1) / SLICE_BLOCK); }

static gwl_status check_shape(int64_t n, int d, int k) {
  if (n < 1 || n > kMaxBatch || d < 1 || d > 4096 || k < 1 || k > 4096)
    return fail(GWL_E_SHAPE, "n=%lld, d=%d, m or G=%d outside [1, 2^30] x [1, 4096] x [1, 4096]", (long long)n, d, k);
  if ((int64_t)k * n > kMaxBatch) return fail(GWL_E_SHAPE, "%d * %lld points exceed 2^30", k, (long long)n);
  // one thread per coordinate of a stepping-out end: the grid must stay below 2^31 threads
  if ((int64_t)k * n * d > ((int64_t)1 << 31))
    return fail(GWL_E_SHAPE, "%d * %lld * %d coordinates exceed 2^31", k, (long long)n, d);
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
  if (!x || !dirn || !u0 || !u1 || (m > 1 && !pts) || !lo || !hi || !jl || !jr)
    return fail(GWL_E_INVALID, "gwl_slice_ends: null pointer");
  hipStream_t s = (hipStream_t)stream;
  if (m > 1)   // one launch: the slots' points and, from each chain's first thread, its interval
    hipLaunchKernelGGL(k_slice_end_points, dim3(grid_of((int64_t)(m - 1) * n * d)), dim3(SLICE_BLOCK), 0, s, n, d, m,
                       x, dirn, u0, u1, pts, lo, hi, jl, jr);
  else
    hipLaunchKernelGGL(k_slice_ends, dim3(grid_of(n)), dim3(SLICE_BLOCK), 0, s, n, m, u0, u1, lo, hi, jl, jr);
  return launched("gwl_slice_ends");
}

gwl_status gwl_slice_ends_select(int64_t n, int d, int m, const double* pts, const double* logl, const double* lmin,
                                 double* lo, double* hi, const double* jl, const double* jr, void* stream) {
  clear_error();
  gwl_status st = check_shape(n, d, m);
  if (st != GWL_OK) return st;
  if (!lo || !hi || !jl || !jr || (m > 1 && (!pts || !logl || !lmin)))
    return fail(GWL_E_INVALID, "gwl_slice_ends_select: null pointer");
  if (m == 1) return GWL_OK;   // no end to step
  if (m - 1 <= WAVE)
    hipLaunchKernelGGL(k_slice_ends_select_lanes, dim3(lane_grid(n, m - 1)), dim3(SLICE_BLOCK), 0, (hipStream_t)stream,
                       n, d, m, pts, logl, lmin, lo, hi, jl);
  else
    hipLaunchKernelGGL(k_slice_ends_select, dim3(grid_of(n)), dim3(SLICE_BLOCK), 0, (hipStream_t)stream, n, d, m, pts,
                       logl, lmin, lo, hi, jl);
  return launched("gwl_slice_ends_select");
}

gwl_status gwl_slice_move_begin(int64_t n, int d, const double* x, double* xn, unsigned char* done, int* list,
                                int64_t* nact, void* stream) {
  clear_error();
  gwl_status st = check_shape(n, d, 1);
  if (st != GWL_OK) return st;
  if (!x || !xn || !done || !list || !nact) return fail(GWL_E_INVALID, "gwl_slice_move_begin: null pointer");
  hipLaunchKernelGGL(k_slice_move_begin, dim3(grid_of(n * d)), dim3(SLICE_BLOCK), 0, (hipStream_t)stream, n, d, x, xn,
                     done, list, nact);
  return launched("gwl_slice_move_begin");
}

gwl_status gwl_slice_move_end(int64_t n, int d, const unsigned char* done, unsigned char* moved, const double* xn,
                              double* x, void* stream) {
  clear_error();
  gwl_status st = check_shape(n, d, 1);
  if (st != GWL_OK) return st;
  if (!done || !moved || !xn || !x) return fail(GWL_E_INVALID, "gwl_slice_move_end: null pointer");
  hipLaunchKernelGGL(k_slice_move_end, dim3(grid_of(n * d)), dim3(SLICE_BLOCK), 0, (hipStream_t)stream, n, d, done,
                     moved, xn, x);
  return launched("gwl_slice_move_end");
}

gwl_status gwl_slice_list_init(int64_t n, int* list, int64_t* nact, void* stream) {
  clear_error();
  if (n < 1 || n > kMaxBatch) return fail(GWL_E_SHAPE, "n=%lld outside [1, 2^30]", (long long)n);
  if (!list || !nact) return fail(GWL_E_INVALID, "gwl_slice_list_init: null pointer");
  hipLaunchKernelGGL(k_slice_list_init, dim3(grid_of(n)), dim3(SLICE_BLOCK), 0, (hipStream_t)stream, n, list, nact);
  return launched("gwl_slice_list_init");
}

gwl_status gwl_slice_draws(int64_t n, int d, int G, const int* list, const int64_t* nact, const double* x,
                           const double* dirn, const double* lo, const double* hi, const double* u, double* t,
                           double* pts, double* a, double* b, int64_t* live, int64_t* nact_next, int64_t* calls,
                           void* stream) {
  clear_error();
  gwl_status st = check_shape(n, d, G);
  if (st != GWL_OK) return st;
  if (!list || !nact || !x || !dirn || !lo || !hi || !u || !t || !pts || !a || !b || !live || !nact_next)
    return fail(GWL_E_INVALID, "gwl_slice_draws: null pointer");
  if (nact_next == nact) return fail(GWL_E_INVALID, "gwl_slice_draws: nact_next must not be nact");
  hipLaunchKernelGGL(k_slice_draws, dim3(grid_of(n * d)), dim3(SLICE_BLOCK), 0, (hipStream_t)stream, n, d, G, list,
                     nact, x, dirn, lo, hi, u, t, pts, a, b, live, nact_next, calls);
  return launched("gwl_slice_draws");
}

gwl_status gwl_slice_select(int64_t n, int d, int G, const int* list, const int64_t* nact, const double* x,
                            const double* dirn, const double* t, const double* logl, const double* lmin,
                            const double* a, const double* b, double* xn, unsigned char* done, double* lo, double* hi,
                            int* list_next, int64_t* nact_next, void* stream) {
  clear_error();
  gwl_status st = check_shape(n, d, G);
  if (st != GWL_OK) return st;
  if (!list || !nact || !x || !dirn || !t || !logl || !lmin || !a || !b || !xn || !done || !lo || !hi || !list_next ||
      !nact_next)
    return fail(GWL_E_INVALID, "gwl_slice_select: null pointer");
  if (list_next == list || nact_next == nact)
    return fail(GWL_E_INVALID, "gwl_slice_select: the next list must not be the current one");
  if (G <= WAVE)
    hipLaunchKernelGGL(k_slice_select_lanes, dim3(lane_grid(n, G)), dim3(SLICE_BLOCK), 0, (hipStream_t)stream, n, d, G,
                       list, nact, x, dirn, t, logl, lmin, a, b, xn, done, lo, hi, list_next, nact_next);
  else
    hipLaunchKernelGGL(k_slice_select, dim3(grid_of(n)), dim3(SLICE_BLOCK), 0, (hipStream_t)stream, n, d, G, list,
                       nact, x, dirn, t, logl, lmin, a, b, xn, done, lo, hi, list_next, nact_next);
  return launched("gwl_slice_select");
}

}  // extern "C"
