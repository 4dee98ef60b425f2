// Several events of uneven duration and batch size in one persistent launch, captured in a
// HIP graph (the batch axis of the paper's parallel prior sampling, section 3, extended over
// events).
//
// Work items are (event, 64-point group, bin chunk) with one chunk length for all events, so
// items cost about the same; events are queued shortest first, items of an event chunk-major.
// Every wavefront of the persistent kernel takes items from an atomic counter until the queue
// is empty; each item writes its own partial sums, which a multi-event epilogue launch adds in
// chunk order (deterministic). A per-event counter stamps the device clock when the last item
// of the event completes. The graph is: reset (counters and start stamp, by a kernel) ->
// per-point set-up for all events -> persistent bin loop -> epilogue for all events.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stddef.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "gwl_bins.h"
#include "gwl_epilogue.h"
#include "gwl_runtime.h"

using namespace gwl;

namespace gwl {

constexpr int MULTI_PT_BLOCK = 128;

struct MultiEvDev {
  const void* tab;         // RowMixed<ND> or RowF64<ND> [M]
  const void* gtab;        // RowGradF64 [M] (adjoint basis, both precisions)
  const EventConst* ec;
  double* coef;            // [NCOEF][Bp]
  double* part;            // [nchunk][NZ][Bp]
  int64_t Bp;
  int M, chunk, nchunk, npg;
  int item0, nitems;       // first item in the queue, item count
  int f64;                 // 1: float64 tables and loop (every event of a float64 plan, and the
                           // relative-binning events of a mixed one)
  int rot;                 // 1: the float64 loop on a uniform grid rotates the detectors' phasors
  double step;             // the uniform grid's spacing (rot)
};

struct MultiIODev {
  const double* theta;     // [B][11]
  double* logl;            // [B]
  double* grad;            // [B][11] or null
  int64_t B;
};

struct MultiCtl {
  unsigned int next;       // queue head
  unsigned int pad;
  unsigned long long t0;   // device clock at the start of the launch
  unsigned long long tend; // device clock at the end of the epilogue
};

__global__ void k_multi_reset(MultiCtl* __restrict__ ctl, unsigned int* __restrict__ done,
                              unsigned long long* __restrict__ tev, int E) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < E) {
    done[i] = 0u;
    tev[i] = 0ull;
  }
  if (i == 0) {
    ctl->next = 0u;
    ctl->pad = 0u;
    ctl->t0 = wall_clock64();
    ctl->tend = 0ull;
  }
}

// device clock stamp (a calibrated event's completion)
__global__ void k_multi_stamp(unsigned long long* __restrict__ t) { *t = wall_clock64(); }

template <int ND>
__global__ __launch_bounds__(MULTI_PT_BLOCK) void k_multi_setup(const MultiEvDev* __restrict__ evs,
                                                                 const EventGeom* __restrict__ geoms,
                                                                 const MultiIODev* __restrict__ io,
                                                                 const int* __restrict__ blk_ev,
                                                                 const int* __restrict__ blk_p0) {
  const int e = blk_ev[blockIdx.x];
  const int64_t p = (int64_t)blk_p0[blockIdx.x] + threadIdx.x;
  const MultiEvDev ev = evs[e];
  const MultiIODev o = io[e];
  if (p >= ev.Bp) return;
  const int64_t pc = p < o.B ? p : o.B - 1;
  double th[NPARAM];
#pragma unroll
  for (int i = 0; i < NPARAM; ++i) th[i] = o.theta[pc * NPARAM + i];
  double rows[NCOEF];
  const bool valid = setup_rows<ND>(th, geoms[e], ev.ec, ev.f64 == 0, rows);
  const double nan = __builtin_nan("");
#pragma unroll
  for (int j = 0; j < NCOEF; ++j) ev.coef[j * ev.Bp + p] = valid ? rows[j] : nan;
}

// Persistent bin loop: one wavefront per item, items from the shared counter. ANYF64: a mixed
// plan that also holds float64 (relative-binning) events, which take the float64 loop.
template <int ND, bool MIXED, bool GRAD, bool ANYF64>
__global__ __launch_bounds__(BLOCK, (ND <= 3 ? (GRAD && MIXED && !ANYF64 ? 5 : 4) : 3)) void k_multi_bins(
    const MultiEvDev* __restrict__ evs, int E, int total, const MultiIODev* __restrict__ io,
    MultiCtl* __restrict__ ctl, unsigned int* __restrict__ done, unsigned long long* __restrict__ tev) {
  constexpr int NZ = nz_of(ND, GRAD);
  constexpr bool TBL = !MIXED || ANYF64;
  __shared__ double2 tbl[TBL ? PH_TBL : 1];  // the float64 phasor table
  if constexpr (TBL) fill_phasor_table(tbl);
  __syncthreads();
  const int lane = threadIdx.x % WAVE;
  for (;;) {
    // One ticket per wavefront. Every lane takes part in the atomic (lane 0 adds 1, the others
    // 0) and the first lane's old value is read back as a scalar, so the loop is wave-uniform:
    // a per-lane broadcast (a shuffle inside lane-divergent control flow) lets the compiler
    // separate the lane that takes the ticket from the lanes that read it, and those then
    // never see the queue advance.
    const unsigned int ticket = atomicAdd(&ctl->next, lane == 0 ? 1u : 0u);
    const int it = (int)__builtin_amdgcn_readfirstlane(ticket);
    if (it >= total) break;
    // event of this item: queue order is event order, item0 increasing
    int e = 0;
    while (e + 1 < E && evs[e + 1].item0 <= it) ++e;
    const MultiEvDev ev = evs[e];
    const int64_t B = io[e].B;
    const int local = it - ev.item0;
    const int c = local / ev.npg;
    const int pg = local - c * ev.npg;
    const int64_t p = (int64_t)pg * WAVE + lane;
    const int64_t pc = p < B ? p : B - 1;
    const int k0 = c * ev.chunk;
    const int k1 = k0 + ev.chunk < ev.M ? k0 + ev.chunk : ev.M;
    double tot[NZ];
    double a[NBASIS], T[ND];
    bool f64path = !MIXED;
    if constexpr (MIXED && ANYF64) f64path = ev.f64 != 0;  // wave-uniform (scalar) branch
    if (!f64path) {
      if constexpr (MIXED) {
        float cr[ND], ci[ND];
        load_coef<ND, float>(ev.coef, ev.Bp, pc, GRAD, a, T, cr, ci);
        bin_loop_mixed<ND, GRAD>((const_as_ptr<RowMixed<ND>>)ev.tab, (const_as_ptr<RowGradF64>)ev.gtab, k0, k1, a,
                                 T, cr, ci, tot);
      }
    } else {
      if constexpr (TBL) {
        double cr[ND], ci[ND];
        load_coef<ND, double>(ev.coef, ev.Bp, pc, GRAD, a, T, cr, ci);
        to_table_units<ND>(a, T);
        if (ev.rot)
          bin_loop_f64_rot<ND, GRAD>((const_as_ptr<RowF64<ND>>)ev.tab, (const_as_ptr<RowGradF64>)ev.gtab, k0, k1, a,
                                     T, cr, ci, tbl, ev.step, tot);
        else
          bin_loop_f64<ND, GRAD>((const_as_ptr<RowF64<ND>>)ev.tab, (const_as_ptr<RowGradF64>)ev.gtab, k0, k1, a, T,
                                 cr, ci, tbl, tot);
      }
    }
    global_as_ptr<double> part = (global_as_ptr<double>)ev.part;
#pragma unroll
    for (int z = 0; z < NZ; ++z) part[((int64_t)c * NZ + z) * ev.Bp + p] = tot[z];
    const unsigned int prev = atomicAdd(&done[e], lane == 0 ? 1u : 0u);
    const unsigned int d = __builtin_amdgcn_readfirstlane(prev);
    if (d + 1u == (unsigned int)ev.nitems && lane == 0) tev[e] = wall_clock64();
  }
}

template <int ND, bool GRAD>
__global__ __launch_bounds__(MULTI_PT_BLOCK) void k_multi_epilogue(const MultiEvDev* __restrict__ evs,
                                                                    const EventGeom* __restrict__ geoms,
                                                                    const MultiIODev* __restrict__ io,
                                                                    const int* __restrict__ blk_ev,
                                                                    const int* __restrict__ blk_p0,
                                                                    MultiCtl* __restrict__ ctl) {
  constexpr int NZ = nz_of(ND, GRAD);
  const int e = blk_ev[blockIdx.x];
  const int64_t p = (int64_t)blk_p0[blockIdx.x] + threadIdx.x;
  const MultiEvDev ev = evs[e];
  const MultiIODev o = io[e];
  const bool scaled = ev.f64 == 0;
  if (p < o.B) {
    const EventConst ec = *ev.ec;
    double acc[NZ];
    gather<NZ>(ev.part, ev.nchunk, ev.Bp, p, acc);
    if (scaled) apply_gain<ND>(ec, acc);
    if constexpr (GRAD) {
      double th[NPARAM];
#pragma unroll
      for (int i = 0; i < NPARAM; ++i) th[i] = o.theta[p * NPARAM + i];
      const double nan = __builtin_nan("");
      bool valid;
      double gout[NPARAM];
      const double v = epilogue_gradient<ND>(acc, th, geoms[e], ec, scaled ? ec.uref : 1.0, valid, gout);
      o.logl[p] = valid ? v : nan;
#pragma unroll
      for (int j = 0; j < NPARAM; ++j) o.grad[p * NPARAM + j] = valid ? gout[j] : nan;
    } else {
      o.logl[p] = epilogue_value_rows<ND, NZ>(acc, ev.coef, ev.Bp, p, ec, scaled ? ec.uref : 1.0);
    }
  }
  if (threadIdx.x == 0) atomicMax(&ctl->tend, wall_clock64());
}

}  // namespace gwl

struct gwl_plan_s {
  int device = 0;
  int E = 0, nd = 0;
  bool mixed = false, grad = false;
  bool anyf64 = false;         // a mixed plan with float64 (relative-binning) events
  std::vector<int64_t> B;
  std::vector<gwl_event> evs;  // the events (event order)
  std::vector<int> cal;        // calibrated events (event index): their own kernels, after the graph
  std::vector<int> order;      // queue position -> event index
  int total = 0, grid = 0, nptblk = 0, chunk = 0;
  bool descending = false;     // queue order: events by descending work instead of ascending
  double clock_khz = 0.0;
  gwl::MultiEvDev* d_evs = nullptr;   // in queue order
  gwl::EventGeom* d_geoms = nullptr;  // in queue order
  gwl::MultiIODev* d_io = nullptr;    // in queue order
  gwl::MultiIODev* h_io = nullptr;    // pinned host staging
  int* d_blk = nullptr;               // [2][nptblk]: event (queue index), first point
  void* d_ctl = nullptr;              // MultiCtl, done[E], tev[E]
  unsigned long long* h_stamps = nullptr;  // pinned: t0, tend, tev[E]
  double* ws = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t io_done = nullptr;
  // calibrated events run on side streams (default priority) after the graph, the calibrated
  // events in turn, each stream in a workspace of the plan's own sized for its largest event
  static constexpr int kCalStreams = 4;
  hipStream_t cal_s[kCalStreams] = {};
  void* cal_ws[kCalStreams] = {};
  size_t cal_ws_bytes[kCalStreams] = {};
  hipEvent_t cal_fork = nullptr;
  hipEvent_t cal_join[kCalStreams] = {};
};

namespace {

// Set to false to switch the multi-event plan off.
constexpr bool kMultiEnabled = true;

size_t ctl_bytes(int E) {
  return sizeof(gwl::MultiCtl) + sizeof(unsigned int) * (size_t)((E + 1) & ~1) + sizeof(unsigned long long) * E;
}

// precision of calibrated event e's own kernels in plan pl (as its single call would take)
bool mixed_cal(const gwl_plan_s* pl, int e) { return pl->mixed && use_mixed(pl->evs[e], GWL_MIXED); }

void plan_free(gwl_plan pl) {
  if (!pl) return;
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  if (pl->cap) (void)hipStreamDestroy(pl->cap);
  if (pl->io_done) (void)hipEventDestroy(pl->io_done);
  for (int i = 0; i < gwl_plan_s::kCalStreams; ++i) {
    if (pl->cal_s[i]) (void)hipStreamDestroy(pl->cal_s[i]);
    if (pl->cal_join[i]) (void)hipEventDestroy(pl->cal_join[i]);
    if (pl->cal_ws[i]) (void)hipFree(pl->cal_ws[i]);
  }
  if (pl->cal_fork) (void)hipEventDestroy(pl->cal_fork);
  if (pl->d_evs) (void)hipFree(pl->d_evs);
  if (pl->d_geoms) (void)hipFree(pl->d_geoms);
  if (pl->d_io) (void)hipFree(pl->d_io);
  if (pl->d_blk) (void)hipFree(pl->d_blk);
  if (pl->d_ctl) (void)hipFree(pl->d_ctl);
  if (pl->ws) (void)hipFree(pl->ws);
  if (pl->h_io) (void)hipHostFree(pl->h_io);
  if (pl->h_stamps) (void)hipHostFree(pl->h_stamps);
  delete pl;
}

template <int ND>
hipError_t enqueue_multi_nd(gwl_plan pl, hipStream_t s) {
  const int E = pl->E;
  unsigned char* ctl = (unsigned char*)pl->d_ctl;
  gwl::MultiCtl* c = (gwl::MultiCtl*)ctl;
  unsigned int* done = (unsigned int*)(ctl + sizeof(gwl::MultiCtl));
  unsigned long long* tev =
      (unsigned long long*)(ctl + sizeof(gwl::MultiCtl) + sizeof(unsigned int) * (size_t)((E + 1) & ~1));
  const int* blk_ev = pl->d_blk;
  const int* blk_p0 = pl->d_blk + pl->nptblk;
  hipLaunchKernelGGL(gwl::k_multi_reset, dim3((E + 255) / 256), dim3(256), 0, s, c, done, tev, E);
  if (pl->nptblk > 0)   // no point outside calibrated events: only the reset and the (empty) queue
    hipLaunchKernelGGL(gwl::k_multi_setup<ND>, dim3(pl->nptblk), dim3(gwl::MULTI_PT_BLOCK), 0, s,
                       (const gwl::MultiEvDev*)pl->d_evs, (const gwl::EventGeom*)pl->d_geoms,
                       (const gwl::MultiIODev*)pl->d_io, blk_ev, blk_p0);
#define GWL_MB(MX, GR, AF)                                                                                         \
  hipLaunchKernelGGL((gwl::k_multi_bins<ND, MX, GR, AF>), dim3(pl->grid), dim3(gwl::BLOCK), 0, s,               \
                     (const gwl::MultiEvDev*)pl->d_evs, E, pl->total, (const gwl::MultiIODev*)pl->d_io, c, done, tev)
  if (pl->mixed) {
    if (pl->anyf64) {
      if (pl->grad) GWL_MB(true, true, true); else GWL_MB(true, false, true);
    } else {
      if (pl->grad) GWL_MB(true, true, false); else GWL_MB(true, false, false);
    }
  } else {
    if (pl->grad) GWL_MB(false, true, false); else GWL_MB(false, false, false);
  }
#undef GWL_MB
  if (pl->nptblk == 0) return hipGetLastError();
  if (pl->grad)
    hipLaunchKernelGGL((gwl::k_multi_epilogue<ND, true>), dim3(pl->nptblk), dim3(gwl::MULTI_PT_BLOCK), 0, s,
                       (const gwl::MultiEvDev*)pl->d_evs, (const gwl::EventGeom*)pl->d_geoms,
                       (const gwl::MultiIODev*)pl->d_io, blk_ev, blk_p0, c);
  else
    hipLaunchKernelGGL((gwl::k_multi_epilogue<ND, false>), dim3(pl->nptblk), dim3(gwl::MULTI_PT_BLOCK), 0, s,
                       (const gwl::MultiEvDev*)pl->d_evs, (const gwl::EventGeom*)pl->d_geoms,
                       (const gwl::MultiIODev*)pl->d_io, blk_ev, blk_p0, c);
  return hipGetLastError();
}

hipError_t enqueue_multi(gwl_plan pl, hipStream_t s) {
  switch (pl->nd) {
    case 1: return enqueue_multi_nd<1>(pl, s);
    case 2: return enqueue_multi_nd<2>(pl, s);
    case 3: return enqueue_multi_nd<3>(pl, s);
    case 4: return enqueue_multi_nd<4>(pl, s);
  }
  return hipErrorInvalidValue;
}

template <int ND>
hipError_t occupancy_nd(bool mixed, bool grad, bool anyf64, int* nblk) {
#define GWL_OCC(MX, GR, AF) \
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(nblk, gwl::k_multi_bins<ND, MX, GR, AF>, gwl::BLOCK, 0)
  if (mixed) {
    if (anyf64) {
      if (grad) GWL_OCC(true, true, true); else GWL_OCC(true, false, true);
    } else {
      if (grad) GWL_OCC(true, true, false); else GWL_OCC(true, false, false);
    }
  } else {
    if (grad) GWL_OCC(false, true, false); else GWL_OCC(false, false, false);
  }
#undef GWL_OCC
}

hipError_t occupancy(int nd, bool mixed, bool grad, bool anyf64, int* nblk) {
  switch (nd) {
    case 1: return occupancy_nd<1>(mixed, grad, anyf64, nblk);
    case 2: return occupancy_nd<2>(mixed, grad, anyf64, nblk);
    case 3: return occupancy_nd<3>(mixed, grad, anyf64, nblk);
    case 4: return occupancy_nd<4>(mixed, grad, anyf64, nblk);
  }
  return hipErrorInvalidValue;
}

}  // namespace

namespace gwl {

// Build a plan with a given chunk length (0: the heuristic) and queue order.
gwl_status build_plan(const gwl_event* evs, int E, const int64_t* B_e, gwl_precision prec, int with_grad,
                      int chunk_req, bool descending, gwl_plan* out) {
  if (!out) return fail(GWL_E_INVALID, "out is null");
  *out = nullptr;
  if (!evs || !B_e) return fail(GWL_E_INVALID, "evs and B_e must be host arrays");
  if (E < 1 || E > 4096) return fail(GWL_E_SHAPE, "E=%d outside [1, 4096]", E);
  if (prec != GWL_FP64 && prec != GWL_MIXED) return fail(GWL_E_INVALID, "unknown precision %d", (int)prec);
  const int nd = evs[0] ? evs[0]->ndet : 0;
  for (int e = 0; e < E; ++e) {
    if (!evs[e]) return fail(GWL_E_INVALID, "event %d is null", e);
    if (evs[e]->ndet != nd) return fail(GWL_E_UNSUPPORTED, "events must share one detector count");
    if (evs[e]->ech.isco) return fail(GWL_E_UNSUPPORTED, "event %d has the ISCO cut-off: not in multi-event plans", e);
    if (evs[e]->device != evs[0]->device) return fail(GWL_E_INVALID, "events must live on one device");
    if (B_e[e] < 0 || B_e[e] > kMaxBatch) return fail(GWL_E_SHAPE, "B_e[%d]=%lld out of range", e, (long long)B_e[e]);
  }
  gwl_status st = check_device(evs[0]->device);
  if (st != GWL_OK) return st;
  if (!kMultiEnabled)
    return fail(GWL_E_UNSUPPORTED, "the persistent multi-event launch is switched off");

  gwl_plan pl = new (std::nothrow) gwl_plan_s();
  if (!pl) return fail(GWL_E_NOMEM, "host allocation failed");
  pl->device = evs[0]->device;
  pl->E = E;
  pl->nd = nd;
  pl->mixed = prec == GWL_MIXED;
  pl->grad = with_grad != 0;
  pl->B.assign(B_e, B_e + E);
  pl->evs.assign(evs, evs + E);
  for (int e = 0; e < E; ++e)
    if (evs[e]->ncal > 0) pl->cal.push_back(e);
  // a mixed plan runs its relative-binning events on the float64 loop, as single calls do
  for (int e = 0; e < E; ++e) pl->anyf64 |= pl->mixed && !use_mixed(evs[e], prec);

  // one chunk length for all events: the largest power of two in [1024, 16384] that still
  // gives at least four items per resident wavefront
  hipError_t err = hipSuccess;
  int occ = 0, ncu = 0, clk = 0;
  err = occupancy(nd, pl->mixed, pl->grad, pl->anyf64, &occ);
  if (err == hipSuccess) err = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, pl->device);
  if (err == hipSuccess) err = hipDeviceGetAttribute(&clk, hipDeviceAttributeWallClockRate, pl->device);
  if (err != hipSuccess) {
    plan_free(pl);
    return hip_fail(err, "device query");
  }
  if (occ < 1) occ = 1;
  pl->grid = occ * ncu;
  pl->clock_khz = (double)clk;
  const int64_t resident = (int64_t)pl->grid * WAVES_PER_BLOCK;
  auto items_for = [&](int chunk) {
    int64_t n = 0;
    for (int e = 0; e < E; ++e) {
      if (B_e[e] == 0 || evs[e]->ncal > 0) continue;
      n += ((B_e[e] + WAVE - 1) / WAVE) * ((evs[e]->M + chunk - 1) / chunk);
    }
    return n;
  };
  int chunk = 1024;
  for (int c = 16384; c >= 1024; c >>= 1) {
    if (items_for(c) >= 4 * resident) {
      chunk = c;
      break;
    }
  }
  if (chunk_req > 0) chunk = chunk_req;
  const int64_t total = items_for(chunk);
  if (total > ((int64_t)1 << 30)) {
    plan_free(pl);
    return fail(GWL_E_SHAPE, "too many work items (%lld)", (long long)total);
  }
  pl->chunk = chunk;
  pl->total = (int)total;

  // queue order: events by ascending (or descending) work, ties by index
  pl->descending = descending;
  pl->order.resize(E);
  std::iota(pl->order.begin(), pl->order.end(), 0);
  std::stable_sort(pl->order.begin(), pl->order.end(), [&](int a, int b) {
    const double wa = (double)B_e[a] * (double)evs[a]->M, wb = (double)B_e[b] * (double)evs[b]->M;
    return descending ? wa > wb : wa < wb;
  });

  // workspace and device tables
  const int NZ = nz_of(nd, pl->grad);
  std::vector<MultiEvDev> hev(E);
  std::vector<EventGeom> hgeo(E);
  std::vector<int> blk_ev, blk_p0;
  size_t ws_doubles = 0;
  int item0 = 0;
  for (int q = 0; q < E; ++q) {
    const int e = pl->order[q];
    const gwl_event ev = evs[e];
    MultiEvDev& d = hev[q];
    memset(&d, 0, sizeof d);
    const int64_t B = evs[e]->ncal > 0 ? 0 : B_e[e];   // calibrated events are not in the queue
    d.npg = (int)((B + WAVE - 1) / WAVE);
    d.Bp = (int64_t)d.npg * WAVE;
    d.M = (int)ev->M;
    d.chunk = chunk;
    d.nchunk = B > 0 ? (int)((ev->M + chunk - 1) / chunk) : 0;
    d.item0 = item0;
    d.nitems = d.npg * d.nchunk;
    item0 += d.nitems;
    d.f64 = use_mixed(ev, prec) ? 0 : 1;
    d.rot = d.f64 && ev->ech.uniform != 0 ? 1 : 0;
    d.step = ev->ech.grid_df;
    d.tab = d.f64 ? ev->tab64 : ev->tab32;
    d.gtab = ev->g64;
    d.ec = ev->ec;
    ws_doubles += (size_t)NCOEF * d.Bp + (size_t)d.nchunk * NZ * d.Bp;
    hgeo[q] = ev->geom;
    for (int64_t p0 = 0; p0 < d.Bp; p0 += MULTI_PT_BLOCK) {
      blk_ev.push_back(q);
      blk_p0.push_back((int)p0);
    }
  }
  pl->nptblk = (int)blk_ev.size();
  err = hipMalloc((void**)&pl->ws, sizeof(double) * (ws_doubles > 0 ? ws_doubles : 1));
  size_t off = 0;
  for (int q = 0; q < E; ++q) {
    MultiEvDev& d = hev[q];
    d.coef = pl->ws + off;
    off += (size_t)NCOEF * d.Bp;
    d.part = pl->ws + off;
    off += (size_t)d.nchunk * NZ * d.Bp;
  }
  std::vector<int> blk(blk_ev);
  blk.insert(blk.end(), blk_p0.begin(), blk_p0.end());
  if (err == hipSuccess) err = hipMalloc((void**)&pl->d_evs, sizeof(MultiEvDev) * E);
  if (err == hipSuccess) err = hipMalloc((void**)&pl->d_geoms, sizeof(EventGeom) * E);
  if (err == hipSuccess) err = hipMalloc((void**)&pl->d_io, sizeof(MultiIODev) * E);
  if (err == hipSuccess) err = hipMalloc((void**)&pl->d_blk, sizeof(int) * (blk.empty() ? 1 : blk.size()));
  if (err == hipSuccess) err = hipMalloc(&pl->d_ctl, ctl_bytes(E));
  if (err == hipSuccess) err = hipHostMalloc((void**)&pl->h_io, sizeof(MultiIODev) * E, hipHostMallocDefault);
  if (err == hipSuccess)
    err = hipHostMalloc((void**)&pl->h_stamps, sizeof(unsigned long long) * (2 + E), hipHostMallocDefault);
  if (err == hipSuccess) err = hipMemcpy(pl->d_evs, hev.data(), sizeof(MultiEvDev) * E, hipMemcpyHostToDevice);
  if (err == hipSuccess) err = hipMemcpy(pl->d_geoms, hgeo.data(), sizeof(EventGeom) * E, hipMemcpyHostToDevice);
  if (err == hipSuccess && !blk.empty())
    err = hipMemcpy(pl->d_blk, blk.data(), sizeof(int) * blk.size(), hipMemcpyHostToDevice);
  if (err == hipSuccess) {
    memset(pl->h_io, 0, sizeof(MultiIODev) * E);
    err = hipMemcpy(pl->d_io, pl->h_io, sizeof(MultiIODev) * E, hipMemcpyHostToDevice);
  }
  if (err == hipSuccess) err = hipEventCreateWithFlags(&pl->io_done, hipEventDisableTiming);
  if (err == hipSuccess) err = hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking);
  if (!pl->cal.empty()) {
    if (err == hipSuccess) err = hipEventCreateWithFlags(&pl->cal_fork, hipEventDisableTiming);
    for (int i = 0; i < gwl_plan_s::kCalStreams && err == hipSuccess; ++i) {
      err = hipStreamCreateWithFlags(&pl->cal_s[i], hipStreamNonBlocking);
      if (err == hipSuccess) err = hipEventCreateWithFlags(&pl->cal_join[i], hipEventDisableTiming);
    }
    int next = 0;
    for (int e : pl->cal) {
      if (pl->B[e] == 0) continue;
      const int i = next++ % gwl_plan_s::kCalStreams;
      pl->cal_ws_bytes[i] = std::max(pl->cal_ws_bytes[i],
                                     call_workspace_bytes(pl->evs[e], pl->B[e], mixed_cal(pl, e), pl->grad));
    }
    for (int i = 0; i < gwl_plan_s::kCalStreams && err == hipSuccess; ++i)
      if (pl->cal_ws_bytes[i] > 0) err = hipMalloc(&pl->cal_ws[i], pl->cal_ws_bytes[i]);
  }
  // capture the whole evaluation once
  if (err == hipSuccess) err = hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal);
  if (err == hipSuccess) {
    hipError_t e1 = enqueue_multi(pl, pl->cap);
    hipError_t e2 = hipStreamEndCapture(pl->cap, &pl->graph);
    err = e1 != hipSuccess ? e1 : e2;
  }
  if (err == hipSuccess) err = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
  if (err != hipSuccess) {
    plan_free(pl);
    return hip_fail(err, "multi-event plan");
  }
  *out = pl;
  return GWL_OK;
}

}  // namespace gwl

extern "C" {

gwl_status gwl_multi_plan_create(const gwl_event* evs, int E, const int64_t* B_e, gwl_precision prec, int with_grad,
                                 gwl_plan* out) {
  clear_error();
  int chunk = 0;
  bool desc = false;
  if (evs && B_e && E >= 1 && E <= 4096) {
    bool ok = true;
    for (int e = 0; e < E; ++e) ok &= evs[e] != nullptr;
    if (ok) choose_multi_shape(evs, E, B_e, prec == GWL_MIXED, with_grad != 0, &chunk, &desc);
  }
  return build_plan(evs, E, B_e, prec, with_grad, chunk, desc, out);
}

gwl_status gwl_multi_plan_create_order(const gwl_event* evs, int E, const int64_t* B_e, gwl_precision prec,
                                       int with_grad, int order, gwl_plan* out) {
  clear_error();
  if (order < 0 || order > 2) return fail(GWL_E_INVALID, "order must be 0 (tuned), 1 (ascending) or 2 (descending)");
  int chunk = 0;
  bool desc = false;
  if (evs && B_e && E >= 1 && E <= 4096) {
    bool ok = true;
    for (int e = 0; e < E; ++e) ok &= evs[e] != nullptr;
    if (ok) choose_multi_shape(evs, E, B_e, prec == GWL_MIXED, with_grad != 0, &chunk, &desc);
  }
  if (order == 1) desc = false;
  if (order == 2) desc = true;
  return build_plan(evs, E, B_e, prec, with_grad, chunk, desc, out);
}

gwl_status gwl_plan_info(gwl_plan pl, int* chunk, int* descending, int64_t* items) {
  clear_error();
  if (!pl) return fail(GWL_E_INVALID, "plan is null");
  if (chunk) *chunk = pl->chunk;
  if (descending) *descending = pl->descending ? 1 : 0;
  if (items) *items = pl->total;
  return GWL_OK;
}

gwl_status gwl_multi_launch(gwl_plan pl, const double* const* theta, double* const* logl, double* const* grad,
                            double* event_latency_us, void* stream) {
  clear_error();
  if (!pl) return fail(GWL_E_INVALID, "plan is null");
  if (!theta || !logl) return fail(GWL_E_INVALID, "theta and logl must be host arrays of device pointers");
  if (pl->grad && !grad) return fail(GWL_E_INVALID, "the plan computes gradients: grad must be given");
  for (int e = 0; e < pl->E; ++e) {
    if (pl->B[e] == 0) continue;
    if (!theta[e] || !logl[e] || (pl->grad && !grad[e]))
      return fail(GWL_E_INVALID, "event %d: null device pointer", e);
  }
  gwl_status st = check_device(pl->device);
  if (st != GWL_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  // the staging buffer is reused: wait until the previous upload has been consumed
  hipError_t err = hipEventSynchronize(pl->io_done);
  if (err != hipSuccess) return hip_fail(err, "plan staging");
  for (int q = 0; q < pl->E; ++q) {
    const int e = pl->order[q];
    pl->h_io[q].theta = theta[e];
    pl->h_io[q].logl = logl[e];
    pl->h_io[q].grad = pl->grad ? grad[e] : nullptr;
    pl->h_io[q].B = pl->evs[e]->ncal > 0 ? 0 : pl->B[e];
  }
  err = hipMemcpyAsync(pl->d_io, pl->h_io, sizeof(MultiIODev) * pl->E, hipMemcpyHostToDevice, s);
  if (err == hipSuccess) err = hipEventRecord(pl->io_done, s);
  if (err == hipSuccess) err = hipGraphLaunch(pl->exec, s);
  if (err != hipSuccess) return hip_fail(err, "multi-event launch");
  // calibrated events: their own set-up, bin-loop and epilogue kernels, each followed by a clock
  // stamp in the event's slot, dealt in turn to the plan's side streams after the graph (one small
  // event at a time leaves most of the chip idle); the caller's stream then waits for them all
  unsigned long long* tev_dev = (unsigned long long*)((unsigned char*)pl->d_ctl + sizeof(MultiCtl) +
                                                      sizeof(unsigned int) * (size_t)((pl->E + 1) & ~1));
  if (!pl->cal.empty()) {
    constexpr int NS = gwl_plan_s::kCalStreams;
    err = hipEventRecord(pl->cal_fork, s);
    for (int i = 0; i < NS && err == hipSuccess; ++i) err = hipStreamWaitEvent(pl->cal_s[i], pl->cal_fork, 0);
    if (err != hipSuccess) return hip_fail(err, "multi-event launch");
    int next = 0;
    for (int e : pl->cal) {
      if (pl->B[e] == 0) continue;
      const int i = next++ % NS;
      hipStream_t cs = pl->cal_s[i];
      st = run_calibrated(pl->evs[e], theta[e], pl->B[e], mixed_cal(pl, e), pl->grad, logl[e],
                          pl->grad ? grad[e] : nullptr, cs, pl->cal_ws[i], pl->cal_ws_bytes[i]);
      if (st != GWL_OK) break;
      int q = 0;
      while (pl->order[q] != e) ++q;
      hipLaunchKernelGGL(k_multi_stamp, dim3(1), dim3(1), 0, cs, tev_dev + q);
      err = hipGetLastError();
      if (err != hipSuccess) break;
    }
    // join, also after a failure, so that nothing queued on a side stream outlives the call's order
    hipError_t jerr = hipSuccess;
    for (int i = 0; i < NS; ++i) {
      hipError_t e1 = hipEventRecord(pl->cal_join[i], pl->cal_s[i]);
      if (e1 == hipSuccess) e1 = hipStreamWaitEvent(s, pl->cal_join[i], 0);
      if (e1 != hipSuccess && jerr == hipSuccess) jerr = e1;
    }
    if (st != GWL_OK) return st;
    if (err != hipSuccess) return hip_fail(err, "multi-event launch");
    if (jerr != hipSuccess) return hip_fail(jerr, "multi-event launch");
  }
  if (event_latency_us) {
    const unsigned char* ctl = (const unsigned char*)pl->d_ctl;
    const size_t tev_off = sizeof(MultiCtl) + sizeof(unsigned int) * (size_t)((pl->E + 1) & ~1);
    err = hipMemcpyAsync(pl->h_stamps, ctl + offsetof(MultiCtl, t0), sizeof(unsigned long long) * 2,
                         hipMemcpyDeviceToHost, s);
    if (err == hipSuccess)
      err = hipMemcpyAsync(pl->h_stamps + 2, ctl + tev_off, sizeof(unsigned long long) * pl->E,
                           hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    if (err != hipSuccess) return hip_fail(err, "latency read-back");
    const unsigned long long t0 = pl->h_stamps[0], tend = pl->h_stamps[1];
    unsigned long long tbins = t0;
    for (int q = 0; q < pl->E; ++q)
      if (pl->evs[pl->order[q]]->ncal == 0) tbins = std::max(tbins, pl->h_stamps[2 + q]);
    // an event's results exist once its last item is done and the final epilogue launch has run
    const double epi_us = tend > tbins ? (double)(tend - tbins) * 1e3 / pl->clock_khz : 0.0;
    for (int q = 0; q < pl->E; ++q) {
      const int e = pl->order[q];
      const unsigned long long te = pl->h_stamps[2 + q];
      const double extra = pl->evs[e]->ncal > 0 ? 0.0 : epi_us;   // calibrated: stamped after its epilogue
      event_latency_us[e] = pl->B[e] == 0 ? 0.0 : (double)(te - t0) * 1e3 / pl->clock_khz + extra;
    }
  }
  return GWL_OK;
}

gwl_status gwl_plan_destroy(gwl_plan pl) {
  plan_free(pl);
  return GWL_OK;
}

}  // extern "C"
