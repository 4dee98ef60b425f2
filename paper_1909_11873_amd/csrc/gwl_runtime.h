// Internal host-side declarations shared by the runtime's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "../../include/gwlike.h"
#include "gwl_common.h"
#include "gwl_launch.h"

// Device workspace of an event on one stream: grown (never shrunk) outside graph capture, reused
// by every later call on that stream; calls on one stream are ordered, so they can share it.
struct gwl_workspace {
  hipStream_t stream = nullptr;
  void* ptr = nullptr;
  size_t bytes = 0;
  unsigned int* cnt = nullptr;       // completion counters of the evaluation kernel: zero between calls
  size_t ncnt = 0;
};

struct gwl_event_s {
  std::mutex ws_mu;                  // guards ws
  std::vector<gwl_workspace> ws;     // one per stream that has called on this event
  int device = 0;
  int ndet = 0;
  int64_t M = 0;                     // rows the bin loop walks (bins, or edges for relative binning)
  int64_t M_full = 0;                // bins of the grid (relative binning), else 0
  std::vector<int64_t> rb_idx;       // the relative-binning edges' bins
  // calibration model (ncal nodes per detector, 0 = none)
  int ncal = 0;
  gwl::RowCal32* cal32 = nullptr;    // [M] window weights
  gwl::RowCal64* cal64 = nullptr;
  float* calt32 = nullptr;           // [M] position t in [0, 1] of each bin in its node interval
  double* calt64 = nullptr;
  double* calB = nullptr;            // per interval: the window's weights as cubics in t [n-1][4][4]
  double* kcal = nullptr;            // per detector: K1 [ncal], K2 [ncal][ncal]
  int cal_j0[gwl::MAXNODE] = {};
  int64_t cal_kb[gwl::MAXNODE] = {};
  double df = 0.0;
  double gmst = 0.0;
  gwl_detector dets[GWL_MAX_DET] = {};
  gwl::EventGeom geom = {};
  void* tab64 = nullptr;             // RowF64<ndet>[M]
  void* tab32 = nullptr;             // RowMixed<ndet>[M]
  gwl::RowGradF32* g32 = nullptr;    // [M]
  gwl::RowGradF64* g64 = nullptr;    // [M]
  double* fgrid = nullptr;           // [M] grid frequencies (ISCO cut-off only)
  double* kcum = nullptr;            // [ndet][M + 1] running sums of the K_det terms (ISCO cut-off only)
  gwl::EventConst* ec = nullptr;     // device copy
  gwl::EventConst ech = {};          // host copy
};

namespace gwl {

constexpr int64_t kMaxBatch = (int64_t)1 << 30;

// Whether a call in precision p runs the mixed-precision bin loop on this event. A
// relative-binning event always runs the float64 loop: its few hundred edge terms are each the
// sum of hundreds of bins, and float32 roundings on them (the stored V_e, the hardware phasor,
// the products) do not average down below the 1e-3 bound on loud events.
inline bool use_mixed(const gwl_event_s* ev, gwl_precision p) { return p == GWL_MIXED && ev->M_full == 0; }

gwl_status fail(gwl_status st, const char* fmt, ...);
gwl_status hip_fail(hipError_t e, const char* what);
void clear_error();
gwl_status check_device(int dev);
gwl_status make_geom(const gwl_detector* dets, int ndet, double gmst, EventGeom& g);
size_t row64_bytes(int nd);
size_t row32_bytes(int nd);
// workspace of an evaluation launch: set-up rows [NCOEF][Bp] unless the kernel does the set-up,
// then workgroup partial sums [G][nz][Bp] for the gradient or when G > 1 (doubles), and npg
// completion counters for the value when G > 1
size_t workspace_bytes(int64_t Bp, const LoopShape& sh, int nd, bool grad);
size_t workspace_counters(const LoopShape& sh, bool grad);

// launch shape of a call (autotuner cache, else a heuristic)
LoopShape choose_shape(const gwl_event_s* ev, int64_t B, bool mixed, bool grad);
LoopShape heuristic_shape(int64_t B, int64_t M, bool mixed, bool grad);
// number of bin chunks of the calibrated loop's adjoint (a heuristic)
int heuristic_nchunk(int64_t B, int64_t M);

// multi-event plans: build with an explicit chunk length (0 = heuristic) and queue order; the
// tuner's cached choice for a workload (chunk 0 and ascending order when none is cached)
gwl_status build_plan(const gwl_event* evs, int E, const int64_t* B_e, gwl_precision prec, int with_grad,
                      int chunk_req, bool descending, gwl_plan* out);
void choose_multi_shape(const gwl_event* evs, int E, const int64_t* B_e, bool mixed, bool grad, int* chunk,
                        bool* descending);
// fill theta[B][P] with valid parameter points (timing inputs; P >= 11, zeros past column 11)
hipError_t fill_theta(double* theta, int64_t B, hipStream_t s, int P = NPARAM);

// live (device, may be null): evaluate only the first *live of the B points
gwl_status run_logl(gwl_event ev, const double* theta, int64_t B, bool mixed, bool grad, const LoopShape& sh,
                    double* logl, double* gradout, hipStream_t s, const int64_t* live = nullptr);
// a call on a calibrated event (its own set-up, bin loop and epilogue kernels) in the workspace
// ws of ws_bytes bytes (at least call_workspace_bytes), which the caller owns
gwl_status run_calibrated(gwl_event ev, const double* theta, int64_t B, bool mixed, bool grad, double* logl,
                          double* gradout, hipStream_t s, void* ws, size_t ws_bytes);

// The event's workspace on stream s, grown to at least `bytes` if needed (zero-filled when it
// grows). Growing is refused while s is capturing a graph (GWL_E_INVALID): the caller reserves it
// beforehand with gwl_event_reserve or an ordinary call of the same size.
gwl_status event_workspace(gwl_event ev, hipStream_t s, size_t bytes, size_t ncnt, void** out,
                           unsigned int** cnt = nullptr);
// Workspace bytes a single-event call of this kind needs.
size_t call_workspace_bytes(const gwl_event_s* ev, int64_t B, bool mixed, bool grad);
hipError_t enqueue_logl(gwl_event ev, const double* theta, int64_t B, bool mixed, bool grad, const LoopShape& sh,
                        double* ws, unsigned int* cnt, double* logl, double* gradout, hipStream_t s,
                        const int64_t* live = nullptr);

}  // namespace gwl
