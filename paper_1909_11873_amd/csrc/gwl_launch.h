// Host-side launch wrappers of the kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include "gwl_common.h"

namespace gwl {

// Shape of one evaluation launch: points in groups of 64 (one wavefront), a workgroup of W
// wavefronts per (point group, chunk group), each wavefront one chunk of `chunk` bins, G
// workgroups per point group (nchunk = W G chunks in all); the items = npg G workgroups are
// dealt either so that the dies take the point groups in turn, each with all G of its
// workgroups (pgmaj), or so that each die takes a contiguous range of chunk groups. `setup`:
// the per-point set-up runs inside the kernel instead of the set-up kernel. `sepepi` (value
// only, G > 1): the G workgroup sums of a point are added and the value formed by a second
// kernel instead of by the last workgroup to finish, which needs no device-scope fences (each
// fence writes back and invalidates the die's L2, which slows every workgroup still in its bin
// loop); with the set-up in the kernel, its first workgroup per point group leaves the rows
// that second kernel reads.
constexpr int MAX_EVAL_WAVES = 16;
struct LoopShape {
  int npg;      // point groups = ceil(B / 64)
  int W;        // wavefronts (chunks) per workgroup
  int G;        // workgroups per point group
  int nchunk;   // W G
  int chunk;    // bins per chunk
  int items;    // workgroups = npg G
  int gper;     // workgroups per die: ceil(npg / NXCD) G (pgmaj), else ceil(items / NXCD)
  int setup;    // 1: set-up inside the evaluation kernel
  int sepepi;   // 1: the value's reduction over the G workgroups and its epilogue in a second kernel
  int pgmaj;    // 1: the dies take the point groups in turn (the set-up rows outweigh the table)
};
LoopShape make_shape(int64_t B, int64_t M, int W, int G, int setup, int sepepi = 0);
size_t eval_lds_doubles(bool mixed, const LoopShape& sh);

// event preparation: per-bin tables, K_det and the float32 scale
hipError_t launch_prep(int nd, const double* data, const double* psd, const double* fgrid, int64_t M, double df,
                       void* tab64, void* tab32, RowGradF32* g32, RowGradF64* g64, double* blockpart, int nblk,
                       EventConst* ec, hipStream_t s);
int prep_blocks(int64_t M);
size_t prep_scratch_doubles(int nd, int64_t M);  // size of `blockpart`

// per-point set-up: theta[B][11] -> coef[NCOEF][Bp]; `scaled` (float32 tables) takes the
// phasor gain from *ec into the adjoint projection rows, ec may be null when it is false
hipError_t launch_setup(int nd, const EventGeom& g, const EventConst* ec, bool scaled, const double* theta, int64_t B,
                        int64_t Bp, double* coef, hipStream_t s);

// evaluation: set-up rows (coef, unless sh.setup), bin loop, reduction over the W chunks of a
// workgroup and, for the value, over its G workgroups (part [G][nz][Bp] and cnt [npg], zero
// between calls, when G > 1) and the float64 epilogue -> logl[B]; for the gradient the
// workgroup sums go to part [G][nz][Bp] for the gradient epilogue
// fgrid [M] and kcum [nd][M + 1] (running sums of the K_det terms) for an event with the ISCO
// cut-off, else both null; rot: a float64 call on a uniform grid may take the detectors after
// the first by rotation (ignored with the cut-off and in mixed precision); live (device, may be
// null): only the first *live points are evaluated and written
hipError_t launch_eval(int nd, bool mixed, bool grad, bool rot, const void* tab, const RowGradF64* gtab, const double* theta,
                       const EventGeom& geo, const EventConst* ec, double* coef, int64_t B, int64_t Bp,
                       int64_t M, const LoopShape& sh, double* part, unsigned int* cnt, double* logl,
                       const double* fgrid, const double* kcum, const int64_t* live, hipStream_t s);

// the value's epilogue after an evaluation launch with sh.sepepi: part [G][nz][Bp] -> logl[B],
// the G sums added in workgroup order (as the last-arriving workgroup adds them), then the value
// from the set-up rows coef; fgrid, kcum (both or neither) for the ISCO cut-off; live as in
// launch_eval
hipError_t launch_value_epilogue(int nd, bool mixed, const EventConst* ec, const double* theta, const double* coef,
                                 int64_t B, int64_t Bp, int G, const double* part, double* logl, const double* fgrid,
                                 const double* kcum, int64_t M, const int64_t* live, hipStream_t s);

// epilogue: partial sums [nchunk][nz][Bp] -> logL[B] (and grad[B][11]); the value alone reads the
// set-up rows `coef`, the gradient evaluates the point model from theta
// `scaled`: the partial sums came from the float32 tables, which hold u / uref
hipError_t launch_epilogue(int nd, bool grad, bool scaled, const EventGeom& g, const EventConst* ec,
                           const double* theta, const double* coef, int64_t B, int64_t Bp, int nchunk,
                           const double* part, double* logl, double* gradout, hipStream_t s,
                           const double* fgrid = nullptr, const double* kcum = nullptr, int64_t M = 0);

// float32 rows from float64 rows: tab32 = (basis, u / ec->uref)
hipError_t launch_prep_mixed(int nd, const void* tab64, int64_t M, const EventConst* ec, void* tab32, hipStream_t s);

// relative binning: edge rows from the fine rows (fine64 etc.), the edge indices eidx[nedge] and
// the fiducial in ec->fa, ec->fT; w is scratch of rb_scratch_doubles(nd, nedge); sets ec->uref
size_t rb_scratch_doubles(int nd, int nedge);
hipError_t launch_rb(int nd, const void* fine64, const RowGradF32* fine32g, const RowGradF64* fine64g,
                     const int64_t* eidx, int nedge, double* w, EventConst* ec, void* tab64, void* tab32,
                     RowGradF32* g32, RowGradF64* g64, hipStream_t s);

// calibrated model: set-up, bin loop and epilogue for theta[B][P], P = 11 + 2 nnode nd;
// kcal per detector K1 [nnode], K2 [nnode][nnode]; calc is scratch [2 nnode nd][Bp]
hipError_t launch_cal(int nd, bool mixed, bool grad, const EventGeom& g, const EventConst* ec, const double* kcal,
                      const void* tab, const void* gtab, const void* calw, const void* calt, const double* calB,
                      const double* theta, int P, int64_t B, int64_t Bp, const CalShape& sh, double* coef,
                      double* calc, double* part, double* logl, double* gradout, hipStream_t s);

// model strain on a grid: out[B][nd][M][2]
hipError_t launch_waveform(int nd, const EventGeom& g, const double* coef, int64_t B, int64_t Bp,
                           const double* fgrid, int64_t M, double* out, hipStream_t s);

}  // namespace gwl
