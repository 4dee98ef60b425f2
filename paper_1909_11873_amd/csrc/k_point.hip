// Per-point kernels: set-up (phase coefficients, time shifts, projection factors) before the
// evaluation kernel, and the adjoint's float64 epilogue after it (the log-likelihood ratio of
// Eq. 2 and its gradient with respect to all 11 parameters; the value alone is finished inside
// the evaluation kernel).
#include <hip/hip_runtime.h>

#include "gwl_bins.h"
#include "gwl_common.h"
#include "gwl_device.h"
#include "gwl_epilogue.h"
#include "gwl_launch.h"
#include "gwl_setup.h"

namespace gwl {

// Set-up: one workgroup of two wavefronts per 64 points. The intrinsic half of the point model
// (phase coefficients, constant phase, amplitude) runs on one wavefront and the extrinsic half
// (sky, orientation, per-detector delays and projection factors) on the other, at once, into
// LDS rows; each wavefront then writes half of the rows, with the phase-range check and the
// adjoint factors taken from the LDS rows as setup_rows takes them (the same rows, bit for bit,
// as one thread running setup_rows; NaN rows for a point outside the model's domain or range).
constexpr int SETUP_WAVES = 2;

template <int ND>
__global__ __launch_bounds__(SETUP_WAVES * WAVE) void k_setup(EventGeom g, const EventConst* __restrict__ ec,
                                                              bool scaled, const double* __restrict__ theta,
                                                              int64_t B, int64_t Bp, double* __restrict__ coef) {
  __shared__ double rows_s[NCOEF * WAVE];
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
  const int lane = (int)(threadIdx.x % WAVE);
  const int64_t p = (int64_t)blockIdx.x * WAVE + lane;   // < Bp: Bp is a multiple of 64
  const int64_t pc = p < B ? p : B - 1;                  // padding lanes repeat the last point
  setup_halves<ND>(w, lane, theta + pc * NPARAM, g, ec, rows_s);
  __syncthreads();
  setup_rows_write<ND>(w, lane, rows_s, ec, scaled, true, coef, Bp, p);
}

hipError_t launch_setup(int nd, const EventGeom& g, const EventConst* ec, bool scaled, const double* theta, int64_t B,
                        int64_t Bp, double* coef, hipStream_t s) {
  if (scaled && !ec) return hipErrorInvalidValue;
  if (Bp % WAVE != 0 || B < 1 || B > Bp) return hipErrorInvalidValue;
  dim3 grid((unsigned)(Bp / WAVE));
#define GWL_SETUP(N) \
  case N: hipLaunchKernelGGL(k_setup<N>, grid, dim3(SETUP_WAVES * WAVE), 0, s, g, ec, scaled, theta, B, Bp, coef); break;
  switch (nd) {
    GWL_SETUP(1)
    GWL_SETUP(2)
    GWL_SETUP(3)
    GWL_SETUP(4)
    default: return hipErrorInvalidValue;
  }
#undef GWL_SETUP
  return hipGetLastError();
}

// With the ISCO cut-off (fgrid and kcum given), <h|h> takes the kept bins' share of K_det; the
// cut moves with the masses in steps, so it adds nothing to the derivative.
//
// One workgroup per 64 points, EPG_WAVES wavefronts (the epilogue needs about 256 registers, so a
// SIMD holds one such wavefront and a CU four): the wavefronts first add the points' partial sums
// over the chunks (in chunk order, each wavefront its share of the sums) into LDS, then each runs
// the dual-number passes of the parameters j = w, w + EPG_WAVES, ...: three passes of latency
// instead of eleven, and four times the SIMDs of one thread per point.
constexpr int EPG_WAVES = 4;
template <int ND>
__global__ __launch_bounds__(EPG_WAVES * WAVE) void k_epilogue_grad(EventGeom g, const EventConst* __restrict__ ec,
                                                                    const double* __restrict__ theta, int64_t B,
                                                                    int64_t Bp, int nchunk, bool scaled,
                                                                    const double* __restrict__ part,
                                                                    double* __restrict__ logl,
                                                                    double* __restrict__ grad,
                                                                    const double* __restrict__ fgrid,
                                                                    const double* __restrict__ kcum, int64_t M) {
  constexpr int NZ = nz_of(ND, true);
  __shared__ double acc_s[NZ][WAVE];
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
  const int lane = (int)(threadIdx.x % WAVE);
  const int64_t p = (int64_t)blockIdx.x * WAVE + lane;   // p < Bp: the partial sums have Bp rows
  for (int z = w; z < NZ; z += EPG_WAVES) {
    double a = 0.0;
#pragma unroll 8
    for (int c = 0; c < nchunk; ++c) a += part[((int64_t)c * NZ + z) * Bp + p];
    acc_s[z][lane] = a;
  }
  __syncthreads();
  if (p >= B) return;
  EventConst e = *ec;
  double acc[NZ];
#pragma unroll
  for (int z = 0; z < NZ; ++z) acc[z] = acc_s[z][lane];
  if (scaled) apply_gain<ND>(e, acc);
  double th[NPARAM];
#pragma unroll
  for (int i = 0; i < NPARAM; ++i) th[i] = theta[p * NPARAM + i];
  if (fgrid) {
    const int kc = isco_bins(th[0], th[1], fgrid, M, e);
#pragma unroll
    for (int d = 0; d < ND; ++d) e.K[d] = kcum[(int64_t)d * (M + 1) + kc];
  }
  const double nan = __builtin_nan("");
  const double uref = scaled ? e.uref : 1.0;
#pragma unroll 1
  for (int j = w; j < NPARAM; j += EPG_WAVES) {
    bool valid;
    double value;
    const double gj = epilogue_gradient_pass<ND>(acc, th, g, e, uref, j, valid, value);
    grad[p * NPARAM + j] = valid ? gj : nan;
    if (j == 0) logl[p] = valid ? value : nan;
  }
}

hipError_t launch_epilogue(int nd, bool grad, bool scaled, const EventGeom& g, const EventConst* ec, const double* theta,
                           const double*, int64_t B, int64_t Bp, int nchunk, const double* part, double* logl,
                           double* gradout, hipStream_t s, const double* fgrid, const double* kcum, int64_t M) {
  if (!grad) return hipErrorInvalidValue;  // the value's epilogue runs in the evaluation kernel
  dim3 grid((unsigned)((B + WAVE - 1) / WAVE));
#define GWL_EPI(N)                                                                                                  \
  case N:                                                                                                           \
    hipLaunchKernelGGL(k_epilogue_grad<N>, grid, dim3(EPG_WAVES * WAVE), 0, s, g, ec, theta, B, Bp, nchunk, scaled, \
                       part, logl, gradout, fgrid, kcum, M);                                                        \
    break;
  switch (nd) {
    GWL_EPI(1)
    GWL_EPI(2)
    GWL_EPI(3)
    GWL_EPI(4)
    default: return hipErrorInvalidValue;
  }
#undef GWL_EPI
  return hipGetLastError();
}

}  // namespace gwl
