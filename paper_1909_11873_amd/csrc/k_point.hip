// Per-point kernels: set-up (phase coefficients, time shifts, projection factors) before the
// bin loop, and the float64 epilogue after it (the log-likelihood ratio of Eq. 2 and, for the
// adjoint, its gradient with respect to all 11 parameters).
#include <hip/hip_runtime.h>

#include "gwl_common.h"
#include "gwl_device.h"
#include "gwl_epilogue.h"
#include "gwl_launch.h"

namespace gwl {

constexpr int PT_BLOCK = 128;

template <int ND>
__global__ __launch_bounds__(PT_BLOCK) void k_setup(EventGeom g, const double* __restrict__ theta, int64_t B,
                                                    int64_t Bp, double* __restrict__ coef) {
  const int64_t p = (int64_t)blockIdx.x * PT_BLOCK + threadIdx.x;
  if (p >= Bp) return;
  double th[NPARAM];
  const int64_t pc = p < B ? p : B - 1;  // padding lanes repeat the last point
#pragma unroll
  for (int i = 0; i < NPARAM; ++i) th[i] = theta[pc * NPARAM + i];
  PointModel<double> pm;
  point_model<double, ND>(th, g, pm);
  const double nan = __builtin_nan("");
  double rows[NCOEF];
#pragma unroll
  for (int j = 0; j < NCOEF; ++j) rows[j] = 0.0;
#pragma unroll
  for (int m = 0; m < NBASIS; ++m) rows[CO_A + m] = pm.a[m];
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    rows[CO_T + d] = pm.tdet[d];
    rows[CO_QR + d] = pm.qr[d];
    rows[CO_QI + d] = pm.qi[d];
  }
  rows[CO_C0] = pm.c0;
  rows[CO_AMP] = pm.amp;
#pragma unroll
  for (int j = 0; j < NCOEF; ++j) coef[j * Bp + p] = pm.valid ? rows[j] : nan;
}

hipError_t launch_setup(int nd, const EventGeom& g, const double* theta, int64_t B, int64_t Bp, double* coef,
                        hipStream_t s) {
  dim3 grid((unsigned)((Bp + PT_BLOCK - 1) / PT_BLOCK));
  switch (nd) {
    case 1: hipLaunchKernelGGL(k_setup<1>, grid, dim3(PT_BLOCK), 0, s, g, theta, B, Bp, coef); break;
    case 2: hipLaunchKernelGGL(k_setup<2>, grid, dim3(PT_BLOCK), 0, s, g, theta, B, Bp, coef); break;
    case 3: hipLaunchKernelGGL(k_setup<3>, grid, dim3(PT_BLOCK), 0, s, g, theta, B, Bp, coef); break;
    case 4: hipLaunchKernelGGL(k_setup<4>, grid, dim3(PT_BLOCK), 0, s, g, theta, B, Bp, coef); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int ND>
__global__ __launch_bounds__(PT_BLOCK) void k_epilogue(EventGeom g, const EventConst* __restrict__ ec,
                                                       const double* __restrict__ theta, int64_t B, int64_t Bp,
                                                       int nchunk, bool scaled, const double* __restrict__ part,
                                                       double* __restrict__ logl) {
  const int64_t p = (int64_t)blockIdx.x * PT_BLOCK + threadIdx.x;
  if (p >= B) return;
  constexpr int NZ = nz_of(ND, false);
  const EventConst e = *ec;
  double acc[NZ];
  gather<NZ>(part, nchunk, Bp, p, acc);
  if (scaled) apply_gain<NZ>(e, acc);
  double th[NPARAM];
#pragma unroll
  for (int i = 0; i < NPARAM; ++i) th[i] = theta[p * NPARAM + i];
  bool valid;
  const double v = epilogue_value<ND, NZ>(acc, th, g, e, scaled ? e.uref : 1.0, valid);
  logl[p] = valid ? v : __builtin_nan("");
}

template <int ND>
__global__ __launch_bounds__(PT_BLOCK) void k_epilogue_grad(EventGeom g, const EventConst* __restrict__ ec,
                                                            const double* __restrict__ theta, int64_t B, int64_t Bp,
                                                            int nchunk, bool scaled, const double* __restrict__ part,
                                                            double* __restrict__ logl, double* __restrict__ grad) {
  const int64_t p = (int64_t)blockIdx.x * PT_BLOCK + threadIdx.x;
  if (p >= B) return;
  constexpr int NZ = nz_of(ND, true);
  const EventConst e = *ec;
  double acc[NZ];
  gather<NZ>(part, nchunk, Bp, p, acc);
  if (scaled) apply_gain<NZ>(e, acc);
  double th[NPARAM], gout[NPARAM];
#pragma unroll
  for (int i = 0; i < NPARAM; ++i) th[i] = theta[p * NPARAM + i];
  bool valid;
  const double v = epilogue_gradient<ND>(acc, th, g, e, scaled ? e.uref : 1.0, valid, gout);
  const double nan = __builtin_nan("");
  logl[p] = valid ? v : nan;
#pragma unroll
  for (int j = 0; j < NPARAM; ++j) grad[p * NPARAM + j] = valid ? gout[j] : nan;
}

hipError_t launch_epilogue(int nd, bool grad, bool scaled, const EventGeom& g, const EventConst* ec, const double* theta,
                           int64_t B, int64_t Bp, int nchunk, const double* part, double* logl, double* gradout,
                           hipStream_t s) {
  dim3 grid((unsigned)((B + PT_BLOCK - 1) / PT_BLOCK));
#define GWL_EPI(N)                                                                                                  \
  case N:                                                                                                           \
    if (grad)                                                                                                       \
      hipLaunchKernelGGL(k_epilogue_grad<N>, grid, dim3(PT_BLOCK), 0, s, g, ec, theta, B, Bp, nchunk, scaled, part, \
                         logl, gradout);                                                                            \
    else                                                                                                            \
      hipLaunchKernelGGL(k_epilogue<N>, grid, dim3(PT_BLOCK), 0, s, g, ec, theta, B, Bp, nchunk, scaled, part, \
                         logl);                                                                                     \
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
