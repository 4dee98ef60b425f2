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
__global__ __launch_bounds__(PT_BLOCK) void k_setup(EventGeom g, const EventConst* __restrict__ ec, bool scaled,
                                                    const double* __restrict__ theta, int64_t B, int64_t Bp,
                                                    double* __restrict__ coef) {
  const int64_t p = (int64_t)blockIdx.x * PT_BLOCK + threadIdx.x;
  if (p >= Bp) return;
  double th[NPARAM];
  const int64_t pc = p < B ? p : B - 1;  // padding lanes repeat the last point
#pragma unroll
  for (int i = 0; i < NPARAM; ++i) th[i] = theta[pc * NPARAM + i];
  double rows[NCOEF];
  const bool valid = setup_rows<ND>(th, g, ec, scaled, rows);
  const double nan = __builtin_nan("");
#pragma unroll
  for (int j = 0; j < NCOEF; ++j) coef[j * Bp + p] = valid ? rows[j] : nan;
}

hipError_t launch_setup(int nd, const EventGeom& g, const EventConst* ec, bool scaled, const double* theta, int64_t B,
                        int64_t Bp, double* coef, hipStream_t s) {
  if (scaled && !ec) return hipErrorInvalidValue;
  dim3 grid((unsigned)((Bp + PT_BLOCK - 1) / PT_BLOCK));
#define GWL_SETUP(N) \
  case N: hipLaunchKernelGGL(k_setup<N>, grid, dim3(PT_BLOCK), 0, s, g, ec, scaled, theta, B, Bp, coef); break;
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

// The value epilogue takes EPI_SPLIT lanes per point for the chunk sums: with one thread per
// point a batch of a few thousand points fills a few dozen CUs, each thread walking every chunk.
constexpr int EPI_SPLIT = 4;

template <int ND>
__global__ __launch_bounds__(PT_BLOCK) void k_epilogue(const EventConst* __restrict__ ec,
                                                       const double* __restrict__ coef, int64_t B, int64_t Bp,
                                                       int nchunk, bool scaled, const double* __restrict__ part,
                                                       double* __restrict__ logl) {
  const int64_t p = ((int64_t)blockIdx.x * PT_BLOCK + threadIdx.x) / EPI_SPLIT;
  const int sub = threadIdx.x & (EPI_SPLIT - 1);
  constexpr int NZ = nz_of(ND, false);
  double acc[NZ];
  gather_split<NZ, EPI_SPLIT>(part, nchunk, Bp, p, sub, p < B, acc);
  if (p >= B || sub != 0) return;
  const EventConst e = *ec;
  if (scaled) apply_gain<ND>(e, acc);
  logl[p] = epilogue_value_rows<ND, NZ>(acc, coef, Bp, p, e, scaled ? e.uref : 1.0);
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
  if (scaled) apply_gain<ND>(e, acc);
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
                           const double* coef, int64_t B, int64_t Bp, int nchunk, const double* part, double* logl,
                           double* gradout, hipStream_t s) {
  dim3 grid((unsigned)((B + PT_BLOCK - 1) / PT_BLOCK));
  dim3 grid_split((unsigned)((B * EPI_SPLIT + PT_BLOCK - 1) / PT_BLOCK));
#define GWL_EPI(N)                                                                                                  \
  case N:                                                                                                           \
    if (grad)                                                                                                       \
      hipLaunchKernelGGL(k_epilogue_grad<N>, grid, dim3(PT_BLOCK), 0, s, g, ec, theta, B, Bp, nchunk, scaled, part, \
                         logl, gradout);                                                                            \
    else                                                                                                            \
      hipLaunchKernelGGL(k_epilogue<N>, grid_split, dim3(PT_BLOCK), 0, s, ec, coef, B, Bp, nchunk, scaled, part,    \
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
