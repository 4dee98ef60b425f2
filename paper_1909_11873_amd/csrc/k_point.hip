// Per-point kernels: set-up (phase coefficients, time shifts, projection factors) before the
// bin loop, and the float64 epilogue after it (the log-likelihood ratio of Eq. 2 and, for the
// adjoint, its gradient with respect to all 11 parameters).
#include <hip/hip_runtime.h>

#include "gwl_common.h"
#include "gwl_device.h"
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

// Sum the per-chunk partials of one point in chunk order (deterministic).
template <int NZ>
__device__ inline void gather(const double* __restrict__ part, int nchunk, int64_t Bp, int64_t p, double (&acc)[NZ]) {
#pragma unroll
  for (int z = 0; z < NZ; ++z) acc[z] = 0.0;
  for (int c = 0; c < nchunk; ++c) {
#pragma unroll
    for (int z = 0; z < NZ; ++z) acc[z] += part[((int64_t)c * NZ + z) * Bp + p];
  }
}

// Divide the measured mean gain of the float32 hardware phasor out of every complex sum.
template <int NZ>
__device__ inline void apply_gain(const EventConst* __restrict__ ec, double (&acc)[NZ]) {
  const double gr = ec->gain_r, gi = ec->gain_i;
#pragma unroll
  for (int z = 0; z < NZ; z += 2) {
    const double re = acc[z], im = acc[z + 1];
    acc[z] = re * gr - im * gi;
    acc[z + 1] = re * gi + im * gr;
  }
}

// logL = sum_det [ uref Re(A E Q_det Z_det) - 1/2 A^2 |Q_det|^2 K_det ],  E = exp(-2 pi i c0).
template <int ND>
__global__ __launch_bounds__(PT_BLOCK) void k_epilogue(EventGeom g, const EventConst* __restrict__ ec,
                                                       const double* __restrict__ theta, int64_t B, int64_t Bp,
                                                       int nchunk, bool scaled, const double* __restrict__ part,
                                                       double* __restrict__ logl) {
  const int64_t p = (int64_t)blockIdx.x * PT_BLOCK + threadIdx.x;
  if (p >= B) return;
  constexpr int NZ = nz_of(ND, false);
  double acc[NZ];
  gather<NZ>(part, nchunk, Bp, p, acc);
  if (scaled) apply_gain<NZ>(ec, acc);
  double th[NPARAM];
#pragma unroll
  for (int i = 0; i < NPARAM; ++i) th[i] = theta[p * NPARAM + i];
  PointModel<double> pm;
  point_model<double, ND>(th, g, pm);
  const double uref = scaled ? ec->uref : 1.0;  // float32 tables hold u / uref
  const double c0 = pm.c0 - rint(pm.c0);
  double es, ecs;
  sincos_cycles_f64(c0, es, ecs);
  const double er = ecs, ei = -es;
  double out = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const double xr = pm.amp * (er * pm.qr[d] - ei * pm.qi[d]);
    const double xi = pm.amp * (er * pm.qi[d] + ei * pm.qr[d]);
    const double dh = uref * (xr * acc[2 * d] - xi * acc[2 * d + 1]);
    const double hh = pm.amp * pm.amp * (pm.qr[d] * pm.qr[d] + pm.qi[d] * pm.qi[d]) * ec->K[d];
    out += dh - 0.5 * hh;
  }
  logl[p] = pm.valid ? out : __builtin_nan("");
}

// Gradient epilogue. The kernel accumulated, per point,
//   Z_det  = sum_k u p,  Z1_det = sum_k f u p,  Ybar_m = sum_k g_m(f_k) sum_det Q_det u p
// with p = exp(-2 pi i (psi_k + f_k T_det)). Then
//   dlogL = sum_det [ uref Re(d(A E Q_det) Z_det) - 1/2 d(A^2 |Q|^2) K_det ]
//         + uref Re(-2 pi i A E [ sum_m da_m Ybar_m + sum_det dT_det Q_det Z1_det ]),
// with every d(.) from forward-mode dual numbers through the same point model.
template <int ND>
__global__ __launch_bounds__(PT_BLOCK) void k_epilogue_grad(EventGeom g, const EventConst* __restrict__ ec,
                                                            const double* __restrict__ theta, int64_t B, int64_t Bp,
                                                            int nchunk, bool scaled, const double* __restrict__ part,
                                                            double* __restrict__ logl, double* __restrict__ grad) {
  const int64_t p = (int64_t)blockIdx.x * PT_BLOCK + threadIdx.x;
  if (p >= B) return;
  typedef Dual<NPARAM> D;
  constexpr int NZ = nz_of(ND, true);
  double acc[NZ];
  gather<NZ>(part, nchunk, Bp, p, acc);
  if (scaled) apply_gain<NZ>(ec, acc);
  D th[NPARAM];
#pragma unroll
  for (int i = 0; i < NPARAM; ++i) th[i] = dvar<NPARAM>(theta[p * NPARAM + i], i);
  PointModel<D> pm;
  point_model<D, ND>(th, g, pm);
  const double uref = scaled ? ec->uref : 1.0;  // float32 tables hold u / uref
  D c0 = pm.c0;
  c0.v -= rint(c0.v);
  const D arg = c0 * kTwoPi;
  const D er = xcos(arg), ei = -xsin(arg);
  D tot = dcst<NPARAM>(0.0);
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const D xr = pm.amp * (er * pm.qr[d] - ei * pm.qi[d]);
    const D xi = pm.amp * (er * pm.qi[d] + ei * pm.qr[d]);
    const D dh = (xr * acc[2 * d] - xi * acc[2 * d + 1]) * uref;
    const D hh = pm.amp * pm.amp * (pm.qr[d] * pm.qr[d] + pm.qi[d] * pm.qi[d]) * ec->K[d];
    tot = tot + dh - 0.5 * hh;
  }
  // P = uref A E (values); moment term Re(-2 pi i P S) = 2 pi Im(P S)
  const double pr = uref * pm.amp.v * er.v, pi_ = uref * pm.amp.v * ei.v;
  double gout[NPARAM];
#pragma unroll
  for (int j = 0; j < NPARAM; ++j) {
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int m = 0; m < NBASIS; ++m) {
      sr += pm.a[m].d[j] * acc[4 * ND + 2 * m];
      si += pm.a[m].d[j] * acc[4 * ND + 2 * m + 1];
    }
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const double z1r = acc[2 * ND + 2 * d], z1i = acc[2 * ND + 2 * d + 1];
      const double qr = pm.qr[d].v, qi = pm.qi[d].v;
      const double dt = pm.tdet[d].d[j];
      sr += dt * (qr * z1r - qi * z1i);
      si += dt * (qr * z1i + qi * z1r);
    }
    gout[j] = tot.d[j] + kTwoPi * (pr * si + pi_ * sr);
  }
  const double nan = __builtin_nan("");
  logl[p] = pm.valid ? tot.v : nan;
#pragma unroll
  for (int j = 0; j < NPARAM; ++j) grad[p * NPARAM + j] = pm.valid ? gout[j] : nan;
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
