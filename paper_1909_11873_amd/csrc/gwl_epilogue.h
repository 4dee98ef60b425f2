// Float64 epilogue of one point, shared by the single-event and multi-event kernels:
// the log-likelihood ratio from the accumulated complex sums and, for the adjoint, its
// gradient with respect to all 11 parameters.
#pragma once

#include <hip/hip_runtime.h>

#include "gwl_common.h"
#include "gwl_device.h"

namespace gwl {

// Divide the measured mean gain of the float32 hardware phasor out of every complex sum.
template <int NZ>
__device__ inline void apply_gain(const EventConst& ec, double (&acc)[NZ]) {
  const double gr = ec.gain_r, gi = ec.gain_i;
#pragma unroll
  for (int z = 0; z < NZ; z += 2) {
    const double re = acc[z], im = acc[z + 1];
    acc[z] = re * gr - im * gi;
    acc[z + 1] = re * gi + im * gr;
  }
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

// logL = sum_det [ uref Re(A E Q_det Z_det) - 1/2 A^2 |Q_det|^2 K_det ],  E = exp(-2 pi i c0).
// `acc` holds Z_det (re, im) first; uref = 1 for float64 tables.
template <int ND, int NZ>
__device__ inline double epilogue_value(const double (&acc)[NZ], const double (&th)[NPARAM], const EventGeom& g,
                                        const EventConst& ec, double uref, bool& valid) {
  PointModel<double> pm;
  point_model<double, ND>(th, g, pm);
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
    const double hh = pm.amp * pm.amp * (pm.qr[d] * pm.qr[d] + pm.qi[d] * pm.qi[d]) * ec.K[d];
    out += dh - 0.5 * hh;
  }
  valid = pm.valid;
  return out;
}

// Gradient. The bin loop accumulated, per point,
//   Z_det  = sum_k u p,  Z1_det = sum_k f u p,  Ybar_m = sum_k g_m(f_k) sum_det Q_det u p
// with p = exp(-2 pi i (psi_k + f_k T_det)). Then
//   dlogL = sum_det [ uref Re(d(A E Q_det) Z_det) - 1/2 d(A^2 |Q|^2) K_det ]
//         + uref Re(-2 pi i A E [ sum_m da_m Ybar_m + sum_det dT_det Q_det Z1_det ]).
// Every d(.) comes from one-direction dual numbers pushed through the same point model, one
// parameter at a time (11 passes; this keeps the register footprint of the epilogue small).
template <int ND>
__device__ inline double epilogue_gradient(const double (&acc)[nz_of(ND, true)], const double (&th)[NPARAM],
                                           const EventGeom& g, const EventConst& ec, double uref, bool& valid,
                                           double (&gout)[NPARAM]) {
  typedef Dual<1> D;
  double value = 0.0;
#pragma unroll 1
  for (int j = 0; j < NPARAM; ++j) {
    D t[NPARAM];
#pragma unroll
    for (int i = 0; i < NPARAM; ++i) {
      t[i].v = th[i];
      t[i].d[0] = (i == j) ? 1.0 : 0.0;
    }
    PointModel<D> pm;
    point_model<D, ND>(t, g, pm);
    D c0 = pm.c0;
    c0.v -= rint(c0.v);
    const D arg = c0 * kTwoPi;
    const D er = xcos(arg), ei = -xsin(arg);
    D tot = dcst<1>(0.0);
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const D xr = pm.amp * (er * pm.qr[d] - ei * pm.qi[d]);
      const D xi = pm.amp * (er * pm.qi[d] + ei * pm.qr[d]);
      const D dh = (xr * acc[2 * d] - xi * acc[2 * d + 1]) * uref;
      const D hh = pm.amp * pm.amp * (pm.qr[d] * pm.qr[d] + pm.qi[d] * pm.qi[d]) * ec.K[d];
      tot = tot + dh - 0.5 * hh;
    }
    // P = uref A E (values); moment term Re(-2 pi i P S) = 2 pi Im(P S)
    const double pr = uref * pm.amp.v * er.v, pi_ = uref * pm.amp.v * ei.v;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int m = 0; m < NBASIS; ++m) {
      sr += pm.a[m].d[0] * acc[4 * ND + 2 * m];
      si += pm.a[m].d[0] * acc[4 * ND + 2 * m + 1];
    }
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const double z1r = acc[2 * ND + 2 * d], z1i = acc[2 * ND + 2 * d + 1];
      const double qr = pm.qr[d].v, qi = pm.qi[d].v;
      const double dt = pm.tdet[d].d[0];
      sr += dt * (qr * z1r - qi * z1i);
      si += dt * (qr * z1i + qi * z1r);
    }
    gout[j] = tot.d[0] + kTwoPi * (pr * si + pi_ * sr);
    value = tot.v;
    valid = pm.valid;
  }
  return value;
}

}  // namespace gwl
