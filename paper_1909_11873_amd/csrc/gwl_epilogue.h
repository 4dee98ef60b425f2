// Float64 per-point work shared by the single-event and multi-event kernels: the set-up rows
// before the bin loop, and the epilogue after it (the log-likelihood ratio from the
// accumulated sums and, for the adjoint, its gradient with respect to all 11 parameters).
#pragma once

#include <hip/hip_runtime.h>

#include "gwl_common.h"
#include "gwl_device.h"

namespace gwl {

// E G: the constant phase factor E = exp(-2 pi i c0) (c0 in cycles) times the gain G. This and
// adjoint_factor spell out their fused multiply-adds, so that every kernel forming c_det rounds
// the same way (the in-kernel set-up and the set-up kernel give bitwise equal gradients).
__device__ inline void phase_gain(double c0raw, double gr, double gi, double& egr, double& egi) {
  const double c0 = c0raw - rint(c0raw);
  double es, ecs;
  sincos_cycles_f64(c0, es, ecs);
  egr = fma(ecs, gr, es * gi);
  egi = fma(ecs, gi, -(es * gr));
}
// c_det = (E G) Q_det
__device__ inline void adjoint_factor(double egr, double egi, double qr, double qi, double& cr, double& ci) {
  cr = fma(egr, qr, -(egi * qi));
  ci = fma(egr, qi, egi * qr);
}

// Whether the phase sum_m a_m g_m(f) + f T_det stays below PHASE_LIMIT cycles on the event's
// grid (a and T after the fiducial's offsets; always true without an event).
template <int ND>
__device__ inline bool rows_in_range(const double* a, const double* T, const EventConst* ec) {
  if (!ec) return true;
  double bound = 0.0, tmax = 0.0;
#pragma unroll
  for (int m = 0; m < NBASIS; ++m) bound = fma(fabs(a[m]), ec->gmax[m], bound);
#pragma unroll
  for (int d = 0; d < ND; ++d) tmax = fmax(tmax, fabs(T[d]));
  return fma(tmax, ec->fmax, bound) < PHASE_LIMIT;
}

// Set-up rows (layout CO_*) of one point; false if the point is outside the model's domain or,
// given the event (ec), its phase could exceed PHASE_LIMIT cycles somewhere on the grid.
// With `scaled` (float32 tables) the event's (gain_r, gain_i) undoes the mean gain of the bin
// loop's phasor (1 for float64 tables). It enters the adjoint projection factors
// c_det = E G Q_det, E = exp(-2 pi i c0), through which the adjoint bin loop keeps only the one
// real part of each moment that the gradient uses. A relative-binning event's fiducial phase
// coefficients and shifts are subtracted from the bin loop's rows (ec may be null: no offsets).
template <int ND>
__device__ inline bool setup_rows(const double (&th)[NPARAM], const EventGeom& g, const EventConst* ec, bool scaled,
                                  double (&rows)[NCOEF]) {
  const double gr = (scaled && ec) ? ec->gain_r : 1.0, gi = (scaled && ec) ? ec->gain_i : 0.0;
  PointModel<double> pm;
  point_model<double, ND>(th, g, pm);
#pragma unroll
  for (int j = 0; j < NCOEF; ++j) rows[j] = 0.0;
#pragma unroll
  for (int m = 0; m < NBASIS; ++m) rows[CO_A + m] = pm.a[m] - (ec ? ec->fa[m] : 0.0);
  double egr, egi;
  phase_gain(pm.c0, gr, gi, egr, egi);
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    rows[CO_T + d] = pm.tdet[d] - (ec ? ec->fT[d] : 0.0);
    rows[CO_QR + d] = pm.qr[d];
    rows[CO_QI + d] = pm.qi[d];
    adjoint_factor(egr, egi, pm.qr[d], pm.qi[d], rows[CO_CR + d], rows[CO_CI + d]);
  }
  rows[CO_C0] = pm.c0;
  rows[CO_AMP] = pm.amp;
  const bool in_range = rows_in_range<ND>(&rows[CO_A], &rows[CO_T], ec);
  return pm.valid && in_range;
}

// The in-kernel set-up in two halves, each writing its rows of one point into the LDS rows
// [NCOEF][WAVE] (lane = point), so that two wavefronts can run them at once. The intrinsic half
// writes CO_A (less the fiducial's), CO_C0 and CO_AMP, NaN for a point outside the model's
// domain; the extrinsic half writes CO_T (less the fiducial's), CO_QR and CO_QI. The phase
// range check and the adjoint factors c_det then come from these rows (rows_in_range,
// phase_gain), with the same arithmetic as setup_rows.
__device__ inline void setup_lds_intrinsic(const double (&th)[NPARAM], const EventConst* ec, double* rows_s, int lane) {
  PointModel<double> pm;
  point_intrinsic<double>(th, pm);
  const double nan = __builtin_nan("");
#pragma unroll
  for (int m = 0; m < NBASIS; ++m) rows_s[(CO_A + m) * WAVE + lane] = pm.valid ? pm.a[m] - (ec ? ec->fa[m] : 0.0) : nan;
  rows_s[CO_C0 * WAVE + lane] = pm.valid ? pm.c0 : nan;
  rows_s[CO_AMP * WAVE + lane] = pm.valid ? pm.amp : nan;
}
template <int ND>
__device__ inline void setup_lds_extrinsic(const double (&th)[NPARAM], const EventGeom& g, const EventConst* ec,
                                           double* rows_s, int lane) {
  PointModel<double> pm;
  point_extrinsic<double, ND>(th, g, pm);
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    rows_s[(CO_T + d) * WAVE + lane] = pm.tdet[d] - (ec ? ec->fT[d] : 0.0);
    rows_s[(CO_QR + d) * WAVE + lane] = pm.qr[d];
    rows_s[(CO_QI + d) * WAVE + lane] = pm.qi[d];
  }
}

// Divide the measured mean gain of the float32 hardware phasor out of the complex sums Z_det
// (the leading 2 ND entries; the adjoint moments carry the gain in c_det). Explicit fused
// multiply-adds: every kernel that applies it rounds alike.
template <int ND, int NZ>
__device__ inline void apply_gain(const EventConst& ec, double (&acc)[NZ]) {
  const double gr = ec.gain_r, gi = ec.gain_i;
#pragma unroll
  for (int z = 0; z < 2 * ND; z += 2) {
    const double re = acc[z], im = acc[z + 1];
    acc[z] = fma(re, gr, -(im * gi));
    acc[z + 1] = fma(re, gi, im * gr);
  }
}

// Sum the per-chunk partials of one point in chunk order (deterministic). The chunk loop is
// unrolled so that several chunks' loads are in flight before their adds, which still run in
// chunk order; with one thread per point this loop is latency-bound otherwise.
template <int NZ>
__device__ inline void gather(const double* __restrict__ part, int nchunk, int64_t Bp, int64_t p, double (&acc)[NZ]) {
#pragma unroll
  for (int z = 0; z < NZ; ++z) acc[z] = 0.0;
#pragma unroll 8
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

// The same value from the point's set-up rows (A, Q_det and c0 as the point model gave them; a
// point outside the model's domain has NaN rows and gets NaN), so the forward epilogue does not
// evaluate the point model a second time.
template <int ND, int NZ>
__device__ inline double epilogue_value_rows(const double (&acc)[NZ], const double* __restrict__ coef, int64_t Bp,
                                             int64_t p, const EventConst& ec, double uref) {
  const double amp = coef[CO_AMP * Bp + p];
  const double c0f = coef[CO_C0 * Bp + p];
  const double c0 = c0f - rint(c0f);
  double es, ecs;
  sincos_cycles_f64(c0, es, ecs);
  const double er = ecs, ei = -es;
  double out = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const double qr = coef[(CO_QR + d) * Bp + p], qi = coef[(CO_QI + d) * Bp + p];
    const double xr = amp * (er * qr - ei * qi);
    const double xi = amp * (er * qi + ei * qr);
    const double dh = uref * (xr * acc[2 * d] - xi * acc[2 * d + 1]);
    const double hh = amp * amp * (qr * qr + qi * qi) * ec.K[d];
    out += dh - 0.5 * hh;
  }
  return out;
}

// Gradient. With w_det = u p, p = exp(-2 pi i (psi_k + f_k T_det)) and y_det = Im(c_det w_det),
// the bin loop accumulated per point
//   Z_det = sum_k w_det,  Z1_det = sum_k f_k y_det,  Y_m = sum_k g_m(f_k) sum_det y_det.
// The phase coefficients a_m and the shifts T_det enter logL only through p, so
//   dlogL = sum_det [ uref Re(d(A E Q_det) Z_det) - 1/2 d(A^2 |Q|^2) K_det ]
//         + 2 pi uref A [ sum_m da_m Y_m + sum_det dT_det Z1_det ]
// (the second line is Re(-2 pi i uref A E G Q_det sum_k (da.g + f_k dT_det) w_det) written
// with c_det = E G Q_det).
// Every d(.) comes from one-direction dual numbers pushed through the same point model, one
// parameter at a time (11 passes; this keeps the register footprint of the epilogue small).
// One pass: the derivative with respect to parameter j; `value` and `valid` are the same in every
// pass (the primal part does not depend on the direction).
template <int ND>
__device__ inline double epilogue_gradient_pass(const double (&acc)[nz_of(ND, true)], const double (&th)[NPARAM],
                                                const EventGeom& g, const EventConst& ec, double uref, int j,
                                                bool& valid, double& value) {
  typedef Dual<1> D;
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
  double sm = 0.0;
#pragma unroll
  for (int m = 0; m < NBASIS; ++m) sm += pm.a[m].d[0] * acc[3 * ND + m];
#pragma unroll
  for (int d = 0; d < ND; ++d) sm += pm.tdet[d].d[0] * acc[2 * ND + d];
  value = tot.v;
  valid = pm.valid;
  return tot.d[0] + kTwoPi * uref * pm.amp.v * sm;
}

template <int ND>
__device__ inline double epilogue_gradient(const double (&acc)[nz_of(ND, true)], const double (&th)[NPARAM],
                                           const EventGeom& g, const EventConst& ec, double uref, bool& valid,
                                           double (&gout)[NPARAM]) {
  double value = 0.0;
#pragma unroll 1
  for (int j = 0; j < NPARAM; ++j) gout[j] = epilogue_gradient_pass<ND>(acc, th, g, ec, uref, j, valid, value);
  return value;
}

}  // namespace gwl
