// Set-up kernels' shared part (section 2, Eq. 2's per-point model): the point model's two halves
// on two wavefronts of a workgroup of 64 points, and the set-up rows written from them.
#pragma once
#include <hip/hip_runtime.h>

#include "gwl_common.h"
#include "gwl_device.h"
#include "gwl_epilogue.h"

namespace gwl {

// The set-up of 64 points by two wavefronts of one workgroup: wavefront 0 runs the intrinsic half
// and wavefront 1 the extrinsic half into the LDS rows rows_s [NCOEF][WAVE] (theta rows of P
// columns, the first 11 the signal parameters); after a barrier, setup_rows_write has each
// wavefront write half of the rows [NCOEF][Bp], with the phase-range check and the adjoint
// factors taken from the LDS rows as setup_rows takes them, so the rows equal setup_rows' bit
// for bit; every row is NaN for a point outside the model's domain or range, or with !ok.
template <int ND>
__device__ inline void setup_halves(int w, int lane, const double* __restrict__ theta_row, const EventGeom& g,
                                    const EventConst* ec, double* rows_s) {
  double th[NPARAM];
#pragma unroll
  for (int i = 0; i < NPARAM; ++i) th[i] = theta_row[i];
  if (w == 0) setup_lds_intrinsic(th, ec, rows_s, lane);
  else setup_lds_extrinsic<ND>(th, g, ec, rows_s, lane);
}
template <int ND>
__device__ inline void setup_rows_write(int w, int lane, const double* rows_s, const EventConst* ec, bool scaled,
                                        bool ok, double* __restrict__ coef, int64_t Bp, int64_t p) {
  double a[NBASIS], T[ND];
#pragma unroll
  for (int m = 0; m < NBASIS; ++m) a[m] = rows_s[(CO_A + m) * WAVE + lane];
#pragma unroll
  for (int d = 0; d < ND; ++d) T[d] = rows_s[(CO_T + d) * WAVE + lane];
  // the intrinsic half leaves NaN rows for a point outside the model's domain
  const bool valid = ok && !isnan(a[0]) && rows_in_range<ND>(a, T, ec);
  const double nan = __builtin_nan("");
  auto put = [&](int j, double v) { coef[j * Bp + p] = valid ? v : nan; };
  if (w == 0) {
#pragma unroll
    for (int m = 0; m < NBASIS; ++m) put(CO_A + m, a[m]);
#pragma unroll
    for (int d = 0; d < MAXDET; ++d) put(CO_T + d, d < ND ? T[d] : 0.0);
    put(CO_C0, rows_s[CO_C0 * WAVE + lane]);
    put(CO_AMP, rows_s[CO_AMP * WAVE + lane]);
  } else {
    const double gr = (scaled && ec) ? ec->gain_r : 1.0, gi = (scaled && ec) ? ec->gain_i : 0.0;
    double egr, egi;
    phase_gain(rows_s[CO_C0 * WAVE + lane], gr, gi, egr, egi);
#pragma unroll
    for (int d = 0; d < MAXDET; ++d) {
      double qr = 0.0, qi = 0.0, cr = 0.0, ci = 0.0;
      if (d < ND) {
        qr = rows_s[(CO_QR + d) * WAVE + lane];
        qi = rows_s[(CO_QI + d) * WAVE + lane];
        adjoint_factor(egr, egi, qr, qi, cr, ci);
      }
      put(CO_QR + d, qr);
      put(CO_QI + d, qi);
      put(CO_CR + d, cr);
      put(CO_CI + d, ci);
    }
  }
}

}  // namespace gwl
