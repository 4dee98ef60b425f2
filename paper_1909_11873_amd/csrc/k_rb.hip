// Relative binning (the variant the paper's section 5 names as the next multiplier): summary
// data of the whitened data against a fiducial waveform h0, on a sparse set of edge
// frequencies, so that the bin loop walks the edges instead of every bin.
//
// In the factored form the kernels use, h_det,k = A Q_det f_k^(-7/6) exp(-2 pi i (psi_k +
// f_k T_det + c0)), and Z_det = sum_k u_k p_k with p_k = exp(-2 pi i (psi_k + f_k T_det)).
// Writing p_k = p0_k rho_k with p0 the fiducial's phasor (its own psi0, T0_det) and replacing
// rho between two adjacent edges by its linear interpolant gives
//   Z_det ~ sum_e V_e rho(f_e),   V_e = sum_k u_k p0_k hat_e(f_k),
// with hat_e the piecewise-linear function that is 1 at edge e and 0 at its neighbours, and
// rho(f_e) = exp(-2 pi i (dpsi(f_e) + f_e dT_det)) the phasor of the phase difference from the
// fiducial. So a relative-binning event is an ordinary event whose rows sit on the edges, whose
// u is V, and whose set-up subtracts the fiducial's coefficients (EventConst::fa, fT). <h|h>
// keeps its exact per-point form A^2 |Q_det|^2 K_det.
#include <hip/hip_runtime.h>

#include "gwl_bins.h"
#include "gwl_common.h"
#include "gwl_device.h"
#include "gwl_launch.h"

namespace gwl {

constexpr int RB_BLOCK = 256;

// One workgroup per span between edges e and e+1: W0 = sum c (1 - t), W1 = sum c t over the
// span's bins with c = u p0 and t = (f - f_e) / (f_{e+1} - f_e). The span covers bins
// [k_e, k_{e+1}), the last span also k_{E-1}. Fixed-order tree reduction (deterministic).
template <int ND>
__global__ __launch_bounds__(RB_BLOCK) void k_rb_spans(const RowF64<ND>* __restrict__ tab64,
                                                       const int64_t* __restrict__ eidx, int nedge,
                                                       const EventConst* __restrict__ ec,
                                                       double* __restrict__ w /* [nspan][2][ND][2] */) {
  __shared__ double red[4 * ND][RB_BLOCK];
  const int s = blockIdx.x;
  const int64_t k0 = eidx[s], k1 = eidx[s + 1];
  const int64_t kend = (s + 2 == nedge) ? k1 + 1 : k1;
  const double f0 = tab64[k0].f, f1 = tab64[k1].f;
  const double inv = 1.0 / (f1 - f0);
  double fa[NBASIS], fT[ND];
#pragma unroll
  for (int m = 0; m < NBASIS; ++m) fa[m] = ec->fa[m];
#pragma unroll
  for (int d = 0; d < ND; ++d) fT[d] = ec->fT[d];
  double acc[4 * ND];
#pragma unroll
  for (int j = 0; j < 4 * ND; ++j) acc[j] = 0.0;
  for (int64_t k = k0 + threadIdx.x; k < kend; k += RB_BLOCK) {
    const RowF64<ND> r = tab64[k];
    const double t = (r.f - f0) * inv;
    const double psi = phase_poly(fa, r.x, r.w, r.w2, r.lnf);
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      double ph = fma(r.f, fT[d], psi);
      ph -= rint(ph);
      double sn, cs;
      sincos_cycles_f64(ph, sn, cs);
      // c = u p0 = (ur + i ui)(cs - i sn)
      const double cr = r.u[2 * d] * cs + r.u[2 * d + 1] * sn;
      const double ci = r.u[2 * d + 1] * cs - r.u[2 * d] * sn;
      acc[4 * d + 0] += (1.0 - t) * cr;
      acc[4 * d + 1] += (1.0 - t) * ci;
      acc[4 * d + 2] += t * cr;
      acc[4 * d + 3] += t * ci;
    }
  }
#pragma unroll
  for (int j = 0; j < 4 * ND; ++j) red[j][threadIdx.x] = acc[j];
  __syncthreads();
  for (int off = RB_BLOCK / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
#pragma unroll
      for (int j = 0; j < 4 * ND; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x < 4 * ND) {
    const int j = threadIdx.x, d = j / 4, q = j % 4;     // q: 0,1 = W0 (re, im); 2,3 = W1
    w[(((int64_t)s * 2 + q / 2) * ND + d) * 2 + (q % 2)] = red[j][0];
  }
}

// One thread per edge: the edge's rows (basis of its bin, u = V_e = W1 of the span before it +
// W0 of the span after it) and its adjoint basis rows. A single edge (one bin) keeps c itself.
template <int ND>
__global__ __launch_bounds__(RB_BLOCK) void k_rb_rows(const RowF64<ND>* __restrict__ fine64,
                                                      const RowGradF32* __restrict__ fine32g,
                                                      const RowGradF64* __restrict__ fine64g,
                                                      const int64_t* __restrict__ eidx, int nedge,
                                                      const double* __restrict__ w, const EventConst* __restrict__ ec,
                                                      RowF64<ND>* __restrict__ tab64, RowGradF32* __restrict__ g32,
                                                      RowGradF64* __restrict__ g64) {
  const int e = blockIdx.x * RB_BLOCK + threadIdx.x;
  if (e >= nedge) return;
  const int64_t k = eidx[e];
  RowF64<ND> r = fine64[k];
  if (nedge == 1) {
    const double psi = phase_poly(ec->fa, r.x, r.w, r.w2, r.lnf);
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      double ph = fma(r.f, ec->fT[d], psi);
      ph -= rint(ph);
      double sn, cs;
      sincos_cycles_f64(ph, sn, cs);
      const double ur = r.u[2 * d], ui = r.u[2 * d + 1];
      r.u[2 * d] = ur * cs + ui * sn;
      r.u[2 * d + 1] = ui * cs - ur * sn;
    }
  } else {
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      double vr = 0.0, vi = 0.0;
      if (e > 0) {                                   // W1 of span e-1
        vr += w[(((int64_t)(e - 1) * 2 + 1) * ND + d) * 2];
        vi += w[(((int64_t)(e - 1) * 2 + 1) * ND + d) * 2 + 1];
      }
      if (e < nedge - 1) {                           // W0 of span e
        vr += w[(((int64_t)e * 2) * ND + d) * 2];
        vi += w[(((int64_t)e * 2) * ND + d) * 2 + 1];
      }
      r.u[2 * d] = vr;
      r.u[2 * d + 1] = vi;
    }
  }
  tab64[e] = r;
  g32[e] = fine32g[k];
  g64[e] = fine64g[k];
}

// One workgroup: the float32 scale for the edge rows, uref = smallest power of two >= max |V|.
template <int ND>
__global__ __launch_bounds__(RB_BLOCK) void k_rb_uref(const RowF64<ND>* __restrict__ tab64, int nedge,
                                                      EventConst* __restrict__ ec) {
  __shared__ double red[RB_BLOCK];
  double m = 0.0;
  for (int e = threadIdx.x; e < nedge; e += RB_BLOCK) {
#pragma unroll
    for (int j = 0; j < 2 * ND; ++j) m = fmax(m, fabs(tab64[e].u[j]));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int off = RB_BLOCK / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double um = red[0];
    ec->uref = (um > 0.0 && isfinite(um)) ? exp2(ceil(log2(um))) : 1.0;
  }
}

template <int ND>
static hipError_t rb_nd(const void* fine64, const RowGradF32* fine32g, const RowGradF64* fine64g, const int64_t* eidx,
                        int nedge, double* w, EventConst* ec, void* tab64, void* tab32, RowGradF32* g32,
                        RowGradF64* g64, hipStream_t s) {
  if (nedge > 1)
    hipLaunchKernelGGL(k_rb_spans<ND>, dim3(nedge - 1), dim3(RB_BLOCK), 0, s, (const RowF64<ND>*)fine64, eidx, nedge,
                       (const EventConst*)ec, w);
  hipLaunchKernelGGL(k_rb_rows<ND>, dim3((nedge + RB_BLOCK - 1) / RB_BLOCK), dim3(RB_BLOCK), 0, s,
                     (const RowF64<ND>*)fine64, fine32g, fine64g, eidx, nedge, (const double*)w,
                     (const EventConst*)ec, (RowF64<ND>*)tab64, g32, g64);
  hipLaunchKernelGGL(k_rb_uref<ND>, dim3(1), dim3(RB_BLOCK), 0, s, (const RowF64<ND>*)tab64, nedge, ec);
  return launch_prep_mixed(ND, tab64, nedge, ec, tab32, s);
}

size_t rb_scratch_doubles(int nd, int nedge) { return (size_t)(nedge > 1 ? nedge - 1 : 1) * 4 * nd; }

hipError_t launch_rb(int nd, const void* fine64, const RowGradF32* fine32g, const RowGradF64* fine64g,
                     const int64_t* eidx, int nedge, double* w, EventConst* ec, void* tab64, void* tab32,
                     RowGradF32* g32, RowGradF64* g64, hipStream_t s) {
  switch (nd) {
    case 1: return rb_nd<1>(fine64, fine32g, fine64g, eidx, nedge, w, ec, tab64, tab32, g32, g64, s);
    case 2: return rb_nd<2>(fine64, fine32g, fine64g, eidx, nedge, w, ec, tab64, tab32, g32, g64, s);
    case 3: return rb_nd<3>(fine64, fine32g, fine64g, eidx, nedge, w, ec, tab64, tab32, g32, g64, s);
    case 4: return rb_nd<4>(fine64, fine32g, fine64g, eidx, nedge, w, ec, tab64, tab32, g32, g64, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace gwl
