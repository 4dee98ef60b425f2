// Per-bin work of the bin loop, shared by the single-event kernels and the persistent
// multi-event kernel: the float64 phase polynomial, the per-detector phasor and the complex
// multiply-accumulate (and, for the adjoint, the extra moments).
#pragma once

#include <hip/hip_runtime.h>

#include "gwl_common.h"
#include "gwl_device.h"
#include "gwl_phasor.h"

namespace gwl {

constexpr int NB = 8;  // bins per float32 block before the float64 flush (mixed precision)

// Float64 phasor by table and short polynomials. The float64 kernels carry the phase in table
// units, 1/N of a cycle (their per-point phase coefficients are scaled by N, a power of two, so
// every product and sum rounds exactly as in cycles): tu = n + y with n = rint(tu), |y| <= 1/2,
// and e^{2 pi i tu / N} = T[n mod N] e^{2 pi i y / N}. T holds (cos, sin) of 2 pi k / N in LDS
// (32 KB per workgroup), copied from a table the compiler builds. With N = 2048,
// |2 pi y / N| <= 1.6e-3, and the Taylor series of sin(2 pi y / N) and cos(2 pi y / N) stop after
// their y^3 and y^4 terms: the first omitted terms are below 7.2e-17 and 2e-20 in absolute value
// (under half a unit in the last place of a result near 1). The series' coefficients are those
// of sin(2 pi y) and cos(2 pi y) divided by powers of N (exact).
constexpr int PH_TBL = 2048;
static __device__ const PhasorTable<PH_TBL> kPhasorTable = make_phasor_table<PH_TBL>();
__device__ __forceinline__ void fill_phasor_table(double2* tbl, int first = 0) {
  // by threads first .. blockDim.x - 1
  for (int k = (int)threadIdx.x - first; k < PH_TBL; k += (int)blockDim.x - first)
    tbl[k] = make_double2(kPhasorTable.e[k].c, kPhasorTable.e[k].s);
}
template <int ND>
__device__ __forceinline__ void to_table_units(double (&a)[NBASIS], double (&T)[ND]) {
#pragma unroll
  for (int m = 0; m < NBASIS; ++m) a[m] *= (double)PH_TBL;
#pragma unroll
  for (int d = 0; d < ND; ++d) T[d] *= (double)PH_TBL;
}
// The integer n comes from adding and subtracting 1.5 * 2^52: for |tu| < 2^51 the sum lies in
// [2^52, 2^53), where the float64 spacing is 1, so it is rounded to the nearest integer (ties to
// even), and its low mantissa bits are n modulo 2^52 in two's complement; the low 11 bits are
// the table index for negative n too. (A float64 -> int32 conversion would clamp beyond 2^31.)
// The set-up keeps |tu| below 2048 * PHASE_LIMIT = 2^50 or marks the point invalid.
__device__ __forceinline__ void sincos_tbl(double tu, const double2* __restrict__ tbl, double& s, double& c) {
  constexpr double N = PH_TBL;
  constexpr double RND = 6755399441055744.0;     // 1.5 * 2^52
  const double t = tu + RND;
  const double n = t - RND;                      // rint(tu), exact
  const double y = tu - n;                       // exact, |y| <= 1/2
  const double2 e = tbl[(unsigned)__double2loint(t) & (PH_TBL - 1)];
  const double z = y * y;
  const double ps = fma(z, -41.34170224039976 / (N * N * N), 6.283185307179586 / N);  // sin(2 pi y / N) / y
  const double sv = ps * y;
  const double pc = fma(fma(z, 64.9393940226683 / (N * N * N * N), -19.739208802178716 / (N * N)), z, 1.0);
  c = fma(e.x, pc, -(e.y * sv));
  s = fma(e.y, pc, e.x * sv);
}

// Member-wise row loads, valid for plain and address-space-qualified table pointers.
template <int ND, class P>
__device__ __forceinline__ RowMixed<ND> load_row_mixed(P tab, int k) {
  RowMixed<ND> r;
  r.f = tab[k].f; r.x = tab[k].x; r.w = tab[k].w; r.w2 = tab[k].w2; r.lnf = tab[k].lnf;
#pragma unroll
  for (int j = 0; j < 2 * ND; ++j) r.u[j] = tab[k].u[j];
  return r;
}
template <int ND, class P>
__device__ __forceinline__ RowF64<ND> load_row_f64(P tab, int k) {
  RowF64<ND> r;
  r.f = tab[k].f; r.x = tab[k].x; r.w = tab[k].w; r.w2 = tab[k].w2; r.lnf = tab[k].lnf;
#pragma unroll
  for (int j = 0; j < 2 * ND; ++j) r.u[j] = tab[k].u[j];
  return r;
}
template <class P>
__device__ __forceinline__ RowGradF32 load_grad_f32(P g, int k) {
  RowGradF32 r;
#pragma unroll
  for (int m = 0; m < NBASIS; ++m) r.g[m] = g[k].g[m];
  r.f = g[k].f;
  return r;
}
template <class P>
__device__ __forceinline__ RowGradF64 load_grad_f64(P g, int k) {
  RowGradF64 r;
  r.g2 = g[k].g2; r.g3 = g[k].g3; r.g6 = g[k].g6; r.g7 = g[k].g7;
  return r;
}

// Horner form of sum_m a_m g_m(f) in x = f^(1/3):  a0 w + w2 (a1 + x (a2 + x (a3 + x (a4 ln f
//   + x (a5 + a6 ln f + x a7))))),  w = f^-5/3, w2 = f^-1.
__device__ __forceinline__ double phase_poly(const double (&a)[NBASIS], double x, double w, double w2, double lnf) {
  double t = fma(a[7], x, fma(a[6], lnf, a[5]));
  t = fma(t, x, a[4] * lnf);
  t = fma(t, x, a[3]);
  t = fma(t, x, a[2]);
  t = fma(t, x, a[1]);
  return fma(w2, t, w * a[0]);
}

// One bin of the mixed-precision loop. The complex sums Z_det go into the float32 block sums z;
// the adjoint's moments (f y_det per detector, g_m y for the eight basis functions) go straight
// into float64 (tot[2 ND ..]), with the basis values in float64: the gradient combines these
// moments with coefficients of both signs that nearly cancel for the mass and spin directions,
// so a float32 rounding on each moment would be magnified there. On this chip a float64 FMA
// issues at the rate of an unpacked float32 one, so this costs about what the float32 block sums
// and their flushes did.
template <int ND, bool GRAD, class GradP>
__device__ __forceinline__ void mixed_bin(const RowMixed<ND> r, GradP gt, int k,
                                          const double (&a)[NBASIS], const double (&T)[ND], const float (&cr)[ND],
                                          const float (&ci)[ND], float (&z)[2 * ND], double (&tot)[nz_of(ND, GRAD)]) {
  const double psi = phase_poly(a, r.x, r.w, r.w2, r.lnf);
  double y = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const double ph = fma(r.f, T[d], psi);
    const float rr = (float)__builtin_amdgcn_fract(ph);  // [0, 1) cycles
    const float cs = __builtin_amdgcn_cosf(rr);
    const float sn = __builtin_amdgcn_sinf(rr);
    const float ur = r.u[2 * d], ui = r.u[2 * d + 1];
    if (!GRAD) {
      // u (cs - i sn)
      z[2 * d] = fmaf(ur, cs, fmaf(ui, sn, z[2 * d]));
      z[2 * d + 1] = fmaf(ui, cs, fmaf(-ur, sn, z[2 * d + 1]));
    } else {
      const float wr = fmaf(ur, cs, ui * sn);
      const float wi = fmaf(ui, cs, -(ur * sn));
      z[2 * d] += wr;
      z[2 * d + 1] += wi;
      const double yd = (double)fmaf(cr[d], wi, ci[d] * wr);  // Im(c_det w)
      tot[2 * ND + d] = fma(r.f, yd, tot[2 * ND + d]);
      y = d == 0 ? yd : y + yd;
    }
  }
  if (GRAD) {
    const RowGradF64 g = load_grad_f64(gt, k);
    const double gm[NBASIS] = {r.w, r.w2, g.g2, g.g3, r.lnf, r.x, g.g6, g.g7};
#pragma unroll
    for (int m = 0; m < NBASIS; ++m) tot[3 * ND + m] = fma(gm[m], y, tot[3 * ND + m]);
  }
}

// The float64 multiply-accumulate of one bin: detector d's phasor cs[d] + i sn[d] against its
// whitened data, into the complex sums (and, for the adjoint, the real moments).
template <int ND, bool GRAD, class GradP>
__device__ __forceinline__ void f64_mac(const RowF64<ND>& r, GradP gt, int k, const double (&cs)[ND],
                                        const double (&sn)[ND], const double (&cr)[ND], const double (&ci)[ND],
                                        double (&z)[nz_of(ND, GRAD)]) {
  double y = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const double ur = r.u[2 * d], ui = r.u[2 * d + 1];
    if (!GRAD) {
      z[2 * d] = fma(ur, cs[d], fma(ui, sn[d], z[2 * d]));
      z[2 * d + 1] = fma(ui, cs[d], fma(-ur, sn[d], z[2 * d + 1]));
    } else {
      const double wr = fma(ur, cs[d], ui * sn[d]);
      const double wi = fma(ui, cs[d], -(ur * sn[d]));
      z[2 * d] += wr;
      z[2 * d + 1] += wi;
      const double yd = fma(cr[d], wi, ci[d] * wr);  // Im(c_det w)
      z[2 * ND + d] = fma(r.f, yd, z[2 * ND + d]);
      y = d == 0 ? yd : y + yd;
    }
  }
  if (GRAD) {
    const RowGradF64 g = load_grad_f64(gt, k);
    const double gm[NBASIS] = {r.w, r.w2, g.g2, g.g3, r.lnf, r.x, g.g6, g.g7};
#pragma unroll
    for (int m = 0; m < NBASIS; ++m) z[3 * ND + m] = fma(gm[m], y, z[3 * ND + m]);
  }
}

template <int ND, bool GRAD, class GradP>
__device__ __forceinline__ void f64_bin(const RowF64<ND> r, GradP gt, int k,
                                        const double (&a)[NBASIS], const double (&T)[ND], const double (&cr)[ND],
                                        const double (&ci)[ND], const double2* __restrict__ tbl,
                                        double (&z)[nz_of(ND, GRAD)]) {
  const double psi = phase_poly(a, r.x, r.w, r.w2, r.lnf);
  double y = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    double sn, cs;
    sincos_tbl(fma(r.f, T[d], psi), tbl, sn, cs);  // phase in table units
    const double ur = r.u[2 * d], ui = r.u[2 * d + 1];
    if (!GRAD) {
      z[2 * d] = fma(ur, cs, fma(ui, sn, z[2 * d]));
      z[2 * d + 1] = fma(ui, cs, fma(-ur, sn, z[2 * d + 1]));
    } else {
      const double wr = fma(ur, cs, ui * sn);
      const double wi = fma(ui, cs, -(ur * sn));
      z[2 * d] += wr;
      z[2 * d + 1] += wi;
      const double yd = fma(cr[d], wi, ci[d] * wr);  // Im(c_det w)
      z[2 * ND + d] = fma(r.f, yd, z[2 * ND + d]);
      y = d == 0 ? yd : y + yd;
    }
  }
  if (GRAD) {
    const RowGradF64 g = load_grad_f64(gt, k);
    const double gm[NBASIS] = {r.w, r.w2, g.g2, g.g3, r.lnf, r.x, g.g6, g.g7};
#pragma unroll
    for (int m = 0; m < NBASIS; ++m) z[3 * ND + m] = fma(gm[m], y, z[3 * ND + m]);
  }
}

// A row with its whitened data zeroed in the lanes whose point is cut off below bin k (the
// optional ISCO cut-off: kc bins kept), so that the bin adds nothing there.
template <int ND, class Row>
__device__ __forceinline__ Row cut_row(Row r, int k, int kc) {
  const bool keep = k < kc;
#pragma unroll
  for (int j = 0; j < 2 * ND; ++j) r.u[j] = keep ? r.u[j] : 0;
  return r;
}

// The bin loop of one wavefront: points in lanes, bins [k0, k1) of one event.
// Mixed precision: the complex sums in float32 over blocks of NB bins, each block added into
// float64; the adjoint moments in float64 throughout (see mixed_bin). CUT: each lane keeps only
// its first kc bins.
template <int ND, bool GRAD, class TabP, class GradP, bool CUT = false>
__device__ __forceinline__ void bin_loop_mixed(TabP tab, GradP gtab,
                                               int k0, int k1, const double (&a)[NBASIS], const double (&T)[ND],
                                               const float (&cr)[ND], const float (&ci)[ND],
                                               double (&tot)[nz_of(ND, GRAD)], int kc = 0) {
  constexpr int NZ = nz_of(ND, GRAD);
  constexpr int NF = 2 * ND;  // float32 block sums
#pragma unroll
  for (int z = 0; z < NZ; ++z) tot[z] = 0.0;
  int k = k0;
  if (k + NB <= k1) {
    // each bin's row is requested ahead of its use, two bins ahead in the forward loop and one
    // in the adjoint (whose registers would lose it a wavefront per SIMD); the tables carry
    // TAB_PAD zero rows after the last bin, so the look-ahead read past a chunk's end stays in
    // bounds
    RowMixed<ND> cur = load_row_mixed<ND>(tab, k), nx1 = load_row_mixed<ND>(tab, k + (GRAD ? 0 : 1));
    for (; k + NB <= k1; k += NB) {
      float z[NF];
#pragma unroll
      for (int j = 0; j < NF; ++j) z[j] = 0.0f;
#pragma unroll 2
      for (int j = 0; j < NB; ++j) {
        if constexpr (GRAD) {
          const RowMixed<ND> nxt = load_row_mixed<ND>(tab, k + j + 1);
          mixed_bin<ND, GRAD, GradP>(CUT ? cut_row<ND>(cur, k + j, kc) : cur, gtab, k + j, a, T, cr, ci, z, tot);
          cur = nxt;
        } else {
          const RowMixed<ND> nx2 = load_row_mixed<ND>(tab, k + j + 2);
          mixed_bin<ND, GRAD, GradP>(CUT ? cut_row<ND>(cur, k + j, kc) : cur, gtab, k + j, a, T, cr, ci, z, tot);
          cur = nx1;
          nx1 = nx2;
        }
      }
#pragma unroll
      for (int j = 0; j < NF; ++j) tot[j] += (double)z[j];
    }
  }
  if (k < k1) {
    float z[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j) z[j] = 0.0f;
    for (; k < k1; ++k) {
      const RowMixed<ND> r = load_row_mixed<ND>(tab, k);
      mixed_bin<ND, GRAD, GradP>(CUT ? cut_row<ND>(r, k, kc) : r, gtab, k, a, T, cr, ci, z, tot);
    }
#pragma unroll
    for (int j = 0; j < NF; ++j) tot[j] += (double)z[j];
  }
}

// Float64: sums in float64 throughout.
template <int ND, bool GRAD, class TabP, class GradP, bool CUT = false>
__device__ __forceinline__ void bin_loop_f64(TabP tab, GradP gtab,
                                             int k0, int k1, const double (&a)[NBASIS], const double (&T)[ND],
                                             const double (&cr)[ND], const double (&ci)[ND],
                                             const double2* __restrict__ tbl, double (&z)[nz_of(ND, GRAD)],
                                             int kc = 0) {
  constexpr int NZ = nz_of(ND, GRAD);
#pragma unroll
  for (int j = 0; j < NZ; ++j) z[j] = 0.0;
  if (k0 >= k1) return;
  // rows requested one bin ahead (two ahead measured no faster here and cost registers)
  RowF64<ND> cur = load_row_f64<ND>(tab, k0);
#pragma unroll 2
  for (int k = k0; k < k1; ++k) {
    const RowF64<ND> nxt = load_row_f64<ND>(tab, k + 1);
    f64_bin<ND, GRAD, GradP>(CUT ? cut_row<ND>(cur, k, kc) : cur, gtab, k, a, T, cr, ci, tbl, z);
    cur = nxt;
  }
}

// Float64 on a uniform grid (f_k = f_0 + k step): the detectors' phases differ only by
// f (T_det - T_0), so detector 0's phasor is looked up per bin and every other detector's is
// detector 0's times r_det(f_k) = exp(2 pi i f_k (T_det - T_0)), a geometric sequence in k with
// ratio exp(2 pi i step (T_det - T_0)). The sequence is restarted from an exact r_det every NROT
// bins, so the recurrence's rounding never acts over more than NROT steps (|T_det - T_0| is at
// most the Earth's light-crossing time, 0.043 s: under 90 cycles at 2 kHz). Per detector after
// the first this replaces the phase shift, the table lookup and the series (15 float64
// instructions and one LDS read) by two complex multiplies (8). a and T are in table units.
//
// The forward pass needs only the sums Z_det = sum_k u_k conj(p_0,k) conj(r_det,k), so it does
// not form each detector's phasor: over a block of bins kb..ke-1 it runs the Horner recurrence
// G <- G rho + u_k conj(p_0,k) (rho = exp(2 pi i step (T_det - T_0))), which leaves
// G = sum_k u_k conj(p_0,k) rho^(ke-1-k), and closes the block with Z_det += G conj(r_det,ke-1),
// r_det taken exactly at the block's last bin. Since |rho| = 1 this is the same sum; the
// recurrence costs one complex multiply-add per bin and detector (8 instructions) where the
// phasor, its rotation and the multiply-accumulate cost 12.
constexpr int NROT = 32;
template <int ND, bool GRAD, class TabP, class GradP>
__device__ __forceinline__ void bin_loop_f64_rot(TabP tab, GradP gtab, int k0, int k1, const double (&a)[NBASIS],
                                                 const double (&T)[ND], const double (&cr)[ND],
                                                 const double (&ci)[ND], const double2* __restrict__ tbl, double step,
                                                 double (&z)[nz_of(ND, GRAD)]) {
  constexpr int NZ = nz_of(ND, GRAD);
#pragma unroll
  for (int j = 0; j < NZ; ++j) z[j] = 0.0;
  if (k0 >= k1) return;
  double D[ND], pr[ND], pim[ND];
  D[0] = 0.0;
  pr[0] = 1.0;
  pim[0] = 0.0;
#pragma unroll
  for (int d = 1; d < ND; ++d) {
    D[d] = T[d] - T[0];
    sincos_tbl(step * D[d], tbl, pim[d], pr[d]);  // the ratio exp(2 pi i step D_d)
  }
  RowF64<ND> cur = load_row_f64<ND>(tab, k0);
  if constexpr (!GRAD) {
    for (int kb = k0; kb < k1; kb += NROT) {
      double gr[ND], gi[ND];
#pragma unroll
      for (int d = 0; d < ND; ++d) gr[d] = gi[d] = 0.0;
      const int ke = kb + NROT < k1 ? kb + NROT : k1;
      double flast = cur.f;
#pragma unroll 2
      for (int k = kb; k < ke; ++k) {
        const RowF64<ND> nxt = load_row_f64<ND>(tab, k + 1);
        const double psi = phase_poly(a, cur.x, cur.w, cur.w2, cur.lnf);
        double c0, s0;
        sincos_tbl(fma(cur.f, T[0], psi), tbl, s0, c0);
        z[0] = fma(cur.u[0], c0, fma(cur.u[1], s0, z[0]));       // u_0 conj(p_0)
        z[1] = fma(cur.u[1], c0, fma(-cur.u[0], s0, z[1]));
#pragma unroll
        for (int d = 1; d < ND; ++d) {
          const double ur = cur.u[2 * d], ui = cur.u[2 * d + 1];
          const double ar = fma(ur, c0, ui * s0), ai = fma(ui, c0, -(ur * s0));  // u_d conj(p_0)
          const double t = gr[d];
          gr[d] = fma(t, pr[d], fma(-gi[d], pim[d], ar));
          gi[d] = fma(t, pim[d], fma(gi[d], pr[d], ai));
        }
        flast = cur.f;
        cur = nxt;
      }
#pragma unroll
      for (int d = 1; d < ND; ++d) {
        double qr, qi;
        sincos_tbl(flast * D[d], tbl, qi, qr);                    // exact r_det at the last bin
        z[2 * d] = fma(gr[d], qr, fma(gi[d], qi, z[2 * d]));     // G conj(r_det)
        z[2 * d + 1] = fma(gi[d], qr, fma(-gr[d], qi, z[2 * d + 1]));
      }
    }
    return;
  }
  for (int kb = k0; kb < k1; kb += NROT) {
    double qr[ND], qi[ND];
    qr[0] = 1.0;
    qi[0] = 0.0;
#pragma unroll
    for (int d = 1; d < ND; ++d) sincos_tbl(cur.f * D[d], tbl, qi[d], qr[d]);  // exact restart
    const int ke = kb + NROT < k1 ? kb + NROT : k1;
#pragma unroll 2
    for (int k = kb; k < ke; ++k) {
      const RowF64<ND> nxt = load_row_f64<ND>(tab, k + 1);
      const double psi = phase_poly(a, cur.x, cur.w, cur.w2, cur.lnf);
      double cs[ND], sn[ND];
      sincos_tbl(fma(cur.f, T[0], psi), tbl, sn[0], cs[0]);
#pragma unroll
      for (int d = 1; d < ND; ++d) {
        cs[d] = fma(cs[0], qr[d], -(sn[0] * qi[d]));
        sn[d] = fma(sn[0], qr[d], cs[0] * qi[d]);
        const double t = qr[d];
        qr[d] = fma(t, pr[d], -(qi[d] * pim[d]));
        qi[d] = fma(t, pim[d], qi[d] * pr[d]);
      }
      f64_mac<ND, GRAD, GradP>(cur, gtab, k, cs, sn, cr, ci, z);
      cur = nxt;
    }
  }
}

// Read-only tables reached through a pointer held in memory (not a kernel argument) are read
// through the constant address space: the compiler can then use scalar loads for wave-uniform
// addresses, as it does for `const __restrict__` kernel arguments.
template <class T>
using const_as_ptr = const __attribute__((address_space(4))) T*;
template <class T>
using global_as_ptr = __attribute__((address_space(1))) T*;

// Per-lane coefficients of point pc from the set-up rows coef[row][Bp].
template <int ND, class QT>
__device__ __forceinline__ void load_coef(const double* __restrict__ coef, int64_t Bp, int64_t pc, bool grad,
                                          double (&a)[NBASIS], double (&T)[ND], QT (&cr)[ND], QT (&ci)[ND]) {
#pragma unroll
  for (int m = 0; m < NBASIS; ++m) a[m] = coef[(CO_A + m) * Bp + pc];
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    T[d] = coef[(CO_T + d) * Bp + pc];
    cr[d] = grad ? (QT)coef[(CO_CR + d) * Bp + pc] : (QT)0;
    ci[d] = grad ? (QT)coef[(CO_CI + d) * Bp + pc] : (QT)0;
  }
}

// The optional ISCO cut-off (GWL_F_ISCO_CUTOFF): the number of grid bins at or below the
// gravitational-wave frequency of the innermost stable circular orbit of the point's total
// mass, f_isco = 1 / (6^(3/2) pi T_sun M) (twice the orbital frequency at r = 6 G M / c^2). The
// grid is increasing; a first guess from its mean spacing is corrected by stepping, with a
// bisection if the guess is far off. Every caller (set-up, evaluation, gradient epilogue) takes
// the same decision in float64.
__device__ inline int isco_bins(double mc, double q, const double* __restrict__ fgrid, int64_t M, const EventConst& ec) {
  const double eta = q / ((1.0 + q) * (1.0 + q));
  const double mtot = mc * pow(eta, -0.6);
  const double fi = 1.0 / (14.696938456699067 * kPi * kTsun * mtot);  // 6^(3/2) = 14.696938456699067
  if (!(fi > 0.0) || !isfinite(fi)) return 0;
  // first index with f > fi
  double g = floor((fi - ec.fmin) / ec.grid_df) + 1.0;
  g = fmin(fmax(g, 0.0), (double)M);
  int64_t k = (int64_t)g;
  for (int it = 0; it < 8; ++it) {
    if (k > 0 && fgrid[k - 1] > fi) --k;
    else if (k < M && fgrid[k] <= fi) ++k;
    else return (int)k;
  }
  int64_t lo = 0, hi = M;  // bisection: f[k] <= fi for k < lo, f[k] > fi for k >= hi
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (fgrid[mid] <= fi) lo = mid + 1;
    else hi = mid;
  }
  return (int)lo;
}

// Largest value of v across the wavefront (every lane gets it, as a scalar).
__device__ inline int wave_max(int v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
  return __builtin_amdgcn_readfirstlane(v);
}

}  // namespace gwl
