// Detector calibration model (paper section 2, "Models and parameter spaces": amplitude and
// phase corrections at frequency nodes, ten per detector): the calibrated model is
//   h_cal,det(f) = h_det(f) (1 + dA_det(f)) exp(i dphi_det(f)),
// dA and dphi cubic Catmull-Rom splines in ln f through the node values (theta columns
// 11 + 2 n det .. : n amplitude values, then n phase values in radians).
//
// The bin loop is the ordinary one with one more complex factor per (point, detector, bin):
// the spline value is a four-term dot product of per-bin weights (RowCal, wave-uniform) with the
// point's four window node values (VGPRs, fixed over a node interval, so chunks never cross an
// interval). <h_cal|h_cal> needs no per-bin work: with K_k = 4 df f_k^-7/3 / S_k,
//   sum_k K_k (1 + dA_k)^2 = K + 2 alpha.K1 + alpha.K2.alpha,
// K1_j = sum_k K_k w_kj and K2_jl = sum_k K_k w_kj w_kl computed once per event (alpha the
// amplitude node values, w_kj the spline weight of node j at bin k).
//
// Adjoint: besides the uncalibrated moments (with w = u p replaced by the calibrated product),
// per detector and window node i the sums sum_k w_ki Re(c q_k) (amplitude) and
// sum_k w_ki Im(c w_cal,k) (phase), q = u p exp(i dphi), w_cal = (1 + dA) q.
#include <hip/hip_runtime.h>

#include "gwl_bins.h"
#include "gwl_common.h"
#include "gwl_device.h"
#include "gwl_epilogue.h"
#include "gwl_launch.h"
#include "gwl_setup.h"

namespace gwl {

// Set-up of a calibrated call: the point model's rows as k_setup writes them (two wavefronts per
// 64 points, one per half of the model), and the calibration node values turned from theta's
// columns 11.. into rows calc [ncal][Bp], each wavefront copying half of them; every row of a
// point with a non-finite node value is NaN.
template <int ND>
__global__ __launch_bounds__(2 * WAVE) void k_setup_cal(EventGeom g, const EventConst* __restrict__ ec, bool scaled,
                                                        const double* __restrict__ theta, int P, int ncal, int64_t B,
                                                        int64_t Bp, double* __restrict__ coef,
                                                        double* __restrict__ calc) {
  __shared__ double rows_s[NCOEF * WAVE];
  __shared__ int ok_s[2][WAVE];
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
  const int lane = (int)(threadIdx.x % WAVE);
  const int64_t p = (int64_t)blockIdx.x * WAVE + lane;   // < Bp: Bp is a multiple of 64
  const int64_t pc = p < B ? p : B - 1;                  // padding lanes repeat the last point
  setup_halves<ND>(w, lane, theta + pc * P, g, ec, rows_s);
  const int half = (ncal + 1) / 2, j0 = w * half, j1 = w == 0 ? half : ncal;
  bool ok = true;
  for (int j = j0; j < j1; ++j) {
    const double v = theta[pc * P + NPARAM + j];
    ok &= isfinite(v);
    calc[(int64_t)j * Bp + p] = v;
  }
  ok_s[w][lane] = ok ? 1 : 0;
  __syncthreads();
  setup_rows_write<ND>(w, lane, rows_s, ec, scaled, ok_s[0][lane] && ok_s[1][lane], coef, Bp, p);
}

// One bin of the calibrated loop. T_ is float (mixed: hardware phasors, float32 products) or
// double (float64: table phasor).
// 1 + dA and dphi come from their cubics in the bin's position t in the node interval (kA, kP:
// coefficients of t^0 .. t^3 for this chunk's interval, 1 included in kA[.][0]); the window
// weights cw (the same cubics' parts per node) serve only the adjoint's node moments.
template <int ND, bool GRAD, class T_, class Row, class CalRow, class GradP>
__device__ __forceinline__ void cal_bin(const Row r, const CalRow cw, T_ t, GradP gt, int k,
                                        const double (&a)[NBASIS], const double (&T)[ND], const T_ (&cr)[ND],
                                        const T_ (&ci)[ND], const T_ (&kA)[ND][4], const T_ (&kP)[ND][4],
                                        const double2* tbl, T_ (&z)[nz_cal(ND, GRAD)]) {
  constexpr bool MIXED = sizeof(T_) == 4;
  constexpr int MA = 3 * ND + NBASIS, MB = MA + 4 * ND;
  const double psi = phase_poly(a, r.x, r.w, r.w2, r.lnf);
  T_ y = 0, fk = 0;
  T_ gm[NBASIS];
  if constexpr (GRAD) {
    if constexpr (MIXED) {
      const RowGradF32 g = load_grad_f32(gt, k);
#pragma unroll
      for (int m = 0; m < NBASIS; ++m) gm[m] = g.g[m];
      fk = g.f;
    } else {
      const RowGradF64 g = load_grad_f64(gt, k);
      gm[0] = r.w; gm[1] = r.w2; gm[2] = g.g2; gm[3] = g.g3; gm[4] = r.lnf; gm[5] = r.x; gm[6] = g.g6; gm[7] = g.g7;
      fk = r.f;
    }
  }
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    // g1 = 1 + dA and dphi at this bin (Horner in t)
    const T_ g1 = fma(fma(fma(kA[d][3], t, kA[d][2]), t, kA[d][1]), t, kA[d][0]);
    const T_ dp = fma(fma(fma(kP[d][3], t, kP[d][2]), t, kP[d][1]), t, kP[d][0]);
    // q = u p exp(i dphi) = u exp(-2 pi i (phi - dphi / 2 pi)): the calibration phase joins the
    // model phase before the phasor, so one phasor (with its gain correction) serves both. The
    // mixed variant subtracts dphi / 2 pi (at most a few hundredths of a cycle) in float32 from
    // the reduced phase; the float64 variant adds it in table units before the reduction.
    T_ cs, sn;
    if constexpr (MIXED) {
      const float rr = fmaf(dp, -0.15915494f, (float)__builtin_amdgcn_fract(fma(r.f, T[d], psi)));
      cs = __builtin_amdgcn_cosf(rr);
      sn = __builtin_amdgcn_sinf(rr);
    } else {
      sincos_tbl(fma(dp, -0.15915494309189535 * PH_TBL, fma(r.f, T[d], psi)), tbl, sn, cs);
    }
    const T_ ur = r.u[2 * d], ui = r.u[2 * d + 1];
    const T_ qr = fma(ur, cs, ui * sn);
    const T_ qi = fma(ui, cs, -(ur * sn));
    if constexpr (!GRAD) {
      z[2 * d] = fma(g1, qr, z[2 * d]);            // calibrated product g1 q
      z[2 * d + 1] = fma(g1, qi, z[2 * d + 1]);
    } else {
      const T_ vr = g1 * qr, vi = g1 * qi;          // calibrated product
      z[2 * d] += vr;
      z[2 * d + 1] += vi;
      const T_ yd = fma(cr[d], vi, ci[d] * vr);     // Im(c w_cal)
      const T_ ya = fma(cr[d], qr, -(ci[d] * qi));  // Re(c q)
      z[2 * ND + d] = fma(fk, yd, z[2 * ND + d]);
      y = d == 0 ? yd : y + yd;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        z[MA + 4 * d + i] = fma(cw.w[i], ya, z[MA + 4 * d + i]);
        z[MB + 4 * d + i] = fma(cw.w[i], yd, z[MB + 4 * d + i]);
      }
    }
  }
  if constexpr (GRAD) {
#pragma unroll
    for (int m = 0; m < NBASIS; ++m) z[3 * ND + m] = fma(gm[m], y, z[3 * ND + m]);
  }
}

// Workgroup -> (chunk, point group) as in the plain loop; a chunk is a piece of one interval
// (intervals are cut into pieces of similar length, so chunks cost about the same).
__device__ __forceinline__ bool locate_cal(const CalShape& sh, int& c, int& j, int64_t& k0, int64_t& k1, int& pg) {
  const int bid = blockIdx.x;
  const int item = (bid % NXCD) * sh.gper + bid / NXCD;
  if (item >= sh.items) return false;
  c = item / sh.nbpg;
  pg = (item - c * sh.nbpg) * WAVES_PER_BLOCK + (int)(threadIdx.x / WAVE);
  if (pg >= sh.npg) return false;
  j = sh.cj[c];
  k0 = sh.ck[c];
  k1 = sh.ck[c + 1];
  return true;
}

// Wavefronts per SIMD the register budget must allow: three for the mixed adjoint up to three
// detectors (its window moments' float64 totals live in LDS for that), otherwise no bound.
template <int ND, bool MIXED, bool GRAD>
constexpr int cal_waves_per_eu() {
  return (MIXED && GRAD && ND <= 3) ? 3 : 1;
}

template <int ND, bool MIXED, bool GRAD>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(cal_waves_per_eu<ND, MIXED, GRAD>()))) void k_bins_cal(const void* __restrict__ tabv, const void* __restrict__ gtabv,
                                                    const void* __restrict__ calwv, const void* __restrict__ caltv,
                                                    const double* __restrict__ calB, const double* __restrict__ coef,
                                                    const double* __restrict__ calc, int64_t B, int64_t Bp,
                                                    CalShape sh, double* __restrict__ part) {
  typedef typename std::conditional<MIXED, float, double>::type T_;
  constexpr int NZ = nz_cal(ND, GRAD);
  __shared__ double2 tbl[MIXED ? 1 : PH_TBL];  // the float64 phasor table
  // mixed adjoint: the float64 totals of the 8 ND window moments stay in LDS (one column per
  // lane, so no barrier), which keeps the kernel at three wavefronts per SIMD instead of two
  constexpr int NNODE = 8 * ND, NZU = NZ - NNODE;
  __shared__ double ntot[MIXED && GRAD ? NNODE : 1][MIXED && GRAD ? BLOCK : 1];
  if constexpr (!MIXED) {
    fill_phasor_table(tbl);
    __syncthreads();
  }
  int c, j, pg;
  int64_t k0, k1;
  if (!locate_cal(sh, c, j, k0, k1, pg)) return;
  const int64_t p = (int64_t)pg * WAVE + (threadIdx.x % WAVE);
  const int64_t pc = p < B ? p : B - 1;
  double a[NBASIS], T[ND];
  T_ cr[ND], ci[ND];
  load_coef<ND, T_>(coef, Bp, pc, GRAD, a, T, cr, ci);
  if constexpr (!MIXED) to_table_units<ND>(a, T);  // the float64 phase runs in 1/PH_TBL cycles
  // this point's amplitude and phase node values in the window of the chunk's interval, turned
  // into the cubics' coefficients: k[p] = sum_i v_i B[i][p] (1 added to the amplitude's k[0])
  T_ kA[ND][4], kP[ND][4];
  {
    const int n = sh.nnode, j0 = sh.j0[j];
    const double* Bj = calB + (int64_t)j * 16;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      T_ va[4], vp[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        va[i] = (T_)calc[(int64_t)(2 * n * d + j0 + i) * Bp + pc];
        vp[i] = (T_)calc[(int64_t)(2 * n * d + n + j0 + i) * Bp + pc];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T_ sa = q == 0 ? (T_)1 : (T_)0, sp = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          sa = fma(va[i], (T_)Bj[i * 4 + q], sa);
          sp = fma(vp[i], (T_)Bj[i * 4 + q], sp);
        }
        kA[d][q] = sa;
        kP[d][q] = sp;
      }
    }
  }
  double tot[NZ];
#pragma unroll
  for (int zz = 0; zz < NZ; ++zz) tot[zz] = 0.0;
  if constexpr (MIXED && GRAD) {
#pragma unroll
    for (int i = 0; i < NNODE; ++i) ntot[i][threadIdx.x] = 0.0;
  }
  // a float32 block's sums into the float64 totals
  auto flush = [&](const float (&z)[NZ]) {
    if constexpr (MIXED && GRAD) {
#pragma unroll
      for (int zz = 0; zz < NZU; ++zz) tot[zz] += (double)z[zz];
#pragma unroll
      for (int i = 0; i < NNODE; ++i) ntot[i][threadIdx.x] += (double)z[NZU + i];
    } else {
#pragma unroll
      for (int zz = 0; zz < NZ; ++zz) tot[zz] += (double)z[zz];
    }
  };
  if constexpr (MIXED) {
    const RowMixed<ND>* tab = (const RowMixed<ND>*)tabv;
    const RowGradF32* gt = (const RowGradF32*)gtabv;
    const RowCal32* cw = (const RowCal32*)calwv;
    const float* ct = (const float*)caltv;
    // float32 blocks of NB bins added into float64; each bin's rows are requested one bin ahead
    // (the tables carry zero padding rows past the last bin). Only the adjoint reads the weights.
    int k = (int)k0;
    const int kend = (int)k1;
    if (k < kend) {
      RowMixed<ND> cur = load_row_mixed<ND>(tab, k);
      RowCal32 cwc;
      if constexpr (GRAD) cwc = cw[k];
      float tc = ct[k];
      for (; k + NB <= kend; k += NB) {
        float z[NZ];
#pragma unroll
        for (int zz = 0; zz < NZ; ++zz) z[zz] = 0.0f;
#pragma unroll 2
        for (int jj = 0; jj < NB; ++jj) {
          const RowMixed<ND> nxt = load_row_mixed<ND>(tab, k + jj + 1);
          RowCal32 cwn;
          if constexpr (GRAD) cwn = cw[k + jj + 1];
          const float tn = ct[k + jj + 1];
          cal_bin<ND, GRAD, float>(cur, cwc, tc, gt, k + jj, a, T, cr, ci, kA, kP, tbl, z);
          cur = nxt;
          if constexpr (GRAD) cwc = cwn;
          tc = tn;
        }
        flush(z);
      }
      if (k < kend) {
        float z[NZ];
#pragma unroll
        for (int zz = 0; zz < NZ; ++zz) z[zz] = 0.0f;
        for (; k < kend; ++k)
          cal_bin<ND, GRAD, float>(load_row_mixed<ND>(tab, k), cw[k], ct[k], gt, k, a, T, cr, ci, kA, kP, tbl, z);
        flush(z);
      }
    }
    if constexpr (GRAD) {
#pragma unroll
      for (int i = 0; i < NNODE; ++i) tot[NZU + i] = ntot[i][threadIdx.x];
    }
  } else {
    const RowF64<ND>* tab = (const RowF64<ND>*)tabv;
    const RowGradF64* gt = (const RowGradF64*)gtabv;
    const RowCal64* cw = (const RowCal64*)calwv;
    const double* ct = (const double*)caltv;
    if (k0 < k1) {
      RowF64<ND> cur = load_row_f64<ND>(tab, (int)k0);
      RowCal64 cwc;
      if constexpr (GRAD) cwc = cw[k0];
      double tc = ct[k0];
      for (int k = (int)k0; k < (int)k1; ++k) {
        const RowF64<ND> nxt = load_row_f64<ND>(tab, k + 1);
        RowCal64 cwn;
        if constexpr (GRAD) cwn = cw[k + 1];
        const double tn = ct[k + 1];
        cal_bin<ND, GRAD, double>(cur, cwc, tc, gt, k, a, T, cr, ci, kA, kP, tbl, tot);
        cur = nxt;
        if constexpr (GRAD) cwc = cwn;
        tc = tn;
      }
    }
  }
#pragma unroll
  for (int zz = 0; zz < NZ; ++zz) part[((int64_t)c * NZ + zz) * Bp + p] = tot[zz];
}

// Epilogue, one workgroup per 64 points. The value alone takes one wavefront. The adjoint takes
// four, which first share the gather: the value sums one component at a time and the window
// moments of one detector and kind (amplitude or phase) at a time, each summed in chunk order.
// Chunks come in interval order and an interval's window of four nodes starts at
// clamp(j - 1, 0, n - 4), which never moves back and moves by at most one node, so a node's
// moment is final once the window has moved past it: the task keeps the window in four
// registers and turns each finished node into its gradient at once. The 11 signal-parameter
// derivatives (one dual-number pass each, the first also giving the value) are then dealt to
// the wavefronts in turn.
constexpr int EPC_WAVES = 4;

// With alpha the point's amplitude node values for a detector: r_i = K1_i + (K2 alpha)_i. The
// effective K_det = K_det + 2 alpha.K1 + alpha.K2.alpha = K_det + sum_i alpha_i (2 K1_i + (r_i - K1_i)),
// and the amplitude node gradient takes 2 r_i.
__device__ __forceinline__ double cal_r(const double* __restrict__ K1, const double* __restrict__ K2,
                                        const double* __restrict__ al, int n, int i) {
  double r = K1[i];
  for (int l = 0; l < n; ++l) r += K2[i * n + l] * al[l];
  return r;
}

template <int ND, bool GRAD>
__global__ __launch_bounds__((GRAD ? EPC_WAVES : 1) * WAVE) void k_epilogue_cal(
    EventGeom g, const EventConst* __restrict__ ec, const double* __restrict__ kcal, const double* __restrict__ theta,
    int P, int64_t B, int64_t Bp, CalShape sh, bool scaled, const double* __restrict__ part, double* __restrict__ logl,
    double* __restrict__ grad) {
  constexpr int NZ = nz_cal(ND, GRAD), NZU = nz_of(ND, GRAD);
  constexpr int MA = 3 * ND + NBASIS, MB = MA + 4 * ND;
  constexpr int NW = GRAD ? EPC_WAVES : 1;
  __shared__ double acc_s[NZU][WAVE];
  __shared__ double ks_s[ND][WAVE];   // K_det's calibration term per point
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
  const int lane = (int)(threadIdx.x % WAVE);
  const int64_t p = (int64_t)blockIdx.x * WAVE + lane;   // p < Bp: the partial sums have Bp rows
  const int n = sh.nnode, nchunk = sh.nchunk;
  if constexpr (GRAD) {
    for (int z = w; z < NZU; z += NW) {
      double a = 0.0;
#pragma unroll 8
      for (int c = 0; c < nchunk; ++c) a += part[((int64_t)c * NZ + z) * Bp + p];
      acc_s[z][lane] = a;
    }
  } else {
    // one wavefront: every component in one chunk loop, so that their loads for several chunks
    // are in flight together
    double a[NZU];
#pragma unroll
    for (int z = 0; z < NZU; ++z) a[z] = 0.0;
#pragma unroll 8
    for (int c = 0; c < nchunk; ++c) {
#pragma unroll
      for (int z = 0; z < NZU; ++z) a[z] += part[((int64_t)c * NZ + z) * Bp + p];
    }
#pragma unroll
    for (int z = 0; z < NZU; ++z) acc_s[z][lane] = a[z];
  }
  const bool live = p < B;
  const double nan = __builtin_nan("");
  const EventConst e = *ec;
  const double uref = scaled ? e.uref : 1.0;
  if constexpr (GRAD) {
    // node gradients: amplitude uref A m_i - 1/2 A^2 |Q_det|^2 2 r_i, phase -uref A m_i
    int t = w - NZU % NW;
    if (t < 0) t += NW;
    if (t < 2 * ND) {
      const int64_t pc = live ? p : B - 1;
      double th[NPARAM];
#pragma unroll
      for (int i = 0; i < NPARAM; ++i) th[i] = theta[pc * P + i];
      PointModel<double> pm;
      point_model<double, ND>(th, g, pm);
      for (; t < 2 * ND; t += NW) {
        const int d = t >> 1, kind = t & 1;
        const double* al = theta + pc * P + NPARAM + 2 * n * d;
        const double* K1 = kcal + (int64_t)d * (n + n * n);
        const double* K2 = K1 + n;
        double hh = 0.0;   // A^2 |Q_det|^2 (selected with constant indices: pm stays in registers)
#pragma unroll
        for (int dd = 0; dd < ND; ++dd)
          if (dd == d) hh = pm.amp * pm.amp * (pm.qr[dd] * pm.qr[dd] + pm.qi[dd] * pm.qi[dd]);
        double* out = grad + pc * P + NPARAM + 2 * n * d + (kind ? n : 0);
        const int base = (kind ? MB : MA) + 4 * d;
        double ks = 0.0;   // the amplitude task also sums K_det's calibration term
        auto finish = [&](int i, double m) {
          double x;
          if (kind) {
            x = -uref * pm.amp * m;
          } else {
            const double r = cal_r(K1, K2, al, n, i);
            ks += al[i] * (2.0 * K1[i] + (r - K1[i]));
            x = uref * pm.amp * m - 0.5 * hh * (2.0 * r);
          }
          if (live) out[i] = pm.valid ? x : nan;
        };
        double win[4] = {0.0, 0.0, 0.0, 0.0};
        int wb = 0;   // the window holds nodes wb .. wb + 3
        for (int c = 0; c < nchunk; ++c) {
          const int j0 = sh.j0[sh.cj[c]];
          for (; wb < j0; ++wb) {
            finish(wb, win[0]);
            win[0] = win[1];
            win[1] = win[2];
            win[2] = win[3];
            win[3] = 0.0;
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) win[i] += part[((int64_t)c * NZ + base + i) * Bp + p];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (wb + i < n) finish(wb + i, win[i]);
        for (int i = wb + 4; i < n; ++i) finish(i, 0.0);
        if (!kind) ks_s[d][lane] = ks;
      }
    }
  } else {
    const int64_t pc = live ? p : B - 1;
    for (int d = 0; d < ND; ++d) {
      const double* al = theta + pc * P + NPARAM + 2 * n * d;
      const double* K1 = kcal + (int64_t)d * (n + n * n);
      const double* K2 = K1 + n;
      double ks = 0.0;
      for (int i = 0; i < n; ++i) ks += al[i] * (2.0 * K1[i] + (cal_r(K1, K2, al, n, i) - K1[i]));
      ks_s[d][lane] = ks;
    }
  }
  __syncthreads();
  if (!live) return;
  double acc[NZU];
#pragma unroll
  for (int z = 0; z < NZU; ++z) acc[z] = acc_s[z][lane];
  if (scaled) apply_gain<ND>(e, acc);
  double th[NPARAM];
#pragma unroll
  for (int i = 0; i < NPARAM; ++i) th[i] = theta[p * P + i];
  EventConst ek = e;
#pragma unroll
  for (int d = 0; d < ND; ++d) ek.K[d] = e.K[d] + ks_s[d][lane];
  bool valid;
  if constexpr (!GRAD) {
    const double v = epilogue_value<ND, NZU>(acc, th, g, ek, uref, valid);
    logl[p] = valid ? v : nan;
  } else {
#pragma unroll 1
    for (int j = w; j < NPARAM; j += NW) {
      double value;
      const double gj = epilogue_gradient_pass<ND>(acc, th, g, ek, uref, j, valid, value);
      grad[p * P + j] = valid ? gj : nan;
      if (j == 0) logl[p] = valid ? value : nan;
    }
  }
}

template <int ND>
static hipError_t cal_nd(bool mixed, bool grad, const EventGeom& g, const EventConst* ec, const double* kcal,
                         const void* tab, const void* gtab, const void* calw, const void* calt, const double* calB,
                         const double* theta, int P, int64_t B, int64_t Bp, const CalShape& sh, double* coef,
                         double* calc, double* part, double* logl, double* gradout, hipStream_t s) {
  const int ncal = 2 * sh.nnode * ND;
  if (Bp % WAVE != 0 || B < 1 || B > Bp) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_setup_cal<ND>, dim3((unsigned)(Bp / WAVE)), dim3(2 * WAVE), 0, s, g, ec, mixed, theta, P, ncal,
                     B, Bp, coef, calc);
  const dim3 grid((unsigned)(sh.gper * NXCD)), block(BLOCK);
#define GWL_CB(MX, GR) \
  hipLaunchKernelGGL((k_bins_cal<ND, MX, GR>), grid, block, 0, s, tab, gtab, calw, calt, calB, (const double*)coef, \
                     (const double*)calc, B, Bp, sh, part)
  if (mixed) {
    if (grad) GWL_CB(true, true); else GWL_CB(true, false);
  } else {
    if (grad) GWL_CB(false, true); else GWL_CB(false, false);
  }
#undef GWL_CB
  const dim3 egrid((unsigned)((B + WAVE - 1) / WAVE));
  if (grad)
    hipLaunchKernelGGL((k_epilogue_cal<ND, true>), egrid, dim3(EPC_WAVES * WAVE), 0, s, g, ec, kcal, theta, P, B, Bp,
                       sh, mixed, (const double*)part, logl, gradout);
  else
    hipLaunchKernelGGL((k_epilogue_cal<ND, false>), egrid, dim3(WAVE), 0, s, g, ec, kcal, theta, P, B, Bp, sh, mixed,
                       (const double*)part, logl, gradout);
  return hipGetLastError();
}

hipError_t launch_cal(int nd, bool mixed, bool grad, const EventGeom& g, const EventConst* ec, const double* kcal,
                      const void* tab, const void* gtab, const void* calw, const void* calt, const double* calB,
                      const double* theta, int P, int64_t B, int64_t Bp, const CalShape& sh, double* coef,
                      double* calc, double* part, double* logl, double* gradout, hipStream_t s) {
  switch (nd) {
#define GWL_CN(N)                                                                                                   \
  case N:                                                                                                           \
    return cal_nd<N>(mixed, grad, g, ec, kcal, tab, gtab, calw, calt, calB, theta, P, B, Bp, sh, coef, calc, part, \
                     logl, gradout, s);
    GWL_CN(1)
    GWL_CN(2)
    GWL_CN(3)
    GWL_CN(4)
#undef GWL_CN
  }
  return hipErrorInvalidValue;
}

}  // namespace gwl
