// The bin loop: for every (point, detector, frequency bin) evaluate the post-Newtonian phase,
// shift it by the detector's arrival time, reduce it modulo one cycle, form the phasor and
// multiply-accumulate it against the event's whitened data (the sum over bins j of Eq. 2), then
// reduce over bins and, for the value, apply the float64 epilogue in the same kernel.
//
// Mapping to CDNA: one lane per parameter point, one wavefront per 64 points, and all lanes
// of a wavefront walk the same bins in lock-step. Every per-bin quantity (frequency basis,
// whitened data) is therefore wave-uniform and arrives through scalar loads into SGPRs,
// while the per-point coefficients live in VGPRs for the whole chunk.
//
// A workgroup holds W wavefronts that share one group of 64 points and take W consecutive
// chunks of the bins; G workgroups cover a point group's bins. The W partial sums of a
// workgroup are added in LDS in wavefront order; with G = 1 the first wavefront then applies
// the epilogue directly, so neither partial sums nor a second kernel are needed. With G > 1 each
// workgroup writes its partial sums and the last one to finish (a counter per point group, after
// an agent-scope release/acquire) adds the G of them in workgroup order: every sum is taken in a
// fixed order, so results are bitwise reproducible for a given shape. The gradient's epilogue
// (eleven forward-mode passes through the point model, over 250 registers) runs as its own kernel
// on the G partial sums.
//
// The per-point set-up (phase coefficients, shifts, projection factors) either comes from the
// set-up kernel's rows or is computed here and handed to every wavefront through LDS
// (sh.setup): the intrinsic half on the first wavefront, the extrinsic half on the second. That
// saves a launch for small calls, at the price of the set-up's registers in this kernel.
//
// Mixed precision: float64 for the phase polynomial, the f T_det term and the reduction to
// [0, 1) cycles (v_fract_f64); float32 for the phasor (hardware sin/cos, which take cycles)
// and the complex multiply-accumulate. The float32 sums run over blocks of NB bins and are
// then added into float64 accumulators (cascaded summation), so float32 rounding never acts
// on more than NB terms at once. The adjoint's moments are accumulated in float64.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "gwl_bins.h"
#include "gwl_common.h"
#include "gwl_device.h"
#include "gwl_epilogue.h"
#include "gwl_launch.h"

namespace gwl {

LoopShape make_shape(int64_t B, int64_t M, int W, int G, int setup, int sepepi) {
  LoopShape s;
  s.npg = (int)((B + WAVE - 1) / WAVE);
  if (W < 1) W = 1;
  if (W > MAX_EVAL_WAVES) W = MAX_EVAL_WAVES;
  if (G < 1) G = 1;
  // no more chunks than bins
  const int64_t gmax = (M + W - 1) / W;
  if (G > gmax) G = (int)(gmax > 0 ? gmax : 1);
  s.W = W;
  s.G = G;
  s.nchunk = W * G;
  s.chunk = (int)((M + s.nchunk - 1) / s.nchunk);
  s.items = s.npg * G;
  // how the dies share the work: by point groups (each die reads its points' set-up rows, 30
  // doubles a point, and the whole per-bin table) when the rows outweigh the table (about 8
  // doubles a bin), else by ranges of chunk groups (each die reads its part of the table and
  // every point's rows): c1 (65,536 points, 16,225 bins) goes by point groups, the 128 s event
  // (4,096 points, 259,585 bins) by chunk groups; so do batches of fewer than 8 point groups,
  // whose workgroups would otherwise not reach every die
  s.pgmaj = (s.npg >= NXCD && (int64_t)s.npg * WAVE * NCOEF >= M * 8) ? 1 : 0;
  s.gper = s.pgmaj ? (s.npg + NXCD - 1) / NXCD * G : (s.items + NXCD - 1) / NXCD;
  s.setup = setup ? 1 : 0;
  s.sepepi = (sepepi && G > 1) ? 1 : 0;
  return s;
}

// Dynamic LDS of a workgroup, in doubles: the set-up rows (NCOEF x 64) when the set-up runs here,
// then the float64 phasor table (PH_TBL double2), which the cross-wavefront reduction reuses, or,
// for mixed precision, the reduction buffer alone ((W - 1) x RED_Z x 64).
constexpr int RED_Z = 4;  // sums reduced per LDS pass
size_t eval_lds_doubles(bool mixed, const LoopShape& sh) {
  const size_t rows = sh.setup ? (size_t)NCOEF * WAVE : 0;
  const size_t red = (size_t)(sh.W - 1) * RED_Z * WAVE;
  const size_t tbl = mixed ? 0 : (size_t)2 * PH_TBL;
  return rows + (red > tbl ? red : tbl);
}

// logL of one point from its reduced sums and set-up values (A, c0, Q_det):
//   sum_det [ uref Re(A E Q_det Z_det) - 1/2 A^2 |Q_det|^2 K_det ],  E = exp(-2 pi i c0).
// The fused multiply-adds are spelled out, so that the evaluation kernel and the separate value
// epilogue round alike.
template <int ND, int NZ>
__device__ inline double value_from_rows(const double (&acc)[NZ], double amp, double c0f, const double (&qr)[ND],
                                         const double (&qi)[ND], const EventConst& ec, double uref) {
  const double c0 = c0f - rint(c0f);
  double es, ecs;
  sincos_cycles_f64(c0, es, ecs);
  const double er = ecs, ei = -es;
  double out = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const double xr = amp * fma(er, qr[d], -(ei * qi[d]));
    const double xi = amp * fma(er, qi[d], ei * qr[d]);
    const double dh = uref * fma(xr, acc[2 * d], -(xi * acc[2 * d + 1]));
    const double hh = amp * amp * fma(qr[d], qr[d], qi[d] * qi[d]) * ec.K[d];
    out += fma(-0.5, hh, dh);
  }
  return out;
}

template <int ND, bool MIXED>
using TabRow = typename std::conditional<MIXED, RowMixed<ND>, RowF64<ND>>::type;

// The tables are `const __restrict__` kernel arguments, so the compiler reads their wave-uniform
// rows with scalar loads.
// Wavefronts per SIMD that the register budget must allow (as the bin loop alone needs): the
// reduction and epilogue after the loop would otherwise let the compiler take registers that
// cost a wavefront per SIMD. The in-kernel set-up needs more and is not bounded.
template <int ND, bool MIXED, bool GRAD, bool SETUP, bool CUT, bool ROT>
constexpr int eval_waves_per_eu() {
  return (SETUP || CUT) ? 1 : (ND > 3 ? 1 : (MIXED ? (GRAD ? 5 : 8) : (GRAD ? 4 : 5)));
}

// CUT: the optional ISCO cut-off; every lane keeps only the bins at or below its point's ISCO
// frequency (isco_bins over fgrid), the wavefront stops at the last bin any of its lanes keeps,
// and <h|h> takes the kept bins' share of K_det from the per-detector running sums kcum
// [ND][M + 1]. ROT (float64, uniform grids): the detectors after the first take their phasors by
// rotation from the first's (bin_loop_f64_rot).
template <int ND, bool MIXED, bool GRAD, bool SETUP, bool CUT, bool ROT>
__global__ __launch_bounds__(WAVE * MAX_EVAL_WAVES)
__attribute__((amdgpu_waves_per_eu(eval_waves_per_eu<ND, MIXED, GRAD, SETUP, CUT, ROT>()))) void k_eval(
    const TabRow<ND, MIXED>* __restrict__ tab, const RowGradF64* __restrict__ gtab, const double* __restrict__ theta,
    EventGeom geo, const EventConst* __restrict__ ec, double* __restrict__ coef, int64_t B, int64_t Bp, int64_t M,
    LoopShape sh, double* __restrict__ part, unsigned int* __restrict__ cnt, double* __restrict__ logl,
    const double* __restrict__ fgrid, const double* __restrict__ kcum, const int64_t* __restrict__ live) {
  constexpr int NZ = nz_of(ND, GRAD);
  extern __shared__ double lds[];
  double* rows_s = lds;                                        // [NCOEF][64] when SETUP
  double* tail = lds + (SETUP ? NCOEF * WAVE : 0);             // table, then the reduction buffer
  double2* tbl = reinterpret_cast<double2*>(tail);

  // sh.pgmaj: each die takes whole point groups, all G workgroups of each (a point group's set-up
  // rows are read by one die only): a contiguous range of point-group-major items (balanced to
  // one item), or, for a live-length call, the point groups in turn (pg = xcd mod NXCD), so that a
  // partly live batch stays spread over the dies. Else each die takes a contiguous range of items,
  // chunk group major (a die reads its part of the per-bin table only).
  const int bid = blockIdx.x;
  const int xcd = bid % NXCD, loc = bid / NXCD;
  int g, pg;
  if (sh.pgmaj && live) {
    const int pgl = loc / sh.G;
    g = loc - pgl * sh.G;
    pg = pgl * NXCD + xcd;
    if (pg >= sh.npg) return;                                  // whole workgroup
  } else if (sh.pgmaj) {
    const int per = (sh.items + NXCD - 1) / NXCD;
    const int item = xcd * per + loc;
    if (loc >= per || item >= sh.items) return;                // whole workgroup
    pg = item / sh.G;
    g = item - pg * sh.G;
  } else {
    const int item = xcd * sh.gper + loc;
    if (item >= sh.items) return;                              // whole workgroup
    g = item / sh.npg;
    pg = item - g * sh.npg;
  }
  // live: only the first *live points are evaluated (a batch whose length the device decides)
  if (live) {
    const int64_t nl = *live;
    B = nl < B ? nl : B;
  }
  if ((int64_t)pg * WAVE >= B) return;                         // whole workgroup
  // the wavefront index is uniform across the wavefront; readfirstlane tells the compiler so, which
  // keeps the chunk's bin range, and with it every table row, in scalar registers
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
  const int lane = (int)(threadIdx.x % WAVE);
  const int64_t p = (int64_t)pg * WAVE + lane;
  const int64_t pc = p < B ? p : B - 1;                        // padding lanes repeat the last point
  const int64_t c = (int64_t)g * sh.W + w;
  const int64_t k0l = c * sh.chunk;
  const int k0 = (int)(k0l < M ? k0l : M);
  int k1 = (int)(k0 + sh.chunk < M ? k0 + sh.chunk : M);
  int kc = 0;
  if constexpr (CUT) {
    kc = isco_bins(theta[pc * NPARAM], theta[pc * NPARAM + 1], fgrid, M, *ec);
    const int kmax = wave_max(kc);
    k1 = k1 < kmax ? k1 : (kmax > k0 ? kmax : k0);
  }

  // the float64 phasor table; with the in-kernel set-up and three or more wavefronts, the ones
  // that do not run a half of the set-up fill it meanwhile
  if constexpr (!MIXED) {
    if (!SETUP || sh.W < 3) fill_phasor_table(tbl);
    else if (w >= 2) fill_phasor_table(tbl, 2 * WAVE);
  }
  // in-kernel set-up: the intrinsic half on wavefront 0, the extrinsic half on wavefront 1 (on
  // wavefront 0 too when the workgroup has one)
  if constexpr (SETUP) {
    const int wx = sh.W > 1 ? 1 : 0;
    if (w == 0 || w == wx) {
      double th[NPARAM];
#pragma unroll
      for (int i = 0; i < NPARAM; ++i) th[i] = theta[pc * NPARAM + i];
      if (w == 0) setup_lds_intrinsic(th, ec, rows_s, lane);
      if (w == wx) setup_lds_extrinsic<ND>(th, geo, ec, rows_s, lane);
    }
  }
  if (SETUP || !MIXED) __syncthreads();

  double a[NBASIS], T[ND];
  double tot[NZ];
  bool in_range = true;
  if constexpr (SETUP) {
#pragma unroll
    for (int m = 0; m < NBASIS; ++m) a[m] = rows_s[(CO_A + m) * WAVE + lane];
#pragma unroll
    for (int d = 0; d < ND; ++d) T[d] = rows_s[(CO_T + d) * WAVE + lane];
    // a point whose phase could leave the supported range gets NaN sums (and value)
    in_range = rows_in_range<ND>(a, T, ec);
    if (!in_range) a[0] = __builtin_nan("");
  }
  // c_det = E G Q_det from the set-up rows (the adjoint's projection factors)
  auto lds_factors = [&](double (&crd)[ND], double (&cid)[ND]) {
    double egr, egi;
    phase_gain(rows_s[CO_C0 * WAVE + lane], (MIXED && ec) ? ec->gain_r : 1.0, (MIXED && ec) ? ec->gain_i : 0.0, egr,
               egi);
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      adjoint_factor(egr, egi, rows_s[(CO_QR + d) * WAVE + lane], rows_s[(CO_QI + d) * WAVE + lane], crd[d], cid[d]);
    }
  };
  if constexpr (MIXED) {
    float cr[ND], ci[ND];
    if constexpr (SETUP) {
#pragma unroll
      for (int d = 0; d < ND; ++d) cr[d] = ci[d] = 0.0f;
      if constexpr (GRAD) {
        double crd[ND], cid[ND];
        lds_factors(crd, cid);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          cr[d] = (float)crd[d];
          ci[d] = (float)cid[d];
        }
      }
    } else {
      load_coef<ND, float>(coef, Bp, pc, GRAD, a, T, cr, ci);
    }
    bin_loop_mixed<ND, GRAD, const TabRow<ND, MIXED>*, const RowGradF64*, CUT>(tab, gtab, k0, k1, a, T, cr, ci, tot,
                                                                                kc);
  } else {
    double cr[ND], ci[ND];
    if constexpr (SETUP) {
#pragma unroll
      for (int d = 0; d < ND; ++d) cr[d] = ci[d] = 0.0;
      if constexpr (GRAD) lds_factors(cr, ci);
    } else {
      load_coef<ND, double>(coef, Bp, pc, GRAD, a, T, cr, ci);
    }
    to_table_units<ND>(a, T);
    if constexpr (ROT)
      bin_loop_f64_rot<ND, GRAD, const TabRow<ND, MIXED>*, const RowGradF64*>(tab, gtab, k0, k1, a, T, cr, ci, tbl,
                                                                              ec->grid_df, tot);
    else
      bin_loop_f64<ND, GRAD, const TabRow<ND, MIXED>*, const RowGradF64*, CUT>(tab, gtab, k0, k1, a, T, cr, ci, tbl,
                                                                                tot, kc);
  }

  // the W chunk sums of this workgroup, added in wavefront order by the first wavefront; the
  // buffer reuses the phasor table's LDS, so every wavefront must be past its bin loop first
  double* red = tail;
  if (sh.W > 1) {
#pragma unroll
    for (int z0 = 0; z0 < NZ; z0 += RED_Z) {
      __syncthreads();
      if (w > 0) {
#pragma unroll
        for (int zz = 0; zz < RED_Z; ++zz)
          if (z0 + zz < NZ) red[((w - 1) * RED_Z + zz) * WAVE + lane] = tot[z0 + zz];
      }
      __syncthreads();
      if (w == 0) {
        for (int v = 1; v < sh.W; ++v) {
#pragma unroll
          for (int zz = 0; zz < RED_Z; ++zz)
            if (z0 + zz < NZ) tot[z0 + zz] += red[((v - 1) * RED_Z + zz) * WAVE + lane];
        }
      }
    }
  }
  if (w != 0) return;

  if (GRAD || sh.G > 1) {
#pragma unroll
    for (int z = 0; z < NZ; ++z) part[((int64_t)g * NZ + z) * Bp + p] = tot[z];
  }
  if constexpr (!GRAD) {
    if (sh.G > 1) {
      if (sh.sepepi) {        // k_value_epilogue adds them
        if constexpr (SETUP) {
          // with the set-up in this kernel, the first workgroup of the point group leaves the
          // rows the epilogue needs (A, c0, Q_det; as the set-up kernel writes them, A NaN for
          // a point outside the phase range)
          if (g == 0) {
            coef[CO_AMP * Bp + p] = in_range ? rows_s[CO_AMP * WAVE + lane] : __builtin_nan("");
            coef[CO_C0 * Bp + p] = rows_s[CO_C0 * WAVE + lane];
#pragma unroll
            for (int d = 0; d < ND; ++d) {
              coef[(CO_QR + d) * Bp + p] = rows_s[(CO_QR + d) * WAVE + lane];
              coef[(CO_QI + d) * Bp + p] = rows_s[(CO_QI + d) * WAVE + lane];
            }
          }
        }
        return;
      }
      // the last of the point group's G workgroups adds the G partial sums in workgroup order
      __threadfence();
      const unsigned int prev = atomicAdd(&cnt[pg], lane == 0 ? 1u : 0u);
      const unsigned int done = __builtin_amdgcn_readfirstlane(prev);
      if (done + 1u != (unsigned int)sh.G) return;
      __threadfence();
#pragma unroll
      for (int z = 0; z < NZ; ++z) tot[z] = 0.0;
#pragma unroll 8
      for (int gg = 0; gg < sh.G; ++gg) {
#pragma unroll
        for (int z = 0; z < NZ; ++z) tot[z] += part[((int64_t)gg * NZ + z) * Bp + p];
      }
      if (lane == 0) cnt[pg] = 0u;                             // ready for the next call
    }
    EventConst e = *ec;
    if constexpr (CUT) {
#pragma unroll
      for (int d = 0; d < ND; ++d) e.K[d] = kcum[(int64_t)d * (M + 1) + kc];
    }
    if (MIXED) apply_gain<ND>(e, tot);
    double qr[ND], qi[ND], amp, c0f;
    if constexpr (SETUP) {
      amp = in_range ? rows_s[CO_AMP * WAVE + lane] : __builtin_nan("");
      c0f = rows_s[CO_C0 * WAVE + lane];
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        qr[d] = rows_s[(CO_QR + d) * WAVE + lane];
        qi[d] = rows_s[(CO_QI + d) * WAVE + lane];
      }
    } else {
      amp = coef[CO_AMP * Bp + pc];
      c0f = coef[CO_C0 * Bp + pc];
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        qr[d] = coef[(CO_QR + d) * Bp + pc];
        qi[d] = coef[(CO_QI + d) * Bp + pc];
      }
    }
    if (p < B) logl[p] = value_from_rows<ND, NZ>(tot, amp, c0f, qr, qi, e, MIXED ? e.uref : 1.0);
  }
}

template <int ND, bool MIXED, bool GRAD>
static hipError_t eval_setup(bool setup, bool cut, bool rot, const void* tab, const RowGradF64* gtab, const double* theta,
                             const EventGeom& geo, const EventConst* ec, double* coef, int64_t B, int64_t Bp,
                             int64_t M, const LoopShape& sh, double* part, unsigned int* cnt, double* logl,
                             const double* fgrid, const double* kcum, const int64_t* live, hipStream_t s) {
  const dim3 grid((unsigned)(sh.gper * NXCD)), block((unsigned)(sh.W * WAVE));
  const size_t lds = eval_lds_doubles(MIXED, sh) * sizeof(double);
  const TabRow<ND, MIXED>* t = (const TabRow<ND, MIXED>*)tab;
#define GWL_EVAL(ST, CU, RO)                                                                                  \
  hipLaunchKernelGGL((k_eval<ND, MIXED, GRAD, ST, CU, RO>), grid, block, lds, s, t, gtab, theta, geo, ec, coef, B, \
                     Bp, M, sh, part, cnt, logl, fgrid, kcum, live)
  if (cut) {
    if (setup) GWL_EVAL(true, true, false); else GWL_EVAL(false, true, false);
  } else if (MIXED || !rot) {
    if (setup) GWL_EVAL(true, false, false); else GWL_EVAL(false, false, false);
  } else {
    if constexpr (!MIXED) {
      if (setup) GWL_EVAL(true, false, true); else GWL_EVAL(false, false, true);
    }
  }
#undef GWL_EVAL
  return hipGetLastError();
}

template <int ND>
static hipError_t eval_nd(bool mixed, bool grad, bool cut, bool rot, const void* tab, const RowGradF64* gtab,
                          const double* theta, const EventGeom& geo, const EventConst* ec, double* coef,
                          int64_t B, int64_t Bp, int64_t M, const LoopShape& sh, double* part, unsigned int* cnt,
                          double* logl, const double* fgrid, const double* kcum, const int64_t* live,
                          hipStream_t s) {
  const bool st = sh.setup != 0;
#define GWL_EV(MX, GR) \
  return eval_setup<ND, MX, GR>(st, cut, rot, tab, gtab, theta, geo, ec, coef, B, Bp, M, sh, part, cnt, logl, fgrid, \
                                kcum, live, s)
  if (mixed) {
    if (grad) GWL_EV(true, true);
    GWL_EV(true, false);
  }
  if (grad) GWL_EV(false, true);
  GWL_EV(false, false);
#undef GWL_EV
}

// The value's epilogue as a kernel of its own (LoopShape::sepepi): one thread per point adds the
// G workgroup sums in workgroup order, as the last-arriving workgroup of k_eval does, and forms
// the value from the set-up rows, so both paths give the same bits.
constexpr int EPI_BLOCK = 256;
template <int ND, bool MIXED, bool CUT>
__global__ __launch_bounds__(EPI_BLOCK) void k_value_epilogue(const EventConst* __restrict__ ec,
                                                              const double* __restrict__ theta,
                                                              const double* __restrict__ coef, int64_t B, int64_t Bp,
                                                              int G, const double* __restrict__ part,
                                                              double* __restrict__ logl, const double* __restrict__ fgrid,
                                                              const double* __restrict__ kcum, int64_t M,
                                                              const int64_t* __restrict__ live) {
  constexpr int NZ = nz_of(ND, false);
  const int64_t p = (int64_t)blockIdx.x * EPI_BLOCK + threadIdx.x;
  if (live) {
    const int64_t nl = *live;
    B = nl < B ? nl : B;
  }
  if (p >= B) return;
  double tot[NZ];
#pragma unroll
  for (int z = 0; z < NZ; ++z) tot[z] = 0.0;
  // workgroup order; unrolled so that several workgroups' loads are in flight before their adds
#pragma unroll 8
  for (int gg = 0; gg < G; ++gg) {
#pragma unroll
    for (int z = 0; z < NZ; ++z) tot[z] += part[((int64_t)gg * NZ + z) * Bp + p];
  }
  EventConst e = *ec;
  if constexpr (CUT) {
    const int kc = isco_bins(theta[p * NPARAM], theta[p * NPARAM + 1], fgrid, M, *ec);
#pragma unroll
    for (int d = 0; d < ND; ++d) e.K[d] = kcum[(int64_t)d * (M + 1) + kc];
  }
  if (MIXED) apply_gain<ND>(e, tot);
  double qr[ND], qi[ND];
  const double amp = coef[CO_AMP * Bp + p], c0f = coef[CO_C0 * Bp + p];
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    qr[d] = coef[(CO_QR + d) * Bp + p];
    qi[d] = coef[(CO_QI + d) * Bp + p];
  }
  logl[p] = value_from_rows<ND, NZ>(tot, amp, c0f, qr, qi, e, MIXED ? e.uref : 1.0);
}

hipError_t launch_value_epilogue(int nd, bool mixed, const EventConst* ec, const double* theta, const double* coef,
                                 int64_t B, int64_t Bp, int G, const double* part, double* logl, const double* fgrid,
                                 const double* kcum, int64_t M, const int64_t* live, hipStream_t s) {
  if (!coef || !part || G < 1) return hipErrorInvalidValue;
  const bool cut = fgrid != nullptr;
  if (cut && !kcum) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((B + EPI_BLOCK - 1) / EPI_BLOCK));
#define GWL_VEPI(N, MX, CU)                                                                                   \
  hipLaunchKernelGGL((k_value_epilogue<N, MX, CU>), grid, dim3(EPI_BLOCK), 0, s, ec, theta, coef, B, Bp, G, \
                     part, logl, fgrid, kcum, M, live)
#define GWL_VEPI_ND(N)                                               \
  case N:                                                            \
    if (mixed) {                                                     \
      if (cut) GWL_VEPI(N, true, true); else GWL_VEPI(N, true, false);    \
    } else {                                                         \
      if (cut) GWL_VEPI(N, false, true); else GWL_VEPI(N, false, false);  \
    }                                                                \
    break;
  switch (nd) {
    GWL_VEPI_ND(1)
    GWL_VEPI_ND(2)
    GWL_VEPI_ND(3)
    GWL_VEPI_ND(4)
    default: return hipErrorInvalidValue;
  }
#undef GWL_VEPI_ND
#undef GWL_VEPI
  return hipGetLastError();
}

hipError_t launch_eval(int nd, bool mixed, bool grad, bool rot, const void* tab, const RowGradF64* gtab, const double* theta,
                       const EventGeom& geo, const EventConst* ec, double* coef, int64_t B, int64_t Bp,
                       int64_t M, const LoopShape& sh, double* part, unsigned int* cnt, double* logl,
                       const double* fgrid, const double* kcum, const int64_t* live, hipStream_t s) {
  if (sh.W < 1 || sh.W > MAX_EVAL_WAVES || sh.G < 1) return hipErrorInvalidValue;
  if ((grad || sh.G > 1) && !part) return hipErrorInvalidValue;
  if (!grad && sh.G > 1 && !sh.sepepi && !cnt) return hipErrorInvalidValue;
  if (!sh.setup && !coef) return hipErrorInvalidValue;
  const bool cut = fgrid != nullptr;
  if (cut && !kcum) return hipErrorInvalidValue;
  switch (nd) {
    case 1: return eval_nd<1>(mixed, grad, cut, rot, tab, gtab, theta, geo, ec, coef, B, Bp, M, sh, part, cnt, logl, fgrid, kcum, live, s);
    case 2: return eval_nd<2>(mixed, grad, cut, rot, tab, gtab, theta, geo, ec, coef, B, Bp, M, sh, part, cnt, logl, fgrid, kcum, live, s);
    case 3: return eval_nd<3>(mixed, grad, cut, rot, tab, gtab, theta, geo, ec, coef, B, Bp, M, sh, part, cnt, logl, fgrid, kcum, live, s);
    case 4: return eval_nd<4>(mixed, grad, cut, rot, tab, gtab, theta, geo, ec, coef, B, Bp, M, sh, part, cnt, logl, fgrid, kcum, live, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace gwl
