// The bin loop: for every (point, detector, frequency bin) evaluate the post-Newtonian phase,
// shift it by the detector's arrival time, reduce it modulo one cycle, form the phasor and
// multiply-accumulate it against the event's whitened data (the sum over bins j of Eq. 2).
//
// Mapping to CDNA: one lane per parameter point, one wavefront per 64 points, and all lanes
// of a wavefront walk the same bins in lock-step. Every per-bin quantity (frequency basis,
// whitened data) is therefore wave-uniform and arrives through scalar loads into SGPRs,
// while the per-point coefficients live in VGPRs for the whole chunk. There is no cross-lane
// reduction: each lane owns its point's sums. Bins are split into chunks only to give the
// chip enough wavefronts; each chunk writes one partial per point, summed in chunk order by
// the epilogue.
//
// Mixed precision: float64 for the phase polynomial, the f T_det term and the reduction to
// [0, 1) cycles (v_fract_f64); float32 for the phasor (hardware sin/cos, which take cycles)
// and the complex multiply-accumulate. The float32 sums run over blocks of NB bins and are
// then added into float64 accumulators (cascaded summation), so float32 rounding never acts
// on more than NB terms at once.
#include <hip/hip_runtime.h>

#include "gwl_common.h"
#include "gwl_device.h"
#include "gwl_launch.h"

namespace gwl {

constexpr int NB = 8;  // bins per float32 block before the float64 flush

LoopShape make_shape(int64_t B, int64_t M, int nchunk) {
  LoopShape s;
  s.npg = (int)((B + WAVE - 1) / WAVE);
  if (nchunk < 1) nchunk = 1;
  if (nchunk > M) nchunk = (int)M;
  s.chunk = (int)((M + nchunk - 1) / nchunk);
  s.nchunk = (int)((M + s.chunk - 1) / s.chunk);
  s.nbpg = (s.npg + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
  s.items = s.nchunk * s.nbpg;
  s.gper = (s.items + NXCD - 1) / NXCD;
  return s;
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

// Decode the workgroup's (chunk, point group) and the lane's point; false if idle.
__device__ __forceinline__ bool locate(const LoopShape& sh, int64_t M, int& c, int& k0, int& k1, int& pg) {
  const int bid = blockIdx.x;
  const int item = (bid % NXCD) * sh.gper + bid / NXCD;  // dies take contiguous item ranges
  if (item >= sh.items) return false;
  c = item / sh.nbpg;
  pg = (item - c * sh.nbpg) * WAVES_PER_BLOCK + (int)(threadIdx.x / WAVE);
  if (pg >= sh.npg) return false;
  k0 = c * sh.chunk;
  k1 = (int)((int64_t)k0 + sh.chunk < M ? k0 + sh.chunk : M);
  return true;
}

// ----------------------------------------------------------------------------------------------
// Mixed precision
// ----------------------------------------------------------------------------------------------
template <int ND, bool GRAD>
struct MixedAcc {
  static constexpr int NZ = nz_of(ND, GRAD);
  float blk[NZ];
  double tot[NZ];
};

template <int ND, bool GRAD>
__device__ __forceinline__ void mixed_bin(const RowMixed<ND>& r, const RowGradF32* __restrict__ gt, int k,
                                          const double (&a)[NBASIS], const double (&T)[ND], const float (&qr)[ND],
                                          const float (&qi)[ND], float (&z)[nz_of(ND, GRAD)]) {
  const double psi = phase_poly(a, r.x, r.w, r.w2, r.lnf);
  float yr = 0.0f, yi = 0.0f;
  float fk = 0.0f;
  if (GRAD) fk = gt[k].f;
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
      z[2 * ND + 2 * d] = fmaf(fk, wr, z[2 * ND + 2 * d]);
      z[2 * ND + 2 * d + 1] = fmaf(fk, wi, z[2 * ND + 2 * d + 1]);
      yr = fmaf(qr[d], wr, fmaf(-qi[d], wi, yr));
      yi = fmaf(qr[d], wi, fmaf(qi[d], wr, yi));
    }
  }
  if (GRAD) {
    const RowGradF32 g = gt[k];
#pragma unroll
    for (int m = 0; m < NBASIS; ++m) {
      z[4 * ND + 2 * m] = fmaf(g.g[m], yr, z[4 * ND + 2 * m]);
      z[4 * ND + 2 * m + 1] = fmaf(g.g[m], yi, z[4 * ND + 2 * m + 1]);
    }
  }
}

template <int ND, bool GRAD>
__global__ __launch_bounds__(BLOCK) void k_bins_mixed(const RowMixed<ND>* __restrict__ tab,
                                                      const RowGradF32* __restrict__ gtab,
                                                      const double* __restrict__ coef, int64_t B, int64_t Bp, int64_t M,
                                                      LoopShape sh, double* __restrict__ part) {
  constexpr int NZ = nz_of(ND, GRAD);
  int c, k0, k1, pg;
  if (!locate(sh, M, c, k0, k1, pg)) return;
  const int64_t p = (int64_t)pg * WAVE + (threadIdx.x % WAVE);
  const int64_t pc = p < B ? p : B - 1;
  double a[NBASIS], T[ND];
  float qr[ND], qi[ND];
#pragma unroll
  for (int m = 0; m < NBASIS; ++m) a[m] = coef[(CO_A + m) * Bp + pc];
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    T[d] = coef[(CO_T + d) * Bp + pc];
    qr[d] = GRAD ? (float)coef[(CO_QR + d) * Bp + pc] : 0.0f;
    qi[d] = GRAD ? (float)coef[(CO_QI + d) * Bp + pc] : 0.0f;
  }
  double tot[NZ];
#pragma unroll
  for (int z = 0; z < NZ; ++z) tot[z] = 0.0;
  int k = k0;
  for (; k + NB <= k1; k += NB) {
    float z[NZ];
#pragma unroll
    for (int j = 0; j < NZ; ++j) z[j] = 0.0f;
#pragma unroll 2
    for (int j = 0; j < NB; ++j) mixed_bin<ND, GRAD>(tab[k + j], gtab, k + j, a, T, qr, qi, z);
#pragma unroll
    for (int j = 0; j < NZ; ++j) tot[j] += (double)z[j];
  }
  if (k < k1) {
    float z[NZ];
#pragma unroll
    for (int j = 0; j < NZ; ++j) z[j] = 0.0f;
    for (; k < k1; ++k) mixed_bin<ND, GRAD>(tab[k], gtab, k, a, T, qr, qi, z);
#pragma unroll
    for (int j = 0; j < NZ; ++j) tot[j] += (double)z[j];
  }
#pragma unroll
  for (int z = 0; z < NZ; ++z) part[((int64_t)c * NZ + z) * Bp + p] = tot[z];
}

// ----------------------------------------------------------------------------------------------
// Float64
// ----------------------------------------------------------------------------------------------
template <int ND, bool GRAD>
__device__ __forceinline__ void f64_bin(const RowF64<ND>& r, const RowGradF64* __restrict__ gt, int k,
                                        const double (&a)[NBASIS], const double (&T)[ND], const double (&qr)[ND],
                                        const double (&qi)[ND], double (&z)[nz_of(ND, GRAD)]) {
  const double psi = phase_poly(a, r.x, r.w, r.w2, r.lnf);
  double yr = 0.0, yi = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    double sn, cs;
    sincos_cycles_f64(fma(r.f, T[d], psi), sn, cs);
    const double ur = r.u[2 * d], ui = r.u[2 * d + 1];
    if (!GRAD) {
      z[2 * d] = fma(ur, cs, fma(ui, sn, z[2 * d]));
      z[2 * d + 1] = fma(ui, cs, fma(-ur, sn, z[2 * d + 1]));
    } else {
      const double wr = fma(ur, cs, ui * sn);
      const double wi = fma(ui, cs, -(ur * sn));
      z[2 * d] += wr;
      z[2 * d + 1] += wi;
      z[2 * ND + 2 * d] = fma(r.f, wr, z[2 * ND + 2 * d]);
      z[2 * ND + 2 * d + 1] = fma(r.f, wi, z[2 * ND + 2 * d + 1]);
      yr = fma(qr[d], wr, fma(-qi[d], wi, yr));
      yi = fma(qr[d], wi, fma(qi[d], wr, yi));
    }
  }
  if (GRAD) {
    const RowGradF64 g = gt[k];
    const double gm[NBASIS] = {r.w, r.w2, g.g2, g.g3, r.lnf, r.x, g.g6, g.g7};
#pragma unroll
    for (int m = 0; m < NBASIS; ++m) {
      z[4 * ND + 2 * m] = fma(gm[m], yr, z[4 * ND + 2 * m]);
      z[4 * ND + 2 * m + 1] = fma(gm[m], yi, z[4 * ND + 2 * m + 1]);
    }
  }
}

template <int ND, bool GRAD>
__global__ __launch_bounds__(BLOCK) void k_bins_f64(const RowF64<ND>* __restrict__ tab,
                                                    const RowGradF64* __restrict__ gtab,
                                                    const double* __restrict__ coef, int64_t B, int64_t Bp, int64_t M,
                                                    LoopShape sh, double* __restrict__ part) {
  constexpr int NZ = nz_of(ND, GRAD);
  int c, k0, k1, pg;
  if (!locate(sh, M, c, k0, k1, pg)) return;
  const int64_t p = (int64_t)pg * WAVE + (threadIdx.x % WAVE);
  const int64_t pc = p < B ? p : B - 1;
  double a[NBASIS], T[ND], qr[ND], qi[ND];
#pragma unroll
  for (int m = 0; m < NBASIS; ++m) a[m] = coef[(CO_A + m) * Bp + pc];
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    T[d] = coef[(CO_T + d) * Bp + pc];
    qr[d] = GRAD ? coef[(CO_QR + d) * Bp + pc] : 0.0;
    qi[d] = GRAD ? coef[(CO_QI + d) * Bp + pc] : 0.0;
  }
  double z[NZ];
#pragma unroll
  for (int j = 0; j < NZ; ++j) z[j] = 0.0;
#pragma unroll 2
  for (int k = k0; k < k1; ++k) f64_bin<ND, GRAD>(tab[k], gtab, k, a, T, qr, qi, z);
#pragma unroll
  for (int j = 0; j < NZ; ++j) part[((int64_t)c * NZ + j) * Bp + p] = z[j];
}

template <int ND>
static hipError_t bins_nd(bool mixed, bool grad, const void* tab, const void* gtab, const void* gtab64,
                          const double* coef, int64_t B, int64_t Bp, int64_t M, const LoopShape& sh, double* part,
                          hipStream_t s) {
  const dim3 grid((unsigned)(sh.gper * NXCD)), block(BLOCK);
  if (mixed) {
    if (grad)
      hipLaunchKernelGGL((k_bins_mixed<ND, true>), grid, block, 0, s, (const RowMixed<ND>*)tab,
                         (const RowGradF32*)gtab, coef, B, Bp, M, sh, part);
    else
      hipLaunchKernelGGL((k_bins_mixed<ND, false>), grid, block, 0, s, (const RowMixed<ND>*)tab,
                         (const RowGradF32*)gtab, coef, B, Bp, M, sh, part);
  } else {
    if (grad)
      hipLaunchKernelGGL((k_bins_f64<ND, true>), grid, block, 0, s, (const RowF64<ND>*)tab,
                         (const RowGradF64*)gtab64, coef, B, Bp, M, sh, part);
    else
      hipLaunchKernelGGL((k_bins_f64<ND, false>), grid, block, 0, s, (const RowF64<ND>*)tab,
                         (const RowGradF64*)gtab64, coef, B, Bp, M, sh, part);
  }
  return hipGetLastError();
}

hipError_t launch_bins(int nd, bool mixed, bool grad, const void* tab, const void* gtab, const void* gtab64,
                       const double* coef, int64_t B, int64_t Bp, int64_t M, const LoopShape& sh, double* part,
                       hipStream_t s) {
  switch (nd) {
    case 1: return bins_nd<1>(mixed, grad, tab, gtab, gtab64, coef, B, Bp, M, sh, part, s);
    case 2: return bins_nd<2>(mixed, grad, tab, gtab, gtab64, coef, B, Bp, M, sh, part, s);
    case 3: return bins_nd<3>(mixed, grad, tab, gtab, gtab64, coef, B, Bp, M, sh, part, s);
    case 4: return bins_nd<4>(mixed, grad, tab, gtab, gtab64, coef, B, Bp, M, sh, part, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace gwl
