// Event preparation (per-bin tables of the factored likelihood) and model strain kernels.
//
// Factoring Eq. 2's inner products for the TaylorF2 model h_det,k = A Q_det f_k^(-7/6)
// exp(-2 pi i Phi_det,k):
//   <d|h>_det = A Re(Q_det E Z_det),  Z_det = sum_k u_k exp(-2 pi i (Phi_det,k - c0)),
//   u_k = 4 df f_k^(-7/6) conj(d_k) / S_k,
//   <h|h>_det = A^2 |Q_det|^2 K_det,  K_det = 4 df sum_k f_k^(-7/3) / S_k,
// so every point-independent per-bin quantity is computed once per event here.
#include <hip/hip_runtime.h>

#include "gwl_common.h"
#include "gwl_device.h"
#include "gwl_launch.h"

namespace gwl {

constexpr int PREP_BLOCK = 256;

int prep_blocks(int64_t M) { return (int)((M + PREP_BLOCK - 1) / PREP_BLOCK); }

// per block: ND K_det terms, max |u|, rejected count, lowest and highest frequency
constexpr int prep_part(int nd) { return nd + 4; }

size_t prep_scratch_doubles(int nd, int64_t M) {
  return (size_t)prep_blocks(M) * prep_part(nd) + (size_t)NGAIN_BLK * 2;
}

// One thread per bin. Writes the float64 row, the adjoint basis rows, and per-block partial
// sums (K_det terms, max |u|, count of rejected inputs, frequency range) reduced in a fixed
// tree order.
template <int ND>
__global__ __launch_bounds__(PREP_BLOCK) void k_prep_bins(const double* __restrict__ data, const double* __restrict__ psd,
                                                          const double* __restrict__ fgrid, int64_t M, double df,
                                                          RowF64<ND>* __restrict__ tab64, RowGradF32* __restrict__ g32,
                                                          RowGradF64* __restrict__ g64, double* __restrict__ blockpart) {
  __shared__ double red[ND + 4][PREP_BLOCK];
  const int64_t k = (int64_t)blockIdx.x * PREP_BLOCK + threadIdx.x;
  double kt[ND], umax = 0.0, bad = 0.0, flo = __builtin_inf(), fhi = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) kt[d] = 0.0;
  if (k < M) {
    const double f = fgrid[k];
    if (!(f > 0.0) || !isfinite(f)) bad += 1.0;
    flo = f;
    fhi = f;
    const double x = cbrt(f);
    const double w2 = 1.0 / f;
    const double w = w2 / (x * x);
    const double lnf = log(f);
    const double f76 = w2 / sqrt(x);   // f^(-7/6)
    const double f73 = w2 * w2 / x;    // f^(-7/3)
    RowF64<ND> row;
    row.f = f; row.x = x; row.w = w; row.w2 = w2; row.lnf = lnf;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const double s = psd[(int64_t)d * M + k];
      const double dr = data[((int64_t)d * M + k) * 2];
      const double di = data[((int64_t)d * M + k) * 2 + 1];
      if (!(s > 0.0) || !isfinite(s) || !isfinite(dr) || !isfinite(di)) bad += 1.0;
      const double sc = 4.0 * df * f76 / s;
      row.u[2 * d] = sc * dr;       // u = 4 df f^-7/6 conj(d) / S
      row.u[2 * d + 1] = -sc * di;
      kt[d] = 4.0 * df * f73 / s;
      umax = fmax(umax, fmax(fabs(row.u[2 * d]), fabs(row.u[2 * d + 1])));
    }
    tab64[k] = row;
    RowGradF32 gr;
    const double g2 = w2 * x, g3 = w2 * x * x, g6 = x * lnf, g7 = x * x;
    gr.g[0] = (float)w; gr.g[1] = (float)w2; gr.g[2] = (float)g2; gr.g[3] = (float)g3;
    gr.g[4] = (float)lnf; gr.g[5] = (float)x; gr.g[6] = (float)g6; gr.g[7] = (float)g7;
    gr.f = (float)f;
    g32[k] = gr;
    RowGradF64 gd;
    gd.g2 = g2; gd.g3 = g3; gd.g6 = g6; gd.g7 = g7;
    g64[k] = gd;
  }
#pragma unroll
  for (int d = 0; d < ND; ++d) red[d][threadIdx.x] = kt[d];
  red[ND][threadIdx.x] = umax;
  red[ND + 1][threadIdx.x] = bad;
  red[ND + 2][threadIdx.x] = flo;
  red[ND + 3][threadIdx.x] = fhi;
  __syncthreads();
  for (int off = PREP_BLOCK / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
#pragma unroll
      for (int d = 0; d < ND; ++d) red[d][threadIdx.x] += red[d][threadIdx.x + off];
      red[ND][threadIdx.x] = fmax(red[ND][threadIdx.x], red[ND][threadIdx.x + off]);
      red[ND + 1][threadIdx.x] += red[ND + 1][threadIdx.x + off];
      red[ND + 2][threadIdx.x] = fmin(red[ND + 2][threadIdx.x], red[ND + 2][threadIdx.x + off]);
      red[ND + 3][threadIdx.x] = fmax(red[ND + 3][threadIdx.x], red[ND + 3][threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x < ND + 4) blockpart[(int64_t)blockIdx.x * prep_part(ND) + threadIdx.x] = red[threadIdx.x][0];
}

// Mean complex gain of the float32 hardware phasor (v_cos_f32, v_sin_f32 take cycles) against
// the float64 reference, over phases r_j = (j + 1/2) / N on [0, 1): per-block partial sums of
// p_hw conj(p_exact), reduced in a fixed tree order.
__global__ __launch_bounds__(PREP_BLOCK) void k_gain_partial(double* __restrict__ gainpart) {
  __shared__ double red[2][PREP_BLOCK];
  const double inv_n = 1.0 / ((double)NGAIN_BLK * PREP_BLOCK * NGAIN_PER);
  double gr = 0.0, gi = 0.0;
  for (int j = 0; j < NGAIN_PER; ++j) {
    const int64_t idx = ((int64_t)blockIdx.x * PREP_BLOCK + threadIdx.x) * NGAIN_PER + j;
    const float r = (float)(((double)idx + 0.5) * inv_n);
    const float ch = __builtin_amdgcn_cosf(r), sh = __builtin_amdgcn_sinf(r);
    double se, ce;
    sincos_cycles_f64((double)r, se, ce);
    gr += (double)ch * ce + (double)sh * se;
    gi += (double)sh * ce - (double)ch * se;
  }
  red[0][threadIdx.x] = gr;
  red[1][threadIdx.x] = gi;
  __syncthreads();
  for (int off = PREP_BLOCK / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      red[0][threadIdx.x] += red[0][threadIdx.x + off];
      red[1][threadIdx.x] += red[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x < 2) gainpart[(int64_t)blockIdx.x * 2 + threadIdx.x] = red[threadIdx.x][0] * inv_n;
}

// One workgroup: fixed-order reduction of the block partials into the event constants.
template <int ND>
__global__ __launch_bounds__(PREP_BLOCK) void k_prep_final(const double* __restrict__ blockpart, int nblk,
                                                           const double* __restrict__ gainpart,
                                                           EventConst* __restrict__ ec) {
  constexpr int NP = prep_part(ND);
  __shared__ double red[NP + 2][PREP_BLOCK];
  double acc[NP + 2];
#pragma unroll
  for (int j = 0; j < NP + 2; ++j) acc[j] = 0.0;
  acc[ND + 2] = __builtin_inf();
  for (int b = threadIdx.x; b < nblk; b += PREP_BLOCK) {
    const double* bp = blockpart + (int64_t)b * NP;
#pragma unroll
    for (int d = 0; d < ND; ++d) acc[d] += bp[d];
    acc[ND] = fmax(acc[ND], bp[ND]);
    acc[ND + 1] += bp[ND + 1];
    acc[ND + 2] = fmin(acc[ND + 2], bp[ND + 2]);
    acc[ND + 3] = fmax(acc[ND + 3], bp[ND + 3]);
  }
  for (int b = threadIdx.x; b < NGAIN_BLK; b += PREP_BLOCK) {
    acc[NP] += gainpart[2 * b];
    acc[NP + 1] += gainpart[2 * b + 1];
  }
#pragma unroll
  for (int j = 0; j < NP + 2; ++j) red[j][threadIdx.x] = acc[j];
  __syncthreads();
  for (int off = PREP_BLOCK / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
#pragma unroll
      for (int d = 0; d < ND; ++d) red[d][threadIdx.x] += red[d][threadIdx.x + off];
      red[ND][threadIdx.x] = fmax(red[ND][threadIdx.x], red[ND][threadIdx.x + off]);
      red[ND + 1][threadIdx.x] += red[ND + 1][threadIdx.x + off];
      red[ND + 2][threadIdx.x] = fmin(red[ND + 2][threadIdx.x], red[ND + 2][threadIdx.x + off]);
      red[ND + 3][threadIdx.x] = fmax(red[ND + 3][threadIdx.x], red[ND + 3][threadIdx.x + off]);
      red[NP][threadIdx.x] += red[NP][threadIdx.x + off];
      red[NP + 1][threadIdx.x] += red[NP + 1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    EventConst e;
#pragma unroll
    for (int d = 0; d < MAXDET; ++d) e.K[d] = d < ND ? red[d][0] : 0.0;
    const double um = red[ND][0];
    // smallest power of two >= max |u| (exact rescaling of the float32 tables)
    e.uref = (um > 0.0 && isfinite(um)) ? exp2(ceil(log2(um))) : 1.0;
    // Z_hw ~ conj(G) Z for coherent sums, so the float32 sums are multiplied by 1 / conj(G)
    const double gr = red[NP][0], gi = red[NP + 1][0];
    const double g2 = gr * gr + gi * gi;
    e.gain_r = gr / g2;
    e.gain_i = gi / g2;
    e.bad = red[ND + 1][0] != 0.0 || !isfinite(um);
    e.pad = 0;
    e.isco = 0;
    e.uniform = 0;
    e.grid_df = 0.0;
    e.fmin = red[ND + 2][0];
    e.fmax = red[ND + 3][0];
    // |g_m| over the band: each basis function is monotone there except f^(1/3) ln f, whose
    // magnitude peaks at f = e^-3 (value 3/e) when the band contains that point
    const double fl = e.fmin, fh = e.fmax;
    const double ga[NBASIS] = {pow(fl, -5.0 / 3.0), 1.0 / fl, pow(fl, -2.0 / 3.0), pow(fl, -1.0 / 3.0),
                               fabs(log(fl)), cbrt(fl), fabs(cbrt(fl) * log(fl)), pow(fl, 2.0 / 3.0)};
    const double gb[NBASIS] = {pow(fh, -5.0 / 3.0), 1.0 / fh, pow(fh, -2.0 / 3.0), pow(fh, -1.0 / 3.0),
                               fabs(log(fh)), cbrt(fh), fabs(cbrt(fh) * log(fh)), pow(fh, 2.0 / 3.0)};
#pragma unroll
    for (int m = 0; m < NBASIS; ++m) e.gmax[m] = fmax(ga[m], gb[m]);
    if (fl < 0.049787068367863944 && fh > 0.049787068367863944) e.gmax[6] = fmax(e.gmax[6], 1.1036383235143269);
#pragma unroll
    for (int m = 0; m < NBASIS; ++m) e.fa[m] = 0.0;
#pragma unroll
    for (int d = 0; d < MAXDET; ++d) e.fT[d] = 0.0;
    *ec = e;
  }
}

// One thread per bin: the mixed-precision row (float64 basis, float32 u / uref).
template <int ND>
__global__ __launch_bounds__(PREP_BLOCK) void k_prep_mixed(const RowF64<ND>* __restrict__ tab64, int64_t M,
                                                           const EventConst* __restrict__ ec,
                                                           RowMixed<ND>* __restrict__ tab32) {
  const int64_t k = (int64_t)blockIdx.x * PREP_BLOCK + threadIdx.x;
  if (k >= M) return;
  const double inv = 1.0 / ec->uref;
  const RowF64<ND> r = tab64[k];
  RowMixed<ND> o;
  o.f = r.f; o.x = r.x; o.w = r.w; o.w2 = r.w2; o.lnf = r.lnf;
#pragma unroll
  for (int j = 0; j < 2 * ND; ++j) o.u[j] = (float)(r.u[j] * inv);
  tab32[k] = o;
}

hipError_t launch_prep_mixed(int nd, const void* tab64, int64_t M, const EventConst* ec, void* tab32, hipStream_t s) {
  const dim3 grid((unsigned)prep_blocks(M));
  switch (nd) {
    case 1: hipLaunchKernelGGL(k_prep_mixed<1>, grid, dim3(PREP_BLOCK), 0, s, (const RowF64<1>*)tab64, M, ec, (RowMixed<1>*)tab32); break;
    case 2: hipLaunchKernelGGL(k_prep_mixed<2>, grid, dim3(PREP_BLOCK), 0, s, (const RowF64<2>*)tab64, M, ec, (RowMixed<2>*)tab32); break;
    case 3: hipLaunchKernelGGL(k_prep_mixed<3>, grid, dim3(PREP_BLOCK), 0, s, (const RowF64<3>*)tab64, M, ec, (RowMixed<3>*)tab32); break;
    case 4: hipLaunchKernelGGL(k_prep_mixed<4>, grid, dim3(PREP_BLOCK), 0, s, (const RowF64<4>*)tab64, M, ec, (RowMixed<4>*)tab32); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int ND>
static hipError_t prep_nd(const double* data, const double* psd, const double* fgrid, int64_t M, double df, void* tab64,
                          void* tab32, RowGradF32* g32, RowGradF64* g64, double* blockpart, int nblk, EventConst* ec,
                          hipStream_t s) {
  // blockpart holds nblk * prep_part(ND) bin partials followed by NGAIN_BLK * 2 gain partials
  double* gainpart = blockpart + (size_t)nblk * prep_part(ND);
  hipLaunchKernelGGL(k_prep_bins<ND>, dim3(nblk), dim3(PREP_BLOCK), 0, s, data, psd, fgrid, M, df,
                     (RowF64<ND>*)tab64, g32, g64, blockpart);
  hipLaunchKernelGGL(k_gain_partial, dim3(NGAIN_BLK), dim3(PREP_BLOCK), 0, s, gainpart);
  hipLaunchKernelGGL(k_prep_final<ND>, dim3(1), dim3(PREP_BLOCK), 0, s, (const double*)blockpart, nblk,
                     (const double*)gainpart, ec);
  hipLaunchKernelGGL(k_prep_mixed<ND>, dim3(nblk), dim3(PREP_BLOCK), 0, s, (const RowF64<ND>*)tab64, M,
                     (const EventConst*)ec, (RowMixed<ND>*)tab32);
  return hipGetLastError();
}

hipError_t launch_prep(int nd, const double* data, const double* psd, const double* fgrid, int64_t M, double df,
                       void* tab64, void* tab32, RowGradF32* g32, RowGradF64* g64, double* blockpart, int nblk,
                       EventConst* ec, hipStream_t s) {
  switch (nd) {
    case 1: return prep_nd<1>(data, psd, fgrid, M, df, tab64, tab32, g32, g64, blockpart, nblk, ec, s);
    case 2: return prep_nd<2>(data, psd, fgrid, M, df, tab64, tab32, g32, g64, blockpart, nblk, ec, s);
    case 3: return prep_nd<3>(data, psd, fgrid, M, df, tab64, tab32, g32, g64, blockpart, nblk, ec, s);
    case 4: return prep_nd<4>(data, psd, fgrid, M, df, tab64, tab32, g32, g64, blockpart, nblk, ec, s);
  }
  return hipErrorInvalidValue;
}

// Model strain on the grid, float64: h_det,k = A Q_det f^-7/6 exp(-2 pi i (psi_k + f_k T_det + c0)).
// Grid: (ceil(M / 256), B); the point's coefficients are block-uniform.
template <int ND>
__global__ __launch_bounds__(PREP_BLOCK) void k_waveform(const double* __restrict__ coef, int64_t Bp,
                                                         const double* __restrict__ fgrid, int64_t M,
                                                         double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * PREP_BLOCK + threadIdx.x;
  const int64_t b = blockIdx.y;
  if (k >= M) return;
  double a[NBASIS];
#pragma unroll
  for (int m = 0; m < NBASIS; ++m) a[m] = coef[(CO_A + m) * Bp + b];
  const double c0 = coef[CO_C0 * Bp + b], amp = coef[CO_AMP * Bp + b];
  const double f = fgrid[k];
  const double x = cbrt(f), w2 = 1.0 / f, w = w2 / (x * x), lnf = log(f);
  double t = fma(a[7], x, fma(a[6], lnf, a[5]));
  t = fma(t, x, a[4] * lnf);
  t = fma(t, x, a[3]);
  t = fma(t, x, a[2]);
  t = fma(t, x, a[1]);
  const double psi = fma(w2, t, w * a[0]) + c0;
  const double mag = amp * w2 / sqrt(x);
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const double T = coef[(CO_T + d) * Bp + b];
    double sn, cs;
    sincos_cycles_f64(fma(f, T, psi), sn, cs);
    const double qr = coef[(CO_QR + d) * Bp + b], qi = coef[(CO_QI + d) * Bp + b];
    // (qr + i qi) (cs - i sn) mag
    double* o = out + ((b * ND + d) * M + k) * 2;
    o[0] = mag * (qr * cs + qi * sn);
    o[1] = mag * (qi * cs - qr * sn);
  }
}

hipError_t launch_waveform(int nd, const EventGeom&, const double* coef, int64_t B, int64_t Bp, const double* fgrid,
                           int64_t M, double* out, hipStream_t s) {
  dim3 grid((unsigned)prep_blocks(M), (unsigned)B);
  switch (nd) {
    case 1: hipLaunchKernelGGL(k_waveform<1>, grid, dim3(PREP_BLOCK), 0, s, coef, Bp, fgrid, M, out); break;
    case 2: hipLaunchKernelGGL(k_waveform<2>, grid, dim3(PREP_BLOCK), 0, s, coef, Bp, fgrid, M, out); break;
    case 3: hipLaunchKernelGGL(k_waveform<3>, grid, dim3(PREP_BLOCK), 0, s, coef, Bp, fgrid, M, out); break;
    case 4: hipLaunchKernelGGL(k_waveform<4>, grid, dim3(PREP_BLOCK), 0, s, coef, Bp, fgrid, M, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gwl
