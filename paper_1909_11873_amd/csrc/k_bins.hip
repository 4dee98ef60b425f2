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
// on more than NB terms at once. The adjoint's moments are accumulated in float64.
#include <hip/hip_runtime.h>

#include "gwl_bins.h"
#include "gwl_common.h"
#include "gwl_device.h"
#include "gwl_launch.h"

namespace gwl {

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

template <int ND, bool GRAD>
__global__ __launch_bounds__(BLOCK) void k_bins_mixed(const RowMixed<ND>* __restrict__ tab,
                                                      const RowGradF64* __restrict__ gtab,
                                                      const double* __restrict__ coef, int64_t B, int64_t Bp, int64_t M,
                                                      LoopShape sh, double* __restrict__ part) {
  constexpr int NZ = nz_of(ND, GRAD);
  int c, k0, k1, pg;
  if (!locate(sh, M, c, k0, k1, pg)) return;
  const int64_t p = (int64_t)pg * WAVE + (threadIdx.x % WAVE);
  const int64_t pc = p < B ? p : B - 1;
  double a[NBASIS], T[ND];
  float cr[ND], ci[ND];
  load_coef<ND, float>(coef, Bp, pc, GRAD, a, T, cr, ci);
  double tot[NZ];
  bin_loop_mixed<ND, GRAD>(tab, gtab, k0, k1, a, T, cr, ci, tot);
#pragma unroll
  for (int z = 0; z < NZ; ++z) part[((int64_t)c * NZ + z) * Bp + p] = tot[z];
}

template <int ND, bool GRAD>
__global__ __launch_bounds__(BLOCK) void k_bins_f64(const RowF64<ND>* __restrict__ tab,
                                                    const RowGradF64* __restrict__ gtab,
                                                    const double* __restrict__ coef, int64_t B, int64_t Bp, int64_t M,
                                                    LoopShape sh, double* __restrict__ part) {
  constexpr int NZ = nz_of(ND, GRAD);
  __shared__ double2 tbl[PH_TBL];
  fill_phasor_table(tbl);  // before any wavefront leaves
  __syncthreads();
  int c, k0, k1, pg;
  if (!locate(sh, M, c, k0, k1, pg)) return;
  const int64_t p = (int64_t)pg * WAVE + (threadIdx.x % WAVE);
  const int64_t pc = p < B ? p : B - 1;
  double a[NBASIS], T[ND], cr[ND], ci[ND];
  load_coef<ND, double>(coef, Bp, pc, GRAD, a, T, cr, ci);
  to_table_units<ND>(a, T);
  double z[NZ];
  bin_loop_f64<ND, GRAD>(tab, gtab, k0, k1, a, T, cr, ci, tbl, z);
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
                         (const RowGradF64*)gtab64, coef, B, Bp, M, sh, part);
    else
      hipLaunchKernelGGL((k_bins_mixed<ND, false>), grid, block, 0, s, (const RowMixed<ND>*)tab,
                         (const RowGradF64*)gtab64, coef, B, Bp, M, sh, part);
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
