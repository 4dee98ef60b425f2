// Layouts shared by the host runtime and the kernels of the batched log-likelihood library.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace gwl {

constexpr int NPARAM = 11;   // parameters per point
constexpr int MAXDET = 4;    // detectors per event
constexpr int NBASIS = 8;    // per-bin phase basis functions g_m(f) (see gwl_device.h)
constexpr int WAVE = 64;     // CDNA wavefront width: one lane per parameter point
constexpr int WAVES_PER_BLOCK = 4;
constexpr int BLOCK = WAVE * WAVES_PER_BLOCK;
constexpr int NXCD = 8;      // MI355X accelerator complex dies; workgroups are dealt round-robin

// Detector geometry of an event, computed once on the host:
// dt = detector tensor (xx, yy, zz, xy, xz, yz), r = vertex position (m).
struct EventGeom {
  int ndet;
  double gmst;
  double dt[MAXDET][6];
  double r[MAXDET][3];
};

// Per-event scalars produced on the device by event preparation.
struct EventConst {
  double K[MAXDET];   // 4 df sum_k f_k^(-7/3) / S_k
  double uref;        // power of two >= max |u|: the float32 tables hold u / uref
  double gain_r;      // 1 / conj(G), G = mean over phases of p_hw conj(p_exact): divides the mean
  double gain_i;      //   complex gain of the hardware float32 phasor out of the float32 sums
  int bad;            // nonzero if an input value was rejected
  int pad;
  int isco;           // 1: the model is zero above the ISCO frequency (GWL_F_ISCO_CUTOFF)
  int uniform;        // 1: every grid step is grid_df to within 8 ulp of fmax (see grid_is_uniform)
  double grid_df;     // (fmax - fmin) / (M - 1): first guess of a frequency's bin, uniform step
  double fmin, fmax;  // lowest and highest grid frequency
  double gmax[NBASIS];// max over [fmin, fmax] of |g_m(f)|: bounds the phase range of a point
  // Relative binning: the fiducial waveform's phase coefficients and detector shifts. The set-up
  // subtracts them, so the bin loop evaluates the phase of h / h0 on the edges. Zero otherwise.
  double fa[NBASIS];
  double fT[MAXDET];
};

// Largest phase, in cycles, that a point may reach on the grid: the float64 bin loops split
// 2048 times the phase into an integer and a remainder in float64, exactly for magnitudes below
// 2^51; a point whose phase bound exceeds PHASE_LIMIT is outside the supported domain (NaN).
constexpr double PHASE_LIMIT = 549755813888.0;  // 2^39

// Phases sampled to measure the hardware phasor gain: NGAIN_BLK workgroups x 256 threads x
// NGAIN_PER phases, uniform on [0, 1) cycles.
constexpr int NGAIN_BLK = 1024;
constexpr int NGAIN_PER = 16;

// Per-bin rows, one row per frequency bin, read wave-uniformly by the bin loop. The row tables
// are allocated with TAB_PAD zero rows after the last bin (look-ahead reads).
constexpr int TAB_PAD = 8;
// Basis: f, x = f^(1/3), w = f^(-5/3), w2 = f^(-1), ln f.
template <int ND>
struct RowMixed {          // float64 basis + float32 u / uref per detector (re, im)
  double f, x, w, w2, lnf;
  float u[2 * ND];
};
template <int ND>
struct RowF64 {            // float64 basis + float64 u per detector (re, im)
  double f, x, w, w2, lnf;
  double u[2 * ND];
};
struct RowGradF32 {        // float32 phase basis g_0..g_7 and f, for the adjoint moments
  float g[NBASIS];
  float f;
};
struct RowGradF64 {        // float64 g_m not already in RowF64: f^-2/3, f^-1/3, f^1/3 ln f, f^2/3
  double g2, g3, g6, g7;
};

static_assert(sizeof(RowMixed<1>) == 48 && sizeof(RowMixed<3>) == 64 && sizeof(RowMixed<4>) == 72, "row layout");
static_assert(sizeof(RowF64<1>) == 56 && sizeof(RowF64<3>) == 88 && sizeof(RowF64<4>) == 104, "row layout");
static_assert(sizeof(RowGradF32) == 36 && sizeof(RowGradF64) == 32, "row layout");

// Per-point coefficient rows written by the set-up kernel, structure of arrays [row][Bp]:
constexpr int CO_A = 0;              // a_0..a_7 phase coefficients (cycles)
constexpr int CO_T = CO_A + NBASIS;  // T_det = t_c + dt_det, MAXDET rows
constexpr int CO_QR = CO_T + MAXDET; // Re Q_det
constexpr int CO_QI = CO_QR + MAXDET;// Im Q_det
constexpr int CO_C0 = CO_QI + MAXDET;// constant phase (cycles)
constexpr int CO_AMP = CO_C0 + 1;    // amplitude A
constexpr int CO_CR = CO_AMP + 1;    // Re c_det, adjoint projection c_det = E G Q_det (MAXDET rows)
constexpr int CO_CI = CO_CR + MAXDET;// Im c_det
constexpr int NCOEF = CO_CI + MAXDET;

// Accumulated sums per point, per bin chunk (partials [chunk][z][Bp]), with w = u p the
// per-bin product of one detector and y_det = Im(c_det w):
//   forward : Z_det = sum w (re, im)                                     -> 2 ND
//   adjoint : + sum f y_det (one real per detector), + sum_k g_m sum_det y_det (m < 8)
//                                                                         -> 3 ND + 8
__host__ __device__ constexpr int nz_of(int nd, bool grad) { return grad ? 3 * nd + NBASIS : 2 * nd; }

// Detector calibration model: per detector, nnode amplitude and nnode phase node values
// interpolated in ln f by a cubic spline whose value at a bin depends on the four nodes around
// it. The weights of those four nodes are per-bin constants; the window of four nodes is fixed
// over a node interval, and the bin loop's chunks never cross an interval.
constexpr int MAXNODE = 16;
struct RowCal32 {
  float w[4];
};
struct RowCal64 {
  double w[4];
};
constexpr int MAXCALCHUNK = 96;
struct CalShape {
  int nnode;              // nodes per detector
  int nchunk;             // chunks; each lies inside one node interval
  int npg, nbpg, items, gper;
  int j0[MAXNODE];        // first node of each interval's window of four
  int cj[MAXCALCHUNK];    // interval of each chunk
  int ck[MAXCALCHUNK + 1];// first bin of each chunk; ck[nchunk] = M
};
// Calibrated sums: Z_det (2 ND); adjoint: + the uncalibrated model's moments (ND + 8) + per
// detector the window moments of the amplitude (4) and phase (4) nodes
__host__ __device__ constexpr int nz_cal(int nd, bool grad) { return grad ? 11 * nd + NBASIS : 2 * nd; }

}  // namespace gwl
