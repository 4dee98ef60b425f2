// Host runtime of the C ABI in include/gwlike.h: argument checking, event tables, workspace,
// launch sequencing, tile choice. All computation happens in the kernels.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/gwlike.h"
#include "gwl_common.h"
#include "gwl_launch.h"
#include "gwl_runtime.h"

using namespace gwl;

namespace gwl {

static thread_local std::string g_err;

gwl_status fail(gwl_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

gwl_status hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) return fail(GWL_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
  return fail(GWL_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_err.clear(); }

size_t row64_bytes(int nd) { return 40 + 16 * (size_t)nd; }
size_t row32_bytes(int nd) { return 40 + 8 * (size_t)nd; }

// Detector tensor and vertex of an L-shaped detector (arms horizontal, azimuths clockwise
// from North) on a spherical Earth.
static void detector_geometry(const gwl_detector& d, double dt[6], double r[3]) {
  const double RE = 6.371e6;
  const double sl = sin(d.lat), cl = cos(d.lat), so = sin(d.lon), co = cos(d.lon);
  const double north[3] = {-sl * co, -sl * so, cl};
  const double east[3] = {-so, co, 0.0};
  double xa[3], ya[3];
  for (int i = 0; i < 3; ++i) {
    xa[i] = cos(d.xarm_az) * north[i] + sin(d.xarm_az) * east[i];
    ya[i] = cos(d.yarm_az) * north[i] + sin(d.yarm_az) * east[i];
  }
  const int ii[6] = {0, 1, 2, 0, 0, 1}, jj[6] = {0, 1, 2, 1, 2, 2};
  for (int m = 0; m < 6; ++m) dt[m] = 0.5 * (xa[ii[m]] * xa[jj[m]] - ya[ii[m]] * ya[jj[m]]);
  r[0] = RE * cl * co;
  r[1] = RE * cl * so;
  r[2] = RE * sl;
}

gwl_status make_geom(const gwl_detector* dets, int ndet, double gmst, EventGeom& g) {
  if (!dets) return fail(GWL_E_INVALID, "dets is null");
  if (ndet < 1 || ndet > GWL_MAX_DET) return fail(GWL_E_SHAPE, "ndet=%d outside [1, %d]", ndet, GWL_MAX_DET);
  if (!isfinite(gmst)) return fail(GWL_E_INVALID, "gmst is not finite");
  memset(&g, 0, sizeof g);
  g.ndet = ndet;
  g.gmst = gmst;
  for (int d = 0; d < ndet; ++d) {
    const gwl_detector& x = dets[d];
    if (!isfinite(x.lat) || !isfinite(x.lon) || !isfinite(x.xarm_az) || !isfinite(x.yarm_az))
      return fail(GWL_E_INVALID, "detector %d has a non-finite angle", d);
    detector_geometry(x, g.dt[d], g.r[d]);
  }
  return GWL_OK;
}

gwl_status check_device(int dev) {
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != dev) return fail(GWL_E_INVALID, "event lives on device %d but device %d is current", dev, cur);
  return GWL_OK;
}

}  // namespace gwl

namespace gwl {

// A grid is uniform when every step f_{k+1} - f_k equals the mean step (f_{M-1} - f_0) / (M - 1)
// to within 8 ulp of the highest frequency: a grid built as f_0 + k df in float64 is uniform.
static bool grid_is_uniform(const std::vector<double>& f, double& step) {
  const size_t M = f.size();
  step = M > 1 ? (f[M - 1] - f[0]) / (double)(M - 1) : 1.0;
  const double tol = 8.0 * ldexp(fabs(f[M - 1]), -52);
  for (size_t k = 0; k + 1 < M; ++k)
    if (!(fabs((f[k + 1] - f[k]) - step) <= tol)) return false;
  return true;
}

// Tables of the optional ISCO cut-off, built on the host in float64 (once per event): the grid
// (which must increase) and per detector the running sums Kc[k] = sum_{j < k} 4 df f_j^(-7/3) / S_j,
// k = 0..M, so that <h|h> of a point cut after its first kc bins is A^2 |Q_det|^2 Kc[kc].
static gwl_status isco_tables(gwl_event ev, const double* fgrid, const double* psd, hipStream_t s) {
  const int64_t M = ev->M;
  const int nd = ev->ndet;
  std::vector<double> f((size_t)M), ps((size_t)M * nd);
  hipError_t e = hipMemcpyAsync(f.data(), fgrid, sizeof(double) * M, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(ps.data(), psd, sizeof(double) * M * nd, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "grid read-back");
  for (int64_t k = 1; k < M; ++k)
    if (!(f[(size_t)k] > f[(size_t)k - 1]))
      return fail(GWL_E_INVALID, "the ISCO cut-off needs an increasing frequency grid (bin %lld)", (long long)k);
  std::vector<double> kc((size_t)(M + 1) * nd);
  for (int d = 0; d < nd; ++d) {
    double acc = 0.0;
    kc[(size_t)d * (M + 1)] = 0.0;
    for (int64_t k = 0; k < M; ++k) {
      acc += 4.0 * ev->df * pow(f[(size_t)k], -7.0 / 3.0) / ps[(size_t)d * M + k];
      kc[(size_t)d * (M + 1) + k + 1] = acc;
    }
  }
  e = hipMalloc((void**)&ev->fgrid, sizeof(double) * M);
  if (e == hipSuccess) e = hipMalloc((void**)&ev->kcum, sizeof(double) * kc.size());
  if (e == hipSuccess) e = hipMemcpy(ev->fgrid, f.data(), sizeof(double) * M, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ev->kcum, kc.data(), sizeof(double) * kc.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "ISCO tables");
  ev->ech.isco = 1;
  ev->ech.grid_df = M > 1 ? (f[(size_t)M - 1] - f[0]) / (double)(M - 1) : 1.0;
  e = hipMemcpy(ev->ec, &ev->ech, sizeof(EventConst), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "ISCO tables");
  return GWL_OK;
}

}  // namespace gwl

// ------------------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------------------
extern "C" {

const char* gwl_last_error(void) { return g_err.c_str(); }

const char* gwl_version(void) { return "gwlike 0.1 (gfx950)"; }

gwl_status gwl_event_create(const double* data, const double* psd, const gwl_detector* dets, int ndet,
                            const double* fgrid, int64_t M, double df, double gmst, unsigned flags, void* stream,
                            gwl_event* out) {
  clear_error();
  if (!out) return fail(GWL_E_INVALID, "out is null");
  *out = nullptr;
  if (!data || !psd || !fgrid) return fail(GWL_E_INVALID, "data, psd and fgrid must be device pointers");
  if (M < 1 || M > (int64_t)1 << 30) return fail(GWL_E_SHAPE, "M=%lld outside [1, 2^30]", (long long)M);
  if (!(df > 0.0) || !isfinite(df)) return fail(GWL_E_INVALID, "df must be finite and positive");
  if (flags & ~(unsigned)GWL_F_ISCO_CUTOFF) return fail(GWL_E_UNSUPPORTED, "flags=0x%x: unknown flags", flags);
  EventGeom g;
  gwl_status st = make_geom(dets, ndet, gmst, g);
  if (st != GWL_OK) return st;

  gwl_event ev = new (std::nothrow) gwl_event_s();
  if (!ev) return fail(GWL_E_NOMEM, "host allocation failed");
  ev->ndet = ndet;
  ev->M = M;
  ev->df = df;
  ev->gmst = gmst;
  ev->geom = g;
  for (int d = 0; d < ndet; ++d) ev->dets[d] = dets[d];
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipGetDevice(&ev->device);
  const int nblk = prep_blocks(M);
  double* blockpart = nullptr;
  if (e == hipSuccess) e = hipMalloc(&ev->tab64, row64_bytes(ndet) * (M + TAB_PAD));
  if (e == hipSuccess) e = hipMalloc(&ev->tab32, row32_bytes(ndet) * (M + TAB_PAD));
  if (e == hipSuccess)
    e = hipMemsetAsync((char*)ev->tab64 + row64_bytes(ndet) * M, 0, row64_bytes(ndet) * TAB_PAD, s);
  if (e == hipSuccess)
    e = hipMemsetAsync((char*)ev->tab32 + row32_bytes(ndet) * M, 0, row32_bytes(ndet) * TAB_PAD, s);
  if (e == hipSuccess) e = hipMalloc((void**)&ev->g32, sizeof(RowGradF32) * M);
  if (e == hipSuccess) e = hipMalloc((void**)&ev->g64, sizeof(RowGradF64) * M);
  if (e == hipSuccess) e = hipMalloc((void**)&ev->ec, sizeof(EventConst));
  if (e == hipSuccess) e = hipMalloc((void**)&blockpart, sizeof(double) * prep_scratch_doubles(ndet, M));
  if (e == hipSuccess)
    e = launch_prep(ndet, data, psd, fgrid, M, df, ev->tab64, ev->tab32, ev->g32, ev->g64, blockpart, nblk, ev->ec, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&ev->ech, ev->ec, sizeof(EventConst), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (blockpart) (void)hipFree(blockpart);
  if (e != hipSuccess) {
    gwl_event_destroy(ev);
    return hip_fail(e, "event preparation");
  }
  if (ev->ech.bad) {
    gwl_event_destroy(ev);
    return fail(GWL_E_INVALID, "rejected inputs: every PSD value and frequency must be finite and positive and "
                               "every data value finite");
  }
  // the grid's step, and whether the float64 loop may carry detector phasors by a fixed rotation
  {
    std::vector<double> fh((size_t)M);
    e = hipMemcpyAsync(fh.data(), fgrid, sizeof(double) * M, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) {
      ev->ech.uniform = grid_is_uniform(fh, ev->ech.grid_df) ? 1 : 0;
      e = hipMemcpyAsync(ev->ec, &ev->ech, sizeof(EventConst), hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      gwl_event_destroy(ev);
      return hip_fail(e, "grid read-back");
    }
  }
  if (flags & GWL_F_ISCO_CUTOFF) {
    st = isco_tables(ev, fgrid, psd, s);
    if (st != GWL_OK) {
      gwl_event_destroy(ev);
      return st;
    }
  }
  *out = ev;
  return GWL_OK;
}

// Relative-binning edges on the grid: the bins where floor(dpsi(f) / eps) changes, plus both
// ends, with dpsi(f) = 2 pi sum_gamma sign(gamma) (f / f_gamma)^gamma over the post-Newtonian
// phase power laws gamma = -5/3, -2/3, 1, 5/3, 7/3 (f_gamma = f_hi for gamma > 0, f_lo below):
// the largest phase difference between two waveforms of the model grows no faster than dpsi.
static std::vector<int64_t> rb_edges(const std::vector<double>& f, double eps) {
  const double flo = f.front(), fhi = f.back();
  const double gam[5] = {-5.0 / 3.0, -2.0 / 3.0, 1.0, 5.0 / 3.0, 7.0 / 3.0};
  auto dpsi = [&](double x) {
    double s = 0.0;
    for (double g : gam) s += (g > 0 ? 1.0 : -1.0) * pow(x / (g > 0 ? fhi : flo), g);
    return 2.0 * M_PI * s;
  };
  std::vector<int64_t> idx{0};
  double prev = floor(dpsi(f[0]) / eps);
  for (size_t k = 1; k < f.size(); ++k) {
    const double c = floor(dpsi(f[k]) / eps);
    if (c != prev) idx.push_back((int64_t)k);
    prev = c;
  }
  if (idx.back() != (int64_t)f.size() - 1) idx.push_back((int64_t)f.size() - 1);
  return idx;
}

gwl_status gwl_event_create_rb(const double* data, const double* psd, const gwl_detector* dets, int ndet,
                               const double* fgrid, int64_t M, double df, double gmst, const double* theta_fid,
                               double eps, unsigned flags, void* stream, gwl_event* out) {
  clear_error();
  if (!out) return fail(GWL_E_INVALID, "out is null");
  *out = nullptr;
  if (!theta_fid) return fail(GWL_E_INVALID, "theta_fid must be a host array of 11 values");
  for (int i = 0; i < NPARAM; ++i)
    if (!isfinite(theta_fid[i])) return fail(GWL_E_INVALID, "theta_fid[%d] is not finite", i);
  if (!(eps > 0.0) || !isfinite(eps)) return fail(GWL_E_INVALID, "eps must be finite and positive");
  if (flags & GWL_F_ISCO_CUTOFF)
    return fail(GWL_E_UNSUPPORTED, "the ISCO cut-off is not available with relative binning");
  gwl_event ev = nullptr;
  gwl_status st = gwl_event_create(data, psd, dets, ndet, fgrid, M, df, gmst, flags, stream, &ev);
  if (st != GWL_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  // grid on the host, edges
  std::vector<double> fh((size_t)M);
  hipError_t e = hipMemcpyAsync(fh.data(), fgrid, sizeof(double) * M, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    gwl_event_destroy(ev);
    return hip_fail(e, "grid read-back");
  }
  const std::vector<int64_t> idx = rb_edges(fh, eps);
  const int nedge = (int)idx.size();
  // fiducial coefficients through the ordinary set-up (no offsets, no gain)
  double *th = nullptr, *coef = nullptr, *w = nullptr;
  int64_t* d_idx = nullptr;
  void *tab64 = nullptr, *tab32 = nullptr;
  RowGradF32* g32 = nullptr;
  RowGradF64* g64 = nullptr;
  std::vector<double> hcoef((size_t)NCOEF * WAVE);
  const int nd = ev->ndet;
  e = hipMalloc((void**)&th, sizeof(double) * NPARAM);
  if (e == hipSuccess) e = hipMalloc((void**)&coef, sizeof(double) * NCOEF * WAVE);
  if (e == hipSuccess) e = hipMemcpyAsync(th, theta_fid, sizeof(double) * NPARAM, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_setup(nd, ev->geom, nullptr, false, th, 1, WAVE, coef, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hcoef.data(), coef, sizeof(double) * NCOEF * WAVE, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  bool fid_ok = e == hipSuccess;
  if (fid_ok) {
    for (int m = 0; m < NBASIS; ++m) {
      ev->ech.fa[m] = hcoef[(size_t)(CO_A + m) * WAVE];
      fid_ok &= isfinite(ev->ech.fa[m]);
    }
    for (int d = 0; d < MAXDET; ++d) ev->ech.fT[d] = d < nd ? hcoef[(size_t)(CO_T + d) * WAVE] : 0.0;
    for (int d = 0; d < nd; ++d) fid_ok &= isfinite(ev->ech.fT[d]);
  }
  if (e == hipSuccess && !fid_ok) {
    (void)hipFree(th);
    (void)hipFree(coef);
    gwl_event_destroy(ev);
    return fail(GWL_E_INVALID, "theta_fid is outside the model's domain");
  }
  // edge tables (the edges are not a uniform grid)
  ev->ech.uniform = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(ev->ec, &ev->ech, sizeof(EventConst), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMalloc((void**)&d_idx, sizeof(int64_t) * nedge);
  if (e == hipSuccess) e = hipMemcpyAsync(d_idx, idx.data(), sizeof(int64_t) * nedge, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMalloc((void**)&w, sizeof(double) * rb_scratch_doubles(nd, nedge));
  if (e == hipSuccess) e = hipMalloc(&tab64, row64_bytes(nd) * (nedge + TAB_PAD));
  if (e == hipSuccess) e = hipMalloc(&tab32, row32_bytes(nd) * (nedge + TAB_PAD));
  if (e == hipSuccess) e = hipMemsetAsync((char*)tab64 + row64_bytes(nd) * nedge, 0, row64_bytes(nd) * TAB_PAD, s);
  if (e == hipSuccess) e = hipMemsetAsync((char*)tab32 + row32_bytes(nd) * nedge, 0, row32_bytes(nd) * TAB_PAD, s);
  if (e == hipSuccess) e = hipMalloc((void**)&g32, sizeof(RowGradF32) * nedge);
  if (e == hipSuccess) e = hipMalloc((void**)&g64, sizeof(RowGradF64) * nedge);
  if (e == hipSuccess) e = launch_rb(nd, ev->tab64, ev->g32, ev->g64, d_idx, nedge, w, ev->ec, tab64, tab32, g32, g64, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&ev->ech, ev->ec, sizeof(EventConst), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(th);
  (void)hipFree(coef);
  if (d_idx) (void)hipFree(d_idx);
  if (w) (void)hipFree(w);
  if (e != hipSuccess) {
    if (tab64) (void)hipFree(tab64);
    if (tab32) (void)hipFree(tab32);
    if (g32) (void)hipFree(g32);
    if (g64) (void)hipFree(g64);
    gwl_event_destroy(ev);
    return hip_fail(e, "relative-binning tables");
  }
  // the event now walks the edges
  (void)hipFree(ev->tab64);
  (void)hipFree(ev->tab32);
  (void)hipFree(ev->g32);
  (void)hipFree(ev->g64);
  ev->tab64 = tab64;
  ev->tab32 = tab32;
  ev->g32 = g32;
  ev->g64 = g64;
  ev->M_full = ev->M;
  ev->M = nedge;
  ev->rb_idx = idx;
  *out = ev;
  return GWL_OK;
}

// Calibration spline tables (host, float64): per bin the Catmull-Rom weights of the four nodes
// around it in ln f, with the linearly extrapolated ghost node beyond either end folded into
// the real end nodes, expressed over the interval's window of four real nodes; the interval
// starts; and per detector K1_j = sum_k K_k w_kj, K2_jl = sum_k K_k w_kj w_kl, K_k = 4 df
// f_k^-7/3 / S_k.
// Catmull-Rom weights of nodes j-1 .. j+2 on interval j as polynomials in t (coefficients of
// t^0 .. t^3), and the ghost nodes at both ends (-1 = 2 v0 - v1, n = 2 v_{n-1} - v_{n-2}) folded
// into the window of four nodes j0[j] .. j0[j] + 3: B[(j * 4 + i) * 4 + p].
static void cal_basis(int n, const int* j0, std::vector<double>& B) {
  const double C[4][4] = {{0.0, -0.5, 1.0, -0.5}, {1.0, 0.0, -2.5, 1.5}, {0.0, 0.5, 2.0, -1.5}, {0.0, 0.0, -0.5, 0.5}};
  B.assign((size_t)(n - 1) * 16, 0.0);
  for (int j = 0; j < n - 1; ++j) {
    double wn[MAXNODE + 2][4] = {};  // over nodes -1 .. n
    for (int i = 0; i < 4; ++i)
      for (int q = 0; q < 4; ++q) wn[j + i][q] += C[i][q];
    for (int q = 0; q < 4; ++q) {
      wn[1][q] += 2.0 * wn[0][q];
      wn[2][q] -= wn[0][q];
      wn[n][q] += 2.0 * wn[n + 1][q];
      wn[n - 1][q] -= wn[n + 1][q];
    }
    for (int i = 0; i < 4; ++i)
      for (int q = 0; q < 4; ++q) B[((size_t)j * 4 + i) * 4 + q] = wn[j0[j] + i + 1][q];
  }
}

static void cal_tables(const std::vector<double>& f, const std::vector<double>& psd, int nd, double df, int n,
                       std::vector<double>& w, std::vector<double>& tloc, int* j0, int64_t* kb,
                       std::vector<double>& kcal) {
  const int64_t M = (int64_t)f.size();
  const double x0 = log(f.front()), x1 = log(f.back());
  const double h = n > 1 ? (x1 - x0) / (n - 1) : 1.0;
  w.assign((size_t)M * 4, 0.0);
  tloc.assign((size_t)M, 0.0);
  std::vector<double> W((size_t)M * n, 0.0);  // weights over all nodes (for K1, K2)
  std::vector<int> jk((size_t)M);
  for (int j = 0; j < n - 1; ++j) j0[j] = std::min(std::max(j - 1, 0), n - 4);
  for (int64_t k = 0; k < M; ++k) {
    double s = (log(f[k]) - x0) / h;
    s = std::min(std::max(s, 0.0), (double)(n - 1));
    const int j = std::min(std::max((int)floor(s), 0), n - 2);
    const double t = s - j;
    tloc[(size_t)k] = t;
    double cw[4] = {0.5 * (-t + 2 * t * t - t * t * t), 0.5 * (2 - 5 * t * t + 3 * t * t * t),
                    0.5 * (t + 4 * t * t - 3 * t * t * t), 0.5 * (-t * t + t * t * t)};  // nodes j-1 .. j+2
    double wn[MAXNODE + 2] = {};  // over nodes -1 .. n
    for (int i = 0; i < 4; ++i) wn[j - 1 + i + 1] += cw[i];
    wn[1] += 2.0 * wn[0];          // ghost -1 = 2 v0 - v1
    wn[2] -= wn[0];
    wn[n] += 2.0 * wn[n + 1];      // ghost n = 2 v_{n-1} - v_{n-2}
    wn[n - 1] -= wn[n + 1];
    for (int i = 0; i < 4; ++i) w[(size_t)k * 4 + i] = wn[j0[j] + i + 1];
    for (int i = 0; i < n; ++i) W[(size_t)k * n + i] = wn[i + 1];
    jk[(size_t)k] = j;
  }
  for (int j = 0; j <= n - 1; ++j) kb[j] = M;
  for (int64_t k = M - 1; k >= 0; --k) kb[jk[(size_t)k]] = k;
  kb[0] = 0;
  for (int j = n - 2; j >= 1; --j) kb[j] = std::min(kb[j], kb[j + 1]);  // empty intervals start where the next does
  kb[n - 1] = M;
  kcal.assign((size_t)nd * (n + n * n), 0.0);
  for (int d = 0; d < nd; ++d) {
    double* K1 = kcal.data() + (size_t)d * (n + n * n);
    double* K2 = K1 + n;
    for (int64_t k = 0; k < M; ++k) {
      const double Kk = 4.0 * df * pow(f[k], -7.0 / 3.0) / psd[(size_t)d * M + k];
      const double* Wk = W.data() + (size_t)k * n;
      for (int i = 0; i < n; ++i) {
        if (Wk[i] == 0.0) continue;
        K1[i] += Kk * Wk[i];
        for (int l = 0; l < n; ++l) K2[i * n + l] += Kk * Wk[i] * Wk[l];
      }
    }
  }
}

}  // extern "C"

namespace gwl {

// Attach calibration tables to an event whose bin loop walks rows at the frequencies `frow`
// (the grid itself, or relative-binning edges): per row the spline weights of its window and its
// position in its node interval, the interval starts in rows, the per-interval cubic basis; the
// spline moments K1, K2 of <h_cal|h_cal> always over every grid bin (fgrid, psd).
static gwl_status attach_cal(gwl_event ev, const std::vector<double>& frow, const std::vector<double>& fgrid,
                             const std::vector<double>& psd, int nnode) {
  const int ndet = ev->ndet;
  const int64_t M = (int64_t)frow.size();
  std::vector<double> w, tl, kc, kc_rows, basis, wfull, tfull;
  int j0full[MAXNODE];
  int64_t kbfull[MAXNODE];
  // the rows' weights (their spline moments are not used: any positive PSD will do), then the
  // moments over the grid
  const std::vector<double> psd_rows((size_t)M * ndet, 1.0);
  cal_tables(frow, psd_rows, ndet, ev->df, nnode, w, tl, ev->cal_j0, ev->cal_kb, kc_rows);
  cal_tables(fgrid, psd, ndet, ev->df, nnode, wfull, tfull, j0full, kbfull, kc);
  cal_basis(nnode, ev->cal_j0, basis);
  std::vector<RowCal32> w32((size_t)M);
  for (int64_t k = 0; k < M; ++k)
    for (int i = 0; i < 4; ++i) w32[(size_t)k].w[i] = (float)w[(size_t)k * 4 + i];
  // TAB_PAD zero rows past the last bin: the bin loops request rows ahead of their bin
  w32.resize((size_t)(M + TAB_PAD));
  for (int64_t k = M; k < M + TAB_PAD; ++k)
    for (int i = 0; i < 4; ++i) w32[(size_t)k].w[i] = 0.0f;
  w.resize((size_t)(M + TAB_PAD) * 4, 0.0);
  tl.resize((size_t)(M + TAB_PAD), 0.0);
  std::vector<float> t32(tl.begin(), tl.end());
  hipError_t e = hipMalloc((void**)&ev->cal32, sizeof(RowCal32) * (M + TAB_PAD));
  if (e == hipSuccess) e = hipMalloc((void**)&ev->cal64, sizeof(RowCal64) * (M + TAB_PAD));
  if (e == hipSuccess) e = hipMalloc((void**)&ev->calt32, sizeof(float) * (M + TAB_PAD));
  if (e == hipSuccess) e = hipMalloc((void**)&ev->calt64, sizeof(double) * (M + TAB_PAD));
  if (e == hipSuccess) e = hipMalloc((void**)&ev->calB, sizeof(double) * basis.size());
  if (e == hipSuccess) e = hipMalloc((void**)&ev->kcal, sizeof(double) * kc.size());
  if (e == hipSuccess) e = hipMemcpy(ev->cal32, w32.data(), sizeof(RowCal32) * (M + TAB_PAD), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ev->cal64, w.data(), sizeof(RowCal64) * (M + TAB_PAD), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ev->calt32, t32.data(), sizeof(float) * (M + TAB_PAD), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ev->calt64, tl.data(), sizeof(double) * (M + TAB_PAD), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ev->calB, basis.data(), sizeof(double) * basis.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ev->kcal, kc.data(), sizeof(double) * kc.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "calibration tables");
  ev->ncal = nnode;
  return GWL_OK;
}

static gwl_status read_grid(const double* fgrid, const double* psd, int ndet, int64_t M, hipStream_t s,
                            std::vector<double>& fh, std::vector<double>& ph) {
  fh.resize((size_t)M);
  ph.resize((size_t)M * ndet);
  hipError_t e = hipMemcpyAsync(fh.data(), fgrid, sizeof(double) * M, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(ph.data(), psd, sizeof(double) * M * ndet, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "grid read-back");
  return GWL_OK;
}

}  // namespace gwl

extern "C" {

gwl_status gwl_event_create_cal(const double* data, const double* psd, const gwl_detector* dets, int ndet,
                                const double* fgrid, int64_t M, double df, double gmst, int nnode, unsigned flags,
                                void* stream, gwl_event* out) {
  clear_error();
  if (!out) return fail(GWL_E_INVALID, "out is null");
  *out = nullptr;
  if (nnode < 4 || nnode > MAXNODE) return fail(GWL_E_SHAPE, "nnode=%d outside [4, %d]", nnode, MAXNODE);
  if (flags & GWL_F_ISCO_CUTOFF)
    return fail(GWL_E_UNSUPPORTED, "the ISCO cut-off is not available with the calibration model");
  gwl_event ev = nullptr;
  gwl_status st = gwl_event_create(data, psd, dets, ndet, fgrid, M, df, gmst, flags, stream, &ev);
  if (st != GWL_OK) return st;
  std::vector<double> fh, ph;
  st = read_grid(fgrid, psd, ndet, M, (hipStream_t)stream, fh, ph);
  if (st == GWL_OK) st = attach_cal(ev, fh, fh, ph, nnode);
  if (st != GWL_OK) {
    gwl_event_destroy(ev);
    return st;
  }
  *out = ev;
  return GWL_OK;
}

gwl_status gwl_event_create_rb_cal(const double* data, const double* psd, const gwl_detector* dets, int ndet,
                                   const double* fgrid, int64_t M, double df, double gmst, const double* theta_fid,
                                   double eps, int nnode, unsigned flags, void* stream, gwl_event* out) {
  clear_error();
  if (!out) return fail(GWL_E_INVALID, "out is null");
  *out = nullptr;
  if (nnode < 4 || nnode > MAXNODE) return fail(GWL_E_SHAPE, "nnode=%d outside [4, %d]", nnode, MAXNODE);
  gwl_event ev = nullptr;
  gwl_status st = gwl_event_create_rb(data, psd, dets, ndet, fgrid, M, df, gmst, theta_fid, eps, flags, stream, &ev);
  if (st != GWL_OK) return st;
  std::vector<double> fh, ph;
  st = read_grid(fgrid, psd, ndet, M, (hipStream_t)stream, fh, ph);
  if (st == GWL_OK) {
    std::vector<double> fe(ev->rb_idx.size());
    for (size_t i = 0; i < fe.size(); ++i) fe[i] = fh[(size_t)ev->rb_idx[i]];
    st = attach_cal(ev, fe, fh, ph, nnode);
  }
  if (st != GWL_OK) {
    gwl_event_destroy(ev);
    return st;
  }
  *out = ev;
  return GWL_OK;
}

gwl_status gwl_event_destroy(gwl_event ev) {
  if (!ev) return GWL_OK;
  for (gwl_workspace& w : ev->ws) {
    if (w.ptr) (void)hipFree(w.ptr);
    if (w.cnt) (void)hipFree(w.cnt);
  }
  ev->ws.clear();
  if (ev->cal32) (void)hipFree(ev->cal32);
  if (ev->cal64) (void)hipFree(ev->cal64);
  if (ev->calt32) (void)hipFree(ev->calt32);
  if (ev->calt64) (void)hipFree(ev->calt64);
  if (ev->calB) (void)hipFree(ev->calB);
  if (ev->kcal) (void)hipFree(ev->kcal);
  if (ev->tab64) (void)hipFree(ev->tab64);
  if (ev->tab32) (void)hipFree(ev->tab32);
  if (ev->g32) (void)hipFree(ev->g32);
  if (ev->g64) (void)hipFree(ev->g64);
  if (ev->fgrid) (void)hipFree(ev->fgrid);
  if (ev->kcum) (void)hipFree(ev->kcum);
  if (ev->ec) (void)hipFree(ev->ec);
  delete ev;
  return GWL_OK;
}

gwl_status gwl_event_rb_info(gwl_event ev, int64_t* nedge, int64_t* nbins) {
  clear_error();
  if (!ev) return fail(GWL_E_INVALID, "event is null");
  if (nedge) *nedge = ev->M_full ? ev->M : 0;
  if (nbins) *nbins = ev->M_full ? ev->M_full : ev->M;
  return GWL_OK;
}

gwl_status gwl_event_info(gwl_event ev, int* ndet, int64_t* M, double* df) {
  clear_error();
  if (!ev) return fail(GWL_E_INVALID, "event is null");
  if (ndet) *ndet = ev->ndet;
  if (M) *M = ev->M;
  if (df) *df = ev->df;
  return GWL_OK;
}

// Calibrated evaluation: chunks are pieces of node intervals; workspace from the stream pool.
// ws_given: a workspace of ws_bytes bytes owned by the caller (a multi-event plan), used instead of
// the event's own workspace on s
static gwl_status run_logl_cal(gwl_event ev, const double* theta, int64_t B, bool mixed, bool grad, double* logl,
                               double* gradout, hipStream_t s, void* ws_given = nullptr, size_t ws_bytes = 0) {
  const int nd = ev->ndet, n = ev->ncal;
  CalShape sh;
  memset(&sh, 0, sizeof sh);
  sh.nnode = n;
  sh.npg = (int)((B + WAVE - 1) / WAVE);
  // chunks of about M / want bins, none crossing a node interval (intervals in ln f hold very
  // different numbers of bins, so each is cut into its own number of pieces)
  // forward: about six rounds of 8192 wavefronts (on the c1 shapes 48 chunks per point group, the
  // count the uncalibrated loop's tuning found best for its own chunked launch, which the calibrated
  // loop keeps; fewer left the chip's second round of wavefronts partly empty); adjoint: the
  // heuristic, since each of its chunks writes 11 N_det + 8 partial sums per point and more chunks
  // measured slower
  const int tuned = grad ? heuristic_nchunk(B, ev->M)
                         : (int)std::min<int64_t>(ev->M, (6 * 8192 + sh.npg - 1) / sh.npg);
  const int want = std::min(tuned, MAXCALCHUNK - (n - 1));
  const int64_t target = std::max<int64_t>(1, (ev->M + want - 1) / want);
  int nc = 0;
  for (int j = 0; j < n - 1; ++j) {
    const int64_t a = ev->cal_kb[j], len = ev->cal_kb[j + 1] - a;
    const int pieces = (int)std::max<int64_t>(1, (len + target - 1) / target);
    if (nc + pieces > MAXCALCHUNK) return fail(GWL_E_INTERNAL, "calibrated loop: too many chunks");
    for (int q = 0; q < pieces; ++q, ++nc) {
      sh.cj[nc] = j;
      sh.ck[nc] = (int)(a + len * q / pieces);
    }
  }
  sh.ck[nc] = (int)ev->M;
  sh.nchunk = nc;
  sh.nbpg = (sh.npg + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
  sh.items = sh.nchunk * sh.nbpg;
  sh.gper = (sh.items + NXCD - 1) / NXCD;
  for (int j = 0; j < n - 1; ++j) sh.j0[j] = ev->cal_j0[j];
  const int64_t Bp = (int64_t)sh.npg * WAVE;
  const int nchunk = sh.nchunk, ncal = 2 * n * nd;
  const size_t bytes = sizeof(double) * ((size_t)NCOEF * Bp + (size_t)ncal * Bp + (size_t)nchunk * nz_cal(nd, grad) * Bp);
  void* ws = ws_given;
  if (ws_given) {
    if (ws_bytes < bytes) return fail(GWL_E_INTERNAL, "calibrated loop: workspace of %zu bytes, %zu needed", ws_bytes, bytes);
  } else {
    gwl_status st = event_workspace(ev, s, bytes, 0, &ws);
    if (st != GWL_OK) return st;
  }
  double* coef = (double*)ws;
  double* calc = coef + (size_t)NCOEF * Bp;
  double* part = calc + (size_t)ncal * Bp;
  hipError_t e = launch_cal(nd, mixed, grad, ev->geom, ev->ec, ev->kcal, mixed ? ev->tab32 : ev->tab64,
                 mixed ? (const void*)ev->g32 : (const void*)ev->g64, mixed ? (const void*)ev->cal32 : (const void*)ev->cal64,
                 mixed ? (const void*)ev->calt32 : (const void*)ev->calt64, ev->calB, theta, NPARAM + ncal, B, Bp, sh,
                 coef, calc, part, logl, gradout, s);
  if (e != hipSuccess) return hip_fail(e, "launch");
  return GWL_OK;
}

static gwl_status logl_common(gwl_event ev, const double* theta, int64_t B, gwl_precision prec, double* logl,
                              double* grad, bool with_grad, void* stream) {
  clear_error();
  if (!ev) return fail(GWL_E_INVALID, "event is null");
  if (B < 0 || B > kMaxBatch) return fail(GWL_E_SHAPE, "B=%lld outside [0, %lld]", (long long)B, (long long)kMaxBatch);
  if (prec != GWL_FP64 && prec != GWL_MIXED) return fail(GWL_E_INVALID, "unknown precision %d", (int)prec);
  if (B == 0) return GWL_OK;
  if (!theta || !logl || (with_grad && !grad)) return fail(GWL_E_INVALID, "theta, logl%s must be device pointers",
                                                           with_grad ? " and grad" : "");
  gwl_status st = check_device(ev->device);
  if (st != GWL_OK) return st;
  const bool mixed = use_mixed(ev, prec);
  if (ev->ncal > 0) return run_logl_cal(ev, theta, B, mixed, with_grad, logl, grad, (hipStream_t)stream);
  const LoopShape sh = choose_shape(ev, B, mixed, with_grad);
  return run_logl(ev, theta, B, mixed, with_grad, sh, logl, grad, (hipStream_t)stream);
}

gwl_status gwl_logl_batch(gwl_event ev, const double* theta, int64_t B, gwl_precision prec, double* logl,
                          void* stream) {
  return logl_common(ev, theta, B, prec, logl, nullptr, false, stream);
}

gwl_status gwl_logl_batch_live(gwl_event ev, const double* theta, int64_t B, const int64_t* live, gwl_precision prec,
                               double* logl, void* stream) {
  clear_error();
  if (!ev) return fail(GWL_E_INVALID, "event is null");
  if (B < 0 || B > kMaxBatch) return fail(GWL_E_SHAPE, "B=%lld outside [0, %lld]", (long long)B, (long long)kMaxBatch);
  if (prec != GWL_FP64 && prec != GWL_MIXED) return fail(GWL_E_INVALID, "unknown precision %d", (int)prec);
  if (!live) return fail(GWL_E_INVALID, "live must be a device pointer");
  if (B == 0) return GWL_OK;
  if (!theta || !logl) return fail(GWL_E_INVALID, "theta and logl must be device pointers");
  if (ev->ncal > 0) return fail(GWL_E_UNSUPPORTED, "gwl_logl_batch_live does not take calibrated events");
  gwl_status st = check_device(ev->device);
  if (st != GWL_OK) return st;
  const bool mixed = use_mixed(ev, prec);
  // the shape for B, with at least enough workgroups per point group that a quarter of the point
  // groups still give every CU two workgroups (chunks of at least 32 bins): a partly live batch
  // then still fills the chip. The G workgroup sums go to the separate epilogue kernel (the
  // set-up in either kernel): at these workgroup counts the last-arriver's device-scope fences
  // cost more than the second launch (on c1 shapes with 8192 points, 240 against 196 us)
  LoopShape sh = choose_shape(ev, B, mixed, false);
  const int64_t want = (4 * 2 * 256 + sh.npg - 1) / sh.npg;
  const int64_t gcap = std::max<int64_t>(1, ev->M / (32 * (int64_t)sh.W));
  const int G = (int)std::min<int64_t>(std::max<int64_t>(sh.G, want), std::max<int64_t>(gcap, sh.G));
  sh = make_shape(B, ev->M, sh.W, G, sh.setup, 1);
  return run_logl(ev, theta, B, mixed, false, sh, logl, nullptr, (hipStream_t)stream, live);
}

gwl_status gwl_logl_grad(gwl_event ev, const double* theta, int64_t B, gwl_precision prec, double* logl, double* grad,
                         void* stream) {
  return logl_common(ev, theta, B, prec, logl, grad, true, stream);
}

gwl_status gwl_event_reserve(gwl_event ev, int64_t B, gwl_precision prec, int with_grad, void* stream) {
  clear_error();
  if (!ev) return fail(GWL_E_INVALID, "event is null");
  if (B < 0 || B > kMaxBatch) return fail(GWL_E_SHAPE, "B=%lld outside [0, %lld]", (long long)B, (long long)kMaxBatch);
  if (prec != GWL_FP64 && prec != GWL_MIXED) return fail(GWL_E_INVALID, "unknown precision %d", (int)prec);
  if (B == 0) return GWL_OK;
  gwl_status st = check_device(ev->device);
  if (st != GWL_OK) return st;
  void* ws = nullptr;
  const bool mixed = use_mixed(ev, prec), grad = with_grad != 0;
  const size_t ncnt = ev->ncal > 0 ? 0 : workspace_counters(choose_shape(ev, B, mixed, grad), grad);
  return event_workspace(ev, (hipStream_t)stream, call_workspace_bytes(ev, B, mixed, grad), ncnt, &ws);
}

gwl_status gwl_launch_shape(gwl_event ev, int64_t B, gwl_precision prec, int with_grad, int* nchunk,
                            int* chunk_bins) {
  clear_error();
  if (!ev) return fail(GWL_E_INVALID, "event is null");
  if (B < 1 || B > kMaxBatch) return fail(GWL_E_SHAPE, "B=%lld outside [1, %lld]", (long long)B, (long long)kMaxBatch);
  if (prec != GWL_FP64 && prec != GWL_MIXED) return fail(GWL_E_INVALID, "unknown precision %d", (int)prec);
  const LoopShape sh = choose_shape(ev, B, use_mixed(ev, prec), with_grad != 0);
  if (nchunk) *nchunk = sh.nchunk;
  if (chunk_bins) *chunk_bins = sh.chunk;
  return GWL_OK;
}

gwl_status gwl_launch_layout(gwl_event ev, int64_t B, gwl_precision prec, int with_grad, int* waves, int* groups,
                             int* setup) {
  clear_error();
  if (!ev) return fail(GWL_E_INVALID, "event is null");
  if (B < 1 || B > kMaxBatch) return fail(GWL_E_SHAPE, "B=%lld outside [1, %lld]", (long long)B, (long long)kMaxBatch);
  if (prec != GWL_FP64 && prec != GWL_MIXED) return fail(GWL_E_INVALID, "unknown precision %d", (int)prec);
  const LoopShape sh = choose_shape(ev, B, use_mixed(ev, prec), with_grad != 0);
  if (waves) *waves = sh.W;
  if (groups) *groups = sh.G;
  if (setup) *setup = sh.setup;
  return GWL_OK;
}

gwl_status gwl_waveform(const double* theta, int64_t B, const gwl_detector* dets, int ndet, const double* fgrid,
                        int64_t M, double gmst, double* out, void* stream) {
  clear_error();
  EventGeom g;
  gwl_status st = make_geom(dets, ndet, gmst, g);
  if (st != GWL_OK) return st;
  if (B < 0 || B > 65535) return fail(GWL_E_SHAPE, "B=%lld outside [0, 65535]", (long long)B);
  if (M < 1 || M > (int64_t)1 << 30) return fail(GWL_E_SHAPE, "M=%lld outside [1, 2^30]", (long long)M);
  if (B == 0) return GWL_OK;
  if (!theta || !fgrid || !out) return fail(GWL_E_INVALID, "theta, fgrid and out must be device pointers");
  hipStream_t s = (hipStream_t)stream;
  const int64_t Bp = (B + WAVE - 1) / WAVE * WAVE;
  double* coef = nullptr;
  hipError_t e = hipMallocAsync((void**)&coef, sizeof(double) * NCOEF * (size_t)Bp, s);
  if (e != hipSuccess) return hip_fail(e, "workspace");
  e = launch_setup(ndet, g, nullptr, false, theta, B, Bp, coef, s);
  if (e == hipSuccess) e = launch_waveform(ndet, g, coef, B, Bp, fgrid, M, out, s);
  hipError_t e2 = hipFreeAsync(coef, s);
  if (e != hipSuccess) return hip_fail(e, "waveform launch");
  if (e2 != hipSuccess) return hip_fail(e2, "workspace release");
  return GWL_OK;
}

}  // extern "C"

namespace gwl {

gwl_status run_calibrated(gwl_event ev, const double* theta, int64_t B, bool mixed, bool grad, double* logl,
                          double* gradout, hipStream_t s, void* ws, size_t ws_bytes) {
  return run_logl_cal(ev, theta, B, mixed, grad, logl, gradout, s, ws, ws_bytes);
}

// The set-up rows [NCOEF][Bp] come first unless the evaluation kernel makes them itself and
// nothing after it reads them (with the separate value epilogue it leaves that kernel's rows there)
static bool coef_in_workspace(const LoopShape& sh, bool grad) { return !sh.setup || (!grad && sh.G > 1 && sh.sepepi); }

size_t workspace_bytes(int64_t Bp, const LoopShape& sh, int nd, bool grad) {
  const size_t coef = coef_in_workspace(sh, grad) ? (size_t)NCOEF * Bp : 0;
  const size_t part = (grad || sh.G > 1) ? (size_t)sh.G * nz_of(nd, grad) * Bp : 0;
  return sizeof(double) * (coef + part);
}

size_t workspace_counters(const LoopShape& sh, bool grad) {
  return (!grad && sh.G > 1 && !sh.sepepi) ? (size_t)sh.npg : 0;
}

// Set-up, bin loop and epilogue on `s`, in the event's workspace for `s`.
gwl_status run_logl(gwl_event ev, const double* theta, int64_t B, bool mixed, bool grad, const LoopShape& sh,
                    double* logl, double* gradout, hipStream_t s, const int64_t* live) {
  const int64_t Bp = (int64_t)sh.npg * WAVE;
  void* ws = nullptr;
  unsigned int* cnt = nullptr;
  gwl_status st = event_workspace(ev, s, workspace_bytes(Bp, sh, ev->ndet, grad), workspace_counters(sh, grad), &ws,
                                  &cnt);
  if (st != GWL_OK) return st;
  hipError_t e = enqueue_logl(ev, theta, B, mixed, grad, sh, (double*)ws, cnt, logl, gradout, s, live);
  if (e != hipSuccess) return hip_fail(e, "launch");
  return GWL_OK;
}

gwl_status event_workspace(gwl_event ev, hipStream_t s, size_t bytes, size_t ncnt, void** out, unsigned int** cnt) {
  *out = nullptr;
  if (cnt) *cnt = nullptr;
  std::lock_guard<std::mutex> lk(ev->ws_mu);
  gwl_workspace* w = nullptr;
  for (gwl_workspace& x : ev->ws)
    if (x.stream == s) w = &x;
  if (w && w->bytes >= bytes && w->ncnt >= ncnt) {
    *out = w->ptr;
    if (cnt) *cnt = w->cnt;
    return GWL_OK;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &cs);
  if (e != hipSuccess) return hip_fail(e, "stream capture status");
  if (cs != hipStreamCaptureStatusNone)
    return fail(GWL_E_INVALID, "the call needs %zu bytes of workspace on a stream that is capturing a graph and has %zu: "
                               "reserve it first (gwl_event_reserve, or one call of this size on that stream outside "
                               "capture)", bytes, w ? w->bytes : (size_t)0);
  if (!w) {
    ev->ws.push_back(gwl_workspace{});
    w = &ev->ws.back();
    w->stream = s;
  }
  const size_t grain = (size_t)2 << 20;
  const size_t nb = std::max(w->bytes, (bytes + grain - 1) / grain * grain);
  const size_t nc = std::max(w->ncnt, (ncnt + 1023) / 1024 * 1024);
  void* p = w->ptr;
  unsigned int* c = w->cnt;
  if (nb > w->bytes) {
    e = hipMalloc(&p, nb);
    if (e != hipSuccess) return hip_fail(e, "workspace");
  }
  if (nc > w->ncnt) {
    e = hipMalloc((void**)&c, nc * sizeof(unsigned int));
    // the kernels leave their counters at zero; a new array starts there
    if (e == hipSuccess) e = hipMemsetAsync(c, 0, nc * sizeof(unsigned int), s);
  }
  // buffers being replaced may still be in use by work queued on s
  const bool replace_ptr = p != w->ptr && w->ptr, replace_cnt = c != w->cnt && w->cnt;
  if (e == hipSuccess && (replace_ptr || replace_cnt)) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    if (p != w->ptr) (void)hipFree(p);
    if (c != w->cnt && c) (void)hipFree(c);
    return hip_fail(e, "workspace");
  }
  if (replace_ptr) (void)hipFree(w->ptr);
  if (replace_cnt) (void)hipFree(w->cnt);
  w->ptr = p;
  w->bytes = nb;
  w->cnt = c;
  w->ncnt = nc;
  *out = p;
  if (cnt) *cnt = c;
  return GWL_OK;
}

size_t call_workspace_bytes(const gwl_event_s* ev, int64_t B, bool mixed, bool grad) {
  const int64_t Bp = (B + WAVE - 1) / WAVE * WAVE;
  if (ev->ncal > 0) {
    // the calibrated loop uses at most MAXCALCHUNK chunks and 2 nnode nd calibration rows
    return sizeof(double) * ((size_t)NCOEF * Bp + (size_t)2 * ev->ncal * ev->ndet * Bp +
                             (size_t)MAXCALCHUNK * nz_cal(ev->ndet, grad) * Bp);
  }
  return workspace_bytes(Bp, choose_shape(ev, B, mixed, grad), ev->ndet, grad);
}

// ---- bin-loop timing (gwl_profile_*) ----
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_events;

static bool prof_begin(hipStream_t s, hipEvent_t& a, hipEvent_t& b) {
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return false;
  }
  if (hipEventCreate(&a) != hipSuccess) return false;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return false;
  }
  (void)hipEventRecord(a, s);
  return true;
}

static void prof_end(hipStream_t s, hipEvent_t a, hipEvent_t b) {
  (void)hipEventRecord(b, s);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_events.emplace_back(a, b);
}

hipError_t enqueue_logl(gwl_event ev, const double* theta, int64_t B, bool mixed, bool grad, const LoopShape& sh,
                        double* ws, unsigned int* cnt, double* logl, double* gradout, hipStream_t s,
                        const int64_t* live) {
  const int64_t Bp = (int64_t)sh.npg * WAVE;
  const bool with_coef = coef_in_workspace(sh, grad);
  double* coef = with_coef ? ws : nullptr;
  double* part = (grad || sh.G > 1) ? ws + (with_coef ? (size_t)NCOEF * Bp : 0) : nullptr;
  hipError_t e = hipSuccess;
  if (!sh.setup) e = launch_setup(ev->ndet, ev->geom, ev->ec, mixed, theta, B, Bp, coef, s);
  hipEvent_t pa = nullptr, pb = nullptr;
  const bool prof = e == hipSuccess && prof_begin(s, pa, pb);
  if (e == hipSuccess)
    e = launch_eval(ev->ndet, mixed, grad, ev->ech.uniform != 0, mixed ? ev->tab32 : ev->tab64, ev->g64, theta,
                    ev->geom, ev->ec, coef, B, Bp, ev->M, sh, part, cnt, logl, ev->fgrid, ev->kcum, live, s);
  // the value's reduction over the G workgroups in its own kernel (timed with the evaluation)
  if (e == hipSuccess && !grad && sh.G > 1 && sh.sepepi)
    e = launch_value_epilogue(ev->ndet, mixed, ev->ec, theta, coef, B, Bp, sh.G, part, logl, ev->fgrid, ev->kcum,
                              ev->M, live, s);
  if (prof) prof_end(s, pa, pb);
  if (e == hipSuccess && grad)
    e = launch_epilogue(ev->ndet, true, mixed, ev->geom, ev->ec, theta, coef, B, Bp, sh.G, part, logl, gradout, s,
                        ev->fgrid, ev->kcum, ev->M);
  return e;
}

}  // namespace gwl

extern "C" {

gwl_status gwl_profile_enable(int on) {
  clear_error();
  std::lock_guard<std::mutex> lk(gwl::g_prof_mu);
  gwl::g_prof_on = on != 0;
  return GWL_OK;
}

gwl_status gwl_profile_read(int64_t* launches, double* total_ms) {
  clear_error();
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  {
    std::lock_guard<std::mutex> lk(gwl::g_prof_mu);
    ev.swap(gwl::g_prof_events);
  }
  double tot = 0.0;
  hipError_t err = hipSuccess;
  for (auto& p : ev) {
    hipError_t e = hipEventSynchronize(p.second);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.first, p.second);
    if (e == hipSuccess) tot += ms;
    else if (err == hipSuccess) err = e;
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  if (launches) *launches = (int64_t)ev.size();
  if (total_ms) *total_ms = tot;
  if (err != hipSuccess) return hip_fail(err, "profile read");
  return GWL_OK;
}

}  // extern "C"
