// Device-side model of one parameter point: TaylorF2 phase coefficients, amplitude,
// detector projection and time delays, written once as templates over the scalar type so
// that the same code gives plain float64 values (per-point set-up) or forward-mode
// derivatives (gradient epilogue).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gwl_common.h"

namespace gwl {

// ---------------------------------------------------------------------------------------------
// Physical constants (SI) of the library's conventions.
// ---------------------------------------------------------------------------------------------
constexpr double kC = 299792458.0;               // m/s
constexpr double kTsun = 4.925490947641267e-6;   // G Msun / c^3, s
constexpr double kMpc = 3.0856775814913673e22;   // m
constexpr double kGammaE = 0.5772156649015329;
constexpr double kPi = 3.141592653589793;
constexpr double kTwoPi = 6.283185307179586;

// ---------------------------------------------------------------------------------------------
// Forward-mode dual numbers: value plus N partial derivatives.
// ---------------------------------------------------------------------------------------------
template <int N>
struct Dual {
  double v;
  double d[N];
};

template <int N>
__device__ inline Dual<N> dcst(double x) {
  Dual<N> r;
  r.v = x;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = 0.0;
  return r;
}
template <int N>
__device__ inline Dual<N> dvar(double x, int i) {
  Dual<N> r = dcst<N>(x);
  r.d[i] = 1.0;
  return r;
}
template <int N>
__device__ inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int N>
__device__ inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int N>
__device__ inline Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r; r.v = -a.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int N>
__device__ inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int N>
__device__ inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v / b.v;
  const double ib = 1.0 / b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
  return r;
}
template <int N> __device__ inline Dual<N> operator+(const Dual<N>& a, double b) { Dual<N> r = a; r.v += b; return r; }
template <int N> __device__ inline Dual<N> operator+(double b, const Dual<N>& a) { return a + b; }
template <int N> __device__ inline Dual<N> operator-(const Dual<N>& a, double b) { Dual<N> r = a; r.v -= b; return r; }
template <int N> __device__ inline Dual<N> operator-(double b, const Dual<N>& a) { return -a + b; }
template <int N>
__device__ inline Dual<N> operator*(const Dual<N>& a, double b) {
  Dual<N> r; r.v = a.v * b;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
  return r;
}
template <int N> __device__ inline Dual<N> operator*(double b, const Dual<N>& a) { return a * b; }
template <int N> __device__ inline Dual<N> operator/(const Dual<N>& a, double b) { return a * (1.0 / b); }
template <int N>
__device__ inline Dual<N> operator/(double a, const Dual<N>& b) {
  Dual<N> r; r.v = a / b.v;
  const double s = -r.v / b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = s * b.d[i];
  return r;
}
// chain rule helper: f(a) with f'(a) = g
template <int N>
__device__ inline Dual<N> dchain(const Dual<N>& a, double fv, double g) {
  Dual<N> r; r.v = fv;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = g * a.d[i];
  return r;
}

// Elementary functions for double and Dual<N>.
__device__ inline double xsin(double a) { return sin(a); }
__device__ inline double xcos(double a) { return cos(a); }
__device__ inline double xlog(double a) { return log(a); }
__device__ inline double xsqrt(double a) { return sqrt(a); }
__device__ inline double xpow(double a, double p) { return pow(a, p); }
__device__ inline double val(double a) { return a; }
template <int N> __device__ inline Dual<N> xsin(const Dual<N>& a) { return dchain(a, sin(a.v), cos(a.v)); }
template <int N> __device__ inline Dual<N> xcos(const Dual<N>& a) { return dchain(a, cos(a.v), -sin(a.v)); }
template <int N> __device__ inline Dual<N> xlog(const Dual<N>& a) { return dchain(a, log(a.v), 1.0 / a.v); }
template <int N> __device__ inline Dual<N> xsqrt(const Dual<N>& a) { double s = sqrt(a.v); return dchain(a, s, 0.5 / s); }
template <int N> __device__ inline Dual<N> xpow(const Dual<N>& a, double p) {
  double fv = pow(a.v, p);
  return dchain(a, fv, p * fv / a.v);
}
template <int N> __device__ inline double val(const Dual<N>& a) { return a.v; }

// ---------------------------------------------------------------------------------------------
// One parameter point, as the bin loop and the epilogue need it.
//
// Phase in cycles, split into a per-bin part and a constant:
//   Psi(f)/(2 pi) = f t_c + sum_m a_m g_m(f) + c0,
//   g = { f^-5/3, f^-1, f^-2/3, f^-1/3, ln f, f^1/3, f^1/3 ln f, f^2/3 }
// which is the TaylorF2 series 3/(128 eta v^5) sum_k phi_k v^k with v^3 = pi M f regrouped by
// powers of f (the ln v of the 2.5PN and 3PN terms split into ln(pi M) and ln f).
// Per detector: T_det = t_c + dt_det; projection factor Q_det = F+ (1+cos^2 i)/2 - i Fx cos i.
// ---------------------------------------------------------------------------------------------
template <class T>
struct PointModel {
  T a[NBASIS];
  T c0;
  T amp;
  T qr[MAXDET], qi[MAXDET];
  T tdet[MAXDET];
  bool valid;
};

// The model splits into an intrinsic half (masses, spins, distance, phase: a_m, c0, A and the
// domain check) and an extrinsic half (sky position, orientation, time: T_det and Q_det), which
// the in-kernel set-up runs on two wavefronts at once.
template <class T>
__device__ inline void point_intrinsic(const T th[NPARAM], PointModel<T>& pm) {
  const T& mc = th[0];
  const T& q = th[1];
  const T& chi1 = th[2];
  const T& chi2 = th[3];
  const T& dl = th[4];
  const T& phic = th[9];

  const double qv = val(q), mcv = val(mc), dlv = val(dl), c1 = val(chi1), c2 = val(chi2);
  bool ok = (qv > 0.0) && (qv <= 1.0) && (mcv > 0.0) && (dlv > 0.0) && (fabs(c1) < 1.0) && (fabs(c2) < 1.0);
#pragma unroll
  for (int i = 0; i < NPARAM; ++i) ok = ok && isfinite(val(th[i]));
  pm.valid = ok;

  const T onepq = q + 1.0;
  const T eta = q / (onepq * onepq);
  const T mtot = mc * xpow(eta, -0.6);
  const T x1 = 1.0 / onepq;  // m1 / M
  const T x2 = q / onepq;    // m2 / M
  const T beta = (113.0 / 12.0 * x1 * x1 + 25.0 / 4.0 * eta) * chi1 + (113.0 / 12.0 * x2 * x2 + 25.0 / 4.0 * eta) * chi2;
  const T sigma = (79.0 / 8.0) * eta * chi1 * chi2;
  const T eta2 = eta * eta;
  const T phi2 = 3715.0 / 756.0 + 55.0 / 9.0 * eta;
  const T phi3 = -16.0 * kPi + 4.0 * beta;
  const T phi4 = 15293365.0 / 508032.0 + 27145.0 / 504.0 * eta + 3085.0 / 72.0 * eta2 - 10.0 * sigma;
  const T c5 = kPi * (38645.0 / 756.0 - 65.0 / 9.0 * eta);
  const T a6c = 11583231236531.0 / 4694215680.0 - 640.0 / 3.0 * kPi * kPi - 6848.0 / 21.0 * kGammaE +
                (-15737765635.0 / 3048192.0 + 2255.0 / 12.0 * kPi * kPi) * eta + 76055.0 / 1728.0 * eta2 -
                127825.0 / 1296.0 * eta2 * eta;
  const T phi7 = kPi * (77096675.0 / 254016.0 + 378515.0 / 1512.0 * eta - 74045.0 / 756.0 * eta2);

  const T pmass = (kPi * kTsun) * mtot;  // pi M in seconds
  const T lpm = xlog(pmass);
  const T p13 = xpow(pmass, 1.0 / 3.0);
  const T pm13 = 1.0 / p13;
  const T pm23 = pm13 * pm13;
  const T pref = 3.0 / (256.0 * kPi) / eta;  // 3/(128 eta) per radian, in cycles
  pm.a[0] = pref * pm23 * pm23 * pm13;      // f^-5/3
  pm.a[1] = pref * phi2 / pmass;            // f^-1
  pm.a[2] = pref * phi3 * pm23;             // f^-2/3
  pm.a[3] = pref * phi4 * pm13;             // f^-1/3
  pm.a[4] = pref * c5;                      // ln f
  pm.a[5] = pref * p13 * (a6c - 6848.0 / 21.0 * (1.3862943611198906 + lpm * (1.0 / 3.0)));  // f^1/3
  pm.a[6] = pref * p13 * (-6848.0 / 63.0);  // f^1/3 ln f
  pm.a[7] = pref * phi7 * p13 * p13;        // f^2/3
  pm.c0 = pref * c5 * (1.0 + lpm) - (phic + kPi / 4.0) * (1.0 / kTwoPi);

  pm.amp = 0.45643546458763845 * 0.46619407703541166 * xpow(kTsun * mc, 5.0 / 6.0) * (kC / kMpc) / dl;
}

template <class T, int ND>
__device__ inline void point_extrinsic(const T th[NPARAM], const EventGeom& g, PointModel<T>& pm) {
  const T& ra = th[5];
  const T& dec = th[6];
  const T& inc = th[7];
  const T& psi = th[8];
  const T& tc = th[10];

  // polarisation basis of the source at (ra - gmst, dec), rotated by psi
  const T h = ra - g.gmst;
  const T ch = xcos(h), sh = xsin(h), cd = xcos(dec), sd = xsin(dec);
  const T cp = xcos(psi), sp = xsin(psi);
  const T k0 = cd * ch, k1 = cd * sh, k2 = sd;
  const T u0 = -(sd * ch), u1 = -(sd * sh), u2 = cd;
  const T v0 = -sh, v1 = ch;
  const T X0 = cp * u0 + sp * v0, X1 = cp * u1 + sp * v1, X2 = cp * u2;
  const T Y0 = cp * v0 - sp * u0, Y1 = cp * v1 - sp * u1, Y2 = -(sp * u2);
  const T ci = xcos(inc);
  const T fpl = 0.5 * (1.0 + ci * ci);
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    // D symmetric: (xx, yy, zz, xy, xz, yz)
    const double* D = g.dt[d];
    const T fp = D[0] * (X0 * X0 - Y0 * Y0) + D[1] * (X1 * X1 - Y1 * Y1) + D[2] * (X2 * X2 - Y2 * Y2) +
                 2.0 * (D[3] * (X0 * X1 - Y0 * Y1) + D[4] * (X0 * X2 - Y0 * Y2) + D[5] * (X1 * X2 - Y1 * Y2));
    const T fx = 2.0 * (D[0] * X0 * Y0 + D[1] * X1 * Y1 + D[2] * X2 * Y2) +
                 2.0 * (D[3] * (X0 * Y1 + X1 * Y0) + D[4] * (X0 * Y2 + X2 * Y0) + D[5] * (X1 * Y2 + X2 * Y1));
    pm.qr[d] = fp * fpl;
    pm.qi[d] = -(fx * ci);
    const double* r = g.r[d];
    pm.tdet[d] = tc - (r[0] * k0 + r[1] * k1 + r[2] * k2) * (1.0 / kC);
  }
}

template <class T, int ND>
__device__ inline void point_model(const T th[NPARAM], const EventGeom& g, PointModel<T>& pm) {
  point_intrinsic<T>(th, pm);
  point_extrinsic<T, ND>(th, g, pm);
}

// ---------------------------------------------------------------------------------------------
// sin(2 pi t), cos(2 pi t) in float64 for any t (cycles). Reduction to a quarter cycle
// around the nearest multiple of 1/4, then Taylor polynomials of sin and cos of
// 2 pi y, |y| <= 1/8 (|angle| <= pi/4), truncated where the next term is below 1e-18.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void sincos_cycles_f64(double t, double& s, double& c) {
  const double qd = rint(4.0 * t);
  const double y = fma(qd, -0.25, t);  // exact: |y| <= 1/8
  const int qi = (int)(int64_t)qd;
  const double z = y * y;
  // sin(2 pi y) = sum_n (-1)^n (2 pi)^(2n+1) y^(2n+1) / (2n+1)!,  n = 0..8
  double ps = 0.10422916220813984;
  ps = fma(ps, z, -0.7181223017785006);
  ps = fma(ps, z, 3.819952584848282);
  ps = fma(ps, z, -15.09464257682299);
  ps = fma(ps, z, 42.058693944897655);
  ps = fma(ps, z, -76.70585975306139);
  ps = fma(ps, z, 81.60524927607506);
  ps = fma(ps, z, -41.34170224039976);
  ps = fma(ps, z, 6.283185307179586);
  const double sv = ps * y;
  // cos(2 pi y) = sum_n (-1)^n (2 pi)^(2n) y^(2n) / (2n)!,  n = 0..8
  double pc = 0.28200596845579123;
  pc = fma(pc, z, -1.714390711088672);
  pc = fma(pc, z, 7.903536371318469);
  pc = fma(pc, z, -26.4262567833744);
  pc = fma(pc, z, 60.24464137187666);
  pc = fma(pc, z, -85.45681720669373);
  pc = fma(pc, z, 64.9393940226683);
  pc = fma(pc, z, -19.739208802178716);
  pc = fma(pc, z, 1.0);
  const double cv = pc;
  // rotate by qi quarter turns
  const bool swap = qi & 1;
  const double S = swap ? cv : sv;
  const double C = swap ? sv : cv;
  s = (qi & 2) ? -S : S;
  c = ((qi + 1) & 2) ? -C : C;
}

}  // namespace gwl
