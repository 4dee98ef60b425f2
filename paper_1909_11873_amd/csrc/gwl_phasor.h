// The float64 phasor table e^{2 pi i k / N}, k = 0..N-1, built by the compiler: each entry from
// the quadrant q = rint(4 k / N) and y = k / N - q / 4 in [-1/8, 1/8] (exact, N a power of two),
// sin and cos of 2 pi y by their Taylor series (|2 pi y| <= pi / 4; the series stop where the
// next term is below 1e-20), then the quarter turn q. Every workgroup of the float64 kernels
// copies it into LDS; it is not recomputed on the device.
#pragma once

#include <hip/hip_runtime.h>

namespace gwl {

struct PhasorEntry {
  double c, s;
};

template <int N>
struct PhasorTable {
  PhasorEntry e[N];
};

constexpr void taylor_sincos_2pi(double y, double& s, double& c) {
  const double th = 6.283185307179586 * y;
  const double z = th * th;
  // sin th = th (1 - z/3! + z^2/5! - ...), cos th = 1 - z/2! + z^2/4! - ..., Horner from the
  // 21st and 20th orders down
  double ps = 0.0, pc = 0.0;
  for (int n = 10; n >= 1; --n) {
    ps = (1.0 - ps * z / ((2.0 * n + 2.0) * (2.0 * n + 3.0)));
    pc = (1.0 - pc * z / ((2.0 * n + 1.0) * (2.0 * n + 2.0)));
  }
  s = th * (1.0 - ps * z / 6.0);
  c = 1.0 - pc * z / 2.0;
}

template <int N>
constexpr PhasorTable<N> make_phasor_table() {
  PhasorTable<N> t{};
  for (int k = 0; k < N; ++k) {
    const int q = (4 * k + N / 2) / N;  // rint(4 k / N), halves rounded up (4 k / N is never a half)
    const double y = (double)(k - q * (N / 4)) / N;
    double s = 0.0, c = 0.0;
    taylor_sincos_2pi(y, s, c);
    switch (q & 3) {
      case 0: t.e[k] = {c, s}; break;
      case 1: t.e[k] = {-s, c}; break;
      case 2: t.e[k] = {-c, -s}; break;
      default: t.e[k] = {s, -c}; break;
    }
  }
  return t;
}

}  // namespace gwl
