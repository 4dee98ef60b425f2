// Unit cube -> parameters for a sampler above the likelihood: nested sampling draws its points
// uniformly in the unit cube and maps them through the prior's inverse CDF (the prior-sampling
// step of static nested sampling, section 2). Priors whose columns are independent and whose
// inverse CDFs take the form g(c0 + c1 u) are covered: g the identity (uniform), the cube root
// (density ~ x^2, e.g. distance), asin (density ~ cos x, e.g. declination) and acos (density
// ~ sin x, e.g. inclination). One thread per element; the column's map and coefficients come
// in the kernel's argument block.
#include <hip/hip_runtime.h>

#include "gwl_runtime.h"

namespace gwl {

constexpr int PRIOR_BLOCK = 256;

struct PriorCols {
  int map[GWL_PRIOR_MAX_DIM];
  double c0[GWL_PRIOR_MAX_DIM];
  double c1[GWL_PRIOR_MAX_DIM];
};

__global__ __launch_bounds__(PRIOR_BLOCK) void k_prior_transform(int64_t total, int d, PriorCols cols,
                                                                 const double* __restrict__ u,
                                                                 double* __restrict__ theta) {
  const int64_t e = (int64_t)blockIdx.x * PRIOR_BLOCK + threadIdx.x;
  if (e >= total) return;
  const int j = (int)(e % d);
  const double v = fmin(fmax(u[e], 0.0), 1.0);
  const double x = fma(cols.c1[j], v, cols.c0[j]);
  double y;
  switch (cols.map[j]) {
    case GWL_MAP_CBRT: y = cbrt(x); break;
    case GWL_MAP_ASIN: y = asin(fmin(fmax(x, -1.0), 1.0)); break;
    case GWL_MAP_ACOS: y = acos(fmin(fmax(x, -1.0), 1.0)); break;
    default: y = x; break;
  }
  theta[e] = y;
}

}  // namespace gwl

using namespace gwl;

extern "C" {

gwl_status gwl_prior_transform(int64_t n, int d, const int* map, const double* c0, const double* c1, const double* u,
                               double* theta, void* stream) {
  clear_error();
  if (n < 1 || n > kMaxBatch || d < 1 || d > GWL_PRIOR_MAX_DIM)
    return fail(GWL_E_SHAPE, "n=%lld, d=%d outside [1, 2^30] x [1, %d]", (long long)n, d, GWL_PRIOR_MAX_DIM);
  if (!map || !c0 || !c1 || !u || !theta) return fail(GWL_E_INVALID, "gwl_prior_transform: null pointer");
  PriorCols cols;
  for (int j = 0; j < d; ++j) {
    if (map[j] < GWL_MAP_LINEAR || map[j] > GWL_MAP_ACOS)
      return fail(GWL_E_INVALID, "column %d: unknown map %d", j, map[j]);
    cols.map[j] = map[j];
    cols.c0[j] = c0[j];
    cols.c1[j] = c1[j];
  }
  for (int j = d; j < GWL_PRIOR_MAX_DIM; ++j) {
    cols.map[j] = GWL_MAP_LINEAR;
    cols.c0[j] = cols.c1[j] = 0.0;
  }
  const int64_t total = n * d;
  hipLaunchKernelGGL(k_prior_transform, dim3((unsigned)((total + PRIOR_BLOCK - 1) / PRIOR_BLOCK)), dim3(PRIOR_BLOCK), 0,
                     (hipStream_t)stream, total, d, cols, u, theta);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? GWL_OK : hip_fail(e, "gwl_prior_transform");
}

}  // extern "C"
