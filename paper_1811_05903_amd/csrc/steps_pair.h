// Pair-weight helpers of libsteps' force kernels (device code): the
// softened force of Sec. 2.2, Eq. 4, divided by r, and the compensated
// running sum.  Included by the open and the periodic pair kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace steps {
namespace {

// ---------------------------------------------------------------------------
// FP64 pair weight, Newtonian branch (r >= h): w = m r^-3.  v_rsq_f64 gives
// y ~ r^-1 to about 2^-24 (measured on gfx950); with e = 1 - r2 y^2,
//   r^-3 = y^3 (1 - e)^(-3/2) = y^3 (1 + 3/2 e + 15/8 e^2 + O(e^3)).
// E2 = true keeps the e^2 term (residual below 2^-68).  E2 = false stops at
// the linear term: the residual 15/8 e^2 is at most ~2e-14 relative per
// pair and about 1e-15 on average, and the weight costs one accumulate-form
// FMA with a literal instead of a two-constant polynomial.
// ---------------------------------------------------------------------------
template <bool E2>
__device__ __forceinline__ double newton_w64(double r2, double m) {
  double y = __builtin_amdgcn_rsq(r2);
  double y2 = y * y;
  double e = fma(-r2, y2, 1.0);
  double t = (m * y) * y2;
  if (E2) return t * fma(e, fma(e, 1.875, 1.5), 1.0);
  return fma(t * e, 1.5, t);
}

// Softened branch of Eq. 4 divided by r, with u = r/h (h = h_i + h_j):
//   u < 1/2      : (1/h^3) (32/3 - 38.4 u^2 + 32 u^3)
//   1/2 <= u < 1 : (1/h^3) (64/3 - 48 u + 38.4 u^2 - 32/3 u^3) - 1/(15 r^3)
// Zero separation contributes nothing (the j != i exclusion of Eq. 8).
// Only reached when r2 <= h^2, so h > 0 whenever r2 > 0.
__device__ __noinline__ double soft_w64(double r2, double h, double m) {
  if (r2 == 0.0) return 0.0;
  double y = __builtin_amdgcn_rsq(r2);
  double e = fma(-r2, y * y, 1.0);
  // r^-1 = y (1 - e)^(-1/2) = y (1 + e/2 + 3/8 e^2 + ...)
  double rinv = y * fma(e, fma(e, 0.375, 0.5), 1.0);
  double r = r2 * rinv;
  double hinv = 1.0 / h;
  double u = r * hinv;
  double hinv3 = hinv * hinv * hinv;
  if (u < 0.5) {
    return m * hinv3 * fma(u * u, fma(32.0, u, -38.4), 32.0 / 3.0);
  }
  double p = fma(u, fma(u, fma(u, -32.0 / 3.0, 38.4), -48.0), 64.0 / 3.0);
  return m * fma(hinv3, p, -(rinv * rinv * rinv) * (1.0 / 15.0));
}

[[maybe_unused]] __device__ __noinline__ float soft_w32(float r2, float h, float m) {
  if (r2 == 0.0f) return 0.0f;
  float rinv = __builtin_amdgcn_rsqf(r2);
  float r = r2 * rinv;
  float hinv = 1.0f / h;
  float u = r * hinv;
  float hinv3 = hinv * hinv * hinv;
  if (u < 0.5f) {
    return m * hinv3 * fmaf(u * u, fmaf(32.0f, u, -38.4f), 32.0f / 3.0f);
  }
  float p = fmaf(u, fmaf(u, fmaf(u, -32.0f / 3.0f, 38.4f), -48.0f), 64.0f / 3.0f);
  return m * fmaf(hinv3, p, -(rinv * rinv * rinv) * (1.0f / 15.0f));
}

// s + c += x with the rounding error of the addition kept in c (Knuth's
// TwoSum, branch-free).  Used to add each tile's partial into the running
// total: in spatial order the running sum can pass through values far
// larger than the final one (the pull of one side of a particle arrives
// before the other side's), and plain addition would lose ~1e-12 of it.
__device__ __forceinline__ void two_sum_add(double &s, double &c, double x) {
  const double t = s + x;
  const double bp = t - s;
  c += (s - (t - bp)) + (x - bp);
  s = t;
}

}  // namespace
}  // namespace steps
