// gfx950 kernels of libsteps other than the pair sum: the softened
// potential (a diagnostic, derived from the kernel of Racz et al. 2018,
// Sec. 2.2 Eq. 4), and the O(N) kick / drift / conversion / reduction
// kernels of the KDK leapfrog (Sec. 2.3 Eqs. 9-11).  The pair-sum kernels
// are in steps_force.hip, the spatial sort in steps_sort.hip.

#include <algorithm>

#include "steps_internal.h"

namespace steps {
namespace {

// ---------------------------------------------------------------------------
// Softened potential, FP64: phi = -1/r for r >= h, else
//   u < 1/2      : (1/h) (-2.8 + 16/3 u^2 - 9.6 u^4 + 6.4 u^5)
//   1/2 <= u < 1 : (1/h) (-3.2 + 1/(15u) + 32/3 u^2 - 16 u^3 + 9.6 u^4
//                          - 32/15 u^5)
// (the integral of Eq. 4 with phi(inf) = 0).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rinv64(double r2) {
  double y = __builtin_amdgcn_rsq(r2);
  double e = fma(-r2, y * y, 1.0);
  return y * fma(e, fma(e, 0.375, 0.5), 1.0);
}

__device__ __noinline__ double soft_phi64(double r2, double h, double m) {
  if (r2 == 0.0) return 0.0;
  double rinv = rinv64(r2);
  double r = r2 * rinv;
  double hinv = 1.0 / h;
  double u = r * hinv;
  double u2 = u * u;
  if (u < 0.5) {
    // -2.8 + u^2 (16/3 + u^2 (-9.6 + 6.4 u))
    return m * hinv * fma(u2, fma(u2, fma(6.4, u, -9.6), 16.0 / 3.0), -2.8);
  }
  // -3.2 + 1/(15u) + u^2 (32/3 + u (-16 + u (9.6 - 32/15 u)))
  double p = fma(u2, fma(u, fma(u, fma(-32.0 / 15.0, u, 9.6), -16.0), 32.0 / 3.0), -3.2);
  return m * (hinv * p + rinv * (1.0 / 15.0));
}

template <int R, int TJ>
__global__ __launch_bounds__(kBlock) void k_potential_f64(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const double *__restrict__ soft, int n, int jchunk,
    double *__restrict__ out) {
  __shared__ double2 tile[3 * TJ];
  const int tid = threadIdx.x;
  const int ibase = blockIdx.x * (kBlock * R) + tid;
  const int jbeg = blockIdx.y * jchunk;
  const int jend = min(n, jbeg + jchunk);
  const double *X = pos, *Y = pos + n, *Z = pos + 2 * (size_t)n;
  double xi[R], yi[R], zi[R], hi[R], acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = ibase + r * kBlock;
    const bool ok = i < n;
    xi[r] = ok ? X[i] : 0.0;
    yi[r] = ok ? Y[i] : 0.0;
    zi[r] = ok ? Z[i] : 0.0;
    hi[r] = ok ? soft[i] : 0.0;
    acc[r] = 0.0;
  }
  for (int jt = jbeg; jt < jend; jt += TJ) {
    __syncthreads();
    for (int k = tid; k < TJ; k += kBlock) {
      const int j = jt + k;
      double2 a = {0.0, 0.0}, b = {0.0, 0.0}, c = {0.0, 0.0};
      if (j < jend) {
        a = double2{X[j], Y[j]};
        b = double2{Z[j], soft[j]};
        c = double2{mass[j], 0.0};
      }
      tile[3 * k] = a;
      tile[3 * k + 1] = b;
      tile[3 * k + 2] = c;
    }
    __syncthreads();
    double t[R];
#pragma unroll
    for (int r = 0; r < R; ++r) t[r] = 0.0;
    for (int k = 0; k < TJ; ++k) {
      const double2 a = tile[3 * k], b = tile[3 * k + 1], c = tile[3 * k + 2];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double dx = a.x - xi[r], dy = a.y - yi[r], dz = b.x - zi[r];
        const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const double h = b.y + hi[r];
        double p;
        if (r2 <= h * h) {
          p = soft_phi64(r2, h, c.x);
        } else {
          p = -c.x * rinv64(r2);
        }
        t[r] += p;
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] += t[r];
  }
  double *o = out + (size_t)blockIdx.y * (size_t)n;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = ibase + r * kBlock;
    if (i < n) o[i] = acc[r];
  }
}

// ---------------------------------------------------------------------------
// O(N) kernels.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_reduce_partials(
    const double *__restrict__ part, int jsplit, int comps, int n,
    double *__restrict__ acc) {
  const size_t total = (size_t)comps * n;
  const size_t k = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= total) return;
  double s = 0.0;
  for (int p = 0; p < jsplit; ++p) s += part[(size_t)p * total + k];
  acc[k] = s;
}

__global__ __launch_bounds__(kBlock) void k_shadow(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const double *__restrict__ soft, int n, float *__restrict__ shadow) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  shadow[i] = (float)pos[i];
  shadow[(size_t)n + i] = (float)pos[(size_t)n + i];
  shadow[2 * (size_t)n + i] = (float)pos[2 * (size_t)n + i];
  shadow[3 * (size_t)n + i] = (float)mass[i];
  shadow[4 * (size_t)n + i] = (float)soft[i];
}

__global__ __launch_bounds__(kBlock) void k_kick_drift(
    double *__restrict__ pos, double *__restrict__ vel,
    const double *__restrict__ S, int n, double hdt, double gA, double radA,
    double drag, double dt) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const size_t k = (size_t)d * n + i;
    const double x = pos[k], s = S[k];
    double v = vel[k];
    v = v + hdt * (gA * s + radA * x - drag * v);
    vel[k] = v;
    pos[k] = x + dt * v;
  }
}

__global__ __launch_bounds__(kBlock) void k_kick_end(
    const double *__restrict__ pos, double *__restrict__ vel,
    const double *__restrict__ S, int n, double hdt, double gA, double radA,
    double inv) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const size_t k = (size_t)d * n + i;
    vel[k] = (vel[k] + hdt * (gA * S[k] + radA * pos[k])) * inv;
  }
}

__global__ __launch_bounds__(kBlock) void k_check_finite(
    const double *__restrict__ p, int64_t count, int *__restrict__ flag) {
  int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  int bad = 0;
  for (; k < count; k += stride) bad |= !isfinite(p[k]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// Energy sums, 6 per block in a fixed order: sum 1/2 m |v|^2,
// sum 1/2 m phi, sum m |x|^2, sum m v (3).  Grid-stride over particles,
// then a fixed-shape tree within the block.
constexpr int kEnergySums = 6;

__global__ __launch_bounds__(kBlock) void k_energy_partial(
    const double *__restrict__ pos, const double *__restrict__ vel,
    const double *__restrict__ mass, const double *__restrict__ phi, int n,
    double *__restrict__ part) {
  __shared__ double red[kEnergySums][kBlock];
  double v[kEnergySums] = {0, 0, 0, 0, 0, 0};
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n;
       i += gridDim.x * kBlock) {
    const double m = mass[i];
    const double vx = vel[i], vy = vel[(size_t)n + i], vz = vel[2 * (size_t)n + i];
    v[0] += 0.5 * m * (vx * vx + vy * vy + vz * vz);
    if (phi) v[1] += 0.5 * m * phi[i];
    if (pos) {
      const double x = pos[i], y = pos[(size_t)n + i], z = pos[2 * (size_t)n + i];
      v[2] += m * (x * x + y * y + z * z);
    }
    v[3] += m * vx;
    v[4] += m * vy;
    v[5] += m * vz;
  }
#pragma unroll
  for (int c = 0; c < kEnergySums; ++c) red[c][threadIdx.x] = v[c];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int c = 0; c < kEnergySums; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < kEnergySums) {
    part[(size_t)blockIdx.x * kEnergySums + threadIdx.x] = red[threadIdx.x][0];
  }
}

__global__ __launch_bounds__(kBlock) void k_energy_final(
    const double *__restrict__ part, int nb, double *__restrict__ out) {
  if (threadIdx.x < kEnergySums) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(size_t)b * kEnergySums + threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// Adaptive step (Eq. 12): per block the smallest 2.8 h_i / |A_i| over its
// particles, A_i = g S_i + rad x_i - drag v_i (the kick's acceleration at
// the start of the step); +inf where A_i = 0.  min is exact, so the result
// does not depend on the order.
__global__ __launch_bounds__(kBlock) void k_dt_partial(
    const double *__restrict__ pos, const double *__restrict__ vel,
    const double *__restrict__ acc, const double *__restrict__ soft, int n,
    double g, double rad, double drag, double *__restrict__ part) {
  __shared__ double red[kBlock];
  double q = INFINITY;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n;
       i += gridDim.x * kBlock) {
    double a2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const size_t k = (size_t)d * n + i;
      const double ad = g * acc[k] + rad * pos[k] - drag * vel[k];
      a2 = fma(ad, ad, a2);
    }
    if (a2 > 0.0) q = fmin(q, 2.8 * soft[i] / sqrt(a2));
  }
  red[threadIdx.x] = q;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void k_dt_final(
    const double *__restrict__ part, int nb, double *__restrict__ out) {
  __shared__ double red[kBlock];
  double q = INFINITY;
  for (int b = threadIdx.x; b < nb; b += kBlock) q = fmin(q, part[b]);
  red[threadIdx.x] = q;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace

int dt_blocks(int n) { return std::max(1, std::min(512, ceil_div(n, kBlock))); }

hipError_t launch_dt_min(const double *pos, const double *vel,
                         const double *acc, const double *soft, int n,
                         double g, double rad, double drag, double *part,
                         double *out, hipStream_t s) {
  const int nb = dt_blocks(n);
  hipLaunchKernelGGL(k_dt_partial, dim3(nb), dim3(kBlock), 0, s, pos, vel, acc,
                     soft, n, g, rad, drag, part);
  hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(kBlock), 0, s, part, nb, out);
  return hipGetLastError();
}

int energy_blocks(int n) { return std::max(1, std::min(512, ceil_div(n, kBlock))); }

hipError_t launch_energy(const double *pos, const double *vel,
                         const double *mass, const double *phi, int n,
                         double *part, double *out, hipStream_t s) {
  const int nb = energy_blocks(n);
  hipLaunchKernelGGL(k_energy_partial, dim3(nb), dim3(kBlock), 0, s, pos, vel,
                     mass, phi, n, part);
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kBlock), 0, s, part, nb, out);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double *part, int jsplit, int n,
                                  double *acc, hipStream_t s) {
  const long long total = 3LL * n;
  hipLaunchKernelGGL(k_reduce_partials, dim3(ceil_div(total, kBlock)),
                     dim3(kBlock), 0, s, part, jsplit, 3, n, acc);
  return hipGetLastError();
}

hipError_t launch_reduce_partials1(const double *part, int jsplit, int n,
                                   double *phi, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(ceil_div(n, kBlock)),
                     dim3(kBlock), 0, s, part, jsplit, 1, n, phi);
  return hipGetLastError();
}

hipError_t launch_potential(const double *pos, const double *mass,
                            const double *soft, int n, int jchunk, int jsplit,
                            double *out, hipStream_t s) {
  constexpr int R = 2, TJ = 128;
  dim3 grid(ceil_div(n, (long long)kBlock * R), jsplit);
  hipLaunchKernelGGL((k_potential_f64<R, TJ>), grid, dim3(kBlock), 0, s, pos,
                     mass, soft, n, jchunk, out);
  return hipGetLastError();
}

hipError_t launch_shadow(const double *pos, const double *mass,
                         const double *soft, int n, float *shadow,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_shadow, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s,
                     pos, mass, soft, n, shadow);
  return hipGetLastError();
}

hipError_t launch_kick_drift(double *pos, double *vel, const double *S, int n,
                             double hdt, double gA, double radA, double drag,
                             double dt, hipStream_t s) {
  hipLaunchKernelGGL(k_kick_drift, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0,
                     s, pos, vel, S, n, hdt, gA, radA, drag, dt);
  return hipGetLastError();
}

hipError_t launch_kick_end(const double *pos, double *vel, const double *S,
                           int n, double hdt, double gA, double radA,
                           double inv, hipStream_t s) {
  hipLaunchKernelGGL(k_kick_end, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0,
                     s, pos, vel, S, n, hdt, gA, radA, inv);
  return hipGetLastError();
}

hipError_t launch_check_finite(const double *p, int64_t count, int *flag,
                               hipStream_t s) {
  long long blocks = (count + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_check_finite, dim3((unsigned)blocks), dim3(kBlock), 0,
                     s, p, count, flag);
  return hipGetLastError();
}

}  // namespace steps
