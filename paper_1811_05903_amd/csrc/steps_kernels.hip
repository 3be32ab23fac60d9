// gfx950 kernels of libsteps: the all-pairs spline-softened pair sum of
// StePS (Racz et al. 2018, Sec. 2.2 Eqs. 3, 4 and 8), its potential, and the
// O(N) kick / drift of the KDK leapfrog (Sec. 2.3 Eqs. 9-11).
//
// Force kernel layout (all precisions):
//   * a workgroup is 256 lanes (4 wave64); each lane holds R i-particles in
//     registers, so a workgroup owns 256*R consecutive i (lane-strided, so
//     the one-off i loads and the stores are coalesced);
//   * grid.y splits the j range into jsplit chunks; each chunk is streamed
//     through LDS in tiles of TJ particles, loaded cooperatively with
//     coalesced SoA reads and read back by every lane as an LDS broadcast;
//   * each lane sums a tile's TJ terms into a per-tile partial and adds the
//     partial to its running total after the tile (blocked summation: the
//     rounding error grows with TJ + N/TJ instead of N);
//   * the softened branch of Eq. 4 is rare (pairs closer than h_i + h_j): it
//     is taken under one divergent branch per j that waves skip when no lane
//     needs it.
// No atomics: the FP64 result is bitwise reproducible for a given launch
// shape.  Partial sums of a j-split are reduced in fixed order.

#include "steps_internal.h"

namespace steps {
namespace {

// ---------------------------------------------------------------------------
// FP64 pair weight.  S_i += w (x_j - x_i) with w = m_j F(r, h) / r.
//
// Newtonian branch (r >= h): w = m r^-3.  v_rsq_f64 gives y ~ r^-1 to about
// 2^-24 (measured on gfx950); with e = 1 - r2 y^2 the exact value is
//   r^-3 = y^3 (1 - e)^(-3/2) = y^3 (1 + 3/2 e + 15/8 e^2 + O(e^3)).
// E2 = true keeps the e^2 term (residual below 2^-68).  E2 = false stops at
// the linear term: the residual 15/8 e^2 is at most ~2e-14 relative per
// pair and about 1e-15 on average, and the weight then costs one
// accumulate-form FMA with a literal instead of a two-constant polynomial.
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

template <int R, int TJ, bool E2>
__global__ __launch_bounds__(kBlock) void k_force_f64(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const double *__restrict__ soft, int n, int jchunk,
    double *__restrict__ out) {
  // one j per 3 x double2: (x, y), (z, h), (m, 0)
  __shared__ double2 tile[3 * TJ];
  const int tid = threadIdx.x;
  const int ibase = blockIdx.x * (kBlock * R) + tid;
  const int jbeg = blockIdx.y * jchunk;
  const int jend = min(n, jbeg + jchunk);
  const double *X = pos, *Y = pos + n, *Z = pos + 2 * (size_t)n;

  double xi[R], yi[R], zi[R], hi[R], ax[R], ay[R], az[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = ibase + r * kBlock;
    const bool ok = i < n;
    xi[r] = ok ? X[i] : 0.0;
    yi[r] = ok ? Y[i] : 0.0;
    zi[r] = ok ? Z[i] : 0.0;
    hi[r] = ok ? soft[i] : 0.0;
    ax[r] = ay[r] = az[r] = 0.0;
  }

  for (int jt = jbeg; jt < jend; jt += TJ) {
    __syncthreads();
    for (int k = tid; k < TJ; k += kBlock) {
      const int j = jt + k;
      double2 a = {0.0, 0.0}, b = {0.0, 0.0}, c = {0.0, 0.0};
      if (j < jend) {  // padding: zero mass at the origin contributes 0
        a = double2{X[j], Y[j]};
        b = double2{Z[j], soft[j]};
        c = double2{mass[j], 0.0};
      }
      tile[3 * k] = a;
      tile[3 * k + 1] = b;
      tile[3 * k + 2] = c;
    }
    __syncthreads();

    double tx[R], ty[R], tz[R];
#pragma unroll
    for (int r = 0; r < R; ++r) tx[r] = ty[r] = tz[r] = 0.0;

#pragma unroll 2
    for (int k = 0; k < TJ; ++k) {
      const double2 a = tile[3 * k], b = tile[3 * k + 1], c = tile[3 * k + 2];
      const double xj = a.x, yj = a.y, zj = b.x, hj = b.y, mj = c.x;
      double dx[R], dy[R], dz[R], r2[R], w[R];
      bool sf[R];
      bool any = false;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        dx[r] = xj - xi[r];
        dy[r] = yj - yi[r];
        dz[r] = zj - zi[r];
        r2[r] = fma(dz[r], dz[r], fma(dy[r], dy[r], dx[r] * dx[r]));
        const double h = hj + hi[r];
        sf[r] = r2[r] <= h * h;  // softened, or zero separation
        any |= sf[r];
        w[r] = newton_w64<E2>(r2[r], mj);
      }
      if (any) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (sf[r]) w[r] = soft_w64(r2[r], hj + hi[r], mj);
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        tx[r] = fma(w[r], dx[r], tx[r]);
        ty[r] = fma(w[r], dy[r], ty[r]);
        tz[r] = fma(w[r], dz[r], tz[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      ax[r] += tx[r];
      ay[r] += ty[r];
      az[r] += tz[r];
    }
  }

  double *o = out + (size_t)blockIdx.y * 3 * (size_t)n;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = ibase + r * kBlock;
    if (i < n) {
      o[i] = ax[r];
      o[(size_t)n + i] = ay[r];
      o[2 * (size_t)n + i] = az[r];
    }
  }
}

// ---------------------------------------------------------------------------
// Mixed precision: the pair arithmetic runs in FP32 on an FP32 shadow of the
// inputs (v_rsq_f32 is accurate to ~2^-23, used as is); each tile's FP32
// partial is added into an FP64 accumulator, or into a Kahan-compensated
// FP32 (sum, compensation) pair.
// ---------------------------------------------------------------------------
__device__ __noinline__ float soft_w32(float r2, float h, float m) {
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

template <int R, int TJ, bool KAHAN>
__global__ __launch_bounds__(kBlock) void k_force_mixed(
    const float *__restrict__ shadow, int n, int jchunk,
    double *__restrict__ out) {
  __shared__ float4 tpos[TJ];  // (x, y, z, h)
  __shared__ float tmass[TJ];
  const int tid = threadIdx.x;
  const int ibase = blockIdx.x * (kBlock * R) + tid;
  const int jbeg = blockIdx.y * jchunk;
  const int jend = min(n, jbeg + jchunk);
  const float *X = shadow, *Y = shadow + n, *Z = shadow + 2 * (size_t)n;
  const float *M = shadow + 3 * (size_t)n, *H = shadow + 4 * (size_t)n;

  float xi[R], yi[R], zi[R], hi[R];
  double ax[R], ay[R], az[R];  // FP64 accumulation
  float sx[R], sy[R], sz[R], cx[R], cy[R], cz[R];  // Kahan accumulation
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = ibase + r * kBlock;
    const bool ok = i < n;
    xi[r] = ok ? X[i] : 0.0f;
    yi[r] = ok ? Y[i] : 0.0f;
    zi[r] = ok ? Z[i] : 0.0f;
    hi[r] = ok ? H[i] : 0.0f;
    ax[r] = ay[r] = az[r] = 0.0;
    sx[r] = sy[r] = sz[r] = cx[r] = cy[r] = cz[r] = 0.0f;
  }

  for (int jt = jbeg; jt < jend; jt += TJ) {
    __syncthreads();
    for (int k = tid; k < TJ; k += kBlock) {
      const int j = jt + k;
      float4 p = {0.0f, 0.0f, 0.0f, 0.0f};
      float m = 0.0f;
      if (j < jend) {
        p = float4{X[j], Y[j], Z[j], H[j]};
        m = M[j];
      }
      tpos[k] = p;
      tmass[k] = m;
    }
    __syncthreads();

    float tx[R], ty[R], tz[R];
#pragma unroll
    for (int r = 0; r < R; ++r) tx[r] = ty[r] = tz[r] = 0.0f;

#pragma unroll 2
    for (int k = 0; k < TJ; ++k) {
      const float4 p = tpos[k];
      const float mj = tmass[k];
      float dx[R], dy[R], dz[R], r2[R], w[R];
      bool sf[R];
      bool any = false;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        dx[r] = p.x - xi[r];
        dy[r] = p.y - yi[r];
        dz[r] = p.z - zi[r];
        r2[r] = fmaf(dz[r], dz[r], fmaf(dy[r], dy[r], dx[r] * dx[r]));
        const float h = p.w + hi[r];
        sf[r] = r2[r] <= h * h;
        any |= sf[r];
        const float y = __builtin_amdgcn_rsqf(r2[r]);
        w[r] = (mj * y) * (y * y);
      }
      if (any) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (sf[r]) w[r] = soft_w32(r2[r], p.w + hi[r], mj);
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        tx[r] = fmaf(w[r], dx[r], tx[r]);
        ty[r] = fmaf(w[r], dy[r], ty[r]);
        tz[r] = fmaf(w[r], dz[r], tz[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (KAHAN) {
        float yv, t;
        yv = tx[r] - cx[r]; t = sx[r] + yv; cx[r] = (t - sx[r]) - yv; sx[r] = t;
        yv = ty[r] - cy[r]; t = sy[r] + yv; cy[r] = (t - sy[r]) - yv; sy[r] = t;
        yv = tz[r] - cz[r]; t = sz[r] + yv; cz[r] = (t - sz[r]) - yv; sz[r] = t;
      } else {
        ax[r] += (double)tx[r];
        ay[r] += (double)ty[r];
        az[r] += (double)tz[r];
      }
    }
  }

  double *o = out + (size_t)blockIdx.y * 3 * (size_t)n;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = ibase + r * kBlock;
    if (i < n) {
      if (KAHAN) {
        o[i] = (double)sx[r] - (double)cx[r];
        o[(size_t)n + i] = (double)sy[r] - (double)cy[r];
        o[2 * (size_t)n + i] = (double)sz[r] - (double)cz[r];
      } else {
        o[i] = ax[r];
        o[(size_t)n + i] = ay[r];
        o[2 * (size_t)n + i] = az[r];
      }
    }
  }
}

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

template <int R, int TJ, bool E2>
hipError_t launch_f64(const ForceLaunch &L, hipStream_t s) {
  dim3 grid(ceil_div(L.n, (long long)kBlock * R), L.jsplit);
  hipLaunchKernelGGL((k_force_f64<R, TJ, E2>), grid, dim3(kBlock), 0, s,
                     L.pos, L.mass, L.soft, L.n, L.jchunk, L.out);
  return hipGetLastError();
}

template <int R, int TJ>
hipError_t launch_mixed(const ForceLaunch &L, hipStream_t s) {
  dim3 grid(ceil_div(L.n, (long long)kBlock * R), L.jsplit);
  if (L.kahan) {
    hipLaunchKernelGGL((k_force_mixed<R, TJ, true>), grid, dim3(kBlock), 0, s,
                       L.shadow, L.n, L.jchunk, L.out);
  } else {
    hipLaunchKernelGGL((k_force_mixed<R, TJ, false>), grid, dim3(kBlock), 0,
                       s, L.shadow, L.n, L.jchunk, L.out);
  }
  return hipGetLastError();
}

// variant 0: FP64 weight with the e^2 correction term; variant 1: without.
const ForceVariant kVariants[] = {
    {kClassF64, 1, 128, 0, launch_f64<1, 128, true>},
    {kClassF64, 2, 128, 0, launch_f64<2, 128, true>},
    {kClassF64, 4, 128, 0, launch_f64<4, 128, true>},
    {kClassF64, 4, 256, 0, launch_f64<4, 256, true>},
    {kClassF64, 8, 128, 0, launch_f64<8, 128, true>},
    {kClassF64, 1, 128, 1, launch_f64<1, 128, false>},
    {kClassF64, 2, 128, 1, launch_f64<2, 128, false>},
    {kClassF64, 4, 128, 1, launch_f64<4, 128, false>},
    {kClassF64, 4, 256, 1, launch_f64<4, 256, false>},
    {kClassF64, 8, 128, 1, launch_f64<8, 128, false>},
    {kClassMixed, 1, 128, 0, launch_mixed<1, 128>},
    {kClassMixed, 2, 256, 0, launch_mixed<2, 256>},
    {kClassMixed, 4, 256, 0, launch_mixed<4, 256>},
    {kClassMixed, 8, 256, 0, launch_mixed<8, 256>},
};

}  // namespace

const ForceVariant *force_variants(int *count) {
  *count = (int)(sizeof(kVariants) / sizeof(kVariants[0]));
  return kVariants;
}

const ForceVariant *find_force_variant(int cls, int r, int tj, int variant) {
  for (const ForceVariant &v : kVariants) {
    if (v.cls == cls && v.r == r && v.tj == tj && v.variant == variant) {
      return &v;
    }
  }
  return nullptr;
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
