// O(N) kernels of the ensemble path of libsteps: many independent
// simulations stepped together (KDK of Racz et al. 2018, Sec. 2.3 Eqs. 9-11,
// with the acceleration of Sec. 2.2 Eq. 8, per member).
//
// The ensemble's state lives in one sorted arena: member a owns the slot
// range [soff[a], soff[a+1]); mid[k] is the member of slot k.  The scalars of
// step s for member a (dt, G/a^3, radial/a^3, drag, ...) sit in a device
// table at [s][a][8], and the step index s is read from a device counter
// that the last kernel of a step advances -- so a captured step replays
// unchanged from one step to the next.

#include <algorithm>

#include "steps_internal.h"

namespace steps {
namespace {

inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

__global__ __launch_bounds__(kBlock) void k_batch_init(int *counter) {
  if (threadIdx.x < 2) counter[threadIdx.x] = 0;
}

// clamped step index (a replay past the table would reuse the last row)
__device__ __forceinline__ int batch_step(const int *counter, int nsteps) {
  return min(max(counter[0], 0), nsteps - 1);
}

// First half-kick at a_s, then drift; FP32 positions for the mixed kernel.
// Thread 0 also clears the work counter of this step's force launch.
__global__ __launch_bounds__(kBlock) void k_batch_kick_drift(
    double *__restrict__ pos, double *__restrict__ vel,
    const double *__restrict__ S, float *__restrict__ shadow,
    const int *__restrict__ mid, int n, const double *__restrict__ table,
    int members, int nsteps, int *counter) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int step = batch_step(counter, nsteps);
  if (i == 0) counter[1] = 0;
  if (i >= n) return;
  const double *t = table + ((size_t)step * members + mid[i]) * kBatchScalars;
  const double hdt = t[0], gA = t[1], radA = t[2], drag = t[3], dt = t[4];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const size_t k = (size_t)d * n + i;
    const double x = pos[k];
    double v = vel[k];
    v = v + hdt * (gA * S[k] + radA * x - drag * v);
    vel[k] = v;
    const double xn = x + dt * v;
    pos[k] = xn;
    if (shadow) shadow[k] = (float)xn;
  }
}

// Second half-kick at a_{s+1}, drag at the end-of-step velocity.
__global__ __launch_bounds__(kBlock) void k_batch_kick_end(
    const double *__restrict__ pos, double *__restrict__ vel,
    const double *__restrict__ S, const int *__restrict__ mid, int n,
    const double *__restrict__ table, int members, int nsteps,
    const int *counter) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int step = batch_step(counter, nsteps);
  const double *t = table + ((size_t)step * members + mid[i]) * kBatchScalars;
  const double hdt = t[0], gA = t[5], radA = t[6], inv = t[7];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const size_t k = (size_t)d * n + i;
    vel[k] = (vel[k] + hdt * (gA * S[k] + radA * pos[k])) * inv;
  }
}

// acc[d][i] = sum over the j-chunk planes c < kc[member of i] of
// part[c][d][i], in plane order (deterministic)
__global__ __launch_bounds__(kBlock) void k_batch_reduce(
    const double *__restrict__ part, int n, const int *__restrict__ mid,
    const int *__restrict__ kc, double *__restrict__ acc) {
  const size_t total = 3 * (size_t)n;
  const size_t q = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= total) return;
  const int i = (int)(q % (size_t)n);
  const int k = kc[mid[i]];
  double s = 0.0;
  for (int c = 0; c < k; ++c) s += part[(size_t)c * total + q];
  acc[q] = s;
}

__global__ void k_batch_advance(int *counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] += 1;
}

__device__ __forceinline__ double bmin(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double bmax(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Box of tile t = slots [beg[t], end[t]) of a [5][stride] SoA (x,y,z,m,h):
// (lo xyz, hi xyz, hmax, 0).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_batch_tile_info(
    const T *__restrict__ soa, int stride, const int *__restrict__ beg,
    const int *__restrict__ end, double *__restrict__ info) {
  __shared__ double part[kBlock / 64][7];
  const int t = blockIdx.x;
  double v[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
  for (int k = beg[t] + threadIdx.x; k < end[t]; k += kBlock) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double x = (double)soa[(size_t)d * stride + k];
      v[d] = fmin(v[d], x);
      v[3 + d] = fmax(v[3 + d], x);
    }
    v[6] = fmax(v[6], (double)soa[4 * (size_t)stride + k]);
  }
#pragma unroll
  for (int c = 0; c < 7; ++c) v[c] = c < 3 ? bmin(v[c]) : bmax(v[c]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int c = 0; c < 7; ++c) part[threadIdx.x >> 6][c] = v[c];
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    const int c = threadIdx.x;
    double r = 0.0;
    if (c < 7) {
      r = part[0][c];
      for (int q = 1; q < kBlock / 64; ++q) {
        r = c < 3 ? fmin(r, part[q][c]) : fmax(r, part[q][c]);
      }
    }
    info[(size_t)t * 8 + c] = r;
  }
}

__device__ __forceinline__ unsigned long long spread3(unsigned v) {
  unsigned long long x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x1f00000000ffffULL;
  x = (x | (x << 16)) & 0x1f0000ff0000ffULL;
  x = (x | (x << 8)) & 0x100f00f00f00f00fULL;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ULL;
  x = (x | (x << 2)) & 0x1249249249249249ULL;
  return x;
}

// key = member in the high bits, Morton code of qbits per axis below it, so
// one stable sort keeps every member inside its own slot range.
__global__ __launch_bounds__(kBlock) void k_batch_morton(
    const double *__restrict__ pos, int n, const double *__restrict__ box,
    const int *__restrict__ mid, int qbits, unsigned long long *__restrict__ keys,
    int *__restrict__ vals) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double top = (double)((1u << qbits) - 1u);
  const double ext = fmax(box[3] - box[0], fmax(box[4] - box[1], box[5] - box[2]));
  const double scale = ext > 0.0 ? top / ext : 0.0;
  unsigned q[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    q[d] = (unsigned)fmin(top, fmax(0.0, (pos[(size_t)d * n + i] - box[d]) * scale));
  }
  const unsigned long long code =
      spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
  keys[i] = ((unsigned long long)mid[i] << (3 * qbits)) | code;
  vals[i] = i;
}

// dst[c * ds + k] = src[c * ss + idx[k]]
__global__ __launch_bounds__(kBlock) void k_gather_cols(
    const double *__restrict__ src, int ss, const int *__restrict__ idx, int n,
    double *__restrict__ dst, int ds, int comps) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  const int i = idx[k];
  for (int c = 0; c < comps; ++c) dst[(size_t)c * ds + k] = src[(size_t)c * ss + i];
}

__global__ __launch_bounds__(kBlock) void k_gather_int(
    const int *__restrict__ src, const int *__restrict__ idx, int n,
    int *__restrict__ dst) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k < n) dst[k] = src[idx[k]];
}

// dst[c * ds + idx[k]] = src[c * ss + k]
__global__ __launch_bounds__(kBlock) void k_scatter_cols(
    const double *__restrict__ src, int ss, const int *__restrict__ idx, int n,
    double *__restrict__ dst, int ds, int comps) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  const int i = idx[k];
  for (int c = 0; c < comps; ++c) dst[(size_t)c * ds + i] = src[(size_t)c * ss + k];
}

}  // namespace

hipError_t launch_batch_init(int *counter, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_init, dim3(1), dim3(64), 0, s, counter);
  return hipGetLastError();
}

hipError_t launch_batch_kick_drift(double *pos, double *vel, const double *S,
                                   float *shadow, const int *mid, int n,
                                   const double *table, int members,
                                   int nsteps, int *counter, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_kick_drift, dim3(ceil_div(std::max(n, 1), kBlock)),
                     dim3(kBlock), 0, s, pos, vel, S, shadow, mid, n, table,
                     members, nsteps, counter);
  return hipGetLastError();
}

hipError_t launch_batch_kick_end(const double *pos, double *vel,
                                 const double *S, const int *mid, int n,
                                 const double *table, int members, int nsteps,
                                 const int *counter, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_kick_end, dim3(ceil_div(std::max(n, 1), kBlock)),
                     dim3(kBlock), 0, s, pos, vel, S, mid, n, table, members,
                     nsteps, counter);
  return hipGetLastError();
}

hipError_t launch_batch_reduce(const double *part, int n, const int *mid,
                               const int *kc, double *acc, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reduce,
                     dim3(ceil_div(std::max(3LL * n, 1LL), kBlock)), dim3(kBlock),
                     0, s, part, n, mid, kc, acc);
  return hipGetLastError();
}

hipError_t launch_batch_advance(int *counter, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(64), 0, s, counter);
  return hipGetLastError();
}

hipError_t launch_batch_tile_info_f64(const double *soa, int stride,
                                      const int *beg, const int *end,
                                      int ntiles, double *info, hipStream_t s) {
  hipLaunchKernelGGL((k_batch_tile_info<double>), dim3(ntiles), dim3(kBlock), 0,
                     s, soa, stride, beg, end, info);
  return hipGetLastError();
}

hipError_t launch_batch_tile_info_f32(const float *soa, int stride,
                                      const int *beg, const int *end,
                                      int ntiles, double *info, hipStream_t s) {
  hipLaunchKernelGGL((k_batch_tile_info<float>), dim3(ntiles), dim3(kBlock), 0,
                     s, soa, stride, beg, end, info);
  return hipGetLastError();
}

hipError_t launch_batch_morton(const double *pos, int n, const double *box,
                               const int *mid, int qbits,
                               unsigned long long *keys, int *vals,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_batch_morton, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0,
                     s, pos, n, box, mid, qbits, keys, vals);
  return hipGetLastError();
}

hipError_t launch_gather_cols(const double *src, int ss, const int *idx, int n,
                              double *dst, int ds, int comps, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_cols, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0,
                     s, src, ss, idx, n, dst, ds, comps);
  return hipGetLastError();
}

hipError_t launch_gather_int(const int *src, const int *idx, int n, int *dst,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_gather_int, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0,
                     s, src, idx, n, dst);
  return hipGetLastError();
}

hipError_t launch_scatter_cols(const double *src, int ss, const int *idx,
                               int n, double *dst, int ds, int comps,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_scatter_cols, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0,
                     s, src, ss, idx, n, dst, ds, comps);
  return hipGetLastError();
}

}  // namespace steps
