// Spatial ordering for the culled pair-sum kernels of libsteps.
//
// Before a culled force evaluation the particles are put in Morton
// (Z-curve) order of their positions: consecutive particles are then close
// in space, so a wave's 64*R particles and a j-tile's TJ particles each fill
// a small box, and most (wave, tile) boxes are far apart compared to the
// softening lengths.  The order is a permutation computed every evaluation
// (positions move every step); sums are formed in the sorted order and
// scattered back to the caller's order at the end.  Everything here is
// deterministic: min/max reductions, a stable radix sort on (key, index).

#include <hip/hip_runtime.h>

#include <algorithm>

#include <hipcub/device/device_radix_sort.hpp>

#include "steps_internal.h"

namespace steps {
namespace {

inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

__device__ __forceinline__ double wmin(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Block-wide reduction of K values: lanes hold v[0..K), mins first then
// maxes (negated mins are not used: each slot says which it is).
template <int K>
__device__ void block_minmax(double (&v)[K], const bool (&is_max)[K],
                             double *out) {
  __shared__ double part[kBlock / 64][K];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = is_max[k] ? wmax(v[k]) : wmin(v[k]);
  if (l == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) part[w][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double r = part[0][k];
      for (int q = 1; q < kBlock / 64; ++q) {
        r = is_max[k] ? fmax(r, part[q][k]) : fmin(r, part[q][k]);
      }
      out[k] = r;
    }
  }
}

// per-block bounding box of the positions: part[b][6] = lo xyz, hi xyz
__global__ __launch_bounds__(kBlock) void k_bbox_partial(
    const double *__restrict__ pos, int n, double *__restrict__ part) {
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  const bool mx[6] = {false, false, false, true, true, true};
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n;
       i += gridDim.x * kBlock) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double x = pos[(size_t)d * n + i];
      v[d] = fmin(v[d], x);
      v[3 + d] = fmax(v[3 + d], x);
    }
  }
  block_minmax<6>(v, mx, part + (size_t)blockIdx.x * 6);
}

__global__ __launch_bounds__(kBlock) void k_bbox_final(
    const double *__restrict__ part, int nb, double *__restrict__ box) {
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  const bool mx[6] = {false, false, false, true, true, true};
  for (int b = threadIdx.x; b < nb; b += kBlock) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double x = part[(size_t)b * 6 + k];
      v[k] = mx[k] ? fmax(v[k], x) : fmin(v[k], x);
    }
  }
  block_minmax<6>(v, mx, box);
}

// spread the low 21 bits of v to every third bit
__device__ __forceinline__ unsigned long long spread3(unsigned v) {
  unsigned long long x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x1f00000000ffffULL;
  x = (x | (x << 16)) & 0x1f0000ff0000ffULL;
  x = (x | (x << 8)) & 0x100f00f00f00f00fULL;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ULL;
  x = (x | (x << 2)) & 0x1249249249249249ULL;
  return x;
}

// 63-bit Morton key of each position on a 2^21 grid over the bounding cube
__global__ __launch_bounds__(kBlock) void k_morton(
    const double *__restrict__ pos, int n, const double *__restrict__ box,
    unsigned long long *__restrict__ keys, int *__restrict__ vals) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double ext = fmax(box[3] - box[0], fmax(box[4] - box[1], box[5] - box[2]));
  const double scale = ext > 0.0 ? 2097151.0 / ext : 0.0;
  unsigned q[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    // fmax/fmin also map NaN to the grid edge
    const double t = fmin(2097151.0, fmax(0.0, (pos[(size_t)d * n + i] - box[d]) * scale));
    q[d] = (unsigned)t;
  }
  keys[i] = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
  vals[i] = i;
}

// sorted SoA copy [x | y | z | m | h] (FP64) and optional FP32 shadow
__global__ __launch_bounds__(kBlock) void k_gather(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const double *__restrict__ soft, const int *__restrict__ perm, int n,
    double *__restrict__ sorted, float *__restrict__ shadow) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  const int i = perm[k];
  const double v[5] = {pos[i], pos[(size_t)n + i], pos[2 * (size_t)n + i],
                       mass[i], soft[i]};
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    if (sorted) sorted[(size_t)c * n + k] = v[c];
    if (shadow) shadow[(size_t)c * n + k] = (float)v[c];
  }
}

// per tile of tj sorted particles: (xlo, ylo, zlo, xhi, yhi, zhi, hmax, 0)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_tile_info(
    const T *__restrict__ soa, int n, int tj, double *__restrict__ info) {
  const int t = blockIdx.x;
  const int beg = t * tj, end = min(n, beg + tj);
  double v[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
  const bool mx[7] = {false, false, false, true, true, true, true};
  for (int k = beg + threadIdx.x; k < end; k += kBlock) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double x = (double)soa[(size_t)d * n + k];
      v[d] = fmin(v[d], x);
      v[3 + d] = fmax(v[3 + d], x);
    }
    v[6] = fmax(v[6], (double)soa[4 * (size_t)n + k]);
  }
  block_minmax<7>(v, mx, info + (size_t)t * 8);
  if (threadIdx.x == 0) info[(size_t)t * 8 + 7] = 0.0;
}

// acc[d][perm[k]] = sum_p part[p][d][k], fixed order over p
__global__ __launch_bounds__(kBlock) void k_reduce_scatter(
    const double *__restrict__ part, int jsplit, int n,
    const int *__restrict__ perm, double *__restrict__ acc) {
  const size_t total = 3 * (size_t)n;
  const size_t q = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= total) return;
  double s = 0.0;
  for (int p = 0; p < jsplit; ++p) s += part[(size_t)p * total + q];
  const size_t d = q / n, k = q - d * n;
  acc[d * n + perm[k]] = s;
}

}  // namespace

int bbox_blocks(int n) { return std::max(1, std::min(1024, ceil_div(n, kBlock))); }

hipError_t launch_bbox(const double *pos, int n, double *part, double *box,
                       hipStream_t s) {
  const int nb = bbox_blocks(n);
  hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(kBlock), 0, s, pos, n, part);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(kBlock), 0, s, part, nb, box);
  return hipGetLastError();
}

hipError_t launch_morton(const double *pos, int n, const double *box,
                         unsigned long long *keys, int *vals, hipStream_t s) {
  hipLaunchKernelGGL(k_morton, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s,
                     pos, n, box, keys, vals);
  return hipGetLastError();
}

hipError_t sort_pairs(void *tmp, size_t *tmp_bytes,
                      const unsigned long long *kin, unsigned long long *kout,
                      const int *vin, int *vout, int n, hipStream_t s) {
  return hipcub::DeviceRadixSort::SortPairs(tmp, *tmp_bytes, kin, kout, vin,
                                            vout, n, 0, 63, s);
}

hipError_t launch_gather(const double *pos, const double *mass,
                         const double *soft, const int *perm, int n,
                         double *sorted, float *shadow, hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s,
                     pos, mass, soft, perm, n, sorted, shadow);
  return hipGetLastError();
}

hipError_t launch_tile_info_f64(const double *sorted, int n, int tj,
                                double *info, hipStream_t s) {
  hipLaunchKernelGGL((k_tile_info<double>), dim3(ceil_div(n, tj)), dim3(kBlock),
                     0, s, sorted, n, tj, info);
  return hipGetLastError();
}

hipError_t launch_tile_info_f32(const float *shadow, int n, int tj,
                                double *info, hipStream_t s) {
  hipLaunchKernelGGL((k_tile_info<float>), dim3(ceil_div(n, tj)), dim3(kBlock),
                     0, s, shadow, n, tj, info);
  return hipGetLastError();
}

hipError_t launch_reduce_scatter(const double *part, int jsplit, int n,
                                 const int *perm, double *acc, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_scatter, dim3(ceil_div(3LL * n, kBlock)),
                     dim3(kBlock), 0, s, part, jsplit, n, perm, acc);
  return hipGetLastError();
}

}  // namespace steps
