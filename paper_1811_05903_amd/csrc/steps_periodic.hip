// gfx950 periodic pair sum of libsteps (StePS, Sec. 2.2, Eqs. 2 and 5): in
// a box of side L the softened force of Eq. 4 is summed over the images
// x_j + n L of every other particle,
//   images = all:     every n with |x_j + n L - x_i| < 2.6 L (the printed
//                     formula: a direct image sum, no Fourier-space part);
//   images = nearest: the leading term only, the nearest image
//                     (quasi-periodic).
// A pair's displacement is first brought to its nearest image,
// d <- d - L rint(d / L) per component (each |d_k| <= L/2); the images
// within 2.6 L of such a d are among the 179 triplets n in [-3, 3]^3 whose
// box [n - 1/2, n + 1/2]^3 (in units of L) comes within 2.6 of the origin,
// listed at compile time below.  A particle's own images cancel in pairs
// (n and -n) and are skipped.  FP64; no spatial sort or culling (a
// periodic box has one resolution throughout); per-tile partials added
// into compensated running totals, j-splits reduced in fixed order.

#include "steps_internal.h"
#include "steps_pair.h"

namespace steps {
namespace {

constexpr int kTJp = 128;  // j-particles per LDS tile
constexpr int kRp = 2;     // i-particles per lane

struct ImageTable {
  int count;
  signed char n[343][3];
};

// n in [-3, 3]^3 with sum_k max(2|n_k| - 1, 0)^2 < (2 * 2.6)^2 = 27.04,
// i.e. the box around n L comes within 2.6 L of the origin.
constexpr ImageTable make_images() {
  ImageTable t{};
  t.count = 0;
  for (int a = -3; a <= 3; ++a) {
    for (int b = -3; b <= 3; ++b) {
      for (int c = -3; c <= 3; ++c) {
        const int qa = 2 * (a < 0 ? -a : a) - 1, qb = 2 * (b < 0 ? -b : b) - 1,
                  qc = 2 * (c < 0 ? -c : c) - 1;
        const int s = (qa > 0 ? qa * qa : 0) + (qb > 0 ? qb * qb : 0) +
                      (qc > 0 ? qc * qc : 0);
        if (s <= 27) {
          t.n[t.count][0] = (signed char)a;
          t.n[t.count][1] = (signed char)b;
          t.n[t.count][2] = (signed char)c;
          ++t.count;
        }
      }
    }
  }
  return t;
}

__constant__ ImageTable kImages = make_images();
static_assert(make_images().count == 179, "image candidate list");

__device__ __forceinline__ double pair_w(double r2, double h, double m) {
  return r2 <= h * h ? soft_w64(r2, h, m) : newton_w64<true>(r2, m);
}

// block (x, y) = (i-block, j-split); split y writes its partial to
// out + y * 3n
template <int IMAGES>
__global__ __launch_bounds__(kBlock) void k_force_periodic(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const double *__restrict__ soft, int n, int jchunk, double L,
    double *__restrict__ out) {
  __shared__ double2 tile[3 * kTJp];
  const int tid = threadIdx.x;
  const int ibase = blockIdx.x * (kBlock * kRp) + (tid >> 6) * (64 * kRp) + (tid & 63);
  const int jbeg = blockIdx.y * jchunk, jend = min(n, jbeg + jchunk);
  const double *X = pos, *Y = pos + n, *Z = pos + 2 * (size_t)n;
  const double invL = 1.0 / L, cut2 = (2.6 * L) * (2.6 * L);

  int ii[kRp];
  double xi[kRp], yi[kRp], zi[kRp], hi[kRp];
  double ax[kRp], ay[kRp], az[kRp], cx[kRp], cy[kRp], cz[kRp];
#pragma unroll
  for (int r = 0; r < kRp; ++r) {
    ii[r] = ibase + 64 * r;
    const int i = min(ii[r], n - 1);
    xi[r] = X[i];
    yi[r] = Y[i];
    zi[r] = Z[i];
    hi[r] = soft[i];
    ax[r] = ay[r] = az[r] = cx[r] = cy[r] = cz[r] = 0.0;
  }

  for (int jt = jbeg; jt < jend; jt += kTJp) {
    __syncthreads();
    for (int k = tid; k < kTJp; k += kBlock) {
      const int j = min(jt + k, jend - 1);
      const double mj = (jt + k < jend) ? mass[j] : 0.0;
      tile[3 * k] = double2{X[j], Y[j]};
      tile[3 * k + 1] = double2{Z[j], mj};
      tile[3 * k + 2] = double2{soft[j], 0.0};
    }
    __syncthreads();
    double tx[kRp], ty[kRp], tz[kRp];
#pragma unroll
    for (int r = 0; r < kRp; ++r) tx[r] = ty[r] = tz[r] = 0.0;
    const int kend = min(kTJp, jend - jt);
    for (int k = 0; k < kend; ++k) {
      const double2 a = tile[3 * k], b = tile[3 * k + 1], c = tile[3 * k + 2];
#pragma unroll
      for (int r = 0; r < kRp; ++r) {
        if (jt + k == ii[r]) continue;  // own images cancel in pairs
        double dx = a.x - xi[r], dy = a.y - yi[r], dz = b.x - zi[r];
        dx = fma(-L, rint(dx * invL), dx);
        dy = fma(-L, rint(dy * invL), dy);
        dz = fma(-L, rint(dz * invL), dz);
        const double h = c.x + hi[r];
        if (IMAGES == 1) {
          const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
          const double w = pair_w(r2, h, b.y);
          tx[r] = fma(w, dx, tx[r]);
          ty[r] = fma(w, dy, ty[r]);
          tz[r] = fma(w, dz, tz[r]);
        } else {
          for (int q = 0; q < kImages.count; ++q) {
            const double ex = fma((double)kImages.n[q][0], L, dx);
            const double ey = fma((double)kImages.n[q][1], L, dy);
            const double ez = fma((double)kImages.n[q][2], L, dz);
            const double r2 = fma(ez, ez, fma(ey, ey, ex * ex));
            if (r2 < cut2) {
              const double w = pair_w(r2, h, b.y);
              tx[r] = fma(w, ex, tx[r]);
              ty[r] = fma(w, ey, ty[r]);
              tz[r] = fma(w, ez, tz[r]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kRp; ++r) {
      two_sum_add(ax[r], cx[r], tx[r]);
      two_sum_add(ay[r], cy[r], ty[r]);
      two_sum_add(az[r], cz[r], tz[r]);
    }
  }
  double *o = out + (size_t)blockIdx.y * 3 * (size_t)n;
#pragma unroll
  for (int r = 0; r < kRp; ++r) {
    const int i = ii[r];
    if (i < n) {
      o[i] = ax[r] + cx[r];
      o[(size_t)n + i] = ay[r] + cy[r];
      o[2 * (size_t)n + i] = az[r] + cz[r];
    }
  }
}

inline int ceil_div_p(long long a, long long b) { return (int)((a + b - 1) / b); }

}  // namespace

int periodic_tile() { return kTJp; }
int periodic_iblocks(int n) { return ceil_div_p(n, (long long)kBlock * kRp); }

hipError_t launch_force_periodic(const double *pos, const double *mass,
                                 const double *soft, int n, double L,
                                 int images, int jchunk, int jsplit,
                                 double *out, hipStream_t s) {
  dim3 grid(periodic_iblocks(n), jsplit);
  if (images == 1) {
    hipLaunchKernelGGL(k_force_periodic<1>, grid, dim3(kBlock), 0, s, pos,
                       mass, soft, n, jchunk, L, out);
  } else {
    hipLaunchKernelGGL(k_force_periodic<2>, grid, dim3(kBlock), 0, s, pos,
                       mass, soft, n, jchunk, L, out);
  }
  return hipGetLastError();
}

}  // namespace steps
