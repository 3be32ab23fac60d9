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
// (n and -n) and are skipped.  FP64, over Morton-sorted particles with
// per-block shortcuts that give the same bits as the per-pair rules (see
// k_force_periodic); per-tile partials added into compensated running
// totals, j-splits reduced in fixed order and scattered back.

#include "steps_internal.h"
#include "steps_pair.h"

namespace steps {
namespace {

constexpr int kTJp = 128;  // j-particles per LDS tile
constexpr int kRp = 2;     // i-particles per lane
// One wave per workgroup: waves take the per-block shortcuts at different
// (wave, tile) blocks, and a workgroup barrier per tile would hold every
// wave to its slowest sibling (measured: 4-wave workgroups gained nothing
// from the shortcuts, 1-wave ones gain the full difference).
constexpr int kWaveBlock = 64;

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

__device__ __forceinline__ double wave_lo(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_hi(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Particles arrive Morton-sorted, with the box (lo xyz, hi xyz, hmax) of
// every tile of kTJp in tinfo.  Per (wave, tile) block, along each axis,
// the displacements d = x_j - x_i lie in [tlo - whi, thi - wlo]; when that
// range over L sits strictly inside (k - 1/2, k + 1/2) for one integer k,
// every pair's nearest image along the axis is the shift -k L (rounding is
// monotone, so the per-pair rint(d / L) is k as well), and the block uses
// it without the per-pair wrap -- the same operations on the same values,
// so the same bits.  Such a block whose minimum-image boxes are farther
// apart than the largest combined softening also skips the softening test.
// With every image (IMAGES = 2), such a block loops only over the candidate
// images whose shifted box comes within 2.6 L; the rest would fail the
// per-pair cut for every pair (the box distance is formed with the same
// operations as r^2, so it bounds it from below exactly).
//
// block (x, y) = (i-block of one wave, j-split); split y writes its
// partial to out + y * 3n
template <int IMAGES>
__global__ __launch_bounds__(kWaveBlock) void k_force_periodic(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const double *__restrict__ soft, int n, int jchunk, double L,
    const double *__restrict__ tinfo, double *__restrict__ out) {
  __shared__ double2 tile[3 * kTJp];
  const int tid = threadIdx.x;
  const int ibase = blockIdx.x * (kWaveBlock * kRp) + tid;
  const int jbeg = blockIdx.y * jchunk, jend = min(n, jbeg + jchunk);
  const double *X = pos, *Y = pos + n, *Z = pos + 2 * (size_t)n;
  const double invL = 1.0 / L, cut2 = (2.6 * L) * (2.6 * L);

  int ii[kRp];
  double xi[kRp], yi[kRp], zi[kRp], hi[kRp];
  double ax[kRp], ay[kRp], az[kRp], cx[kRp], cy[kRp], cz[kRp];
  double wl[3] = {INFINITY, INFINITY, INFINITY};
  double wh[3] = {-INFINITY, -INFINITY, -INFINITY};
  double whm = 0.0;
#pragma unroll
  for (int r = 0; r < kRp; ++r) {
    ii[r] = ibase + 64 * r;
    const int i = min(ii[r], n - 1);
    xi[r] = X[i];
    yi[r] = Y[i];
    zi[r] = Z[i];
    hi[r] = soft[i];
    ax[r] = ay[r] = az[r] = cx[r] = cy[r] = cz[r] = 0.0;
    if (ii[r] < n) {
      wl[0] = fmin(wl[0], xi[r]); wh[0] = fmax(wh[0], xi[r]);
      wl[1] = fmin(wl[1], yi[r]); wh[1] = fmax(wh[1], yi[r]);
      wl[2] = fmin(wl[2], zi[r]); wh[2] = fmax(wh[2], zi[r]);
      whm = fmax(whm, hi[r]);
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    wl[c] = wave_lo(wl[c]);
    wh[c] = wave_hi(wh[c]);
  }
  whm = wave_hi(whm);

  for (int jt = jbeg; jt < jend; jt += kTJp) {
    __syncthreads();
    for (int k = tid; k < kTJp; k += kWaveBlock) {
      const int j = min(jt + k, jend - 1);
      const double mj = (jt + k < jend) ? mass[j] : 0.0;
      tile[3 * k] = double2{X[j], Y[j]};
      tile[3 * k + 1] = double2{Z[j], mj};
      tile[3 * k + 2] = double2{soft[j], 0.0};
    }
    __syncthreads();

    // the block's shift per axis, the wrapped displacement range [dl, dh]
    // and the minimum-image gap
    const double *ti = tinfo + (size_t)(jt / kTJp) * 8;
    bool uniform = true;
    double ks[3], dl[3], dh[3], g2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double dmn = ti[c] - wh[c], dmx = ti[3 + c] - wl[c];
      const double fmn = dmn * invL, fmx = dmx * invL;
      const double kc = rint(fmn);
      uniform = uniform && fmn > kc - 0.5 && fmx < kc + 0.5;
      ks[c] = kc;
      dl[c] = fma(-L, kc, dmn);
      dh[c] = fma(-L, kc, dmx);
      const double g = fmax(0.0, fmax(dl[c], -dh[c]));
      g2 = fma(g, g, g2);
    }
    const double hs = ti[6] + whm;
    const bool uni = __builtin_amdgcn_readfirstlane((int)uniform) != 0;
    const bool far = uni && __builtin_amdgcn_readfirstlane(
                                (int)(g2 > fmax(hs * hs * (1.0 + 1e-6), 1e-30))) != 0;

    // candidate images of a uniform block (every image): bit q of cm[q / 64]
    unsigned long long cm[3] = {0ull, 0ull, 0ull};
    if (IMAGES == 2 && uni) {
#pragma unroll
      for (int w = 0; w < 3; ++w) {
        const int q = 64 * w + tid;
        bool keep = false;
        if (q < kImages.count) {
          double gg[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double nl = fma((double)kImages.n[q][c], L, dl[c]);
            const double nh = fma((double)kImages.n[q][c], L, dh[c]);
            gg[c] = fmax(0.0, fmax(nl, -nh));
          }
          keep = fma(gg[2], gg[2], fma(gg[1], gg[1], gg[0] * gg[0])) < cut2;
        }
        cm[w] = __ballot(keep);
      }
    }

    double tx[kRp], ty[kRp], tz[kRp];
#pragma unroll
    for (int r = 0; r < kRp; ++r) tx[r] = ty[r] = tz[r] = 0.0;
    const int kend = min(kTJp, jend - jt);
    if (IMAGES == 1 && far) {
      // one shift for the block, no softening, no coincident pairs
      for (int k = 0; k < kend; ++k) {
        const double2 a = tile[3 * k], b = tile[3 * k + 1];
#pragma unroll
        for (int r = 0; r < kRp; ++r) {
          const double dx = fma(-L, ks[0], a.x - xi[r]);
          const double dy = fma(-L, ks[1], a.y - yi[r]);
          const double dz = fma(-L, ks[2], b.x - zi[r]);
          const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
          const double w = newton_w64<true>(r2, b.y);
          tx[r] = fma(w, dx, tx[r]);
          ty[r] = fma(w, dy, ty[r]);
          tz[r] = fma(w, dz, tz[r]);
        }
      }
    } else {
      for (int k = 0; k < kend; ++k) {
        const double2 a = tile[3 * k], b = tile[3 * k + 1], c = tile[3 * k + 2];
#pragma unroll
        for (int r = 0; r < kRp; ++r) {
          if (jt + k == ii[r]) continue;  // own images cancel in pairs
          double dx = a.x - xi[r], dy = a.y - yi[r], dz = b.x - zi[r];
          if (uni) {
            dx = fma(-L, ks[0], dx);
            dy = fma(-L, ks[1], dy);
            dz = fma(-L, ks[2], dz);
          } else {
            dx = fma(-L, rint(dx * invL), dx);
            dy = fma(-L, rint(dy * invL), dy);
            dz = fma(-L, rint(dz * invL), dz);
          }
          const double h = c.x + hi[r];
          if (IMAGES == 1) {
            const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            const double w = pair_w(r2, h, b.y);
            tx[r] = fma(w, dx, tx[r]);
            ty[r] = fma(w, dy, ty[r]);
            tz[r] = fma(w, dz, tz[r]);
          } else if (uni) {
#pragma unroll
            for (int wd = 0; wd < 3; ++wd) {
              unsigned long long mk = cm[wd];
              while (mk) {
                const int q = 64 * wd + __builtin_ctzll(mk);
                mk &= mk - 1;
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
int periodic_iblocks(int n) { return ceil_div_p(n, (long long)kWaveBlock * kRp); }

hipError_t launch_force_periodic(const double *pos, const double *mass,
                                 const double *soft, int n, double L,
                                 int images, int jchunk, int jsplit,
                                 const double *tinfo, double *out,
                                 hipStream_t s) {
  // tinfo is indexed by tile from each split's start: splits tile-aligned
  if (jchunk <= 0 || jchunk % kTJp != 0 || !tinfo ||
      (long long)jchunk * jsplit < n) {
    return hipErrorInvalidValue;
  }
  dim3 grid(periodic_iblocks(n), jsplit);
  if (images == 1) {
    hipLaunchKernelGGL(k_force_periodic<1>, grid, dim3(kWaveBlock), 0, s, pos,
                       mass, soft, n, jchunk, L, tinfo, out);
  } else {
    hipLaunchKernelGGL(k_force_periodic<2>, grid, dim3(kWaveBlock), 0, s, pos,
                       mass, soft, n, jchunk, L, tinfo, out);
  }
  return hipGetLastError();
}

}  // namespace steps
