// gfx950 periodic pair sum of libsteps (StePS, Sec. 2.2, Eqs. 2 and 5): in
// a box of side L the softened force of Eq. 4 is summed over the images
// x_j + n L of every other particle,
//   images = all:     every n with |x_j + n L - x_i| < 2.6 L (the printed
//                     formula: a direct image sum, no Fourier-space part);
//   images = nearest: the leading term only, the nearest image
//                     (quasi-periodic).
// The plain rule brings a pair's displacement to its nearest image,
// d <- d - L rint(d / L) per component (each |d_k| <= L/2); the images
// within 2.6 L of such a d are among the 179 triplets n in [-3, 3]^3 whose
// box [n - 1/2, n + 1/2]^3 (in units of L) comes within 2.6 of the origin,
// listed at compile time below.  A particle's own images cancel in pairs
// (n and -n) and are skipped.  FP64, over Morton-sorted particles; blocks
// of (128 i, 128 j) whose displacement ranges allow it take the shifts or
// image lists once per block instead of per pair (see k_force_periodic);
// per-tile partials added into compensated running totals, j-splits
// reduced in fixed order and scattered back.

#include <type_traits>

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

// m r^-3 with the e^2 term of the correction to v_rsq_f64 (e = 1 - r^2 y^2,
// r^-3 = y^3 (1 + 3/2 e + 15/8 e^2 + O(e^3))), written as
// t (1 + 3/2 e (1 + 5/4 e)) with t = m y^3: each constant is an operand of
// its own instruction, so none has to be rebuilt in a register per pair.
// The image sums cancel heavily, so the periodic kernel keeps the e^2 term.
__device__ __forceinline__ double newton_w64_e2(double r2, double m) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double y2 = y * y;
  const double e = fma(-r2, y2, 1.0);
  const double t = (m * y) * y2;
  const double q = e * fma(e, 1.25, 1.0);
  return fma(t * q, 1.5, t);
}

__device__ __forceinline__ double pair_w(double r2, double h, double m) {
  return r2 <= h * h ? soft_w64(r2, h, m) : newton_w64_e2(r2, m);
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
// it without the per-pair wrap (the same operations on the same values, so
// the same bits).  Such a block whose minimum-image boxes are farther apart
// than the largest combined softening also skips the softening test, and
// applies the shift to its i positions once (x_j - (x_i + k L): rounded at
// the scale of the positions, as the per-pair difference already is).
// With every image (IMAGES = 2), a block takes its candidate images from
// the raw displacement range instead (no wrap), image by image over the
// whole tile: an image whose shifted box lies wholly inside 2.6 L and
// beyond the softening needs no per-pair test, the others keep the cut and
// softening tests; only blocks too wide for eight shifts per axis (particles
// stored far outside the box) wrap each pair and test all 179 candidates.
//
// block (x, y) = (i-block of one wave, j-split); split y writes its
// partial to out + y * 3n.  At most 128 VGPRs, four waves per SIMD (the
// every-image kernel spills a few block-level values outside its pair
// loops to get there).
template <int IMAGES>
__global__ __launch_bounds__(kWaveBlock, 4) void k_force_periodic(
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
    // and the minimum-image gap; the raw (unwrapped) range [rl, rh]
    // Along an axis whose range straddles one half-box (rint of its ends k
    // and k + 1) every pair takes shift k or k + 1, so the wrapped values
    // lie in [lo - k L, L/2] or [-L/2, hi - (k + 1) L] (rounding is
    // monotone): the gap is the nearer of the two.  wrap: bit c set when
    // axis c needs the per-pair wrap.
    const double *ti = tinfo + (size_t)(jt / kTJp) * 8;
    int wrap = 0;
    double ks[3], dl[3], dh[3], rl[3], rh[3], g2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double dmn = ti[c] - wh[c], dmx = ti[3 + c] - wl[c];
      const double fmn = dmn * invL, fmx = dmx * invL;
      const double kc = rint(fmn), kh = rint(fmx);
      const bool ua = fmn > kc - 0.5 && fmx < kc + 0.5;
      wrap |= ua ? 0 : 1 << c;
      ks[c] = kc;
      rl[c] = dmn;
      rh[c] = dmx;
      dl[c] = fma(-L, kc, dmn);
      dh[c] = fma(-L, kc, dmx);
      double g = 0.0;
      if (kh == kc) {
        g = fmax(0.0, fmax(dl[c], -dh[c]));
      } else if (kh == kc + 1.0) {
        g = fmin(fmax(0.0, dl[c]), fmax(0.0, -fma(-L, kh, dmx)));
      }
      g2 = fma(g, g, g2);
    }
    const double hs = ti[6] + whm;
    wrap = __builtin_amdgcn_readfirstlane(wrap);
    const bool uni = wrap == 0;
    // every pair of the block beyond the largest combined softening
    const bool nosoft = __builtin_amdgcn_readfirstlane(
                            (int)(g2 > fmax(hs * hs * (1.0 + 1e-6), 1e-30))) != 0;
    const bool far = uni && nosoft;
    const int kend = min(kTJp, jend - jt);

    // Every image (IMAGES = 2) from the raw displacement range: the image
    // shifts n that can bring a raw displacement of the block within 2.6 L
    // lie in [floor((-2.6 L - rh) / L), ceil((2.6 L - rl) / L)] per axis (a
    // superset: the rounding of the quotients is far below one unit).  With
    // at most 8 per axis, lane t tests the shifts (lo_x + t % 8, lo_y + t / 8)
    // for each lo_z + z, and ballots which boxes come within 2.6 L, which of
    // those lie beyond the largest combined softening (no softening test)
    // and which of these lie wholly inside 2.6 L (no per-pair test at all);
    // the margins are far above the rounding of the per-pair terms.  Blocks
    // holding a particle's own pair take the tested loop, which skips it
    // (its images cancel in pairs).  Wider blocks (particles far outside
    // the box) take the per-pair wrap below.
    int nlo[3] = {0, 0, 0}, ncnt[3] = {0, 0, 0};
    bool raw = IMAGES == 2;
    if (IMAGES == 2) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double sl = floor((-2.6 * L - rh[c]) * invL);
        const double sh = ceil((2.6 * L - rl[c]) * invL);
        const bool ok = sl >= -1.0e6 && sh <= 1.0e6 && sh - sl < 8.0;  // NaN: false
        raw = raw && ok;
        nlo[c] = __builtin_amdgcn_readfirstlane(ok ? (int)sl : 0);
        ncnt[c] = __builtin_amdgcn_readfirstlane(ok ? (int)(sh - sl) + 1 : 0);
      }
      raw = __builtin_amdgcn_readfirstlane((int)raw) != 0;
    }

    double tx[kRp], ty[kRp], tz[kRp];
#pragma unroll
    for (int r = 0; r < kRp; ++r) tx[r] = ty[r] = tz[r] = 0.0;
    if (IMAGES == 1 && far) {
      // one shift for the block, applied to the i side once: the image
      // x_j - k L is at x_j - (x_i + k L); no softening, no coincident pairs
      double qx[kRp], qy[kRp], qz[kRp];
#pragma unroll
      for (int r = 0; r < kRp; ++r) {
        qx[r] = fma(ks[0], L, xi[r]);
        qy[r] = fma(ks[1], L, yi[r]);
        qz[r] = fma(ks[2], L, zi[r]);
      }
      for (int k = 0; k < kend; ++k) {
        const double2 a = tile[3 * k], b = tile[3 * k + 1];
#pragma unroll
        for (int r = 0; r < kRp; ++r) {
          const double dx = a.x - qx[r], dy = a.y - qy[r], dz = b.x - qz[r];
          const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
          const double w = newton_w64_e2(r2, b.y);
          tx[r] = fma(w, dx, tx[r]);
          ty[r] = fma(w, dy, ty[r]);
          tz[r] = fma(w, dz, tz[r]);
        }
      }
    } else if (IMAGES == 2 && raw) {
      const int i0 = blockIdx.x * (kWaveBlock * kRp);
      const bool own = jt < i0 + kWaveBlock * kRp && jt + kend > i0;
      const int lx = tid & 7, ly = tid >> 3;
      const double nx = (double)(nlo[0] + lx), ny = (double)(nlo[1] + ly);
      const double ax0 = fma(nx, L, rl[0]), ax1 = fma(nx, L, rh[0]);
      const double ay0 = fma(ny, L, rl[1]), ay1 = fma(ny, L, rh[1]);
      const double gx = fmax(0.0, fmax(ax0, -ax1)), gy = fmax(0.0, fmax(ay0, -ay1));
      const double fx = fmax(fabs(ax0), fabs(ax1)), fy = fmax(fabs(ay0), fabs(ay1));
      const bool lane_ok = lx < ncnt[0] && ly < ncnt[1];
      const double soft2 = fmax(hs * hs * (1.0 + 1e-6), 1e-30);
      for (int z = 0; z < ncnt[2]; ++z) {
        // this z-slice's images: within 2.6 L (mk); of those, beyond the
        // softening in a block without an own pair (msoft); of these, wholly
        // inside 2.6 L (minside)
        const double nz = (double)(nlo[2] + z);
        const double az0 = fma(nz, L, rl[2]), az1 = fma(nz, L, rh[2]);
        const double gz = fmax(0.0, fmax(az0, -az1)), fz = fmax(fabs(az0), fabs(az1));
        const double gg = fma(gz, gz, fma(gy, gy, gx * gx));
        const double ff = fma(fz, fz, fma(fy, fy, fx * fx));
        const bool kp = lane_ok && gg < cut2 * (1.0 + 1e-9);
        const bool sf = kp && !own && gg > soft2;
        unsigned long long mk = __ballot(kp);
        const unsigned long long msoft = __ballot(sf);
        const unsigned long long minside = __ballot(sf && ff < cut2 * (1.0 - 1e-9));
        while (mk) {
          const int bit = __builtin_ctzll(mk);
          mk &= mk - 1;
          // image x_j + n L: displacement x_j - (x_i - n L)
          const double sx = (double)(nlo[0] + (bit & 7));
          const double sy = (double)(nlo[1] + (bit >> 3));
          double qx[kRp], qy[kRp], qz[kRp];
#pragma unroll
          for (int r = 0; r < kRp; ++r) {
            qx[r] = fma(-sx, L, xi[r]);
            qy[r] = fma(-sy, L, yi[r]);
            qz[r] = fma(-nz, L, zi[r]);
          }
          // no softening test; inside 2.6 L no cut test either (the lanes
          // of a wave hold nearby i, so the cut mostly branches uniformly)
          auto unsoftened = [&](auto cut_tag) {
            constexpr bool CUT = decltype(cut_tag)::value;
#pragma unroll 2
            for (int k = 0; k < kend; ++k) {
              const double2 a = tile[3 * k], b = tile[3 * k + 1];
#pragma unroll
              for (int r = 0; r < kRp; ++r) {
                const double ex = a.x - qx[r], ey = a.y - qy[r], ez = b.x - qz[r];
                const double r2 = fma(ez, ez, fma(ey, ey, ex * ex));
                if (!CUT || r2 < cut2) {
                  const double w = newton_w64_e2(r2, b.y);
                  tx[r] = fma(w, ex, tx[r]);
                  ty[r] = fma(w, ey, ty[r]);
                  tz[r] = fma(w, ez, tz[r]);
                }
              }
            }
          };
          if ((minside >> bit) & 1) {
            unsoftened(std::false_type{});
          } else if ((msoft >> bit) & 1) {
            unsoftened(std::true_type{});
          } else {
            for (int k = 0; k < kend; ++k) {
              const double2 a = tile[3 * k], b = tile[3 * k + 1], c = tile[3 * k + 2];
#pragma unroll
              for (int r = 0; r < kRp; ++r) {
                if (jt + k == ii[r]) continue;  // own images cancel in pairs
                const double ex = a.x - qx[r], ey = a.y - qy[r], ez = b.x - qz[r];
                const double r2 = fma(ez, ez, fma(ey, ey, ex * ex));
                if (r2 < cut2) {
                  const double w = pair_w(r2, c.x + hi[r], b.y);
                  tx[r] = fma(w, ex, tx[r]);
                  ty[r] = fma(w, ey, ty[r]);
                  tz[r] = fma(w, ez, tz[r]);
                }
              }
            }
          }
        }
      }
    } else if (IMAGES == 1) {
      // the per-pair wrap only along the axes that need it (the others
      // shift by k L: the same bits), and no softening test where every
      // pair lies beyond the largest combined softening (such a block holds
      // no coincident or own pair: its gap is positive)
      auto nearest = [&](auto wx, auto wy, auto wz, auto soft_tag) {
        constexpr bool WX = decltype(wx)::value, WY = decltype(wy)::value,
                       WZ = decltype(wz)::value, SOFT = decltype(soft_tag)::value;
        for (int k = 0; k < kend; ++k) {
          const double2 a = tile[3 * k], b = tile[3 * k + 1], c = tile[3 * k + 2];
#pragma unroll
          for (int r = 0; r < kRp; ++r) {
            if (SOFT && jt + k == ii[r]) continue;  // own images cancel in pairs
            double dx = a.x - xi[r], dy = a.y - yi[r], dz = b.x - zi[r];
            dx = fma(-L, WX ? rint(dx * invL) : ks[0], dx);
            dy = fma(-L, WY ? rint(dy * invL) : ks[1], dy);
            dz = fma(-L, WZ ? rint(dz * invL) : ks[2], dz);
            const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            const double w = SOFT ? pair_w(r2, c.x + hi[r], b.y) : newton_w64_e2(r2, b.y);
            tx[r] = fma(w, dx, tx[r]);
            ty[r] = fma(w, dy, ty[r]);
            tz[r] = fma(w, dz, tz[r]);
          }
        }
      };
      using T = std::true_type;
      using F = std::false_type;
      auto by_soft = [&](auto wx, auto wy, auto wz) {
        if (nosoft) {
          nearest(wx, wy, wz, F{});
        } else {
          nearest(wx, wy, wz, T{});
        }
      };
      switch (wrap) {
        case 0: by_soft(F{}, F{}, F{}); break;
        case 1: by_soft(T{}, F{}, F{}); break;
        case 2: by_soft(F{}, T{}, F{}); break;
        case 3: by_soft(T{}, T{}, F{}); break;
        case 4: by_soft(F{}, F{}, T{}); break;
        case 5: by_soft(T{}, F{}, T{}); break;
        case 6: by_soft(F{}, T{}, T{}); break;
        default: by_soft(T{}, T{}, T{}); break;
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
          {
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
