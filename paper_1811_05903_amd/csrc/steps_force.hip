// gfx950 pair-sum kernels of libsteps: the all-pairs spline-softened sum of
// StePS (Racz et al. 2018, Sec. 2.2 Eqs. 3, 4 and 8),
//   S_i = sum_{j != i} m_j F(r_ij, h_i + h_j) (x_j - x_i) / r_ij.
//
// Layout common to every variant:
//   * a workgroup is 256 lanes = 4 wave64.  Wave w of block b owns the
//     64*R consecutive particles starting at b*256*R + w*64*R; lane l holds
//     i = start + 64*r + l for r < R in registers (coalesced loads/stores);
//   * grid.y splits the j range into jsplit chunks (multiples of TJ); each
//     chunk streams through LDS in tiles of TJ particles, staged with
//     coalesced SoA reads and read back by every lane as broadcasts (the
//     symmetric kernel instead runs a 1-D grid of chunk pairs, each pair
//     evaluated once for both particles);
//   * a lane sums a tile's terms into a per-tile partial and adds it to its
//     running total after the tile (blocked summation: rounding grows with
//     TJ + N/TJ rather than N; in FP64 the running total is also
//     compensated); no atomics, so a launch shape gives a
//     bitwise-reproducible result.
//
// The softened branch of Eq. 4 applies only to pairs closer than
// h_i + h_j.  Two ways to handle it:
//   * CULL = false: every pair is tested (h add, h^2, compare) and a wave
//     takes the softened branch only when one of its lanes needs it;
//   * CULL = true: particles arrive sorted along a space-filling curve, the
//     host has computed each j-tile's bounding box and largest softening,
//     and each wave computes the same for its own i.  When the boxes are
//     farther apart than the two largest softenings combined, no pair of the
//     (wave, tile) block can be softened or coincident, and the wave runs a
//     loop with the Newtonian weight only -- no per-pair test at all.
//     Otherwise it runs the tested loop.

#include <algorithm>

#include "steps_internal.h"
#include "steps_pair.h"

namespace steps {
namespace {

// ---------------------------------------------------------------------------
// wave-level helpers for the culling test
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
// a value equal on every lane, moved to scalar registers
__device__ __forceinline__ double uniform(double v) {
  unsigned long long b = __double_as_longlong(v);
  unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

// Wave box: (xlo, ylo, zlo, xhi, yhi, zhi, hmax) over the wave's valid i.
template <int R, typename T>
__device__ __forceinline__ void wave_box(const T *xi, const T *yi, const T *zi,
                                         const T *hi, const bool *valid,
                                         double wb[7]) {
  double lo[3] = {INFINITY, INFINITY, INFINITY};
  double up[3] = {-INFINITY, -INFINITY, -INFINITY};
  double hm = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (valid[r]) {
      lo[0] = fmin(lo[0], (double)xi[r]); up[0] = fmax(up[0], (double)xi[r]);
      lo[1] = fmin(lo[1], (double)yi[r]); up[1] = fmax(up[1], (double)yi[r]);
      lo[2] = fmin(lo[2], (double)zi[r]); up[2] = fmax(up[2], (double)zi[r]);
      hm = fmax(hm, (double)hi[r]);
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    wb[d] = uniform(wave_min(lo[d]));
    wb[3 + d] = uniform(wave_max(up[d]));
  }
  wb[6] = uniform(wave_max(hm));
}

// True when no pair between the wave box and the tile box
// (tile info: xlo, ylo, zlo, xhi, yhi, zhi, hmax) can be closer than the
// largest combined softening, nor coincide.
__device__ __forceinline__ bool tile_is_far(const double *__restrict__ ti,
                                            const double wb[7]) {
  const double gx = fmax(0.0, fmax(ti[0] - wb[3], wb[0] - ti[3]));
  const double gy = fmax(0.0, fmax(ti[1] - wb[4], wb[1] - ti[4]));
  const double gz = fmax(0.0, fmax(ti[2] - wb[5], wb[2] - ti[5]));
  const double d2 = gx * gx + gy * gy + gz * gz;
  const double hs = ti[6] + wb[6];
  const bool far = d2 > fmax(hs * hs * (1.0 + 1e-6), 1e-30);
  return __builtin_amdgcn_readfirstlane((int)far) != 0;
}

// ---------------------------------------------------------------------------
// One block's share of the sum, FP64.  The block owns the 256*R particles
// [i0, min(i0 + 256 R, iend)) and sums over j in [jbeg, jend).  SoA arrays
// have component stride `stride`; tinfo (CULL) points at the info of the
// tile that starts at jbeg, tiles being consecutive from there.  Results go
// to out[c * stride + i].  LDS tile: per j three double2 = (x, y), (z, m),
// (h, -).  Must be called by all threads of the block.
// ---------------------------------------------------------------------------
template <int R, int TJ, bool E2, bool CULL>
__device__ __forceinline__ void force_block_f64(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const double *__restrict__ soft, int stride, int i0, int iend, int jbeg,
    int jend, const double *__restrict__ tinfo, double *__restrict__ out,
    double2 *tile) {
  const int tid = threadIdx.x;
  const int ibase = i0 + (tid >> 6) * (64 * R) + (tid & 63);
  const double *X = pos, *Y = pos + stride, *Z = pos + 2 * (size_t)stride;

  double xi[R], yi[R], zi[R], hi[R];
  double ax[R], ay[R], az[R], cx[R], cy[R], cz[R];  // total + compensation
  bool valid[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = ibase + 64 * r;
    valid[r] = i < iend;
    xi[r] = valid[r] ? X[i] : 0.0;
    yi[r] = valid[r] ? Y[i] : 0.0;
    zi[r] = valid[r] ? Z[i] : 0.0;
    hi[r] = valid[r] ? soft[i] : 0.0;
    ax[r] = ay[r] = az[r] = cx[r] = cy[r] = cz[r] = 0.0;
  }
  double wb[7];
  if (CULL) wave_box<R, double>(xi, yi, zi, hi, valid, wb);

  for (int jt = jbeg; jt < jend; jt += TJ) {
    __syncthreads();
    for (int k = tid; k < TJ; k += kBlock) {
      // entries past the end repeat the last particle with zero mass: they
      // add nothing and never sit outside the tile's box
      const int j = min(jt + k, jend - 1);
      const double mj = (jt + k < jend) ? mass[j] : 0.0;
      tile[3 * k] = double2{X[j], Y[j]};
      tile[3 * k + 1] = double2{Z[j], mj};
      tile[3 * k + 2] = double2{soft[j], 0.0};
    }
    __syncthreads();

    bool far = false;
    if (CULL) far = tile_is_far(tinfo + (size_t)((jt - jbeg) / TJ) * 8, wb);

    double tx[R], ty[R], tz[R];
#pragma unroll
    for (int r = 0; r < R; ++r) tx[r] = ty[r] = tz[r] = 0.0;

    if (far) {
#pragma unroll 2
      for (int k = 0; k < TJ; ++k) {
        const double2 a = tile[3 * k], b = tile[3 * k + 1];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double dx = a.x - xi[r], dy = a.y - yi[r], dz = b.x - zi[r];
          const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
          const double w = newton_w64<E2>(r2, b.y);
          tx[r] = fma(w, dx, tx[r]);
          ty[r] = fma(w, dy, ty[r]);
          tz[r] = fma(w, dz, tz[r]);
        }
      }
    } else {
#pragma unroll 2
      for (int k = 0; k < TJ; ++k) {
        const double2 a = tile[3 * k], b = tile[3 * k + 1], c = tile[3 * k + 2];
        const double xj = a.x, yj = a.y, zj = b.x, mj = b.y, hj = c.x;
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
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      two_sum_add(ax[r], cx[r], tx[r]);
      two_sum_add(ay[r], cy[r], ty[r]);
      two_sum_add(az[r], cz[r], tz[r]);
    }
  }

#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = ibase + 64 * r;
    if (i < iend) {
      out[i] = ax[r] + cx[r];
      out[(size_t)stride + i] = ay[r] + cy[r];
      out[2 * (size_t)stride + i] = az[r] + cz[r];
    }
  }
}

// ---------------------------------------------------------------------------
// One block's share, FP64, with both contractions of the far field on the
// matrix cores.  Relative to a centre c (the j-tile's box centre), with
// u = x - c and q = |u|^2, a pair's squared distance is a Gram product
//   r_ij^2 = q_i + sum_k (-2 u_i, 1)_k (u_j, q_j)_k,
// and the tile's contribution to S_i is a matrix product minus a rank-one
// term,
//   sum_j m_j r_ij^-3 (x_j - x_i) = sum_j w_ij (u_j) - u_i sum_j w_ij,
// both sums being one product of the weight matrix with (m_j u_j, m_j).
// v_mfma_f64_4x4x4_4b forms 4 blocks of (4 x 4) += (4 x 4)(4 x 4) per
// wave, so one instruction yields r^2 for 64 pairs (16 i by 4 j) and a
// second accumulates their weights; the vector ALU is left with the rsqrt
// and four operations per pair.  The output lane layout of the first
// product is the A-operand layout of the second, so the weights never
// move between lanes.  On gfx950 FP64 matrix and vector work share one
// pipe (they do not co-issue), so the gain is only the operations saved:
// per 64 pairs two MFMAs cost 8 vector slots and replace about 11.
//
// The Gram form loses about eps (|u_i| + |u_j|)^2 of r^2.  It is used only
// for (wave, tile) blocks that are Newtonian (as in the culled kernels) and
// well separated: |c_i - c_t| + |e_i| + |e_t| <= kSep * gap, where c, e are
// the boxes' centres and half-diagonals and gap is their distance; then the
// relative error of r^2 is below ~2 kSep^2 eps (8e-15 for kSep = 6, under
// the first-order rsqrt residual that the VALU kernel accepts).  Other
// blocks take the direct per-pair loop (one particle per lane, softening
// tested where the boxes are near).  The wave owns 64 consecutive sorted
// particles.
//
// Lane roles of v_mfma_f64_4x4x4_4b on gfx950, lane l = n + 4 b + 16 k
// for A (row n) and B (column n) with K index k, and l = n + 4 b + 16 m for
// D (row m, column n), b the block.
// ---------------------------------------------------------------------------
constexpr double kSep = 6.0;
// The symmetric kernels send more blocks to the matrix cores: with
// kSepSym = 12 the Gram form's r^2 error stays below ~2 kSepSym^2 eps =
// 3.2e-14 relative (measured 5% faster than 6 at N = 2^18, with unchanged
// errors against the oracle).
constexpr double kSepSym = 12.0;

__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// every lane of a quad (4 consecutive lanes) takes the quad's lane 3 (DPP
// quad_perm [3, 3, 3, 3])
__device__ __forceinline__ double quad_bcast3(double v) {
  const unsigned long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, 0xFF, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), 0xFF, 0xF,
                                          0xF, true);
  return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) |
                              (unsigned)lo);
}

// v rotated right by N lanes within each row of 16 lanes (DPP row_ror)
template <int N>
__device__ __forceinline__ double row_ror(double v) {
  static_assert(N > 0 && N < 16, "row_ror takes 1..15");
  const unsigned long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, 0x120 + N, 0xF,
                                          0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), 0x120 + N,
                                          0xF, 0xF, true);
  return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) |
                              (unsigned)lo);
}

// every lane takes the value of lane (l + 1) mod 64 (DPP wave_rol:1)
__device__ __forceinline__ double wave_rol1(double v) {
  const unsigned long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, 0x134, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), 0x134, 0xF,
                                          0xF, true);
  return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) |
                              (unsigned)lo);
}

// ---------------------------------------------------------------------------
// A (wave, tile) block of the symmetric FP64 kernels off the matrix cores,
// each pair once (the pair term is antisymmetric, Sec. 2.2 Eq. 8).  Lane l
// holds i = wave base + l; the tile is taken in parts of 64 j, and in step t
// of a part lane l pairs its i with j = (l + t) mod 64 of the part, read
// from LDS, so no two lanes share a j within a step.  One weight w per pair
// serves both sides: the i-side sums m_j w (x_j - x_i) stay in the lane; the
// j-side sums m_i w (x_i - x_j) travel with their j, every lane taking its
// right neighbour's sums after each step (the sums of the j it meets next).
// After 64 steps lane l holds the sums of j = l of the part, stored to
// jb[3 k + c] (k the tile index of the j).  Blocks whose pairs all lie
// beyond their softening radius (farw) skip the softening test.  Lanes past
// the end of the chunk carry zero mass.  Additions run in a fixed order.
// ---------------------------------------------------------------------------
template <int TJ>
__device__ __forceinline__ void near_block_f64(const double2 *tile, double xi,
                                               double yi, double zi, double hi,
                                               double mi, bool farw, int l,
                                               double &tx, double &ty,
                                               double &tz, double *jb) {
  tx = ty = tz = 0.0;
  for (int p = 0; p < TJ / 64; ++p) {
    double jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll 2
    for (int t = 0; t < 64; ++t) {
      const int k = 64 * p + ((l + t) & 63);
      const double2 a = tile[3 * k], b = tile[3 * k + 1];
      const double dx = a.x - xi, dy = a.y - yi, dz = b.x - zi;
      const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
      double w = newton_w64<true>(r2, 1.0);
      if (!farw) {
        const double h = tile[3 * k + 2].x + hi;
        if (r2 <= h * h) w = soft_w64(r2, h, 1.0);
      }
      const double wi = b.y * w, wj = mi * w;
      tx = fma(wi, dx, tx);
      ty = fma(wi, dy, ty);
      tz = fma(wi, dz, tz);
      jx = wave_rol1(fma(-wj, dx, jx));
      jy = wave_rol1(fma(-wj, dy, jy));
      jz = wave_rol1(fma(-wj, dz, jz));
    }
    const int k = 64 * p + l;
    jb[3 * k] = jx;
    jb[3 * k + 1] = jy;
    jb[3 * k + 2] = jz;
  }
}

template <int TJ>
__device__ __forceinline__ void force_block_f64_mfma(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const double *__restrict__ soft, int stride, int i0, int iend, int jbeg,
    int jend, const double *__restrict__ tinfo, double *__restrict__ out,
    double2 *tile, double *gram, double *bmat, int ostride = -1,
    int obase = 0) {
  // results go to out[c * ostride + i - obase] (ostride < 0: stride)
  const size_t os = ostride < 0 ? (size_t)stride : (size_t)ostride;
  const int tid = threadIdx.x;
  const int l = tid & 63;
  const int wbase = i0 + (tid >> 6) * 64;
  const int last = iend - 1;
  const double *X = pos, *Y = pos + stride, *Z = pos + 2 * (size_t)stride;

  // direct loop: lane l owns particle wbase + l
  const bool valid = wbase + l < iend;
  const int ip = min(wbase + l, last);
  const double xi = X[ip], yi = Y[ip], zi = Z[ip], hi = soft[ip];
  // matrix path: lane l is i-slot (l & 3) of block (l >> 2) & 3 in the
  // operands (particle 16 r + (l & 15)), K index l >> 4, and holds component
  // (l & 3) of particle 16 r + 4 ((l >> 2) & 3) + (l >> 4) in the output
  const int kk = l >> 4, cc = l & 3;
  const double *Pc = cc == 0 ? X : (cc == 1 ? Y : Z);
  double gx[4], gy[4], gz[4], dc[4], sum[4], cmp[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ig = min(wbase + 16 * r + (l & 15), last);
    gx[r] = X[ig];
    gy[r] = Y[ig];
    gz[r] = Z[ig];
    const int id = min(wbase + 16 * r + 4 * ((l >> 2) & 3) + (l >> 4), last);
    dc[r] = cc < 3 ? Pc[id] : 0.0;
    sum[r] = cmp[r] = 0.0;
  }
  double wb[7];
  {
    const double xs[1] = {xi}, ys[1] = {yi}, zs[1] = {zi}, hs[1] = {hi};
    const bool vs[1] = {valid};
    wave_box<1, double>(xs, ys, zs, hs, vs, wb);
  }
  const double wc[3] = {0.5 * (wb[0] + wb[3]), 0.5 * (wb[1] + wb[4]),
                        0.5 * (wb[2] + wb[5])};
  const double we = 0.5 * sqrt((wb[3] - wb[0]) * (wb[3] - wb[0]) +
                               (wb[4] - wb[1]) * (wb[4] - wb[1]) +
                               (wb[5] - wb[2]) * (wb[5] - wb[2]));

  for (int jt = jbeg; jt < jend; jt += TJ) {
    const double *ti = tinfo + (size_t)((jt - jbeg) / TJ) * 8;
    const double ct[3] = {0.5 * (ti[0] + ti[3]), 0.5 * (ti[1] + ti[4]),
                          0.5 * (ti[2] + ti[5])};
    __syncthreads();
    for (int k = tid; k < TJ; k += kBlock) {
      const int j = min(jt + k, jend - 1);
      const double mj = (jt + k < jend) ? mass[j] : 0.0;
      const double xj = X[j], yj = Y[j], zj = Z[j];
      tile[3 * k] = double2{xj, yj};
      tile[3 * k + 1] = double2{zj, mj};
      tile[3 * k + 2] = double2{soft[j], 0.0};
      const double ux = xj - ct[0], uy = yj - ct[1], uz = zj - ct[2];
      const double mm = -1.5 * mj;
      gram[4 * k] = ux;
      gram[4 * k + 1] = uy;
      gram[4 * k + 2] = uz;
      gram[4 * k + 3] = fma(uz, uz, fma(uy, uy, ux * ux));
      bmat[4 * k] = mm * ux;
      bmat[4 * k + 1] = mm * uy;
      bmat[4 * k + 2] = mm * uz;
      bmat[4 * k + 3] = mm;
    }
    __syncthreads();

    // box gap and separation, uniform over the wave
    const double gxv = fmax(0.0, fmax(ti[0] - wb[3], wb[0] - ti[3]));
    const double gyv = fmax(0.0, fmax(ti[1] - wb[4], wb[1] - ti[4]));
    const double gzv = fmax(0.0, fmax(ti[2] - wb[5], wb[2] - ti[5]));
    const double d2 = gxv * gxv + gyv * gyv + gzv * gzv;
    const double hs = ti[6] + wb[6];
    const bool far = d2 > fmax(hs * hs * (1.0 + 1e-6), 1e-30);
    const double te = 0.5 * sqrt((ti[3] - ti[0]) * (ti[3] - ti[0]) +
                                 (ti[4] - ti[1]) * (ti[4] - ti[1]) +
                                 (ti[5] - ti[2]) * (ti[5] - ti[2]));
    const double cd = sqrt((wc[0] - ct[0]) * (wc[0] - ct[0]) +
                           (wc[1] - ct[1]) * (wc[1] - ct[1]) +
                           (wc[2] - ct[2]) * (wc[2] - ct[2]));
    const bool sep = far && (cd + we + te) <= kSep * sqrt(d2);
    const bool use_mfma = __builtin_amdgcn_readfirstlane((int)sep) != 0;

    double part[4];
    if (use_mfma) {
      double b1[4], qi[4], d2acc[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double ux = gx[r] - ct[0], uy = gy[r] - ct[1], uz = gz[r] - ct[2];
        const double uk = kk == 0 ? ux : (kk == 1 ? uy : uz);
        b1[r] = kk < 3 ? -2.0 * uk : 1.0;
        qi[r] = fma(uz, uz, fma(uy, uy, ux * ux));
        d2acc[r] = 0.0;
      }
      const int arow = 4 * (l & 3) + kk;  // gram[4 (4g + (l & 3)) + k]
      const int brow = 4 * kk + cc;       // bmat[4 (4g + k) + c]
      // not unrolled: measured 2% faster than unrolling by 2 (the four
      // independent r chains already give the scheduler enough to interleave)
#pragma unroll 1
      for (int g = 0; g < TJ / 4; ++g) {
        const double a1 = gram[16 * g + arow];
        const double b2 = bmat[16 * g + brow];
        double rr[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) rr[r] = mfma4(a1, b1[r], qi[r]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double y = __builtin_amdgcn_rsq(rr[r]);
          const double y2 = y * y;
          const double t = fma(rr[r], y2, -5.0 / 3.0);
          const double w = (y * y2) * t;  // -(2/3) r^-3 (1 + 3/2 e)
          d2acc[r] = mfma4(w, b2, d2acc[r]);
        }
      }
      // column 3 holds sum_j m_j r^-3; subtract u_i times it
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double s3 = __shfl(d2acc[r], l | 3);
        const double ctc = cc == 0 ? ct[0] : (cc == 1 ? ct[1] : ct[2]);
        const double ui = cc < 3 ? dc[r] - ctc : 0.0;
        part[r] = fma(-ui, s3, d2acc[r]);
      }
    } else {
      double tx = 0.0, ty = 0.0, tz = 0.0;
      if (__builtin_amdgcn_readfirstlane((int)far)) {
#pragma unroll 4
        for (int k = 0; k < TJ; ++k) {
          const double2 a = tile[3 * k], b = tile[3 * k + 1];
          const double dx = a.x - xi, dy = a.y - yi, dz = b.x - zi;
          const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
          const double w = newton_w64<true>(r2, b.y);
          tx = fma(w, dx, tx);
          ty = fma(w, dy, ty);
          tz = fma(w, dz, tz);
        }
      } else {
#pragma unroll 2
        for (int k = 0; k < TJ; ++k) {
          const double2 a = tile[3 * k], b = tile[3 * k + 1], c = tile[3 * k + 2];
          const double dx = a.x - xi, dy = a.y - yi, dz = b.x - zi;
          const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
          const double h = c.x + hi;
          double w = newton_w64<true>(r2, b.y);
          if (r2 <= h * h) w = soft_w64(r2, h, b.y);
          tx = fma(w, dx, tx);
          ty = fma(w, dy, ty);
          tz = fma(w, dz, tz);
        }
      }
      // to the output layout: component cc of particle 16 r + 4 b + (l >> 4)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int src = 16 * r + 4 * ((l >> 2) & 3) + (l >> 4);
        const double vx = __shfl(tx, src), vy = __shfl(ty, src), vz = __shfl(tz, src);
        part[r] = cc == 0 ? vx : (cc == 1 ? vy : (cc == 2 ? vz : 0.0));
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) two_sum_add(sum[r], cmp[r], part[r]);
  }

#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int id = wbase + 16 * r + 4 * ((l >> 2) & 3) + (l >> 4);
    if (cc < 3 && id < iend) out[(size_t)cc * os + id - obase] = sum[r] + cmp[r];
  }
}

// ---------------------------------------------------------------------------
// Symmetric FP64 evaluation (Newton's third law).  The pair term of Eq. 8
// is antisymmetric: the pull of j on i is m_j F/r (x_j - x_i) and that of
// i on j is m_i F/r (x_i - x_j), with the same F(r, h_i + h_j)/r.  The sorted
// particles are cut into chunks of C (a multiple of 256) and a workgroup
// takes one unit (R, s), R <= s, of chunk pairs.  For R < s it evaluates
// each pair of chunk R x chunk s once and keeps both sides:
//   * i-side (chunk R): the weights summed against (m_j u_j, m_j) in
//     registers, as in force_block_f64_mfma, written to plane s of iplane;
//   * j-side (chunk s): the same weights summed against (m_i u_i, m_i).  In
//     the matrix-core path pair (i, j) sits in lane n + 4b + 16m, i the
//     row n of block b and j the row m; a product on v_mfma_f64_4x4x4_4b
//     contracts over the high lane index, so the weights are transposed
//     within each 4 x 4 block (lane permute) before the second product, and
//     the four blocks' partials are added across lanes.  A near block
//     takes each pair once in near_block_f64 (both sides from one weight).
//     Each wave leaves its per-tile j sums in LDS; after the tile they are
//     added in wave order and then into the unit's compensated accumulator
//     (value, error) [6][C] in global memory, which only this workgroup
//     touches.
// A diagonal unit (R == s) sums its chunk one-sided into plane s.  Every
// output word has one writer and a fixed order of additions, so a launch
// shape gives a bitwise-reproducible result.
// ---------------------------------------------------------------------------
template <int TJ>
__device__ __forceinline__ void sym_block_f64(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const double *__restrict__ soft, int stride, int i0, int iend, int jbeg,
    int jend, const double *__restrict__ tinfo, double *__restrict__ out,
    double *__restrict__ jacc, int chunk, bool first, double2 *tile,
    double *gram, double *bmat, double *jbuf) {
  static_assert(TJ == kBlock, "one thread per tile particle in the j-side sum");
  const int tid = threadIdx.x;
  const int l = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wbase = i0 + wv * 64;
  const int last = iend - 1;
  const int nw = max(0, min(64, iend - wbase));  // valid i of this wave
  const double *X = pos, *Y = pos + stride, *Z = pos + 2 * (size_t)stride;
  double *jb = jbuf + (size_t)wv * TJ * 3;  // this wave's [TJ][3] j sums

  const bool valid = wbase + l < iend;
  const int ip = min(wbase + l, last);
  const double xi = X[ip], yi = Y[ip], zi = Z[ip], hi = soft[ip];
  // matrix path roles as in force_block_f64_mfma; lane l also holds the mass
  // of particle 16 r + 4 ((l >> 2) & 3) + (l >> 4) (zero past iend, so that
  // padding lanes add nothing to the j-side)
  const int kk = l >> 4, cc = l & 3;
  const double *Pc = cc == 0 ? X : (cc == 1 ? Y : Z);
  // (the operand-layout coordinates and masses are re-read from cache per
  // tile rather than held, to keep the register count at three waves)
  double dc[4], sum[4], cmp[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int id = wbase + 16 * r + 4 * ((l >> 2) & 3) + (l >> 4);
    dc[r] = cc < 3 ? Pc[min(id, last)] : 0.0;
    sum[r] = cmp[r] = 0.0;
  }
  double wb[7];
  {
    const double xs[1] = {xi}, ys[1] = {yi}, zs[1] = {zi}, hs[1] = {hi};
    const bool vs[1] = {valid};
    wave_box<1, double>(xs, ys, zs, hs, vs, wb);
  }
  const double wc[3] = {0.5 * (wb[0] + wb[3]), 0.5 * (wb[1] + wb[4]),
                        0.5 * (wb[2] + wb[5])};
  const double we = 0.5 * sqrt((wb[3] - wb[0]) * (wb[3] - wb[0]) +
                               (wb[4] - wb[1]) * (wb[4] - wb[1]) +
                               (wb[5] - wb[2]) * (wb[5] - wb[2]));
  // transpose within 4 x 4 blocks: lane n + 4b + 16m reads n' = m, m' = n
  const int tsrc = ((l >> 4) & 3) | (l & 12) | ((l & 3) << 4);

  for (int jt = jbeg; jt < jend; jt += TJ) {
    const double *ti = tinfo + (size_t)((jt - jbeg) / TJ) * 8;
    const double ct[3] = {0.5 * (ti[0] + ti[3]), 0.5 * (ti[1] + ti[4]),
                          0.5 * (ti[2] + ti[5])};
    __syncthreads();
    for (int k = tid; k < TJ; k += kBlock) {
      const int j = min(jt + k, jend - 1);
      const double mj = (jt + k < jend) ? mass[j] : 0.0;
      const double xj = X[j], yj = Y[j], zj = Z[j];
      tile[3 * k] = double2{xj, yj};
      tile[3 * k + 1] = double2{zj, mj};
      tile[3 * k + 2] = double2{soft[j], 0.0};
      const double ux = xj - ct[0], uy = yj - ct[1], uz = zj - ct[2];
      const double mm = -1.5 * mj;
      gram[4 * k] = ux;
      gram[4 * k + 1] = uy;
      gram[4 * k + 2] = uz;
      gram[4 * k + 3] = fma(uz, uz, fma(uy, uy, ux * ux));
      bmat[4 * k] = mm * ux;
      bmat[4 * k + 1] = mm * uy;
      bmat[4 * k + 2] = mm * uz;
      bmat[4 * k + 3] = mm;
    }
    const bool jown = jt + tid < jend;
    const size_t jl = (size_t)(jt + tid - jbeg);
    __syncthreads();

    const double gxv = fmax(0.0, fmax(ti[0] - wb[3], wb[0] - ti[3]));
    const double gyv = fmax(0.0, fmax(ti[1] - wb[4], wb[1] - ti[4]));
    const double gzv = fmax(0.0, fmax(ti[2] - wb[5], wb[2] - ti[5]));
    const double d2 = gxv * gxv + gyv * gyv + gzv * gzv;
    const double hs = ti[6] + wb[6];
    const bool far = d2 > fmax(hs * hs * (1.0 + 1e-6), 1e-30);
    const double te = 0.5 * sqrt((ti[3] - ti[0]) * (ti[3] - ti[0]) +
                                 (ti[4] - ti[1]) * (ti[4] - ti[1]) +
                                 (ti[5] - ti[2]) * (ti[5] - ti[2]));
    const double cd = sqrt((wc[0] - ct[0]) * (wc[0] - ct[0]) +
                           (wc[1] - ct[1]) * (wc[1] - ct[1]) +
                           (wc[2] - ct[2]) * (wc[2] - ct[2]));
    const bool sep = far && (cd + we + te) <= kSepSym * sqrt(d2);
    const bool use_mfma = __builtin_amdgcn_readfirstlane((int)sep) != 0;

    double part[4] = {0.0, 0.0, 0.0, 0.0};
    if (nw == 0) {
      // a wave past the end of the chunk: nothing on either side
      for (int k = l; k < 3 * TJ; k += 64) jb[k] = 0.0;
    } else if (use_mfma) {
      double b1[4], qi[4], d2acc[4], bi[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ig = min(wbase + 16 * r + (l & 15), last);
        const double ux = X[ig] - ct[0], uy = Y[ig] - ct[1], uz = Z[ig] - ct[2];
        const double uk = kk == 0 ? ux : (kk == 1 ? uy : uz);
        b1[r] = kk < 3 ? -2.0 * uk : 1.0;
        qi[r] = fma(uz, uz, fma(uy, uy, ux * ux));
        d2acc[r] = 0.0;
        const int id = wbase + 16 * r + 4 * ((l >> 2) & 3) + (l >> 4);
        const double m = id < iend ? mass[min(id, last)] : 0.0;
        const double ctc = cc == 0 ? ct[0] : (cc == 1 ? ct[1] : ct[2]);
        bi[r] = -1.5 * m * (cc < 3 ? dc[r] - ctc : 1.0);
      }
      const int arow = 4 * (l & 3) + kk;
      const int brow = 4 * kk + cc;
      // j-side of group g: lane c + 4b + 16m sums, over the i of block b,
      // w (m_i u_i, m_i)_c for j = 4g + m (two chains of two products);
      // the four blocks are added with row rotations (DPP), component c < 3
      // becomes D_c - u_{j,c} D_3 (D_3 broadcast within the quad, u from
      // gram at the lane's own (m, c)), and lanes b = 0 store.  Pipelined
      // one group behind the i-side, so that the lane permutes of a group
      // land while the next one is computed.
      double wt[4], ujp = 0.0;
      auto jside = [&](int g) {
        double j0 = mfma4(wt[0], bi[0], 0.0);
        double j1 = mfma4(wt[2], bi[2], 0.0);
        j0 = mfma4(wt[1], bi[1], j0);
        j1 = mfma4(wt[3], bi[3], j1);
        double jd = j0 + j1;
        jd += row_ror<4>(jd);
        jd += row_ror<8>(jd);
        const double f = fma(-ujp, quad_bcast3(jd), jd);
        if ((l & 12) == 0 && cc < 3) jb[3 * (4 * g + kk) + cc] = f;
      };
      double a1n = gram[arow], b2n = bmat[brow], ujn = gram[brow];
      // unrolled by 32 (half the tile): measured 3% faster at N = 2^18 than
      // by two, which was 2-4% faster than none; same 168 VGPRs
#pragma unroll 32
      for (int g = 0; g < TJ / 4; ++g) {
        const double a1 = a1n, b2 = b2n;
        const int gn = min(g + 1, TJ / 4 - 1);
        a1n = gram[16 * gn + arow];
        b2n = bmat[16 * gn + brow];
        double rr[4], w[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) rr[r] = mfma4(a1, b1[r], qi[r]);
        if (g > 0) jside(g - 1);
        ujp = ujn;
        ujn = gram[16 * gn + brow];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double y = __builtin_amdgcn_rsq(rr[r]);
          const double y2 = y * y;
          const double t = fma(rr[r], y2, -5.0 / 3.0);
          w[r] = (y * y2) * t;  // -(2/3) r^-3 (1 + 3/2 e)
          d2acc[r] = mfma4(w[r], b2, d2acc[r]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) wt[r] = __shfl(w[r], tsrc);
      }
      jside(TJ / 4 - 1);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double s3 = __shfl(d2acc[r], l | 3);
        const double ctc = cc == 0 ? ct[0] : (cc == 1 ? ct[1] : ct[2]);
        const double ui = cc < 3 ? dc[r] - ctc : 0.0;
        part[r] = fma(-ui, s3, d2acc[r]);
      }
    } else {
      // near block: each pair once, lane = i; i-side sums moved into the
      // matrix-core output layout
      double tx, ty, tz;
      near_block_f64<TJ>(tile, xi, yi, zi, hi, valid ? mass[ip] : 0.0,
                         __builtin_amdgcn_readfirstlane((int)far) != 0, l, tx,
                         ty, tz, jb);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int src = 16 * r + 4 * ((l >> 2) & 3) + (l >> 4);
        const double vx = __shfl(tx, src), vy = __shfl(ty, src), vz = __shfl(tz, src);
        part[r] = cc == 0 ? vx : (cc == 1 ? vy : (cc == 2 ? vz : 0.0));
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) two_sum_add(sum[r], cmp[r], part[r]);
    // this thread's accumulator entry (j = jt + tid), read while the other
    // waves finish
    double acc6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (!first && jown) {
#pragma unroll
      for (int c = 0; c < 6; ++c) acc6[c] = jacc[(size_t)c * chunk + jl];
    }
    __syncthreads();

    // tile's j-side: the four waves' sums in order, into the accumulator
    if (jown) {
      const int k = tid;
      double f[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        f[c] = ((jbuf[3 * k + c] + jbuf[3 * (TJ + k) + c]) +
                jbuf[3 * (2 * TJ + k) + c]) + jbuf[3 * (3 * TJ + k) + c];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (first) {
          acc6[c] = f[c];
          acc6[3 + c] = 0.0;
        } else {
          two_sum_add(acc6[c], acc6[3 + c], f[c]);
        }
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) jacc[(size_t)c * chunk + jl] = acc6[c];
    }
  }

#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int id = wbase + 16 * r + 4 * ((l >> 2) & 3) + (l >> 4);
    if (cc < 3 && id < iend) out[(size_t)cc * stride + id] = sum[r] + cmp[r];
  }
}

// ---------------------------------------------------------------------------
// Symmetric FP64 evaluation, j-quad layout (variant 30).  Same units, plane
// and accumulator layout, reduction and near-block path as sym_block_f64;
// the far blocks assign the matrix-core lanes the other way round.  In
// v_mfma_f64_4x4x4_4b the four blocks now hold four different j-quads
// against the same four i (an i-quad), and a wave sweeps its 16 i-quads for
// each group of 16 j:
//   * Gram product: r^2 (i row ii, j column jj of block b) = q_j +
//     (-2 u_i, q_i) . (u_j, 1), lane jj + 4b + 16 ii;
//   * j-side: the weights are already the A operand of a product that
//     contracts over the i of the quad (lane bits 4-5), so one MFMA per
//     i-quad, chained over the 16 i-quads, gives the j sums of all 64 i of
//     the wave: no cross-lane reduction per group;
//   * i-side: the weights transposed within each 4 x 4 block (lane permute)
//     are the A operand of the product with the j operand -1.5 m_j (u_j, 1);
//     each i-quad keeps its own accumulator, whose four blocks (one per
//     j-quad) are added once per pass over the unit's j chunk.
// Positions are taken relative to the centre cb of the i-block's box (not
// of the tile's), so the i operands stay in registers for the whole pass;
// the separation test bounds |u_i| + |u_j| by |c_w - cb| + e_w +
// |c_t - cb| + e_t, and the Gram error stays below ~2 kSepSym^2 eps as
// before.  The i-side rank-one term -u_i D_3 is linear in the sums and is
// applied once at the end of the pass.
// ---------------------------------------------------------------------------
template <int TJ>
__device__ __forceinline__ void sym_block_f64_q(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const double *__restrict__ soft, int stride, int i0, int iend, int jbeg,
    int jend, const double *__restrict__ tinfo,
    const double *__restrict__ iinfo, double *__restrict__ out,
    double *__restrict__ jacc, int chunk, bool first, double2 *tile,
    double *gT, double *qT, double *bT, double *jbuf, int ostride = -1,
    int obase = 0) {
  static_assert(TJ == kBlock, "one thread per tile particle in the j-side sum");
  constexpr int NQ = 16;  // i-quads of a wave
  // i-side results go to out[c * ostride + i - obase] (ostride < 0: stride)
  const size_t os = ostride < 0 ? (size_t)stride : (size_t)ostride;
  const int tid = threadIdx.x;
  const int l = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wbase = i0 + wv * 64;
  const int last = iend - 1;
  const int nw = max(0, min(64, iend - wbase));  // valid i of this wave
  const double *X = pos, *Y = pos + stride, *Z = pos + 2 * (size_t)stride;
  double *jb = jbuf + (size_t)wv * TJ * 3;  // this wave's [TJ][3] j sums

  const bool valid = wbase + l < iend;
  const int ip = min(wbase + l, last);
  const double xi = X[ip], yi = Y[ip], zi = Z[ip], hi = soft[ip];
  const int kk = l >> 4, cc = l & 3;
  const double *Pc = cc == 0 ? X : (cc == 1 ? Y : Z);
  double wb[7];
  {
    const double xs[1] = {xi}, ys[1] = {yi}, zs[1] = {zi}, hs[1] = {hi};
    const bool vs[1] = {valid};
    wave_box<1, double>(xs, ys, zs, hs, vs, wb);
  }
  // centre of the i-block's box (uniform over the workgroup)
  const double cb[3] = {0.5 * (iinfo[0] + iinfo[3]), 0.5 * (iinfo[1] + iinfo[4]),
                        0.5 * (iinfo[2] + iinfo[5])};
  const double ccb = cc == 0 ? cb[0] : (cc == 1 ? cb[1] : cb[2]);
  // |u_i| bound of this wave: |c_w - cb| + e_w
  const double aw =
      sqrt((0.5 * (wb[0] + wb[3]) - cb[0]) * (0.5 * (wb[0] + wb[3]) - cb[0]) +
           (0.5 * (wb[1] + wb[4]) - cb[1]) * (0.5 * (wb[1] + wb[4]) - cb[1]) +
           (0.5 * (wb[2] + wb[5]) - cb[2]) * (0.5 * (wb[2] + wb[5]) - cb[2])) +
      0.5 * sqrt((wb[3] - wb[0]) * (wb[3] - wb[0]) +
                 (wb[4] - wb[1]) * (wb[4] - wb[1]) +
                 (wb[5] - wb[2]) * (wb[5] - wb[2]));

  // i operands of the 16 i-quads, fixed for the pass: ag = (-2 u_i, q_i) at
  // lane ii + 4b + 16k (i = 4q + ii), bi = -1.5 m_i (u_i, 1) at lane
  // c + 4b + 16ii (i = 4q + ii; zero mass past iend)
  double ag[NQ], bi[NQ], acci[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int ia = min(wbase + 4 * q + cc, last);
    const double ux = X[ia] - cb[0], uy = Y[ia] - cb[1], uz = Z[ia] - cb[2];
    ag[q] = kk == 0 ? -2.0 * ux
                    : (kk == 1 ? -2.0 * uy
                               : (kk == 2 ? -2.0 * uz : fma(uz, uz, fma(uy, uy, ux * ux))));
    const int ib = wbase + 4 * q + kk;
    const int ibc = min(ib, last);
    const double m = ib < iend ? mass[ibc] : 0.0;
    bi[q] = -1.5 * m * (cc < 3 ? Pc[ibc] - ccb : 1.0);
    acci[q] = 0.0;
  }
  // near-block i-side sums (output layout: component cc of particle
  // 16 r + 4 ((l >> 2) & 3) + (l >> 4)), compensated
  double sum[4], cmp[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) sum[r] = cmp[r] = 0.0;
  // transpose within 4 x 4 blocks: lane n + 4b + 16m reads n' = m, m' = n
  const int tsrc = ((l >> 4) & 3) | (l & 12) | ((l & 3) << 4);
  // this lane's j-side slot in a group of 16 j: j = 16 G + 4 b + jj, b the
  // block, jj = l >> 4, component cc
  const int jslot = (l & 12) + kk;
  // Far i-side fold: add each quad's four j-quad blocks (row rotations),
  // keep quad q = 4r + b in the lanes of block b, form S = D_c - u_{i,c} D_3
  // and add it into the compensated running sums; the accumulators restart.
  // Done every kFoldTiles tiles and at the end of the pass, so that a plain
  // matrix-core accumulation never spans more than 512 j per block.
  constexpr int kFoldTiles = 8;
  auto fold_far = [&]() {
    double part[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double v = acci[q];
      v += row_ror<4>(v);
      v += row_ror<8>(v);
      if (((l >> 2) & 3) == (q & 3)) part[q >> 2] = v;
      acci[q] = 0.0;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int id = wbase + 16 * r + 4 * ((l >> 2) & 3) + (l >> 4);
      const double ui = cc < 3 ? Pc[min(id, last)] - ccb : 0.0;
      const double f = fma(-ui, quad_bcast3(part[r]), part[r]);
      two_sum_add(sum[r], cmp[r], cc < 3 ? f : 0.0);
    }
  };

  for (int jg = jbeg; jg < jend; jg += kFoldTiles * TJ) {
    const int jgend = min(jend, jg + kFoldTiles * TJ);
    for (int jt = jg; jt < jgend; jt += TJ) {
      const double *ti = tinfo + (size_t)((jt - jbeg) / TJ) * 8;
      // No barrier before staging: every wave finished reading the previous
      // tile before the barrier that precedes the previous tile's j-side sum,
      // and that sum reads only jbuf, which staging does not touch.
      {
        const int k = tid;
        const int j = min(jt + k, jend - 1);
        const double mj = (jt + k < jend) ? mass[j] : 0.0;
        const double xj = X[j], yj = Y[j], zj = Z[j];
        tile[3 * k] = double2{xj, yj};
        tile[3 * k + 1] = double2{zj, mj};
        tile[3 * k + 2] = double2{soft[j], 0.0};
        const double ux = xj - cb[0], uy = yj - cb[1], uz = zj - cb[2];
        const int G = k >> 4, jl = k & 15;
        gT[64 * G + jl] = ux;
        gT[64 * G + 16 + jl] = uy;
        gT[64 * G + 32 + jl] = uz;
        gT[64 * G + 48 + jl] = 1.0;
        qT[k] = fma(uz, uz, fma(uy, uy, ux * ux));
        const double mm = -1.5 * mj;
        const int bo = 64 * G + 16 * (jl & 3) + 4 * (jl >> 2);
        bT[bo] = mm * ux;
        bT[bo + 1] = mm * uy;
        bT[bo + 2] = mm * uz;
        bT[bo + 3] = mm;
      }
      const bool jown = jt + tid < jend;
      const size_t jl = (size_t)(jt + tid - jbeg);
      __syncthreads();

      const double gxv = fmax(0.0, fmax(ti[0] - wb[3], wb[0] - ti[3]));
      const double gyv = fmax(0.0, fmax(ti[1] - wb[4], wb[1] - ti[4]));
      const double gzv = fmax(0.0, fmax(ti[2] - wb[5], wb[2] - ti[5]));
      const double d2 = gxv * gxv + gyv * gyv + gzv * gzv;
      const double hs = ti[6] + wb[6];
      const bool far = d2 > fmax(hs * hs * (1.0 + 1e-6), 1e-30);
      const double bt =
          sqrt((0.5 * (ti[0] + ti[3]) - cb[0]) * (0.5 * (ti[0] + ti[3]) - cb[0]) +
               (0.5 * (ti[1] + ti[4]) - cb[1]) * (0.5 * (ti[1] + ti[4]) - cb[1]) +
               (0.5 * (ti[2] + ti[5]) - cb[2]) * (0.5 * (ti[2] + ti[5]) - cb[2])) +
          0.5 * sqrt((ti[3] - ti[0]) * (ti[3] - ti[0]) +
                     (ti[4] - ti[1]) * (ti[4] - ti[1]) +
                     (ti[5] - ti[2]) * (ti[5] - ti[2]));
      const bool sep = far && (aw + bt) <= kSepSym * sqrt(d2);
      const bool use_mfma = __builtin_amdgcn_readfirstlane((int)sep) != 0;

      if (nw == 0) {
        // a wave past the end of the chunk: nothing on either side
        for (int k = l; k < 3 * TJ; k += 64) jb[k] = 0.0;
      } else if (use_mfma) {
        // each group's operands are read one group ahead; the 16 groups of
        // the tile fully unrolled (measured 2.9% faster at 2^21 than a loop
        // of one group per iteration, 247 VGPRs and no spills)
        double bgn = gT[l], cjn = qT[l & 15], bjn = bT[l];
#pragma unroll
        for (int G = 0; G < TJ / 16; ++G) {
          const double bg = bgn, cj = cjn, bj = bjn;
          const int Gn = min(G + 1, TJ / 16 - 1);
          bgn = gT[64 * Gn + l];
          cjn = qT[16 * Gn + (l & 15)];
          bjn = bT[64 * Gn + l];
          double aj = 0.0;
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const double rr = mfma4(ag[q], bg, cj);
            const double y = __builtin_amdgcn_rsq(rr);
            const double y2 = y * y;
            const double t = fma(rr, y2, -5.0 / 3.0);
            const double w = (y * y2) * t;  // -(2/3) r^-3 (1 + 3/2 e)
            aj = mfma4(w, bi[q], aj);
            acci[q] = mfma4(__shfl(w, tsrc), bj, acci[q]);
          }
          // j-side of the group: D_c - u_{j,c} D_3 (D_3 from the quad's lane 3)
          const double uj = gT[64 * G + 16 * cc + (l & 12) + kk];
          const double f = fma(-uj, quad_bcast3(aj), aj);
          if (cc < 3) jb[3 * (16 * G + jslot) + cc] = f;
        }
      } else {
        // near block: each pair once (lane = i), i-side results moved into
        // the output layout
        double tx, ty, tz;
        near_block_f64<TJ>(tile, xi, yi, zi, hi, valid ? mass[ip] : 0.0,
                           __builtin_amdgcn_readfirstlane((int)far) != 0, l,
                           tx, ty, tz, jb);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int src = 16 * r + 4 * ((l >> 2) & 3) + (l >> 4);
          const double vx = __shfl(tx, src), vy = __shfl(ty, src), vz = __shfl(tz, src);
          two_sum_add(sum[r], cmp[r],
                      cc == 0 ? vx : (cc == 1 ? vy : (cc == 2 ? vz : 0.0)));
        }
      }
      // this thread's accumulator entry (j = jt + tid), read while the other
      // waves finish
      double acc6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      if (!first && jown) {
#pragma unroll
        for (int c = 0; c < 6; ++c) acc6[c] = jacc[(size_t)c * chunk + jl];
      }
      __syncthreads();

      // tile's j-side: the four waves' sums in order, into the accumulator
      if (jown) {
        const int k = tid;
        double f[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          f[c] = ((jbuf[3 * k + c] + jbuf[3 * (TJ + k) + c]) +
                  jbuf[3 * (2 * TJ + k) + c]) + jbuf[3 * (3 * TJ + k) + c];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (first) {
            acc6[c] = f[c];
            acc6[3 + c] = 0.0;
          } else {
            two_sum_add(acc6[c], acc6[3 + c], f[c]);
          }
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) jacc[(size_t)c * chunk + jl] = acc6[c];
      }
    }
    fold_far();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int id = wbase + 16 * r + 4 * ((l >> 2) & 3) + (l >> 4);
    if (cc < 3 && id < iend) out[(size_t)cc * os + id - obase] = sum[r] + cmp[r];
  }
}

// ---------------------------------------------------------------------------
// One block's share, mixed precision: pair arithmetic in FP32 on an FP32
// shadow [5][stride] (x, y, z, m, h); v_rsq_f32 (~2^-23) used as is.  Each
// tile's FP32 partial is added into an FP64 accumulator, or into a
// Kahan-compensated FP32 (sum, compensation) pair.  The inner loops use
// only two-operand VGPR forms of the FP32 ops, which gfx950 issues from two
// waves per cycle.  LDS tile: float4 (x, y, z, m) and float h.
// ---------------------------------------------------------------------------
template <int R, int TJ, bool KAHAN, bool CULL>
__device__ __forceinline__ void force_block_mixed(
    const float *__restrict__ shadow, int stride, int i0, int iend, int jbeg,
    int jend, const double *__restrict__ tinfo, double *__restrict__ out,
    int ostride, int obase, float4 *tpos, float *tsoft) {
  const int tid = threadIdx.x;
  const int ibase = i0 + (tid >> 6) * (64 * R) + (tid & 63);
  const float *X = shadow, *Y = shadow + stride, *Z = shadow + 2 * (size_t)stride;
  const float *M = shadow + 3 * (size_t)stride, *H = shadow + 4 * (size_t)stride;

  float xi[R], yi[R], zi[R], hi[R];
  bool valid[R];
  double ax[R], ay[R], az[R];                      // FP64 accumulation
  float sx[R], sy[R], sz[R], cx[R], cy[R], cz[R];  // Kahan accumulation
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = ibase + 64 * r;
    valid[r] = i < iend;
    xi[r] = valid[r] ? X[i] : 0.0f;
    yi[r] = valid[r] ? Y[i] : 0.0f;
    zi[r] = valid[r] ? Z[i] : 0.0f;
    hi[r] = valid[r] ? H[i] : 0.0f;
    ax[r] = ay[r] = az[r] = 0.0;
    sx[r] = sy[r] = sz[r] = cx[r] = cy[r] = cz[r] = 0.0f;
  }
  double wb[7];
  if (CULL) wave_box<R, float>(xi, yi, zi, hi, valid, wb);

  for (int jt = jbeg; jt < jend; jt += TJ) {
    __syncthreads();
    for (int k = tid; k < TJ; k += kBlock) {
      const int j = min(jt + k, jend - 1);
      const float mj = (jt + k < jend) ? M[j] : 0.0f;
      tpos[k] = float4{X[j], Y[j], Z[j], mj};
      tsoft[k] = H[j];
    }
    __syncthreads();

    bool far = false;
    if (CULL) far = tile_is_far(tinfo + (size_t)((jt - jbeg) / TJ) * 8, wb);

    float tx[R], ty[R], tz[R];
#pragma unroll
    for (int r = 0; r < R; ++r) tx[r] = ty[r] = tz[r] = 0.0f;

    if (far) {
#pragma unroll 2
      for (int k = 0; k < TJ; ++k) {
        const float4 p = tpos[k];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const float dx = p.x - xi[r], dy = p.y - yi[r], dz = p.z - zi[r];
          const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
          const float y = __builtin_amdgcn_rsqf(r2);
          const float w = (p.w * y) * (y * y);
          tx[r] = fmaf(w, dx, tx[r]);
          ty[r] = fmaf(w, dy, ty[r]);
          tz[r] = fmaf(w, dz, tz[r]);
        }
      }
    } else {
#pragma unroll 2
      for (int k = 0; k < TJ; ++k) {
        const float4 p = tpos[k];
        const float hj = tsoft[k];
        float dx[R], dy[R], dz[R], r2[R], w[R];
        bool sf[R];
        bool any = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          dx[r] = p.x - xi[r];
          dy[r] = p.y - yi[r];
          dz[r] = p.z - zi[r];
          r2[r] = fmaf(dz[r], dz[r], fmaf(dy[r], dy[r], dx[r] * dx[r]));
          const float h = hj + hi[r];
          sf[r] = r2[r] <= h * h;
          any |= sf[r];
          const float y = __builtin_amdgcn_rsqf(r2[r]);
          w[r] = (p.w * y) * (y * y);
        }
        if (any) {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            if (sf[r]) w[r] = soft_w32(r2[r], hj + hi[r], p.w);
          }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          tx[r] = fmaf(w[r], dx[r], tx[r]);
          ty[r] = fmaf(w[r], dy[r], ty[r]);
          tz[r] = fmaf(w[r], dz[r], tz[r]);
        }
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

#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = ibase + 64 * r;
    if (i < iend) {
      double *o = out + (i - obase);
      if (KAHAN) {
        o[0] = (double)sx[r] - (double)cx[r];
        o[(size_t)ostride] = (double)sy[r] - (double)cy[r];
        o[2 * (size_t)ostride] = (double)sz[r] - (double)cz[r];
      } else {
        o[0] = ax[r];
        o[(size_t)ostride] = ay[r];
        o[2 * (size_t)ostride] = az[r];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Single-simulation kernels: block (x, y) = (i-block, j-split); split y
// writes its partial to out + y * 3n.
// ---------------------------------------------------------------------------
template <int R, int TJ, bool E2, bool CULL>
__global__ __launch_bounds__(kBlock) void k_force_f64(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const double *__restrict__ soft, int n, int jchunk,
    const double *__restrict__ tinfo, double *__restrict__ out) {
  __shared__ double2 tile[3 * TJ];
  const int jbeg = blockIdx.y * jchunk;
  force_block_f64<R, TJ, E2, CULL>(
      pos, mass, soft, n, blockIdx.x * (kBlock * R), n, jbeg,
      min(n, jbeg + jchunk), CULL ? tinfo + (size_t)(jbeg / TJ) * 8 : nullptr,
      out + (size_t)blockIdx.y * 3 * (size_t)n, tile);
}

template <int TJ>
__global__ __launch_bounds__(kBlock) void k_force_f64_mfma(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const double *__restrict__ soft, int n, int jchunk,
    const double *__restrict__ tinfo, double *__restrict__ out) {
  __shared__ double2 tile[3 * TJ];
  __shared__ double gram[4 * TJ];
  __shared__ double bmat[4 * TJ];
  const int jbeg = blockIdx.y * jchunk;
  force_block_f64_mfma<TJ>(pos, mass, soft, n, blockIdx.x * kBlock, n,
                           jbeg, min(n, jbeg + jchunk),
                           tinfo + (size_t)(jbeg / TJ) * 8,
                           out + (size_t)blockIdx.y * 3 * (size_t)n, tile,
                           gram, bmat);
}

// Symmetric FP64 kernel: block u is unit (R, s).  Units u < Q(Q-1)/2 are the
// off-diagonal pairs in column order (u = s(s-1)/2 + R, R < s); the Q
// diagonal units (lighter) come last.  iplane is [Q][3][n]; unit u < Q(Q-1)/2
// owns jacc + u * 6C.
template <int TJ>
__global__ __launch_bounds__(kBlock, 3) void k_force_f64_sym(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const double *__restrict__ soft, int n, int chunk, int nchunks,
    const double *__restrict__ tinfo, double *__restrict__ iplane,
    double *__restrict__ jacc) {
  __shared__ double2 tile[3 * TJ];
  __shared__ double gram[4 * TJ];
  __shared__ double bmat[4 * TJ];
  __shared__ double jbuf[4 * TJ * 3];
  const int nsym = nchunks * (nchunks - 1) / 2;
  const int u = blockIdx.x;
  int R, s;
  if (u < nsym) {
    s = (int)((1.0 + sqrt(1.0 + 8.0 * (double)u)) * 0.5);
    while (s * (s - 1) / 2 > u) --s;
    while ((s + 1) * s / 2 <= u) ++s;
    R = u - s * (s - 1) / 2;
  } else {
    R = s = u - nsym;
  }
  const int ibeg = R * chunk, iend = min(n, ibeg + chunk);
  const int jbeg = s * chunk, jend = min(n, jbeg + chunk);
  double *out = iplane + (size_t)s * 3 * (size_t)n;
  const double *ti = tinfo + (size_t)(jbeg / TJ) * 8;
  if (R == s) {
    for (int i0 = ibeg; i0 < iend; i0 += kBlock) {
      force_block_f64_mfma<TJ>(pos, mass, soft, n, i0, iend, jbeg, jend, ti,
                               out, tile, gram, bmat);
    }
    return;
  }
  double *ja = jacc + (size_t)u * 6 * (size_t)chunk;
  for (int i0 = ibeg; i0 < iend; i0 += kBlock) {
    sym_block_f64<TJ>(pos, mass, soft, n, i0, iend, jbeg, jend, ti, out, ja,
                      chunk, i0 == ibeg, tile, gram, bmat, jbuf);
  }
}

// Symmetric FP64 kernel, j-quad layout of the far blocks (variant 30):
// units, planes and accumulators as k_force_f64_sym.  Its far loop holds
// the i operands of 16 i-quads and their accumulators in registers, so the
// kernel runs two workgroups per CU.
template <int TJ>
__global__ __launch_bounds__(kBlock, 2) void k_force_f64_symq(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const double *__restrict__ soft, int n, int chunk, int nchunks,
    const double *__restrict__ tinfo, double *__restrict__ iplane,
    double *__restrict__ jacc) {
  __shared__ double2 tile[3 * TJ];
  __shared__ double gram[4 * TJ];
  __shared__ double bmat[4 * TJ];
  __shared__ double qj[TJ];
  __shared__ double jbuf[4 * TJ * 3];
  const int nsym = nchunks * (nchunks - 1) / 2;
  const int u = blockIdx.x;
  int R, s;
  if (u < nsym) {
    s = (int)((1.0 + sqrt(1.0 + 8.0 * (double)u)) * 0.5);
    while (s * (s - 1) / 2 > u) --s;
    while ((s + 1) * s / 2 <= u) ++s;
    R = u - s * (s - 1) / 2;
  } else {
    R = s = u - nsym;
  }
  const int ibeg = R * chunk, iend = min(n, ibeg + chunk);
  const int jbeg = s * chunk, jend = min(n, jbeg + chunk);
  double *out = iplane + (size_t)s * 3 * (size_t)n;
  const double *ti = tinfo + (size_t)(jbeg / TJ) * 8;
  if (R == s) {
    for (int i0 = ibeg; i0 < iend; i0 += kBlock) {
      force_block_f64_mfma<TJ>(pos, mass, soft, n, i0, iend, jbeg, jend, ti,
                               out, tile, gram, bmat);
    }
    return;
  }
  double *ja = jacc + (size_t)u * 6 * (size_t)chunk;
  for (int i0 = ibeg; i0 < iend; i0 += kBlock) {
    sym_block_f64_q<TJ>(pos, mass, soft, n, i0, iend, jbeg, jend, ti,
                        tinfo + (size_t)(i0 / TJ) * 8, out, ja, chunk,
                        i0 == ibeg, tile, gram, qj, bmat, jbuf);
  }
}

// acc[d][perm[p]] for p in chunk k: planes k .. Q-1 of iplane, then the
// (value, error) accumulators of units (R, k), R < k, in that order,
// compensated
__global__ __launch_bounds__(kBlock) void k_reduce_sym(
    const double *__restrict__ iplane, const double *__restrict__ jacc, int n,
    int chunk, int nchunks, const int *__restrict__ perm,
    double *__restrict__ acc) {
  const size_t total = 3 * (size_t)n;
  const size_t q = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= total) return;
  const int d = (int)(q / n), p = (int)(q - (size_t)d * n);
  const int k = p / chunk, loc = p - k * chunk;
  double s = 0.0, c = 0.0;
  for (int t = k; t < nchunks; ++t) {
    two_sum_add(s, c, iplane[(size_t)t * total + (size_t)d * n + p]);
  }
  const size_t base = (size_t)k * (k - 1) / 2;
  for (int R = 0; R < k; ++R) {
    const double *ja = jacc + (base + R) * 6 * (size_t)chunk;
    two_sum_add(s, c, ja[(size_t)d * chunk + loc]);
    c += ja[(size_t)(3 + d) * chunk + loc];
  }
  acc[(size_t)d * n + perm[p]] = s + c;
}

template <int R, int TJ, bool KAHAN, bool CULL>
__global__ __launch_bounds__(kBlock) void k_force_mixed(
    const float *__restrict__ shadow, int n, int jchunk,
    const double *__restrict__ tinfo, double *__restrict__ out) {
  __shared__ float4 tpos[TJ];
  __shared__ float tsoft[TJ];
  const int jbeg = blockIdx.y * jchunk;
  force_block_mixed<R, TJ, KAHAN, CULL>(
      shadow, n, blockIdx.x * (kBlock * R), n, jbeg, min(n, jbeg + jchunk),
      CULL ? tinfo + (size_t)(jbeg / TJ) * 8 : nullptr,
      out + (size_t)blockIdx.y * 3 * (size_t)n, n, 0, tpos, tsoft);
}

// ---------------------------------------------------------------------------
// Symmetric mixed-precision evaluation (Newton's third law, Sec. 2.2 Eq. 8:
// the pair term is antisymmetric), on the units and output layout of the
// FP64 symmetric kernel.  In an off-diagonal unit (R, s) each wave takes
// 64 R particles of chunk R (R per lane) against every 256-particle tile of
// chunk s, the tile in four parts of 64.  In step t of a part, lane l pairs
// its particles with particle (l + t) mod 64 of the part, read from LDS: over
// 64 steps every lane meets every j of the part once, and within a step no
// two lanes share a j.  One FP32 weight w' = F(r, h)/r per pair serves both
// sides: the i-side sums m_j w' d in registers, and the lane's R terms
// m_i w' d of the step are added into the wave's own FP32 j-sums in LDS by
// plain read-modify-write (one lane per address and step, so the order of
// additions is fixed; LDS float atomics measured 7x slower overall).  Per tile,
// the i-side partial is added into FP64 (or a Kahan FP32 pair), and the four
// waves' j-sums are added in wave order into the unit's (value, error)
// accumulator: FP64 TwoSum, or a Kahan FP32 step kept as (sum, -comp).  The
// cross-lane traffic goes through the LDS pipe, so the vector ALU issues only
// the pair arithmetic: one v_rsq_f32 per unordered pair instead of two.
// ---------------------------------------------------------------------------
// Orders one rotation step's LDS j-sum stores before the next step's loads.
// Step t + 1 of lane l - 1 reads the word that lane l wrote in step t; from
// one thread's view the two addresses differ, so without a fence the
// compiler could move the load above the store.  The hardware needs no wait:
// a wave's LDS instructions execute in issue order.  The empty asm with a
// memory clobber is a compiler-only barrier (it emits no instruction).
__device__ __forceinline__ void lds_step_fence() { asm volatile("" ::: "memory"); }

template <int R, bool KAHAN, bool REFINE = false>
__device__ __forceinline__ void sym_block_mixed(
    const float *__restrict__ shadow, int stride, int i0, int iend, int jbeg,
    int jend, const double *__restrict__ tinfo, double *__restrict__ out,
    int ostride, int obase, double *__restrict__ jacc, int chunk, bool first,
    float4 *tpos, float *tsoft, float *jl) {
  constexpr int TJ = 256;
  static_assert(TJ == kBlock, "one thread per tile particle");
  const int tid = threadIdx.x;
  const int l = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wbase = i0 + wv * 64 * R;
  const int last = iend - 1;
  const float *X = shadow, *Y = shadow + stride, *Z = shadow + 2 * (size_t)stride;
  const float *M = shadow + 3 * (size_t)stride, *H = shadow + 4 * (size_t)stride;
  float *jw = jl + (size_t)wv * 3 * TJ;  // this wave's j-sums [3][TJ]

  // lanes past iend take the position of the last particle (inside the wave
  // box, so far tiles keep r > 0) and zero mass
  float xi[R], yi[R], zi[R], mi[R], hi[R];
  bool valid[R];
  double ax[R], ay[R], az[R];                      // FP64 accumulation
  float sx[R], sy[R], sz[R], cx[R], cy[R], cz[R];  // Kahan accumulation
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = wbase + 64 * r + l;
    valid[r] = i < iend;
    const int ic = min(i, last);
    xi[r] = X[ic];
    yi[r] = Y[ic];
    zi[r] = Z[ic];
    hi[r] = H[ic];
    mi[r] = valid[r] ? M[ic] : 0.0f;
    ax[r] = ay[r] = az[r] = 0.0;
    sx[r] = sy[r] = sz[r] = cx[r] = cy[r] = cz[r] = 0.0f;
  }
  const bool live = wbase < iend;  // wave-uniform: any valid i
  double wb[7];
  wave_box<R, float>(xi, yi, zi, hi, valid, wb);

  for (int jt = jbeg; jt < jend; jt += TJ) {
    // No barrier before staging: every wave finished reading the previous
    // tile before the barrier that precedes the previous tile's j-side sum,
    // and that sum reads only jl.  A wave clears its own j-sums after the
    // staging barrier, when no thread is still reading them.
    {
      const int j = min(jt + tid, jend - 1);
      tpos[tid] = float4{X[j], Y[j], Z[j], (jt + tid < jend) ? M[j] : 0.0f};
      tsoft[tid] = H[j];
    }
    __syncthreads();
    for (int k = l; k < 3 * TJ; k += 64) jw[k] = 0.0f;
    lds_step_fence();  // the zeros before the rotation's first loads

    const bool far = tile_is_far(tinfo + (size_t)((jt - jbeg) / TJ) * 8, wb);
    float tx[R], ty[R], tz[R];
#pragma unroll
    for (int r = 0; r < R; ++r) tx[r] = ty[r] = tz[r] = 0.0f;
    if (live && far) {
      // two parts of 64 j per step (j and j + 64 of the same rotation):
      // one address computation and one loop step serve 2 R pairs
      static_assert(TJ % 128 == 0, "the far loop takes parts in pairs");
      for (int q = 0; q < TJ; q += 128) {
#pragma unroll 2
        for (int t = 0; t < 64; ++t) {
          const int jj = q + ((l + t) & 63);
          const float4 pa = tpos[jj], pb = tpos[jj + 64];
          // these j's running sums, read before the pair arithmetic that
          // hides their latency (plain read-modify-write: one lane per
          // address within a step; the words lane l writes here are read by
          // lane l - 1 in the next step, ordered by lds_step_fence below)
          float ax_ = jw[jj], ay_ = jw[TJ + jj], az_ = jw[2 * TJ + jj];
          float bx_ = jw[jj + 64], by_ = jw[TJ + jj + 64], bz_ = jw[2 * TJ + jj + 64];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const float4 p = h ? pb : pa;
            float jx = h ? bx_ : ax_, jy = h ? by_ : ay_, jz = h ? bz_ : az_;
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const float dx = p.x - xi[r], dy = p.y - yi[r], dz = p.z - zi[r];
              const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
              const float y = __builtin_amdgcn_rsqf(r2);
              const float y2 = y * y;
              float y3 = y2 * y;
              if (REFINE) {
                // one Newton step on r^-3: with e = 1 - r^2 y^2,
                // r^-3 = y^3 (1 + 3/2 e) + O(e^2)
                const float e = fmaf(-r2, y2, 1.0f);
                y3 = fmaf(1.5f * e, y3, y3);
              }
              const float wi = p.w * y3, wj = mi[r] * y3;
              tx[r] = fmaf(wi, dx, tx[r]);
              ty[r] = fmaf(wi, dy, ty[r]);
              tz[r] = fmaf(wi, dz, tz[r]);
              jx = fmaf(wj, dx, jx);
              jy = fmaf(wj, dy, jy);
              jz = fmaf(wj, dz, jz);
            }
            if (h) {
              bx_ = jx; by_ = jy; bz_ = jz;
            } else {
              ax_ = jx; ay_ = jy; az_ = jz;
            }
          }
          jw[jj] = ax_;
          jw[TJ + jj] = ay_;
          jw[2 * TJ + jj] = az_;
          jw[jj + 64] = bx_;
          jw[TJ + jj + 64] = by_;
          jw[2 * TJ + jj + 64] = bz_;
          lds_step_fence();
        }
      }
    } else if (live) {
      // one part of 64 j per step; SOFT: softening tested per pair
      // (coincident pairs take the softened branch, which gives 0)
      auto part = [&](int q, auto soft_tag) {
        constexpr bool SOFT = decltype(soft_tag)::value;
#pragma unroll 2
        for (int t = 0; t < 64; ++t) {
          const int jj = q + ((l + t) & 63);
          const float4 p = tpos[jj];
          const float hj = tsoft[jj];
          float jx = jw[jj], jy = jw[TJ + jj], jz = jw[2 * TJ + jj];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const float dx = p.x - xi[r], dy = p.y - yi[r], dz = p.z - zi[r];
            const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            const float y = __builtin_amdgcn_rsqf(r2);
            const float y2 = y * y;
            float w = y2 * y;
            if (REFINE) w = fmaf(1.5f * fmaf(-r2, y2, 1.0f), w, w);
            if (SOFT) {
              const float h = hj + hi[r];
              if (r2 <= h * h) w = soft_w32(r2, h, 1.0f);
            }
            const float wi = p.w * w, wj = mi[r] * w;
            tx[r] = fmaf(wi, dx, tx[r]);
            ty[r] = fmaf(wi, dy, ty[r]);
            tz[r] = fmaf(wi, dz, tz[r]);
            jx = fmaf(wj, dx, jx);
            jy = fmaf(wj, dy, jy);
            jz = fmaf(wj, dz, jz);
          }
          jw[jj] = jx;
          jw[TJ + jj] = jy;
          jw[2 * TJ + jj] = jz;
          lds_step_fence();
        }
      };
      for (int q = 0; q < TJ; q += 64) {
        // the tile failed the box test; a part whose every j lies beyond
        // the largest combined softening from the wave's box skips the
        // per-pair test (same margin as the tile test)
        const float4 pj = tpos[q + l];
        const double gx = fmax(0.0, fmax((double)pj.x - wb[3], wb[0] - (double)pj.x));
        const double gy = fmax(0.0, fmax((double)pj.y - wb[4], wb[1] - (double)pj.y));
        const double gz = fmax(0.0, fmax((double)pj.z - wb[5], wb[2] - (double)pj.z));
        const double hs = (double)tsoft[q + l] + wb[6];
        const bool jfar = gx * gx + gy * gy + gz * gz > fmax(hs * hs * (1.0 + 1e-6), 1e-30);
        if (__builtin_amdgcn_ballot_w64(!jfar) == 0) {
          part(q, std::false_type{});
        } else {
          part(q, std::true_type{});
        }
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
    // this thread's accumulator entry (j = jt + tid), read while the other
    // waves finish
    const bool jown = jt + tid < jend;
    const size_t jo = (size_t)(jt + tid - jbeg);
    double acc6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (!first && jown) {
#pragma unroll
      for (int c = 0; c < 6; ++c) acc6[c] = jacc[(size_t)c * chunk + jo];
    }
    __syncthreads();
    if (jown) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        // the pull of i on j is m_i w' (x_i - x_j) = -(m_i w' d)
        if (KAHAN) {
          // the waves' sums added in FP32, then a Kahan FP32 step; the
          // accumulator keeps (sum, -compensation), so that value + error
          // is the compensated total
          const float f = -(((jl[c * TJ + tid] + jl[(3 + c) * TJ + tid]) +
                             jl[(6 + c) * TJ + tid]) +
                            jl[(9 + c) * TJ + tid]);
          if (first) {
            acc6[c] = (double)f;
            acc6[3 + c] = 0.0;
          } else {
            const float s0 = (float)acc6[c], c0 = -(float)acc6[3 + c];
            const float yv = f - c0, t = s0 + yv;
            acc6[3 + c] = -(double)((t - s0) - yv);
            acc6[c] = (double)t;
          }
        } else {
          // the waves' FP32 sums (64 R terms each) are added in FP64
          const double f = -((((double)jl[c * TJ + tid] +
                               (double)jl[(3 + c) * TJ + tid]) +
                              (double)jl[(6 + c) * TJ + tid]) +
                             (double)jl[(9 + c) * TJ + tid]);
          if (first) {
            acc6[c] = f;
            acc6[3 + c] = 0.0;
          } else {
            two_sum_add(acc6[c], acc6[3 + c], f);
          }
        }
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) jacc[(size_t)c * chunk + jo] = acc6[c];
    }
  }

#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = wbase + 64 * r + l;
    if (valid[r]) {
      double *o = out + (i - obase);
      if (KAHAN) {
        o[0] = (double)sx[r] - (double)cx[r];
        o[(size_t)ostride] = (double)sy[r] - (double)cy[r];
        o[2 * (size_t)ostride] = (double)sz[r] - (double)cz[r];
      } else {
        o[0] = ax[r];
        o[(size_t)ostride] = ay[r];
        o[2 * (size_t)ostride] = az[r];
      }
    }
  }
}

// Symmetric mixed kernel: the unit grid of k_force_f64_sym; diagonal units
// run the one-sided mixed block (same accumulation) into plane s.
template <int R, bool KAHAN, bool REFINE>
__global__ __launch_bounds__(kBlock, 4) void k_force_mixed_sym(
    const float *__restrict__ shadow, int n, int chunk, int nchunks,
    const double *__restrict__ tinfo, double *__restrict__ iplane,
    double *__restrict__ jacc) {
  __shared__ float4 tpos[256];
  __shared__ float tsoft[256];
  __shared__ float jl[4 * 3 * 256];
  const int nsym = nchunks * (nchunks - 1) / 2;
  const int u = blockIdx.x;
  int cr, cs;
  if (u < nsym) {
    cs = (int)((1.0 + sqrt(1.0 + 8.0 * (double)u)) * 0.5);
    while (cs * (cs - 1) / 2 > u) --cs;
    while ((cs + 1) * cs / 2 <= u) ++cs;
    cr = u - cs * (cs - 1) / 2;
  } else {
    cr = cs = u - nsym;
  }
  const int ibeg = cr * chunk, iend = min(n, ibeg + chunk);
  const int jbeg = cs * chunk, jend = min(n, jbeg + chunk);
  double *out = iplane + (size_t)cs * 3 * (size_t)n;
  const double *ti = tinfo + (size_t)(jbeg / 256) * 8;
  if (cr == cs) {
    for (int i0 = ibeg; i0 < iend; i0 += kBlock * R) {
      force_block_mixed<R, 256, KAHAN, true>(shadow, n, i0, iend, jbeg, jend,
                                             ti, out, n, 0, tpos, tsoft);
    }
    return;
  }
  double *ja = jacc + (size_t)u * 6 * (size_t)chunk;
  for (int i0 = ibeg; i0 < iend; i0 += kBlock * R) {
    sym_block_mixed<R, KAHAN, REFINE>(shadow, n, i0, iend, jbeg, jend, ti, out, n, 0,
                              ja, chunk, i0 == ibeg, tpos, tsoft, jl);
  }
}

// ---------------------------------------------------------------------------
// Ensemble kernels: a persistent grid pulls work items from an atomic
// counter until none are left (every block then returns, so the grid always
// drains).  Item k is the block of particles [it.x, it.y) of one member
// against a tile-aligned part [it.z, it.w) of that member's range (all of
// it, or one of its j-chunks); tbase[k] is the index of that part's first
// tile in tinfo, and islot[k] (if given) the output plane the item writes,
// one plane per j-chunk, reduced afterwards in fixed order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int next_item(int *counter, int *slot) {
  __syncthreads();  // everyone has read the previous item
  if (threadIdx.x == 0) *slot = atomicAdd(counter, 1);
  __syncthreads();
  return *slot;
}

template <int R, int TJ, bool E2>
__global__ __launch_bounds__(kBlock) void k_batch_force_f64(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const double *__restrict__ soft, int stride, const int4 *__restrict__ items,
    const int *__restrict__ tbase, const int *__restrict__ islot, int nitems,
    const double *__restrict__ tinfo, double *__restrict__ out, int *counter) {
  __shared__ double2 tile[3 * TJ];
  __shared__ int slot;
  for (int it = next_item(counter, &slot); it < nitems;
       it = next_item(counter, &slot)) {
    const int4 w = items[it];
    double *o = islot ? out + (size_t)islot[it] * 3 * (size_t)stride : out;
    force_block_f64<R, TJ, E2, true>(pos, mass, soft, stride, w.x, w.y, w.z,
                                     w.w, tinfo + (size_t)tbase[it] * 8, o,
                                     tile);
  }
}

template <int TJ>
__global__ __launch_bounds__(kBlock) void k_batch_force_f64_mfma(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const double *__restrict__ soft, int stride, const int4 *__restrict__ items,
    const int *__restrict__ tbase, const int *__restrict__ islot, int nitems,
    const double *__restrict__ tinfo, double *__restrict__ out, int *counter) {
  __shared__ double2 tile[3 * TJ];
  __shared__ double gram[4 * TJ];
  __shared__ double bmat[4 * TJ];
  __shared__ int slot;
  for (int it = next_item(counter, &slot); it < nitems;
       it = next_item(counter, &slot)) {
    const int4 w = items[it];
    double *o = islot ? out + (size_t)islot[it] * 3 * (size_t)stride : out;
    force_block_f64_mfma<TJ>(pos, mass, soft, stride, w.x, w.y, w.z, w.w,
                             tinfo + (size_t)tbase[it] * 8, o, tile, gram,
                             bmat);
  }
}

template <int R, int TJ, bool KAHAN>
__global__ __launch_bounds__(kBlock) void k_batch_force_mixed(
    const float *__restrict__ shadow, int stride, const int4 *__restrict__ items,
    const int *__restrict__ tbase, const int *__restrict__ islot, int nitems,
    const double *__restrict__ tinfo, double *__restrict__ out, int *counter) {
  __shared__ float4 tpos[TJ];
  __shared__ float tsoft[TJ];
  __shared__ int slot;
  for (int it = next_item(counter, &slot); it < nitems;
       it = next_item(counter, &slot)) {
    const int4 w = items[it];
    double *o = islot ? out + (size_t)islot[it] * 3 * (size_t)stride : out;
    force_block_mixed<R, TJ, KAHAN, true>(shadow, stride, w.x, w.y, w.z, w.w,
                                          tinfo + (size_t)tbase[it] * 8, o,
                                          stride, 0, tpos, tsoft);
  }
}

// Symmetric ensemble kernel, mixed precision: block u is unit u of the
// layout, a chunk pair (R, s), R <= s, of one member: items[u] = (ibeg,
// iend, jbeg, jend) in the sorted arena, tbase[u] the tile of jbeg, and
// islot[u] its slot of usum, [9][chunk] doubles: the i-side sums of chunk
// R's particles, then the (value, error) j-side accumulator of chunk s's.
// A diagonal unit (ibeg == jbeg) sums its chunk one-sided into the i-side.
// Units are of nearly equal cost, so the grid is one workgroup per unit.
template <int R, bool KAHAN>
__global__ __launch_bounds__(kBlock, 4) void k_batch_force_mixed_sym(
    const float *__restrict__ shadow, int stride, const int4 *__restrict__ units,
    const int *__restrict__ tbase, const int *__restrict__ uslot, int nunits,
    const double *__restrict__ tinfo, double *__restrict__ usum, int chunk) {
  __shared__ float4 tpos[256];
  __shared__ float tsoft[256];
  __shared__ float jl[4 * 3 * 256];
  const int u = blockIdx.x;
  if (u >= nunits) return;
  const int4 w = units[u];
  const double *ti = tinfo + (size_t)tbase[u] * 8;
  double *slot = usum + (size_t)uslot[u] * 9 * (size_t)chunk;
  if (w.x == w.z) {
    for (int i0 = w.x; i0 < w.y; i0 += kBlock * R) {
      force_block_mixed<R, 256, KAHAN, true>(shadow, stride, i0, w.y, w.z, w.w,
                                             ti, slot, chunk, w.x, tpos, tsoft);
    }
    return;
  }
  for (int i0 = w.x; i0 < w.y; i0 += kBlock * R) {
    sym_block_mixed<R, KAHAN>(shadow, stride, i0, w.y, w.z, w.w, ti, slot,
                              chunk, w.x, slot + 3 * (size_t)chunk, chunk,
                              i0 == w.x, tpos, tsoft, jl);
  }
}

// Symmetric ensemble kernel, FP64: the units and slots of
// k_batch_force_mixed_sym, each off-diagonal unit run by the j-quad block of
// k_force_f64_symq, each diagonal unit by the one-sided matrix-core block.
// Tiles of 256 run from each member's start, so the tile of an i-block is
// that of the unit's j-range shifted by (ibeg - jbeg) / 256.
template <int TJ>
__global__ __launch_bounds__(kBlock, 2) void k_batch_force_f64_sym(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const double *__restrict__ soft, int stride, const int4 *__restrict__ units,
    const int *__restrict__ tbase, const int *__restrict__ uslot, int nunits,
    const double *__restrict__ tinfo, double *__restrict__ usum, int chunk) {
  __shared__ double2 tile[3 * TJ];
  __shared__ double gram[4 * TJ];
  __shared__ double bmat[4 * TJ];
  __shared__ double qj[TJ];
  __shared__ double jbuf[4 * TJ * 3];
  const int u = blockIdx.x;
  if (u >= nunits) return;
  const int4 w = units[u];
  const double *ti = tinfo + (size_t)tbase[u] * 8;
  double *slot = usum + (size_t)uslot[u] * 9 * (size_t)chunk;
  if (w.x == w.z) {
    for (int i0 = w.x; i0 < w.y; i0 += kBlock) {
      force_block_f64_mfma<TJ>(pos, mass, soft, stride, i0, w.y, w.z, w.w, ti,
                               slot, tile, gram, bmat, chunk, w.x);
    }
    return;
  }
  const double *ib = ti + (ptrdiff_t)((w.x - w.z) / TJ) * 8;
  for (int i0 = w.x; i0 < w.y; i0 += kBlock) {
    sym_block_f64_q<TJ>(pos, mass, soft, stride, i0, w.y, w.z, w.w, ti,
                        ib + (size_t)((i0 - w.x) / TJ) * 8, slot,
                        slot + 3 * (size_t)chunk, chunk, i0 == w.x, tile, gram,
                        qj, bmat, jbuf, chunk, w.x);
  }
}

// acc[d][p] for arena slot p of member a = mid[p], in chunk k of that
// member: the i-side sums of units (k, t), t = k .. Q_a - 1, then the j-side
// (value, error) accumulators of units (R, k), R < k, compensated, in that
// order.  Unit (R, s) of member a sits in slot ubase[a] + s (s + 1) / 2 + R.
__global__ __launch_bounds__(kBlock) void k_batch_reduce_sym(
    const double *__restrict__ usum, int n, const int *__restrict__ mid,
    const int *__restrict__ moff, const int *__restrict__ mq,
    const int *__restrict__ mubase, int chunk, double *__restrict__ acc) {
  const size_t total = 3 * (size_t)n;
  const size_t q = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= total) return;
  const int d = (int)(q / n), p = (int)(q - (size_t)d * n);
  const int a = mid[p];
  const int loc0 = p - moff[a];
  const int k = loc0 / chunk, loc = loc0 - k * chunk;
  const int nq = mq[a];
  const size_t ub = (size_t)mubase[a], S = 9 * (size_t)chunk;
  double s = 0.0, c = 0.0;
  for (int t = k; t < nq; ++t) {
    two_sum_add(s, c, usum[(ub + (size_t)t * (t + 1) / 2 + k) * S +
                           (size_t)d * chunk + loc]);
  }
  const size_t row = ub + (size_t)k * (k + 1) / 2;
  for (int r = 0; r < k; ++r) {
    const double *js = usum + (row + r) * S + 3 * (size_t)chunk;
    two_sum_add(s, c, js[(size_t)d * chunk + loc]);
    c += js[(size_t)(3 + d) * chunk + loc];
  }
  acc[q] = s + c;
}

// ---------------------------------------------------------------------------
// launchers and the variant table
// ---------------------------------------------------------------------------
inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

template <int R, int TJ, bool E2, bool CULL>
hipError_t launch_f64(const ForceLaunch &L, hipStream_t s) {
  dim3 grid(ceil_div(L.n, (long long)kBlock * R), L.jsplit);
  hipLaunchKernelGGL((k_force_f64<R, TJ, E2, CULL>), grid, dim3(kBlock), 0, s,
                     L.pos, L.mass, L.soft, L.n, L.jchunk, L.tinfo, L.out);
  return hipGetLastError();
}

template <int TJ>
hipError_t launch_f64_mfma(const ForceLaunch &L, hipStream_t s) {
  dim3 grid(ceil_div(L.n, (long long)kBlock), L.jsplit);
  hipLaunchKernelGGL((k_force_f64_mfma<TJ>), grid, dim3(kBlock), 0, s, L.pos,
                     L.mass, L.soft, L.n, L.jchunk, L.tinfo, L.out);
  return hipGetLastError();
}

// Units of the symmetric kernel: Q chunks of jchunk particles (Q = jsplit)
// must cover [0, n) with every chunk non-empty; checked here, before the
// launch, since the kernel indexes iplane, jacc and tinfo by chunk.
template <int TJ, bool QUAD>
hipError_t launch_f64_sym(const ForceLaunch &L, hipStream_t s) {
  const int q = L.jsplit;
  if (L.jchunk <= 0 || L.jchunk % TJ != 0 || q < 1 || q > 4096 ||
      (long long)(q - 1) * L.jchunk >= L.n ||
      (long long)q * L.jchunk < L.n || (q > 1 && !L.jacc) || !L.tinfo) {
    return hipErrorInvalidValue;
  }
  const int units = q * (q + 1) / 2;
  if (QUAD) {
    hipLaunchKernelGGL((k_force_f64_symq<TJ>), dim3(units), dim3(kBlock), 0, s,
                       L.pos, L.mass, L.soft, L.n, L.jchunk, q, L.tinfo, L.out,
                       L.jacc);
  } else {
    hipLaunchKernelGGL((k_force_f64_sym<TJ>), dim3(units), dim3(kBlock), 0, s,
                       L.pos, L.mass, L.soft, L.n, L.jchunk, q, L.tinfo, L.out,
                       L.jacc);
  }
  return hipGetLastError();
}

// Symmetric mixed kernel: the chunk layout is checked as for the FP64
// symmetric kernel.
template <int R, bool REFINE>
hipError_t launch_mixed_sym(const ForceLaunch &L, hipStream_t s) {
  const int q = L.jsplit;
  if (!L.shadow || L.jchunk <= 0 || L.jchunk % 256 != 0 || q < 1 ||
      q > 4096 || (long long)(q - 1) * L.jchunk >= L.n ||
      (long long)q * L.jchunk < L.n || (q > 1 && !L.jacc) || !L.tinfo) {
    return hipErrorInvalidValue;
  }
  const int units = q * (q + 1) / 2;
  if (L.kahan) {
    hipLaunchKernelGGL((k_force_mixed_sym<R, true, REFINE>), dim3(units), dim3(kBlock),
                       0, s, L.shadow, L.n, L.jchunk, q, L.tinfo, L.out, L.jacc);
  } else {
    hipLaunchKernelGGL((k_force_mixed_sym<R, false, REFINE>), dim3(units),
                       dim3(kBlock), 0, s, L.shadow, L.n, L.jchunk, q, L.tinfo,
                       L.out, L.jacc);
  }
  return hipGetLastError();
}

template <int R, int TJ, bool CULL>
hipError_t launch_mixed(const ForceLaunch &L, hipStream_t s) {
  dim3 grid(ceil_div(L.n, (long long)kBlock * R), L.jsplit);
  if (L.kahan) {
    hipLaunchKernelGGL((k_force_mixed<R, TJ, true, CULL>), grid, dim3(kBlock),
                       0, s, L.shadow, L.n, L.jchunk, L.tinfo, L.out);
  } else {
    hipLaunchKernelGGL((k_force_mixed<R, TJ, false, CULL>), grid,
                       dim3(kBlock), 0, s, L.shadow, L.n, L.jchunk, L.tinfo,
                       L.out);
  }
  return hipGetLastError();
}

// Persistent ensemble launch: grid = CUs x resident blocks per CU.
template <typename K>
int persistent_grid(K kernel) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
          hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, 0) !=
          hipSuccess) {
    (void)hipGetLastError();
    return 2048;
  }
  return std::max(1, cus * std::max(1, per));
}

template <int R, int TJ, bool E2>
hipError_t launch_batch_f64(const BatchLaunch &L, hipStream_t s) {
  static const int grid = persistent_grid(k_batch_force_f64<R, TJ, E2>);
  hipLaunchKernelGGL((k_batch_force_f64<R, TJ, E2>), dim3(grid), dim3(kBlock),
                     0, s, L.pos, L.mass, L.soft, L.stride, L.items, L.tbase, L.islot,
                     L.nitems, L.tinfo, L.out, L.counter);
  return hipGetLastError();
}

template <int TJ>
hipError_t launch_batch_f64_mfma(const BatchLaunch &L, hipStream_t s) {
  static const int grid = persistent_grid(k_batch_force_f64_mfma<TJ>);
  hipLaunchKernelGGL((k_batch_force_f64_mfma<TJ>), dim3(grid), dim3(kBlock), 0,
                     s, L.pos, L.mass, L.soft, L.stride, L.items, L.tbase, L.islot,
                     L.nitems, L.tinfo, L.out, L.counter);
  return hipGetLastError();
}

hipError_t launch_batch_f64_sym(const BatchLaunch &L, hipStream_t s) {
  if (!L.usum || L.chunk <= 0 || L.chunk % 256 != 0 || L.nitems < 0) {
    return hipErrorInvalidValue;
  }
  if (L.nitems == 0) return hipSuccess;
  hipLaunchKernelGGL((k_batch_force_f64_sym<256>), dim3(L.nitems), dim3(kBlock),
                     0, s, L.pos, L.mass, L.soft, L.stride, L.items, L.tbase,
                     L.islot, L.nitems, L.tinfo, L.usum, L.chunk);
  return hipGetLastError();
}

template <int R>
hipError_t launch_batch_mixed_sym(const BatchLaunch &L, hipStream_t s) {
  if (!L.usum || L.chunk <= 0 || L.chunk % 256 != 0 || L.nitems < 0) {
    return hipErrorInvalidValue;
  }
  if (L.nitems == 0) return hipSuccess;
  if (L.kahan) {
    hipLaunchKernelGGL((k_batch_force_mixed_sym<R, true>), dim3(L.nitems),
                       dim3(kBlock), 0, s, L.shadow, L.stride, L.items, L.tbase,
                       L.islot, L.nitems, L.tinfo, L.usum, L.chunk);
  } else {
    hipLaunchKernelGGL((k_batch_force_mixed_sym<R, false>), dim3(L.nitems),
                       dim3(kBlock), 0, s, L.shadow, L.stride, L.items, L.tbase,
                       L.islot, L.nitems, L.tinfo, L.usum, L.chunk);
  }
  return hipGetLastError();
}

template <int R, int TJ>
hipError_t launch_batch_mixed(const BatchLaunch &L, hipStream_t s) {
  if (L.kahan) {
    static const int grid = persistent_grid(k_batch_force_mixed<R, TJ, true>);
    hipLaunchKernelGGL((k_batch_force_mixed<R, TJ, true>), dim3(grid),
                       dim3(kBlock), 0, s, L.shadow, L.stride, L.items,
                       L.tbase, L.islot, L.nitems, L.tinfo, L.out, L.counter);
  } else {
    static const int grid = persistent_grid(k_batch_force_mixed<R, TJ, false>);
    hipLaunchKernelGGL((k_batch_force_mixed<R, TJ, false>), dim3(grid),
                       dim3(kBlock), 0, s, L.shadow, L.stride, L.items,
                       L.tbase, L.islot, L.nitems, L.tinfo, L.out, L.counter);
  }
  return hipGetLastError();
}

// variant bits: 1 = FP64 weight without the e^2 term; 2 = sorted input with
// (wave, tile) culling of the softening test; 4 = matrix-core far field
// (with 2: sorted input; a wave owns 64 particles, so it is listed as r = 1);
// 8 = symmetric units (FP64: with 2 and 4; mixed: with 2; jsplit is the
// chunk count); 16 = FP64 symmetric: the j-quad layout of the far blocks;
// mixed symmetric: one Newton step on the FP32 r^-3.
#define F64_SET(R)                                                  \
  {kClassF64, R, 128, 0, launch_f64<R, 128, true, false>},          \
      {kClassF64, R, 128, 1, launch_f64<R, 128, false, false>},     \
      {kClassF64, R, 128, 2, launch_f64<R, 128, true, true>},       \
      {kClassF64, R, 128, 3, launch_f64<R, 128, false, true>}
#define MIXED_SET(R, TJ)                                            \
  {kClassMixed, R, TJ, 0, launch_mixed<R, TJ, false>},              \
      {kClassMixed, R, TJ, 2, launch_mixed<R, TJ, true>}

const ForceVariant kVariants[] = {
    F64_SET(1),         F64_SET(2),         F64_SET(4),         F64_SET(8),
    {kClassF64, 1, 128, 6, launch_f64_mfma<128>},
    {kClassF64, 1, 256, 6, launch_f64_mfma<256>},
    {kClassF64, 1, 256, 14, launch_f64_sym<256, false>},
    {kClassF64, 1, 256, 30, launch_f64_sym<256, true>},
    MIXED_SET(1, 128),  MIXED_SET(2, 256),  MIXED_SET(4, 256),  MIXED_SET(8, 256),
    {kClassMixed, 2, 256, 10, launch_mixed_sym<2, false>},
    {kClassMixed, 4, 256, 10, launch_mixed_sym<4, false>},
    {kClassMixed, 2, 256, 26, launch_mixed_sym<2, true>},
    {kClassMixed, 4, 256, 26, launch_mixed_sym<4, true>},
};

// ensemble variants: always culled (the ensemble keeps its state sorted)
const BatchVariant kBatchVariants[] = {
    {kClassF64, 2, 128, 2, launch_batch_f64<2, 128, true>},
    {kClassF64, 2, 128, 3, launch_batch_f64<2, 128, false>},
    {kClassF64, 4, 128, 2, launch_batch_f64<4, 128, true>},
    {kClassF64, 4, 128, 3, launch_batch_f64<4, 128, false>},
    {kClassF64, 1, 128, 6, launch_batch_f64_mfma<128>},
    {kClassF64, 1, 256, 30, launch_batch_f64_sym},
    {kClassMixed, 1, 128, 2, launch_batch_mixed<1, 128>},
    {kClassMixed, 2, 256, 2, launch_batch_mixed<2, 256>},
    {kClassMixed, 4, 256, 2, launch_batch_mixed<4, 256>},
    {kClassMixed, 2, 256, 10, launch_batch_mixed_sym<2>},
    {kClassMixed, 4, 256, 10, launch_batch_mixed_sym<4>},
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

hipError_t launch_reduce_sym(const double *iplane, const double *jacc, int n,
                             int chunk, int nchunks, const int *perm,
                             double *acc, hipStream_t s) {
  if (n <= 0 || chunk <= 0 || nchunks < 1 ||
      (long long)(nchunks - 1) * chunk >= n ||
      (long long)nchunks * chunk < n || (nchunks > 1 && !jacc)) {
    return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k_reduce_sym, dim3(ceil_div(3LL * n, kBlock)),
                     dim3(kBlock), 0, s, iplane, jacc, n, chunk, nchunks, perm,
                     acc);
  return hipGetLastError();
}

hipError_t launch_batch_reduce_sym(const double *usum, int n, const int *mid,
                                   const int *moff, const int *mq,
                                   const int *mubase, int chunk, double *acc,
                                   hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (chunk <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_batch_reduce_sym, dim3(ceil_div(3LL * n, kBlock)),
                     dim3(kBlock), 0, s, usum, n, mid, moff, mq, mubase, chunk,
                     acc);
  return hipGetLastError();
}

const BatchVariant *batch_variants(int *count) {
  *count = (int)(sizeof(kBatchVariants) / sizeof(kBatchVariants[0]));
  return kBatchVariants;
}

}  // namespace steps
