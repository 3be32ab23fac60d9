/*
 * CPU FP64 oracle for the StePS direct-summation path (Racz et al. 2018,
 * "StePS: A Multi-GPU Cosmological N-body Code for Compactified
 * Simulations").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, constant table or
 * helper with the GPU library; the two meet only through the seeded input
 * generator.
 *
 * Everything here is the plain definition, written for a reader checking it
 * against the paper by eye: one particle i at a time, every j in index
 * order, no blocking, no reordering, FP64 throughout, compensated
 * (Neumaier) sums so that the oracle's own rounding stays far below the GPU
 * tolerance.  Build with -O2 -ffp-contract=off and no fast-math.
 *
 * Readings of points the paper leaves open:
 *   - The three branches of the spline kernel (Sec. 2.2, Eq. 4) use strict
 *     inequalities at r = h/2 and r = h; here u < 1/2 is the inner branch,
 *     1/2 <= u < 1 the middle one and u >= 1 the Newtonian one.  Value and
 *     slope are continuous at both joins, so the choice is harmless.
 *   - The middle branch is printed across a line break as "... -" followed by
 *     "- 48 r^2/h^4 ..."; the doubled sign is a typesetting artefact and is
 *     read as a single minus (this is the reading that makes r^2 F equal the
 *     enclosed mass of the cubic-spline density, which the tests check).
 *   - h in F(r, h) is the support radius, where the force becomes exactly
 *     1/r^2; a pair uses h = h_i + h_j (Sec. 2.2, Eqs. 2 and 8).
 *   - A pair at zero separation (the excluded self term j = i of Eq. 8, or
 *     coincident particles) contributes nothing.
 *   - The effective radial term of Eq. 8, (4 pi G / 3) rho x, is taken with
 *     the physical mean density rho_crit Omega_m / a^3, i.e. it is
 *     (Omega_m H0^2 / 2) x / a^3.  With that reading a uniform comoving ball
 *     at rest stays at rest for every a; the tests pin it.
 *   - The time step belonging to a step in a is the exact cosmic-time
 *     interval dt = integral_a^{a+da} da' / (a' H(a')) (Eq. 1), evaluated by
 *     adaptive quadrature; Eq. 13 is its first-order limit and is not used.
 *   - The acceleration of Eq. 8 depends on the velocity through the Hubble
 *     drag -2 H v, and the paper does not say which velocity a kick uses.
 *     Each half-kick evaluates A at its own end of the step: the first one
 *     at (x_n, v_n, a_n), explicitly; the second at (x_{n+1}, v_{n+1},
 *     a_{n+1}), which is linear in v_{n+1} and solved in closed form.  This
 *     is the reading under which the KDK of Eq. 11 is second order and time
 *     reversible, as the paper states for its integrator (taking the drag at
 *     the half-step velocity in the second kick makes it first order).  The
 *     G-free pair sum S is carried between steps so that each step makes
 *     exactly one O(N^2) evaluation.
 *   - The adaptive step of Eq. 12 is one global step, the smallest of the
 *     particles' proposals, with eta_i = 2.8 h_i as printed (the text calls
 *     it Plummer-equivalent although the spline's phi(0) = -2.8/h would make
 *     that h/2.8; the printed factor is kept) and |A_i| the magnitude of the
 *     kick's acceleration of Eq. 8 at the start of the step.
 *   - Reversed gravity, for the glass relaxation of Sec. 3, flips the sign
 *     of G in both the pair term and the radial term of Eq. 8 (the latter
 *     is the gravity of the matter outside); the drag is unchanged.
 *   - Periodic boxes (Eqs. 2 and 5): the paper names Ewald summation, but
 *     the formula it prints -- and this oracle -- is the direct sum over
 *     the images within 2.6 L, with no Fourier-space part.  A particle's
 *     own images cancel in pairs and are left out; the quasi-periodic
 *     option keeps the nearest image, ties broken to even.  Eq. 2 has no
 *     radial term.
 *
 * Units: Mpc, Gyr, solar masses.  H0 is given in km/s/Mpc.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- unit constants, derived here from IAU values --------------------- */
/* 1 pc = au * 648000 / pi with au = 149597870700 m; 1 Gyr = 1e9 Julian yr. */
static double oracle_mpc_in_m(void) {
  const double pi = 3.14159265358979323846;
  return 149597870700.0 * 648000.0 / pi * 1.0e6;
}
static double oracle_gyr_in_s(void) { return 365.25 * 86400.0 * 1.0e9; }

/* km/s expressed in Mpc/Gyr. */
double oracle_kms_to_mpc_per_gyr(void) {
  return 1.0e3 * oracle_gyr_in_s() / oracle_mpc_in_m();
}

/* Newton's constant in Mpc^3 / (Msun Gyr^2) from the solar mass parameter
 * GM_sun = 1.32712440018e20 m^3 s^-2. */
double oracle_G(void) {
  double mpc = oracle_mpc_in_m(), gyr = oracle_gyr_in_s();
  return 1.32712440018e20 * gyr * gyr / (mpc * mpc * mpc);
}

/* ---- the softened pair force, Sec. 2.2, Eqs. 3-4 ---------------------- */

/* Scalar force kernel F(r, h) of Eq. 4 (G-free), written term by term as
 * the paper prints it: the force per unit mass at distance r from a unit
 * mass softened with support radius h.  For h == 0 every r > 0 is in the
 * Newtonian branch. */
double oracle_kernel_F(double r, double h) {
  if (h <= 0.0 || r >= h) {
    return 1.0 / (r * r);
  }
  double h2 = h * h, h3 = h2 * h, h4 = h2 * h2, h5 = h4 * h, h6 = h3 * h3;
  double r2 = r * r, r3 = r2 * r, r4 = r2 * r2;
  if (r < 0.5 * h) {
    return 32.0 * r4 / h6 - 38.4 * r3 / h5 + 32.0 * r / (3.0 * h3);
  }
  return -32.0 * r4 / (3.0 * h6) + 38.4 * r3 / h5 - 48.0 * r2 / h4 +
         64.0 * r / (3.0 * h3) - 1.0 / (15.0 * r2);
}

/* Softened potential kernel phi(r, h) (G-free, per unit mass).  The paper
 * gives only the force; phi is its integral, fixed by phi(r) = -1/r for
 * r >= h and d phi / d r = F(r, h), so that the force is -grad phi. */
double oracle_kernel_phi(double r, double h) {
  if (h <= 0.0 || r >= h) {
    return -1.0 / r;
  }
  double u = r / h, u2 = u * u, u3 = u2 * u, u4 = u2 * u2, u5 = u4 * u;
  if (u < 0.5) {
    return (-2.8 + 16.0 / 3.0 * u2 - 9.6 * u4 + 6.4 * u5) / h;
  }
  return (-3.2 + 1.0 / (15.0 * u) + 32.0 / 3.0 * u2 - 16.0 * u3 + 9.6 * u4 -
          32.0 / 15.0 * u5) / h;
}

/* ---- compensated summation -------------------------------------------- */
typedef struct {
  double s, c;
} nsum;

static void nsum_add(nsum *a, double t) {
  double s = a->s + t;
  if (fabs(a->s) >= fabs(t)) {
    a->c += (a->s - s) + t;
  } else {
    a->c += (t - s) + a->s;
  }
  a->s = s;
}
static double nsum_get(const nsum *a) { return a->s + a->c; }

/* ---- pair sum S_i, Sec. 2.2 Eq. 8 (first term, G-free) ---------------- */

/*
 * S_i = sum_{j != i} m_j F(|x_j - x_i|, h_i + h_j) (x_j - x_i) / |x_j - x_i|
 *
 * so that the comoving pair acceleration of Eq. 8 is G S_i / a^3 (Eq. 3 puts
 * the minus sign on x_i - x_j; here it is absorbed into x_j - x_i).
 *
 * pos is SoA [3][n] (all x, then all y, then all z); mass and soft are [n].
 * If idx is NULL the sum is formed for every i (ni must equal n); otherwise
 * for the ni particles idx[k], written to row k of acc ([3][ni]).  kappa, if
 * not NULL, receives the conditioning ratio
 * |sum_j |m_j F d / r|| / |S_i| (component-wise absolute sums), used to
 * stratify errors.  nthreads <= 0 uses the OpenMP default.
 * Returns 0, or -1 on a bad argument.
 */
int oracle_forces(int64_t n, const double *pos, const double *mass,
                  const double *soft, int64_t ni, const int64_t *idx,
                  double *acc, double *kappa, int nthreads) {
  if (n < 0 || ni < 0 || (n > 0 && (!pos || !mass || !soft)) ||
      (ni > 0 && !acc) || (!idx && ni != n)) {
    return -1;
  }
  const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
  for (int64_t k = 0; k < ni; ++k) {
    int64_t i = idx ? idx[k] : k;
    nsum sx = {0, 0}, sy = {0, 0}, sz = {0, 0};
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
      double r = sqrt(dx * dx + dy * dy + dz * dz);
      if (r == 0.0) continue;
      double f = mass[j] * oracle_kernel_F(r, soft[i] + soft[j]) / r;
      nsum_add(&sx, f * dx);
      nsum_add(&sy, f * dy);
      nsum_add(&sz, f * dz);
      ax += fabs(f * dx);
      ay += fabs(f * dy);
      az += fabs(f * dz);
    }
    double gx = nsum_get(&sx), gy = nsum_get(&sy), gz = nsum_get(&sz);
    acc[k] = gx;
    acc[ni + k] = gy;
    acc[2 * ni + k] = gz;
    if (kappa) {
      double num = sqrt(ax * ax + ay * ay + az * az);
      double den = sqrt(gx * gx + gy * gy + gz * gz);
      kappa[k] = den > 0.0 ? num / den : INFINITY;
    }
  }
  return 0;
}

/* Softened potential Phi_i = sum_{j != i} m_j phi(r_ij, h_i + h_j), G-free
 * (a diagnostic; the paper is silent on it).  Same layout rules as
 * oracle_forces. */
int oracle_potential(int64_t n, const double *pos, const double *mass,
                     const double *soft, int64_t ni, const int64_t *idx,
                     double *phi, int nthreads) {
  if (n < 0 || ni < 0 || (n > 0 && (!pos || !mass || !soft)) ||
      (ni > 0 && !phi) || (!idx && ni != n)) {
    return -1;
  }
  const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
  for (int64_t k = 0; k < ni; ++k) {
    int64_t i = idx ? idx[k] : k;
    nsum s = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
      double r = sqrt(dx * dx + dy * dy + dz * dz);
      if (r == 0.0) continue;
      nsum_add(&s, mass[j] * oracle_kernel_phi(r, soft[i] + soft[j]));
    }
    phi[k] = nsum_get(&s);
  }
  return 0;
}

/* ---- periodic pair sum, Sec. 2.2 Eqs. 2 and 5 ------------------------- */

/*
 * Periodic box of side L: the pair term of Eq. 2 with the force of Eq. 5,
 * which sums the softened force over the images x_j + n L of every other
 * particle.
 *   images = 2: every integer triplet n with |x_j + n L - x_i| < 2.6 L (the
 *               cut the paper uses);
 *   images = 1: the leading term only -- the nearest image (the
 *               quasi-periodic option).
 * The nearest image of d = x_j - x_i is d - L nearbyint(d / L) per component
 * (ties to even: a pair exactly L/2 apart along an axis has two nearest
 * images, and this picks one).  The image sum starts from it and tests every
 * n in [-3, 3]^3, which holds every image within 2.6 L of a nearest-image
 * displacement (each |d_k| <= L/2).  Particle i's own images cancel in
 * pairs (n and -n) and are left out.  G-free, like oracle_forces.
 * Returns 0, or -1 on a bad argument.
 */
int oracle_forces_periodic(int64_t n, const double *pos, const double *mass,
                           const double *soft, double L, int images,
                           int64_t ni, const int64_t *idx, double *acc,
                           int nthreads) {
  if (n < 0 || ni < 0 || (n > 0 && (!pos || !mass || !soft)) ||
      (ni > 0 && !acc) || (!idx && ni != n) || !(L > 0.0) ||
      (images != 1 && images != 2)) {
    return -1;
  }
  const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
  const double cut2 = (2.6 * L) * (2.6 * L);
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
  for (int64_t k = 0; k < ni; ++k) {
    int64_t i = idx ? idx[k] : k;
    nsum sx = {0, 0}, sy = {0, 0}, sz = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double d[3] = {X[j] - X[i], Y[j] - Y[i], Z[j] - Z[i]};
      for (int c = 0; c < 3; ++c) d[c] -= L * nearbyint(d[c] / L);
      double h = soft[i] + soft[j];
      int lim = images == 1 ? 0 : 3;
      for (int a = -lim; a <= lim; ++a) {
        for (int b = -lim; b <= lim; ++b) {
          for (int e = -lim; e <= lim; ++e) {
            double ex = d[0] + a * L, ey = d[1] + b * L, ez = d[2] + e * L;
            double r2 = ex * ex + ey * ey + ez * ez;
            if (images == 2 && !(r2 < cut2)) continue;
            double r = sqrt(r2);
            if (r == 0.0) continue;
            double f = mass[j] * oracle_kernel_F(r, h) / r;
            nsum_add(&sx, f * ex);
            nsum_add(&sy, f * ey);
            nsum_add(&sz, f * ez);
          }
        }
      }
    }
    acc[k] = nsum_get(&sx);
    acc[ni + k] = nsum_get(&sy);
    acc[2 * ni + k] = nsum_get(&sz);
  }
  return 0;
}

/* ---- background cosmology, Sec. 2.2 Eq. 1 and Sec. 2.3 Eq. 13 -------- */

typedef struct {
  double H0;      /* km/s/Mpc */
  double omega_m;
  double omega_l;
  double omega_r;
  double omega_k; /* given explicitly */
  double G;       /* Mpc^3 / (Msun Gyr^2) */
  int newtonian_test; /* 1: a == 1, H == 0, no radial term, dt = da */
  int reversed_gravity; /* 1: G -> -G in the pair and the radial term */
  int images;           /* 0: open sphere (Eq. 8); 1, 2: periodic box of
                           side box_L (Eq. 2) with the image rule of
                           oracle_forces_periodic, and no radial term */
  double box_L;
} oracle_cosmo;

/* G and the radial coefficient Omega_m H0^2 / 2 as the equations of motion
 * use them: both change sign under reversed gravity (the glass relaxation of
 * Sec. 3 integrates Eq. 8 with gravity reversed; the radial term stands for
 * the gravity of the matter outside, so it is reversed with it). */
static double oracle_G_eff(const oracle_cosmo *c) {
  return c->reversed_gravity ? -c->G : c->G;
}

/* Hubble rate H(a) in 1/Gyr from the first Friedmann equation (Eq. 1). */
double oracle_hubble(double a, const oracle_cosmo *c) {
  double h0 = c->H0 * oracle_kms_to_mpc_per_gyr();
  double e2 = c->omega_m / (a * a * a) + c->omega_r / (a * a * a * a) +
              c->omega_l + c->omega_k / (a * a);
  return h0 * sqrt(e2);
}

/* integrand of dt = da / (a H(a)) */
static double oracle_dtda(double a, const oracle_cosmo *c) {
  return 1.0 / (a * oracle_hubble(a, c));
}

static double simpson_rec(const oracle_cosmo *c, double lo, double hi,
                          double flo, double fmid, double fhi, double whole,
                          double tol, int depth) {
  double mid = 0.5 * (lo + hi);
  double lm = 0.5 * (lo + mid), rm = 0.5 * (mid + hi);
  double flm = oracle_dtda(lm, c), frm = oracle_dtda(rm, c);
  double left = (mid - lo) / 6.0 * (flo + 4.0 * flm + fmid);
  double right = (hi - mid) / 6.0 * (fmid + 4.0 * frm + fhi);
  double diff = left + right - whole;
  if (depth <= 0 || fabs(diff) <= 15.0 * tol) {
    return left + right + diff / 15.0;
  }
  return simpson_rec(c, lo, mid, flo, flm, fmid, left, 0.5 * tol, depth - 1) +
         simpson_rec(c, mid, hi, fmid, frm, fhi, right, 0.5 * tol, depth - 1);
}

/* Cosmic time elapsed while the scale factor goes from a to a + da:
 * dt = integral_a^{a+da} da' / (a' H(a')), by adaptive Simpson quadrature
 * to a relative tolerance of about 1e-15.  da may be negative. */
double oracle_dt(double a, double da, const oracle_cosmo *c) {
  if (c->newtonian_test) return da;
  if (da == 0.0) return 0.0;
  double lo = a, hi = a + da, sgn = 1.0;
  if (hi < lo) {
    double t = lo;
    lo = hi;
    hi = t;
    sgn = -1.0;
  }
  double flo = oracle_dtda(lo, c), fhi = oracle_dtda(hi, c);
  double fmid = oracle_dtda(0.5 * (lo + hi), c);
  double whole = (hi - lo) / 6.0 * (flo + 4.0 * fmid + fhi);
  double tol = 1e-16 * fabs(whole);
  return sgn * simpson_rec(c, lo, hi, flo, fmid, fhi, whole, tol, 40);
}

/* ---- kick-drift-kick, Sec. 2.3 Eqs. 9-11 with the acceleration of Eq. 8 */

/* Kick K(dt) (Eq. 9): v <- v + A dt, with A the right-hand side of Eq. 8
 * at scale factor a:
 *   A_i = G S_i / a^3 + (Omega_m H0^2 / 2) x_i / a^3 - 2 H(a) v_i.
 * end == 0: A is taken at the velocity before the kick (v' = v + A(v) dt).
 * end == 1: A is taken at the velocity after it, v' = v + A(v') dt, i.e.
 *           v' = (v + (G S + radial x) dt / a^3) / (1 + 2 H dt).
 * In the Newtonian test mode A_i = G S_i and the two coincide. */
static void oracle_kick(int64_t n, const double *pos, double *vel,
                        const double *S, double a, double dt,
                        const oracle_cosmo *c, int end) {
  double G = oracle_G_eff(c);
  double ainv3 = 1.0, radial = 0.0, drag = 0.0;
  if (!c->newtonian_test) {
    double h0 = c->H0 * oracle_kms_to_mpc_per_gyr();
    ainv3 = 1.0 / (a * a * a);
    radial = c->images ? 0.0 : 0.5 * c->omega_m * h0 * h0;
    if (c->reversed_gravity) radial = -radial;
    drag = 2.0 * oracle_hubble(a, c);
  }
  for (int d = 0; d < 3; ++d) {
    for (int64_t i = 0; i < n; ++i) {
      double x = pos[d * n + i], v = vel[d * n + i], s = S[d * n + i];
      double g = G * s * ainv3 + radial * x * ainv3;
      if (end) {
        vel[d * n + i] = (v + g * dt) / (1.0 + drag * dt);
      } else {
        vel[d * n + i] = v + (g - drag * v) * dt;
      }
    }
  }
}

/* Drift D(dt) (Eq. 10): x <- x + v dt. */
static void oracle_drift(int64_t n, double *pos, const double *vel,
                         double dt) {
  for (int64_t k = 0; k < 3 * n; ++k) {
    pos[k] = pos[k] + vel[k] * dt;
  }
}

/*
 * One KDK step (Eq. 11), U(dt) = K(dt/2) D(dt) K(dt/2), from scale factor a
 * to a + da.  On entry S must hold the pair sum of the current positions; on
 * exit pos, vel and S are those of the new time.  One pair-sum evaluation.
 * Returns 0, or -1 on a bad argument.
 */
int oracle_kdk_step(int64_t n, double *pos, double *vel, const double *mass,
                    const double *soft, double *S, double a, double da,
                    const oracle_cosmo *c, int nthreads) {
  if (n < 0 || !c || (n > 0 && (!pos || !vel || !mass || !soft || !S))) {
    return -1;
  }
  if (!c->newtonian_test && (a <= 0.0 || a + da <= 0.0)) return -1;
  double dt = oracle_dt(a, da, c);
  oracle_kick(n, pos, vel, S, a, 0.5 * dt, c, 0);
  oracle_drift(n, pos, vel, dt);
  int rc = c->images
               ? oracle_forces_periodic(n, pos, mass, soft, c->box_L,
                                        c->images, n, NULL, S, nthreads)
               : oracle_forces(n, pos, mass, soft, n, NULL, S, NULL, nthreads);
  if (rc) return rc;
  oracle_kick(n, pos, vel, S, a + da, 0.5 * dt, c, 1);
  return 0;
}

/* ---- adaptive time step, Sec. 2.3 Eq. 12 ------------------------------ */

/*
 * Global step from the criterion of Eq. 12: particle i proposes
 * sqrt(2 eta_i eps / |A_i|) with eta_i = 2.8 h_i (as printed), and the step
 * is the smallest proposal, capped at dt_max.  A_i is the acceleration the
 * kick of Eq. 9 applies -- the right-hand side of Eq. 8 -- at the start of
 * the step: G S_i / a^3 + (Omega_m H0^2 / 2) x_i / a^3 - 2 H(a) v_i, with S
 * the pair sum of the current positions.  A particle with A_i = 0 proposes
 * no limit.  *da_out is the step in the scale factor whose cosmic-time
 * interval (oracle_dt) equals *dt_out, found by bisection; in the Newtonian
 * test mode A_i = G S_i and da = dt.  Returns 0, or -1 on a bad argument.
 */
int oracle_adaptive_dt(int64_t n, const double *pos, const double *vel,
                       const double *soft, const double *S, double a,
                       const oracle_cosmo *c, double eps, double dt_max,
                       double *dt_out, double *da_out) {
  if (n < 0 || !c || !dt_out || !da_out ||
      (n > 0 && (!pos || !vel || !soft || !S))) {
    return -1;
  }
  if (!(eps > 0.0) || !(dt_max > 0.0)) return -1;
  if (!c->newtonian_test && !(a > 0.0)) return -1;
  double ainv3 = 1.0, radial = 0.0, drag = 0.0;
  if (!c->newtonian_test) {
    double h0 = c->H0 * oracle_kms_to_mpc_per_gyr();
    ainv3 = 1.0 / (a * a * a);
    radial = c->images ? 0.0 : 0.5 * c->omega_m * h0 * h0;
    if (c->reversed_gravity) radial = -radial;
    drag = 2.0 * oracle_hubble(a, c);
  }
  double G = oracle_G_eff(c);
  double dt = dt_max;
  for (int64_t i = 0; i < n; ++i) {
    double A2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      double x = pos[d * n + i], v = vel[d * n + i], s = S[d * n + i];
      double Ad = G * s * ainv3 + radial * x * ainv3 - drag * v;
      A2 += Ad * Ad;
    }
    if (A2 > 0.0) {
      double eta = 2.8 * soft[i];
      double prop = sqrt(2.0 * eta * eps / sqrt(A2));
      if (prop < dt) dt = prop;
    }
  }
  *dt_out = dt;
  if (c->newtonian_test) {
    *da_out = dt;
    return 0;
  }
  /* bracket, then bisect: oracle_dt(a, .) increases with da */
  double lo = 0.0, hi = a;
  for (int k = 0; k < 200 && oracle_dt(a, hi, c) < dt; ++k) hi *= 2.0;
  for (int k = 0; k < 200 && hi - lo > 1e-17 * hi; ++k) {
    double mid = 0.5 * (lo + hi);
    if (oracle_dt(a, mid, c) < dt) {
      lo = mid;
    } else {
      hi = mid;
    }
  }
  *da_out = 0.5 * (lo + hi);
  return 0;
}

/* ---- comoving energies, for the Layzer-Irvine check -------------------- */

/*
 * The paper states no energy diagnostic; this one follows from Eq. 8.  With
 * the canonical momentum p = m a^2 dx/dt, Eq. 8 reads dp/dt = -grad U_c / a
 * for the comoving potential energy
 *   U_c = (G/2) sum_{i != j} m_i m_j phi(r_ij, h_i + h_j)
 *         - (Omega_m H0^2 / 4) sum_i m_i |x_i|^2,
 * whose gradient is the pair force plus the radial term (Omega_m H0^2 / 2) x.
 * With K = (1/2) sum m a^2 |v|^2 and W = U_c / a this gives the cosmic energy
 * equation d(K + W)/dt = -H (2K + W).  In the Newtonian test mode a = 1 and
 * the radial term is absent.
 *
 * out[0] = K, out[1] = W, out[2] = pair part of U_c, out[3] = radial part,
 * out[4..6] = sum m a^2 v (peculiar momentum; not conserved: the radial term
 * pushes outwards).  Returns 0, or -1 on a bad argument.
 */
int oracle_energy(int64_t n, const double *pos, const double *vel,
                  const double *mass, const double *soft, double a,
                  const oracle_cosmo *c, double *out, int nthreads) {
  if (n < 0 || !c || !out || (n > 0 && (!pos || !vel || !mass || !soft))) {
    return -1;
  }
  if (c->newtonian_test) a = 1.0;
  if (!(a > 0.0)) return -1;
  double *phi = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  if (!phi) return -1;
  int rc = oracle_potential(n, pos, mass, soft, n, NULL, phi, nthreads);
  if (rc) {
    free(phi);
    return rc;
  }
  double h0 = c->H0 * oracle_kms_to_mpc_per_gyr();
  double rad = c->newtonian_test ? 0.0 : 0.25 * c->omega_m * h0 * h0;
  double G = oracle_G_eff(c);
  if (c->reversed_gravity) rad = -rad;
  nsum kin = {0, 0}, upair = {0, 0}, urad = {0, 0};
  nsum px = {0, 0}, py = {0, 0}, pz = {0, 0};
  for (int64_t i = 0; i < n; ++i) {
    double vx = vel[i], vy = vel[n + i], vz = vel[2 * n + i];
    double x = pos[i], y = pos[n + i], z = pos[2 * n + i];
    nsum_add(&kin, 0.5 * mass[i] * a * a * (vx * vx + vy * vy + vz * vz));
    nsum_add(&upair, 0.5 * G * mass[i] * phi[i]);
    nsum_add(&urad, -rad * mass[i] * (x * x + y * y + z * z));
    nsum_add(&px, mass[i] * a * a * vx);
    nsum_add(&py, mass[i] * a * a * vy);
    nsum_add(&pz, mass[i] * a * a * vz);
  }
  free(phi);
  out[0] = nsum_get(&kin);
  out[2] = nsum_get(&upair);
  out[3] = nsum_get(&urad);
  out[1] = (out[2] + out[3]) / a;
  out[4] = nsum_get(&px);
  out[5] = nsum_get(&py);
  out[6] = nsum_get(&pz);
  return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
