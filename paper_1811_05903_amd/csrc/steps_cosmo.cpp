// Background cosmology for libsteps (host only): the first Friedmann
// equation (Racz et al. 2018, Sec. 2.2 Eq. 1) and the cosmic-time length of
// a step in the scale factor.
//
// The paper integrates a(t) with RK4 alongside its time steps (Sec. 2.3) and
// gives the first-order relation dt = da / (a H(a)) (Eq. 13).  Here a step
// is specified in a, and its length in t is the exact interval
//     dt = integral_a^{a+da} da' / (a' H(a')) = integral d(ln a') / H(a'),
// evaluated with composite 8-point Gauss-Legendre quadrature in ln a, panel
// count doubled until two successive values agree to 1e-15 relative.

#include "steps_cosmo.h"

#include <cmath>

namespace steps {

namespace {
// 1 pc = au * 648000 / pi, au = 149597870700 m (IAU 2012); 1 Gyr = 1e9
// Julian years of 365.25 days.
constexpr double kPi = 3.14159265358979323846;
constexpr double kMpcMetres = 149597870700.0 * 648000.0 / kPi * 1.0e6;
constexpr double kGyrSeconds = 365.25 * 86400.0 * 1.0e9;
// Solar mass parameter GM_sun in m^3 s^-2 (IAU 2009 TCB-compatible value).
constexpr double kGMsun = 1.32712440018e20;

// 8-point Gauss-Legendre nodes and weights on [-1, 1].
constexpr double kGLx[4] = {0.1834346424956498049394761, 0.5255324099163289858177390,
                            0.7966664774136267395915539, 0.9602898564975362316835609};
constexpr double kGLw[4] = {0.3626837833783619829651504, 0.3137066458778872873379622,
                            0.2223810344533744705443560, 0.1012285362903762591525314};
}  // namespace

double kms_to_mpc_per_gyr() { return 1.0e3 * kGyrSeconds / kMpcMetres; }

double newton_G() {
  return kGMsun * kGyrSeconds * kGyrSeconds /
         (kMpcMetres * kMpcMetres * kMpcMetres);
}

Background::Background(double H0_kms, double om, double ol, double orad,
                       double ok, double G, bool newtonian,
                       bool reversed_gravity, bool periodic_box)
    : h0(H0_kms * kms_to_mpc_per_gyr()), omega_m(om), omega_l(ol),
      omega_r(orad), omega_k(ok),
      g((reversed_gravity ? -1.0 : 1.0) * (G > 0.0 ? G : newton_G())),
      newtonian_test(newtonian), reversed(reversed_gravity),
      periodic(periodic_box) {}

double Background::e2(double a) const {
  const double ia = 1.0 / a;
  return ((omega_r * ia + omega_m) * ia + omega_k) * ia * ia + omega_l;
}

double Background::hubble(double a) const {
  if (newtonian_test) return 0.0;
  return h0 * std::sqrt(e2(a));
}

// composite Gauss-Legendre of 1/H over ln a in [s0, s1] with `panels`
// panels; returns false if H^2 <= 0 at a node.
static bool gl_dt(const Background &b, double s0, double s1, int panels,
                  double *out) {
  const double w = (s1 - s0) / panels;
  double total = 0.0;
  for (int p = 0; p < panels; ++p) {
    const double mid = s0 + (p + 0.5) * w, half = 0.5 * w;
    double acc = 0.0;
    for (int k = 0; k < 4; ++k) {
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        const double a = std::exp(mid + sgn * half * kGLx[k]);
        const double e2 = b.e2(a);
        if (!(e2 > 0.0)) return false;
        acc += kGLw[k] / std::sqrt(e2);
      }
    }
    total += acc * half;
  }
  *out = total / b.h0;
  return true;
}

bool Background::step_dt(double a, double da, double *dt) const {
  if (newtonian_test) {
    *dt = da;
    return true;
  }
  if (da == 0.0) {
    *dt = 0.0;
    return true;
  }
  if (!(e2(a) > 0.0) || !(e2(a + da) > 0.0)) return false;
  const double s0 = std::log(a), s1 = std::log(a + da);
  double prev = 0.0;
  if (!gl_dt(*this, s0, s1, 1, &prev)) return false;
  for (int panels = 2; panels <= 4096; panels *= 2) {
    double cur;
    if (!gl_dt(*this, s0, s1, panels, &cur)) return false;
    if (std::fabs(cur - prev) <= 1e-15 * std::fabs(cur)) {
      *dt = cur;
      return true;
    }
    prev = cur;
  }
  *dt = prev;
  return true;
}

bool Background::da_for_dt(double a, double dt, double *da) const {
  if (newtonian_test) {
    *da = dt;
    return true;
  }
  if (!(dt > 0.0) || !(a > 0.0) || !(e2(a) > 0.0)) return false;
  double x = dt * a * hubble(a);  // first-order start: da = a H dt
  for (int it = 0; it < 60; ++it) {
    double t = 0.0;
    if (!(a + x > 0.0) || !step_dt(a, x, &t)) return false;
    const double step = (t - dt) * (a + x) * hubble(a + x);
    double nx = x - step;
    if (!(nx > 0.0)) nx = 0.5 * x;  // stay on the positive side
    if (std::fabs(nx - x) <= 1e-15 * nx) {
      *da = nx;
      return true;
    }
    x = nx;
  }
  *da = x;
  return std::isfinite(x) && x > 0.0;
}

}  // namespace steps
