// Background cosmology of libsteps (host only); see steps_cosmo.cpp.
#pragma once

namespace steps {

double kms_to_mpc_per_gyr();
double newton_G();  // Mpc^3 / (Msun Gyr^2)

struct Background {
  double h0;  // 1/Gyr
  double omega_m, omega_l, omega_r, omega_k;
  double g;   // Mpc^3 / (Msun Gyr^2), negative for reversed gravity
  bool newtonian_test;
  bool reversed;  // G -> -G in the pair and radial terms
  bool periodic;  // periodic box (Eq. 2): no radial term

  Background(double H0_kms, double om, double ol, double orad, double ok,
             double G, bool newtonian, bool reversed_gravity = false,
             bool periodic_box = false);
  // E(a)^2 = Omega_m a^-3 + Omega_r a^-4 + Omega_k a^-2 + Omega_Lambda
  double e2(double a) const;
  // H(a) in 1/Gyr (0 in the Newtonian test mode)
  double hubble(double a) const;
  // cosmic time from a to a + da; false if H^2 <= 0 on the way
  bool step_dt(double a, double da, double *dt) const;
  // the da > 0 whose step_dt is dt (> 0): Newton's method on step_dt, whose
  // derivative in da is 1 / ((a + da) H(a + da)); false if it fails
  bool da_for_dt(double a, double dt, double *da) const;
  // radial-term coefficient Omega_m H0^2 / 2 (the (4 pi G / 3) rho_bar of
  // Eq. 8 with rho_bar = Omega_m rho_crit, rho_crit = 3 H0^2 / (8 pi G))
  // (negative for reversed gravity)
  double radial() const {
    return newtonian_test || periodic
               ? 0.0
               : (reversed ? -0.5 : 0.5) * omega_m * h0 * h0;
  }
};

}  // namespace steps
