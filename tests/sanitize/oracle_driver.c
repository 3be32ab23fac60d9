/*
 * Runs every oracle entry point once on small inputs, for a build with
 * -fsanitize=address,undefined (host memory errors and undefined
 * behaviour in the oracle).  Includes the oracle's single source file.
 */
#include "../../oracle/oracle.c"

#include <stdio.h>

static double frand(unsigned *s) {
  *s = *s * 1664525u + 1013904223u;
  return (*s >> 8) * (1.0 / 16777216.0);
}

int main(void) {
  enum { N = 37 };
  double pos[3 * N], vel[3 * N], mass[N], soft[N], S[3 * N], phi[N], kap[N];
  double e[7], dt = 0.0, da = 0.0;
  unsigned seed = 12345u;
  for (int i = 0; i < N; ++i) {
    for (int d = 0; d < 3; ++d) {
      pos[d * N + i] = 10.0 * frand(&seed);
      vel[d * N + i] = frand(&seed) - 0.5;
    }
    mass[i] = 1e11 * (0.5 + frand(&seed));
    soft[i] = 0.1 + frand(&seed);
  }
  pos[3] = pos[5]; pos[N + 3] = pos[N + 5]; pos[2 * N + 3] = pos[2 * N + 5];
  soft[7] = 0.0;
  oracle_cosmo c = {70.0, 0.3, 0.7, 0.0, 0.0, oracle_G(), 0, 0, 0, 0.0};
  int64_t idx[3] = {0, 5, N - 1};
  double Ssub[9];
  int rc = 0;
  rc |= oracle_forces(N, pos, mass, soft, N, NULL, S, kap, 2);
  rc |= oracle_forces(N, pos, mass, soft, 3, idx, Ssub, NULL, 1);
  rc |= oracle_potential(N, pos, mass, soft, N, NULL, phi, 2);
  rc |= oracle_energy(N, pos, vel, mass, soft, 0.4, &c, e, 2);
  rc |= oracle_adaptive_dt(N, pos, vel, soft, S, 0.4, &c, 1e-2, 1.0, &dt, &da);
  rc |= oracle_kdk_step(N, pos, vel, mass, soft, S, 0.4, da, &c, 2);
  oracle_cosmo cp = c;
  cp.images = 2;
  cp.box_L = 10.0;
  rc |= oracle_forces_periodic(N, pos, mass, soft, 10.0, 2, N, NULL, S, 2);
  rc |= oracle_forces_periodic(N, pos, mass, soft, 10.0, 1, N, NULL, S, 2);
  rc |= oracle_kdk_step(N, pos, vel, mass, soft, S, 0.4, 0.01, &cp, 2);
  oracle_cosmo cr = c;
  cr.reversed_gravity = 1;
  rc |= oracle_kdk_step(N, pos, vel, mass, soft, S, 0.4, 0.01, &cr, 2);
  /* bad arguments are refused, not dereferenced */
  if (oracle_forces(-1, pos, mass, soft, 0, NULL, S, NULL, 1) != -1) rc |= 1;
  if (oracle_forces_periodic(N, pos, mass, soft, 0.0, 2, N, NULL, S, 1) != -1) rc |= 1;
  double t = oracle_dt(0.1, 0.5, &c) + oracle_hubble(0.5, &c) +
             oracle_kernel_F(0.3, 1.0) + oracle_kernel_phi(0.7, 1.0);
  printf("oracle driver: rc=%d dt=%g check=%g\n", rc, dt, t);
  return rc != 0;
}
