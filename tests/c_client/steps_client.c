/*
 * A plain C client of libsteps (no Python, no C++): builds a small particle
 * set with its own generator, computes the pair sum with steps_forces,
 * takes one KDK step with steps_step, checks that a bad call is refused
 * with a message, and writes inputs and outputs to a binary file for the
 * test to compare with the oracle.
 *
 *   steps_client <n> <out.bin>
 *
 * out.bin: int64 n, then doubles pos[3n], vel[3n], mass[n], soft[n],
 * S[3n] (of pos), a, da, H0, omega_m, omega_l, and after the step
 * pos[3n], vel[3n], S[3n].
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "steps.h"

static uint64_t lcg = 0x2545F4914F6CDD1DULL;
static double uniform01(void) {
  lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
  return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

#define CHECK_HIP(x)                                                  \
  do {                                                                \
    if ((x) != hipSuccess) {                                          \
      fprintf(stderr, "HIP error at %s:%d\n", __FILE__, __LINE__);    \
      return 2;                                                       \
    }                                                                 \
  } while (0)

#define CHECK_STEPS(x)                                                 \
  do {                                                                 \
    int rc_ = (x);                                                     \
    if (rc_ != STEPS_OK) {                                             \
      fprintf(stderr, "steps error %d: %s\n", rc_, steps_last_error()); \
      return 3;                                                        \
    }                                                                  \
  } while (0)

int main(int argc, char **argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s <n> <out.bin>\n", argv[0]);
    return 1;
  }
  const int64_t n = atoll(argv[1]);
  if (n < 2 || n > (1 << 20)) return 1;
  const size_t v3 = 3 * (size_t)n, b3 = v3 * sizeof(double), b1 = (size_t)n * sizeof(double);
  double *pos = malloc(b3), *vel = malloc(b3), *mass = malloc(b1), *soft = malloc(b1);
  double *S0 = malloc(b3), *pos1 = malloc(b3), *vel1 = malloc(b3), *S1 = malloc(b3);
  if (!pos || !vel || !mass || !soft || !S0 || !pos1 || !vel1 || !S1) return 1;
  for (int64_t i = 0; i < n; ++i) {
    for (int d = 0; d < 3; ++d) {
      pos[d * n + i] = 100.0 * (uniform01() - 0.5);
      vel[d * n + i] = 2.0 * (uniform01() - 0.5);
    }
    mass[i] = 1e11 * (0.5 + uniform01());
    soft[i] = 0.2 + 0.3 * uniform01();
  }
  double *dp, *dv, *dm, *dh, *da_;
  CHECK_HIP(hipMalloc((void **)&dp, b3));
  CHECK_HIP(hipMalloc((void **)&dv, b3));
  CHECK_HIP(hipMalloc((void **)&da_, b3));
  CHECK_HIP(hipMalloc((void **)&dm, b1));
  CHECK_HIP(hipMalloc((void **)&dh, b1));
  CHECK_HIP(hipMemcpy(dp, pos, b3, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(dv, vel, b3, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(dm, mass, b1, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(dh, soft, b1, hipMemcpyHostToDevice));

  /* a refused call: the output aliases an input */
  if (steps_forces(dp, dm, dh, n, dp) != STEPS_E_INVAL ||
      strstr(steps_last_error(), "overlap") == NULL) {
    fprintf(stderr, "aliasing was not refused\n");
    return 4;
  }

  CHECK_STEPS(steps_forces(dp, dm, dh, n, da_));
  CHECK_HIP(hipDeviceSynchronize());
  CHECK_HIP(hipMemcpy(S0, da_, b3, hipMemcpyDeviceToHost));

  steps_cosmology c;
  c.H0 = 70.0;
  c.omega_m = 0.3;
  c.omega_l = 0.7;
  c.omega_r = 0.0;
  c.omega_k = 0.0;
  c.G = 0.0;
  c.mode = STEPS_COMOVING_SPHERICAL;
  c.flags = 0;
  const double a = 0.5, da = 0.01;
  CHECK_STEPS(steps_step(dp, dv, dm, dh, n, da_, a, da, &c));
  CHECK_HIP(hipDeviceSynchronize());
  CHECK_HIP(hipMemcpy(pos1, dp, b3, hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(vel1, dv, b3, hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(S1, da_, b3, hipMemcpyDeviceToHost));

  FILE *f = fopen(argv[2], "wb");
  if (!f) return 5;
  const double scal[5] = {a, da, c.H0, c.omega_m, c.omega_l};
  fwrite(&n, sizeof(n), 1, f);
  fwrite(pos, 1, b3, f);
  fwrite(vel, 1, b3, f);
  fwrite(mass, 1, b1, f);
  fwrite(soft, 1, b1, f);
  fwrite(S0, 1, b3, f);
  fwrite(scal, sizeof(double), 5, f);
  fwrite(pos1, 1, b3, f);
  fwrite(vel1, 1, b3, f);
  fwrite(S1, 1, b3, f);
  fclose(f);
  hipFree(dp);
  hipFree(dv);
  hipFree(da_);
  hipFree(dm);
  hipFree(dh);
  printf("steps_client: n=%lld, %s\n", (long long)n, steps_version());
  return 0;
}
