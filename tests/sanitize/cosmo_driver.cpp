// Exercises the library's host-side background code (Friedmann H(a), the
// cosmic-time interval of a step in a, and its inverse) for a build with
// -fsanitize=address,undefined.
#include <cmath>
#include <initializer_list>
#include <cstdio>

#include "steps_cosmo.h"

int main() {
  int bad = 0;
  const steps::Background lcdm(67.74, 0.3089, 0.6911, 0.0, 0.0, 0.0, false);
  const steps::Background curved(70.0, 0.3, 0.5, 1e-4, 0.2 - 1e-4, 0.0, false);
  const steps::Background newton(70.0, 0.3, 0.7, 0.0, 0.0, 1.0, true, true);
  const steps::Background periodic(70.0, 0.3, 0.7, 0.0, 0.0, 0.0, false, false, true);
  for (const steps::Background *b : {&lcdm, &curved, &newton, &periodic}) {
    for (double a : {0.02, 0.1, 0.5, 1.0}) {
      double dt = 0.0, da = 0.0;
      if (!b->step_dt(a, 0.1 * a, &dt)) bad |= 1;
      if (!b->da_for_dt(a, dt, &da)) bad |= 2;
      if (std::fabs(da - 0.1 * a) > 1e-12 * a) bad |= 4;
      (void)b->hubble(a);
      (void)b->radial();
    }
  }
  double dt = 0.0;
  // H^2 <= 0 on the way is reported, not computed through
  const steps::Background closed(70.0, 1.0, -2.0, 0.0, 2.0, 0.0, false);
  if (closed.step_dt(1.0, 1.0, &dt)) bad |= 8;
  std::printf("cosmo driver: bad=%d\n", bad);
  return bad;
}
