/* The C ABI used from plain C (no C++ and no HIP headers in the caller):
 * host-only entry points and argument validation, which need no GPU. */
#include <stdio.h>
#include <string.h>

#include "mpcd.h"

int main(void) {
  mpcd_params p;
  memset(&p, 0, sizeof p);
  p.n_cells[0] = p.n_cells[1] = p.n_cells[2] = 50;
  p.a = 1.0;
  p.alpha = 2.2689280275926285; /* 130 degrees */
  p.dt = 0.1;
  p.kT = 1.0;
  p.seed = 1;
  p.solvent_mass = 1.0;
  p.precision = MPCD_FP32;
  p.thermostat = 1;
  p.grid_shift = 1;
  p.flags = MPCD_TILE_4x4x4;
  p.collision = MPCD_SRD;
  int64_t peak = 0, held = 0;
  if (mpcd_footprint(&p, 1000000, 10, 1, &peak, &held) != MPCD_OK) {
    printf("footprint failed: %s\n", mpcd_last_error());
    return 1;
  }
  printf("footprint %lld %lld\n", (long long)peak, (long long)held);
  p.a = -1.0;
  const mpcd_status st = mpcd_footprint(&p, 10, 1, 1, &peak, &held);
  printf("bad cell size: %d (%s)\n", (int)st, mpcd_last_error());
  if (st != MPCD_EINVAL) return 2;
  p.a = 1.0;
  p.flags = 7 << MPCD_TILE_SHIFT; /* no such tile shape */
  if (mpcd_footprint(&p, 10, 1, 1, &peak, &held) != MPCD_EINVAL) return 3;
  mpcd_ctx ctx = NULL;
  if (mpcd_create(NULL, 0, NULL, NULL, 0, NULL, NULL, NULL, 0, NULL, &ctx) != MPCD_EINVAL || ctx)
    return 4;
  return 0;
}
