/* Drives every entry point of the CPU oracle on small cases so that the
 * address and undefined-behaviour sanitizers can watch it (built and run by
 * tests/test_oracle_sanitizers.py on the CPU). */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "btrirt_oracle.h"

static or_case base_case(int nx, int ny) {
  or_case c = {0};
  c.nx = nx;
  c.ny = ny;
  c.param_mode = OR_PARAM_DIMENSIONLESS;
  c.Ra = 1e5; c.Pr = 1.0; c.Ste = 1.0; c.Ma = 0.1;
  c.Cp = 1.0; c.Th = 1.0; c.Tm = 0.0; c.rho0 = 1.0;
  c.heater_center = 0.5; c.heater_width = 0.25;
  c.k0_g = c.k2_g = c.k0_f = c.k1_f = NAN;
  c.darcy_c = c.darcy_eps = NAN;
  return c;
}

static int run(or_case c, int steps, unsigned seed) {
  or_state *st = or_create(&c);
  if (!st) return 1;
  const size_t n = (size_t)c.nx * c.ny * OR_Q;
  double *f = malloc(n * sizeof(double)), *g = malloc(n * sizeof(double));
  double *fld = malloc((size_t)c.nx * c.ny * 6 * sizeof(double));
  if (!f || !g || !fld) return 2;
  or_init_solid(st);
  or_step(st, steps);
  or_init_gaussian(st, 0.5, 1.0, 2.0);
  or_step(st, 3);
  or_init_liquid(st, 0.7);
  srand(seed);
  for (size_t k = 0; k < n; ++k) {
    f[k] = 0.1 * (1.0 + 0.1 * rand() / RAND_MAX);
    g[k] = 0.1 * (2.5 * rand() / RAND_MAX - 0.5);
  }
  or_set_populations(st, f, g);
  or_step(st, steps);
  or_get_populations(st, f, g);
  const size_t m = (size_t)c.nx * c.ny;
  or_fields(st, fld, fld + m, fld + 2 * m, fld + 3 * m, fld + 4 * m, fld + 5 * m);
  or_stats s;
  or_get_stats(st, &s);
  const or_params *p = or_get_params(st);
  double fo[OR_Q], go[OR_Q], mac[6];
  or_collide_cell(p, f, g, fo, go, mac);
  double T, fl, geq[OR_Q], feq[OR_Q];
  or_enthalpy_map(0.3, 1.0, 0.0, 1.0, &T, &fl);
  or_geq(0.3, T, 0.01, -0.02, 1.0, geq);
  or_feq(1.0, 0.01, -0.02, 1.0, feq);
  or_destroy(st);
  free(f);
  free(g);
  free(fld);
  return s.finite ? 0 : 3;
}

int main(void) {
  or_set_threads(2);
  int rc = 0;
  or_case c = base_case(40, 20);
  rc |= run(c, 60, 1);
  c.periodic_x = 1;
  rc |= run(c, 20, 2);
  c = base_case(1, 12);
  c.periodic_x = 1;
  c.heater_width = 1.0;
  rc |= run(c, 20, 3);
  c = base_case(33, 17);
  c.periodic_x = c.periodic_y = 1;
  rc |= run(c, 20, 4);
  for (int model = OR_SOLID_DARCY; model <= OR_SOLID_PBB; ++model) {
    c = base_case(24, 12);
    c.solid_model = model;
    rc |= run(c, 30, 5 + model);
  }
  c = base_case(0, 4);  /* invalid: rejected without touching memory */
  if (or_create(&c) != NULL) rc |= 4;
  printf("oracle driver: %s\n", rc ? "FAILED" : "ok");
  return rc;
}
