/*
 * btrirt_oracle.c -- plain FP64 CPU oracle for the B-TriRT melting step.
 *
 * TEST INFRASTRUCTURE ONLY (see btrirt_oracle.h): used by the tests, the smoke
 * check and the benchmark's CPU-baseline leg; never by the product library.
 *
 * Written to be read against the paper: one cell at a time, two lattices,
 * collide into a post-collision lattice, then pull-stream with the wall rules.
 * Build with -ffp-contract=off so every product and sum is rounded as written.
 */
#include "btrirt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D2Q9 lattice, Sec. 2: weights 4/9, 1/9 (i = 1..4), 1/36 (i = 5..8).  The
 * velocity set and cs^2 = 1/3 are not printed; the standard ordering is used. */
static const int CX[OR_Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[OR_Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[OR_Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double W[OR_Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                               1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0;

struct or_state {
  or_params p;
  double *f, *g;   /* pre-collision populations at time t, [i][y][x] */
  double *fs, *gs; /* post-collision populations, same layout */
  long step;
  double E0;         /* sum of H at t = 0 */
  double qsum, qcmp; /* compensated running sum of the heater flux Q(1..t) */
};

/* Neumaier compensated summation: the running sum is s + c. */
static void nsum_add(double *s, double *c, double x) {
  double t = *s + x;
  if (fabs(*s) >= fabs(x))
    *c += (*s - t) + x;
  else
    *c += (x - t) + *s;
  *s = t;
}

static int valid_rate(double k) { return isfinite(k) && k > 0.0 && k < 2.0; }

int or_derive(const or_case *cs, or_params *p) {
  memset(p, 0, sizeof(*p));
  if (cs->nx < 1 || cs->ny < 1) return -1;
  if (!(cs->Cp > 0.0) || !(cs->rho0 > 0.0) || !isfinite(cs->Th) || !isfinite(cs->Tm))
    return -1;
  p->nx = cs->nx;
  p->ny = cs->ny;
  p->periodic_x = cs->periodic_x != 0;
  p->periodic_y = cs->periodic_y != 0;
  p->Cp = cs->Cp;
  p->Th = cs->Th;
  p->Tm = cs->Tm;
  p->rho0 = cs->rho0;
  if (cs->param_mode == OR_PARAM_DIMENSIONLESS) {
    /* Reading of Sec. 3.2: Ra = g*beta*dT*l^3/(nu*alpha), Pr = nu/alpha, with the
     * cavity height l = ny and the free-fall velocity sqrt(g*beta*dT*l) fixed
     * to Ma*cs.  Ste = Cp*dT/L (latent heat). */
    double dT = cs->Th - cs->Tm;
    if (!(cs->Ra > 0.0) || !(cs->Pr > 0.0) || !(cs->Ste > 0.0) || !(cs->Ma > 0.0) ||
        !(dT > 0.0))
      return -1;
    double U = cs->Ma * sqrt(CS2);
    p->nu = U * (double)cs->ny * sqrt(cs->Pr / cs->Ra);
    p->alpha = p->nu / cs->Pr;
    p->gbeta = U * U / ((double)cs->ny * dT);
    p->latent = cs->Cp * dT / cs->Ste;
  } else if (cs->param_mode == OR_PARAM_LATTICE) {
    p->nu = cs->nu;
    p->alpha = cs->alpha;
    p->gbeta = cs->gbeta;
    p->latent = cs->latent;
  } else {
    return -1;
  }
  if (!(p->nu > 0.0) || !(p->alpha > 0.0) || !isfinite(p->gbeta) || !(p->latent >= 0.0) ||
      !isfinite(p->latent))
    return -1;
  /* Eq. (4): 1/k1 = alpha/(cs^2 dt) + 1/2. */
  p->k1_g = 1.0 / (p->alpha / CS2 + 0.5);
  /* Eq. (5): k1 + k2 = 2 unless the caller overrides k2. */
  p->k2_g = isnan(cs->k2_g) ? 2.0 - p->k1_g : cs->k2_g;
  p->k0_g = isnan(cs->k0_g) ? 1.0 : cs->k0_g;
  /* Flow (reading): the stress moment carries the viscosity the same way. */
  p->k2_f = 1.0 / (p->nu / CS2 + 0.5);
  p->k0_f = isnan(cs->k0_f) ? 1.0 : cs->k0_f;
  p->k1_f = isnan(cs->k1_f) ? 1.0 : cs->k1_f;
  if (!valid_rate(p->k0_g) || !valid_rate(p->k1_g) || !valid_rate(p->k2_g) ||
      !valid_rate(p->k0_f) || !valid_rate(p->k1_f) || !valid_rate(p->k2_f))
    return -1;
  /* Heated strip (Sec. 3.2), reading for cell-centred nodes: cell x is heated
   * when its centre x + 1/2 lies in [(C - D/2) nx, (C + D/2) nx]. */
  if (!isfinite(cs->heater_center) || !isfinite(cs->heater_width)) return -1;
  p->heater_lo = 1;
  p->heater_hi = 0;
  if (cs->heater_width > 0.0 && !p->periodic_y) {
    double xa = (cs->heater_center - 0.5 * cs->heater_width) * (double)cs->nx;
    double xb = (cs->heater_center + 0.5 * cs->heater_width) * (double)cs->nx;
    double lo = ceil(xa - 0.5), hi = floor(xb - 0.5);
    if (lo < 0.0) lo = 0.0;
    if (hi > (double)(cs->nx - 1)) hi = (double)(cs->nx - 1);
    if (lo <= hi) {
      p->heater_lo = (int)lo;
      p->heater_hi = (int)hi;
    }
  }
  p->n_heater = p->heater_hi >= p->heater_lo ? p->heater_hi - p->heater_lo + 1 : 0;
  /* Solid-phase treatment of the flow (reading; the paper names none). */
  if (cs->solid_model < OR_SOLID_SCALE || cs->solid_model > OR_SOLID_PBB) return -1;
  p->solid_model = cs->solid_model;
  p->darcy_c = isnan(cs->darcy_c) ? 1e3 : cs->darcy_c;
  p->darcy_eps = isnan(cs->darcy_eps) ? 1e-3 : cs->darcy_eps;
  if (!(p->darcy_c >= 0.0) || !isfinite(p->darcy_c) || !(p->darcy_eps > 0.0) ||
      !isfinite(p->darcy_eps))
    return -1;
  return 0;
}

/* Sec. 2, below Eq. (1): H = Cp*T + fl*L with an isothermal melting point Tm.
 * Explicit branches keep T = Tm exactly inside the mushy range. */
void or_enthalpy_map(double H, double Cp, double Tm, double latent, double *T, double *fl) {
  double Hs = Cp * Tm;          /* enthalpy of solid at the melting point */
  double Hl = Cp * Tm + latent; /* enthalpy of liquid at the melting point */
  if (H <= Hs) {
    *fl = 0.0;
    *T = H / Cp;
  } else if (H >= Hl) {
    *fl = 1.0;
    *T = Tm + (H - Hl) / Cp;
  } else {
    *fl = (H - Hs) / latent;
    *T = Tm;
  }
}

/* Eq. (3): enthalpy equilibrium. */
void or_geq(double H, double T, double ux, double uy, double Cp, double geq[OR_Q]) {
  for (int i = 0; i < OR_Q; ++i) {
    if (i == 0) {
      geq[i] = H - Cp * T + W[0] * Cp * T;
    } else {
      double cu = CX[i] * ux + CY[i] * uy;
      geq[i] = W[i] * Cp * T * (1.0 + cu / CS2);
    }
  }
}

/* Flow equilibrium (reading): incompressible D2Q9 form with reference density
 * rho0, so the first moment is rho0*u and no division by rho occurs. */
void or_feq(double rho, double ux, double uy, double rho0, double feq[OR_Q]) {
  double uu = ux * ux + uy * uy;
  for (int i = 0; i < OR_Q; ++i) {
    double cu = CX[i] * ux + CY[i] * uy;
    feq[i] = W[i] * (rho + rho0 * (cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2)));
  }
}

/* Q_i : M for Q_i = c_i c_i - cs^2 I and a symmetric 2x2 tensor M. */
static double qcontract(int i, double mxx, double mxy, double myy) {
  double qxx = CX[i] * CX[i] - CS2;
  double qxy = CX[i] * CY[i];
  double qyy = CY[i] * CY[i] - CS2;
  return qxx * mxx + 2.0 * qxy * mxy + qyy * myy;
}

/* Eq. (2) for one distribution: the non-equilibrium part relaxes with k0, its
 * first moment M1 with k1 and its second moment M2 with k2. */
static void btrirt_update(const double p[OR_Q], const double peq[OR_Q], double k0, double k1,
                          double k2, const double src[OR_Q], double out[OR_Q]) {
  double neq[OR_Q];
  double m1x = 0.0, m1y = 0.0, m2xx = 0.0, m2xy = 0.0, m2yy = 0.0;
  for (int j = 0; j < OR_Q; ++j) {
    neq[j] = p[j] - peq[j];
    m1x += CX[j] * neq[j];
    m1y += CY[j] * neq[j];
    m2xx += CX[j] * CX[j] * neq[j];
    m2xy += CX[j] * CY[j] * neq[j];
    m2yy += CY[j] * CY[j] * neq[j];
  }
  for (int i = 0; i < OR_Q; ++i) {
    double cm1 = CX[i] * m1x + CY[i] * m1y;
    double qm2 = qcontract(i, m2xx, m2xy, m2yy);
    out[i] = p[i] - k0 * neq[i] - (k1 - k0) * W[i] * cm1 / CS2 -
             (k2 - k0) * W[i] * qm2 / (2.0 * CS2 * CS2);
    if (src) out[i] += src[i];
  }
}

void or_collide_cell(const or_params *p, const double f[OR_Q], const double g[OR_Q],
                     double fout[OR_Q], double gout[OR_Q], double macro[6]) {
  /* (a) total enthalpy */
  double H = 0.0;
  for (int i = 0; i < OR_Q; ++i) H += g[i];
  /* (b) temperature and liquid fraction */
  double T, fl;
  or_enthalpy_map(H, p->Cp, p->Tm, p->latent, &T, &fl);
  /* (c) flow moments, buoyancy, velocity.  Reading: Boussinesq force
   * rho0*g*beta*(T - Tm) along +y.  The solid is held still by one of three
   * readings (or_case.solid_model):
   *   SCALE: u = fl (j + F/2)/rho0, the fluid velocity scaled by the liquid
   *          fraction;
   *   DARCY: an enthalpy-porosity drag F_d = -A rho0 u with the Carman-Kozeny
   *          factor A = C (1-fl)^2/(fl^3+eps), taken at the half step like
   *          the body force, rho0 u = j + (F + F_d)/2, so
   *          u = (j + F/2)/(rho0 (1 + A/2)); the collision is forced by
   *          F + F_d;
   *   PBB:   u = (j + F/2)/rho0 as for a free fluid; after the collision the
   *          flow populations are partly bounced back, f_i <- (1 - ns) f_i* +
   *          ns f_opp(i) with the pre-collision f and solid fraction
   *          ns = 1 - fl. */
  double rho = 0.0, jx = 0.0, jy = 0.0;
  for (int i = 0; i < OR_Q; ++i) {
    rho += f[i];
    jx += CX[i] * f[i];
    jy += CY[i] * f[i];
  }
  double Fx = 0.0;
  double Fy = p->rho0 * p->gbeta * (T - p->Tm);
  double ux, uy, ns = 0.0;
  if (p->solid_model == OR_SOLID_DARCY) {
    double A = p->darcy_c * (1.0 - fl) * (1.0 - fl) / (fl * fl * fl + p->darcy_eps);
    ux = (jx + 0.5 * Fx) / (p->rho0 * (1.0 + 0.5 * A));
    uy = (jy + 0.5 * Fy) / (p->rho0 * (1.0 + 0.5 * A));
    Fx -= A * p->rho0 * ux;
    Fy -= A * p->rho0 * uy;
  } else if (p->solid_model == OR_SOLID_PBB) {
    ux = (jx + 0.5 * Fx) / p->rho0;
    uy = (jy + 0.5 * Fy) / p->rho0;
    ns = 1.0 - fl;
  } else {
    ux = fl * (jx + 0.5 * Fx) / p->rho0;
    uy = fl * (jy + 0.5 * Fy) / p->rho0;
  }
  /* (d) flow collision: Eq. (2) with (k0_f, k1_f, k2_f) plus a forcing term
   * projected on the first and second Hermite moments (reading). */
  double feq[OR_Q], force[OR_Q];
  or_feq(rho, ux, uy, p->rho0, feq);
  double sxx = 2.0 * ux * Fx, sxy = ux * Fy + uy * Fx, syy = 2.0 * uy * Fy; /* uF + Fu */
  for (int i = 0; i < OR_Q; ++i) {
    double cF = CX[i] * Fx + CY[i] * Fy;
    force[i] = W[i] * ((1.0 - 0.5 * p->k1_f) * cF / CS2 +
                       (1.0 - 0.5 * p->k2_f) * qcontract(i, sxx, sxy, syy) / (2.0 * CS2 * CS2));
  }
  btrirt_update(f, feq, p->k0_f, p->k1_f, p->k2_f, force, fout);
  if (p->solid_model == OR_SOLID_PBB)
    for (int i = 0; i < OR_Q; ++i) fout[i] = (1.0 - ns) * fout[i] + ns * f[OPP[i]];
  /* (e) enthalpy collision: Eq. (2) with g_eq of Eq. (3). */
  double geq[OR_Q];
  or_geq(H, T, ux, uy, p->Cp, geq);
  btrirt_update(g, geq, p->k0_g, p->k1_g, p->k2_g, NULL, gout);
  if (macro) {
    macro[0] = T;
    macro[1] = fl;
    macro[2] = H;
    macro[3] = ux;
    macro[4] = uy;
    macro[5] = rho;
  }
}

static size_t cell_count(const or_params *p) { return (size_t)p->nx * (size_t)p->ny; }

static int is_heater(const or_params *p, int x) {
  return x >= p->heater_lo && x <= p->heater_hi;
}

/* Enthalpy entering through the strip, from the incoming (pre-collision)
 * populations of the heated bottom cells: each anti-bounce-back link adds
 * g_in - g_out = 2*(g_i - w_i*Cp*Th). */
static double heater_flux(const or_params *p, const double *g) {
  size_t n = cell_count(p);
  double s = 0.0, c = 0.0;
  for (int x = p->heater_lo; x <= p->heater_hi; ++x) {
    for (int i = 0; i < OR_Q; ++i) {
      if (CY[i] != 1) continue;
      nsum_add(&s, &c, 2.0 * (g[(size_t)i * n + (size_t)x] - W[i] * p->Cp * p->Th));
    }
  }
  return s + c;
}

or_state *or_create(const or_case *cs) {
  or_params p;
  if (or_derive(cs, &p) != 0) return NULL;
  or_state *st = (or_state *)calloc(1, sizeof(or_state));
  if (!st) return NULL;
  st->p = p;
  size_t n = (size_t)OR_Q * cell_count(&p);
  st->f = (double *)calloc(n, sizeof(double));
  st->g = (double *)calloc(n, sizeof(double));
  st->fs = (double *)calloc(n, sizeof(double));
  st->gs = (double *)calloc(n, sizeof(double));
  if (!st->f || !st->g || !st->fs || !st->gs) {
    or_destroy(st);
    return NULL;
  }
  or_init_solid(st);
  return st;
}

void or_destroy(or_state *st) {
  if (!st) return;
  free(st->f);
  free(st->g);
  free(st->fs);
  free(st->gs);
  free(st);
}

const or_params *or_get_params(const or_state *st) { return &st->p; }

static double total_enthalpy(const or_state *st) {
  size_t n = cell_count(&st->p);
  double s = 0.0, c = 0.0;
  for (size_t k = 0; k < n; ++k) {
    double H = 0.0;
    for (int i = 0; i < OR_Q; ++i) H += st->g[(size_t)i * n + k];
    nsum_add(&s, &c, H);
  }
  return s + c;
}

static void reset_clock(or_state *st) {
  st->step = 0;
  st->qsum = 0.0;
  st->qcmp = 0.0;
  st->E0 = total_enthalpy(st);
}

/* Initial state from a temperature field at rest: liquid where T > Tm, solid
 * otherwise; g at the equilibrium of Eq. (3) with u = 0, f_i = w_i*rho0. */
static void init_from_temperature(or_state *st, const double *Tfield) {
  const or_params *p = &st->p;
  size_t n = cell_count(p);
  for (size_t k = 0; k < n; ++k) {
    double T = Tfield[k];
    double fl = T > p->Tm ? 1.0 : 0.0;
    double H = p->Cp * T + fl * p->latent;
    double geq[OR_Q], feq[OR_Q];
    or_geq(H, T, 0.0, 0.0, p->Cp, geq);
    or_feq(p->rho0, 0.0, 0.0, p->rho0, feq);
    for (int i = 0; i < OR_Q; ++i) {
      st->g[(size_t)i * n + k] = geq[i];
      st->f[(size_t)i * n + k] = feq[i];
    }
  }
  reset_clock(st);
}

void or_init_solid(or_state *st) {
  size_t n = cell_count(&st->p);
  double *T = (double *)malloc(n * sizeof(double));
  for (size_t k = 0; k < n; ++k) T[k] = st->p.Tm;
  init_from_temperature(st, T);
  free(T);
}

void or_init_liquid(or_state *st, double T0) {
  size_t n = cell_count(&st->p);
  double *T = (double *)malloc(n * sizeof(double));
  for (size_t k = 0; k < n; ++k) T[k] = T0;
  init_from_temperature(st, T);
  free(T);
}

void or_init_gaussian(or_state *st, double T0, double amp, double sigma) {
  const or_params *p = &st->p;
  size_t n = cell_count(p);
  double *T = (double *)malloc(n * sizeof(double));
  for (int y = 0; y < p->ny; ++y) {
    for (int x = 0; x < p->nx; ++x) {
      double dx = (x + 0.5) - 0.5 * p->nx;
      double dy = (y + 0.5) - 0.5 * p->ny;
      T[(size_t)y * p->nx + x] = T0 + amp * exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma));
    }
  }
  init_from_temperature(st, T);
  free(T);
}

void or_set_populations(or_state *st, const double *f, const double *g) {
  size_t n = (size_t)OR_Q * cell_count(&st->p);
  memcpy(st->f, f, n * sizeof(double));
  memcpy(st->g, g, n * sizeof(double));
  reset_clock(st);
}

void or_get_populations(const or_state *st, double *f, double *g) {
  size_t n = (size_t)OR_Q * cell_count(&st->p);
  if (f) memcpy(f, st->f, n * sizeof(double));
  if (g) memcpy(g, st->g, n * sizeof(double));
}

static void collide_all(or_state *st) {
  const or_params *p = &st->p;
  size_t n = cell_count(p);
#pragma omp parallel for schedule(static)
  for (int y = 0; y < p->ny; ++y) {
    for (int x = 0; x < p->nx; ++x) {
      size_t k = (size_t)y * p->nx + x;
      double f[OR_Q], g[OR_Q], fo[OR_Q], go[OR_Q];
      for (int i = 0; i < OR_Q; ++i) {
        f[i] = st->f[(size_t)i * n + k];
        g[i] = st->g[(size_t)i * n + k];
      }
      or_collide_cell(p, f, g, fo, go, NULL);
      for (int i = 0; i < OR_Q; ++i) {
        st->fs[(size_t)i * n + k] = fo[i];
        st->gs[(size_t)i * n + k] = go[i];
      }
    }
  }
}

/* Left-hand side of Eq. (2): pull streaming.  A link whose upstream cell lies
 * outside a non-periodic side crosses a wall half-way between nodes; it is
 * reflected into the same cell (no-slip bounce-back for f, zero-flux
 * bounce-back for g), except that a link entering a heated bottom cell through
 * the bottom wall takes the anti-bounce-back value that fixes T = Th there. */
static void stream_all(or_state *st) {
  const or_params *p = &st->p;
  size_t n = cell_count(p);
#pragma omp parallel for schedule(static)
  for (int y = 0; y < p->ny; ++y) {
    for (int x = 0; x < p->nx; ++x) {
      size_t k = (size_t)y * p->nx + x;
      for (int i = 0; i < OR_Q; ++i) {
        int sx = x - CX[i], sy = y - CY[i];
        int outside = 0;
        if (sx < 0 || sx >= p->nx) {
          if (p->periodic_x)
            sx = (sx + p->nx) % p->nx;
          else
            outside = 1;
        }
        int below = 0;
        if (sy < 0 || sy >= p->ny) {
          if (p->periodic_y) {
            sy = (sy + p->ny) % p->ny;
          } else {
            outside = 1;
            below = sy < 0;
          }
        }
        double *fi = st->f + (size_t)i * n;
        double *gi = st->g + (size_t)i * n;
        if (!outside) {
          size_t ks = (size_t)sy * p->nx + sx;
          fi[k] = st->fs[(size_t)i * n + ks];
          gi[k] = st->gs[(size_t)i * n + ks];
        } else {
          int o = OPP[i];
          fi[k] = st->fs[(size_t)o * n + k];
          if (below && is_heater(p, x))
            gi[k] = -st->gs[(size_t)o * n + k] + 2.0 * W[i] * p->Cp * p->Th;
          else
            gi[k] = st->gs[(size_t)o * n + k];
        }
      }
    }
  }
}

void or_step(or_state *st, long nsteps) {
  for (long s = 0; s < nsteps; ++s) {
    collide_all(st);
    stream_all(st);
    st->step += 1;
    nsum_add(&st->qsum, &st->qcmp, heater_flux(&st->p, st->g));
  }
}

void or_fields(const or_state *st, double *T, double *fl, double *H, double *ux, double *uy,
               double *rho) {
  const or_params *p = &st->p;
  size_t n = cell_count(p);
  for (size_t k = 0; k < n; ++k) {
    double f[OR_Q], g[OR_Q], fo[OR_Q], go[OR_Q], m[6];
    for (int i = 0; i < OR_Q; ++i) {
      f[i] = st->f[(size_t)i * n + k];
      g[i] = st->g[(size_t)i * n + k];
    }
    or_collide_cell(p, f, g, fo, go, m);
    if (T) T[k] = m[0];
    if (fl) fl[k] = m[1];
    if (H) H[k] = m[2];
    if (ux) ux[k] = m[3];
    if (uy) uy[k] = m[4];
    if (rho) rho[k] = m[5];
  }
}

void or_get_stats(const or_state *st, or_stats *out) {
  const or_params *p = &st->p;
  size_t n = cell_count(p);
  double sfl = 0.0, cfl = 0.0, sH = 0.0, cH = 0.0, sr = 0.0, cr = 0.0, umax = 0.0;
  int finite = 1;
  for (size_t k = 0; k < (size_t)OR_Q * n; ++k) {
    if (!isfinite(st->f[k]) || !isfinite(st->g[k])) finite = 0;
  }
  for (size_t k = 0; k < n; ++k) {
    double f[OR_Q], g[OR_Q], fo[OR_Q], go[OR_Q], m[6];
    for (int i = 0; i < OR_Q; ++i) {
      f[i] = st->f[(size_t)i * n + k];
      g[i] = st->g[(size_t)i * n + k];
    }
    or_collide_cell(p, f, g, fo, go, m);
    nsum_add(&sfl, &cfl, m[1]);
    nsum_add(&sH, &cH, m[2]);
    nsum_add(&sr, &cr, m[5]);
    double u = sqrt(m[3] * m[3] + m[4] * m[4]);
    if (u > umax) umax = u;
  }
  memset(out, 0, sizeof(*out));
  out->step = st->step;
  out->melt_fraction = (sfl + cfl) / (double)n;
  out->total_H = sH + cH;
  out->mass = sr + cr;
  out->max_u = umax;
  out->heater_q = heater_flux(p, st->g);
  out->heat_in_cum = st->qsum + st->qcmp;
  out->budget_residual = out->total_H - st->E0 - out->heat_in_cum;
  /* Nusselt number (reading): flux per unit heater length, scaled by the
   * conductive flux alpha*Cp*(Th - Tm)/ny across the cavity height. */
  double dT = p->Th - p->Tm;
  out->nusselt = (p->n_heater > 0 && dT != 0.0)
                     ? (double)p->ny * out->heater_q / ((double)p->n_heater * p->alpha * p->Cp * dT)
                     : 0.0;
  out->fourier = p->alpha * (double)st->step / ((double)p->ny * (double)p->ny);
  out->finite = finite;
}

void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
