/*
 * btrirt_oracle.h -- plain FP64 CPU oracle for the block triple-relaxation-time
 * (B-TriRT) lattice Boltzmann melting step of Zhao, Wu, Chai & Shi (arXiv
 * 1909.13086).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this code; only the test suite, the package smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no source with the GPU path.
 *
 * What it computes (all in lattice units dx = dt = 1, c = 1, cs^2 = 1/3):
 *   - Sec. 2, Eq. (1): total-enthalpy energy equation, H = Cp*T + fl*L;
 *   - Sec. 2, Eq. (2): the B-TriRT update, applied to the enthalpy populations
 *     g (equilibrium of Eq. (3), k1 from Eq. (4), k2 = 2 - k1 from Eq. (5)) and,
 *     as a reading of the paper, to the Boussinesq flow populations f;
 *   - Sec. 3.2: cavity with no-slip adiabatic walls and a bottom strip held at
 *     Th, the PCM starting solid at Tm;
 *   - how the solid holds the flow still, which the paper does not state: three
 *     readings (velocity scaled by the liquid fraction, Carman-Kozeny drag,
 *     partial bounce-back), see OR_SOLID_*.
 * Every reading of a point the paper leaves open is stated beside the code that
 * takes it.  Storage is two lattices with pull streaming; this is the plain
 * reference, not a fast solver.
 *
 * Parity status: every function here is pinned by CPU tests against closed forms,
 * invariants or independently coded special cases (moment identities of the
 * equilibria and projections, the SRT limit, the enthalpy map, the Neumann
 * (Stefan) solution of Eqs. (6)-(7), Gaussian diffusion, conservation, the
 * discrete heater budget, Poiseuille flow, mirror symmetry and quiescence; for
 * the solid readings: the drag's half-step momentum balance, the bounce-back's
 * affine mix of a free-fluid collision and a full reflection).
 * The coupled high-Rayleigh cavity itself has no printed numbers in the paper:
 * beyond those properties its trajectories are "parity unpinned".
 */
#ifndef BTRIRT_ORACLE_H
#define BTRIRT_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define OR_Q 9

/* How the physical parameters are given. */
enum { OR_PARAM_DIMENSIONLESS = 0, OR_PARAM_LATTICE = 1 };

/* How the flow is held still in solid and mushy cells (the paper does not
 * say; readings, see or_collide_cell):
 *   OR_SOLID_SCALE: fluid velocity scaled by the liquid fraction;
 *   OR_SOLID_DARCY: enthalpy-porosity drag -A rho0 u, A = C (1-fl)^2/(fl^3+eps);
 *   OR_SOLID_PBB:   partial bounce-back of the flow populations with solid
 *                   fraction 1 - fl. */
enum { OR_SOLID_SCALE = 0, OR_SOLID_DARCY = 1, OR_SOLID_PBB = 2 };

/* Problem statement.  Any relaxation rate left as NaN takes its default. */
typedef struct {
  int nx, ny;               /* cells along x (horizontal) and y (vertical, y=0 heated bottom) */
  int periodic_x, periodic_y;
  int param_mode;           /* OR_PARAM_DIMENSIONLESS or OR_PARAM_LATTICE */
  double Ra, Pr, Ste, Ma;   /* dimensionless mode (Sec. 3.2) */
  double nu, alpha, gbeta, latent; /* lattice mode: viscosity, diffusivity, g*beta, latent heat */
  double Cp, Th, Tm, rho0;
  double heater_center, heater_width; /* strip centre C and width D, fractions of nx */
  double k0_g, k2_g;        /* enthalpy rates; k1_g always follows Eq. (4) */
  double k0_f, k1_f;        /* flow rates; k2_f always follows the viscosity */
  int solid_model;          /* OR_SOLID_* */
  double darcy_c, darcy_eps; /* OR_SOLID_DARCY constants; NaN -> 1e3 and 1e-3 */
} or_case;

/* Lattice parameters derived from an or_case. */
typedef struct {
  int nx, ny, periodic_x, periodic_y;
  double nu, alpha, gbeta, latent, Cp, Th, Tm, rho0;
  double k0_g, k1_g, k2_g, k0_f, k1_f, k2_f;
  int heater_lo, heater_hi; /* heater cells x in [heater_lo, heater_hi] on row y=0; none if lo>hi */
  int n_heater;
  int solid_model;
  double darcy_c, darcy_eps;
} or_params;

typedef struct {
  long step;
  double melt_fraction;   /* mean liquid fraction over all cells */
  double nusselt;         /* heater-averaged wall Nusselt number from the link flux */
  double heater_q;        /* enthalpy entering through the strip in the step that produced this state */
  double total_H;         /* sum of H over all cells */
  double heat_in_cum;     /* sum of heater_q over steps 1..t */
  double budget_residual; /* total_H(t) - total_H(0) - heat_in_cum */
  double mass;            /* sum of rho */
  double max_u;           /* max |u| */
  double fourier;         /* alpha * t / ny^2 */
  int finite;             /* 1 if every population is finite */
} or_stats;

typedef struct or_state or_state;

/* Derives lattice parameters.  Returns 0, or -1 for an invalid case. */
int or_derive(const or_case *cs, or_params *out);

or_state *or_create(const or_case *cs);   /* NULL on invalid input */
void or_destroy(or_state *st);
const or_params *or_get_params(const or_state *st);

/* Initial states (all at t = 0, u = 0, f_i = w_i*rho0). */
void or_init_solid(or_state *st);                      /* H = Cp*Tm everywhere (Sec. 3.2) */
void or_init_liquid(or_state *st, double T0);          /* liquid at T0 > Tm */
void or_init_gaussian(or_state *st, double T0, double amp, double sigma);
/* Raw pre-collision populations, layout [i][y][x], 9*nx*ny doubles each. */
void or_set_populations(or_state *st, const double *f, const double *g);
void or_get_populations(const or_state *st, double *f, double *g);

void or_step(or_state *st, long nsteps);

/* Macroscopic fields of the current (pre-collision) state, [y][x]; any may be NULL. */
void or_fields(const or_state *st, double *T, double *fl, double *H,
               double *ux, double *uy, double *rho);
void or_get_stats(const or_state *st, or_stats *out);

/* Single-cell pieces, exported so tests can pin them one by one. */
void or_enthalpy_map(double H, double Cp, double Tm, double latent, double *T, double *fl);
void or_geq(double H, double T, double ux, double uy, double Cp, double geq[OR_Q]);
void or_feq(double rho, double ux, double uy, double rho0, double feq[OR_Q]);
/* One collision of a single cell: f,g pre-collision in, post-collision out;
 * macro[6] = {T, fl, H, ux, uy, rho} (may be NULL). */
void or_collide_cell(const or_params *p, const double f[OR_Q], const double g[OR_Q],
                     double fout[OR_Q], double gout[OR_Q], double macro[6]);

int or_num_threads(void);
void or_set_threads(int n); /* OpenMP threads for the row loops (results do not depend on it) */

#ifdef __cplusplus
}
#endif
#endif
