/*
 * lbm.h -- C ABI of the gfx950 B-TriRT lattice Boltzmann melting library.
 *
 * The library advances cavities of phase-change material heated locally from
 * below (Zhao, Wu, Chai & Shi, arXiv 1909.13086, Sec. 3.2) with the block
 * triple-relaxation-time update of Sec. 2, Eq. (2), on a D2Q9 lattice:
 *   - enthalpy populations g: equilibrium of Eq. (3), k1 from the thermal
 *     diffusivity by Eq. (4), k2 = 2 - k1 by Eq. (5) unless overridden;
 *   - Boussinesq flow populations f: Eq. (2) with a second-order equilibrium
 *     and a Hermite-projected buoyancy force; the solid is immobilised by
 *     scaling the velocity with the liquid fraction;
 *   - total enthalpy H = Cp*T + fl*L (Sec. 2, under Eq. (1)) with isothermal
 *     melting at Tm;
 *   - no-slip adiabatic walls (half-way bounce-back) and a bottom strip held at
 *     Th (anti-bounce-back), Sec. 3.2.
 * Lattice units throughout: dx = dt = 1, c = 1, cs^2 = 1/3.
 *
 * Conventions shared by every call:
 *   - All functions return int: LBM_OK (0) or a negative LBM_E* code; no
 *     exception crosses the ABI.  lbm_last_error() gives a message for the last
 *     failure on the calling thread.
 *   - Pointers named "host" are host memory owned by the caller.  Device
 *     memory is allocated by the library unless the caller lends a buffer to
 *     lbm_set_case; lent memory stays owned by the caller and must outlive the
 *     slot (until lbm_release or lbm_destroy).
 *   - Field and population layout on the host: field-major, then row-major
 *     idx = y*nx + x, y = 0 the heated bottom wall.  Populations: plane i of
 *     the D2Q9 set c_0=(0,0), c_1=(1,0), c_2=(0,1), c_3=(-1,0), c_4=(0,-1),
 *     c_5=(1,1), c_6=(-1,1), c_7=(-1,-1), c_8=(1,-1), so f[i*nx*ny + y*nx + x].
 *   - Work is ordered on the context's HIP stream.  lbm_step only enqueues;
 *     lbm_reduce, lbm_fields, lbm_series, lbm_state_* and lbm_sync block until
 *     the stream has drained.  A context is not thread-safe.
 *   - A batched launch whose device work list is inconsistent (a bookkeeping
 *     fault of the library, never expected) advances nothing and raises a
 *     device error word; the next blocking call (or the next chunk of
 *     lbm_step_many) returns LBM_EDEVICE and clears it.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,    /* invalid argument or case */
  LBM_ENOMEM = -2,    /* HBM budget or device memory exhausted; nothing was changed */
  LBM_EDEVICE = -3,   /* HIP runtime error */
  LBM_EUNSTABLE = -4, /* state is no longer finite (returned with the stats) */
  LBM_ESTATE = -5,    /* wrong slot state (unused slot, busy server, ...) */
  LBM_ENOTSUP = -6    /* combination not supported */
};

enum { LBM_FP64 = 0, LBM_FP32_SHIFTED = 1 };
enum { LBM_PATTERN_AA = 0, LBM_PATTERN_AB = 1 };
enum { LBM_PARAM_DIMENSIONLESS = 0, LBM_PARAM_LATTICE = 1 };
enum { LBM_INIT_SOLID_AT_TM = 0, LBM_INIT_LIQUID_T0 = 1, LBM_INIT_GAUSSIAN = 2 };
enum {
  LBM_FIELD_T = 1,
  LBM_FIELD_FL = 2,
  LBM_FIELD_H = 4,
  LBM_FIELD_UX = 8,
  LBM_FIELD_UY = 16,
  LBM_FIELD_RHO = 32
};
#define LBM_ALL (-1)

typedef struct lbm_ctx lbm_ctx;

/*
 * How the solid and mushy cells hold the flow still.  The paper does not say;
 * three readings are offered:
 *   LBM_SOLID_SCALE  fluid velocity u = fl (j + F/2)/rho0, scaled by the
 *                    liquid fraction (default);
 *   LBM_SOLID_DARCY  enthalpy-porosity drag -A rho0 u with the Carman-Kozeny
 *                    factor A = C (1 - fl)^2 / (fl^3 + eps), taken at the half
 *                    step with the buoyancy: u = (j + F/2) / (rho0 (1 + A/2)),
 *                    and the collision forced by buoyancy plus drag;
 *   LBM_SOLID_PBB    partial bounce-back: u = (j + F/2)/rho0 as for a free
 *                    fluid, then f_i <- (1 - ns) f_i* + ns f_opp(i) with the
 *                    pre-collision populations and solid fraction ns = 1 - fl.
 */
enum { LBM_SOLID_SCALE = 0, LBM_SOLID_DARCY = 1, LBM_SOLID_PBB = 2 };

/*
 * Problem statement of one cavity (Sec. 3.2).  Physical inputs come either
 * as dimensionless groups (param_mode = LBM_PARAM_DIMENSIONLESS: Ra, Pr, Ste
 * and the lattice Mach number Ma of the free-fall velocity, with the cavity
 * height ny as length scale) or directly in lattice units
 * (LBM_PARAM_LATTICE: nu, alpha, gbeta, latent).  A rate given as NaN takes
 * its default: k0_g = 1, k2_g = 2 - k1_g (Eq. (5)), k0_f = k1_f = 1.
 */
typedef struct {
  int32_t nx, ny;           /* cells, >= 1 each */
  int32_t precision;        /* LBM_FP64 or LBM_FP32_SHIFTED */
  int32_t pattern;          /* LBM_PATTERN_AA (in place) or LBM_PATTERN_AB (two lattices) */
  int32_t param_mode;       /* LBM_PARAM_* */
  int32_t periodic_x, periodic_y;
  int32_t init;             /* LBM_INIT_* */
  double Ra, Pr, Ste, Ma;   /* dimensionless mode */
  double nu, alpha, gbeta, latent; /* lattice mode */
  double Cp, Th, Tm, rho0;
  double heater_center, heater_width; /* strip centre C and width D as fractions of nx
                                       (Sec. 3.2); cell x is heated when its centre x + 1/2
                                       lies in [(C - D/2) nx, (C + D/2) nx].  A strip that
                                       reaches past a side wall is clipped to the cavity
                                       (only its cells inside are heated); width 0 or a
                                       periodic y direction means no strip. */
  double k0_g, k2_g, k0_f, k1_f;
  double T0, gauss_amp, gauss_sigma; /* LBM_INIT_LIQUID_T0 / LBM_INIT_GAUSSIAN */
  int32_t solid_model;      /* LBM_SOLID_*: how the solid holds the flow still */
  int32_t reserved;         /* 0 */
  double darcy_c, darcy_eps; /* LBM_SOLID_DARCY constants C and eps; NaN -> 1e3 and 1e-3 */
} lbm_case;

/* Lattice parameters derived from a case (Eqs. (4)-(5) and the flow closure). */
typedef struct {
  double nu, alpha, gbeta, latent;
  double k0_g, k1_g, k2_g, k0_f, k1_f, k2_f;
  int32_t heater_lo, heater_hi, n_heater; /* heated cells x in [lo, hi] of row y = 0 */
  int32_t pitch;                          /* device row pitch in cells */
  double darcy_c, darcy_eps;              /* drag constants in use (LBM_SOLID_DARCY) */
} lbm_lattice;

/* Per-cavity diagnostics of the current state, computed in FP64 with
 * compensated sums. */
typedef struct {
  int64_t step;
  double melt_fraction;   /* mean liquid fraction (Sec. 3.2, liquid fraction curves) */
  double nusselt;         /* ny*Q/(n_heater*alpha*Cp*(Th-Tm)) from the strip flux Q */
  double heater_q;        /* enthalpy entering through the strip in the last step */
  double total_H;         /* sum of H over all cells */
  double heat_in_cum;     /* strip enthalpy summed over every step so far */
  double budget_residual; /* total_H - total_H(at load) - heat_in_cum */
  double mass;            /* sum of rho */
  double max_u;           /* max |u| */
  double fourier;         /* alpha*step/ny^2 */
  int32_t finite;         /* 1 when every population is finite */
  int32_t parity;         /* storage parity of the in-place pattern */
} lbm_stats;

/* ---- host-only calls (no GPU needed) ------------------------------------ */

/* Message for an error code; never NULL. */
const char *lbm_strerror(int code);
/* Message of the last failure on this thread (empty when none). */
const char *lbm_last_error(void);
/* Validates a case and derives its lattice parameters.  LBM_EINVAL with a
 * message for an invalid case (rates outside (0,2), non-positive viscosity or
 * diffusivity, non-positive Ra/Pr/Ste/Ma or Th <= Tm in dimensionless mode,
 * unknown enums, sizes < 1). */
int lbm_derive(const lbm_case *cs, lbm_lattice *out);
/* Device bytes one slot of this case occupies (population planes, per-column
 * strip-flux accumulators, diagnostics at load); 0 for an invalid case.
 * A lent buffer must be at least this large and 256-byte aligned. */
size_t lbm_footprint(const lbm_case *cs);
/* Library version string. */
const char *lbm_version(void);

/* ---- context and slots ---------------------------------------------------- */

/* Creates a context on `device`.  hip_stream: a hipStream_t to order all work
 * on (e.g. the current PyTorch stream), or NULL for a stream of its own.
 * hbm_budget: bytes of slot footprints the context may hold at once (0 = no
 * limit beyond device memory).  max_slots: resident cavities, >= 1. */
int lbm_create(lbm_ctx **out, int device, void *hip_stream, size_t hbm_budget, int max_slots);
/* Frees every slot the library allocated, graphs and scratch.  NULL is a no-op. */
void lbm_destroy(lbm_ctx *c);
/* Admits a cavity: validates the case, reserves its footprint against the
 * budget (LBM_ENOMEM without side effects when it does not fit), binds
 * memory (dev_buf of buf_bytes >= lbm_footprint, or NULL to let the library
 * allocate) and enqueues the initial state of cs->init at step 0.  With a
 * lent buffer nothing waits for the device; library allocation may. */
int lbm_set_case(lbm_ctx *c, const lbm_case *cs, void *dev_buf, size_t buf_bytes, int *slot_out);
/* Returns a slot's footprint to the budget and frees library-owned memory. */
int lbm_release(lbm_ctx *c, int slot);

/* ---- the hot path --------------------------------------------------------- */

/* Enqueues nsteps time steps of Eq. (2) (collide, stream, wall rules) for one
 * slot, or for every resident slot with slot = LBM_ALL (one batched launch
 * per step covers all cavities).  Asynchronous. */
int lbm_step(lbm_ctx *c, int slot, int64_t nsteps);
/* Advances slots[j] by nsteps[j] steps (each >= 0) in batched launches: one
 * launch per step covers every listed cavity still short of its count, so
 * requests of different lengths share the device (continuous batching).
 * Asynchronous.  Each result equals that of lbm_step on the slot alone. */
int lbm_step_many(lbm_ctx *c, int count, const int32_t *slots, const int64_t *nsteps);
/* Capacity of one cache group of the batched launch (default 192 MiB): within
 * a chunk of graph-replayed steps, each group of cavities whose footprints
 * sum to at most this advances through all its steps before the next group,
 * so its populations stay in the last-level cache.  A cavity whose footprint
 * exceeds it steps on the single-cavity path (as lbm_step would) instead.
 * LBM_EINVAL below 1 MiB. */
int lbm_set_group_bytes(lbm_ctx *c, size_t bytes);
/* Diagnostics of the current state.  Blocks.  Returns LBM_EUNSTABLE (with
 * *out filled) when a population is not finite. */
int lbm_reduce(lbm_ctx *c, int slot, lbm_stats *out);
/* Macroscopic fields of the current state (Sec. 2): T and fl from the total
 * enthalpy H = sum g_i through H = Cp T + fl L with melting at Tm (below
 * Eq. (1)); the velocity u = fl (j + F/2)/rho0 of the solid-phase reading in
 * use (u as defined for LBM_SOLID_DARCY / LBM_SOLID_PBB above) and rho = sum f_i.
 * For each bit of mask, in the order T, fl, H, ux, uy, rho, one nx*ny plane
 * of doubles (row-major, y = 0 the heated wall) into host; n is the capacity
 * of host in doubles.  LBM_EINVAL for an empty mask or a short buffer;
 * LBM_ENOMEM when the device staging buffer cannot grow.  Blocks. */
int lbm_fields(lbm_ctx *c, int slot, uint32_t mask, double *host, size_t n);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lbm_fields
 * with its device staging in a fixed array of 16 MiB (2^24 bytes) of static
 * device memory instead of a buffer the context grows with hipMalloc.  Each
 * GPU the library runs on holds its own copy of that array from the first
 * context on it until the process ends; the call itself allocates nothing.
 * Same arguments, layout and results as lbm_fields (bit for bit).
 * LBM_EINVAL when the requested planes need more than 16 MiB (8 bytes per
 * cell and field: one field of 2048x1024 cells, or all six of 512x512).
 * Every call on one GPU, from any context or thread of the process, shares
 * the array: calls that overlap in time on one GPU race and must be
 * serialised by the caller.  Blocks. */
int lbm_fields_noalloc(lbm_ctx *c, int slot, uint32_t mask, double *host, size_t n);

/* Records diagnostics every `every` steps into a device ring of `capacity`
 * entries while lbm_step runs (every = 0 stops).  Clears earlier entries. */
int lbm_set_report(lbm_ctx *c, int slot, int64_t every, int32_t capacity);
/* Copies up to max recorded diagnostics to host; *count gets the number. */
int lbm_series(lbm_ctx *c, int slot, lbm_stats *host, int32_t max, int32_t *count);

/* Raw pre-collision populations (FP64, layout above, 9*nx*ny each).  Load
 * resets the step counter and the strip-flux budget to zero. */
int lbm_state_load(lbm_ctx *c, int slot, const double *f, const double *g, size_t n);
int lbm_state_save(lbm_ctx *c, int slot, double *f, double *g, size_t n);

/* Checkpoint / resume.  A checkpoint is the slot's device region exactly as
 * stored (populations in their precision, layout and storage parity, the
 * per-column strip flux, the diagnostics at load) behind a header with the
 * case, the step counter and the parity; lbm_checkpoint_bytes gives its size
 * (0 for an unused slot).  Loading needs a slot of the same size, precision
 * and pattern; the restored slot takes the checkpoint's case, and stepping on
 * from it reproduces the uninterrupted run bit for bit.  Both block. */
size_t lbm_checkpoint_bytes(lbm_ctx *c, int slot);
int lbm_checkpoint_save(lbm_ctx *c, int slot, void *host, size_t n);
/* Every check (header, embedded case derived as lbm_set_case would, its
 * precision, pattern and region size against the header and the slot) runs
 * before anything is copied: on LBM_EINVAL the slot is unchanged. */
int lbm_checkpoint_load(lbm_ctx *c, int slot, const void *host, size_t n);
/* Host-only, needs no GPU: validates a checkpoint of n bytes as
 * lbm_checkpoint_load does (without the slot comparison) and returns its case
 * and step counter (either output may be NULL).  LBM_EINVAL with a message
 * for a corrupt, truncated or inconsistent checkpoint. */
int lbm_checkpoint_info(const void *host, size_t n, lbm_case *cs, int64_t *step);

/* ---- execution control ---------------------------------------------------- */

enum {
  LBM_LAUNCH_XCD_BANDS = 1,  /* each of the 8 XCDs gets a contiguous band of tiles */
  LBM_LAUNCH_NONTEMPORAL = 2, /* population loads/stores bypass cache retention */
  LBM_LAUNCH_ALTERNATE = 4,  /* tiles walked backwards on every other step */
  LBM_LAUNCH_ZIGZAG = 8,     /* fused kernels: odd row segments walked downwards,
                                so neighbouring segments share halo rows in the L2 */
  LBM_LAUNCH_STAGED = 16     /* two-step kernel: rows copied into LDS one row ahead
                                by asynchronous global-to-LDS loads (three-step
                                kernels stage in FP32 and not in FP64 regardless) */
};
/* Tile of the single-cavity step kernels for a precision: bx threads along x
 * (multiple of 64), by rows per block (bx*by <= 256), cpl rows per lane (1, 2
 * or 4) and LBM_LAUNCH_* flags.  Default 256, 1, 1,
 * LBM_LAUNCH_XCD_BANDS | LBM_LAUNCH_ALTERNATE | LBM_LAUNCH_ZIGZAG | LBM_LAUNCH_STAGED.
 * Results do not depend on the tile or the flags. */
int lbm_set_launch(lbm_ctx *c, int precision, int bx, int by, int cpl, int flags);
int lbm_get_launch(lbm_ctx *c, int precision, int *bx, int *by, int *cpl, int *flags);
/* Temporal blocking of the two-lattice pattern: with steps_per_launch = 2, 3
 * or (FP32 only) 4 a single launch advances a LBM_PATTERN_AB slot by that
 * many steps, reading its lattice once and writing the other once.  Each
 * wavefront walks a strip of 62 (two steps), 60 (three) or 58 (four) columns
 * along a segment of segment_rows rows, 1 to 64, keeping three-row windows
 * of the intermediate steps in registers (FP64 three-step launches keep the
 * second window in LDS and load rows directly; the LBM_LAUNCH_STAGED flag
 * applies to two-step launches).  Batched launches fuse at most three steps.
 * Segment rows are stored per depth (2, 3 and 4); segment_rows = 0 keeps the
 * stored value.  lbm_get_fusion returns the segment rows of the current
 * depth.  Launches never fuse steps across a report step, and step counts
 * that are not a multiple end with shorter launches.  Batched launches
 * (lbm_step_many) fuse as many steps as the slot's single-cavity launches.
 * Results equal those of single steps bit for bit.  Default: 3 steps per
 * launch in segments of 4 rows (FP64) or 6 rows (FP32), four-step segments
 * of 6 rows; two-step segments of 2 rows (FP64) or 4 rows (FP32).  Until
 * lbm_set_fusion or lbm_autotune sets it, the default follows each cavity's
 * size: FP64 cavities below 2^18 cells take two steps per launch, FP32
 * cavities of 2^21 cells or more take four; when some segment length of 1,
 * 2, 3, 4, 6 or 8 rows lets every wavefront of the launch be resident on
 * the device at once, the rows are those minimising resident passes x rows
 * collided per segment x max(rho, resident wavefronts per SIMD), rho = 4
 * (FP64) or 1.5 (FP32), else the default rows stand (lbm_slot_fusion shows
 * the result).  Batched launches choose their segment rows per cache group
 * so that the group's segments fill the device's wavefronts evenly;
 * lbm_get_fusion returns the nominal values.  LBM_EINVAL for
 * steps_per_launch outside 1..4 (4 with LBM_FP64) or segment_rows outside
 * 0..64. */
int lbm_set_fusion(lbm_ctx *c, int precision, int steps_per_launch, int segment_rows);
int lbm_get_fusion(lbm_ctx *c, int precision, int *steps_per_launch, int *segment_rows);
/* Steps per captured HIP graph replayed by lbm_step (0 = plain launches). */
int lbm_set_graph_chunk(lbm_ctx *c, int chunk);
/* Times the candidates on a scratch cavity of the given size and precision
 * and selects the fastest: block shape, rows per lane and walk flags of the
 * one-step kernels, segment rows and staged or direct rows of the two-step
 * kernel, segment rows of the three-step kernel (and in FP32 of the four-step
 * kernel), and then two, three or four steps per launch by the time per step
 * (unless the context runs single steps)
 * (lbm_set_launch, lbm_set_fusion).  When cache_path is not NULL the choice is
 * recorded there (JSON, one entry per precision and power-of-two size class:
 * bx, by, cpl, flags, us per one-step launch, segment rows and us per launch
 * of the two-step kernel, the same of the three-step kernel and in FP32 of
 * the four-step kernel) and a cached entry is reused. */
int lbm_autotune(lbm_ctx *c, int precision, int nx, int ny, const char *cache_path);
/* Measurement aid: the streaming ceiling of the lattice layout, against which
 * the step kernels' memory rate is read (no lattice arithmetic).  Allocates
 * one buffer of `bytes` (in place, LBM_PATTERN_AA) or two (LBM_PATTERN_AB),
 * rounded down to whole 64-cell chunks of 18 FP64 planes, and times
 * `launches` launches (1 .. 100000) on the context stream after two untimed
 * ones: each wavefront reads one chunk and writes it back in place or to the
 * other buffer, in the order the step kernels use (XCD bands, direction and,
 * for two buffers, source and destination alternating between launches).
 * *us gets the mean time per launch in microseconds; the bytes moved per
 * launch are twice the buffer size.  Buffers are freed before return.
 * LBM_EINVAL for NULL arguments, a bad pattern or count, or fewer bytes than
 * one chunk; LBM_ENOMEM if the buffers do not fit; LBM_EDEVICE on a HIP
 * error.  Waits for the context stream before and after. */
int lbm_stream_probe(lbm_ctx *c, size_t bytes, int pattern, int launches, double *us);
/* Waits for all work on the context stream. */
int lbm_sync(lbm_ctx *c);
/* The hipStream_t the context orders its work on. */
int lbm_stream(lbm_ctx *c, void **stream);
/* Step counter, parity and footprint of a slot. */
int lbm_slot_info(lbm_ctx *c, int slot, int64_t *step, int32_t *parity, size_t *bytes);
/* Steps per launch and segment rows that lbm_step uses for this slot (1 for
 * in-place slots), after the default fusion has followed the cavity size
 * (lbm_set_fusion).  LBM_EINVAL for a bad slot or NULL outputs. */
int lbm_slot_fusion(lbm_ctx *c, int slot, int *steps_per_launch, int *segment_rows);

#ifdef __cplusplus
}
#endif
#endif
