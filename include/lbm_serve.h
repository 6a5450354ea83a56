/*
 * lbm_serve.h -- request loop with continuous batching over an lbm context.
 *
 * Melting solves (cavities of Sec. 3.2 of arXiv 1909.13086, each a problem
 * statement plus a number of time steps) arrive at given times.  The loop
 * admits a queued request as soon as its device footprint fits the HBM budget
 * and a slot is free (first fit in arrival order), keeps admitted lattices
 * resident, and advances every resident cavity together in chunks of batched
 * launches (lbm_step_many), so work that arrives while others run shares the
 * device.  A request leaves when its step count is reached; its final
 * diagnostics are kept and its memory returns to the budget.
 *
 * Conventions of include/lbm.h apply (return codes, lbm_last_error).  Times
 * are seconds since lbm_server_run started, on the host's steady clock.
 */
#ifndef LBM_SERVE_H
#define LBM_SERVE_H

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_server lbm_server;

enum {
  LBM_REQ_QUEUED = 0,
  LBM_REQ_RESIDENT = 1,
  LBM_REQ_DONE = 2,
  LBM_REQ_FAILED = 3,   /* state went non-finite; slot freed, others unaffected */
  LBM_REQ_REJECTED = 4  /* footprint exceeds the whole budget */
};

typedef struct {
  int32_t id, status, precision, pad;
  int64_t steps, cells;
  double t_arrival, t_admit, t_done;
  size_t bytes;         /* device footprint while resident */
  lbm_stats stats;      /* diagnostics after the last step */
} lbm_request;

typedef struct {
  int32_t completed, failed, rejected, max_resident;
  int64_t chunks;
  double makespan_s;          /* first arrival to last result */
  double p50_s, p99_s, mean_s, max_s; /* time to result: arrival to result */
  double mlups;               /* lattice updates of completed requests / makespan, 1e6/s */
  double busy_frac;           /* share of the makespan with work resident */
  size_t peak_bytes;          /* largest resident footprint */
} lbm_serve_summary;

/* Creates a request loop.  ctx: the context whose slots hold the lattices
 * (its max_slots bounds residency), or NULL for a host-only stand-in
 * executor that advances at fake_mlups (1e6 lattice updates per second) and
 * produces no physics, for testing the scheduling on a machine without a
 * GPU.  hbm_budget: bytes of footprints resident at once (> 0); with a GPU
 * context the loop reserves this much device memory once and lends parts of
 * it to the admitted slots.  chunk: steps per batched chunk (>= 1). */
int lbm_server_create(lbm_server **out, lbm_ctx *ctx, size_t hbm_budget, int chunk,
                      double fake_mlups);
void lbm_server_destroy(lbm_server *s);
/* Queues a request arriving at arrival_s (>= 0); *id numbers requests from
 * 0 in submission order.  The case is validated here (LBM_EINVAL). */
int lbm_server_submit(lbm_server *s, const lbm_case *cs, int64_t steps, double arrival_s,
                      int32_t *id);
/* Replays the arrivals in real time divided by time_scale (time_scale = 2
 * runs arrivals twice as fast) and returns when every request has finished,
 * failed or been rejected.  Blocks. */
int lbm_server_run(lbm_server *s, double time_scale);
/* Called by lbm_server_run, on its thread, each time a request leaves the
 * loop (done, failed or rejected), with the request's final record; user is
 * passed through.  The callback must not call into the server.  fn = NULL
 * removes it.  Set before lbm_server_run. */
typedef void (*lbm_request_fn)(const lbm_request *r, void *user);
int lbm_server_on_finish(lbm_server *s, lbm_request_fn fn, void *user);
int lbm_server_request(lbm_server *s, int32_t id, lbm_request *out);
int lbm_server_summary(lbm_server *s, lbm_serve_summary *out);

#ifdef __cplusplus
}
#endif
#endif
