/*
 * mg_serve.h -- C ABI of the multigrid solve server: continuous batching of independent
 * 2D solves of mixed sizes on one GPU.
 *
 * What is served.  Each request is one solve L_h u = f of the fourth-order Poisson
 * problem of mg.h (section 2.1 problem, section 2.3 eq. L_h_2d_4o operator, the section
 * 2.2 cycle) at its own side n = 2^k + 1, with the cycle, coarse operators, precision
 * and tolerance of the server's base configuration.  Solving requests in batches is not
 * part of the method; it changes only which problems share a kernel launch.
 *
 * How.  Requests of one side share a batch: one handle that holds `slots` problems of
 * that size, every level array laid out [slot][n_l * n_l], one stopping state per slot,
 * and the solve step (a gamma-cycle in FP64, or one refinement step in mixed precision)
 * captured once into a HIP graph whose kernels take the slot from the grid's third
 * dimension.  Batches run on their own streams (or on streams shared by a group of
 * sizes, stream_groups), so batches of different sizes overlap on the device.  A worker thread owned by the server replays each busy batch in
 * chunks, reads every slot's stopping flag after a chunk, copies finished solutions out
 * and admits waiting requests into the freed slots between two replays: a request that
 * arrives while others run joins the next replay of its size's batch.
 *
 * Admission.  A batch's device footprint (mg_serve_batch_bytes) counts against the
 * server's HBM budget.  A request whose size has no batch gets one if the budget allows
 * (slots = as many as fit, at most max_slots); otherwise idle batches are released,
 * least recently used first, and if that does not free enough the request waits.
 *
 * Determinism.  Slot k of a batched launch computes exactly what an unbatched handle
 * computes on the same data (same kernels, same per-slot reduction order), so a
 * request's result does not depend on what else is being served.
 *
 * Memory and threads.  f and u of a request are device FP64 arrays of n*n values on
 * the server's device; the server reads f and writes u until that request completes.
 * Submit, poll, stats and destroy may be called from any one thread at a time; the
 * worker thread makes all HIP calls of the batches.
 */
#ifndef MG_SERVE_H
#define MG_SERVE_H

#include <stddef.h>

#include "mg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mg_server_s *mg_server;

typedef struct {
  mg_config base;     /* every field but n applies to all requests; dim must be 2 */
  size_t hbm_budget;  /* device bytes the server may hold in batches */
  int max_slots;      /* most problems per batch (1..1024) */
  int chunk_steps;    /* solve steps per launch between two reads of the flags (1..64) */
  int stream_groups;  /* 0: each batch on a stream of its own; 1..3: batches share that many
                         streams by side (3: n <= 257, n <= 1025, larger; 2: n <= 1025,
                         larger; 1: one stream), so that the replays of small problems never
                         wait in a hardware queue behind those of large ones */
} mg_server_config;

typedef struct {
  long long tag;       /* the caller's tag from mg_server_submit */
  int n;               /* side of the problem */
  int status;          /* mg_status of the solve (MG_OK, MG_ENOCONV, MG_ENUMERIC) */
  double t_submit;     /* seconds on the monotonic clock: submitted, */
  double t_admit;      /*   admitted into a slot, */
  double t_done;       /*   result copied out and observed by the server */
  mg_result result;    /* as mg_solve fills it */
} mg_completion;

typedef struct {
  long long submitted, completed, rejected;
  int queued;              /* waiting for a slot */
  int active;              /* admitted, not yet completed */
  int peak_active;
  int batches;             /* live batches */
  long long batches_created, batches_released;
  size_t bytes_held;       /* device bytes of live batches */
  size_t peak_bytes_held;
  long long replays;       /* graph replays launched */
} mg_server_stats;

/* Device bytes a batch of `slots` problems of side n takes under base (0 if invalid). */
size_t mg_serve_batch_bytes(const mg_config *base, int n, int slots);

/* Creates a server on the current device and starts its worker thread.  MG_EINVAL for a
 * bad configuration; nothing is allocated on the device until requests arrive. */
mg_status mg_server_create(const mg_server_config *cfg, mg_server *out);

/* Queues a solve of side n.  f, u: device FP64 arrays of n*n values (u is overwritten
 * with the solution; its input value is ignored: every solve starts from zero).
 * MG_EINVAL for a bad side or null buffers; MG_ENOMEM if a single slot of this side
 * exceeds the whole budget (the request is rejected, not queued). */
mg_status mg_server_submit(mg_server s, long long tag, int n, const double *f, double *u);

/* Moves up to max finished requests into out and returns how many; waits up to
 * timeout_s seconds for the first one (0: do not wait).  Returns -1 on a bad argument
 * and -MG_EDEVICE after a HIP failure in the worker (mg_last_error has the message). */
int mg_server_poll(mg_server s, mg_completion *out, int max, double timeout_s);

mg_status mg_server_stats_get(mg_server s, mg_server_stats *out);

/* Stops the worker (finishing nothing further), releases every batch.  Requests not yet
 * completed are dropped; their u is left unspecified. */
mg_status mg_server_destroy(mg_server s);

/* Seconds on the clock the completion times use. */
double mg_server_clock(void);

#ifdef __cplusplus
}
#endif
#endif
