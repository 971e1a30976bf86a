/*
 * ib_lbm_server.h — request loop that serves many independent IB-LBM cases
 * on one GPU with continuous batching.
 *
 * A server owns one worker thread and one batch (ib_lbm_batch_*).  Requests
 * (a lattice configuration, its bodies and a step count) are queued by
 * ib_lbm_server_submit from any host thread.  The worker admits queued
 * requests in arrival order while the sum of the resident requests' device
 * footprints (ib_lbm_footprint) stays within the HBM budget and the number of
 * resident requests stays within max_resident; an admitted request's lattice,
 * markers and history live on the device until it completes.  All resident
 * requests advance together: each scheduling round queues up to `quantum`
 * batch steps (one collide-stream launch per collision model and one IB
 * launch for every body of every resident request), each request stopping at
 * its own step count.  Requests that have reached their count are retired
 * (forces and optional fields copied to the host, device memory released)
 * and queued requests take their place in the next round, so work that
 * arrives while others run joins the running batch.
 *
 * A request's result does not depend on what else is resident: the
 * collide-stream update of a node and the IB pass of a body read only that
 * request's own state, and every reduction has a fixed order, so a request
 * served in a mix is bitwise identical to the same case stepped alone with
 * the same precision and spreading mode.
 *
 * Threading: submit, wait, stats and last_error may be called from any host
 * thread; destroy from one thread once.  Every HIP call is made by the
 * worker thread on the server's stream, on the device that was current when
 * the server was created.
 */
#ifndef IB_LBM_SERVER_H
#define IB_LBM_SERVER_H

#include "ib_lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define IB_LBM_SERVER_MAX_BODIES 8

/* Returned by ib_lbm_server_wait when the request is not complete by the
 * time limit (not an error). */
#define IB_LBM_PENDING 1

typedef struct ib_lbm_server ib_lbm_server;

/* hbm_budget: device bytes the resident requests may hold together
 * (0 -> 16 GiB); a request larger than the whole budget is rejected with
 * IB_LBM_E_NOMEM.  max_resident: resident requests at once (0 -> 64).
 * quantum: most batch steps queued between two scheduling decisions
 * (0 -> 256); a round is shortened to the smallest remaining step count of
 * the resident requests, so a request is retired as soon as it completes.
 * graph_steps: > 0 replays batch steps from a captured hipGraph of that many
 * steps.  launch: collide-stream launch shape (block_x = 0 -> the library's
 * default).  stream: hipStream_t the worker enqueues on; NULL -> a private
 * non-blocking stream owned by the server. */
typedef struct {
  uint32_t abi_version; /* IB_LBM_ABI_VERSION */
  int32_t precision;    /* IB_LBM_FP64 | IB_LBM_FP32_SHIFTED, for every request */
  uint64_t hbm_budget;
  int32_t max_resident;
  int32_t quantum;
  int32_t graph_steps;
  int32_t spread;       /* IB_LBM_SPREAD_GATHER | IB_LBM_SPREAD_ATOMIC */
  ib_lbm_launch launch;
  void *stream;
} ib_lbm_server_config;

/* One case.  lattice.precision must equal the server's; lattice.stream and
 * lattice.alloc are ignored (the server's stream and hipMalloc are used).
 * rho/ux/uy: optional caller-owned host arrays of nx*ny doubles that receive
 * ib_lbm_fields() of the final state before the request completes; they must
 * stay valid until ib_lbm_server_wait has returned the request's result.
 * The request struct itself is copied by submit. */
typedef struct {
  ib_lbm_config lattice;
  int32_t n_bodies; /* 0 .. IB_LBM_SERVER_MAX_BODIES */
  ib_lbm_body_desc bodies[IB_LBM_SERVER_MAX_BODIES];
  int64_t steps;    /* >= 0 */
  double *rho, *ux, *uy;
} ib_lbm_request;

/* status: IB_LBM_OK, or why the request failed: E_INVALID (configuration or
 * body rejected by ib_lbm_create / ib_lbm_add_body), E_RANGE (a support left
 * the lattice or two bodies met: the case stopped early, steps_done tells
 * where), E_DIVERGED (non-finite force), E_NOMEM (larger than the budget, or
 * the allocation failed), E_DEVICE.  Times are seconds since the server was
 * created, on a monotonic clock: submitted, admitted (device memory taken)
 * and finished (result on the host). */
typedef struct {
  int64_t id;
  int32_t status;
  int32_t n_bodies;
  int64_t steps_done;
  uint64_t footprint;
  double t_submit, t_admit, t_finish;
  ib_lbm_body_state body[IB_LBM_SERVER_MAX_BODIES];
} ib_lbm_result;

/* node_updates: sum of nx*ny*steps_done over completed requests.
 * busy_seconds: wall time during which at least one request was resident.
 * rounds: scheduling rounds (each queues one batch of steps). */
typedef struct {
  int64_t submitted, admitted, completed, failed;
  int64_t resident, queued;
  uint64_t resident_bytes, peak_resident_bytes;
  int64_t peak_resident;
  int64_t node_updates;
  int64_t rounds;
  double busy_seconds;
  double now;
} ib_lbm_server_stats;

/* Create a server and start its worker thread. */
ib_lbm_status ib_lbm_server_create(const ib_lbm_server_config *cfg, ib_lbm_server **out);

/* Queue a request (host struct copied); *id receives its identifier. */
ib_lbm_status ib_lbm_server_submit(ib_lbm_server *srv, const ib_lbm_request *req, int64_t *id);

/* Wait up to timeout_s seconds (< 0: no limit) for request `id`.  Returns
 * IB_LBM_OK with *out filled once it has completed (successfully or not:
 * see out->status), IB_LBM_PENDING on time-out, IB_LBM_E_INVALID for an
 * unknown id.  A completed result can be read any number of times. */
ib_lbm_status ib_lbm_server_wait(ib_lbm_server *srv, int64_t id, double timeout_s, ib_lbm_result *out);

/* Counters of the server (host copy). */
ib_lbm_status ib_lbm_server_stats_get(ib_lbm_server *srv, ib_lbm_server_stats *out);

/* Block until every submitted request has completed. */
ib_lbm_status ib_lbm_server_drain(ib_lbm_server *srv);

/* Finish the requests already submitted, stop the worker and free
 * everything the server holds. */
ib_lbm_status ib_lbm_server_destroy(ib_lbm_server *srv);

/* Message of the last internal failure (empty when none). */
const char *ib_lbm_server_last_error(const ib_lbm_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* IB_LBM_SERVER_H */
