/*
 * gs_serve.h - request loop serving projection renders (Eq. 7) and volume
 * queries (Eq. 4, Sec. 3.2.2) for many resident Gaussian models on one GPU.
 *
 * A server owns worker threads, each with its own HIP stream and gs_plan.
 *
 * Continuous batching (batching = 1).  When a run starts, the server measures
 * the tile-list entries of one view of every (model, detector size) and of
 * one volume query of every (model, grid shape) in the trace, and reserves
 * each worker's plan (forward only) and two output slots within its share of
 * hbm_budget_bytes: batches of up to max_batch_views views of the largest
 * model, and the largest volume query, or fewer views per batch if that does
 * not fit.  A worker takes the oldest queued request and, for a projection,
 * every other queued projection with the same detector size, of any model,
 * while the batch stays within the reservation; all their views render in one
 * launch (gs_project_fwd_multi).  It enqueues the batch and goes back to the
 * queue without waiting: up to two batches per worker are on the device
 * while newly arrived requests are admitted.  Nothing is allocated and no
 * stream is synchronized per batch, and the device memory in use stays within
 * the budget.  A request that cannot fit its worker's reservation alone fails
 * with GS_ENOMEM in its status; a batch whose tile lists overflow the
 * reservation (the entry estimate was short) is served again request by
 * request.  A request's result equals the same request run alone up to the
 * FP32 order of partial sums (a batch may split tile lists differently).
 *
 * Graph replay (batching = 2): continuous batching in which a projection
 * batch replays a HIP graph captured, when the run starts, for its shape
 * (views padded to a multiple of 8 above 8, detector size, model size class: models
 * whose binning chunk counts share a power of two).  The batch's request
 * state, its views and each view's Gaussian set, is copied to device memory
 * before the replay; the graph's kernels read it there, and its results are
 * copied to the requests' outputs after it.  Volume queries are launched
 * directly.  Results equal those of batching = 1 up to the FP32 order of
 * partial sums.
 *
 * Per request (batching = 0): the plain path, one request per launch on an
 * allocating plan, waited for, with admission while the estimated memory of
 * the work in flight stays within hbm_budget_bytes.
 *
 * All pointers to Gaussians and outputs are device pointers owned by the
 * caller; they must stay valid until gs_server_run returns.  One
 * gs_server_run at a time per server.
 */
#ifndef GS_SERVE_H
#define GS_SERVE_H

#include "gs.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gs_server gs_server;

typedef struct {
  int32_t n_workers;         /* >= 1 (threads, each with a stream and a plan) */
  int32_t batching;          /* 0: plain, one request per launch; 1: continuous batching;
                                2: continuous batching with graph replay */
  int32_t max_batch_views;   /* >= 1, views per merged projection launch */
  float cutoff;              /* Mahalanobis cutoff of every request (> 0, INFINITY = none) */
  int64_t hbm_budget_bytes;  /* > 0: device memory of the workers' workspaces (continuous)
                                or of the work in flight (plain) */
} gs_server_config;

typedef enum { GS_REQ_PROJECT = 0, GS_REQ_VOLUME = 1 } gs_request_kind;

/* One request of a trace (host struct).  Projection: n_views views (all the
 * same detector size) written to out [n_views][h][w].  Volume: grid written to
 * out [nz][ny][nx].  out may be NULL: the result is then written to worker
 * scratch memory and discarded (load generation). */
typedef struct {
  int32_t kind;            /* gs_request_kind */
  int32_t model;           /* id from gs_server_add_model */
  double arrival_s;        /* arrival time, seconds after the start of the run */
  int32_t n_views;
  const gs_view *views;    /* (host) projection views */
  gs_grid grid;            /* volume grid */
  float *out;              /* device output or NULL */
} gs_request;

/* Per-request result (host). */
typedef struct {
  double start_s;          /* when a worker started it (seconds after run start) */
  double done_s;           /* when its result was complete on the device */
  double latency_s;        /* done_s - arrival_s */
  int32_t batch_size;      /* requests that shared its launch */
  int32_t status;          /* gs_status */
} gs_request_result;

GS_API gs_status gs_server_create(const gs_server_config *cfg, gs_server **out);
GS_API void gs_server_destroy(gs_server *srv);

/* Register a resident model; returns its id in *model_id. */
GS_API gs_status gs_server_add_model(gs_server *srv, const gs_gaussians *g, int32_t *model_id);

/* Replay a trace in real time: request i is enqueued at its arrival time
 * (time_scale stretches or compresses the arrival times; 0 enqueues all at
 * once).  Returns when every request has completed; results[i] (host) is
 * filled, *wall_s is the run's duration.  Returns the first non-OK request
 * status, if any, after all requests have finished. */
GS_API gs_status gs_server_run(gs_server *srv, const gs_request *reqs, int64_t n, double time_scale,
                               gs_request_result *results, double *wall_s);

/* Device bytes the workers reserved for the last continuous run (0 for the
 * plain path or before a run). */
GS_API gs_status gs_server_reserved_bytes(const gs_server *srv, int64_t *bytes);

#ifdef __cplusplus
}
#endif

#endif /* GS_SERVE_H */
