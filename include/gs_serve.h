/*
 * gs_serve.h - request loop serving projection renders (Eq. 7) and volume
 * queries (Eq. 4) for many resident Gaussian models on one GPU.
 *
 * A server owns worker threads, each with its own HIP stream and gs_plan, so
 * that requests admitted together overlap on the device.  With batching on,
 * a worker that takes a projection request also takes the queued projection
 * requests of the same model with the same detector size (up to
 * max_batch_views views) and renders all their views in one launch; results
 * are then copied to each request's output.  Admission: a request (or batch)
 * starts only while the estimated device memory of the work in flight stays
 * within hbm_budget_bytes; a request that alone exceeds it fails with
 * GS_ENOMEM in its status.  Results do not depend on which requests share a
 * batch beyond FP32 summation order.
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
  int32_t batching;          /* 0: one request per launch; 1: merge same-model projections */
  int32_t max_batch_views;   /* >= 1, views per merged projection launch */
  float cutoff;              /* Mahalanobis cutoff of every request (> 0, INFINITY = none) */
  int64_t hbm_budget_bytes;  /* > 0: estimated device memory allowed in flight */
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

#ifdef __cplusplus
}
#endif

#endif /* GS_SERVE_H */
