/*
 * pp_server.h - C ABI of the photon server in libpp: continuous batching of
 * events submitted concurrently by many CPU clients.
 *
 * The paper's new chain connects several client processes to one photon
 * server, which aggregates light-emitting steps from many events and
 * clients to keep the GPU busy (Sec. 4, propagation-client and
 * instance-count paragraphs), and replaces whole-event memory residency,
 * whose power-law size made memory use unpredictable, with queues of
 * bounded size (Sec. 3, memory paragraph; Sec. 4, queue paragraph). Here the
 * clients are threads of one process calling pp_server_submit.
 *
 * A scheduler thread owns the context. It admits waiting requests into a
 * new device batch whenever a launch slot is free and their device memory
 * fits the budget, so requests that arrive while others are on the GPU join
 * the next launch, and up to max_inflight launches run at once on separate
 * HIP streams. Each request's hits are returned to it alone: because
 * randomness is keyed by (seed, event id, photon index), a request gives the
 * same hits alone and in any mix. Requests whose event id already appears in
 * the batch being formed wait for the next one.
 */
#ifndef PP_SERVER_H_
#define PP_SERVER_H_

#include <stdint.h>

#include "pp.h"
#include "pp_surrogate.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pp_server pp_server;

typedef struct {
  uint32_t max_inflight;      /* launches in flight at once (default 4) */
  uint32_t max_batch_events;  /* events per launch (default 4096) */
  uint64_t hbm_budget_bytes;  /* device bytes the batches in flight may hold (default 200e9) */
  uint64_t max_batch_photons; /* a batch closes once it holds this many photons (default 2e8) */
} pp_server_config;

typedef struct {
  double t_submit_s, t_launch_s, t_done_s; /* steady-clock seconds of one process-wide clock */
  uint64_t photons, n_hits;
  uint32_t batch_events;                    /* events in the launch that carried this request */
  uint32_t reserved;
} pp_request_info;

typedef struct {
  uint64_t submitted, completed, launches, deferred;
  uint64_t bytes_in_use, peak_bytes_in_use;
  uint64_t photons_completed;
} pp_server_stats;

/* Pure admission policy (exported for host-side tests): given the queued
 * requests in arrival order (device bytes and event id of each), the bytes
 * in use and the budget, marks in take[] (0/1) the requests admitted into
 * the next batch: in order, each request that fits the remaining budget and
 * whose event id is not already taken, up to max_events requests and until
 * max_photons photons are reached (photons[] per request). Returns the
 * number taken. */
uint32_t pp_server_admit_plan(uint32_t n, const uint64_t *bytes, const uint32_t *event_ids,
                              const uint64_t *photons, uint64_t bytes_in_use, uint64_t budget,
                              uint32_t max_events, uint64_t max_photons, uint8_t *take);

/* Device bytes a request of n_sources sources and n_photons photons holds
 * while on the device (the admission cost). */
uint64_t pp_server_request_bytes(uint32_t n_sources, uint64_t n_photons);

/* Starts a server owning ctx (ice and geometry loaded; the caller must not
 * use ctx until pp_server_destroy). cfg may be NULL for defaults. If sur is
 * not NULL, every request also gets the surrogate's expected hits per
 * module for its sources (Cherenkov sources only). */
pp_status pp_server_create(pp_context *ctx, const pp_server_config *cfg, pp_surrogate *sur, pp_server **out);

/* Drains all queued and running requests, then stops the scheduler. */
void pp_server_destroy(pp_server *srv);

/* Thread-safe. Queues one request (an event: sources sharing one event id,
 * or any sources whose event ids are all distinct from other requests in
 * flight) and returns a ticket. PP_EBUDGET if it alone exceeds the budget;
 * PP_EINVAL on invalid sources (same validation as pp_submit). */
pp_status pp_server_submit(pp_server *srv, const pp_source *sources, uint32_t n, uint64_t *ticket);

/* Thread-safe. Blocks until the request is done, copies its hits to out
 * and, if dom_expected is not NULL and a surrogate is attached, n_doms
 * expected hits per module; fills *info; the ticket is then forgotten. If
 * the request has more than cap hits, returns PP_ETRUNC with info->n_hits
 * set and keeps the result, so the call can be repeated with a larger
 * buffer. */
pp_status pp_server_wait(pp_server *srv, uint64_t ticket, pp_hit *out, uint64_t cap, float *dom_expected,
                         pp_request_info *info);

/* Thread-safe snapshot of the counters. */
pp_status pp_server_get_stats(pp_server *srv, pp_server_stats *out);

/* Message of the last scheduler error (empty if none). */
const char *pp_server_last_error(pp_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* PP_SERVER_H_ */
