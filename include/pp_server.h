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
 * Device-resident photon queue. At creation the server allocates, once, a
 * device arena within its HBM budget: a ring of source records, a ring of
 * work-queue entries (chunks of at most 256 photon ids of one source), and
 * per launch slot a counter block and a hit buffer. A scheduler thread owns
 * the context. It moves waiting requests into the rings as soon as ring
 * space frees up (one asynchronous copy per admission round from pinned
 * host memory), so the photons of admitted events wait on the device, and it
 * launches the propagation kernel over a contiguous window of the queue
 * whenever a launch slot is free: requests that arrive while others are on
 * the GPU join the next launch, and up to max_inflight launches run at once
 * on separate HIP streams. No device memory is allocated per request or per
 * launch; only a launch whose hits overflow its slot's buffer gets a
 * temporary larger one, within the budget, and is run again.
 *
 * Each request's hits are returned to it alone: because randomness is keyed
 * by (seed, event id, photon index), a request gives the same hits alone and
 * in any mix. Requests whose event id already appears in a launch being
 * formed wait for the next one.
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

/* Zero picks the default. The arena is sized from the budget B: per launch
 * slot a hit buffer of min(2^20, B / 4 / max_inflight / 32 B) hits, a
 * chunk ring of min(2^22, B / 4 / 16 B) entries and a source ring of
 * min(2^16, B / 16 / 80 B) records, each at least 64 (about 197 MiB at the
 * default budget with 4 slots). What the budget leaves beyond the arena
 * bounds the temporary buffers of overflowing launches. */
typedef struct {
  uint32_t max_inflight;      /* launches in flight at once (default 4) */
  uint32_t max_batch_events;  /* events per launch (default 4096) */
  uint64_t hbm_budget_bytes;  /* device bytes the server may hold (default 200e9) */
  uint64_t max_batch_photons; /* a launch closes once it holds this many photons (default 2e8) */
} pp_server_config;

typedef struct {
  double t_submit_s, t_launch_s, t_done_s; /* steady-clock seconds of one process-wide clock */
  uint64_t photons, n_hits;
  uint32_t batch_events;                    /* events in the launch that carried this request */
  uint32_t reserved;
} pp_request_info;

typedef struct {
  uint64_t submitted, completed, launches;
  uint64_t deferred;             /* admission rounds in which a waiting request did not fit the rings */
  uint64_t bytes_in_use;         /* queue bytes held by admitted requests (source records + queue entries) */
  uint64_t peak_bytes_in_use;    /*   and their peak */
  uint64_t photons_completed;
  uint64_t arena_bytes;          /* device bytes allocated at creation (rings, counters, hit buffers) */
  uint64_t overflow_bytes_peak;  /* largest temporary hit buffer of an overflowing launch (0: none) */
  uint64_t shared_requests;      /* requests that shared their launch with at least one other */
  uint64_t overlapped_launches;  /* launches enqueued while another launch was still running */
  double gpu_busy_s;             /* union of the launches' device intervals (HIP events) */
  double gpu_span_s;             /* from the first launch's start to the last one's end, same clock */
} pp_server_stats;

/* Device queue bytes a request of n_sources sources and n_photons photons
 * holds while admitted (its source records and work-queue entries, with
 * chunks of 256 photon ids): the admission cost. */
uint64_t pp_server_request_bytes(uint32_t n_sources, uint64_t n_photons);

/* Starts a server owning ctx (ice and geometry loaded; the caller must not
 * use ctx until pp_server_destroy) and allocates its device arena. cfg may be
 * NULL for defaults. If sur is not NULL, every request also gets the
 * surrogate's expected hits per module for its sources (Cherenkov sources
 * only), computed beside its Monte Carlo. PP_EBUDGET if the budget cannot
 * hold the smallest arena (about 10 KB per launch slot); PP_ENOMEM if the
 * arena cannot be allocated. */
pp_status pp_server_create(pp_context *ctx, const pp_server_config *cfg, pp_surrogate *sur, pp_server **out);

/* Drains all queued and running requests, then stops the scheduler and frees
 * the arena. */
void pp_server_destroy(pp_server *srv);

/* Thread-safe. Queues one request (an event: sources sharing one event id,
 * or any sources whose event ids are all distinct from other requests in
 * flight) and returns a ticket. PP_EBUDGET if it can never fit the queue
 * rings; PP_EINVAL on invalid sources (same validation as pp_submit). */
pp_status pp_server_submit(pp_server *srv, const pp_source *sources, uint32_t n, uint64_t *ticket);

/* Thread-safe. Blocks until the request is done, copies its hits to out
 * and, if dom_expected is not NULL and a surrogate is attached, n_doms
 * expected hits per module; fills *info; the ticket is then forgotten. If
 * the request has more than cap hits, returns PP_ETRUNC with info->n_hits
 * set and keeps the result, so the call can be repeated with a larger
 * buffer. PP_EINVAL for an unknown ticket, or one that another waiter has
 * collected meanwhile. */
pp_status pp_server_wait(pp_server *srv, uint64_t ticket, pp_hit *out, uint64_t cap, float *dom_expected,
                         pp_request_info *info);

/* Thread-safe snapshot of the counters. */
pp_status pp_server_get_stats(pp_server *srv, pp_server_stats *out);

/* Message of the last scheduler error (empty if none). */
const char *pp_server_last_error(pp_server *srv);

/* Load generator in native threads, so that a measurement sees the server
 * rather than the calling language's client loop. n_clients threads each
 * take the events c, c + n_clients, c + 2 n_clients, ... of events[] (one
 * source per event) in order and
 *   rate_per_s > 0 (open loop): submit them at exponentially distributed
 *     intervals of mean n_clients / rate_per_s seconds (random stream of
 *     client c: seed + c), collecting finished requests between arrivals;
 *   rate_per_s == 0 (closed loop): keep `outstanding` requests in flight,
 *     submitting the next event whenever the oldest one finishes;
 * until duration_s seconds have passed or the client's events run out, then
 * wait for everything outstanding. For each finished request, its latency
 * (submit to done, seconds) goes to latency_s (the first cap of them) and
 * its photons and hits are summed. *n_done, *photons_done, *hits_done and
 * *wall_s (start of the first client to end of the last) are set.
 * PP_EINVAL on zero clients, a closed loop with outstanding == 0, or NULL
 * outputs; the first failing request's status otherwise. */
pp_status pp_server_run_clients(pp_server *srv, const pp_source *events, uint64_t n_events, uint32_t n_clients,
                                double rate_per_s, uint32_t outstanding, double duration_s, uint64_t seed,
                                double *latency_s, uint64_t cap, uint64_t *n_done, uint64_t *photons_done,
                                uint64_t *hits_done, double *wall_s);

#ifdef __cplusplus
}
#endif

#endif /* PP_SERVER_H_ */
