/*
 * mi_server.h -- a request loop that serves all-pairs MI requests on one GPU
 * with continuous batching (the operation itself is the one of mi.h: binary
 * MI of every column pair, paper Section 1 Eq. 1, computed as in Sections 2-3).
 *
 * A server owns a host thread and a small pool of HIP streams ("slots").
 * Clients submit requests whose data already lives on the device; the server
 *   - admits waiting requests in arrival order while a slot is free and the
 *     memory of everything in flight stays within the HBM budget,
 *   - launches the requests admitted together as one batch on a free slot:
 *     a few small requests as plain launches back to back, many as one
 *     persistent launch pulling work units of all of them, a large request
 *     alone, so work of newly admitted requests runs on the device next to
 *     requests that are still running,
 *   - sizes batches by an estimate of each request's device time: a large
 *     request (about 250 us or more alone) runs by itself; with two or more
 *     slots, slot 0 runs large requests one at a time and the other slots
 *     run batches of small requests (up to about 400 us of summed work);
 *     small requests may start before a large request that waits for slot
 *     0, but a request that waits for budget is never overtaken,
 *   - detects completion with events (per request for plain launches, per
 *     batch for a persistent launch) and records each request's latency from
 *     submission to completion.
 * A request's results are bitwise the same whether it runs alone or in a
 * batch (counts are exact integers and MI is a pure function of them).
 *
 * Memory charged to a request: X (m * ldx bytes), out (4 n^2), the optional
 * outputs, and the library scratch it needs (split-K workspace; the FP4 copy
 * of X, m * ceil(n / 2) bytes with the pitch rounded up to 16, when the
 * request runs the FP4 Gram (mi_problem.gram); otherwise a repacked copy of X
 * when its layout is not 16-byte aligned).  Requests take the byte layout.
 *
 * Thread safety: submit, poll and wait may be called from any thread.  The
 * caller keeps X and the outputs alive until the ticket has completed.
 */
#ifndef MI_SERVER_H_
#define MI_SERVER_H_

#include <stddef.h>
#include <stdint.h>

#include "mi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mi_server mi_server;

/* Create a server on the current device.  hbm_budget_bytes: cap on the memory
 * of all admitted, unfinished requests (> 0).  max_slots: concurrent batches
 * (streams), 1..64.  max_queue: bound on waiting requests (0 = 65536). */
mi_status mi_server_create(mi_server** server, size_t hbm_budget_bytes, int32_t max_slots, int32_t max_queue);

/* Submit a request (copied; validate must be 0).  Non-blocking.
 * MI_ERR_BUDGET if the request alone exceeds the budget, MI_ERR_QUEUE_FULL if
 * the waiting queue is full, MI_ERR_INVALID_ARG for a bad problem. */
mi_status mi_server_submit(mi_server* server, const mi_problem* p, uint64_t* ticket);

/* MI_OK if the ticket has completed (its outputs are ready), MI_ERR_NOT_READY
 * if not, MI_ERR_UNKNOWN_TICKET if it was never issued or already collected. */
mi_status mi_server_poll(mi_server* server, uint64_t ticket);

/* Block until the ticket completes or timeout_s seconds pass (<= 0: no limit).
 * On MI_OK, *latency_s (may be NULL) receives submission-to-completion time
 * and the ticket is collected.  MI_ERR_TIMEOUT leaves the ticket pending; a
 * request that failed on the device returns its error and is collected. */
mi_status mi_server_wait(mi_server* server, uint64_t ticket, double timeout_s, double* latency_s);

/* Counters since creation. */
typedef struct mi_server_stats {
  uint64_t submitted, completed, rejected, batches;
  uint64_t max_in_flight;        /* most requests admitted at once */
  size_t max_bytes_in_flight;    /* most budget in use at once */
  size_t bytes_in_flight;        /* budget in use now */
} mi_server_stats;
mi_status mi_server_get_stats(mi_server* server, mi_server_stats* stats);

/* Finish all submitted requests, stop the loop and free the server. */
mi_status mi_server_destroy(mi_server* server);

#ifdef __cplusplus
}
#endif

#endif /* MI_SERVER_H_ */
