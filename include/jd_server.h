/*
 * jd_server.h -- request server of libjd: continuous batching of many
 * gradient-iteration requests (the paper's Section 5, Algorithm 5.4 with the
 * stochastic Armijo rule, eq. Stochastic_Armijo; one request = one optimal
 * control problem with its own d, M, N, rate and seed) on one GPU.
 *
 * Device memory: the caller hands the server one device arena; every admitted
 * request's control, target, trajectory and workspace are carved out of it
 * (first fit, 256-byte aligned) and returned when the request completes.  A
 * request is admitted when a slot (max_active) and an arena extent of
 * jd_server_request_bytes() are free, in arrival order, with smaller requests
 * allowed to pass a larger one that does not fit yet.  The server allocates
 * no device memory; it creates n_streams HIP streams (default priority) and
 * max_active pinned host headers.
 *
 * Execution: admitted requests are spread over the streams; each request's
 * iteration runs the same kernels as jd_optimize (forward sweep, adjoint
 * sweep, reductions, Armijo trials on the same counters, the line search
 * decided on the device), so a request's result is bit-identical alone and in
 * any mix.  The server enqueues a few iterations of a request at a time and
 * looks at it again when they have completed.  jd_server_progress never
 * blocks: it advances every request whose last enqueued batch has completed
 * and admits queued requests.  A request that fails after it was queued
 * (admission, enqueueing, a device error) ends with that error as its status
 * and returns no control; its memory is reused only after its stream has
 * drained.
 *
 * Threading: one host thread drives a server.  Errors as in jd.h.
 */
#ifndef JD_SERVER_H
#define JD_SERVER_H

#include "jd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct jd_server jd_server;

/* Device bytes one request occupies while admitted (0 if invalid). */
size_t jd_server_request_bytes(const jd_problem* prob, const jd_run* run);

/* arena: device memory of arena_bytes (caller-owned, must outlive the
 * server); max_active >= 1 admitted requests at once; 1 <= n_streams <= 16. */
int jd_server_create(void* arena, size_t arena_bytes, int32_t max_active, int32_t n_streams,
                     jd_server** out);

/* Queue one request.  prob's host arrays and xd_host (host, N*d FP64; prob->xd
 * is ignored) and u0_host (host, N*d FP64, NULL = zeros) are copied; run->dump
 * must be NULL.  Returns JD_EWORKSPACE if the request can never fit the arena.
 * *ticket identifies the request. */
int jd_server_submit(jd_server* s, const jd_problem* prob, const double* xd_host,
                     const jd_run* run, const jd_opt* opt, const double* u0_host,
                     int64_t* ticket);

/* Non-blocking scheduling step: advances finished steps, admits queued
 * requests; reports the counts (each pointer may be NULL). */
int jd_server_progress(jd_server* s, int32_t* n_active, int32_t* n_queued, int64_t* n_completed);

/* Result of a finished request: final control (host, N*d), per-iteration log
 * (host, up to opt->n_max entries), iterations done, and the request's status
 * (JD_OK, JD_ELINESEARCH with u at the last accepted iterate, JD_ENONFINITE).
 * JD_EAGAIN while the request is not finished.  A result is returned once;
 * afterwards the ticket is unknown (JD_EINVAL). */
int jd_server_result(jd_server* s, int64_t ticket, double* u_host, jd_iter_log* log,
                     int32_t* iters, int32_t* status);

/* Times of a finished request in seconds on the server's host clock, while
 * its result has not been taken: *queued = admission - submission (all of its
 * time if it was never admitted), *service = completion - admission.  The
 * server sees a completion at the first jd_server_progress after the device
 * has finished, so both are as fine as the caller's polling.  JD_EAGAIN while
 * the request runs, JD_EINVAL for an unknown ticket; either pointer may be
 * NULL. */
int jd_server_times(jd_server* s, int64_t ticket, double* queued, double* service);

/* Waits for all streams, then frees the server (not the arena). */
int jd_server_destroy(jd_server* s);

#ifdef __cplusplus
}
#endif

#endif /* JD_SERVER_H */
