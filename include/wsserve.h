/*
 * wsserve -- request-serving engine over the wsconv apply and
 * Lippmann-Schwinger solver, for AMD Instinct MI355X (gfx950).
 *
 * Requests (applies of A_n, Section 2.1 eq. An, and Nystrom solves of the
 * Lippmann-Schwinger equation, Section 3.3 eq. descretls) of different grid
 * sizes and kernels arrive one at a time from any host thread.  The engine
 * keeps `streams` device streams busy: whenever a stream's worker is free it
 * takes the next job (continuous batching), which is
 *   - an apply together with up to max_batch - 1 other pending applies that
 *     share its plan (kernel, n, precision), run as one conv_apply launch
 *     (with mix_plans, also applies of other grid sizes and kernels whose
 *     plans are built, run as one conv_apply_multi launch), or
 *   - one LS solve, whose GMRES state stays on the device for the whole solve.
 * All device memory comes from one caller-owned arena: the built plans (kernel
 * moments and twiddles, cached and evicted least recently used first) and each
 * job's staging buffers and scratch.  A job is admitted only when its footprint
 * fits in the arena; younger jobs that fit may go ahead of one that does not,
 * a bounded number of times.  The engine never calls hipMalloc.
 *
 * Inputs and outputs are HOST arrays ([n][n], first index x1, as in wsconv.h),
 * always in FP64 / complex128 whatever the engine precision; page-locked
 * memory lets the copies run asynchronously.  The caller keeps a request's
 * arrays alive and unmodified until serve_wait reports it done.
 * With precision WS_FP32 an apply runs in FP32 (twiddles formed in FP64 and
 * rounded once to FP32) and an LS solve runs as FP32 GMRES with FP64
 * iterative refinement; with WS_FP64 both run in FP64.  Each result is the
 * same whether its request ran alone or batched with others: bitwise within
 * one plan's launches, and to rounding (the same arithmetic in another
 * kernel) when mix_plans joins plans.
 *
 * Calls that overlap on one engine are safe from several host threads.
 * Return codes are those of wsconv.h; conv_last_error() holds the message.
 */
#ifndef WSSERVE_H
#define WSSERVE_H

#include "wsconv.h"

#ifdef __cplusplus
extern "C" {
#endif

#define WS_REQ_APPLY 0
#define WS_REQ_LS    1

typedef struct {
    int precision;     /* WS_FP64 or WS_FP32 (see above) */
    int streams;       /* concurrent device streams, 1..16 (1 = one job at a time) */
    int max_batch;     /* applies sharing a plan merged into one launch, 1..1024 */
    int max_plans;     /* plans kept built in the arena, >= 1 */
    int max_skips;     /* times younger jobs may be admitted past the oldest blocked one, >= 0 */
    int mix_plans;     /* 1: applies with different plans (all real-kernel, or all Helmholtz) whose
                          plans are built share one conv_apply_multi launch; 0: same plan only */
} ws_serve_config;

typedef struct {
    int kind;                 /* WS_REQ_APPLY or WS_REQ_LS */
    ws_kernel kernel;         /* WS_REQ_LS: must be WS_HELMHOLTZ */
    int n;                    /* grid side, power of two in [16, 2048]; period b = 2, default a.  The
                                 density (LS: the contrast) must vanish beyond 0.39 of (1/2, 1/2),
                                 the support for which the default a is valid at b = 2 (Section 2.1) */
    const void* input;        /* host.  Apply: density, float64 (WS_LOG, WS_POWER) or complex128
                                 (WS_HELMHOLTZ).  LS: incident field u_inc, complex128 */
    const double* contrast;   /* host, LS only: m = 1 - mu, float64 [n][n] */
    void* output;             /* host, same element type as input (LS: the solution, complex128) */
    double tol;               /* LS: target true relative residual */
    int restart;              /* LS: GMRES restart length, 1..200 */
    int max_matvecs;          /* LS: bound on operator applications */
} ws_request;

typedef struct {
    int    status;     /* WS_OK; for LS also WS_LS_MAXIT / WS_LS_BREAKDOWN; < 0 on failure */
    int    batch;      /* requests served by the same launch */
    double t_submit;   /* engine clock (serve_now) at serve_submit */
    double t_start;    /* when its job was admitted to a stream */
    double t_done;     /* when its output was complete in host memory */
    ws_ls_info ls;     /* LS only */
} ws_result;

typedef struct {
    unsigned long long submitted, completed, launches, plan_builds, plan_evictions;
    size_t arena_bytes, arena_peak_bytes;
    int cached_plans, pending;
} ws_serve_stats;

/* Device bytes one request needs on its own (its plan, buffers and scratch);
 * serve_submit rejects a request above the arena size.  Host only. */
int serve_footprint(const ws_serve_config* cfg, const ws_request* req, size_t* bytes);

/* Create an engine over `arena` (device memory of the current HIP device,
 * 256-byte aligned, arena_bytes long, owned by the caller and untouched by it
 * until serve_destroy returns).  Starts one worker thread per stream. */
int serve_create(const ws_serve_config* cfg, void* arena, size_t arena_bytes, void** engine);

/* Queue a request; *ticket identifies it in serve_wait.  Checks the request on
 * the host (WS_EINVAL / WS_EUNSUPPORTED as conv_plan_query and ls_solve would,
 * or WS_EINVAL when its footprint exceeds the arena).  Never blocks on the GPU. */
int serve_submit(void* engine, const ws_request* req, unsigned long long* ticket);

/* Wait up to timeout_s seconds (< 0: no limit) for a request.  Returns 1 and
 * fills *out when it is done (each ticket is reported once), 0 on time-out,
 * WS_EINVAL for an unknown ticket. */
int serve_wait(void* engine, unsigned long long ticket, double timeout_s, ws_result* out);

/* Seconds on the engine clock (steady clock, zero at serve_create). */
double serve_now(void* engine);

int serve_stats(void* engine, ws_serve_stats* out);

/* Finish every queued request, stop the workers and release the plans.
 * Results not yet collected are discarded. */
void serve_destroy(void* engine);

#ifdef __cplusplus
}
#endif
#endif /* WSSERVE_H */
