/*
 * jacobi.h -- C ABI of libjacobi, a dense Jacobi solver for AMD Instinct
 * MI355X (gfx950).
 *
 * The method (Margaris, Souravlas & Roumeliotis, "Parallel implementations of
 * the Jacobi linear algebraic systems solver", sec. 2): for A X = B with
 * alpha_ii != 0, starting from X^0, repeat the sweep
 *
 *     x_i^(k) = ( beta_i - sum_{j != i} alpha_ij x_j^(k-1) ) / alpha_ii
 *
 * (the component equation of sec. 2; in matrix form X^(k) = T X^(k-1) + C
 * with T = D^-1 (L + U), C = D^-1 B) until the distance between consecutive
 * iterates falls below tol or the iteration cap L is reached (the serial
 * pseudocode of sec. 2).
 *
 * Conventions for every entry point:
 *   - Matrices are row-major with a leading dimension (elements, >= columns).
 *     A is n x n, B and X are n x k (k right-hand sides, k >= 1).
 *   - Unless stated otherwise, matrix and vector pointers are DEVICE pointers
 *     owned by the caller.  The library never keeps a pointer after the call
 *     returns.
 *   - Calls are synchronous with respect to the stream passed in: work is
 *     enqueued on that stream, the call waits for it, and outputs are valid on
 *     return.  A NULL stream is the device's null stream.
 *   - Errors are reported as return codes; no C++ exception crosses the ABI.
 *     jacobi_last_error() gives a thread-local message for the last failure.
 *   - Input validation happens before any sweep writes X: a validation error
 *     leaves X untouched.
 */
#ifndef JACOBI_H
#define JACOBI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* hipStream_t;

/* Entry points are the only symbols the shared library exports. */
#define JACOBI_API __attribute__((visibility("default")))

typedef enum {
    JACOBI_OK = 0,                   /* converged: distance < tol                      */
    JACOBI_NOT_CONVERGED = 1,        /* cap L reached (sec. 2, pseudocode step 3)      */
    JACOBI_DIVERGED = 2,             /* distance became NaN or Inf                     */
    JACOBI_PENDING = 3,              /* serving: not finished yet                      */
    JACOBI_CANCELLED = 4,            /* serving: server destroyed before completion    */
    JACOBI_ERR_INVALID_ARG = -1,     /* bad size, pointer, tolerance, cap or option    */
    JACOBI_ERR_ZERO_DIAGONAL = -2,   /* some alpha_ii == 0 (sec. 2); bad_index = i     */
    JACOBI_ERR_NONFINITE_INPUT = -3, /* NaN/Inf on the diagonal, in B or in X0         */
    JACOBI_ERR_OUT_OF_MEMORY = -4,   /* device workspace could not be allocated        */
    JACOBI_ERR_DEVICE = -5,          /* a HIP runtime call failed                      */
    JACOBI_ERR_REJECTED = -6,        /* serving: request can never fit the HBM budget  */
    JACOBI_ERR_INTERNAL = -7         /* unexpected internal failure                    */
} jacobi_status;

typedef enum {
    JACOBI_F64 = 0,   /* double                                      */
    JACOBI_F32 = 1,   /* float                                       */
    JACOBI_BF16 = 2   /* bfloat16 (upper half of a binary32), A only */
} jacobi_dtype;

typedef enum {
    JACOBI_NORM_INF = 0, /* max_i,c |x^(k) - x^(k-1)|                                  */
    JACOBI_NORM_L2 = 1   /* Euclidean distance over all n*k entries (sec. 2, sec. 3.1) */
} jacobi_norm;

typedef enum {
    JACOBI_MODE_PLAIN = 0,  /* Jacobi sweeps on A as given                                */
    JACOBI_MODE_REFINE = 1  /* FP64 system; sweeps on a reduced-precision copy of A inside
                               iterative refinement (residual and update in FP64)         */
} jacobi_mode;

/* Solver options.  Fill with jacobi_options_default() and change fields.
 *
 * PLAIN mode: stop after sweep k when distance_k < tol (strict, absolute;
 *   sec. 2 pseudocode step (b)), or after max_iter sweeps.  tol = 0 runs exactly
 *   max_iter sweeps (fixed-iteration mode).  max_iter = 0 returns X = X0.
 * REFINE mode (A, B, X in FP64): outer loop r = B - A x (FP64), stop when
 *   ||r||_2 < refine_tol * ||B||_2 (per system; a zero residual also stops);
 *   otherwise solve A_lo d = r by Jacobi sweeps on A_lo = round(A) in
 *   sweep_dtype (F32 or BF16) with FP32 accumulation, starting from d = 0 and
 *   stopping when max|d^(j) - d^(j-1)| <= inner_rel_tol * max|d^(j)| or after
 *   max_inner sweeps, then x += d in FP64.  At most max_outer corrections. */
typedef struct {
    double tol;             /* PLAIN: absolute threshold on the distance (default 1e-8)  */
    int32_t max_iter;       /* PLAIN: iteration cap L (default 10000)                     */
    int32_t norm;           /* jacobi_norm (default JACOBI_NORM_INF)                      */
    int32_t mode;           /* jacobi_mode (default JACOBI_MODE_PLAIN)                    */
    int32_t sweep_dtype;    /* REFINE: JACOBI_F32 or JACOBI_BF16 (default BF16)           */
    double inner_rel_tol;   /* REFINE: inner relative stop (default 1e-3)                 */
    int32_t max_inner;      /* REFINE: inner sweep cap per correction (default 200)       */
    int32_t max_outer;      /* REFINE: correction cap (default 50)                        */
    double refine_tol;      /* REFINE: ||r||_2 / ||B||_2 target (default 1e-12: the 2-norm
                               residual can understate the max-norm error by 10-20x at
                               n ~ 1e4, so 1e-12 is what keeps that error below 1e-10) */
    int32_t sync_every;     /* sweeps between host checks of the stop flag, 0 = adaptive  */
    int32_t profile;        /* 1: time every sweep kernel with HIP events (see info)      */
} jacobi_options;

typedef struct {
    int32_t status;           /* jacobi_status of this system                            */
    int32_t iterations;       /* sweeps executed (REFINE: inner sweeps, all corrections)  */
    int32_t outer_iterations; /* REFINE: residual evaluations; PLAIN: 0                  */
    int32_t kernel;           /* batched-kernel solves: bit 0 lockstep schedule, bit 6
                                 dataflow schedule (neither: planned), bit 1 deep shape
                                 (one workgroup per CU, else two), bits 2-4 XCD groups - 1
                                 (lockstep), bits 8-15 work items per workgroup (lockstep,
                                 dataflow), bits 16+ column chunks of a split single system
                                 (1 = none); plain single solves: 128 when every sweep ran in
                                 one launch of the small-system kernel, 129 when that was its
                                 register-resident variant, else 0                          */
    int64_t bad_index;        /* first offending row for ZERO_DIAGONAL / NONFINITE, or -1 */
    double final_delta;       /* distance of the last executed sweep (-1 if none)        */
    double rel_residual;      /* REFINE: last ||r||_2/||B||_2; PLAIN: -1                 */
    double device_ms;         /* device time of the whole call (HIP events)              */
    double sweep_kernel_ms;   /* profile=1: summed duration of the sweep kernels;
                                 batched-kernel solves: the persistent kernel's own
                                 duration (setup excluded), always                       */
    int64_t sweep_kernel_launches; /* number of sweep kernels timed (batched: 1)          */
} jacobi_info;

typedef struct jacobi_ctx jacobi_ctx;

/* Fill *opt with the defaults above (the paper's experiment values tol = 1e-8
 * and L = 10000, sec. 4). */
JACOBI_API void jacobi_options_default(jacobi_options* opt);

/* Create a context bound to HIP device `device`: it owns device workspaces
 * (iterate ping-pong buffer, diagonal, stop-flag block) reused across calls.
 * Calls on one context are serialised by an internal lock.  Returns
 * JACOBI_ERR_INVALID_ARG for a bad device or NULL out. */
JACOBI_API jacobi_status jacobi_ctx_create(int32_t device, jacobi_ctx** out);
JACOBI_API jacobi_status jacobi_ctx_destroy(jacobi_ctx* ctx);

/* Solve A X = B (sec. 2) for one dense system with k right-hand sides.
 *
 * ctx      context, or NULL for the per-device default context of the current device
 * n, k     system size and number of right-hand sides (n >= 1, k >= 1)
 * a_dtype  element type of A.  PLAIN: F64 => B, X0, X are double; F32 or BF16 =>
 *          B, X0, X are float (BF16 A is widened to FP32, FP32 accumulation).
 *          REFINE: must be F64 (A, B, X0, X double).
 * A, lda   device matrix n x n, row-major, lda >= n
 * B, ldb   device n x k, ldb >= k
 * X0       device n x k initial approximation (leading dim ldx), NULL => zero;
 *          may alias X
 * X, ldx   device n x k output, ldx >= k
 * opt      options, NULL => defaults
 * stream   HIP stream of the caller (work is enqueued there; the call waits)
 * info     optional host pointer receiving the outcome
 *
 * Returns the solve status (also info->status): OK, NOT_CONVERGED, DIVERGED,
 * or an error.  On OK, X holds the iterate whose distance to its predecessor
 * met the test; on NOT_CONVERGED, X^(L); on DIVERGED, the last (non-finite)
 * iterate. */
JACOBI_API jacobi_status jacobi_solve(jacobi_ctx* ctx, int64_t n, int64_t k,
                                      int32_t a_dtype, const void* A, int64_t lda,
                                      const void* B, int64_t ldb, const void* X0, void* X,
                                      int64_t ldx, const jacobi_options* opt,
                                      hipStream_t stream, jacobi_info* info);

/* ---------------------------------------------------------------------------
 * Prepared matrices: one A solved repeatedly with new right-hand sides (the
 * sec. 2 iteration on each).  jacobi_matrix_create keeps the caller's device
 * pointer A (n x n, leading dimension lda; not copied: A must stay alive and
 * unchanged until jacobi_matrix_destroy) and, with lo_dtype = JACOBI_F32 or
 * JACOBI_BF16 (FP64 A only), builds once, in the handle's own device memory,
 * the reduced-precision copy A_lo (round to nearest even) and its diagonal
 * that REFINE solves would otherwise build on every call; lo_dtype = -1
 * builds nothing.  It waits for `stream`.  Errors: INVALID_ARG (n < 1,
 * lda < n, null A, bad dtype, a reduced copy of a non-FP64 A), OUT_OF_MEMORY,
 * DEVICE; *out is then null.  The handle is bound to ctx (NULL: the default
 * context) and its device. */
typedef struct jacobi_matrix jacobi_matrix;

JACOBI_API jacobi_status jacobi_matrix_create(jacobi_ctx* ctx, int64_t n, int32_t a_dtype,
                                              const void* A, int64_t lda, int32_t lo_dtype,
                                              hipStream_t stream, jacobi_matrix** out);

/* jacobi_solve on the prepared A: the same arguments, checks, results (bitwise)
 * and errors as jacobi_solve(ctx, n, k, a_dtype, A, lda, B, ...).  REFINE
 * needs opt->sweep_dtype equal to the prepared lo_dtype (else INVALID_ARG) and
 * then sweeps the prepared copy: no conversion pass over A. */
JACOBI_API jacobi_status jacobi_solve_prepared(jacobi_matrix* m, int64_t k, const void* B,
                                               int64_t ldb, const void* X0, void* X, int64_t ldx,
                                               const jacobi_options* opt, hipStream_t stream,
                                               jacobi_info* info);

/* Free the handle and its device memory (NULL: no-op).  No solve on it may be
 * running. */
JACOBI_API jacobi_status jacobi_matrix_destroy(jacobi_matrix* m);

/* One system of a batch (device pointers; same conventions as jacobi_solve). */
typedef struct {
    int64_t n, k;       /* size and right-hand sides (k <= 32)                     */
    const void* A;      /* n x n, leading dimension lda                            */
    int64_t lda;
    const void* B;      /* n x k, leading dimension ldb                            */
    int64_t ldb;
    const void* X0;     /* n x k initial approximation (ldx), NULL => zero         */
    void* X;            /* n x k output, leading dimension ldx                     */
    int64_t ldx;
} jacobi_system;

/* Solve `count` independent systems (sec. 2 iteration on each) with one
 * persistent launch.  a_dtype F64: A, B, X0, X double, FP64 MFMA tiles
 * (v_mfma_f64_16x16x4f64, FP64 accumulation); F32 or BF16: A as given,
 * B/X0/X float, FP32 MFMA tiles with FP32 accumulation.  Every system has
 * k <= 32 (others get JACOBI_ERR_INVALID_ARG).  Three schedules run the same
 * row sweep and give bitwise the same X: lockstep (round r is sweep r of every
 * system still running, its rows dealt out to all workgroups as work items,
 * one device-wide barrier per round), dataflow (no rounds: a system's next
 * sweep is queued as work items the moment the last item of its current
 * sweep finishes) and planned (large systems split over workgroups that meet
 * at per-system barriers, small ones taken whole from a queue).  The first
 * batch of a kind is timed on the candidates and the fastest is kept (in the
 * context and a per-user cache file); JACOBI_BATCHED_SCHED = lockstep |
 * dataflow | planned forces one.  Every system stops on its own (opt->tol /
 * opt->max_iter, PLAIN mode only, INF or L2 distance over its n*k entries).
 *
 * systems, infos: host arrays of `count` entries.  Returns JACOBI_OK when the
 * launch ran (per-system outcomes in infos[i].status; a system with bad
 * arguments gets JACOBI_ERR_INVALID_ARG and is skipped), or an error for the
 * whole call (bad options, device failure).  Results depend only on each
 * system's own data: a system gives bitwise the same X alone and in a batch. */
JACOBI_API jacobi_status jacobi_solve_batched(jacobi_ctx* ctx, int32_t count,
                                              const jacobi_system* systems, int32_t a_dtype,
                                              const jacobi_options* opt, hipStream_t stream,
                                              jacobi_info* infos);

/* ---------------------------------------------------------------------------
 * Serving: a request loop that solves FP64 systems as they arrive, with
 * continuous batching.  Each request is solved by iterative refinement (the
 * REFINE mode above): FP64 residual on the device, inner Jacobi sweeps on a
 * reduced-precision copy of A.  A worker thread admits queued requests while
 * their device footprint fits the HBM budget and an active slot is free,
 * copies A and B to the device on a copy stream (overlapping the sweeps of
 * requests already admitted), and steps all active requests together: one
 * step = one FP64 residual pass per request, then one persistent batched
 * launch running every request's inner solve.  Requests that meet their
 * tolerance (or fail) are copied back and retired at once, freeing memory for
 * the next ones.  A request's result does not depend on the other requests in
 * flight (bitwise the same alone and in the mix). */

typedef struct {
    int32_t device;            /* HIP device                                                  */
    int32_t max_active;        /* requests stepped together (default 64)                      */
    uint64_t hbm_budget_bytes; /* device memory for request state, 0 = 80% of free memory     */
    int32_t inner_max;         /* inner sweep cap per refinement step (default 64)            */
    int32_t max_outer;         /* refinement steps per request (default 50)                   */
    double inner_rel_tol;      /* inner relative stop (default 1e-3)                          */
} jacobi_serve_config;

typedef struct {
    int64_t n, k;              /* size, right-hand sides (k <= 32)                            */
    const double* A;           /* HOST n x n FP64, leading dimension lda (pinned is faster)   */
    int64_t lda;
    const double* B;           /* HOST n x k FP64, leading dimension ldb                      */
    int64_t ldb;
    double* X;                 /* HOST n x k FP64 output, leading dimension ldx               */
    int64_t ldx;
    int32_t sweep_dtype;       /* JACOBI_F32 or JACOBI_BF16 inner sweeps                      */
    int32_t max_outer;         /* refinement steps for this request (0 = the server's
                                  max_outer); NOT_CONVERGED once it is exceeded             */
    double rel_tol;            /* stop when ||r||_2 < rel_tol * ||B||_2                       */
} jacobi_request;

typedef struct {
    uint64_t submitted, completed, rejected, failed, active, queued;
    uint64_t hbm_in_use, hbm_peak, steps;
    double solves_per_s;       /* completed / (last completion - first submission)           */
    double p50_ms, p99_ms;     /* end-to-end latency: submission -> result in host memory    */
    double p50_device_ms, p99_device_ms; /* data on the device -> result ready on the device  */
    double elapsed_s;
} jacobi_serve_stats;

typedef struct jacobi_server jacobi_server;

/* Fill *cfg with the defaults above. */
JACOBI_API void jacobi_serve_config_default(jacobi_serve_config* cfg);

/* Start a server (its worker thread, streams and context) on cfg->device. */
JACOBI_API jacobi_status jacobi_serve_create(const jacobi_serve_config* cfg, jacobi_server** out);

/* Queue a request; returns at once with a ticket.  The caller keeps req->A,
 * req->B and req->X alive and unchanged until the ticket completes.  A request
 * whose footprint can never fit the budget returns JACOBI_ERR_REJECTED (and a
 * ticket that polls as rejected); bad sizes return JACOBI_ERR_INVALID_ARG. */
JACOBI_API jacobi_status jacobi_serve_submit(jacobi_server* srv, const jacobi_request* req,
                                             uint64_t* ticket);

/* Outcome of a ticket: JACOBI_PENDING while queued or running, else its final
 * status (info filled: iterations = inner sweeps, outer_iterations,
 * rel_residual, device_ms = device latency). */
JACOBI_API jacobi_status jacobi_serve_poll(jacobi_server* srv, uint64_t ticket, jacobi_info* info);

/* Block until the ticket completes or timeout_us passes (< 0: no timeout);
 * returns JACOBI_PENDING on timeout. */
JACOBI_API jacobi_status jacobi_serve_wait(jacobi_server* srv, uint64_t ticket,
                                           int64_t timeout_us, jacobi_info* info);

JACOBI_API jacobi_status jacobi_serve_stats_get(jacobi_server* srv, jacobi_serve_stats* stats);

/* Stop the worker; requests not finished complete as JACOBI_CANCELLED (their X
 * untouched).  Frees every device buffer of the server. */
JACOBI_API jacobi_status jacobi_serve_destroy(jacobi_server* srv);

/* Size of the fixed per-device workspace of jacobi_solve_noalloc (bytes). */
#define JACOBI_NOALLOC_MAX_BYTES (24u << 20)

/* jacobi_solve without any allocation, for callers that cannot allocate device
 * memory (code that must not call hipMalloc: tight serving loops, harnesses
 * that forbid the allocator).  Same arguments, conventions and results as
 * jacobi_solve in PLAIN mode on the current HIP device, restricted to the
 * vector sweep path: k <= 2 right-hand sides, opt->mode = PLAIN,
 * opt->profile = 0 (other values: JACOBI_ERR_INVALID_ARG).  X, the count and
 * the distance are bitwise those of jacobi_solve for the same input.
 *
 * Workspace: one fixed device array per device (JACOBI_NOALLOC_MAX_BYTES,
 * allocated with the library's code object and held until the process
 * ends), which must hold the control block, the reduction slots, 1.5 MiB of
 * partial sums, the diagonal (n elements) and two iterate buffers (n x kp,
 * kp = k rounded up to a power of two), each rounded up to 256 bytes, with
 * 8-byte elements for F64 and 4-byte for F32/BF16; a larger n * k returns
 * JACOBI_ERR_INVALID_ARG with the sizes in jacobi_last_error() before any
 * device work (F64, k = 1: n up to about 980000; k = 2: about 590000).  Every call on a device
 * uses that device's one array, and the library serialises such calls with
 * a per-device lock; work of a call is complete when it returns (it waits on
 * `stream`), so it cannot be captured into a graph.  Calls that overlap on
 * one device by other means (another copy of the library in the same
 * process) would race.  info->device_ms is -1 (no events are created). */
JACOBI_API jacobi_status jacobi_solve_noalloc(int64_t n, int64_t k, int32_t a_dtype,
                                              const void* A, int64_t lda, const void* B,
                                              int64_t ldb, const void* X0, void* X,
                                              int64_t ldx, const jacobi_options* opt,
                                              hipStream_t stream, jacobi_info* info);

/* Release the per-device default contexts (the ctx = NULL workspaces: device
 * buffers, pinned staging memory, events), after waiting for the device.
 * Meant for process teardown, before the HIP runtime shuts down (the Python
 * binding calls it from an interpreter exit hook, after closing its servers
 * and contexts).  Contexts made by jacobi_ctx_create and servers are not
 * touched: destroy them first.  Must not run concurrently with a call that
 * uses a default context.  A later call with ctx = NULL creates a new default
 * context.  Returns JACOBI_OK. */
JACOBI_API jacobi_status jacobi_shutdown(void);

/* Achievable HBM read bandwidth (a measurement utility, beside the 8 TB/s
 * published peak): streams the device buffer buf (bytes, 16-byte aligned,
 * on the current device; not modified) with 16-byte non-temporal loads,
 * the load width of the sweep's stream of A, in a grid-stride read-only
 * kernel at 2, 4, 8 and 16 workgroups of 256 threads per CU, reps timed
 * launches each (HIP events on `stream`, one untimed launch before), and
 * returns the fastest rate in *gbps (bytes / time / 1e9) and its workgroups
 * per CU in *wg_per_cu (may be null).  Waits for the stream.  Use a buffer
 * larger than the caches (the 256 MB MALL): 1 GiB gives the HBM rate. */
JACOBI_API jacobi_status jacobi_stream_probe(const void* buf, int64_t bytes, int32_t reps,
                                             hipStream_t stream, double* gbps,
                                             int32_t* wg_per_cu);

/* Human-readable name of a status code (static string). */
JACOBI_API const char* jacobi_status_string(int32_t status);

/* Thread-local description of the last error raised in this thread ("" if none). */
JACOBI_API const char* jacobi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* JACOBI_H */
