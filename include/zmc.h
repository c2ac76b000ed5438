/*
 * zmc.h -- C ABI of the MI355X (gfx950) multi-function direct Monte Carlo library.
 *
 * The operation (paper: "Multi-function Integrations" and "Solution method"):
 * many integrands, each with its own form, dimension (1..12) and box domain
 * (Eq. (1): a cos(k.x) + b sin(k.x); Eq. (2): |x1+x2|, |x1+x2-x3|; plus
 * Gaussian and product-polynomial forms), are each integrated by direct Monte
 * Carlo: N uniform samples x_i in the box give
 *
 *     F_hat = V * (1/N) * sum f(x_i),   V = prod_j (hi_j - lo_j),
 *     SE    = V * sqrt(s^2 / N),        s^2 = (sum f^2 - (sum f)^2 / N) / (N - 1),
 *
 * a value with an error bar for every integral (Fig. 1 caption).  Samples are
 * counter-based and taken four at a time: coordinate j of sample i of a
 * d-dimensional function with seed s is output word i mod 4 of the
 * Philox4x32-10 block with key (s mod 2^32, s >> 32) and counter
 * (b mod 2^32, b >> 32, 0, 0), b = (i / 4) * d + j; the word r becomes
 * u = (2*(r mod 2^23) + 1) * 2^-24 and x_j = lo_j + (hi_j - lo_j) * u.  A
 * function's result therefore depends only on its own description, never on
 * the rest of the batch, the launch shape or the tuning.
 *
 * Conventions for every entry point:
 *   - Return an mc_status; nothing throws across the boundary.  On failure
 *     mc_last_error(ctx) holds a message (thread-local when ctx is NULL).
 *   - Host arrays (mc_function[], mc_result[]) are caller-owned; the library
 *     copies what it needs before returning.
 *   - `stream` arguments are hipStream_t values passed as void* (NULL = the
 *     null stream).  Work is enqueued asynchronously on that stream.
 *   - A context is externally synchronized: one thread at a time.
 *   - Testing aid for the error paths: MC_FAULT_HIP=n in the environment when a
 *     context is created makes the n-th checked HIP runtime call the library
 *     makes from then on report failure without being made (out of memory for
 *     allocations, hipErrorUnknown otherwise), once; every mc_create re-arms
 *     the countdown from the variable or, without it, disarms it.
 *   - Log level: MC_LOG in the environment when a context is created sets what
 *     the library writes to stderr, one line per event prefixed "[zmc] ":
 *     0 or unset nothing; 1 every failure an entry point returns, with its
 *     message; 2 also context creation, resident-kernel launches and stops,
 *     tuning choices and promotions to FP64; 3 also every launch and every
 *     admitted request.  Logging never changes a result.
 */
#ifndef ZMC_H
#define ZMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MC_MAX_DIM 12
#define MC_N_PARAMS 32

typedef enum {
    MC_OK = 0,
    MC_NOT_READY = 1,              /* results not finished yet (non-blocking query) */
    MC_ERR_INVALID_ARG = -1,       /* NULL pointer, n_samples < 2, bad config field */
    MC_ERR_UNSUPPORTED_FAMILY = -2,
    MC_ERR_BAD_DIM = -3,           /* dim outside 1..12 */
    MC_ERR_BAD_BOUNDS = -4,        /* lo/hi not finite or lo >= hi */
    MC_ERR_BAD_PARAMS = -5,        /* non-finite parameter, sigma <= 0, bad degree */
    MC_ERR_OUT_OF_MEMORY = -6,     /* device or pinned allocation failed (any HIP call returning out of memory) */
    MC_ERR_ADMISSION = -7,         /* request can never fit the context's capacity */
    MC_ERR_HIP = -8,               /* a HIP runtime call failed (message has the HIP string) */
    MC_ERR_NO_DEVICE = -9,         /* no usable gfx950 device, or device call on a validate-only context */
    MC_ERR_ABORTED = -10,          /* work stopped by mc_abort before it finished */
    MC_ERR_UNKNOWN_REQUEST = -11,  /* request id never issued or results already taken */
    MC_ERR_COMPILE = -12           /* a run-time family did not compile (log in mc_last_error) */
} mc_status;

typedef enum {
    MC_FAMILY_HARMONIC = 0,      /* f = a cos(k.x) + b sin(k.x)         params: a, b, k[0..d)     (Eq. 1) */
    MC_FAMILY_ABS_LINEAR = 1,    /* f = a |c0 + c.x|                    params: a, c0, c[0..d)    (Eq. 2) */
    MC_FAMILY_GAUSSIAN = 2,      /* f = A exp(-|x - mu|^2 / (2 s^2))    params: A, s, mu[0..d)          */
    MC_FAMILY_POLY_PRODUCT = 3,  /* f = prod_j (1 + p_j x_j^{n_j})      params: -, -, p[0..d), n[0..d)  */
    MC_FAMILY_USER0 = 16         /* first id handed out by mc_register_family (16 .. 16 + 7)           */
} mc_family;

#define MC_MAX_USER_FAMILIES 8

/* Parameter layout inside mc_function.params: params[0], params[1] are the two
 * scalars; params[2 + j] is the first per-dimension vector (k, c, mu or p) and
 * params[14 + j] the second (POLY_PRODUCT degrees n_j, integers 0..8 stored as
 * doubles).  Unused entries are ignored but must be finite. */
#define MC_PARAM_V0 2
#define MC_PARAM_W0 14

typedef enum {
    MC_PREC_FP32_EVAL = 0,   /* FP32 sample mapping and evaluation, per-lane compensated FP32 sums,
                                FP64 cross-lane reduction, variance and finalize.  A function FP32
                                cannot resolve is re-run in FP64 and its result says so: spread too
                                small (sigma / rms below 400 * 2^-24 * sqrt(N)), values or squares
                                out of FP32 range (non-finite sums: |f| beyond about 2^60; mean
                                square below 2^-120 or zero: |f| below about 2^-60).  An Eq. (1)
                                function whose phase bound 1 + 2 sum_j |k_j| (hi_j - lo_j) / 2 pi
                                exceeds 4096 revolutions, and a product-polynomial or run-time-family
                                function (which sees x in FP32 absolute coordinates) with
                                K sqrt(N) > 24200, K = max_j max(|lo_j|, |hi_j|) / (hi_j - lo_j), are
                                evaluated in FP64 from the start (for a parameter grid: the whole grid,
                                if any point exceeds it), as is every function of N >= 1.8e9, which the
                                sigma / rms check would always send to FP64. */
    MC_PREC_FP64 = 1         /* FP64 evaluation in the reference operation order, FP64 sums */
} mc_precision;

/* One integrand (472 bytes, no padding). */
typedef struct mc_function {
    uint32_t family;             /* mc_family */
    uint32_t dim;                /* 1..MC_MAX_DIM */
    uint64_t n_samples;          /* N >= 2, at most 2^40 */
    uint64_t seed;               /* Philox key = (seed mod 2^32, seed >> 32) */
    double lo[MC_MAX_DIM];       /* box, entries >= dim ignored */
    double hi[MC_MAX_DIM];
    double params[MC_N_PARAMS];
} mc_function;

/* One result (48 bytes). */
typedef struct mc_result {
    double mean;                 /* F_hat */
    double std_error;            /* SE */
    double sum_f;                /* S1 = sum f(x_i) */
    double sum_f2;               /* S2 = sum f(x_i)^2 */
    uint64_t n;                  /* N */
    int32_t status;              /* MC_OK, MC_ERR_ABORTED, or MC_ERR_HIP if the launch's records failed the
                                    kernels' checks or the result's precision disagrees with its schedule */
    uint32_t precision;          /* mc_precision the result was computed in */
} mc_result;

/* Context flags. */
#define MC_VALIDATE_ONLY 0x1u    /* host-only context: mc_submit validates and packs, no device is touched */
#define MC_NO_GRAPH 0x2u         /* launch kernels directly instead of replaying captured HIP graphs */
#define MC_NO_PROMOTE 0x4u       /* evaluate every function of an FP32 request in FP32: no FP64 re-runs and no
                                    FP64 choice at submit (unresolvable integrands come back as FP32 gave them) */
#define MC_RESIDENT 0x8u         /* serve through one resident kernel instead of launches: see "Resident
                                    contexts" below */

typedef struct mc_config {
    int32_t device;              /* HIP device ordinal */
    uint32_t flags;              /* MC_VALIDATE_ONLY | MC_NO_GRAPH | MC_NO_PROMOTE | MC_RESIDENT */
    uint32_t max_functions;      /* device function slots, at most 2^24 (0: 1 << 16); each also takes
                                    1 KiB of pinned host memory (the packed-record mirror) */
    uint32_t max_tiles_per_run;  /* tiles one mc_run may launch, at most 2^28; the rest waits (0: 1 << 20).
                                    MC_RESIDENT: tiles that may wait unread in the ring (0: two per workgroup) */
    uint64_t max_partials;       /* device tile-partial slots, 16 bytes each, at most 2^32 - 1 (0: 1 << 22) */
    uint64_t mem_budget_bytes;   /* upper bound on device memory the context holds (0: no bound) */
    void* workspace;             /* optional caller-owned device memory for every device buffer */
    uint64_t workspace_bytes;    /* its size; see mc_workspace_size */
    uint32_t blocks_per_cu;      /* persistent-kernel workgroups per CU (0: tuned/default) */
    uint32_t policy;             /* MC_SCHED_FAIR (0), MC_SCHED_FIFO or MC_SCHED_SRPT: how mc_run shares a launch */
} mc_config;

/* Scheduling policies for the tiles of one launch (results never depend on them). */
#define MC_SCHED_FAIR 0u  /* every active request gets an equal share of the launch (small requests finish fast) */
#define MC_SCHED_FIFO 1u  /* fill the launch from the oldest request on */
#define MC_SCHED_SRPT 2u  /* fill the launch from the request with the least remaining work on (estimated
                             evaluation cost of its tiles not yet launched); ties go to the older request.
                             Shortest waits below saturation; under sustained overload the largest requests
                             can wait indefinitely (FAIR bounds every request's share) */

typedef struct mc_ctx mc_ctx;

/* Fill *cfg with defaults (device 0, everything else 0). */
mc_status mc_config_init(mc_config* cfg);

/* Device bytes a context created from *cfg needs (so a caller can pass its own workspace). */
mc_status mc_workspace_size(const mc_config* cfg, uint64_t* bytes);

/* Create a context on cfg->device.  Allocates the function table, tile-partial
 * arena, staging buffers and (unless MC_NO_GRAPH) captures the launch graphs.
 * With MC_VALIDATE_ONLY nothing touches a device.  Paper, "Solution method":
 * the integrations run on the GPU; a context is the device state (one GPU)
 * that every later call of the path uses.  *out is owned by the caller until
 * mc_destroy.  Errors: MC_ERR_INVALID_ARG (NULL or out-of-range config field),
 * MC_ERR_NO_DEVICE, MC_ERR_OUT_OF_MEMORY, MC_ERR_HIP; nothing is left
 * allocated on failure. */
mc_status mc_create(const mc_config* cfg, mc_ctx** out);

/* Wait for the context's outstanding work and free everything it owns. */
mc_status mc_destroy(mc_ctx* ctx);

/* Validate and queue n functions as one request evaluated in `precision`.
 * Paper, "Multi-function Integrations" (Eq. (1), Eq. (2)): a batch of
 * integrands that differ in form, dimension and domain, each one row of the
 * caller's table (family, dim, params, box, n_samples, seed).
 * The whole request is rejected on the first invalid function (its index is in
 * mc_last_error); nothing partial is queued.  Requests are admitted to the device
 * in submission order as function slots and partial memory free up (at submit
 * if they fit, else in a later mc_run).  Admission packs the table into pinned
 * host memory; with no launch in flight it is uploaded at once on the library's
 * own upload stream, otherwise each record goes up with the stage kernel of the
 * first launch that runs that function.  A request that could never fit returns
 * MC_ERR_ADMISSION.  *out_request_id identifies it.  Once validated the request
 * is queued: if a HIP call of the admission tried at submit fails, the request
 * stays queued, unadmitted, and the next mc_run tries again (and reports a
 * failure that persists). */
mc_status mc_submit(mc_ctx* ctx, const mc_function* fns, size_t n, int32_t precision,
                    uint64_t* out_request_id);

/* One axis of a parameter grid: point k (0 <= k < count) sets
 * params[param] = start + (double)k * step (the product rounded, then the sum). */
typedef struct mc_grid_axis {
    uint32_t param;              /* index into mc_function.params, 0..31 */
    uint32_t count;              /* points on this axis, >= 1 */
    double start;
    double step;
} mc_grid_axis;

#define MC_MAX_GRID_AXES 4

/* Submit one integrand form over a Cartesian grid of parameter values, as one
 * request (the paper's functional mode: a single integrand with a large
 * parameter space, program summary, "Solution method" and "Additional
 * comments").  Function i, 0 <= i < prod_a count_a, is `base` with each axis's
 * parameter set to its point k_a, where (k_0, k_1, ...) are the mixed-radix
 * digits of i with axis 0 varying fastest, and seed = base->seed + i (so with
 * base seed (b << 32) function i draws the stream (b << 32) | i).  Every
 * function is validated as in mc_submit (first failing index in mc_last_error);
 * results come back in order i through mc_results.  Errors: as mc_submit, plus
 * MC_ERR_INVALID_ARG for n_axes outside 1..MC_MAX_GRID_AXES, a param index
 * above 31, two axes on one parameter, a zero count, or a seed range that would
 * wrap 2^64. */
mc_status mc_submit_grid(mc_ctx* ctx, const mc_function* base, const mc_grid_axis* axes, uint32_t n_axes,
                         int32_t precision, uint64_t* out_request_id);

/* Paper, "Solution method": direct Monte Carlo of every admitted function on
 * the GPU (uniform samples in its box, sum f and sum f^2 per function).
 * Admit what fits, then enqueue one launch of the batched path on `stream`, as
 * kernels only: a stage kernel that copies the launch's work list (and the
 * records of functions admitted or promoted while launches were in flight) from
 * pinned host memory, preceded by the record-building kernel of any parameter
 * grid admitted under load, the persistent kernels over the admitted (function,
 * sample-segment) tiles, a finalize kernel for every function whose last tile
 * is in this launch, and a publish kernel that writes those results to pinned
 * host memory and then marks the launch done.  Returns without waiting (the
 * library reads completion from that mark, not from the stream).  Launches
 * nothing and returns MC_OK when no admitted work is pending, or MC_NOT_READY
 * when all launch slots are still in flight (call again later).  The stream
 * must stay valid until the launch has completed.  MC_ERR_HIP /
 * MC_ERR_OUT_OF_MEMORY: a HIP call failed; what happens to the launch being
 * built is described at mc_results. */
mc_status mc_run(mc_ctx* ctx, void* stream);

/* Ids of requests that completed since the previous call (their results can be
 * taken without waiting): up to `cap` ids into completed[], the count in *n. */
mc_status mc_poll(mc_ctx* ctx, uint64_t* completed, size_t cap, size_t* n);

/* Number of requests submitted but not yet complete, and tiles still waiting for a launch. */
mc_status mc_pending(mc_ctx* ctx, uint64_t* requests, uint64_t* tiles);

/* Paper, Fig. 1 caption and "Solution method": each integral comes back as a
 * value with an error bar -- mean V * S1 / N and standard error
 * V * sqrt((S2 - S1^2 / N) / ((N - 1) N)) (mc_result, with S1, S2, N and the
 * precision used).
 * Copy the n results of a request into out (n must equal the request size).
 * blocking = 0: MC_NOT_READY if the request is not finished (runs are still
 * needed, or launched work has not completed).  blocking != 0: calls mc_run on
 * the null stream as needed and waits.  Results can be taken once; the
 * request's device resources are released when it completes.
 * After an mc_run that failed with MC_ERR_HIP: if the failure came before the
 * launch's finalize kernel was handed to the stream, the launch is taken back
 * (kernels already handed over are waited for) and every request is as it was:
 * the next mc_run launches the same work, with bitwise the same results.  A
 * failure from the finalize kernel on, or one after which the stream cannot be
 * drained, loses the work of every request in that launch: those requests take
 * no further launches, and mc_results (blocking or not) returns MC_ERR_HIP for
 * them once no launch in flight refers to them, and releases them (their ids
 * are then unknown). */
mc_status mc_results(mc_ctx* ctx, uint64_t request_id, mc_result* out, size_t n, int blocking);

/* Ask running persistent kernels to stop fetching tiles.  Every request submitted
 * (or restored) before the call completes with status MC_ERR_ABORTED on its
 * unfinished functions (mc_results returns MC_ERR_ABORTED); the next mc_run waits
 * for the launches in flight, then clears the request so later work runs
 * normally.  Requests submitted after the call, also before that mc_run, are not
 * affected. */
mc_status mc_abort(mc_ctx* ctx);

/* Cancel one request (a serving loop whose client went away): none of its
 * work not yet handed to the GPU runs, and work already there is discarded.
 * It completes -- mc_poll reports it, mc_results returns MC_ERR_ABORTED --
 * once no kernel refers to its device slots any more: at once if it was still
 * queued or none of its work is in flight, else when the launches holding its
 * work have been collected (a resident context stops its running launch for
 * that, which starts again at once).  Results already in stay; every other
 * result carries MC_ERR_ABORTED.  Other requests are unaffected, bit for bit.
 * A request already complete, or lost to a failed launch, is left as it is.
 * Errors: MC_ERR_UNKNOWN_REQUEST, MC_ERR_HIP. */
mc_status mc_cancel(mc_ctx* ctx, uint64_t request_id);

/* Checkpoint and resume of one request.  A function's state is its result
 * once finished, and otherwise the partial sums of the tiles it has run (its
 * samples are addressed by counter, paper "Solution method": which points a
 * tile draws never depends on when it runs), so a request snapshotted part way
 * and restored later -- in another context, process or machine with the same
 * library version -- completes with results bitwise equal to a run without the
 * interruption.
 *
 * mc_snapshot waits for the launches in flight -- in a resident context it
 * stops the running launch, which starts again once the snapshot is written
 * (after a size query it stays stopped until the next call that runs work, so
 * the size holds for an mc_snapshot that follows at once) --, then
 * writes request `request_id`'s state into buf[0 .. *bytes): its functions (a
 * grid as its expanded table), their tiling and progress, the results already
 * in, and the partials of the tiles run (16 bytes per tile; native byte
 * order).  With buf NULL it only stores the size into *bytes.  The request
 * stays in the context unchanged (continue it, abort it, or take its
 * results).  Snapshots do not depend on the engine: one taken in a launch
 * context restores into a resident one and the other way round.  A request
 * that uses run-time families carries their source texts.  Errors:
 * MC_ERR_INVALID_ARG (cap smaller than needed -- *bytes holds the size --, an
 * aborted or failed request), MC_ERR_UNKNOWN_REQUEST, MC_ERR_HIP.
 *
 * mc_restore checks a snapshot (format, version, every function as mc_submit
 * does, tiling and progress against the functions) and queues it as a new
 * request whose id it stores into *out_request_id; its saved partials go to
 * the device when it is admitted (a resident context stops its running launch
 * for that copy).  Functions whose results were in complete at once; the
 * restoring context's MC_NO_PROMOTE setting applies to FP32 results not yet
 * in.  Run-time families are found by source text among those registered on
 * the restoring context (in any order; the request takes this context's ids).
 * Errors: MC_ERR_INVALID_ARG (not a snapshot of this library version,
 * inconsistent or truncated), MC_ERR_UNSUPPORTED_FAMILY (a run-time family
 * whose source is not registered here), the validation codes of mc_submit,
 * MC_ERR_ADMISSION. */
mc_status mc_snapshot(mc_ctx* ctx, uint64_t request_id, void* buf, size_t cap, size_t* bytes);
mc_status mc_restore(mc_ctx* ctx, const void* buf, size_t bytes, uint64_t* out_request_id);

/* The plain baseline path: for each function one kernel launch with a grid
 * sized to its N (one thread per 4 samples) and a second launch that reduces
 * the block partials, FP64 evaluation, no batching and no graph.  Synchronous:
 * returns when out[0..n) holds the results. */
mc_status mc_integrate_plain_fp64(mc_ctx* ctx, const mc_function* fns, size_t n, mc_result* out,
                                  void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): mc_integrate_plain_fp64
 * with the same arguments and bitwise the same results, but calling no
 * hipMalloc, hipFree or other allocating routine.  Its working set (the copied
 * table, the packed records, the results and the block partials) lives in a
 * fixed 24 MiB array in the library's code object, one per GPU, held until the
 * process ends; mc_create looks up its address on the context's device.
 * Limits: n <= 4096 functions, n_samples <= 2^30 per function (larger inputs
 * return MC_ERR_INVALID_ARG and run nothing).  The array is shared by every
 * call on a GPU and keeps the last call's contents: calls that overlap on one
 * GPU (from several threads, contexts or streams) race and must be serialized
 * by the caller.  Synchronous on `stream`; errors as mc_integrate_plain_fp64. */
mc_status mc_integrate_plain_fp64_noalloc(mc_ctx* ctx, const mc_function* fns, size_t n, mc_result* out,
                                          void* stream);

/* Tuning of the batched path: workgroups per CU for the persistent kernel and,
 * per (precision, family, dim), log2 of the segments each wave takes per tile.
 * Results never depend on these (the reduction tree is fixed per function). */
mc_status mc_get_tuning(mc_ctx* ctx, uint32_t* blocks_per_cu, uint8_t* seg_log2 /* [2][4][12] */);
mc_status mc_set_tuning(mc_ctx* ctx, uint32_t blocks_per_cu, const uint8_t* seg_log2 /* [2][4][12] or NULL */);

/* Time candidate tunings on synthetic functions of every (family, dim) in
 * `precision` and keep the fastest: workgroups per CU (FP32 kernel) first, then
 * the tile size per (family, dim), stopping when `budget_seconds` is spent (a
 * trial in progress finishes).  Blocks until done; uses `stream`; call it on a
 * context with no requests of its own in flight.  Results never change.
 * With MC_TUNE_CACHE naming a text file in the environment, a line for this
 * device kind, compute-unit count, library version and precision is taken
 * from the file instead of timing (the last matching line wins; malformed
 * lines are ignored), and a tuning that was timed is appended to it. */
mc_status mc_autotune(mc_ctx* ctx, int32_t precision, void* stream, double budget_seconds);

/* Kernel timing of the most recent completed direct-launch mc_run (persistent
 * kernels, and finalize with publish, in milliseconds, from HIP events on the
 * launch stream). */
mc_status mc_last_run_timing(mc_ctx* ctx, double* main_ms, double* finalize_ms);

/* Cumulative counters of a context since it was created (completed launches only). */
typedef struct mc_stats {
    uint64_t launches;           /* completed launches */
    uint64_t tiles32, tiles64;   /* tiles run by the FP32 and FP64 persistent kernels */
    uint64_t functions;          /* function results produced (promoted ones count twice) */
    uint64_t samples;            /* integrand evaluations in those tiles */
    uint64_t promoted;           /* FP32 functions re-run in FP64 */
    uint64_t bad_records;        /* records that failed the kernels' bounds checks (always 0 unless corrupt) */
    double fp32_ms;              /* direct launches: sum of FP32 persistent-kernel time (HIP events on the launch stream) */
    double fp64_ms;              /* direct launches: sum of FP64 persistent-kernel time */
    double finalize_ms;          /* direct launches: sum of finalize and publish time */
    double graph_ms;             /* graph launches: sum of whole-graph time (every kernel of the launch) */
} mc_stats;

mc_status mc_get_stats(mc_ctx* ctx, mc_stats* out);

/* The points at which the library samples function `f` (direct Monte Carlo:
 * uniform points in the box, paper "Solution method"): samples
 * [first, first + count) as count x f->dim doubles, row-major, into the host
 * array `out`, computed on the device by the batched kernels' Philox generator
 * and FP64 mapping x = fma(hi - lo, u, lo).  The FP32 evaluation uses the same
 * uniforms u.  For reproducing or auditing a result; synchronous on `stream`.
 * Errors: as mc_submit's validation of f; MC_ERR_INVALID_ARG if the range is
 * empty, leaves [0, n_samples) or holds more than 2^26 samples. */
mc_status mc_sample_points(mc_ctx* ctx, const mc_function* f, uint64_t first, uint64_t count, double* out,
                           void* stream);

/* Register an integrand family given as source text, compiled at run time for
 * gfx950 (hipRTC).  The paper's program integrates functions of arbitrary form
 * written by the user (program summary, "Nature of problem"; the multi-function
 * class of "Solution method"); this is that capability for the batched kernels.
 *
 * `source` must define, at namespace scope,
 *     template <class T>
 *     __device__ T mc_user_integrand(const T* x, const T* p, uint32_t dim);
 * x[0..dim) is the sample point inside the function's box, p[0..32) its
 * mc_function.params, T = float for MC_PREC_FP32_EVAL and double for MC_PREC_FP64
 * (FP32 evaluation sees x and p rounded to float; sums and the finalize stay as
 * for the built-in families, including FP32 -> FP64 promotion and the
 * absolute-coordinate rule of MC_PREC_FP32_EVAL; what the caller's code itself
 * loses in FP32 -- e.g. sin of a large argument -- the library cannot see, so such
 * integrands should be submitted in MC_PREC_FP64).  HIP device math
 * (sinf, exp, ...) is available.  The source is copied; the id written to
 * *family_out (MC_FAMILY_USER0 + k, k < MC_MAX_USER_FAMILIES, in registration
 * order) goes into mc_function.family for mc_submit on this context only.
 * mc_integrate_plain_fp64 accepts built-in families only.
 *
 * Errors: MC_ERR_INVALID_ARG (NULL argument, or all 8 ids used), MC_ERR_COMPILE
 * (the compiler log is in mc_last_error), MC_ERR_HIP (module load).  On a
 * validate-only context the source is compiled but not loaded.  The caller's
 * code runs unchecked inside the library's kernels: an out-of-bounds access in
 * it faults like any kernel.  Launches on a context with registered families
 * are enqueued directly, not as captured graphs.  A resident context
 * (MC_RESIDENT) compiles its resident kernel again with every family it has
 * registered (a few tens of seconds), stops its running launch, and launches
 * the new kernel in its place.  Compiled code is kept for the life of the
 * process, by source: registering the same families again, in this or another
 * context, compiles nothing. */
mc_status mc_register_family(mc_ctx* ctx, const char* source, uint32_t* family_out);

/* Message of the last failure on ctx (or of the calling thread when ctx is NULL). */
const char* mc_last_error(mc_ctx* ctx);

/* Samples per segment (the unit each wave reduces; a function's reduction tree
 * is built over its segments), and the library's version string. */
uint32_t mc_segment_samples(void);
const char* mc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ZMC_H */
