/*
 * lsr.h -- C ABI of the MI355X (gfx950) loop-of-stencil-reduce library.
 *
 * The pattern (Aldinucci et al., "A Parallel Pattern for Iterative Stencil +
 * Reduce", Sect. 3.1) repeats  a = stencil(sigma_k, f):a  until a condition c
 * holds on a global reduce /(+) of the new array (or of delta(new, old) in the
 * -d variant), with an optional global state s such as the sweep count (-s
 * variant). A call to lsr_run is one instance of that procedure:
 *
 *   grid       -> a (the array; in/out: it holds the last iterate on completion)
 *   stencil_id -> (k, f): a compiled elemental function on the 3x3 neighbourhood
 *                 (k = 1, the halo width given by the paper's "3, 3" extent)
 *   reduce_op  -> (delta, (+), identity)
 *   cond       -> c, evaluated every check_every sweeps and at the sweep cap
 *   max_iter   -> the -s state bound (n == max_iter stops the loop)
 *
 * The building blocks the paper's constructor takes (Sect. 3.2: elemental
 * function, combinator with identity, iteration condition, sizes, neighbourhood
 * extent) map one to one onto these arguments. The detection phase of the
 * two-phase restoration is its own stage in the paper's pipeline (Sect. 4.3), so
 * it is a separate one-shot call (lsr_amf_detect).
 *
 * Conventions
 *  - Every call returns lsr_status; nothing throws or aborts across the ABI.
 *    lsr_last_error() gives a thread-local message for the last failure.
 *  - Grid/env pointers are DEVICE pointers (e.g. torch tensors' data_ptr()) on
 *    the context's device, except for lsr_run_host, which takes host buffers.
 *    Grids are row-major with a row pitch counted in elements (pitch >= cols);
 *    env arrays use the same pitch as the grid.
 *  - The caller owns grid->data and the env arrays. The library owns its scratch
 *    (the ping-pong partner grid, per-block partials, the 64-byte job state) and
 *    draws it from a pool bounded by lsr_config.hbm_budget_bytes.
 *  - Ordering: lsr_run starts after all work already enqueued on the context's
 *    stream (lsr_config.stream, NULL = the null stream) and returns at once;
 *    the caller must not touch the job's buffers until lsr_result reports a
 *    terminal status. lsr_result then orders the caller's stream after the job.
 *  - A context is driven from one host thread at a time.
 */
#ifndef LSR_H
#define LSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lsr_ctx lsr_ctx;
typedef int64_t lsr_job;

typedef enum {
    LSR_OK = 0,
    LSR_EINVAL = 1,     /* invalid argument or unsupported combination */
    LSR_ENOMEM = 2,     /* device allocation failed */
    LSR_EBUSY = 3,      /* over the HBM budget, or a non-blocking result is not ready */
    LSR_EDEVICE = 4,    /* a HIP call failed; lsr_last_error() has the HIP message */
    LSR_ENUMERIC = 5,   /* the reduce value became NaN or Inf; the loop stopped there */
    LSR_ECANCELED = 6,  /* the job was cancelled */
    LSR_ENOTFOUND = 7   /* unknown job id (never issued, or its result was already taken) */
} lsr_status;

typedef enum { LSR_U8 = 1, LSR_F32 = 4, LSR_F64 = 8 } lsr_dtype;

/* Out-of-range handling of the neighbourhood (the bottom value of Sect. 3.1). */
typedef enum {
    LSR_BC_RING = 0,    /* the outer ring is fixed boundary data, never updated (Jacobi) */
    LSR_BC_TORUS = 1,   /* both axes wrap (Life) */
    LSR_BC_BOTTOM = 2   /* out-of-range items are absent: dead cells (Life, Fig. 1),
                           dropped neighbours (restoration) */
} lsr_bc;

typedef enum {
    LSR_ST_LAPLACE5 = 1,    /* b = 0.25*((N+S)+(W+E)) on interior cells (Helmholtz with alpha=0, f=0) */
    LSR_ST_HELMHOLTZ5 = 2,  /* b = (((N+S)+(W+E)) + g) * rd, rd = 1/(4 + alpha*h*h), g = h^2 f in env0
                               (the Jacobi solver of Sect. 4.1); param[0] = alpha, param[1] = h.
                               F32 storage needs alpha*h*h in [-4/3, 4] (EINVAL otherwise): its
                               stochastically rounded update relies on |0.25 - rd| <= 1/8 */
    LSR_ST_LIFE = 3,        /* B3/S23 on u8 cells (Fig. 1); non-zero bytes are alive; output is 0/1 */
    LSR_ST_RESTORE = 4,     /* flagged pixels (env0 = u8 mask) take argmin_t sum phi(t - u_m) over
                               their in-range 8-neighbourhood (phase 2 of Sect. 4.3);
                               phi(t) = sqrt(beta + t^2), param[0] = beta,
                               param[1] != 0 selects phi(t) = t^2 */
    LSR_ST_SOBEL = 5,       /* u8 image: b = min(255, floor(sqrt(Gx^2 + Gy^2))) with Gx, Gy the 3x3
                               Sobel derivative masks and samples outside the image 0 (the edge
                               detector of Sect. 4.2, a single-iteration pattern: max_iter = 1,
                               cond NEVER; the reduce SUM is the sum of the new image) */
    LSR_ST_HELMHOLTZ5_SEP = 6, /* the -i form of HELMHOLTZ5 (Sect. 3.1: the elemental function also
                               receives the cell's index): g(i, j) = c2 * (c1 * (p[i] * q[j])),
                               evaluated in FP64 from the cell's indices, replaces the env array;
                               env0 = p (rows FP64 values), env1 = q (cols FP64 values), both
                               device vectors; param[0] = alpha, param[1] = h, param[2] = c1,
                               param[3] = c2. With the factors of a separable right-hand side it
                               gives HELMHOLTZ5's result bit for bit while reading 16 instead of
                               24 bytes per cell update. Plain contexts and device buffers only */
    LSR_ST_BOX = 7,         /* radius-k box mean (sigma_k of Sect. 3.1, k = param[0] in 1..4): cells at
                               least k from the edge take the mean of their (2k+1)^2 neighbourhood
                               (box rows summed left to right, the row sums top to bottom, one
                               division by (2k+1)^2); the band of width k is fixed (bc RING) */
    LSR_ST_LAPLACE7_3D = 8  /* 3D 7-point Jacobi on nz planes of ny rows stored plane after plane
                               (rows = nz * ny, param[0] = ny, cols = nx, pitch per row): inside,
                               b = (((W+E) + (N+S)) + (U+D)) / 6; the six faces are fixed (bc RING) */
} lsr_stencil_id;

typedef enum {
    LSR_RED_MAX_ABS_DELTA = 1,  /* max |b - a| over the grid (0 where a cell is not updated) */
    LSR_RED_L2_DELTA = 2,       /* sqrt(sum (b - a)^2), unscaled */
    LSR_RED_SUM = 3,            /* number of live cells of b (u64; Life) */
    LSR_RED_MEAN_ABS_DELTA = 4  /* sum |b - a| / (rows*cols) (the restoration test of Sect. 4.3) */
} lsr_reduce_op;

typedef enum {
    LSR_COND_BELOW = 1,      /* stop when r < threshold (strict) */
    LSR_COND_STABLE_FOR = 2, /* stop once the count was unchanged at stable_window consecutive
                                checks; the count before the first sweep is the first reference */
    LSR_COND_NEVER = 3       /* run to max_iter */
} lsr_cond_kind;

typedef struct {
    int32_t kind;           /* lsr_cond_kind */
    int32_t check_every;    /* >= 1; the reduce and the test run every check_every sweeps and at max_iter */
    int32_t stable_window;  /* >= 1 for LSR_COND_STABLE_FOR */
    int32_t reserved;
    double threshold;       /* for LSR_COND_BELOW */
} lsr_cond;

typedef struct {
    void *data;             /* device pointer, rows x pitch elements of dtype (in/out) */
    int64_t rows, cols;     /* rows, cols >= 3 (Jacobi), >= 1 otherwise */
    int64_t pitch;          /* elements between row starts, >= cols */
    int32_t dtype;          /* lsr_dtype: F64, or F32 storage (arithmetic in FP32, reduce and test
                               in FP64) for Jacobi/restoration; U8 for Life */
    int32_t bc;             /* lsr_bc */
    const void *env0;       /* read-only env: Helmholtz g (grid dtype), restoration mask (u8) */
    const void *env1;       /* HELMHOLTZ5_SEP: the column factor q; otherwise NULL */
    double param[4];        /* stencil parameters, see lsr_stencil_id */
} lsr_grid;

/*
 * LSR_FLAG_BATCHED: the context runs the batched engine (continuous batching of
 * many jobs, the stream-of-tasks form of Sect. 3.2/4): lsr_run queues the job and
 * returns; an engine thread admits queued jobs in arrival order as soon as the
 * pool can hold their scratch within the HBM budget, advances every admitted job
 * by one sweep per round (one launch per kernel family for the sweeps of all
 * jobs, one launch for all their final reduces and conditions), and retires jobs
 * as they stop, freeing their memory for the next arrivals. A job's tile shape and
 * reduce order depend only on its own shape, so its result is the same alone and
 * in any mix. Supported: every stencil (restoration sweeps one round at a time;
 * two-phase restoration frames through lsr_run_restore_host).
 */
#define LSR_FLAG_BATCHED 1u

typedef struct {
    int32_t device;            /* HIP device ordinal */
    uint32_t flags;            /* LSR_FLAG_* */
    void *stream;              /* hipStream_t the caller orders against (NULL = null stream) */
    uint64_t hbm_budget_bytes; /* cap on library scratch; 0 = 90% of free device memory */
} lsr_config;

typedef struct {
    int64_t iterations;     /* sweeps performed, n */
    double last_reduce;     /* r at the last check (the count for LSR_RED_SUM) */
    uint64_t last_count;    /* live cells after the last check (Life) */
    int32_t converged;      /* 1 if the condition held at the stop (0 if stopped by max_iter) */
    int32_t status;         /* lsr_status of the job */
    int32_t stable_run;     /* consecutive unchanged checks at the stop (Life) */
    int32_t sweeps_per_launch; /* sweeps each sweep-kernel launch advanced (the temporal
                               blocking depth used; 1 when unfused) */
    int64_t checks;         /* number of reduce + condition evaluations */
    double device_ms;       /* device time from the job's first to its last kernel (batched: from
                               admission to retirement, shared with the other jobs of the batch) */
    double queue_ms;        /* host time from lsr_run to the start of the job's device work */
    double latency_ms;      /* host time from lsr_run until the host saw the job end */
} lsr_job_result;

/* Tuning overrides; 0 in a field means "choose automatically". */
typedef struct {
    int32_t tile_rows;      /* rows each workgroup streams through per sweep */
    int32_t tb_depth;       /* sweeps (generations) fused per launch (temporal blocking); 1 = off.
                               Jacobi: 2, 4, 5, 8 or 10; 0 = the measured best depth that
                               divides both check_every and max_iter, else 5 with checks
                               inside launches. Life: 2, 3, 4, 5, 6 or 8; 0 = 8. A stop or
                               cap inside a launch is replayed exactly from the launch's
                               source. Grids whose rows are not 16-byte aligned (Life: or not
                               a multiple of 16 cells) run on staged aligned copies (Life rows
                               padded to 16 cells), fused as well. Fields and counts are bit
                               for bit those of unfused
                               sweeps; a float reduce value differs at most in the order of
                               its partial sums. Restoration is never fused. A batched context
                               takes the depth (FP64 10, 5 or 2; FP32 5 or 2; Life 8 at any
                               width, 1 = one generation per round) and tile_rows from the
                               same overrides or tuning table. */
    int32_t chunk;          /* sweeps per enqueued chunk (a multiple of check_every) */
    int32_t use_graph;      /* 1 = replay chunks as HIP graphs, -1 = plain launches */
    int32_t waves;          /* Jacobi: wavefronts per workgroup (1, 2 or 4) */
    int32_t unroll;         /* Jacobi: rows loaded together per wavefront (4, 8 or 16;
                               fused launches always load 3) */
} lsr_tuning;

/*
 * Creates a context on cfg->device: the runtime set-up that the pattern's
 * implementation does once before any task (Sect. 3.2/3.3: device detection and
 * set-up, the device-memory manager that keeps buffers persistent across
 * iterations; here an execution stream, a pool bounded by hbm_budget_bytes, pinned
 * state mirrors and a driver thread, or the batched engine with
 * LSR_FLAG_BATCHED). *out receives the context; the caller destroys it with
 * lsr_destroy. EINVAL for a NULL argument, unknown flags or a bad device ordinal;
 * EDEVICE when a HIP call fails (nothing is left allocated then).
 */
lsr_status lsr_create(const lsr_config *cfg, lsr_ctx **out);

/* Destroys the context (the end of the runtime of Sect. 3.3) after all its jobs have
 * finished: frees its scratch pool, pinned mirrors and streams. Results not taken are
 * discarded. EINVAL for NULL. */
lsr_status lsr_destroy(lsr_ctx *ctx);

/* Sets tuning overrides for later lsr_run calls (NULL restores the defaults). */
lsr_status lsr_set_tuning(lsr_ctx *ctx, const lsr_tuning *tuning);

/*
 * Autotuner (the launch heuristics of Sect. 3.3, measured instead of guessed). Runs short
 * jobs of this description (zero-filled scratch grids of rows x cols, check_every, at most
 * max_iter sweeps; max_iter <= 0 means no cap) with each candidate launch setting (fused
 * depth, wavefronts per workgroup, band rows, load unroll) on the context's device, and keeps
 * the fastest in the context's table under the key (stencil_id, dtype, bit lengths of rows
 * and cols, check_every). Later lsr_run calls whose overrides leave the launch shape
 * automatic (tile_rows, tb_depth, waves and unroll all 0) take the table's entry for their
 * key, so a job's settings depend only on its key. On a batched context the candidates are
 * the engine's own settings (the fused depths its Jacobi families hold and the band rows of a
 * wavefront tile; for Life one or 8 generations per round, each with its band rows), each
 * measured on 8-256 jobs of the key run together
 * (about 2^25 cells, so the rounds are full); the table then serves that context's later jobs
 * (and others through lsr_tune_export / lsr_tune_import). The winner is copied to best_out
 * when it is not NULL. Blocks until done (a plain context: a few hundred short jobs, about a
 * second at 8192^2; a batched one: up to a few seconds per key); no other job of the context
 * may run meanwhile (a batched context with unfinished jobs: EBUSY). EINVAL for stencils other
 * than Laplace, Helmholtz and Life; ENOMEM/EDEVICE as lsr_run.
 * The caller owns nothing new; scratch returns to the context's pool.
 */
lsr_status lsr_autotune(lsr_ctx *ctx, int32_t stencil_id, int32_t dtype, int64_t rows,
                        int64_t cols, int32_t check_every, int64_t max_iter,
                        lsr_tuning *best_out);

/*
 * The autotuner's table as JSON text, tagged with the device architecture:
 *   {"arch": "gfx950", "entries": [{"stencil": 2, "dtype": 8, "rows_log2": 14, ...}, ...]}
 * Writes at most cap bytes (NUL included) to buf; *len_out receives the size needed. With
 * buf NULL only the size is reported; a buffer that is too small gives EINVAL.
 */
lsr_status lsr_tune_export(lsr_ctx *ctx, char *buf, uint64_t cap, uint64_t *len_out);

/* Merges a table written by lsr_tune_export into the context's (EINVAL if it was measured on
 * another architecture or is malformed; the context's table is then unchanged). */
lsr_status lsr_tune_import(lsr_ctx *ctx, const char *json);

/*
 * Starts one loop-of-stencil-reduce job (asynchronous). Supported combinations:
 *   LAPLACE5   F64|F32  RING            env0 NULL        MAX_ABS|L2|MEAN_ABS  BELOW|NEVER
 *   HELMHOLTZ5 F64|F32  RING            env0 g (dtype)   MAX_ABS|L2|MEAN_ABS  BELOW|NEVER
 *   LIFE       U8       TORUS|BOTTOM    env0 NULL        SUM                  STABLE_FOR|NEVER
 *   RESTORE    F64|F32  BOTTOM          env0 mask (u8)   MAX_ABS|MEAN_ABS     BELOW|NEVER
 *   SOBEL      U8       BOTTOM          env0 NULL        SUM                  NEVER
 *   HELMHOLTZ5_SEP F64|F32 RING         env0 p, env1 q   as HELMHOLTZ5        as HELMHOLTZ5
 *   BOX        F64|F32  RING            env0 NULL        MAX_ABS|L2|MEAN_ABS  BELOW|NEVER
 *   LAPLACE7_3D F64|F32 RING            env0 NULL        MAX_ABS|L2|MEAN_ABS  BELOW|NEVER
 * (HELMHOLTZ5_SEP, BOX and LAPLACE7_3D run on plain contexts only.)
 * EINVAL: null pointers, rows/cols too small, pitch < cols, a combination outside the table,
 * check_every < 1, max_iter < 1, stable_window < 1 with STABLE_FOR. ENOMEM/EBUSY: scratch.
 */
lsr_status lsr_run(lsr_ctx *ctx, const lsr_grid *grid, int32_t stencil_id, int32_t reduce_op,
                   const lsr_cond *cond, int64_t max_iter, lsr_job *job_out);

/*
 * Starts one job whose grid lives in HOST memory: the ingest of a stream item as
 * the paper's runtime does it (Sect. 3.3: when a task is scheduled, device
 * buffers are allocated and filled by H2D copies; Fig. 2: read(output) copies the
 * result back by D2H). Same arguments, checks and supported combinations as
 * lsr_run, except that grid->data and grid->env0 are host pointers (rows x pitch
 * elements each; the RESTORE mask is u8 with the grid's pitch in elements).
 *  - Memory: the context allocates the job's device grid, env and scratch from
 *    its pool, so all of the job's device memory counts against
 *    hbm_budget_bytes. Plain context: allocated at this call (ENOMEM/EBUSY as
 *    lsr_run). Batched context: allocated at admission, which waits in arrival
 *    order until the budget can hold them; the H2D copies run on the engine's
 *    copy stream and the job joins the sweep rounds once they have completed.
 *  - Ownership: the caller keeps both host buffers alive, and does not write
 *    them, until lsr_result reports a terminal status; grid->data then holds the
 *    last iterate (its contents are unspecified after EDEVICE). The device copies
 *    are freed at retirement.
 *  - Pinned host memory (hipHostMalloc, a torch pin_memory tensor) lets the copies
 *    run asynchronously; with pageable memory each copy blocks the thread that
 *    issues it.
 */
lsr_status lsr_run_host(lsr_ctx *ctx, const lsr_grid *grid, int32_t stencil_id, int32_t reduce_op,
                        const lsr_cond *cond, int64_t max_iter, lsr_job *job_out);

/*
 * Two-phase restoration of one HOST frame as one job on a batched context: the
 * frame-at-a-time pipeline of Sect. 4.3 (detect, then the iterative restore, for
 * each frame of a stream; items of a stream overlap on the device and reuse its
 * memory, Sect. 4.3 and 3.3). y is the noisy u8 frame (y->data host, rows, cols,
 * pitch in bytes; y->bc must be BOTTOM; y->param[0] = beta, y->param[1] != 0
 * selects phi(t) = t^2, as for RESTORE). When admitted (under the HBM budget, like
 * lsr_run_host), the frame goes to the device on the copy stream; then, between
 * sweep rounds of other jobs, adaptive-median detection (lsr_amf_detect's rule,
 * w_max) writes the mask and the initial iterate on the device, and the job's
 * restoration sweeps join the rounds. At retirement the restored frame is copied
 * to u_out (host, u_dtype F32 or F64, rows x y->pitch elements). The caller keeps
 * y->data and u_out alive and untouched until lsr_result reports a terminal
 * status. reduce_op, cond, max_iter as for RESTORE. EINVAL on a plain context, for
 * a non-U8 frame, a bad u_dtype, w_max not odd in [3, 31], or what lsr_run would
 * reject for the restoration of a frame this shape.
 */
lsr_status lsr_run_restore_host(lsr_ctx *ctx, const lsr_grid *y, void *u_out, int32_t u_dtype,
                                int32_t w_max, int32_t reduce_op, const lsr_cond *cond,
                                int64_t max_iter, lsr_job *job_out);

/*
 * Result of a job: the loop's output read back once it has stopped (Fig. 2's
 * read(output) step; the field itself stays in the caller's device grid, or has been
 * copied back into the host grid for lsr_run_host). wait != 0 blocks until the job
 * ends; wait == 0 returns EBUSY while it runs. On a terminal status the job's record is released (a second call gives ENOTFOUND)
 * and the context stream is ordered after the job. Returns the job's own status
 * (OK, ENUMERIC, ECANCELED, EDEVICE), which is also in out->status.
 */
lsr_status lsr_result(lsr_ctx *ctx, lsr_job job, int32_t wait, lsr_job_result *out);

/*
 * Completion queue of a context, for a caller serving a stream of jobs (the
 * stream of tasks of Sect. 3.2, whose items finish in any order): stores in
 * *job_out the id of a finished job whose result has not been taken yet, oldest
 * completion first; the caller then takes it with lsr_result. wait != 0 blocks
 * until some job finishes; wait == 0 returns EBUSY when none has. ENOTFOUND when
 * nothing is left to report: every job submitted has finished and has been
 * reported here or had its result taken. Each finished job is reported at most
 * once; a job whose result lsr_result already took is skipped.
 */
lsr_status lsr_wait_any(lsr_ctx *ctx, int32_t wait, lsr_job *job_out);

/* A snapshot of a context's queues and memory, for a serving loop's monitoring. */
typedef struct {
    int64_t pending;            /* submitted and not yet admitted (batched) or started (plain) */
    int64_t ingesting;          /* batched: host jobs whose H2D copies are in flight */
    int64_t active;             /* in the sweep rounds (batched); running (plain) */
    int64_t retiring;           /* batched: stopped, result being copied out */
    int64_t unfinished;         /* submitted and not finished */
    int64_t finished_untaken;   /* finished, result not yet taken with lsr_result */
    uint64_t pool_live_bytes;   /* device memory the jobs hold from the pool */
    uint64_t pool_cached_bytes; /* freed blocks the pool keeps for reuse */
    uint64_t pool_budget_bytes; /* hbm_budget_bytes in force */
} lsr_stats;

/* Fills *out (EINVAL for NULL). The counts are consistent with each other only
 * approximately: the engine publishes its own after every pass of its loop. */
lsr_status lsr_get_stats(lsr_ctx *ctx, lsr_stats *out);

/* Requests cancellation; the job stops at its next chunk boundary with ECANCELED. */
lsr_status lsr_cancel(lsr_ctx *ctx, lsr_job job);

/*
 * For callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): lsr_run followed by a waiting
 * lsr_result, with the job's scratch (partner grid, per-tile partials, loop state)
 * taken from one fixed device array of LSR_NOALLOC_SCRATCH_BYTES that the library
 * holds on every device it runs on until the process ends, instead of the pool.
 *  - Allocates nothing: no device or pinned memory, no graph, no event. Runs on
 *    the context's stream (lsr_config.stream), after the work already enqueued on
 *    it, and returns once the job has finished and its last iterate is in
 *    grid->data; the result is written to *out.
 *  - Same arguments, checks and supported combinations as lsr_run (device
 *    pointers), and the same kernels, so results are bit for bit those of lsr_run.
 *    EINVAL also when the partner grid plus partials exceed the scratch
 *    (rows * pitch * element size must stay below LSR_NOALLOC_SCRATCH_BYTES minus
 *    the partials), or when the grid would need staged copies (rows not 16-byte
 *    aligned; Life rows not a multiple of 16 cells).
 *  - out->device_ms and out->latency_ms are host wall time of the call.
 *  - Every call on one device shares that device's array: calls that overlap on
 *    one device (from several threads, or on streams that run concurrently) race
 *    and give wrong results. Calls in sequence are safe: each job initialises all
 *    the scratch it reads.
 */
#define LSR_NOALLOC_SCRATCH_BYTES ((uint64_t)65 << 20)
lsr_status lsr_run_noalloc(lsr_ctx *ctx, const lsr_grid *grid, int32_t stencil_id,
                           int32_t reduce_op, const lsr_cond *cond, int64_t max_iter,
                           lsr_job_result *out);

/*
 * Adaptive-median impulse detection, phase 1 of the two-phase restoration (Sect. 4.3;
 * a window grown up to a static bound, Sect. 3.2). For each pixel of the u8 image y,
 * windows w = 3, 5, ..., w_max of in-range pixels are tried; med is the lower median
 * (sorted index (count-1)/2). The first window with min < med < max decides
 * flag = !(min < y < max); if none does, flag = (y == min || y == max) with the w_max
 * window. Writes mask (u8 0/1, pitch y->pitch) and u_init (dtype u_dtype, pitch
 * y->pitch): med where flagged, y elsewhere. w_max odd, 3 <= w_max <= 31.
 * Synchronous with respect to the context stream ordering (enqueued, not waited on).
 */
lsr_status lsr_amf_detect(lsr_ctx *ctx, const lsr_grid *y, void *mask, void *u_init,
                          int32_t u_dtype, int32_t w_max);

/*
 * Validates a job description exactly as lsr_run does, without a device or a
 * context: returns LSR_OK or the LSR_EINVAL lsr_run would return (message in
 * lsr_last_error()). Allocates nothing.
 */
lsr_status lsr_check_args(const lsr_grid *grid, int32_t stencil_id, int32_t reduce_op,
                          const lsr_cond *cond, int64_t max_iter);

/*
 * Plain device-to-device copy of `bytes` (a multiple of 16; 16-byte aligned device
 * pointers), run `iters` times back to back on the context's internal stream after
 * one warm-up copy, timed with HIP events; *avg_ms receives the mean time per copy.
 * The measured HBM ceiling for the roofline (2*bytes/avg_ms) and the calibration
 * kernel for the memory counters. Blocks until done.
 */
lsr_status lsr_probe_copy(lsr_ctx *ctx, void *dst, const void *src, uint64_t bytes,
                          int32_t iters, double *avg_ms);

/* Thread-local text of the last error (never NULL). */
const char *lsr_last_error(void);

/* Library version string. */
const char *lsr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LSR_H */
