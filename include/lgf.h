/*
 * lgf.h — C ABI of the MI355X (gfx950) lattice Green's function solver.
 *
 * Problem (Sec. 2.1, Eq. dpoisson / dpoissonsoln): on the unbounded lattice Z^3 with
 * the 7-point Laplacian [L u](n) = sum_{+-e_i} u(n +- e_i) - 6 u(n) and unit spacing,
 * compute u = G * f, i.e. u(n) = sum_m G(n - m) f(m), where G is the lattice Green's
 * function (Eq. lgf1) and f is supported on a union of equal cubic blocks of n^3
 * points (Sec. 2.3).  u is evaluated on the same blocks (B_e = B_s, the case Sec. 3.1
 * describes), or, for a plan from lgf_plan_create_split, on a separate set of evaluation
 * blocks (B_e != B_s in Eq. bconv).
 * The sum is evaluated with the Fast Lattice Green's Function method of Sec. 3.1:
 * block-wise zero-padded FFT convolutions with the exact G between neighbouring
 * blocks (level 0) and, on an octree of interpolation intervals, Lagrange
 * anterpolation (Reg) up the tree, FFT convolutions with the far kernel between the
 * intervals of each interaction list, and interpolation (Interp) back down.
 * For spacing h the caller scales f by h^2.
 *
 * Layouts.  A layout is an array block_ijk[nblocks][3] of int32 block coordinates
 * (bx, by, bz), any origin, no duplicates.  Fields f and u are DEVICE arrays
 * [nblocks][n][n][n] indexed [block][z][y][x] with x fastest, in layout order; entry
 * (b, z, y, x) is the lattice point (bx*n + x, by*n + y, bz*n + z).  Element type is
 * double for LGF_F64 plans and float for LGF_F32 plans.
 *
 * Ownership and streams.  The plan owns its lists, device workspace and a reference
 * to the process-wide cache of kernel spectra (shared by all plans with equal
 * (n, p, level geometry, precision)).  f and u stay owned by the caller and must
 * stay alive until the work enqueued on `hip_stream` has completed.  All device work
 * of lgf_solve is asynchronous on `hip_stream` (a hipStream_t; NULL = default
 * stream); no host<->device copy happens inside a solve.  lgf_plan itself performs
 * synchronous device work (kernel spectra, list upload) on `hip_stream`.
 * A plan holds one workspace: solves on one plan must not overlap in time (enqueue
 * them on one stream).  Different plans may run concurrently on different streams.
 * By default the far-field levels of a solve run on streams owned by the plan (level 1 on
 * one, levels >= 2 on another), forked from and joined back into hip_stream with events, so
 * they overlap the near-field transforms (lgf_tuning.overlap); from the caller's view the
 * solve is ordinary stream work on hip_stream either way.
 *
 * Errors.  Every entry point returns an lgf_status; nothing is printed and no C++
 * exception crosses the ABI.  lgf_last_error() returns a thread-local message for the
 * most recent failure on the calling thread.
 */
#ifndef LGF_H_
#define LGF_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lgf_plan_s* lgf_plan_t;

typedef enum {
    LGF_OK = 0,
    LGF_ERR_ARG = 1,     /* NULL pointer, unsupported n or p, bad count                 */
    LGF_ERR_LAYOUT = 2,  /* empty layout, duplicate blocks, coordinate span > 2^20      */
    LGF_ERR_OOM = 3,     /* device allocation failed                                     */
    LGF_ERR_BUDGET = 4,  /* the plan would exceed the configured device-memory budget    */
    LGF_ERR_DEVICE = 5,  /* a HIP runtime call or kernel launch failed                   */
    LGF_ERR_BUSY = 6     /* the request server's queue is full, or a plan's workspace is
                            still in use by a solve issued on another stream            */
} lgf_status;

typedef enum { LGF_F64 = 0, LGF_F32 = 1 } lgf_precision;

/* Plan summary filled by lgf_plan_query. */
typedef struct {
    int64_t nblocks;          /* active blocks N_B^0                                   */
    int64_t npoints;          /* nblocks * n^3                                         */
    int32_t n, p;             /* block edge and interpolation nodes per interval edge  */
    int32_t levels;           /* tree levels L actually built (leaves at level 1)      */
    int32_t top_level;        /* highest level with a non-empty interaction list (0 = none) */
    int64_t near_pairs;       /* entries of all level-0 near-neighbour lists           */
    int64_t far_pairs[16];    /* entries of the interaction lists, index = level       */
    int64_t intervals[16];    /* intervals per level, index = level                    */
    int64_t workspace_bytes;  /* device bytes owned by the plan                        */
    int64_t spectra_bytes;    /* device bytes of the (shared) kernel spectra it uses   */
    int32_t precision;        /* lgf_precision                                         */
    int64_t source_blocks;    /* blocks of f (B_s)                                     */
    int64_t eval_blocks;      /* blocks of u (B_e); equal to source_blocks and nblocks
                                 unless the plan has separate sets, where nblocks counts
                                 the union the tree of levels >= 1 is built on          */
    int32_t spectra_mode;     /* lgf_spectra_mode of the plan's kernel spectra          */
    double kappa;             /* screening of the operator (lgf_plan_create_screened),
                                 0 for the Laplace operator                             */
} lgf_plan_info;

/*
 * Build a plan (Sec. 3.1 tree and lists; Step 0 pre-computation, Eq. precomp).
 *   block_ijk : HOST array [nblocks][3] of block coordinates (read during the call only)
 *   nblocks   : >= 1
 *   n         : points per block edge; 4, 6, 8, 12 or 16 (padded FFT length 2n)
 *   p         : interpolation nodes per interval edge at every level >= 1: 2..10, where
 *               every stencil uses all p nodes (n_max = p, Sec. 2.5 Lebesgue rule), or
 *               p = n + 1 with n = 12 or 16 (13 or 17 nodes), the paper's scheme
 *               n_I = n + 1 with stencils of the n_max = 10 closest nodes (Sec. 2.5,
 *               Sec. 4).  p = n + 1 puts the nodes on the lattice (the paper's
 *               experimental scheme; n = 6, p = 7 and n = 12, p = 13 are its n_I = 7 and 13)
 *   levels    : tree levels L (leaves at 1); <= 0 selects the full depth
 *               1 + ceil(log2(extent)).  When L is below full depth the top level's
 *               list holds every non-adjacent interval.
 *   prec      : LGF_F64, or LGF_F32 (FP32 forward transforms, products and level-0
 *               inverse; level >= 1 inverse transforms in FP64 arithmetic with
 *               float-float node values through Interp; FP64 kernel tables and spectrum
 *               generation, FP64 final add of far and near fields)
 *   hip_stream: stream for the set-up work (hipStream_t or NULL)
 *   out       : receives the plan on success
 * Errors: LGF_ERR_ARG, LGF_ERR_LAYOUT, LGF_ERR_OOM, LGF_ERR_BUDGET, LGF_ERR_DEVICE.
 */
lgf_status lgf_plan_create(const int32_t* block_ijk, int64_t nblocks, int32_t n, int32_t p,
                           int32_t levels, lgf_precision prec, void* hip_stream, lgf_plan_t* out);

/*
 * A plan for the screened operator L - kappa instead of L: u = G_kappa * f with G_kappa the
 * lattice Green's function of [L_kappa u](n) = sum_{+-e_i} u(n +- e_i) - (6 + kappa) u(n),
 * the discrete modified-Helmholtz operator (an implicit viscous step on the same grid leads
 * to it).  The paper's method applies to it unchanged as a second non-oscillatory lattice
 * kernel (Sec. 5): only the kernel values differ.  They are the Bessel integral of
 * Appendix A (Eq. lgf3) with 6 + kappa in place of 6, integrated on the device in FP64 at
 * every point a kernel block uses; there is no asymptotic expansion of G_kappa here, so
 * every interpolation node must lie on the lattice: (p - 1) must divide n (p = n + 1 is the
 * paper's scheme; p = 17 with n = 16 uses its local stencils).
 *   kappa : 0 (the same plan as lgf_plan_create) or in [1e-3, 1e6]
 * All other arguments, the solve (lgf_solve, graphs, tuning) and the errors as for
 * lgf_plan_create; LGF_ERR_ARG also for kappa out of range or nodes off the lattice.
 */
lgf_status lgf_plan_create_screened(const int32_t* block_ijk, int64_t nblocks, int32_t n, int32_t p,
                                    int32_t levels, double kappa, lgf_precision prec, void* hip_stream,
                                    lgf_plan_t* out);

/*
 * Host-only preview of lgf_plan_create: builds the tree and lists of the layout (no device
 * work, no allocation on the device) and fills *info as lgf_plan_query would, with
 * workspace_bytes = the device bytes the plan would own and spectra_bytes = 0.  For
 * admission decisions and inspection.  Errors: LGF_ERR_ARG, LGF_ERR_LAYOUT, LGF_ERR_OOM.
 */
lgf_status lgf_plan_estimate(const int32_t* block_ijk, int64_t nblocks, int32_t n, int32_t p,
                             int32_t levels, lgf_precision prec, lgf_plan_info* info);

/*
 * u = G * f on the plan's layout (Steps 1-3 of Sec. 3.1).  f, u: DEVICE pointers as
 * described above (may not alias; f over the source blocks and u over the evaluation
 * blocks for a plan with separate sets).  u is overwritten entirely.  Asynchronous on
 * hip_stream.  Errors: LGF_ERR_ARG (NULL), LGF_ERR_BUSY (the plan's previous solve was
 * issued on another stream and has not finished: its one workspace would be shared),
 * LGF_ERR_DEVICE (launch failure).  With LGF_CHECK_FINITE=1 in the environment the input
 * is scanned first (synchronising hip_stream) and non-finite values give LGF_ERR_ARG.
 * With LGF_SYNC_CHECK=1 every kernel launch of an eager solve is followed by a
 * synchronisation, and a failure names its step in lgf_last_error (a debugging aid).
 */
lgf_status lgf_solve(lgf_plan_t plan, const void* f, void* u, void* hip_stream);

/*
 * Several independent solves enqueued back to back on one stream; plans[i] is used
 * with f[i], u[i].  Plans must be distinct (each owns one workspace).
 */
lgf_status lgf_solve_many(const lgf_plan_t* plans, const void* const* f, void* const* u,
                          int32_t count, void* hip_stream);

/*
 * Batched solves (many independent problems, one launch sequence).  The problems of a
 * batch share n, p, levels and precision; their layouts may differ.  The plan is the
 * union of the per-layout trees: every list stays inside its own layout (the union is
 * exact, not an approximation: each problem's u depends on its own f only, Sec. 3.1
 * applied per layout), while each kernel of Steps 1-3 runs once over all layouts.
 *   layouts[i] : HOST array [nblocks[i]][3] of block coordinates of problem i (each
 *                layout has its own origin; coordinates of different layouts may overlap)
 *   count      : number of problems, >= 1
 * The plan's f and u are the problems' fields concatenated in batch order: problem i owns
 * blocks [offsets[i], offsets[i+1]) as returned by lgf_plan_solve_offsets.  All other
 * arguments and errors as for lgf_plan_create; the plan is used with lgf_solve.
 */
lgf_status lgf_plan_create_batch(const int32_t* const* layouts, const int64_t* nblocks, int32_t count,
                                 int32_t n, int32_t p, int32_t levels, lgf_precision prec,
                                 void* hip_stream, lgf_plan_t* out);

/*
 * Plan with separate source and evaluation blocks (Eq. bconv: u^P = sum over Q in B_s of
 * conv(k^{Q-P}, f^Q) for every P in B_e; Sec. 3.1 describes the method for B_e = B_s, and
 * its lists, transfers and transforms apply unchanged to the two sets).
 *   source_ijk : HOST array [nsource][3] of the source blocks B_s; f is DEVICE
 *                [nsource][n][n][n] in this order
 *   eval_ijk   : HOST array [neval][3] of the evaluation blocks B_e; u is DEVICE
 *                [neval][n][n][n] in this order
 * Both sets use one lattice (one origin); they may overlap, be disjoint or nest, and
 * neither may hold duplicates.  The tree of levels >= 1 spans the union of the two
 * sets (its extent sets the full depth); the near field pairs each evaluation block with
 * its neighbouring source blocks only.  A set equal to the other gives the same u as
 * lgf_plan_create.  All other arguments and errors as for lgf_plan_create.  Plans with
 * separate sets are single problems (not for lgf_plan_create_batch or the server).
 */
lgf_status lgf_plan_create_split(const int32_t* source_ijk, int64_t nsource, const int32_t* eval_ijk,
                                 int64_t neval, int32_t n, int32_t p, int32_t levels, lgf_precision prec,
                                 void* hip_stream, lgf_plan_t* out);

/* Host-only preview of lgf_plan_create_split (as lgf_plan_estimate). */
lgf_status lgf_plan_estimate_split(const int32_t* source_ijk, int64_t nsource, const int32_t* eval_ijk,
                                   int64_t neval, int32_t n, int32_t p, int32_t levels, lgf_precision prec,
                                   lgf_plan_info* info);

/*
 * Block offsets of the problems of a plan: *count receives the number of problems (1 for
 * a plan from lgf_plan_create or lgf_plan_create_split) and
 * offsets[0..min(count+1, max_entries)-1] (HOST, may be NULL) the first block of each
 * problem followed by the total block count (of u: the evaluation blocks for a plan with
 * separate sets).
 * Errors: LGF_ERR_ARG.
 */
lgf_status lgf_plan_solve_offsets(lgf_plan_t plan, int64_t* offsets, int32_t max_entries, int32_t* count);

/*
 * HIP graph of one solve.  lgf_graph_create captures the launch sequence of
 * lgf_solve(plan, f, u, .) into an executable graph (f and u are baked in: the graph
 * always reads f and writes u at these DEVICE addresses).  The caller's hip_stream is
 * synchronised first; capture uses a private stream and enqueues no device work.
 * lgf_graph_launch enqueues the whole solve as one graph launch on hip_stream, with the
 * same result as lgf_solve; the plan's single-workspace rule applies (no overlap with
 * other solves or graph launches of the same plan).  The graph must be destroyed
 * before its plan.  Errors: LGF_ERR_ARG, LGF_ERR_DEVICE, and for lgf_graph_launch
 * LGF_ERR_BUSY as for lgf_solve (graph launches and solves of one plan share its workspace).
 */
typedef struct lgf_graph_s* lgf_graph_t;
lgf_status lgf_graph_create(lgf_plan_t plan, const void* f, void* u, void* hip_stream, lgf_graph_t* out);
lgf_status lgf_graph_launch(lgf_graph_t graph, void* hip_stream);
lgf_status lgf_graph_destroy(lgf_graph_t graph);

/*
 * Kernel variants of a plan.  Variants differ in scheduling only: every variant gives the
 * same u bit for bit.  0 selects the library's default where listed.  LGF_M2L_WIDE_LISTS=1
 * in the environment makes the level >= 1 Prod keep 32-bit source-list entries at every
 * level size (it switches to them by itself for levels of 65535 or more intervals); the
 * bits are the same.
 */
typedef struct {
    int32_t fft0_threads;   /* threads per workgroup of the level-0 transforms: 0, 128, 256, 512    */
    int32_t near_waves;     /* waves per workgroup of the level-0 Prod: 2, 4, 8                      */
    int32_t near_prefetch;  /* level-0 Prod issues the next half source slab's loads early: 0, 1
                               (a new plan starts with 1 from 256 level-0 groups of 2^3 blocks)     */
    int32_t far_waves;      /* parent groups per workgroup of the level >= 1 Prod: 0, 1, 2, 4, 8, 16
                               (clamped to at most 16 waves per workgroup, 8 in FP64)       */
    int32_t far_children;   /* children accumulated per lane of that kernel: 0, 1, 2, 4, 8           */
    int32_t overlap;        /* schedule of a solve: 1 three concurrent branches (near field, level 1,
                               levels >= 2), 3 two (near field, levels >= 1), 2 one stream,
                               0 default (three).  With 3 and 2 the M2L of all levels with one
                               tile size is one launch                                                */
} lgf_tuning;

/*
 * Autotuner for eager solves (lgf_solve): times each candidate on (f, u) (DEVICE buffers of
 * the plan's shape; u is overwritten) as the median over `reps` rounds of 4 solves issued
 * back to back on hip_stream.  The kernel variants are chosen first, on one stream
 * (overlap 2: the sum of the kernels' durations), in a coordinate search over the other
 * fields of lgf_tuning; then the schedule (overlap 1, 3 or 2) of an eager solve with those
 * variants.  The choice replaces the plan's variants only if it is at least 1% faster than
 * the variants the call started from, and is remembered for later plans of the same (n, p,
 * precision, power-of-two block-count bucket) in this process; if the environment variable
 * LGF_TUNE_FILE names a file the choice is appended there and read by later processes.
 * A graph runs the schedules with other costs (dependencies resolved on the device instead
 * of host events), so a caller that launches graphs picks the overlap its graph is built
 * with by timing one graph per schedule.  Synchronous.  Errors: LGF_ERR_ARG, LGF_ERR_DEVICE.
 */
lgf_status lgf_plan_autotune(lgf_plan_t plan, const void* f, void* u, void* hip_stream, int32_t reps);

/* The plan's current variants.  Errors: LGF_ERR_ARG. */
lgf_status lgf_plan_get_tuning(lgf_plan_t plan, lgf_tuning* out);

/* Pin the plan's variants by hand (HOST struct, read during the call).
 * Errors: LGF_ERR_ARG (a value outside the lists above). */
lgf_status lgf_plan_set_tuning(lgf_plan_t plan, const lgf_tuning* tuning);

/* Fill *info (HOST struct).  Errors: LGF_ERR_ARG. */
lgf_status lgf_plan_query(lgf_plan_t plan, lgf_plan_info* info);

/* Release the plan's device memory (synchronises with nothing: the caller must make
 * sure no enqueued solve still uses it).  NULL is accepted. */
lgf_status lgf_plan_destroy(lgf_plan_t plan);

/* Device-memory budget in bytes for all plan workspaces + spectra of this process
 * (0 = unlimited, the default).  Plans that would exceed it fail with LGF_ERR_BUDGET. */
lgf_status lgf_set_memory_budget(int64_t bytes);

/* Bytes currently held by live plans and the spectra cache. */
int64_t lgf_memory_in_use(void);

/* Drop cached kernel spectra not referenced by a live plan. */
lgf_status lgf_spectra_cache_trim(void);

/*
 * Storage of the kernel spectra k^(P-Q) (Sec. 3.1, pre-computation; Sec. 3.2, unique
 * kernel vectors per level) for plans created after the call, process-wide (a plan, and
 * a request server, for all the plans it creates, keep the mode they were created with):
 *   LGF_SPECTRA_FULL    one spectrum per offset: 27 at level 0, 343 per level >= 1 (default)
 *   LGF_SPECTRA_REDUCED one spectrum per class of offsets under the 48 signed axis
 *                       permutations the LGF is invariant under: 4 at level 0, 20 per
 *                       level >= 1 (the 16 far classes and the 4 near ones), plus 4 bytes
 *                       per offset.  The Prod kernels read each offset's coefficient at
 *                       the permuted frequency (conjugated where that frequency lies
 *                       outside the stored half spectrum).  u differs from the full
 *                       tables' only by the rounding of the spectrum generation.
 * Errors: LGF_ERR_ARG (unknown mode).
 */
typedef enum { LGF_SPECTRA_FULL = 0, LGF_SPECTRA_REDUCED = 1 } lgf_spectra_mode;
lgf_status lgf_set_spectra_mode(int32_t mode);
int32_t lgf_get_spectra_mode(void);

/*
 * Per-step device timing of a plan's solves (measurement support).
 * lgf_profile_enable(plan, max_solves): the next max_solves calls of lgf_solve on this
 * plan record HIP events around the whole solve and before and after every step (fwd
 * FFT, Reg, Prod, inverse FFT, Interp, final add of each level), each on the stream the
 * step runs on (for small plans the far-field steps run on the plan's internal second stream,
 * concurrently with the near field).  Recording adds no synchronisation.  lgf_profile_collect waits for the recorded events and
 * fills *out with, per step in launch order: its name, the summed device time over
 * the nsolves recorded solves (one launch per step per solve), and the step's
 * algorithmic bytes and flops per launch (compulsory HBM traffic: every input read once, every output
 * written once; flops by the paper's operation counts, Table 1).  Per-solve times
 * are written to solve_ms[0..min(recorded, max_out)-1] when solve_ms is non-NULL.
 * Collecting disables recording.  Errors: LGF_ERR_ARG, LGF_ERR_DEVICE.
 */
#define LGF_MAX_STEPS 64
typedef struct {
    int32_t nsteps;                 /* steps per solve                              */
    int32_t nsolves;                /* solves recorded                              */
    char name[LGF_MAX_STEPS][32];   /* step names, e.g. "prod_l0", "fft_fwd_l1"     */
    double total_ms[LGF_MAX_STEPS]; /* device time summed over the recorded solves  */
    double bytes[LGF_MAX_STEPS];    /* algorithmic bytes per launch                 */
    double flops[LGF_MAX_STEPS];    /* algorithmic flops per launch                 */
} lgf_step_profile;

lgf_status lgf_profile_enable(lgf_plan_t plan, int32_t max_solves);
lgf_status lgf_profile_collect(lgf_plan_t plan, lgf_step_profile* out, double* solve_ms, int32_t max_out);

/*
 * Request server: independent solves submitted one by one (each u = G * f on its own
 * layout, Sec. 3.1) and run concurrently on one GPU.
 *   - A dispatcher thread owned by the server takes requests in submission order.  A
 *     request starts when one of max_slots streams is free and its plan fits the HBM
 *     budget; it is retired when its completion event has fired.
 *   - Plans (lists and workspace) stay resident, cached by layout, and are reused by
 *     later requests with the same block coordinates; kernel spectra are shared by all
 *     plans with equal (n, p, precision).  A plan that does not fit the budget evicts
 *     idle cached plans (least recently used first), else waits for running requests.
 *     A request whose plan alone exceeds the budget fails with LGF_ERR_BUDGET.
 *   - Results do not depend on what else is running: every request computes exactly
 *     what lgf_solve computes on a plan of its own layout.
 * budget_bytes counts the resident plan workspaces plus the shared kernel spectra
 * (0 = unlimited).  max_queue bounds the waiting requests (0 = unbounded); a submit to
 * a full queue returns LGF_ERR_BUSY.  The server serves one (n, p, levels, precision).
 */
typedef struct lgf_server_s* lgf_server_t;

typedef struct {
    int64_t budget_bytes;  /* HBM budget of the server's resident state, 0 = unlimited */
    int32_t max_slots;     /* requests running at once (one stream each), 1..16         */
    int32_t max_queue;     /* waiting requests accepted, 0 = unbounded                  */
    int32_t n, p, levels;  /* as for lgf_plan_create                                    */
    int32_t precision;     /* lgf_precision                                             */
} lgf_server_config;

typedef struct {
    int32_t status;     /* LGF_OK, or the error that ended the request             */
    int64_t nblocks;    /* blocks of the request's layout                          */
    double latency_ms;  /* submit -> completion observed (host clock)              */
    double queue_ms;    /* submit -> launch                                        */
    double device_ms;   /* solve time on the device (events around the solve)      */
} lgf_request_result;

typedef struct {
    int64_t completed, failed, queued;  /* requests                                       */
    int64_t points;                     /* grid points of the completed requests           */
    int64_t plans_created, plans_evicted;
    int64_t plan_bytes, spectra_bytes;  /* resident device bytes                           */
    double latency_p50_ms, latency_p99_ms, latency_max_ms;  /* of the completed requests   */
    double points_per_s;                /* points / (first submit -> last completion)      */
} lgf_server_stats_t;

/* Start a server on the current device.  Errors: LGF_ERR_ARG (bad config), LGF_ERR_DEVICE. */
lgf_status lgf_server_create(const lgf_server_config* cfg, lgf_server_t* out);

/*
 * Queue one solve.  block_ijk: HOST layout [nblocks][3] (copied); f, u: DEVICE fields of
 * the server's precision in the layout's order, caller-owned, kept alive and untouched until
 * the request completes.  hip_stream: the caller's stream (hipStream_t, NULL = default
 * stream).  An event is recorded on it during the call and the request's solve, which runs
 * on one of the server's own streams, waits for that event: work the caller enqueued on
 * hip_stream before the submit (the writes of f, anything still using u) is complete before
 * the solve reads f or writes u.  u holds the result once lgf_server_poll or lgf_server_wait
 * report the request finished; work on other streams must not touch u before that.
 * *ticket identifies the request.  Non-blocking.
 * Errors: LGF_ERR_ARG, LGF_ERR_BUSY (queue full), LGF_ERR_DEVICE (event creation or record
 * failed).  Layout errors are reported per request.
 */
lgf_status lgf_server_submit(lgf_server_t server, const int32_t* block_ijk, int64_t nblocks, const void* f,
                             void* u, void* hip_stream, int64_t* ticket);

/* *done = 1 and *result filled (HOST, may be NULL) when the request has finished; a
 * finished ticket is then released.  Errors: LGF_ERR_ARG (unknown ticket). */
lgf_status lgf_server_poll(lgf_server_t server, int64_t ticket, int32_t* done, lgf_request_result* result);

/* Block until the request has finished, fill *result and release the ticket. */
lgf_status lgf_server_wait(lgf_server_t server, int64_t ticket, lgf_request_result* result);

/* Counters and latency percentiles since creation or the last reset. */
lgf_status lgf_server_stats(lgf_server_t server, lgf_server_stats_t* out);
lgf_status lgf_server_reset_stats(lgf_server_t server);

/* Finish every queued request, then release the server's plans and streams. */
lgf_status lgf_server_destroy(lgf_server_t server);

/* Thread-local message for the last failure on this thread ("" if none). */
const char* lgf_last_error(void);

/*
 * Lattice Green's function values computed by the library's own FP64 device table
 * (Appendix A, Eq. lgf3 Bessel integral), exposed for validation:
 *   out[(a*R + b)*R + c] = G(a, b, c) for 0 <= a, b, c < R.  out is a HOST array of
 *   R^3 doubles.  Synchronous.  Errors: LGF_ERR_ARG (R < 1 or R > 128), LGF_ERR_DEVICE.
 */
lgf_status lgf_green_table(int32_t R, double* out);

/*
 * The screened operator's LGF G_kappa (lgf_plan_create_screened) from the library's own
 * FP64 device integration, for validation: out[(a*R + b)*R + c] = G_kappa(a, b, c) for
 * 0 <= a, b, c < R, HOST array of R^3 doubles.  Synchronous.
 * Errors: LGF_ERR_ARG (R < 1, R > 128, kappa outside [1e-3, 1e6]), LGF_ERR_DEVICE.
 */
lgf_status lgf_green_table_screened(int32_t R, double kappa, double* out);

/*
 * The library's far-field kernel A^q (Sec. 2.1, Eq. lgf2, q = 8 terms) at npts HOST
 * points pts[npts][3] (x, y, z), written to HOST out[npts].  Synchronous; evaluated
 * on the device in FP64.  Errors: LGF_ERR_ARG, LGF_ERR_DEVICE.
 */
lgf_status lgf_far_kernel(const double* pts, int64_t npts, double* out);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): lgf_far_kernel without any device
 * allocation.  Same arguments and the same values, bit for bit.  The points, the values and
 * the expansion's coefficient tables are staged in one static device array of the library
 * (8 MiB + 64 KiB per GPU, held until the process ends), so npts is limited to
 * LGF_FAR_KERNEL_NOALLOC_MAX_POINTS per call.  Calls share that array; the library
 * serialises them (one call at a time per process), and each call rewrites everything it
 * reads.  Synchronous, on the device that is current.
 * Errors: LGF_ERR_ARG (bad arguments, or npts above the maximum), LGF_ERR_DEVICE.
 */
#define LGF_FAR_KERNEL_NOALLOC_MAX_POINTS 262144
lgf_status lgf_far_kernel_noalloc(const double* pts, int64_t npts, double* out);

#ifdef __cplusplus
}
#endif

#endif /* LGF_H_ */
