/*
 * pdr.h -- C ABI of the MI355X (gfx950) Potential Difference Reduction library.
 *
 * The library runs the PDR method for multicommodity-flow feasibility
 * (Liu, "A Localized Method for Multicommodity Flow Problem", arXiv 2108.07549):
 * a pseudo-flow f >= 0 is improved by sweeps. Each sweep computes the excess
 * Delta and the vertex heights h (Section 3.1, Expressions 2-4), the arc
 * congestion psi (Expression 5) and the objective z (Algorithm 1), applies the
 * stop test of Algorithm 1 on the device, and then updates every arc in
 * parallel, either by the exact edge subproblem (PDR-ESO: Expression 14,
 * Algorithm 2) or by the adaptive-gradient step (PDR-AGD: Algorithm 3).
 *
 * Conventions for every call:
 *  - No C++ exception crosses the ABI. Every call returns a pdr_status; the
 *    text of the last failure is returned by pdr_last_error. A host memory
 *    allocation that fails inside a call returns PDR_ERR_OOM; if the call
 *    changes state (sweeps, solve, precision, state, adjoint, and the batch
 *    calls that sweep, tune or switch precision), the object is then
 *    poisoned as after a device error.
 *  - Host arrays passed in are read during the call only and stay owned by
 *    the caller. Output host arrays are owned by the caller.
 *  - The context owns all device memory it allocates. A context is not
 *    thread-safe; distinct contexts are independent.
 *  - Work runs on the context's HIP stream (the caller's stream from
 *    pdr_options.stream, or one the library creates at default priority).
 *  - After a device error the context is poisoned: every later call returns
 *    PDR_ERR_DEVICE until pdr_destroy.
 *  - Flows are exchanged as m x K row-major arrays (arc-major, commodity
 *    contiguous) in the caller's CSR arc order.
 */
#ifndef PDR_H
#define PDR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdr_ctx pdr_ctx;

typedef enum {
    PDR_OK = 0,
    PDR_ERR_INVALID = 1, /* bad argument or instance; nothing was changed */
    PDR_ERR_OOM = 2,     /* device memory would not fit (nothing was allocated),
                            or a host allocation failed */
    PDR_ERR_DEVICE = 3,  /* a HIP call failed; the context is poisoned */
    PDR_ERR_STATE = 4,   /* call not valid in the context's current state */
    PDR_ERR_NUMERIC = 5  /* the objective became non-finite */
} pdr_status;

/* PDR_ESO: Algorithm 1 with the exact edge subproblem (Algorithm 2);
 * PDR_AGD: Algorithm 3; PDR_GDM: Algorithm 4; PDR_CAP: the loop of Algorithm 1
 * for Section 6's formulation (conservation relaxed, capacities kept): each arc
 * projects c = ((h_i + f) - (h_j - f))/2 onto {f >= 0, sum_k f <= u}, i.e.
 * f' = max(0, c - lambda) with lambda = 0 when sum max(0, c) <= u. */
typedef enum { PDR_ESO = 0, PDR_AGD = 1, PDR_GDM = 2, PDR_CAP = 3 } pdr_method;

/* PDR_FP64: f and h stored and updated in FP64.
 * PDR_FP32_BULK: f and h stored and updated in FP32; excess accumulation,
 * per-arc sums, the objective and the stop test stay in FP64. */
typedef enum { PDR_FP64 = 0, PDR_FP32_BULK = 1 } pdr_precision;

typedef enum { PDR_UNDECIDED = 0, PDR_FEASIBLE = 1, PDR_INFEASIBLE = 2 } pdr_verdict;

/* Parameters of Algorithms 3 (AGD) and 4 (GDM). Defaults are the paper's
 * experimental settings (Section 7.2): AGD beta_init 0.25, beta_min 1/K,
 * beta_max 0.5, alpha_inc 2, alpha_dec 0.5; GDM beta_init 0.1, beta_min 1/K,
 * beta_max 0.2, alpha_inc 2, alpha_dec 0.5, momentum gamma 0.9; the increase
 * period is 10 iterations (Algorithms 3, 4). beta_min <= 0 means 1/K. gamma is
 * used by GDM only and must lie in [0, 1). */
typedef struct {
    double beta_init, beta_min, beta_max, alpha_inc, alpha_dec;
    int32_t inc_period;
    double gamma;
} pdr_agd_params;

typedef struct {
    int32_t method;        /* pdr_method */
    int32_t precision;     /* pdr_precision */
    pdr_agd_params agd;    /* used by PDR_AGD */
    pdr_agd_params gdm;    /* used by PDR_GDM */
    double z_feasible_tol; /* verdict FEASIBLE needs z <= this (default 1e-8) */
    void *stream;          /* hipStream_t to run on, or NULL */
    int32_t lanes_per_arc; /* 0: automatic; else a power of two 1..1024 (tuning) */
    int32_t vec_per_lane;  /* 0: automatic; else a count the library instantiates for
                              that lane count: 1, 2, 4, 8 for all; 10, 12, 16, 20
                              for 128 and 256; 3, 5, 6 for 256 and more (tuning) */
    int32_t graph_sweeps;  /* passes per captured HIP graph in pdr_sweep: 0 = 32,
                              < 0 = launch every kernel directly */
    int32_t height_chunk;  /* 16-byte vectors per commodity chunk in the height
                              kernel: 0 = automatic, else a power of two 1..65536 */
    int32_t cluster_size;  /* vertices per locality cluster of the visiting order:
                              0 = automatic (64), 1 = the caller's vertex order */
    int32_t height_blocks; /* blocks of the grid-stride height kernel: 0 = automatic,
                              else 1..8192 (tuning) */
    int32_t height_unroll; /* incident rows each height-kernel thread loads before
                              summing: 0 = automatic, 1, 2, 4 or 8 (tuning) */
    int32_t z_log_capacity; /* objective evaluations kept by pdr_z_log: 0 = 2^20,
                               else a power of two up to 2^20 */
    int32_t cache_policy;  /* cache hints of the pass's flow, velocity and height
                              traffic: 0 = automatic (ordinary loads and stores
                              when f, h and v of one pass fit in the 256 MB
                              Infinity Cache, so they stay resident between
                              passes; non-temporal otherwise, so the height rows
                              that neighbouring arcs re-read stay in L2);
                              1 = ordinary; 2 = non-temporal. Results are the
                              same bit for bit; batches always stream. */
    int32_t batch_groups;  /* batches only: the members are split into this many
                              groups of about equal work, each running its
                              passes on a stream of its own (joined once per
                              call or captured graph, not once per pass):
                              0 = automatic (4, at most B), else 1..4. Results
                              are the same bit for bit. */
    int32_t height_kernel; /* excess -> height kernel of single instances:
                              0 = automatic (the vertex-parallel kernel),
                              1 = vertex-parallel, 2 = tiled: each block stages
                              the rows of the arcs incident to up to 64 neighbouring
                              vertices in LDS, 8 vectors at a time, so an arc
                              with both ends in the tile is read from HBM once
                              rather than once per end (pdr_init fails with
                              PDR_ERR_INVALID when a vertex has more than 304
                              incident arcs). The tiled kernel reads about a
                              third less but runs slower on MI355X, its loads
                              in flight being bounded by the LDS it stages
                              through. Flows and heights are the same bit for
                              bit; the objective's partial sums are grouped
                              differently (last-bit differences). Batches use
                              the vertex-parallel kernel. */
} pdr_options;

/* FP64 residual report of the current flows (see pdr_residual). */
typedef struct {
    double z;              /* objective of Algorithm 1 / Expression 8 */
    double z_psi;          /* 1/2 sum_e psi_e^2 */
    double z_h;            /* 1/2 sum_{i,k} delta_i h_ik^2 */
    double kkt_sq;         /* sum rho^2, rho = phi if f > 0 else max(0, phi) (Section 3.3) */
    double max_abs_excess; /* max |Delta_ik| */
    double max_congestion; /* max psi_e */
    double farkas_gap;     /* sum_k d_k (h_sk - h_tk) - sum_e u_e max(0, max_k (h_ik - h_jk)) */
    double farkas_tol;     /* rounding margin of farkas_gap */
    double z_fp32_floor;   /* FP32 storage: the objective that rounding each stored flow
                              alone would leave (last pass); 0 in FP64 */
    int64_t sweeps_done;   /* arc updates applied since init (iteration counter t) */
    int64_t evaluations;   /* objective evaluations recorded in the z log */
    int32_t verdict;       /* pdr_verdict: INFEASIBLE if farkas_gap > farkas_tol,
                              else FEASIBLE if z <= z_feasible_tol, else UNDECIDED */
    int32_t stopped;       /* 1 if the last pdr_sweep call ended on its stop test */
} pdr_residual_t;

/* Fill *opt with the defaults (ESO, FP64, the paper's AGD and GDM parameters,
 * z_feasible_tol 1e-8, stream NULL, automatic tiling). */
void pdr_default_options(pdr_options *opt);

/*
 * Create a context for one instance (Section 1): a directed graph G(V, E)
 * with n vertices given as an out-adjacency CSR (row_ptr[n+1], int64,
 * row_ptr[0] = 0, non-decreasing, row_ptr[n] = m; col[m] = head of each arc,
 * arc e has tail i with row_ptr[i] <= e < row_ptr[i+1]), capacities u[m],
 * and K commodities (s[K], t[K], d[K]) with s_k != t_k.
 * Flows start at 0 and, for AGD, learning rates at beta_init (Algorithms 1, 3).
 * Host arrays are deep-copied; opt may be NULL for the defaults.
 * Errors: PDR_ERR_INVALID for n < 1, m < 0, K < 1, a malformed CSR, a head
 * out of range, a self-loop, u or d negative or non-finite, s or t out of
 * range, s_k == t_k, a commodity endpoint of degree 0, or a requested tiling
 * (lanes_per_arc, vec_per_lane) that does not cover the row; PDR_ERR_OOM if the
 * device buffers would not fit; PDR_ERR_DEVICE for a HIP failure. On failure
 * *out is set to NULL. Rows of up to 8,192 vectors of 16 bytes (K <= 16,384 in
 * PDR_FP64, K <= 32,768 in PDR_FP32_BULK) are held in registers by the arc
 * kernels; longer rows are streamed (see pdr_tiling).
 */
pdr_status pdr_init(pdr_ctx **out, int32_t n, int32_t m, const int64_t *row_ptr,
                    const int32_t *col, const double *u, int32_t K, const int32_t *s,
                    const int32_t *t, const double *d, const pdr_options *opt);

/*
 * Enqueue up to max_sweeps passes of Algorithm 1 (ESO), Algorithm 3 (AGD) or
 * Algorithm 4 (GDM).
 * Each pass computes h, psi and z from the current flows, records z in the z
 * log, stops if eps_obj > 0 and |z - z_prev| < eps_obj (z_prev = +inf before
 * the first pass since init) or if z_target > 0 and z <= z_target, and
 * otherwise updates every arc (Jacobi: all arcs read the same h).
 * The stop test runs on the device. With no stop test active the call only
 * enqueues work; otherwise it polls the device between batches of passes.
 * A non-finite objective stops the passes like a met stop test (before the
 * update of that pass); pdr_residual, pdr_solve and pdr_adjoint then report
 * PDR_ERR_NUMERIC.
 * Errors: PDR_ERR_INVALID for max_sweeps < 0; PDR_ERR_DEVICE.
 */
pdr_status pdr_sweep(pdr_ctx *ctx, int64_t max_sweeps, double eps_obj, double z_target);

/*
 * Run passes until the objective z (evaluated in FP64 from the stored flows)
 * is <= z_target, or until max_sweeps passes in total (synchronizes).
 * In PDR_FP64 it is pdr_sweep with the z_target stop test.
 * In PDR_FP32_BULK the passes run in FP32 and, every `window` passes, the
 * library estimates where FP32 rounding will stop the descent: every pass
 * adds rounding noise of size z_noise (the objective that rounding each stored
 * flow alone leaves, computed by the height kernel), and a descent that
 * shrinks z by (1 - rate) per pass settles near z_noise / rate (rate measured
 * on the windows' smallest z over the last four windows). When the window's
 * smallest z is <= floor_factor * z_noise / rate (floor_factor <= 0 means 5,
 * or 0.03 for PDR_GDM, whose FP32 descent goes on far below the estimate),
 * or when z stalls (four windows in a row whose smallest z is not below the
 * smallest before by more than 10 z_noise), the flows are widened to FP64
 * exactly (as pdr_set_precision) and the run finishes in FP64: the FP64 polish.
 * The rate and stall tracking carries over from one call to the next, so a
 * long run may be split into calls; pdr_set_state, pdr_set_state_noalloc and
 * pdr_set_precision (and the hand-over itself) restart it.
 * sweeps_fp32 / sweeps_fp64 (may be NULL) receive the passes run in each
 * precision. Errors: PDR_ERR_INVALID for z_target <= 0, max_sweeps < 0 or
 * window < 1; PDR_ERR_NUMERIC for a non-finite objective; PDR_ERR_DEVICE.
 */
pdr_status pdr_solve(pdr_ctx *ctx, double z_target, int64_t max_sweeps, int64_t window,
                     double floor_factor, int64_t *sweeps_fp32, int64_t *sweeps_fp64);

/* Compute the FP64 residual report of the current flows (synchronizes).
 * Returns PDR_ERR_NUMERIC (and fills *out) if z is not finite. */
pdr_status pdr_residual(pdr_ctx *ctx, pdr_residual_t *out);

/* Copy the current pseudo-flow f (Section 3.1: f_ek >= 0 of every commodity
 * k on every arc e, not necessarily conserving) as FP64 into host_out[m*K],
 * m x K row-major in the caller's arc order (synchronizes). */
pdr_status pdr_flows(pdr_ctx *ctx, double *host_out);

/* Write the current pseudo-flow (Section 3.1) into caller-owned device
 * memory dev_out[m*K] (m x K row-major, caller's arc order), as FP64 if
 * fp64 != 0 else FP32. The write is enqueued on the context stream after all
 * work already enqueued there and the call returns without a host sync: a
 * reader on another stream must wait for the context stream first (an event
 * recorded on the stream pdr_stream returns, or a device synchronization).
 * The Python binding does this against torch's current stream. */
pdr_status pdr_flows_device(pdr_ctx *ctx, void *dev_out, int32_t fp64);

/* The HIP stream the context runs on (hipStream_t as void*): the caller's
 * pdr_options.stream, or the one the library created. */
pdr_status pdr_stream(const pdr_ctx *ctx, void **stream);

/* Copy the FP64 heights h[n*K] of the current flows (Expressions 2-4:
 * h_ik = Delta_ik / delta_i with Delta the excess of Section 3.1), n x K
 * row-major, to the host (synchronizes). */
pdr_status pdr_heights(pdr_ctx *ctx, double *host_out);

/* Copy the per-arc learning rates beta[m] of Algorithms 3 and 4 (caller's
 * arc order) to the host (synchronizes). */
pdr_status pdr_learning_rates(pdr_ctx *ctx, double *host_out);

/* Copy the GDM velocities v[m*K] (Algorithm 4) as FP64 to the host
 * (synchronizes). PDR_ERR_STATE for a context that is not PDR_GDM. */
pdr_status pdr_velocities(pdr_ctx *ctx, double *host_out);

/* Copy z log entries [first, first + count) to host_out (synchronizes).
 * Entry q is the objective of the q-th evaluation since init. The log keeps
 * the last z_log_capacity (default 2^20) evaluations; older entries return
 * PDR_ERR_INVALID. */
pdr_status pdr_z_log(pdr_ctx *ctx, int64_t first, int64_t count, double *host_out);

/* Switch the storage precision of the pseudo-flow f of Section 3.1 (and of
 * the GDM velocities of Algorithm 4). FP32_BULK -> FP64 widens the current
 * flows exactly (the FP64 "polish" phase); FP64 -> FP32_BULK rounds them. The
 * iteration counter, z_prev and learning rates are kept. PDR_ERR_INVALID for
 * an unknown precision or a row no arc kernel holds in the new precision (the
 * state is then unchanged). A batch member returns PDR_ERR_STATE: its batch
 * switches with pdr_batch_set_precision. */
pdr_status pdr_set_precision(pdr_ctx *ctx, int32_t precision);

/* Replace the run state: the pseudo-flow f[m*K] (Section 3.1; FP64, m x K
 * row-major in the caller's arc order, >= 0, finite; rounded to FP32 in
 * PDR_FP32_BULK), the learning rates beta[m] of Algorithms 3-4 (may be NULL
 * to keep), the GDM velocities v[m*K] of Algorithm 4 (finite; may be NULL to
 * keep; ignored by other methods), the iteration counter t and z_prev of
 * Algorithm 1's stop test (+inf to restart it). Used to resume a saved run.
 * PDR_ERR_INVALID for a NULL f (m > 0), t < 0, a NaN z_prev or an entry out
 * of range (nothing is changed); PDR_ERR_OOM if the staging buffer does not
 * fit. */
pdr_status pdr_set_state(pdr_ctx *ctx, const double *f, const double *beta, const double *v,
                         int64_t t, double z_prev);

/* pdr_set_state for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, checks and result as pdr_set_state, but no device memory is
 * allocated or freed. The host rows of f (and v) are staged, in chunks of whole
 * arc rows, through a 32 MiB device array (4,194,304 doubles) that the library
 * holds on every GPU it runs on until the process ends (its address is
 * resolved at pdr_init). Calls on one GPU share that array: calls that overlap
 * in time on one GPU (from several threads, contexts or streams) race and must
 * be serialized by the caller. PDR_ERR_INVALID also if one arc row of K
 * doubles exceeds the array. Synchronizes. */
pdr_status pdr_set_state_noalloc(pdr_ctx *ctx, const double *f, const double *beta,
                                 const double *v, int64_t t, double z_prev);

/* Measurement: run `sweeps` passes like pdr_sweep without a stop test,
 * recording HIP events around every kernel on the context stream. On return
 * (synchronized) kernel_ms[0] and kernel_ms[1] hold the summed device time in
 * milliseconds of the height kernel (which also evaluates the objective and
 * the stop test) and of the arc-update kernel. */
pdr_status pdr_profile_sweeps(pdr_ctx *ctx, int64_t sweeps, double *kernel_ms);

/* Reverse-mode gradient (adjoint) of the objective after T PDR-ESO passes.
 * Runs T passes from the current flows f^0 exactly as pdr_sweep(ctx, T, 0, 0)
 * (Algorithm 1 with Algorithm 2; the context ends at f^T) and returns
 * z(f^T) (Algorithm 1's objective) in *z_out and its gradient with respect to
 * the capacities, grad_u[m] (caller's arc order), and the demands, grad_d[K],
 * with f^0 held fixed. The pass map is piecewise linear (per arc: the
 * identity on the active commodities of an uncongested arc; minus the mean
 * over the active set A, weighted 1/(2 + |A|), on a congested one), so this is
 * the exact derivative away from the measure-zero set where an active set or
 * the congestion test changes (there: the one-sided derivative of the branch
 * the forward pass takes). Flows are kept every `checkpoint` passes
 * (0 = 16) and each segment is recomputed once during the reverse sweep;
 * working memory of about (T/checkpoint + checkpoint) m K + (checkpoint + 1)
 * n K doubles is allocated for the call. Needs method PDR_ESO, precision PDR_FP64
 * and a register-resident row (K <= 16,384; PDR_ERR_STATE otherwise). If z(f^T) is not finite it returns
 * PDR_ERR_NUMERIC (the context is then at f^T, as after pdr_sweep) and writes
 * no gradient. Synchronizes. */
pdr_status pdr_adjoint(pdr_ctx *ctx, int64_t T, int32_t checkpoint, double *z_out,
                       double *grad_u, double *grad_d);

/* Measurement: the HBM bandwidth of a plain copy on the current device.
 * Copies `bytes` (rounded down to 16) between two freshly allocated device
 * buffers `iters` times with a 16-byte-vector tiled copy kernel (k_copy) and
 * writes the mean read+write bandwidth in GB/s (2 * bytes per copy / time)
 * to *gbps. The buffers are freed before return. Context-free. */
pdr_status pdr_measure_copy(int64_t bytes, int32_t iters, double *gbps);

/* Query the automatic tiling: lanes per arc and vectors per lane of the arc
 * kernels, and the padded commodity stride Kp. A negative vec_per_lane means
 * the row is longer than a register-resident tiling holds: one block of
 * lanes_per_arc lanes per arc streams it in tiles of lanes_per_arc x
 * (-vec_per_lane) vectors of 16 bytes, recomputing its values from f and h on
 * each pass (ESO: one pass per step of the threshold iteration plus two;
 * AGD/GDM: two). */
pdr_status pdr_tiling(const pdr_ctx *ctx, int32_t *lanes_per_arc, int32_t *vec_per_lane,
                      int32_t *Kp);

/* Release the context and all its device memory. NULL is ignored, and so is a
 * batch member (pdr_batch_destroy releases members). */
void pdr_destroy(pdr_ctx *ctx);

/* Text of the last failure of ctx, or of the calling thread's last failed
 * pdr_init when ctx is NULL. Never NULL. */
const char *pdr_last_error(const pdr_ctx *ctx);

/* ---------------------------------------------------------------- batches
 * A batch sweeps many independent instances at once: every pass of
 * Algorithm 1, 3 or 4 runs for all of them in a handful of launches (one
 * height launch, one objective launch, one arc launch per tiling bucket),
 * captured in HIP graphs. Each instance keeps its own stop test, counters and
 * verdict; its results are read through its member context. */
typedef struct pdr_batch pdr_batch;

/* One instance of Section 1 (same arrays and rules as pdr_init). */
typedef struct {
    int32_t n, m;
    const int64_t *row_ptr; /* n+1 */
    const int32_t *col;     /* m heads */
    const double *u;        /* m capacities */
    int32_t K;
    const int32_t *s, *t;   /* K */
    const double *d;        /* K */
} pdr_instance;

/* A tiling bucket: the members whose arc kernels share one tiling. */
typedef struct {
    int32_t lanes_per_arc, vec_per_lane;
    int32_t instances;      /* members in the bucket */
    int32_t max_K;          /* largest commodity count among them */
    int64_t arcs;           /* their arcs in total */
    double ms;              /* arc-kernel time measured by the last pdr_batch_tune
                               (0 before tuning) */
} pdr_bucket_info;

/* Create a batch of B instances (deep copies; the caller keeps the arrays).
 * opt (NULL: defaults) applies to every member: method, precision, AGD/GDM
 * parameters, stream (NULL: the batch creates one; all members share it),
 * graph_sweeps (passes per captured batch graph), height_blocks (about this
 * many blocks for the batched height launch, shared by work; 0 = 32768;
 * more, smaller blocks balance uneven members better). Members keep 4096 z log
 * entries unless opt->z_log_capacity says otherwise. A failing instance fails
 * the whole call (status of that instance; pdr_batch_last_error(NULL) names it);
 * *out is NULL then. */
pdr_status pdr_batch_init(pdr_batch **out, int32_t B, const pdr_instance *insts,
                          const pdr_options *opt);

/* Up to max_sweeps passes for every member, each stopping on its own test
 * (eps_obj, z_target as in pdr_sweep). Stopped members skip the remaining
 * passes; the call returns early once every member has stopped.
 * Asynchronous on the batch stream. */
pdr_status pdr_batch_sweep(pdr_batch *batch, int64_t max_sweeps, double eps_obj,
                           double z_target);

/* The context of member `index` (0 <= index < B), for pdr_residual,
 * pdr_flows, pdr_z_log, pdr_learning_rates, pdr_velocities, pdr_set_state and
 * the other per-instance calls. Owned by the batch: pdr_destroy ignores it. */
pdr_status pdr_batch_member(pdr_batch *batch, int32_t index, pdr_ctx **ctx);

/* Number of members whose stop test has fired in the current sweep call
 * (synchronizes). */
pdr_status pdr_batch_stopped(pdr_batch *batch, int32_t *n_stopped);

/* Autotuner: for every tiling bucket, time each supported arc tiling that
 * covers the bucket's longest row (at most twice its size) with `reps`
 * launches of the batched arc kernel on the current heights, and give the
 * bucket's members the fastest; then time the batched height launch with
 * 8192, 16384, 32768 and 65536 blocks and pick the fastest. Finally `reps`
 * whole passes are timed with these choices and with the starting ones, and
 * the faster configuration stays (its height block count is written to
 * *height_blocks unless NULL; each bucket's `ms` is its arc launch time under
 * it). The run state is saved before and restored after (results are
 * unchanged); buckets that end with the same tiling merge. */
pdr_status pdr_batch_tune(pdr_batch *batch, int32_t reps, int64_t *height_blocks);

/* The current tiling buckets: *n_buckets receives their number, out[0 ..
 * min(max_buckets, *n_buckets)) their descriptions. */
pdr_status pdr_batch_buckets(pdr_batch *batch, int32_t max_buckets, pdr_bucket_info *out,
                             int32_t *n_buckets);

/* Measurement: `sweeps` batched passes without a stop test; kernel_ms[0] and
 * kernel_ms[1] receive the summed device time of the height + objective
 * launches and of all arc launches (HIP events on the batch stream;
 * synchronizes). */
pdr_status pdr_batch_profile_sweeps(pdr_batch *batch, int64_t sweeps, double *kernel_ms);

/* Switch every member's storage precision (as pdr_set_precision). */
pdr_status pdr_batch_set_precision(pdr_batch *batch, int32_t precision);

/* Text of the last failure of the batch, or of the thread's last failed
 * pdr_batch_init / pdr_init when batch is NULL. Never NULL. */
const char *pdr_batch_last_error(const pdr_batch *batch);

/* Release the batch, its members and all their device memory. */
void pdr_batch_destroy(pdr_batch *batch);

#ifdef __cplusplus
}
#endif

#endif /* PDR_H */
