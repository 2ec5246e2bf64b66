/*
 * ot_assoc.h - entropy-regularised optimal-transport device association on
 * AMD Instinct MI355X (gfx950).
 *
 * The library solves the regularised OT problem of eq. (5) of "Computational
 * Optimal Transport for 5G Massive C-RAN Device Association" (Sec. III-B):
 *
 *     min_pi  sum_ij C_ij pi_ij + eps sum_ij pi_ij (log pi_ij - 1)
 *     s.t.    sum_j pi_ij = a_i  (device traffic, the paper's p = lambda)
 *             sum_i pi_ij = b_j  (RRH load target, the paper's q)
 *
 * with the Sinkhorn iteration of Sec. III-B, written on log-domain dual
 * potentials f_i, g_j so that pi_ij = exp((f_i + g_j - C_ij) / eps) (the KKT
 * form of the Lagrangian, Sec. III-B). The cost is either a dense matrix, a
 * rate matrix R_ij with C_ij = (1/R_ij) / scale (Sec. IV, cost choice (ii):
 * load per unit traffic), or device/RRH geometry from which the rates of the
 * downlink model of Sec. II-A are regenerated on the fly and never stored.
 *
 * Conventions for every call
 *   - Return value: OT_OK (0), a warning (> 0) or an error (< 0). No
 *     exception, abort or exit crosses this boundary. On error the outputs are
 *     left untouched and ot_assoc_last_error() describes the cause.
 *   - Ownership: the caller owns every pointer it passes. Marginals,
 *     positions and host-memory matrices are copied into the handle's device
 *     workspace. One exception avoids copying large matrices: a DENSE or
 *     RATES matrix in device memory is referenced, not copied, and must stay
 *     valid and unchanged until the next call on the handle that takes a cost
 *     descriptor (ot_assoc_plan and ot_assoc_time_sweep read it again). The
 *     handle owns its device workspace, or borrows the caller's
 *     (ot_assoc_options.workspace) until ot_assoc_destroy.
 *   - Layout: matrices are row-major I x J (devices are rows, RRHs are
 *     columns) with leading dimension J, contiguous. Positions are I x 2 and
 *     J x 2 float arrays of (x, y) in metres.
 *   - Memory spaces: OT_MEM_HOST pointers are ordinary host memory;
 *     OT_MEM_DEVICE pointers are device memory of the handle's device
 *     (e.g. torch tensors' data_ptr()).
 *   - Synchrony: every call returns with its outputs final. Work is issued on
 *     the stream given at creation; with NULL the handle creates its own
 *     stream, which is ordered after earlier work on the legacy default stream.
 *   - Threading: a handle is used by one host thread at a time; distinct
 *     handles may be used concurrently.
 */
#ifndef OT_ASSOC_H
#define OT_ASSOC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ot_assoc ot_assoc; /* opaque solver handle */

typedef enum {
    OT_OK = 0,
    OT_WARN_MAXITER = 1, /* max_iter reached before tol; the result is valid */
    OT_EINVAL = -1,      /* an argument failed validation */
    OT_ENOMEM = -2,      /* device or host allocation failed */
    OT_EDEVICE = -3,     /* a HIP runtime call failed */
    OT_ENUMERIC = -4,    /* a non-finite residual or potential appeared */
    OT_ESTATE = -5       /* call made in the wrong state (e.g. plan before solve) */
} ot_status;

/* Cost kinds: DENSE (a matrix C_ij), RATES (a matrix R_ij, C = (1/R) / scale:
 * the load per unit traffic of Sec. IV, choice (ii)), GEOMETRY (the same cost
 * regenerated from positions with the downlink model below) and EUCLID
 * (C_ij = ||x_i - X_j|| / scale from the positions in `geom`, metres: Sec. IV
 * choice (i); the radio fields of `geom` are not used). */
typedef enum { OT_COST_DENSE = 0, OT_COST_RATES = 1, OT_COST_GEOMETRY = 2, OT_COST_EUCLID = 3 } ot_cost_kind;
typedef enum { OT_MEM_HOST = 0, OT_MEM_DEVICE = 1 } ot_mem;
typedef enum { OT_F32 = 0, OT_F64 = 1 } ot_dtype;

/* Arithmetic of the Sinkhorn sweeps. In both modes the potentials f, g are
 * kept in FP64 and the returned plan's statistics are computed in FP64.
 *   OT_PREC_FP32: sweeps use FP32 exponentials (and, for geometry costs, an
 *     FP32 cost functor) until the residual stalls or meets tol, then FP64
 *     sweeps polish the iterate until the FP64 residual meets tol.
 *   OT_PREC_FP64: every sweep is FP64. */
typedef enum { OT_PREC_FP32 = 0, OT_PREC_FP64 = 1 } ot_precision;

/* Downlink geometry (Sec. II-A): R_ij = W log2(1 + SINR_ji) with
 *   SINR_ji = P G_ji / (sum_{k != j} P G_ki + N0),
 *   G_ji = ref_gain * max(d_ij, min_dist_m)^(-pathloss_exp) * 10^(sigma X_ij / 10),
 * X_ij standard normal from the counter-based draw: h = SplitMix64 output
 * for state shadow_key ^ (i * 2^32 + j); u1, u2 = (high, low 32 bits of h
 * + 1/2) * 2^-32; X = sqrt(-2 ln u1) cos(2 pi u2) (Box-Muller). */
typedef struct {
    const float *dev_xy; /* I x 2, metres, in the descriptor's memory space */
    const float *rrh_xy; /* J x 2, metres, in the descriptor's memory space */
    double tx_power_w;   /* P (same for every RRH, all at full power) */
    double ref_gain;     /* K0: gain at 1 m */
    double pathloss_exp; /* alpha */
    double min_dist_m;   /* d_min */
    double shadow_sigma_db;
    double noise_w;      /* N0 */
    double bandwidth_hz; /* W */
    uint64_t shadow_key;
} ot_geometry;

/* The association instance (C, a, b). a (I) and b (J) are FP64 and live in
 * the memory space `mem`, as do `data` and the geometry arrays. */
typedef struct {
    ot_cost_kind kind;
    int64_t I, J;
    ot_mem mem;
    ot_dtype dtype;   /* element type of `data` (DENSE / RATES) */
    const void *data; /* DENSE: C_ij; RATES: R_ij > 0 */
    double scale;     /* RATES / GEOMETRY: C_ij = (1 / R_ij) / scale; EUCLID: C_ij = ||x_i - X_j|| / scale; scale > 0 */
    ot_geometry geom; /* GEOMETRY (all fields) and EUCLID (dev_xy, rrh_xy only) */
    int64_t ld;       /* DENSE / RATES: row stride of `data` in elements (0 = J, else >= J;
                         the padding entries are never used as costs) */
} ot_cost_desc;

typedef struct {
    int device;         /* HIP device ordinal */
    void *stream;       /* hipStream_t to issue work on; NULL = a stream owned by the handle */
    ot_precision precision;
    int polish_iters;   /* FP64 iterations run before the first exact check (default 1) */
    int chunk;          /* iterations per graph launch between host checks (default 8) */
    int use_graphs;     /* capture iteration chunks in HIP graphs (default 1) */
    int sweep_blocks;   /* 0 = choose automatically; else workgroups per sweep */
    int sweep_waves;    /* 0 = choose automatically; 4 or 8 waves per workgroup (dense FP32 costs) */
    int sweep_rows;     /* 0 = choose automatically; else 1, 2, 4 or 8 row steps in flight per wave */
    int sweep_lanes;    /* 0 = choose automatically; else 16, 32 or 64 lanes per row */
    int batch_tune;     /* ot_assoc_solve_batch: 1 (default) times the (waves, rows per part)
                           candidates once per batch shape (device and histogram of the
                           instances' log2 I, log2 J buckets) and keeps the default 8, 128 unless
                           another is 3 % faster; the choice is cached for the process and, when
                           the environment variable OT_ASSOC_TUNE_CACHE names a file, read from
                           and appended to it, so a later process takes it without timing (a
                           batch's results are bitwise reproducible for one choice); 0 uses 8, 128 */
    int persistent;     /* ot_assoc_solve, FP32 precision: 1 (default) runs the FP32 phase as one
                           cooperative launch that keeps the cost in LDS when the instance fits
                           (about I * J <= 9.8e6 cells on 256 CUs; dense FP32, FP32 rates or
                           geometry costs); 0 always uses graph-captured chunks of launches */
    int check_every;    /* ot_assoc_solve: the stop rule (residual below tol, or the FP32 residual
                           stalled) is evaluated only after iterations k that are multiples of
                           check_every (default 1: after every iteration); max_iter always stops.
                           The residual itself is formed in every sweep either way. */
    void* workspace;    /* optional caller-owned device memory on `device` (e.g. a torch tensor's
                           data_ptr()), at least ot_assoc_workspace_size() bytes, 256-byte aligned,
                           valid and not otherwise used until ot_assoc_destroy. Every device buffer
                           of the single-instance calls (ot_assoc_solve, _plan, _potentials,
                           _set_potentials, _cost_median, _materialize_cost, the loads, evaluation,
                           maxSINR and Alg. 2 calls and the timers) is carved from it, so those
                           calls allocate no device memory; bytes beyond the required size stage
                           host-memory DENSE / RATES matrices (a host matrix that does not fit
                           gives OT_ENOMEM). NULL (default): the library allocates one block of
                           that size itself. The batch, snapshot and serving engines keep their
                           own device pools either way. */
    size_t workspace_bytes; /* size of `workspace` (0 when workspace is NULL) */
    int snapshot_k_split;   /* ot_assoc_solve_snapshots: 1 (default) holds the stabilised kernel
                               in BF16 high and low parts (three BF16 products per GEMM step,
                               marginals about 1e-6 of the FP64 problem's); 0 in BF16 alone
                               (two products and half the kernel bytes per GEMM; 3e-4 on the
                               20000 x 400 x 64 layout, up to about 1.1e-3 on a distance cost) */
} ot_assoc_options;

typedef struct {
    int32_t iterations;      /* full (row + column) iterations of the returned iterate */
    int32_t fp64_iterations; /* FP64 sweeps run by the solve (polish and exact phases) */
    int32_t status;          /* ot_status of the solve */
    int32_t flags;           /* OT_RESULT_* bits */
    double marginal_violation; /* (sum_i |rowsum_i - a_i| + sum_j |colsum_j - b_j|) / sum(a), FP64 */
    double objective;          /* <C, pi> (transport cost) */
    double reg_objective;      /* <C, pi> + eps sum pi (log pi - 1), eq. (5) */
    double dual_objective;     /* <f, a> + <g, b> - eps sum pi */
    double seconds;            /* device time of the solve (HIP events) */
} ot_assoc_result;

/* ot_assoc_result.flags: the FP32 phase ran as one cooperative launch with the
   cost held in LDS (ot_assoc_options.persistent). */
#define OT_RESULT_PERSISTENT 1
/* ot_assoc_result.flags of a snapshot (ot_assoc_solve_snapshots): its status
   refers to tol on the BF16 problem, and the exact FP64 check of its
   potentials found a marginal violation of at least tol. */
#define OT_RESULT_CHECK_ABOVE_TOL 2

/* Fills *opt with the defaults listed above (device 0, default stream). */
ot_status ot_assoc_default_options(ot_assoc_options *opt);

/* Bytes of caller workspace (ot_assoc_options.workspace) a handle for
 * instances up to I_max x J_max needs: the O(I_max + J_max) vectors, the
 * per-workgroup partials, the cooperative phase's exchange block and a
 * work region of 2 (I_max + J_max) doubles. Pure host arithmetic (no
 * device is touched). Errors: OT_EINVAL for sizes out of range or NULL. */
ot_status ot_assoc_workspace_size(int64_t I_max, int64_t J_max, size_t *bytes);

/* Creates a handle able to solve instances up to I_max x J_max on
 * opt->device (opt NULL = defaults). Takes its device buffers from
 * opt->workspace when given, else allocates one block of
 * ot_assoc_workspace_size() bytes, plus (only without a caller workspace) an
 * I x ld staging matrix when a host-memory dense or rate cost is later passed.
 * Errors: OT_EINVAL (I_max or J_max out of range, a workspace that is too
 * small or misaligned, check_every < 0), OT_ENOMEM, OT_EDEVICE. */
ot_status ot_assoc_create(ot_assoc **h, int64_t I_max, int64_t J_max, const ot_assoc_options *opt);

/* Solves one instance (eq. (5) with the Sinkhorn iteration of Sec. III-B).
 *   eps > 0: regularisation strength; tol >= 0: stop when the total absolute
 *   marginal residual of the iterate, relative to sum(a), is below tol (the
 *   stop rule of the paper's Sinkhorn-vs-LP experiment); max_iter >= 1.
 *   warm_start != 0 starts from the handle's current potentials (those of
 *   the previous solve of the same shape, or set by ot_assoc_set_potentials);
 *   otherwise from g = 0 (the all-ones column scaling of the algorithm).
 * Validation (OT_EINVAL, nothing written): 1 <= I <= I_max, 1 <= J <= J_max;
 * a_i > 0, b_j > 0, all finite; |sum a - sum b| <= 1e-12 sum a; eps > 0 and
 * finite; tol >= 0; max_iter >= 1; scale > 0 for RATES / GEOMETRY / EUCLID; geometry
 * constants positive (noise_w >= 0, shadow_sigma_db >= 0). Dense costs and
 * rates are checked on the device (non-finite C or R <= 0 give OT_EINVAL).
 * Returns OT_OK, OT_WARN_MAXITER (result valid, tol not met) or an error.
 * `out` may be NULL. */
ot_status ot_assoc_solve(ot_assoc *h, const ot_cost_desc *cost, const double *a, const double *b, double eps,
                         double tol, int32_t max_iter, int warm_start, ot_assoc_result *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve of
 * ot_assoc_solve for a dense FP32 cost in device memory, with no handle. It
 * allocates nothing: every device buffer of the solve (potentials of both
 * parities, workgroup partials, the cooperative exchange block, the control
 * block) lives in a fixed array of about 9 MiB that the library holds on each
 * GPU it runs on until the process ends; the caller passes inputs and outputs.
 * Limits: 1 <= I <= 32768, 1 <= J <= 512 (larger instances give OT_EINVAL).
 *   device, stream: the GPU and the hipStream_t (NULL: the legacy default stream).
 *   C: I x ld FP32 row-major in device memory (ld = 0 means J); a (I), b (J):
 *   FP64 device marginals; f (I), g (J): FP64 device outputs, the potentials
 *   of the returned iterate (with warm_start != 0 also the starting potentials).
 *   eps, tol, max_iter and the validation are those of ot_assoc_solve; `out`
 *   (host, may be NULL) gets the result with seconds = 0 (no timing events).
 * Calls on one GPU share the array: calls that overlap on one GPU (several
 * host threads, or streams not ordered with each other) race and must be
 * serialised by the caller. Each call rewrites every part of the array it
 * reads. Errors: as ot_assoc_solve; the message is ot_assoc_last_error(NULL). */
ot_status ot_assoc_solve_static(int device, void *stream, const float *C, int64_t I, int64_t J, int64_t ld,
                                const double *a, const double *b, double eps, double tol, int32_t max_iter,
                                int warm_start, double *f, double *g, ot_assoc_result *out);

/* Writes the plan pi_ij = exp((f_i + g_j - C_ij) / eps) of the last
 * successful solve (the output step of the Sinkhorn algorithm) into the
 * caller's I x J row-major buffer of element type `dtype` in space `mem`,
 * computed in FP64 from the retained cost. Errors: OT_ESTATE before any
 * successful solve or after ot_assoc_cost_median / ot_assoc_materialize_cost
 * replaced the retained cost, OT_EINVAL for NULL pi. */
ot_status ot_assoc_plan(ot_assoc *h, void *pi, ot_mem mem, ot_dtype dtype);

/* Asks the following solves on the handle to write their plan (as
 * ot_assoc_plan would, element type `dtype`) into the device buffer pi of
 * `capacity` elements, from the cells their final exact check computes
 * anyway, so that the plan takes no pass over the cost of its own (Sec. III-B
 * output step). A solve writes it only when its I x J fits in capacity; pi
 * must stay valid while it is set; NULL stops it. A following
 * ot_assoc_plan(h, pi, OT_MEM_DEVICE, dtype) with the same buffer and type
 * after such a solve returns at once; any other plan call, and a solve that
 * ends without that check (rejected inputs, a numeric failure) or did not
 * write it, computes the plan as before. The solves of ot_assoc_adaptive do
 * not write it. Errors: OT_EINVAL for a bad dtype. */
ot_status ot_assoc_set_plan_output(ot_assoc *h, void *pi, ot_dtype dtype, int64_t capacity);

/* Copies out the FP64 potentials (f: I, g: J) of the last solve. Either
 * pointer may be NULL. Errors: OT_ESTATE before any solve. */
ot_status ot_assoc_potentials(ot_assoc *h, double *f, double *g, ot_mem mem);

/* Sets the potentials used by the next warm-started solve of an I x J
 * instance. Errors: OT_EINVAL on sizes out of range or NULL pointers. */
ot_status ot_assoc_set_potentials(ot_assoc *h, const double *f, const double *g, int64_t I, int64_t J, ot_mem mem);

/* Lower median (element floor((IJ - 1) / 2) in sorted order) of the I*J
 * values 1/R_ij of a RATES or GEOMETRY descriptor (of the distances
 * ||x_i - X_j|| of an EUCLID one), computed on the device in FP32 by radix
 * selection over the regenerated values; the normalisation of the cost
 * C = (1/R)/median. The descriptor's `scale` is ignored.
 * Errors: OT_EINVAL (bad descriptor or sizes), OT_EDEVICE. */
ot_status ot_assoc_cost_median(ot_assoc *h, const ot_cost_desc *cost, double *median_out);

/* Writes the FP32 cost C_ij of a RATES, GEOMETRY or EUCLID descriptor into the
 * caller's device buffer C (I x J row-major): the materialised form of the
 * cost that the geometry sweeps regenerate on the fly. */
ot_status ot_assoc_materialize_cost(ot_assoc *h, const ot_cost_desc *cost, float *C_dev);

/* ------------------------------------------------ association quality --
 * Loads and completion times of Sec. II-B, the maxSINR rule of Sec. II-A /
 * IV and the Adaptive Sinkhorn Association of Sec. IV (Alg. 2). The cost is
 * read as the load per unit traffic, C_ij = (1/R_ij) / scale (cost choice
 * (ii) of Sec. IV): then the transport plan x of a solve with row sums
 * a_i = lambda_i / sum(lambda) gives the association pi_ij = x_ij / a_i and
 *   rho_j = sum_i lambda_i pi_ij / (mu R_ij) = kappa load_j,
 *   load_j = sum_i C_ij x_ij,  kappa = sum(lambda) scale / mu,
 * with 1/mu the mean job size. */

/* Per-RRH load of the last successful solve's plan: load_j = sum_i C_ij x_ij
 * in FP64 (the FP64 cost, x = exp((f + g - C)/eps)). loads: J doubles in
 * `mem`. After ot_assoc_adaptive (J <= 512) the loads were summed by the
 * solves' final exact checks and are copied out; otherwise they take one
 * pass over the cost. Errors: OT_ESTATE before a successful solve (or after
 * a call that replaced the handle's cost). */
ot_status ot_assoc_rrh_loads(ot_assoc *h, double *loads, ot_mem mem);

typedef struct {
    double max_rho;             /* max_j rho_j */
    double mean_completion;     /* (1/I) sum_i T_i in the unit of tau; +inf if a device uses an RRH with rho >= 1 */
    double objective;           /* sum_i T_i, the objective of eq. (1); +inf as above */
    int32_t overloaded_rrhs;    /* RRHs with rho_j >= 1 */
    int32_t devices_overloaded; /* devices with a positive share on such an RRH */
} ot_eval_result;

/* Association quality of the last successful solve (Sec. II-B):
 *   rho_j = kappa load_j;  E[N_j] = rho_j / (1 - rho_j) (mean number of jobs
 *   under processor sharing; +inf when rho_j >= 1);
 *   T_i = (tau / a_i) sum_j C_ij x_ij / (1 - rho_j), the average completion
 *   time of device i (tau = scale / mu for C = (1/R) / scale).
 * rho and EN: J doubles in `mem` (either may be NULL); out is required.
 * Errors: OT_EINVAL (kappa or tau not positive and finite, out NULL),
 * OT_ESTATE before a successful solve. */
ot_status ot_assoc_evaluate(ot_assoc *h, double kappa, double tau, double *rho, double *EN, ot_mem mem,
                            ot_eval_result *out);

/* maxSINR rule: every device to the RRH of lowest cost, i.e. highest rate
 * (lowest index on ties; decided on the FP64 cost), and the traffic it
 * induces, Lambda_j = sum of a_i over the devices associated to j (the RRH
 * marginal q of Lemma 1). a: I doubles; assoc: I int32 (may be NULL);
 * Lambda: J doubles; all in cost->mem. Replaces the handle's retained cost:
 * a later ot_assoc_plan / loads / evaluate needs a new solve.
 * Errors: as ot_assoc_solve for the descriptor and a (values checked). */
ot_status ot_assoc_maxsinr(ot_assoc *h, const ot_cost_desc *cost, const double *a, int32_t *assoc, double *Lambda);

typedef struct {
    int32_t solves;          /* Sinkhorn solves run */
    int32_t best;            /* index (from 0) of the returned solve */
    int32_t iterations;      /* Sinkhorn iterations over all solves */
    int32_t status;          /* ot_status of the returned solve */
    double max_load;         /* max_j load_j of the returned solve */
    double first_max_load;   /* max_j load_j of the first solve (q_j = sum(a) / J) */
    double delta;            /* the step used */
} ot_adaptive_result;

/* Adaptive Sinkhorn Association (Sec. IV, Alg. 2): starting from q_j =
 * sum(a) / J, solve (eps, tol, max_iter as ot_assoc_solve), find the RRH of
 * highest load j* (lowest index on ties), move delta of its traffic to the
 * others (q_j* -= delta, q_j += delta / (J - 1)), and repeat. Readings of
 * the paper's open points: delta <= 0 selects 0.01 sum(a) / J; the loop
 * stops when a solve's maximum load does not fall below the best one so far,
 * when q_j* - delta would not stay positive, or after max_outer solves; the
 * result is the solve with the lowest maximum load, whose potentials and
 * plan the handle then holds (ot_assoc_plan / potentials / loads /
 * evaluate), solved for the returned q. Solves after the first warm-start
 * from the previous one. q: J doubles on the HOST (output); jstar: max_outer
 * int32 on the host, the j* picked after each solve (may be NULL).
 * Errors: as ot_assoc_solve; OT_EINVAL for max_outer < 1 or q / out NULL. */
ot_status ot_assoc_adaptive(ot_assoc *h, const ot_cost_desc *cost, const double *a, double eps, double tol,
                            int32_t max_iter, double delta, int32_t max_outer, double *q, int32_t *jstar,
                            ot_adaptive_result *out);

/* (instrumentation) Average device duration, in milliseconds, of one launch
 * of the fused sweep kernel that the last successful solve used (same cost,
 * shape and launch configuration; FP32 exponentials if fp64 == 0, else FP64).
 * Runs `reps` (1..4096) extra sweeps back to back on the handle's stream
 * between one pair of HIP events (so the figure includes the gap between
 * dependent launches), then restores the solve's potentials and control
 * state, so a later ot_assoc_plan / ot_assoc_potentials is unaffected.
 * Errors: OT_ESTATE before a successful solve, OT_EINVAL for bad reps. */
ot_status ot_assoc_time_sweep(ot_assoc *h, int32_t reps, int fp64, double *ms_per_launch);

/* (instrumentation) HBM read ceiling: average device duration, in
 * milliseconds, of a read-only streaming kernel over `bytes` (a multiple of
 * 16, >= 16) of device memory at `buf` (16-byte aligned; only read), run
 * `reps` (1..4096) times back to back on the handle's stream between one pair
 * of HIP events. Bytes / duration is the read bandwidth the device sustains
 * for a plain coalesced stream, the ceiling beside which the sweeps' HBM
 * figures are read. Errors: OT_EINVAL for bad arguments, OT_EDEVICE. */
ot_status ot_assoc_time_read(ot_assoc *h, const void *buf, size_t bytes, int32_t reps, double *ms_per_launch);

/* (test hook) Makes the next cooperative FP32 launch started by the calling
 * thread withhold the new g at its `iteration`-th iteration (1-based; 0
 * cancels) and bound every wait at a few milliseconds, so that the waits
 * after it end by giving up: every workgroup then leaves the kernel normally
 * and that solve returns OT_EDEVICE ("gave up waiting") with no solution
 * held; the next solve on the handle runs as usual. For tests of the
 * give-up path. Errors: OT_EINVAL for a negative iteration. */
ot_status ot_assoc_test_hold_exchange(int32_t iteration);

/* (instrumentation) Device duration, in milliseconds, of the cooperative
 * launch that ran the FP32 phase of the last successful solve (HIP events on
 * the handle's stream right around that one launch: the LDS fill and every
 * FP32 iteration), and the number of FP32 iterations it ran.
 * Errors: OT_ESTATE if the last solve did not use the cooperative launch
 * (see ot_assoc_result.flags). */
ot_status ot_assoc_fast_phase_time(ot_assoc *h, double *ms, int32_t *iterations);

/* (instrumentation) Number of device allocations (hipMalloc) the library has
 * made in this process so far, over all handles and engines: a caller that
 * passes a workspace can check that its solves allocate nothing. */
int64_t ot_assoc_device_allocations(void);

/* Frees the handle and its device workspace (a caller's workspace is left
 * to the caller). NULL-safe. */
void ot_assoc_destroy(ot_assoc *h);

/* Human-readable description of the last error on this handle ("" if none).
 * The string is owned by the handle and valid until its next call. With
 * h == NULL it describes the last failed ot_assoc_create or
 * ot_assoc_solve_static on this thread. */
const char *ot_assoc_last_error(const ot_assoc *h);

/* ------------------------------------------------------------ batched solves
 * Many independent association instances solved together, as one engine:
 * each is the problem of eq. (5) with its own cost, marginals and eps, solved
 * by the same Sinkhorn iterations (Sec. III-B) and the same phases as
 * ot_assoc_solve with OT_PREC_FP32 (FP32 sweeps, FP64 polish, exact FP64
 * check, FP64 sweeps if the check misses tol). Instances advance together,
 * three persistent launches per iteration, captured in HIP graphs; an
 * instance leaves the work lists as soon as it is done, so uneven sizes and
 * iteration counts cost only their own work.
 *
 * Every cost is held as a padded FP32 row-major matrix: a DENSE FP32 matrix in
 * device memory whose J and row stride (ld, else J) are multiples of 4 and whose
 * base is 16-byte aligned is referenced in place (keep it valid until the
 * next batch on the handle); other DENSE / RATES inputs (host or device, FP32
 * or FP64) are converted, GEOMETRY and EUCLID inputs (device memory; positions
 * read at admission) are materialised (scale <= 0 takes the median of 1/R, or
 * of the distances, which
 * waits on the host). Cost values are not screened: a non-finite cost ends
 * that instance with OT_ENUMERIC. 1 <= J <= 512; a[k] and b[k] live in costs[k].mem
 * (GEOMETRY, EUCLID: device memory). eps[k] > 0 per instance; tol and max_iter are
 * shared. out[k] (may be NULL) receives instance k's result; `seconds` is the
 * device time of the whole batch.
 *
 * Returns OT_OK when every instance met tol, OT_WARN_MAXITER if some stopped
 * at max_iter, OT_ENUMERIC if some failed numerically (see out[k].status),
 * OT_EINVAL / OT_ENOMEM with nothing solved when an input is invalid or the
 * batch does not fit (4096 instances, 2^20 row parts of 64 rows, 90% of free
 * device memory). The previous batch's instances are released first. */
ot_status ot_assoc_solve_batch(ot_assoc *h, int n, const ot_cost_desc *costs, const double *const *a,
                               const double *const *b, const double *eps, double tol, int32_t max_iter,
                               ot_assoc_result *out);

/* Launch configuration the last batch ran with (chosen by the autotuner when
 * batch_tune is set): waves per FP32 sweep workgroup and rows per work item.
 * OT_ESTATE before any batch. */
ot_status ot_assoc_batch_config(ot_assoc *h, int *waves, int *rows_per_part);

/* Potentials (f: I, g: J, FP64) of instance k of the last batch, into host or
 * device memory. OT_ESTATE before a batch, OT_EINVAL for a bad k. */
ot_status ot_assoc_batch_potentials(ot_assoc *h, int k, double *f, double *g, ot_mem mem);

/* Plan of instance k of the last batch, pi_ij = exp((f_i + g_j - C_ij) / eps)
 * (the KKT form of Sec. III-B) with the FP32 cost the batch used, I x J
 * row-major, FP32 or FP64. */
ot_status ot_assoc_batch_plan(ot_assoc *h, int k, void *pi, ot_mem mem, ot_dtype dtype);

/* -------------------------------------------------------- traffic snapshots
 * B (1..64) traffic snapshots of one layout: marginals a_s (row s of A, B x I
 * row-major) over one cost C and one RRH marginal b, each the problem of
 * eq. (5). Solved together in the scaling form of the Sinkhorn iteration
 * (Sec. III-B): a reference solve of the mean snapshot (single-instance path)
 * gives potentials (fbar, gbar) that stabilise the kernel
 * K = exp((fbar + gbar - C) / eps); the half-steps u_s = a_s / (K v_s) and
 * v_s = b / (K^T u_s) of all snapshots are two GEMMs on the matrix cores
 * with BF16 operands: K, u and v each split into high and low BF16 parts
 * (about 16 significant bits), three products per step (hi.hi, hi.lo,
 * lo.hi), FP32 accumulation. The iteration stops when every snapshot's column
 * residual of the BF16 problem is below tol (relative to sum a_s) or after
 * max_iter iterations. out[s] reports the common iteration count and the
 * exact FP64 check of snapshot s's potentials fbar + eps ln u_s,
 * gbar + eps ln v_s against C (for RATES / GEOMETRY / EUCLID, its FP32 materialised
 * form): the violation reflects the split-BF16 arithmetic and FP32
 * accumulation (well below 1e-3), not tol. out[s].status is OT_OK when the
 * BF16 problem met tol; out[s].flags has OT_RESULT_CHECK_ABOVE_TOL when the
 * exact check's violation is nevertheless at least tol.
 * A and b live in cost->mem (GEOMETRY, EUCLID: device). Afterwards the handle's
 * single-instance state (ot_assoc_plan / ot_assoc_potentials) is the
 * reference solve, converged to a marginal violation below 1e-3 only (it
 * conditions the kernel; the snapshots are solved to tol). Errors: OT_EINVAL for bad arguments or marginals,
 * OT_ENOMEM, OT_EDEVICE. */
ot_status ot_assoc_solve_snapshots(ot_assoc *h, const ot_cost_desc *cost, int B, const double *A, const double *b,
                                   double eps, double tol, int32_t max_iter, ot_assoc_result *out);

/* Potentials of snapshot s of the last snapshot solve (f: I, g: J, FP64). */
ot_status ot_assoc_snapshot_potentials(ot_assoc *h, int s, double *f, double *g, ot_mem mem);

/* ------------------------------------------------------------------ serving
 * A request server over the batched engine: requests (one association solve
 * per scheduling instant) are queued on submit and admitted, oldest first, as
 * instance slots, work-list room and the device-memory budget allow, while
 * earlier requests are still iterating; every ot_serve_progress call admits
 * what fits, runs one chunk of iterations of everything in flight and returns
 * the requests that finished. A request with a nonzero layout_key starts from
 * the potentials that the last finished request of the same key (same I x J)
 * left resident, and leaves its own; resident sets are evicted least recently
 * used first when memory or keep_layouts runs out. A request's result does
 * not depend on what else is in flight (fixed-order reductions per instance).
 * Every buffer a request points to must stay valid and unchanged until its
 * completion is returned. One thread per server. */
typedef struct ot_serve ot_serve;

typedef struct {
    int device;
    void *stream;          /* hipStream_t; NULL = a stream owned by the server */
    double budget_bytes;   /* device memory for requests and resident potentials
                              (0 = 90% of free memory, at most 256 GiB) */
    int max_slots;         /* requests in flight (0 = 1024) */
    int max_items;         /* row parts in flight (0 = 2^19) */
    int polish_iters;      /* FP64 sweeps before the exact check (default 1) */
    int sweep_waves;       /* 4 or 8 waves per sweep workgroup (default 8) */
    int rows_per_part;     /* 64, 128 or 256 rows per work item (default 128) */
    int keep_layouts;      /* resident potential sets kept (0 = 4096) */
} ot_serve_options;

typedef struct {
    ot_cost_desc cost;     /* as for ot_assoc_solve_batch */
    const double *a, *b;   /* marginals, in cost.mem (GEOMETRY, EUCLID: device memory) */
    double eps, tol;
    int32_t max_iter;
    int32_t reserved;
    uint64_t layout_key;   /* 0: cold start; else warm start / keep potentials under this key */
    uint64_t user_tag;     /* returned with the completion */
} ot_request;

typedef struct {
    uint64_t ticket, user_tag, layout_key;
    int32_t warm;          /* 1 if the solve started from resident potentials */
    int32_t reserved;
    double t_submit, t_admit, t_done; /* host steady clock, seconds (ot_serve_now) */
    ot_assoc_result result; /* result.status < 0: the request was rejected or failed */
} ot_completion;

ot_status ot_serve_default_options(ot_serve_options *opt);
/* Errors: OT_EINVAL for bad options, OT_EDEVICE / OT_ENOMEM from the device. */
ot_status ot_serve_create(ot_serve **s, const ot_serve_options *opt);
/* Queues a request (validated for shape and settings now, marginals at
 * admission); *ticket identifies its completion. Never waits on the GPU. */
ot_status ot_serve_submit(ot_serve *s, const ot_request *req, uint64_t *ticket);
/* Admits, runs one chunk, and writes up to max_out completions to out
 * (*n_out of them); later completions wait for the next call. A request that
 * can never fit is completed with OT_ENOMEM. */
ot_status ot_serve_progress(ot_serve *s, ot_completion *out, int max_out, int *n_out);
/* Requests queued / in flight, resident potential sets, device bytes held. */
ot_status ot_serve_counts(const ot_serve *s, int *queued, int *running, int *resident, double *bytes_in_use);
/* Resident potentials of a layout (f: I, g: J), into host or device memory. */
ot_status ot_serve_potentials(ot_serve *s, uint64_t layout_key, double *f, double *g, ot_mem mem);
/* The clock of the completion timestamps. */
double ot_serve_now(void);
const char *ot_serve_last_error(const ot_serve *s);
void ot_serve_destroy(ot_serve *s);

#ifdef __cplusplus
}
#endif

#endif /* OT_ASSOC_H */
