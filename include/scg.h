/*
 * libscg: total-variation superiorized conjugate gradient for parallel-beam
 * CT on AMD Instinct MI355X (gfx950).
 *
 * The library solves the least-squares problem of the paper's Introduction,
 *     minimise f(x) = 1/2 ||y - A x||^2,
 * with the superiorized CG family of its third section: the iteration stops
 * as soon as f(x_{k-1/2}) <= eps, and every step is preceded by a TV-reducing
 * perturbation x_{k+1/2} = x_k + gamma_k v_k (eq. superiorization, with
 * gamma taken from gamma_l = gamma0 a^l, eq. gamma_sequence).
 *
 * Geometry (the paper fixes parallel rays, angles uniform over [0, 180 deg)
 * and the image/detector sizes; the remaining conventions are this
 * library's): the image has N x N unit pixels, pixel (i, j) (row i from the
 * top, column j from the left) has centre x_j = j - (N-1)/2,
 * y_i = (N-1)/2 - i and flat index i*N + j. Angle a has theta_a = a*pi/n_a,
 * bin b has centre t_b = b - (n_b-1)/2, ray (a, b) is the line
 * x cos theta_a + y sin theta_a = t_b, and sinograms are angle-major with flat
 * index a*n_b + b. A's entry for (ray, pixel) is the length of the ray inside
 * the pixel's closed unit square; a ray lying on a pixel edge gives each side
 * half of it.
 *
 * Conventions for every entry point:
 *   - Return value: SCG_OK (0) or a negative status; nothing throws across
 *     the ABI. scg_strerror() names a status.
 *   - Vectors are raw device pointers owned by the caller. The library never
 *     frees caller memory and never keeps a caller pointer after returning.
 *   - Element type follows the precision argument: SCG_F32 -> float,
 *     SCG_F64 -> double. In SCG_F32 the operators, TV and vector updates run
 *     in FP32 while the CG scalars (alpha, beta), the residual norm and the
 *     eps test are accumulated and evaluated in FP64.
 *   - `stream` is a hipStream_t (NULL = the default stream). Work is enqueued
 *     on it; calls that return host scalars synchronise it.
 *   - A plan owns small device scratch buffers: calls that share a plan must
 *     not overlap in time (use one plan per concurrent stream).
 */
#ifndef SCG_H
#define SCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define SCG_OK            0
#define SCG_EINVAL       -1   /* invalid argument (size, pointer, parameter)     */
#define SCG_ENOMEM       -2   /* device allocation failed / workspace too small  */
#define SCG_EDEVICE      -3   /* HIP runtime error                               */
#define SCG_ENOCONV      -4   /* max_iter steps done and f > eps still holds     */
#define SCG_ENAN         -5   /* a non-finite CG scalar appeared                 */
#define SCG_EBREAKDOWN   -6   /* ||A p||^2 = 0 for a new direction p             */
#define SCG_EAGAIN       -7   /* no free slot / memory in a batch                */
#define SCG_EINPROGRESS  -8   /* batch ticket still running                      */
#define SCG_ENOTFOUND    -9   /* unknown batch ticket                            */

/* ---- enums ------------------------------------------------------------- */
typedef enum { SCG_F32 = 0, SCG_F64 = 1 } scg_prec;

typedef enum {
    SCG_CG = 0,      /* Alg. CG (unsuperiorized, recursive gradient)           */
    SCG_S_CG = 1,    /* Alg. S-CG with CG-PR-STEP                              */
    SCG_S_CG_CD = 2, /* Alg. S-CG-CD with CG-CD-STEP (conjugate-descent beta)  */
    SCG_S_PCG = 3,   /* Alg. S-PCG with PCG-PR-STEP (filtered preconditioner)  */
    SCG_S_CG_K = 4,  /* Alg. S-CG-K: perturbed(x_k), then CG-K (K = restart_k  */
                     /* CG-STEPs) restarted from the perturbed point           */
    SCG_S_CG_3OP = 5,/* Alg. S-CG with CG-PR-STEP evaluated with q = A p kept  */
                     /* by linearity: beta = (A g')^T q / ||q||^2 and          */
                     /* q' = -A g' + beta q, so a step applies A twice and A^T */
                     /* once (h = A^T A p is never formed). The same iterates  */
                     /* as SCG_S_CG in exact arithmetic; q accumulates the     */
                     /* rounding of its recursion (Sec. 3 (CG-PR-STEP))        */
    SCG_PCG = 6,     /* Alg. PCG with PCG-STEP (unsuperiorized): z = M g is   */
                     /* the filtered backprojection of the residual, which is */
                     /* carried recursively with g; f is evaluated at every x  */
    SCG_S_PCG_K = 7  /* Alg. S-PCG-K: perturbed(x_k), then PCG-K (K =         */
                     /* restart_k PCG-STEPs) restarted from the perturbed      */
                     /* point                                                  */
} scg_variant;

/* flags of scg_params.flags */
#define SCG_FLAG_NO_PERTURB 1u   /* skip perturbed(): x_{k+1/2} = x_k           */

/* ---- plain structs ----------------------------------------------------- */
typedef struct {
    int32_t n;          /* image side N (N x N pixels), >= 2                    */
    int32_t n_angles;   /* angles uniform over [0, 180 deg), >= 1              */
    int32_t n_bins;     /* unit-width detector bins, >= 1                       */
} scg_geom;

typedef struct {
    int32_t variant;     /* scg_variant                                           */
    int32_t prec;        /* scg_prec                                              */
    double  eps;         /* stop when f(x_{k-1/2}) <= eps; must be > 0            */
    double  gamma0;      /* gamma_l = gamma0 * a^l; >= 0 (0: no perturbation)     */
    double  a;           /* 0 < a < 1 (the paper's experiments use 0.975)         */
    int32_t max_iter;    /* cap on the number of steps after the initial one     */
    int32_t max_trials;  /* cap on trials of perturbed() per step, 1..1024        */
    double  tv_kappa;    /* 0: exact isotropic TV; > 0: sqrt(a^2+b^2+kappa^2)     */
    double  precond_mu;  /* mu of the filter c(w) (S-PCG); <= 0 selects 2 pi / P  */
    uint32_t flags;      /* SCG_FLAG_*                                            */
    int32_t restart_k;   /* K of SCG_S_CG_K / SCG_S_PCG_K: steps per pass, 1..64   */
                         /* (default 2)                                        */
} scg_params;

typedef struct {
    int32_t status;       /* SCG_OK, SCG_ENOCONV, SCG_ENAN or SCG_EBREAKDOWN      */
    int32_t k;            /* the paper's counter k when the loop ended; the       */
                          /* output is x_{k-1/2} (SCG_S_CG_K, SCG_S_PCG_K: passes */
                          /* made, 0 when f(x0) <= eps; SCG_CG, SCG_PCG: steps    */
                          /* made, the output is x_k)                             */
    int32_t steps;        /* steps executed after the initial one (passes for    */
                          /* SCG_S_CG_K and SCG_S_PCG_K)                          */
    int32_t trials_total; /* TV trials made by perturbed()                        */
    int32_t ell;          /* final value of the gamma counter l                   */
    int32_t reserved;
    double  f_out;        /* f at the output (FP64 accumulation)                  */
    double  tv_out;       /* TV of the output image (terms summed in FP64)        */
} scg_report;

/* One entry per step k = 1, 2, ... (the step that forms x_{k+1/2}, x_{k+1}). */
typedef struct {
    int32_t k;
    int32_t accepted;     /* index of the accepted trial in this step, -1: none   */
    int32_t trials;       /* trials made in this step                             */
    int32_t ell;          /* l after the step's perturbation                      */
    double  f_half;       /* f(x_{k+1/2})                                         */
    double  tv_x;         /* TV(x_k)                                              */
    double  gamma;        /* step used (0: unperturbed)                           */
    double  beta;
    double  alpha;
} scg_trace_entry;

typedef struct scg_plan scg_plan;

/* ---- plans ------------------------------------------------------------- */

/* Creates a plan for geometry *g on HIP device `device`: FP64 angle tables
 * (cos/sin evaluated in double and snapped to 0/+-1 within 1e-12) are built on
 * the host and uploaded, and the plan's scratch is allocated. *out is set to
 * NULL on failure. Errors: SCG_EINVAL (sizes: 2 <= N <= 2880, and the
 * projector's (angle group, 128-bin chunk) blocks at most 65536, about
 * n_angles / 4 * ceil(n_bins / 128)), SCG_ENOMEM, SCG_EDEVICE. The
 * preconditioning filter (SCG_S_PCG, SCG_PCG, SCG_S_PCG_K, scg_filter)
 * transforms P = 2^ceil(log2(2 n_bins)) complex points in LDS: it needs
 * n_bins <= 8192 in SCG_F32 and n_bins <= 4096 in SCG_F64 and returns
 * SCG_EINVAL otherwise. Its tables are allocated here, so solves allocate
 * nothing for it. */
int scg_plan_create(const scg_geom *g, int device, scg_plan **out);

/* Frees a plan and its device memory (NULL is accepted). The caller must
 * have synchronised every stream that used the plan. */
void scg_plan_destroy(scg_plan *plan);

/* Device bytes the caller must provide to scg_solve for these parameters. */
int scg_workspace_bytes(const scg_plan *plan, const scg_params *params, size_t *bytes);

/* ---- operators --------------------------------------------------------- */

/* y = A x (the discrete line integrals of the Introduction). x: N*N
 * elements, y: n_angles*n_bins elements, both device pointers of the type
 * given by `prec`. The plan's scratch holds a padded copy of x. */
int scg_project(scg_plan *plan, int prec, const void *x, void *y, void *stream);

/* x = A^T y, the exact transpose of scg_project (a pixel-driven gather). */
int scg_backproject(scg_plan *plan, int prec, const void *y, void *x, void *stream);

/* TV(x) (isotropic forward differences over the (N-1)^2 interior terms,
 * sqrt(a^2 + b^2 + kappa^2) per term) into *tv_host, and optionally a
 * subgradient of TV at x into s (device, N*N elements; NULL to skip). Terms
 * are computed in the precision `prec` and summed in FP64. Synchronises. */
int scg_tv(scg_plan *plan, int prec, const void *x, double kappa, void *s, double *tv_host,
           void *stream);

/* The preconditioning filter F^T C F of the paper's Filters for
 * Preconditioning section applied to every projection of r: zero padding to
 * P = 2^ceil(log2(2 n_bins)) samples, DFT, multiplication by
 * c(w) = (|w| + mu)(0.54 + 0.46 cos w) at w_m = 2 pi m / P, inverse DFT,
 * first n_bins samples kept. mu <= 0 selects 2 pi / P. r and out: device,
 * n_angles * n_bins elements of the precision's type. The transform runs
 * in the precision `prec` (radix-2, twiddles from FP64 host values).
 * SCG_EINVAL: n_bins above the precision's bound (see scg_plan_create). A
 * plan holds one spectrum (one mu) per precision at a time: a call with
 * another mu rewrites it, so calls and solves that share a plan and
 * precision must not overlap with different mu (a batch refuses such a
 * submit with SCG_EINVAL). */
int scg_filter(scg_plan *plan, int prec, double mu, const void *r, void *out, void *stream);

/* ---- solver ------------------------------------------------------------ */

/* Runs params->variant from x0 on data y (device, n_angles*n_bins) and
 * writes the output x_{k-1/2} to x_out (device, N*N). x0 may be NULL
 * (the zero image). ws/ws_bytes: device workspace of at least
 * scg_workspace_bytes(); the library allocates nothing during the solve.
 * rep (host) receives the report. trace (host, may be NULL) receives up to
 * trace_cap entries, one per step. forced (host, may be NULL) replays
 * perturbation decisions: for step k, forced[2(k-1)] is the number of trials
 * and forced[2(k-1)+1] the accepted trial index (-1: none) to use instead of
 * the TV tests, for the first forced_len steps. Returns rep->status on a
 * completed solve, or an argument/device error. Synchronises `stream`. */
int scg_solve(scg_plan *plan, const scg_params *params, const void *y, const void *x0,
              void *x_out, void *ws, size_t ws_bytes, scg_report *rep,
              scg_trace_entry *trace, int32_t trace_cap, const int32_t *forced,
              int32_t forced_len, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc): scg_solve with
 * the workspace taken from a static device array of the library instead of
 * a caller buffer. Same arguments, results and statuses as scg_solve
 * (bitwise the same output and report for the same inputs and launch
 * shapes), without ws/ws_bytes; kernel timing (scg_profile) is not applied.
 * The call allocates no device memory. Limit: scg_workspace_bytes() for
 * the parameters must not exceed scg_static_workspace_bytes() (32 MiB: FP32
 * up to about 700 x 700 pixels, FP64 up to 512 x 512 with 720 x 729 rays);
 * larger problems return SCG_ENOMEM. Each device holds one such array for
 * the life of the process, shared by every call on that device, which
 * keeps the previous call's contents (the solve initialises everything it
 * reads). Calls that overlap in time on one device race on it: callers
 * serialise them (one stream, or waits between streams). */
int scg_solve_static(scg_plan *plan, const scg_params *params, const void *y, const void *x0,
                     void *x_out, scg_report *rep, scg_trace_entry *trace, int32_t trace_cap,
                     const int32_t *forced, int32_t forced_len, void *stream);

/* Bytes of the static workspace of scg_solve_static (per device). */
size_t scg_static_workspace_bytes(void);

/* ---- launch shapes ----------------------------------------------------- */

/* Launch shapes of the two operators; results do not depend on them beyond
 * FP rounding order (the backprojector's angle split adds the groups' partial
 * sums in a fixed order, so each choice is itself deterministic). The
 * mirrored backprojector takes angle theta's parameters for pi - theta (a
 * trig table made exactly symmetric about the vertical axis), which moves
 * A^T by about 1e-13 relative in FP64; in the filtered variants' solves only
 * h = A^T q runs mirrored (their two-sinogram backprojection and z' = A^T r~
 * with its dot run on every tile). The mirrored projector does the same
 * for A (each ray (a, b) with a <= n_a / 2 also forms ray (n_a - a, b) from
 * the image mirrored about the vertical axis). */
typedef struct {
    int32_t project_groups;     /* 2 or 4: angle groups of 128 rays per projector block
                                   (256 or 512 threads; twice that in the mirrored
                                   form, whose two halves trace the same rays)        */
    int32_t backproject_split;  /* 1, 2 or 4 (8 with backproject_mirror): angle split
                                   inside each 16 x 16 pixel tile (128 threads each) */
    int32_t project_angles;     /* 8 or 4: angles per projector block                 */
    int32_t swizzle;            /* 1: consecutive blocks of a launch share an XCD
                                   (chiplet and its L2), 0: hardware order            */
    int32_t backproject_mirror; /* 1: each backprojector thread also forms the pixels
                                   mirrored about the vertical axis from the same
                                   footprint (half the tiles), 0: every tile      */
    int32_t project_mirror;     /* 1: each projector thread also forms the ray of the
                                   mirror angle n_a - a from the same crossings and
                                   weights (blocks over the angles a <= n_a / 2),
                                   0: every angle                                  */
} scg_tuning;

/* Current shapes for precision prec. */
int scg_plan_get_tuning(const scg_plan *plan, int prec, scg_tuning *out);

/* Sets the shapes used by every later call on the plan for precision prec.
 * SCG_EINVAL for values other than the ones listed above. */
int scg_plan_set_tuning(scg_plan *plan, int prec, const scg_tuning *in);

/* Times A and A^T for every candidate shape on the plan's geometry (ones as
 * input, HIP events on `stream`): after a warm-up, each candidate is timed
 * in two rounds of 10 launches and keeps its faster mean. The swizzle flag,
 * shared by both operators, is the one whose best projector and best
 * backprojector times sum lowest; the fastest shapes under it are kept for
 * precision prec and written to *chosen (may be NULL). Allocates and frees
 * one image and one sinogram of scratch; synchronises the stream. */
int scg_plan_autotune(scg_plan *plan, int prec, void *stream, scg_tuning *chosen);

/* ---- kernel timing ----------------------------------------------------- */

/* Kernel classes for scg_profile. */
#define SCG_KC_PROJECT     0   /* forward projector A                          */
#define SCG_KC_BACKPROJECT 1   /* backprojector A^T (single or dual)            */
#define SCG_KC_TV          2   /* TV and subgradient                            */
#define SCG_KC_TRIALS      3   /* perturbation trials                           */
#define SCG_KC_VECTOR      4   /* direction, image and perturbation updates     */
#define SCG_KC_STAGE       5   /* image staging for the projector               */
#define SCG_KC_FILTER      6   /* preconditioning filter                        */
#define SCG_KC_CONTROL     7   /* per-iteration control                         */
#define SCG_KC_COUNT       8

typedef struct {
    int64_t launches;       /* launches that did their work                  */
    double  total_ms;       /* their summed event-to-event time              */
    int64_t tail_launches;  /* launches that returned at once: enqueued after
                               the solve had stopped (the last batch of
                               iterations ran past the stop), or behind a
                               trial search that suspended the solve until
                               the host enqueued the rest of its step         */
    double  tail_ms;        /* their summed time                              */
} scg_kernel_time;

/* Times every kernel launch of the classes in class_mask (bit c = class c)
 * that scg_solve enqueues on this plan, with a HIP event recorded on the
 * solve's stream before and after the launch. 0 turns timing off. Resets the
 * accumulated totals. */
int scg_profile(scg_plan *plan, uint32_t class_mask);

/* Times only one launch in `every` (>= 1; 1 = all, the default) of each
 * timed class, counting from the last scg_profile call: an event recorded
 * between two launches delays the second by a few microseconds, so a sampled
 * solve runs almost as fast as an untimed one. Resets the sampling phase. */
int scg_profile_every(scg_plan *plan, int32_t every);

/* Accumulated launches and milliseconds per class since the last
 * scg_profile call; out must hold SCG_KC_COUNT entries. */
int scg_profile_read(scg_plan *plan, scg_kernel_time *out);

/* ---- batch engine ------------------------------------------------------ */

/* Many solves resident on one device at once, of any geometry, precision and
 * variant, advanced together: each call of scg_batch_step runs `iters` loop
 * iterations of every active solve with one kernel launch per phase of the
 * iteration covering all solves of a group (same precision, variant and
 * launch shape), the whole iteration captured as a HIP graph that is reused
 * until the set of solves changes. A solve's result is bitwise the one
 * scg_solve gives for the same inputs, parameters and launch shape.
 *
 * Workspaces come from one device arena allocated at creation; a solve is
 * admitted when a slot is free and the arena has room for its workspace
 * (scg_workspace_bytes), otherwise scg_batch_submit returns SCG_EAGAIN.
 * Buffers passed to scg_batch_submit (y, x0, x_out) and the plan must stay
 * valid until the ticket has been retired (scg_batch_poll no longer returns
 * SCG_EINPROGRESS). Work runs on the batch's own stream (scg_batch_stream);
 * callers that produce y on another stream order it before submitting with
 * scg_batch_wait_stream.
 * A batch is not thread-safe. */
typedef struct scg_batch scg_batch;

#define SCG_BATCH_NO_GRAPH 1u   /* enqueue iterations kernel by kernel          */

typedef struct {
    int32_t  active;        /* solves on the device                             */
    int32_t  slots;         /* max_slots                                        */
    int32_t  groups;        /* groups of the current set                       */
    int32_t  graph_updates; /* changes of the set applied to the current graph */
                            /* in place (same launches, new parameters)        */
    uint64_t arena_bytes;
    uint64_t arena_used;    /* workspace bytes of the active solves             */
    uint64_t submitted;
    uint64_t retired;
    uint64_t macro_steps;   /* iterations run (each over all active solves)     */
    uint64_t graph_builds;  /* executable graphs instantiated (a change of the */
                            /* set whose launches differ, or the first one)    */
    uint64_t rebuild_ns;    /* host time spent recomposing the set (groups,    */
                            /* descriptors, admission launch, graph capture,   */
                            /* instantiation or update)                        */
} scg_batch_stats;

/* Creates a batch on `device` with an arena of arena_bytes and at most
 * max_slots concurrent solves (flags: SCG_BATCH_*). */
int scg_batch_create(int device, size_t arena_bytes, int max_slots, uint32_t flags,
                     scg_batch **out);

/* Waits for the batch's stream and frees everything it owns. */
void scg_batch_destroy(scg_batch *batch);

/* Admits a solve (scg_solve's arguments without trace and replay): takes a
 * slot and arena room for its workspace and prepares its descriptor on the
 * host. Its device set-up (state, zeroed sinogram pads, start image) and its
 * initial step run at the start of the next scg_batch_step, together with
 * those of the other solves submitted since the last step. *ticket
 * identifies it. SCG_EAGAIN: no slot or arena room now (retry after a
 * step). */
int scg_batch_submit(scg_batch *batch, scg_plan *plan, const scg_params *params,
                     const void *y, const void *x0, void *x_out, uint64_t *ticket);

/* Runs `iters` iterations of every active solve (a finished solve's kernels
 * return at once), then reads all solves' states and retires the finished
 * ones: their output image and TV are written and their reports kept for
 * scg_batch_poll. Returns the number of solves still active (>= 0) or a
 * negative status. Synchronises the batch's stream. */
int scg_batch_step(scg_batch *batch, int iters);

/* SCG_OK and *rep (may be NULL) for a retired ticket, whose report is then
 * dropped; SCG_EINPROGRESS while it runs; SCG_ENOTFOUND otherwise. */
int scg_batch_poll(scg_batch *batch, uint64_t ticket, scg_report *rep);

/* Removes an active solve without a report (SCG_ENOTFOUND if unknown). */
int scg_batch_cancel(scg_batch *batch, uint64_t ticket);

int scg_batch_get_stats(const scg_batch *batch, scg_batch_stats *out);

/* The hipStream_t the batch runs on. */
void *scg_batch_stream(const scg_batch *batch);

/* Orders the batch's later work (the staging of the next submissions, the
 * steps) after the work already enqueued on `stream`, a hipStream_t of the
 * batch's device (NULL: the null stream), without blocking the host: an
 * event recorded on `stream` that the batch's stream waits for. For callers
 * that produce y or x0 on a stream of their own; call it before
 * scg_batch_submit. A solve's output is complete once the scg_batch_step
 * that retires it has returned (the step synchronises the batch's stream).
 * SCG_EDEVICE if the event cannot be recorded or waited for. */
int scg_batch_wait_stream(scg_batch *batch, void *stream);

/* Fills *params with the library's defaults: S-CG, FP32, a = 0.975,
 * max_iter = 1000, max_trials = 100, kappa = 0, mu = 2 pi / P; eps and
 * gamma0 are set to 0 and must be provided. */
void scg_default_params(scg_params *params);

const char *scg_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* SCG_H */
