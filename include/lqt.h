/*
 * lqt.h -- C ABI of the MI355X (gfx950) linear-quadratic tracker solver.
 *
 * The solver computes, for each LQT instance, the value functions (S_k, v_k),
 * the control gains (K_k, d_k), the optimal trajectory x_k and the optimal
 * controls u_k with the temporal parallelisation of Sarkka & Garcia-Fernandez,
 * "Temporal Parallelisation of Dynamic Programming and Linear Quadratic
 * Control" (arXiv 2104.03186):
 *
 *   - problem (Section II-B): x_{k+1} = F_k x_k + c_k + L_k u_k, running cost
 *     1/2 (H_k x_k - r_k)^T X_k (H_k x_k - r_k) + 1/2 u_k^T U_k u_k for
 *     k = 0..T-1, terminal cost 1/2 (H_T x_T - r_T)^T X_T (H_T x_T - r_T);
 *     X_k symmetric positive semi-definite, U_k symmetric positive definite;
 *   - value function V_k(x) = const + 1/2 x^T S_k x - v_k^T x (Section II-B);
 *   - control law u_k = -K_k x_k + d_k with
 *     K_k = (L_k^T S_{k+1} L_k + U_k)^{-1} L_k^T S_{k+1} F_k and
 *     d_k = (L_k^T S_{k+1} L_k + U_k)^{-1} L_k^T (v_{k+1} - S_{k+1} c_k),
 *     i.e. d_k = K^v_k v_{k+1} - K^c_k c_k of the control law in Section II-B;
 *   - S_k, v_k come from a reverse associative scan over the one-step elements
 *     (A, b, C, eta, J) of Section IV-B with the combination rule of
 *     Section IV-A; x_k comes from a forward scan over the closed-loop affine
 *     maps x_{k+1} = (F_k - L_k K_k) x_k + c_k + L_k d_k (Section IV-C,
 *     Method 1).
 *
 * Memory: every array pointer inside lqt_problem and lqt_outputs is a DEVICE
 * pointer on the plan's device, row-major and contiguous; r and every output
 * array must be 16-byte aligned (LQT_EINVAL otherwise).  The caller owns all
 * input and output buffers; they must stay valid until the work that reads or
 * writes them has completed (stream-ordered for lqt_solve; until lqt_poll
 * returns something other than LQT_EAGAIN for lqt_submit).  The library owns
 * its workspace and frees it in lqt_destroy.
 *
 * Errors: every entry point returns an lqt_status and never throws.  Argument
 * errors are reported synchronously (LQT_EINVAL) before any work is enqueued.
 * Numerical failures are reported per instance through lqt_outputs.status;
 * a failing instance never alters the outputs of other instances.
 * lqt_last_error returns a human-readable description of the last synchronous
 * error of a plan.
 *
 * Thread safety: the calls on one plan are serialised by a lock inside the
 * plan, so a plan may be shared by host threads.  The device workspace of a
 * plan is shared by the work it enqueues (lqt_solve, lqt_nl_iterate and
 * lqt_fs_solve each reuse their own region on every call): work of one plan
 * enqueued on different streams must be ordered by the caller, or each
 * stream given its own plan.  The serving interface (lqt_submit) manages
 * its own streams and memory.
 */
#ifndef LQT_H
#define LQT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LQT_OK = 0,
    LQT_EINVAL = 1,      /* invalid argument (dimension, pointer, horizon)          */
    LQT_ENOMEM = 2,      /* device memory or the plan's memory budget is exhausted */
    LQT_ENOTPD = 3,      /* U_k or L_k^T S_{k+1} L_k + U_k not positive definite   */
    LQT_ENONFINITE = 4,  /* a non-finite value appeared in the solution            */
    LQT_EAGAIN = 5,      /* lqt_poll: the request has not completed yet            */
    LQT_EBUSY = 6,       /* lqt_submit: the in-flight queue is full                */
    LQT_EHIP = 7,        /* a HIP runtime call failed                              */
    LQT_ENOTSUP = 8      /* a dimension or precision the library does not provide */
} lqt_status;

typedef enum {
    LQT_PREC_FP64 = 0,   /* all arithmetic and all outputs in IEEE double          */
    LQT_PREC_MIXED = 1   /* outputs in float; the scan arithmetic stays in double  */
} lqt_precision;
/* LQT_PREC_MIXED: every combination, solve and product of the scan is carried
 * in double and only the stored results are rounded to float (relative error
 * of order 1e-7 per result family against the double solution).  The vector
 * units issue non-packed float and double instructions at the same rate, so
 * float arithmetic would buy no speed on these paths and would cost accuracy
 * in the C and b chains of the combination rule (Section IV-A); the float
 * results halve the output traffic, which bounds the small-n pipeline. */

/* How the optimal trajectory (x, u) is recovered after the backward pass
 * (Section IV-C).  LQT_TRAJ_MAPS (Method 1): parallel scan of the closed-loop
 * affine maps x_{k+1} = (F_k - L_k K_k) x_k + c~_k.  LQT_TRAJ_PREFIX
 * (Method 2): a forward scan of the same LQT elements, initialised by the
 * element (A, b, C, eta, J) = (0, x_0, 0, 0, 0) (the conditional value
 * function from the given x_0), then x_k = (I + C_{0,k} S_k)^{-1}(b_{0,k} +
 * C_{0,k} v_k) and u_k = -K_k x_k + d_k.  The element scan does not depend
 * on the backward pass and runs on a second stream owned by the plan,
 * concurrently with it (joined before the forward walk, so the solve stays
 * ordered on the caller's stream) on the lane pipeline (nx <= 4).  On the
 * chunked engines the forward prefixes at the chunk starts come from the
 * chunk elements of the backward pass (one combination per chunk, after the
 * steps of the first chunk), then every chunk walks its steps.  It reads S
 * and v, held in library workspace when the caller does not take them; with
 * LQT_PREC_MIXED the instances are solved with double results in workspace
 * and rounded to float afterwards (x_k is solved from S_k and v_k, which
 * float rounding would make too inaccurate for the 1e-5 bound). */
typedef enum {
    LQT_TRAJ_MAPS = 0,
    LQT_TRAJ_PREFIX = 1
} lqt_trajectory;

/* Bits of lqt_problem.per_step: a set bit means the matrix has a leading time
 * axis of length T (one matrix per step k = 0..T-1); a clear bit means one
 * matrix serves every step. */
enum {
    LQT_PS_F = 1, LQT_PS_c = 2, LQT_PS_L = 4, LQT_PS_H = 8, LQT_PS_X = 16, LQT_PS_U = 32
};

/* One LQT instance (Section II-B).  n = nx states, m = nu controls,
 * p = ny tracked outputs at steps 0..T-1, pT = nyT tracked outputs at T. */
typedef struct {
    int32_t nx, nu, ny, nyT;
    int64_t T;            /* number of control steps, T >= 1; states x_0..x_T     */
    uint32_t per_step;    /* LQT_PS_* bits                                          */
    const double *F;      /* [n][n]   or [T][n][n]                                  */
    const double *c;      /* [n]      or [T][n]; NULL means c_k = 0                 */
    const double *L;      /* [n][m]   or [T][n][m]                                  */
    const double *H;      /* [p][n]   or [T][p][n]                                  */
    const double *X;      /* [p][p]   or [T][p][p], symmetric PSD                   */
    const double *U;      /* [m][m]   or [T][m][m], symmetric PD                    */
    const double *r;      /* [T][p]   reference r_0..r_{T-1}                        */
    const double *HT;     /* [pT][n]  terminal output matrix                        */
    const double *XT;     /* [pT][pT] terminal weight, symmetric PSD                */
    const double *rT;     /* [pT]     terminal reference r_T                        */
    const double *x0;     /* [n]      initial state                                 */
    /* Generalised stage cost (Section IV-D): with M or s given, the running
     * cost is 1/2 (H x - r)^T X (H x - r) + (H x - r)^T M (u - s)
     * + 1/2 (u - s)^T U (u - s), the joint weight [X M; M^T U] symmetric PSD
     * and U PD.  Both NULL: the cost above (M = 0, s = 0).  The library
     * transforms the instance to the standard form (Z = U^{-1} M^T:
     * F - L Z H, c_k + L Z r_k + L s_k, X - M Z), solves it and maps the
     * results back (K_k + Z H, d_k + Z r_k + s_k, u_k - Z (H x_k - r_k) + s_k;
     * S, v and x are those of the transformed instance).  It needs L, H, X
     * and U shared by every step (LQT_ENOTSUP otherwise) and takes T n
     * (plus T n^2 with per-step F, plus (T + 1) n when u is taken without x)
     * doubles of extra workspace per instance. */
    const double *M;      /* [p][m]   cross weight; NULL means M = 0                */
    const double *s;      /* [T][m]   control reference s_0..s_{T-1}; NULL means 0  */
} lqt_problem;

/* Outputs of one instance.  Element type is double for LQT_PREC_FP64 and
 * float for LQT_PREC_MIXED.  S and v may be NULL (not written).  K and d may
 * be NULL only when x and u are also NULL.  x and u may be NULL together
 * (the forward pass is then skipped). */
typedef struct {
    void *S;              /* [T+1][n][n] value-function matrices S_0..S_T           */
    void *v;              /* [T+1][n]    value-function vectors  v_0..v_T           */
    void *K;              /* [T][m][n]   feedback gains K_0..K_{T-1}                */
    void *d;              /* [T][m]      feed-forward terms d_0..d_{T-1}            */
    void *x;              /* [T+1][n]    optimal states x_0..x_T                    */
    void *u;              /* [T][m]      optimal controls u_0..u_{T-1}              */
    int32_t *status;      /* optional device int32: the instance's lqt_status       */
} lqt_outputs;

typedef struct {
    int32_t device;           /* HIP device ordinal                                 */
    int32_t max_nx, max_nu;   /* largest dimensions the plan will accept            */
    lqt_precision prec;
    size_t hbm_budget_bytes;  /* cap on library-owned device memory (0: no cap)     */
    int64_t max_steps;        /* workspace is pre-sized for this many total steps   */
    int32_t max_inflight;     /* lqt_submit queue depth (0: default)                */
    lqt_trajectory trajectory; /* forward pass (0: LQT_TRAJ_MAPS)                   */
} lqt_plan_desc;

typedef struct lqt_plan_s *lqt_plan_t;

/* Create a plan: validates the descriptor, selects the device, allocates the
 * workspace for desc->max_steps steps.  On success *out receives the plan. */
lqt_status lqt_plan(const lqt_plan_desc *desc, lqt_plan_t *out);

/* Solve `count` independent instances, enqueued on `stream` (a hipStream_t;
 * NULL is the default stream).  Stream-ordered and asynchronous: returns once
 * the work is enqueued.  probs[i] is solved into outs[i].  Synchronous
 * argument errors return LQT_EINVAL/LQT_ENOTSUP/LQT_ENOMEM with nothing
 * enqueued.  The workspace grows (synchronously) when a call needs more than
 * it holds. */
lqt_status lqt_solve(lqt_plan_t plan, const lqt_problem *probs, const lqt_outputs *outs,
                     int32_t count, void *stream);

/* Allocation-free solve, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Solves one instance like lqt_solve (same routing, kernels and
 * results, bit for bit, as lqt_solve on the same plan), stream-ordered and
 * asynchronous, but keeps the whole workspace in a fixed 64 MiB device array
 * of the library instead of plan memory: it calls no hipMalloc, hipFree or
 * other allocating routine (and records no timing events).  The array exists
 * once per device, is held until the process ends, and is shared by every
 * lqt_solve_noalloc call on that device, whatever the plan: calls whose work
 * overlaps on one device (different streams, or host threads with different
 * plans) race on it and must be ordered by the caller.  The solve writes every
 * workspace value before reading it, so nothing needs clearing between calls.
 * Limits: the instance's workspace must fit 64 MiB (LQT_ENOMEM otherwise,
 * nothing enqueued); e.g. an nx = 4, nu = 2 instance of T = 10^6 that passes K
 * and d needs about 33 MB.  Argument errors as lqt_solve (LQT_EINVAL,
 * LQT_ENOTSUP); LQT_EHIP if the array's device address could not be read when
 * the plan was created. */
lqt_status lqt_solve_noalloc(lqt_plan_t plan, const lqt_problem *prob, const lqt_outputs *out, void *stream);

/* Autotuner.  Times the given instances (solved into outs, stream-ordered on
 * `stream`, synchronous) with several chunk lengths for every launch group
 * (size class 8, 16, 32, 64 x wavefront / workgroup engine) present, and
 * keeps the fastest for later solves of this plan: the chunk length of an
 * instance becomes about T / div steps (at least 16) with div in
 * {1, 4, 16, 64, 256}; div = 1 solves every instance of the group as one
 * chunk (sequential down-sweep, no element fold), which pays when the batch
 * alone fills the GPU.  Untuned groups keep the default (about 64 chunks of
 * 16 to 256 steps).  chosen (may be NULL) receives the div of the 8 groups
 * (index 2 * class_index + engine; 0 = default).  The chunking changes
 * the association order of the scan, so results of a tuned plan differ from
 * an untuned one by rounding only; within a plan a result never depends on
 * the batch it is solved in. */
lqt_status lqt_tune(lqt_plan_t plan, const lqt_problem *probs, const lqt_outputs *outs,
                    int32_t count, void *stream, int32_t *chosen);

/* Graph replay of repeated calls (for callers that solve the same buffers
 * again and again: a batch re-solved with new references, an iterated
 * linearisation restarted from a new nominal).  With enable set, lqt_solve
 * and lqt_nl_iterate record the launch sequence of a call the first time its
 * signature is seen -- every argument's dimensions, per-step bits and device
 * pointers, not the data -- as a HIP graph (stream capture on a stream of
 * the plan), and replay that graph on the caller's stream for later calls
 * with the same signature: one graph launch instead of every kernel launch
 * and host-side preparation.  A replay performs the recorded work on the
 * current contents of the same buffers, so its results equal those of a
 * direct call bit for bit.  Each recorded signature owns its workspace:
 * replays of one signature must be ordered by the caller like any work of
 * the plan.  At most 64 signatures are kept (the set is cleared when full);
 * lqt_set_routing, lqt_tune and disabling clear it.  While per-kernel timing
 * is enabled calls run directly.  Off by default. */
lqt_status lqt_set_graphs(lqt_plan_t plan, int32_t enable);

/* Number of signatures currently recorded as graphs (negative lqt_status on
 * error). */
int32_t lqt_graphs_recorded(lqt_plan_t plan);

/* Routing and chunking overrides of one plan (testing, tuning and the
 * block-length study of Section V-C).  They apply to the plan's later
 * lqt_solve, lqt_tune, lqt_submit and lqt_nl_iterate calls; other plans are
 * not affected.  Every field 0 selects the automatic choice:
 *   path:       1 = the lane pipeline wherever it applies (nx <= 4, nu <= nx,
 *               any T), 2 = the chunked engines for every instance, 3 = the
 *               batched lane kernel wherever it applies (nx <= 4, nu <= nx,
 *               time-invariant except c, any T);
 *   block:      1 = instances of the size classes 16 and 32 stay on the
 *               wavefront engine even when they are time-invariant;
 *   lane_chunk: steps per lane of the lane pipeline, 1..1024;
 *   wave_chunk: steps per chunk of the chunked engines, 1..4096 (takes
 *               precedence over a tuned chunk length);
 *   tree:       how the chunked engines scan an instance's chunks (the value
 *               at every chunk start from the chunk elements, the state at
 *               every chunk start from the chunk maps): 1 = as trees,
 *               recursive doubling in about log2(chunks) dependent steps
 *               (Section II-C), for every instance of two chunks or more,
 *               with chunks of 8 to 64 steps (about as many chunks as the
 *               GPU runs side by side) unless wave_chunk or lqt_tune fixes
 *               the length; 2 = as walks over the chunks in sequence; 0 =
 *               trees from 128 chunks on.  Trees do about log2(chunks) times
 *               the work of the walks: they pay when a launch has too few
 *               instances to fill the GPU (a lone instance, for latency).
 * The chunking and the tree choice change only the association order of the
 * scan.  NULL restores the automatic choices.  LQT_EINVAL for values outside
 * these ranges. */
typedef struct {
    int32_t path;
    int32_t block;
    int32_t lane_chunk;
    int32_t wave_chunk;
    int32_t tree;
} lqt_routing;

lqt_status lqt_set_routing(lqt_plan_t plan, const lqt_routing *routing);

/* Serving interface (continuous batching).  lqt_submit queues one instance
 * and returns at once with *ticket.  Requests wait in one FIFO per lane:
 * short solves (the batched lane kernel, the lane pipeline, and chunked
 * solves with a short critical path) and long ones (chunked solves of long
 * horizon or large size class); each of the plan's serving streams belongs to
 * one lane, so a short request is never batched with, or queued behind, a
 * long one.  Whenever a stream is idle, the longest prefix of its lane's
 * queue whose workspace fits one free range of the plan's serving pool
 * (hbm_budget_bytes, or 8 GiB when that is 0) becomes one batch on that
 * stream.  Several batches run on the device at once; a request that arrives
 * while others are running joins the next batch of its lane as soon as a
 * stream and pool memory are free.  Nothing overtakes the head of a lane;
 * a head waiting for memory is protected (the other lane launches only
 * batches that leave it room), so no request starves.  Batching never
 * changes a result: every instance is solved exactly as by lqt_solve alone.
 * Progress is made inside lqt_submit and lqt_poll and by a progress thread
 * of the plan (started by the first lqt_submit, stopped by lqt_destroy).
 *   LQT_ENOMEM: the request alone needs more than the serving pool.
 *   LQT_EBUSY:  max_inflight requests are already queued or running.
 * Once a request is queued, lqt_submit returns LQT_OK; a failure to launch
 * its batch is its status, returned by lqt_poll.
 * The caller's input and output buffers must stay valid until lqt_poll has
 * returned something other than LQT_EAGAIN for the ticket. */
lqt_status lqt_submit(lqt_plan_t plan, const lqt_problem *prob, const lqt_outputs *out,
                      uint64_t *ticket);

/* LQT_EAGAIN while the request is queued or running; afterwards the
 * instance's status (LQT_OK on success).  A ticket may be polled to
 * completion once. */
lqt_status lqt_poll(lqt_plan_t plan, uint64_t ticket);

/* Counters of the serving interface since the plan was created. */
typedef struct {
    int64_t submitted;        /* requests accepted by lqt_submit                    */
    int64_t completed;        /* requests whose batch has finished                  */
    int64_t batches;          /* batches launched                                   */
    int32_t queued;           /* requests waiting for a stream or pool memory       */
    int32_t running_batches;  /* batches on the device now                          */
    int32_t max_running_batches; /* most batches ever on the device at once         */
    int32_t max_batch;        /* largest batch launched (requests)                  */
    size_t pool_bytes;        /* size of the serving pool                           */
    size_t pool_in_use;       /* bytes held by running batches                      */
    size_t pool_peak;         /* most bytes ever held at once                       */
} lqt_serve_stats;

lqt_status lqt_serve_stats_read(lqt_plan_t plan, lqt_serve_stats *out);

/* Iterated linearisation for nonlinear dynamics (the nonlinear extension of Section IV-D): starting
 * from a nominal trajectory (xbar, ubar), each iteration linearises the
 * dynamics by the first-order Taylor expansion about the nominal,
 * x_{k+1} = F_k x_k + c_k + L_k u_k with F_k = df/dx, L_k = df/du at
 * (xbar_k, ubar_k) and c_k = f(xbar_k, ubar_k) - F_k xbar_k - L_k ubar_k,
 * solves that LQT (the plan's scan, routing and trajectory method) and takes
 * its optimal (x, u) as the next nominal.  Output and control maps are linear
 * (h(x) = H x, g(u) = u); the cost is that of lqt_problem. */
typedef enum {
    /* Unicycle of the nonlinear experiment (Section VI-E): x = (p_x, p_y,
     * theta, speed), u = (acceleration, turn rate), f(x, u) = (p_x + speed
     * cos(theta) dt_k, p_y + speed sin(theta) dt_k, theta + turn rate dt_k,
     * speed + acceleration dt_k); nx = 4, nu = 2. */
    LQT_NL_UNICYCLE = 0
} lqt_nl_model;

typedef struct {
    lqt_nl_model model;
    int32_t ny, nyT;      /* tracked outputs at steps 0..T-1 and at T               */
    int64_t T;
    uint32_t per_step;    /* LQT_PS_H, LQT_PS_X, LQT_PS_U bits (as in lqt_problem)  */
    const double *dt;     /* [T]       step lengths dt_k                            */
    const double *H, *X, *U, *r, *HT, *XT, *rT, *x0;  /* as in lqt_problem        */
} lqt_nl_problem;

/* Run `iterations` (>= 1) linearise-and-solve rounds on `stream`
 * (stream-ordered, asynchronous, like lqt_solve).  x ([T+1][nx]) and u
 * ([T][nu]), device arrays of the plan's output type, hold the nominal
 * trajectory on entry and the last round's optimal states and controls on
 * return (the round solves from x_0 = prob->x0; xbar_0 is the first
 * expansion point).  change (optional, device, [iterations] doubles)
 * receives max_{k,i} |u_new - u_nominal| of each round, a convergence
 * measure; status (optional, device int32) the first failing round's
 * lqt_status, else LQT_OK.  Workspace: (n^2 + n m + n + m) T doubles of
 * linearised model beside the solve's own.  Argument errors (LQT_EINVAL,
 * nothing enqueued): unknown model, per_step bits other than H, X, U, NULL
 * pointers, iterations < 1, the model's nx, nu above the plan's maxima, and
 * the checks of lqt_solve on the linearised instance. */
lqt_status lqt_nl_iterate(lqt_plan_t plan, const lqt_nl_problem *prob, int32_t iterations, void *x, void *u,
                          double *change, int32_t *status, void *stream);

/* Finite state and control spaces (Section III-D): x_k in {0..D_x-1},
 * u_k in {0..D_u-1}, x_{k+1} = f_k(x_k, u_k), stage cost l_k(x_k, u_k),
 * terminal cost l_T(x_T).  The value functions V_k(x) = min_u { l_k(x, u) +
 * V_{k+1}(f_k(x, u)) } come from a reverse scan whose elements are the
 * one-step conditional value functions V_{k->k+1}(x, y) = min { l_k(x, u) :
 * f_k(x, u) = y } (D_x x D_x, +inf where y is unreachable) combined by the
 * min-plus product (the combination rule of Section III-B); the control law
 * u_k(x) is the minimising control (the smallest index among equal minima),
 * and the trajectory from x_0 follows by composing the closed-loop maps
 * x -> f_k(x, u_k(x)) (Method 1 of Section III-C).  Costs are doubles;
 * with integer-valued costs every sum is exact and the results do not
 * depend on the association order of the scan. */
enum { LQT_FS_NEXT = 1, LQT_FS_COST = 2 };  /* per_step bits of lqt_fs_problem */

typedef struct {
    int32_t nstates, ncontrols;  /* D_x in 1..32, D_u in 1..32                           */
    int64_t T;                   /* control steps, T >= 1                                */
    uint32_t per_step;           /* LQT_FS_* bits: table with a leading time axis        */
    const int32_t *next;         /* [D_x][D_u] or [T][D_x][D_u]: f_k(x, u); -1 = control not admissible */
    const double *cost;          /* [D_x][D_u] or [T][D_x][D_u]: l_k(x, u)               */
    const double *cost_T;        /* [D_x] terminal cost                                  */
    int32_t x0;                  /* initial state                                        */
} lqt_fs_problem;

typedef struct {
    double *V;        /* [T+1][D_x] value functions (+inf: no admissible continuation), or NULL */
    int32_t *u;       /* [T][D_x] control law (-1 where no control is admissible), or NULL      */
    int32_t *x;       /* [T+1] optimal trajectory from x0, or NULL                               */
    int32_t *ux;      /* [T] the controls applied along it, or NULL                              */
    int32_t *status;  /* optional device int32: LQT_OK, or LQT_ENONFINITE when no admissible path leaves x0 */
} lqt_fs_outputs;

/* Solve one finite-state problem on `stream` (stream-ordered, asynchronous).
 * All pointers are device pointers; next, cost, cost_T and the outputs
 * are caller-owned.  LQT_EINVAL (nothing enqueued): D_x or D_u outside
 * 1..32, T < 1, x0 outside 0..D_x-1, NULL tables, unknown per_step bits.
 * Next-state entries outside -1..D_x-1 are treated as not admissible.
 * Workspace: about (D_x^2 + 2 D_x) NC doubles for NC = min(2048, T / 16)
 * blocks of consecutive steps, plus D_x T int32 (the closed-loop maps of
 * every step) and, when u is NULL, D_x T int32 for the control law. */
lqt_status lqt_fs_solve(lqt_plan_t plan, const lqt_fs_problem *prob, const lqt_fs_outputs *out, void *stream);

/* Wait for all work of the plan, then release it and its workspace. */
lqt_status lqt_destroy(lqt_plan_t plan);

/* Per-kernel timing (diagnostics, tracing).  While enabled, every kernel the
 * plan launches is bracketed by HIP events recorded on the launch stream, so
 * the device timeline of each kernel can be read back.  Disabled by default. */
typedef struct {
    const char *name;     /* kernel (stage) name, owned by the library           */
    int64_t launches;     /* launches accumulated since the last read            */
    double total_ms;      /* summed device time of those launches                */
} lqt_stage_time;

lqt_status lqt_profile_enable(lqt_plan_t plan, int32_t enable);

/* Restrict the timing to the launches of one stage (NULL: every stage), so
 * that only that kernel is bracketed by events. */
lqt_status lqt_profile_select(lqt_plan_t plan, const char *stage);

/* Waits for the recorded events, writes up to `max` per-stage totals (in
 * first-launch order) into out, clears the accumulators and returns the
 * number of stages (negative lqt_status on failure). */
int32_t lqt_profile_read(lqt_plan_t plan, lqt_stage_time *out, int32_t max);

/* Description of the last synchronous error of the plan ("" if none).
 * The string is owned by the plan.  NULL plan: the last plan-creation error. */
const char *lqt_last_error(lqt_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* LQT_H */
