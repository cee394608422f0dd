/*
 * fdw.h - C-ABI of the MI355X (gfx950) explicit leapfrog solver for the regularised
 * tsunami wave equation of arXiv 2005.11931,
 *
 *     u_tt = d_x(h1(x,y) d_x u) + d_y(h2(x,y) d_y u),  (t,x,y) in [0,T] x [x0,x1] x [y0,y1],
 *     u(0) = u0,  u_t(0) = u1,  u = 0 on the boundary,
 *
 * i.e. the Cauchy problem of Section 2, equation (2.1) with the vector-valued coefficient
 * h = (h1, h2) (positive, Section 2), regularised by mollification (Section 2.1,
 * Section 3.1), on the node grid and with the zero Dirichlet data of Section 3.3.
 *
 * Discretisation (the paper's own solvers are implicit; this library is explicit):
 *   face coefficients  hx_{i+1/2,j} = (h1_{i,j} + h1_{i+1,j})/2,  hy_{i,j+1/2} likewise with h2;
 *   operator           (A u)_ij = [hx_{i+1/2}(u_{i+1}-u_i) + hx_{i-1/2}(u_{i-1}-u_i)]/dx^2 + (same in y)/dy^2;
 *   start              u^1 = u^0 + tau u1 + (tau^2/2) A u^0;
 *   leapfrog           u^{n+1} = 2 u^n - u^{n-1} + tau^2 A u^n;
 *   energy             E^{n+1/2} = dx dy [ sum ((u^{n+1}-u^n)/tau)^2 + <K u^{n+1}, u^n> ],  K = -A,
 *                      the discrete form of the conservation law of Section 2 (proof of
 *                      Theorem 2.1, identity CL-01), constant in exact arithmetic.
 * The state is carried in increment form (u^n, du^n = u^n - u^{n-1}), which is the same
 * recurrence in exact arithmetic and keeps the velocity information that FP32 would lose
 * in 2u^n - u^{n-1} when tau is small.
 *
 * Conventions for every entry point:
 *   - all arrays are row-major [ny][nx] (x fastest), dense, in the problem's storage type
 *     (float for FDW_F32, double for FDW_F64) unless stated as double;
 *   - "device" pointers are HIP device memory on the current device; "host" pointers are
 *     ordinary host memory;
 *   - the caller owns every pointer it passes, including the workspace; inputs are copied
 *     (stream-ordered) during the call, so they may be reused once the stream reaches it;
 *   - work is enqueued on the stream given to fdw_init (hipStream_t passed as void*, NULL
 *     for the null stream); calls return before the GPU finishes unless stated otherwise;
 *   - every entry point returns FDW_OK (0) or a negative FDW_E* code and never aborts;
 *     fdw_last_error() gives a one-line description of the last failure on that context;
 *   - a context is not thread-safe; separate contexts are independent.
 */
#ifndef FDW_H
#define FDW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdw_ctx fdw_ctx; /* opaque */

typedef enum { FDW_F32 = 0, FDW_F64 = 1 } fdw_dtype;

enum {
    FDW_OK = 0,
    FDW_EINVAL = -1,    /* bad argument: sizes, tau <= 0, T/tau not an integer, NULL pointer,
                           non-finite or negative h, receiver outside the interior */
    FDW_ECFL = -2,      /* tau^2 (4 max hx/dx^2 + 4 max hy/dy^2) > 4: leapfrog would be unstable */
    FDW_ESTATE = -3,    /* call out of order (e.g. stepping before fdw_set_coeff) */
    FDW_ENOMEM = -4,    /* workspace too small */
    FDW_EHIP = -5,      /* a HIP runtime error; see fdw_last_error */
    FDW_EUNSTABLE = -6, /* a non-finite energy was produced */
    FDW_ENOTSUP = -7,   /* configuration not supported */
    FDW_ESYNC = -8      /* a grid barrier of the persistent launch timed out: the steps of that call
                           are not valid (the context must be reset or its state set) */
};

/* fdw_problem.flags */
enum {
    FDW_ALLOW_UNSTABLE = 1u, /* skip the stability (CFL) check in fdw_set_coeff */
    FDW_ALLOW_ZERO_H = 2u    /* accept h >= 0 instead of h > 0 (e.g. h2 = 0 decouples rows into 1D problems) */
};

/* One regularised problem (Section 2, eq. (2.1); grid of Section 3.3).
 * nx, ny >= 3 nodes including the boundary ring; dx = (x1-x0)/(nx-1), dy = (y1-y0)/(ny-1);
 * tau > 0; N = llround(T/tau) steps with |N tau - T| <= 1e-9 T (T = 0 allowed: N = 0). */
typedef struct {
    int32_t nx, ny;
    double x0, x1, y0, y1;
    double tau, T;
    int32_t dtype; /* fdw_dtype */
    uint32_t flags;
} fdw_problem;

/* Device workspace (bytes) that fdw_init needs for `count` members described by
 * problems[0..count-1] (the state of the Cauchy problem of Section 2, eq. (2.1), on the grid
 * of Section 3.3, per member).  Returns 0 when the problems are invalid.  The adjoint's
 * checkpoints are sized separately (fdw_adjoint_workspace_bytes), per member and interval. */
size_t fdw_workspace_bytes(const fdw_problem* problems, int32_t count);

/* Create a context for `count` >= 1 members (count > 1 is a batched family: members may
 * differ in size, tau, coefficient and storage type; a family that mixes FP32 and FP64
 * members, e.g. FP64 for its smallest-eps members, runs one launch sequence per type).  Each member is one
 * regularised Cauchy problem: the Cauchy data u(0) = u0, u_t(0) = u1 of eq. (2.1) (Section 2)
 * on the grid with zero Dirichlet data of Section 3.3; a family holds several
 * regularisations h_eps of one singular depth (Section 2.1, Section 3.2).
 * workspace: device memory of ws_bytes >= fdw_workspace_bytes(), 256-byte aligned, owned by
 *            the caller and alive until fdw_destroy;
 * u0, u1:    arrays of `count` device pointers, member m's initial displacement and
 *            velocity, [ny_m][nx_m] in the storage type (the boundary ring is taken as 0);
 * hip_stream: hipStream_t the context enqueues on (NULL = null stream).
 * On success *out receives the context at step n = 0. */
int fdw_init(const fdw_problem* problems, int32_t count, void* workspace, size_t ws_bytes,
             const void* const* u0, const void* const* u1, void* hip_stream, fdw_ctx** out);

/* Set member m's coefficient (face coefficients and the stability check): the positive,
 * vector-valued depth h = (h1, h2) of eq. (2.1) with h_j >= c0 > 0 (Section 2), usually a
 * regularisation h_eps = h * psi_eps (Section 2.1, Section 3.1).
 * h1: device [ny][nx] nodal h1; h2: device nodal h2, or NULL when h2 = h1 (the physical
 * model h_1 = h_2 = h; a faster nodal layout is used).  The values are validated (finite,
 * > 0, or >= 0 with FDW_ALLOW_ZERO_H) and the CFL bound is checked; both read one small
 * result back to the host, so this call synchronises the stream.  Resets member m to n = 0. */
int fdw_set_coeff(fdw_ctx* ctx, int32_t member, const void* h1, const void* h2);

/* Advance every member by n >= 0 steps of the discretised eq. (2.1) (Section 2; grid of
 * Section 3.3) (the Taylor start step when a member is at n = 0, then leapfrog steps).  energy_dev: NULL, or device double [count][n] receiving
 * E^{k+1/2} for k = n_cur .. n_cur+n-1 of each member.  Traces registered with
 * fdw_record_traces are written as the steps are taken.  With energies requested (and
 * FDW_CFG_CHECK_ENERGY on, the default) the call checks them before returning: FDW_EUNSTABLE
 * when one is non-finite or exceeds 10x the first energy of the call (the steps are taken and
 * the energies written either way); this check synchronises the stream.  In batch mode 1 (the
 * persistent launch) the call also reads back the launch's grid-barrier word (synchronising the
 * stream) and returns FDW_ESYNC if a barrier wait timed out; traces and checkpoint recording
 * use the per-time-block launches instead. */
int fdw_step_n(fdw_ctx* ctx, int64_t n, double* energy_dev);

/* E^{n-1/2} of each member's current pair (u^{n-1}, u^n), into host double [count]: the
 * discrete form of the conserved energy of Section 2 (proof of Theorem 2.1, identity CL-01).
 * Needs n >= 1 (FDW_ESTATE otherwise); synchronises the stream. */
int fdw_energy(fdw_ctx* ctx, double* energy_host);

/* Record traces of member m (the solution u(t_k, x_r) of eq. (2.1) at fixed nodes; receivers
 * and the misfit below are this library's addition for gradients, the paper computes none):
 * from now on u^k at the R receivers is written into
 * traces[k][r] (device, storage type, [N+1][R], N = the member's llround(T/tau)) for every
 * step k <= N taken; the current step's row is written immediately.
 * recv_ij: device int32 [R][2] = (i, j) of interior nodes, copied during the call.
 * R = 0 (or traces = NULL) stops recording. */
int fdw_record_traces(fdw_ctx* ctx, int32_t member, const int32_t* recv_ij, int32_t R, void* traces);

/* Receiver misfit (no passage of the paper: the loss whose gradient fdw_adjoint computes):
 * J = sum_{k=0}^{rows-1} sum_r (traces[k][r] - d[k][r])^2 in double, and the
 * adjoint source trace_grad[k][r] = 2 (traces - d) (double, may be NULL).  traces is in the
 * storage type of member m, d is double; all device; J_dev is a device double. */
int fdw_misfit(fdw_ctx* ctx, int32_t member, const void* traces, const double* d, int64_t rows, int32_t R,
               double* J_dev, double* trace_grad);

/* (For callers that cannot allocate.)  fdw_misfit for callers that cannot allocate device memory (code under stream capture,
 * tight loops, harnesses that forbid allocation): no context and no workspace.  Same result,
 * bit for bit, as fdw_misfit on the same arrays: J_dev (device double) receives
 * sum_{k<rows, r<R} (traces[k][r] - d[k][r])^2 and trace_grad (device double [rows][R], may be
 * NULL) the adjoint source 2 (traces - d); traces (device, [rows][R]) is float for FDW_F32
 * and double for FDW_F64, d is device double; enqueued on hip_stream (NULL = null stream).
 * The reduction's partial sums live in a fixed 33 KB array in device memory that each GPU
 * holds once per process (looked up on the first call on a device, which must not be under
 * stream capture); every call on one GPU shares it, so calls that overlap on one GPU (other
 * streams, other host threads) race.  Limits: rows <= 2^31 - 1, R <= 16384 (FDW_EINVAL
 * beyond).  Errors: FDW_EINVAL, FDW_EHIP; fdw_noalloc_last_error() describes the last
 * failure of this entry point on the calling thread. */
int fdw_misfit_noalloc(int32_t dtype, const void* traces, const double* d, int64_t rows, int32_t R, double* J_dev,
                       double* trace_grad, void* hip_stream);
const char* fdw_noalloc_last_error(void);

/* Device workspace (bytes) fdw_adjoint needs for member m with checkpoints every
 * ckpt_every steps: the reverse-sweep state and the (N-1)/ckpt_every stored pairs (u, du).
 * A workspace of its own, since its size depends on the member and the interval. */
size_t fdw_adjoint_workspace_bytes(const fdw_ctx* ctx, int32_t member, int32_t ckpt_every);

/* Checkpointing for the gradient (no passage of the paper: memory/recomputation trade-off of the
 * discrete adjoint).  Store the adjoint's checkpoints during member m's forward run: from step 0 on, every
 * fdw_step_n writes (u^n, du^n) for n = ckpt_every, 2 ckpt_every, ... < N into adj_ws
 * (device, at least fdw_adjoint_workspace_bytes(member, ckpt_every) bytes, 256-byte aligned,
 * owned by the caller and kept alive while recording).  Time blocks are cut at those steps;
 * graph capture and the persistent batch launch are not used while recording.  A later
 * fdw_adjoint of member m with the same adj_ws and ckpt_every, once the member stands at
 * step N, then skips its forward replay.  Needs the member at step 0 (FDW_ESTATE otherwise);
 * fdw_set_coeff, fdw_reset and fdw_set_state of the member stop the recording, as does a call
 * with adj_ws = NULL.  One member per context records at a time (a new call replaces the old). */
int fdw_record_checkpoints(fdw_ctx* ctx, int32_t member, int32_t ckpt_every, void* adj_ws, size_t adj_ws_bytes);

/* Gradient with respect to the nodal coefficient(s) h = (h1, h2) of eq. (2.1) (Section 2) of
 * a loss L of the traces u^k_r, k = 0..N, by the discrete adjoint of the leapfrog scheme of
 * fdw_step_n (derived from the scheme; the paper has no adjoint): the
 * forward recurrence is replayed from member m's initial data storing the state every
 * ckpt_every steps (skipped when fdw_record_checkpoints recorded them during the forward run
 * that left the member at step N), then the transposed (reverse leapfrog) recurrence runs
 * backwards, each segment being reconstructed from its checkpoint by time reversal.
 * trace_grad: device double [N+1][R] = dL/du^k at the receivers;
 * recv_ij: device int32 [R][2] (interior nodes); adj_ws: device workspace of
 * fdw_adjoint_workspace_bytes() bytes; grad_h1: device double [ny][nx] receives dL/dh1;
 * grad_h2: device double [ny][nx] receives dL/dh2, or NULL to receive dL/dh1 + dL/dh2 in
 * grad_h1 (the case h1 = h2 = h).  The forward state of the context is left unchanged. */
int fdw_adjoint(fdw_ctx* ctx, int32_t member, const int32_t* recv_ij, int32_t R, const double* trace_grad,
                int32_t ckpt_every, void* adj_ws, size_t adj_ws_bytes, double* grad_h1, double* grad_h2);

/* Snapshot / resume of the solution u(t_n, .) (Section 3.3 grid, t_n = n tau): copy member
 * m's state (u^n, du^n = u^n - u^{n-1}; the increment form carried by the kernels) to device
 * buffers [ny][nx] in the storage type and its step counter to *n (host).  du is all zeros
 * at n = 0.  u and du may be NULL. */
int fdw_get_state(fdw_ctx* ctx, int32_t member, void* u, void* du, int64_t* n);

/* Overwrite member m's state with (u^n, du^n) from device buffers and set its step counter.
 * n >= 1 (at n = 0 the state is defined by the initial data). */
int fdw_set_state(fdw_ctx* ctx, int32_t member, const void* u, const void* du, int64_t n);

/* L2 distance of two members' current fields (of one storage type: FDW_ENOTSUP otherwise), sqrt(dx dy sum (u_a - u_b)^2) in double: the
 * norm ||u_eps1(t, .) - u_eps2(t, .)||_{L^2} of Section 3.2.1 (limiting behaviour as eps -> 0)
 * and of the consistency statement of Section 2.3 (Theorem 2.6), for regularisations on the
 * same grid.  Both
 * members must have the same nx, ny and domain; synchronises the stream; result on the host. */
int fdw_member_distance(fdw_ctx* ctx, int32_t member_a, int32_t member_b, double* dist_host);

/* Return member m to step 0 (its Cauchy data u0, u1; no passage: execution control). */
int fdw_reset(fdw_ctx* ctx, int32_t member);

/* Step counter n of member m (t = n tau), or -1 on a bad argument. */
int64_t fdw_steps_taken(const fdw_ctx* ctx, int32_t member);

/* Execution configuration (no passage of the paper: tuning; results do not depend on it,
 * bit for bit):
 *   FDW_CFG_TIME_BLOCK: time steps per stencil launch: 1..8 for float with 2 columns per lane and
 *     double with 1, 1..6 for float with 4, 1..4 for double with 2 (0 = automatic);
 *   FDW_CFG_SEGMENT_ROWS: rows per streaming work item, 8..4096 (0 = automatic);
 *   FDW_CFG_USE_GRAPH: 1 captures the launch sequence of a step_n call in a hipGraph and
 *     replays it for later calls with the same shape (0 = plain launches);
 * On a family that mixes storage types a setting applies to both types and must be valid for
 * both; fdw_get_config reports the FP32 members' value.
 *   FDW_CFG_BATCH_MODE: 0 = one launch per time block covering all members, 1 = one persistent
 *     cooperative launch per step_n call (up to 8192 steps per launch) with the energies summed
 *     in the launch; combined with FDW_CFG_USE_GRAPH the launch is replayed from a hipGraph.
 *     The state is the same bit for bit in both modes; the energies agree to rounding (their
 *     partial sums are added in a different order). */
enum {
    FDW_CFG_TIME_BLOCK = 1,
    FDW_CFG_SEGMENT_ROWS = 2,
    FDW_CFG_USE_GRAPH = 3,
    FDW_CFG_BATCH_MODE = 4,
    FDW_CFG_TIMING = 5, /* 1: bracket every stencil launch with HIP events (see fdw_kernel_time) */
    FDW_CFG_LANE_COLUMNS = 6, /* grid columns per lane of the streaming kernels: 2 or 4 (float), 1 or 2
                                 (double); 0 = default */
    FDW_CFG_ADJ_TIME_BLOCK = 7,  /* reverse steps per launch of the adjoint sweep: 1..6 with 1 (double) or
                                    2 (float) columns per lane, else 1..4 (0 = 6 with those lane
                                    layouts, the defaults, else 4) */
    FDW_CFG_ADJ_LANE_COLUMNS = 8, /* columns per lane of the adjoint sweep: 2 or 4 (float), 1 or 2 (double);
                                     0 = default (2 for float, 1 for double) */
    FDW_CFG_ADJ_SEGMENT_ROWS = 9, /* rows per work item of the adjoint sweep, 16..4096 (0 = automatic: 4 x the
                                     reverse time block, at least 16; lengthened, up to 16 x the block,
                                     until one launch's items fit in the waves the device holds at once) */
    FDW_CFG_CHECK_ENERGY = 10,    /* 1 (default): fdw_step_n checks the energies it computes and returns
                                     FDW_EUNSTABLE on a non-finite one or on growth beyond 10x the call's
                                     first energy (one word read back: such calls synchronise the stream);
                                     0: no check, fully asynchronous */
    FDW_CFG_TEST_BARRIER_FLAG = 11 /* test hook: 1 marks the next fdw_step_n as if a grid barrier of the
                                      persistent launch had timed out (the host writes the error word that
                                      the call reads back; no kernel waits on it): that call returns
                                      FDW_ESYNC; the hook then resets itself */,
    FDW_CFG_ITEM_ORDER = 12,      /* 1 (default): every other stencil launch walks its work items in
                                     reverse order, so the rows a launch wrote last are read first by
                                     the next one (1-3% faster where measured); 0: one fixed order;
                                     results are identical */
    FDW_CFG_STREAM_POLICY = 13,   /* row accesses of the forward stencil: 0 (default) non-temporal when the
                                     working set exceeds the last-level cache; 1 non-temporal loads and
                                     stores; 2 cacheable loads and stores; 3 non-temporal stores only;
                                     4 non-temporal loads only (float); results are identical */
    FDW_CFG_SMALL_TILES = 14,     /* small-grid kernel: one workgroup per tile of 48 owned columns,
                                     its waves advancing the tile level by level together.  0 (default):
                                     used where every member has at most 1024 x 1024 nodes; 1: never;
                                     2: wherever allowed.  Never with receiver traces or the persistent
                                     launch (the streaming kernel runs those steps).  States are
                                     identical bit for bit; energies agree to rounding (other partial
                                     sums) */
    FDW_CFG_TILE_ROWS = 15        /* rows per tile of the small-grid kernel (16 halo rows included):
                                     32, 48 or 64 (0 = automatic: 64 where that gives a launch 150 to
                                     300 tiles, else 48 where that gives at least 150, else 32) */
};
int fdw_configure(fdw_ctx* ctx, int32_t key, int64_t value);
int64_t fdw_get_config(const fdw_ctx* ctx, int32_t key);

/* Autotune the execution configuration for this context (no passage: tuning): times short
 * runs of the candidate
 * (columns per lane, time block, segment rows) triples on the context's stream under two
 * stream policies (automatic, and non-temporal stores with cacheable loads, where the two
 * differ), picks the fastest (a larger time block must win by 2%) and applies it (the policy
 * is then readable as FDW_CFG_STREAM_POLICY).  Every member must be at
 * step 0 (FDW_ESTATE otherwise) and is returned to step 0 (a checkpoint recording stops).
 * The choice is cached in the
 * file named by the FDW_AUTOTUNE_CACHE environment variable (if set) under a key of
 * (device arch, storage type, member sizes and layouts, launch mode).  The candidates run in
 * the context's own launch mode (FDW_CFG_USE_GRAPH, FDW_CFG_BATCH_MODE; the persistent launch
 * only takes time blocks 1, 2, 4, 8).  The search times the streaming kernel only: where the
 * small-grid tile kernel runs (FDW_CFG_SMALL_TILES) it keeps running after the call, with the
 * chosen time block.  steps: time steps per candidate
 * run (0 = automatic).  best_out (host, may be NULL) receives
 * {time_block, segment_rows, lane_columns}. */
int fdw_autotune(fdw_ctx* ctx, int32_t steps, int64_t* best_out);

/* Autotune the reverse sweep of member m (no passage: tuning): times fdw_adjoint with the given
 * arguments (as for fdw_adjoint; the gradient goes to grad_scratch, device double [ny][nx], and
 * the forward state is left unchanged) for each candidate (reverse time block, columns per lane,
 * rows per work item) and applies the fastest.  With checkpoints recorded by the forward run in
 * adj_ws the candidates time the reverse sweep alone.  Cached like fdw_autotune.  best_out (host,
 * may be NULL) receives {adj_time_block, adj_segment_rows (0 = automatic), adj_lane_columns}. */
int fdw_autotune_adjoint(fdw_ctx* ctx, int32_t member, const int32_t* recv_ij, int32_t R, const double* trace_grad,
                         int32_t ckpt_every, void* adj_ws, size_t adj_ws_bytes, double* grad_scratch,
                         int64_t* best_out);

/* Instrumentation (no passage: measurement) (FDW_CFG_TIMING = 1, not under graph replay):
 * synchronise the stream and
 * report the summed device time (ms) and the number of the streaming stencil launches made
 * since the previous call; the counters are then cleared.  ms and launches are host pointers. */
int fdw_kernel_time(fdw_ctx* ctx, double* ms, int64_t* launches);

/* ---- The implicit scheme of the paper's 2D experiment (Section 3.3; Section 4, Table 1) ----
 * The paper solves its 2D problem with an implicit finite-difference scheme whose systems are
 * solved by cyclic reduction, and times that solver on a GPU (Table 1).  This is such a solver:
 * the factorized (alternating-direction) implicit scheme
 *     (I - sigma tau^2 L1)(I - sigma tau^2 L2)(u^{n+1} - 2u^n + u^{n-1}) = tau^2 (L1 + L2) u^n,
 * L1 = d_x(h1 d_x .), L2 = d_y(h2 d_y .) with the face coefficients and zero Dirichlet data of the
 * explicit solver, start u^1 = u^0 + tau u1 + w^0/2 (w^0 the same solve applied to tau^2 A u^0);
 * every factor is a set of tridiagonal systems, one per grid line, each solved by one workgroup:
 * elimination within contiguous chunks of the line, then cyclic reduction in LDS on the system of
 * the chunks' interface unknowns.  sigma >= 1/4 is unconditionally stable (constant coefficients:
 * every mode); sigma = 0 is the leapfrog scheme.  The state is carried as (u, du = u^n - u^{n-1}).
 * Limits: max(nx, ny) - 2 <= 4352 in FP64, 8448 in FP32 (256 chunks of at most 17 / 33 unknowns
 * per line; FDW_ENOTSUP beyond). */
typedef struct fdw_adi fdw_adi; /* opaque */

/* Device workspace (bytes) of one implicit solver for problem p (0 if p is invalid). */
size_t fdw_adi_workspace_bytes(const fdw_problem* p);

/* Create an implicit solver at step 0: p as for fdw_init (one member); sigma >= 0 the implicit
 * weight (0.25 recommended); workspace as for fdw_init (256-byte aligned, caller-owned);
 * u0, u1, h1: device [ny][nx] in the storage type; h2 device or NULL (h2 = h1).  h is validated
 * (finite, > 0, or >= 0 with FDW_ALLOW_ZERO_H) and for sigma < 1/4 the stability bound
 * tau^2 (4 max hx/dx^2 + 4 max hy/dy^2)(1 - 4 sigma) <= 4 is checked (FDW_ECFL; skipped with
 * FDW_ALLOW_UNSTABLE); both read results back, so this call synchronises the stream. */
int fdw_adi_init(const fdw_problem* p, double sigma, void* workspace, size_t ws_bytes, const void* u0, const void* u1,
                 const void* h1, const void* h2, void* hip_stream, fdw_adi** out);

/* Advance by n >= 0 steps (the start step first when at step 0); asynchronous. */
int fdw_adi_step_n(fdw_adi* s, int64_t n);

/* Copy (u^n, du^n) to device buffers [ny][nx] (either may be NULL) and the step counter to *n. */
int fdw_adi_get_state(fdw_adi* s, void* u, void* du, int64_t* n);

/* Return to step 0. */
int fdw_adi_reset(fdw_adi* s);

const char* fdw_adi_last_error(const fdw_adi* s);
void fdw_adi_destroy(fdw_adi* s);

/* Error reporting and teardown (no passage: execution control).  fdw_last_error: one line on the
 * context's last failure (owned by the context, valid until its next call); fdw_status_string:
 * static text of a status code; fdw_destroy: releases the host side of a context (the caller
 * still owns the workspace), NULL is ignored. */
const char* fdw_last_error(const fdw_ctx* ctx);
const char* fdw_status_string(int status);
void fdw_destroy(fdw_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
