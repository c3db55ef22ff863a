/*
 * rt.h -- C ABI of librtsc, an MI355X (gfx950) implementation of the short-
 * characteristics radiative transfer solver of Davis, Stone & Jiang (2012),
 * "A Radiation Transfer Solver for Athena using Short Characteristics".
 *
 * The library computes, on one GPU:
 *   - the formal solution J = Lambda[S] of the static transfer equation
 *     n.grad I = chi_tot (S - I) (section 2, eq. radtrans) by short
 *     characteristics on a Cartesian grid whose vertices are cell centres
 *     (section 3.3, eq. rtdisc, bilinear face interpolation): first order (psi+ = 0,
 *     S linear in optical depth along the segment) or second order (S a quadratic
 *     Bezier curve whose control point uses the downwind S, clamped so no new
 *     extrema appear);
 *   - the Jacobi accelerated Lambda iteration with the diagonal operator
 *     Lambda* (section 3.4, eq. dsjacobi) for S = (1 - eps) J + eps B
 *     (section 2, eq. sourcefunc), stopped by eq. conv, and its Gauss-Seidel form
 *     (section 3.4, horizontal planes as the blocks of the ordering);
 *   - the moments J, H, K (section 3.2, eqs. Jsum/Hsum/Ksum), the variable
 *     Eddington tensor f = K/J and the heating rate Q_rad (section 4).
 *
 * Conventions shared by every entry point
 *   - Field layout: C order [nf][nz][ny][nx] (x fastest), one value per vertex and
 *     frequency bin.  "cells" = nx*ny*nz.  The caller's field arrays (chi, eps, B,
 *     S, J, Lambda* and the moments outputs) are FP64 or, with
 *     rt_problem_desc.in_dtype = RT_DTYPE_F32, FP32; they are passed as void*.
 *     The library computes in FP64 (and in FP32 inside the RT_F32 sweeps) either
 *     way: FP32 arrays are widened on the device when read and rounded when written.
 *     Fixed incident intensities (I_fixed) are always FP64.
 *   - Device pointers are HIP device memory on the device that holds the problem:
 *     the device of its context (rt_context_create), or, created without one, the
 *     device current at creation.  Every call on a problem (and on a server) makes
 *     that device current for its duration and restores the caller's on return.
 *     Host pointers are ordinary host memory.  The caller owns every buffer it
 *     passes and must keep device buffers alive until the stream work has finished.
 *     The library owns the per-problem state it allocates (internal copies of the
 *     fields, Lambda*, the periodic memory, scratch) and frees it in
 *     rt_problem_destroy.
 *   - Every argument is validated before any device work is queued: a call that
 *     returns RT_E_INVALID has changed nothing.  The reason is kept in
 *     rt_last_error(): per context for calls on its problems, servers and batches,
 *     and per host thread for every call.  No call throws.
 *   - Streams are hipStream_t values passed as void* (NULL = the null stream).
 *   - A problem, and a context, is used by one host thread at a time.
 *   - Environment: RTSC_TILE_ORDER_SEED = n (n != 0) when a problem is created makes
 *     each launch of the tile wavefront take the tiles of its stage in an order
 *     shuffled with seed n.  Tiles of one stage are independent, so results are
 *     bitwise those of the default order; the switch exists to check that.
 */
#ifndef RTSC_RT_H
#define RTSC_RT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RT_OK = 0,
    RT_NOT_CONVERGED = 1,   /* results valid but max_iter reached */
    RT_E_INVALID = -1,      /* bad argument; nothing was done */
    RT_E_OOM = -2,          /* device allocation failed */
    RT_E_HIP = -3,          /* a HIP runtime call failed */
    RT_E_NONFINITE = -4,    /* a residual became NaN or Inf */
    RT_E_UNSUPPORTED = -5,  /* valid request the library does not implement */
    RT_E_BUSY = -6          /* rt_server_poll, rt_problem_destroy: a request is queued or running */
} rt_status;

/* Sweep arithmetic.  RT_F64 integrates I itself in FP64 ("plain form").
 * RT_F32 integrates D = I - S in FP32 (algebraically the same recurrence);
 * Lambda*, the ALI update, residuals and all sums stay FP64 in both. */
typedef enum { RT_F64 = 0, RT_F32 = 1 } rt_precision;

/* Element type of the caller's field arrays (rt_problem_desc.in_dtype). */
typedef enum { RT_DTYPE_F64 = 0, RT_DTYPE_F32 = 1 } rt_dtype;

/* Boundary kinds (section 3.5): intensity entering through a face is zero
 * (VACUUM), the thermal source function B of the boundary vertex (THERMAL),
 * a caller-given array (FIXED), or the intensity the previous sweep produced
 * at the opposite face (PERIODIC; both faces of the axis must be periodic). */
typedef enum { RT_BC_VACUUM = 0, RT_BC_THERMAL = 1, RT_BC_PERIODIC = 2, RT_BC_FIXED = 3 } rt_bc_kind;

/* Execution of the tile wavefront of one formal solution (section 3.1).
 * RT_SCHED_STAGES: one launch per tile hyperplane (the default).
 * RT_SCHED_PERSISTENT: one launch per formal solution; workgroups draw tiles in
 * hyperplane order from a per-octant counter and wait on completion flags of their
 * upwind neighbours (each wait bounded in time: a wait that runs out makes the call
 * return RT_E_HIP).  Built for RT_SC_LINEAR with RT_INTERP_BILINEAR; other
 * combinations get RT_E_UNSUPPORTED, and so does Gauss-Seidel with it. */
typedef enum { RT_SCHED_DEFAULT = 0, RT_SCHED_STAGES = 1, RT_SCHED_PERSISTENT = 2 } rt_schedule;

/* Order of the short-characteristic integration (section 3.3, eq. rtdisc).
 * RT_SC_LINEAR: S varies linearly in optical depth between the upwind point and the
 * vertex, I0 = I- e^-dtau + psi- S- + psi0 S0.
 * RT_SC_BEZIER: S is the quadratic Bezier curve from S0 to S- with control point
 * Sc = S0 - (dtau-/2) dS/dtau, the slope taken from the parabola through S-, S0 and
 * the downwind S+ (interpolated at the mirror image of the upwind point, optical depth
 * dtau+ = trapezoid of chi0 and chi+), then clamped to [min(S-, S0), max(S-, S0)];
 * I0 = I- e^-dtau + alpha S- + beta S0 + gamma Sc.  Where dtau+ = 0 the one-sided
 * slope (S0 - S-)/dtau- is used.  Lambda* (section 3.4) is sum_k w_k beta_k. */
typedef enum { RT_SC_LINEAR = 0, RT_SC_BEZIER = 1 } rt_sc_order;

/* Interpolation of the upwind intensity I- on the upwind face (section 3.3).
 * RT_INTERP_BILINEAR: bilinear in the 2 x 2 face vertices (tile wavefront sweep).
 * RT_INTERP_QUADRATIC: monotone quadratic on the 3 x 3 vertices of the upwind plane
 * (per line a quadratic Bezier curve whose control point, from the parabola through
 * the three points, is clamped between the two bracketing values: no overshoot,
 * positivity kept), along a then b.  Its stencil reaches the downwind side, so each
 * ray is swept plane by plane along the axis it crosses first; in-plane periodic
 * wraps read this sweep's values, and outside a non-periodic in-plane face the
 * downwind side (an outgoing face) repeats the value in line with the vertex.  S and
 * chi stay bilinear.  Requires order RT_SC_LINEAR.  In a batch (and in the server) such
 * a problem runs its own launches within the batch's iterations. */
typedef enum { RT_INTERP_BILINEAR = 0, RT_INTERP_QUADRATIC = 1 } rt_interp;

typedef struct {
    int32_t nx, ny, nz;       /* grid vertices per axis, each in [1, 8000], nx*ny*nz < 2^31 */
    int32_t nf;               /* frequency bins, >= 1 */
    double dx, dy, dz;        /* vertex spacing, > 0 */
    int32_t n_mu;             /* angle set LQ_{n_mu}, n_mu in {2,4,6,8,10,12}; used when mu == NULL */
    int32_t na;               /* number of rays when mu != NULL (multiple of 8) */
    const double *mu;         /* host [na][3] direction cosines or NULL; na/8 rays per octant */
    const double *w;          /* host [na] ray weights summing to 1 (with mu) */
    const double *w_nu;       /* host [nf] frequency quadrature weights, or NULL for all 1 */
    int32_t bc_lo[3];         /* rt_bc_kind at the low face of x, y, z */
    int32_t bc_hi[3];         /* rt_bc_kind at the high face of x, y, z */
    const double *I_fixed[6]; /* device, faces lo-x hi-x lo-y hi-y lo-z hi-z for RT_BC_FIXED:
                                 [nf][na][n2][n1], (n1, n2) the face's in-plane axes in
                                 increasing order (x-faces: y,z; y-faces: x,z; z-faces: x,y) */
    int32_t precision;        /* rt_precision */
    int32_t tile;             /* tile edge for the sweep (0 = default) */
    int32_t schedule;         /* rt_schedule: how the tile wavefront is executed */
    int32_t order;            /* rt_sc_order: first- or second-order segments */
    int32_t interp;           /* rt_interp: bilinear or monotone quadratic upwind intensity */
    int32_t in_dtype;         /* rt_dtype of the caller's field arrays (0 = FP64) */
} rt_problem_desc;

typedef struct rt_problem rt_problem;

/*
 * A context: one HIP device and the last error of the calls made through it.
 * rt_context_create -- device: a HIP device ordinal (RT_E_INVALID if there is no such
 *   device).  Problems created in the context live on that device; batches and servers
 *   given the context run there.  NULL may be passed wherever a context is taken: the
 *   device current at the call is used and errors are kept per thread only.
 * rt_context_destroy -- frees the context; its problems and servers must be destroyed
 *   first.
 */
typedef struct rt_context rt_context;

rt_status rt_context_create(int32_t device, rt_context **out);
rt_status rt_context_destroy(rt_context *ctx);

/* Human-readable text of a status; the last failure recorded in a context (ctx), or
 * on the calling thread (ctx = NULL).  The text stays valid until the next call on
 * the same thread. */
const char *rt_status_string(rt_status s);
const char *rt_last_error(const rt_context *ctx);

/*
 * rt_quadrature -- the level-symmetric angle set of section 3.2: n_a = n_mu (n_mu + 2)
 * rays, identical in every octant and invariant under 90-degree rotations.  The
 * directions per octant are (mu_i, mu_j, mu_k) with i + j + k = n_mu/2 + 2 and
 * mu_i^2 = mu_1^2 + (i - 1) 2 (1 - 3 mu_1^2)/(n_mu - 2); mu_1 and one weight per
 * permutation class satisfy sum_k w_k mu_x^2p = 1/(2p+1), p = 0, 2..n_mu/2.
 * mu_out: host [n_mu(n_mu+2)][3]; w_out: host [n_mu(n_mu+2)]; either may be NULL
 * to query *na_out only.  Octant-major order: octant o has the signs
 * (-1)^(o&1), (-1)^(o>>1&1), (-1)^(o>>2&1) on x, y, z.
 */
rt_status rt_quadrature(int32_t n_mu, double *mu_out, double *w_out, int32_t *na_out);

/* Device bytes rt_problem_create would allocate for this description. */
rt_status rt_problem_bytes(const rt_problem_desc *desc, size_t *bytes);

/* Create the per-problem device state on the context's device (ctx may be NULL: the
 * current device). */
rt_status rt_problem_create(rt_context *ctx, const rt_problem_desc *desc, rt_problem **out);
/* Frees the problem's device state.  RT_E_BUSY (nothing freed) while a server
 * request on the problem is queued or running. */
rt_status rt_problem_destroy(rt_problem *p);

/*
 * rt_problem_set_fields -- radiative properties per vertex and bin (section 2,
 * eq. sourcefunc; section 3.1): chi = chi_abs + chi_sc (> 0 or 0), eps =
 * chi_abs/chi_tot in [0, 1], B the thermal source function.  Device
 * [nf][nz][ny][nx] in the problem's in_dtype.  The values are copied (widened to
 * FP64); the caller may reuse its buffers once the stream has passed this call.
 * Computes Lambda* (the diagonal of section 3.4) and resets the periodic memory to
 * its cold state.
 */
rt_status rt_problem_set_fields(rt_problem *p, const void *chi, const void *eps,
                                const void *B, void *stream);

/* Forget the previous sweep: periodic ghosts read S of the wrapped vertex on the
 * next sweep (cold start of the periodic iteration, section 3). */
rt_status rt_problem_reset_periodic(rt_problem *p, void *stream);

/*
 * Checkpoint and resume of the periodic memory.  Besides S (the caller's), the only
 * state an iteration hands to the next is what section 3's iteration for periodic
 * boundaries keeps: the intensities each ray carried out of its periodic faces on the
 * last sweep, which the next sweep reads as ghosts (or, on a cold problem, the flag
 * that S of the wrapped vertex stands in for them).  Saving that memory with S and
 * loading both into a problem of the same description continues an ALI (warm_start =
 * 1) with bitwise the results of the uninterrupted run, in this or another process.
 *
 * rt_problem_state_bytes -- size of the saved state (a header, the per-bin slot
 *   selectors and the periodic buffers, about nf * na * 2 * (sum over periodic axes of
 *   the face's vertices) * 8 bytes; for the quadratic interpolation the plane buffers
 *   nf * na * 2 * (largest face) reals plus, in FP32, nf * na * (largest face) * 8).
 * rt_problem_save_state -- write the state to dst (host or device, `bytes` >= the
 *   size above, else RT_E_INVALID).  Synchronises the stream first: the state is the
 *   one left by the work queued before the call.
 * rt_problem_load_state -- read a state saved from a problem with the same shape, bin
 *   count, angle set, precision, interpolation and periodic axes (else RT_E_INVALID,
 *   and the problem is unchanged).  rt_problem_set_fields resets the periodic memory,
 *   so load after setting the fields.  Synchronises the stream first.
 * Neither call may overlap a batch or a server solve of the same problem.
 */
rt_status rt_problem_state_bytes(rt_problem *p, size_t *bytes);
rt_status rt_problem_save_state(rt_problem *p, void *dst, size_t bytes, void *stream);
rt_status rt_problem_load_state(rt_problem *p, const void *src, size_t bytes, void *stream);

/*
 * rt_formal_solve -- one formal solution J = Lambda[S] (section 3.4, eq. formalsol):
 * every ray is integrated once over the grid (section 3.3).  Periodic ghosts come
 * from the previous sweep of this problem (section 3's iteration for periodic
 * boundaries) or, after create/reset, from S.  S: device [nf][cells] (read); J:
 * device [nf][cells] (written); lambda_star: device [nf][cells] or NULL, receives
 * Lambda*_ii = sum_k w_k psi0_k; all in the problem's in_dtype.  Asynchronous on the
 * stream, except with RT_SCHED_PERSISTENT outside stream capture: then the call
 * synchronises the stream after the sweep to read the dependency-wait flag, and
 * returns RT_E_HIP if a wait ran out (under capture that check is skipped).
 */
rt_status rt_formal_solve(rt_problem *p, const void *S, void *J, void *lambda_star,
                          void *stream);

typedef struct {
    double delta_c;        /* stop when max |dS|/S <= delta_c (eq. conv) */
    int32_t max_iter;      /* give up after this many iterations (RT_NOT_CONVERGED) */
    int32_t fixed_iters;   /* > 0: run exactly this many iterations, no test */
    int32_t per_bin_stop;  /* non-zero: a bin stops as soon as it converges */
    int32_t warm_start;    /* 0: S0 = B; 1: S0 = S_inout; 2: S0 = eps B + (1-eps) J_inout */
    int32_t check_every;   /* iterations between host checks of convergence (0 = default) */
} rt_ali_opts;

typedef struct {
    int32_t iterations;       /* largest iteration count over bins */
    int32_t bins_converged;
    double max_rel_dS;        /* largest last residual over bins */
    double seconds;           /* host wall time of the call */
} rt_ali_stats;

/*
 * rt_ali_solve -- Jacobi ALI (section 3.4).  Iteration n: J^n = Lambda[S^n];
 *   dS = ((1-eps) J^n + eps B - S^n) / (1 - (1-eps) Lambda*)   (eq. dsjacobi)
 *   S^{n+1} = S^n + dS;  r = max over cells with S^{n+1} != 0 of |dS|/|S^{n+1}|  (eq. conv)
 * per bin, in FP64.  On return S_inout holds S^{n+1} and J_out holds J^n of each
 * bin's last iteration.  Start values per opts->warm_start; S_inout, J_out: device
 * [nf][cells] in the problem's in_dtype (with FP32 arrays the iteration runs on FP64
 * copies the library keeps, and S and J are rounded to FP32 at the end).
 * Synchronises the stream every check_every iterations to read the convergence
 * flags; stats (host, may be NULL) reports them.
 * Returns RT_OK, RT_NOT_CONVERGED or RT_E_NONFINITE (outputs then undefined).
 */
rt_status rt_ali_solve(rt_problem *p, const rt_ali_opts *opts, void *S_inout, void *J_out,
                       rt_ali_stats *stats, void *stream);

/*
 * rt_ali_solve_gs -- Gauss-Seidel ALI (section 3.4: the update of eq. dsjacobi is
 * applied as soon as J of a vertex is complete, so later short characteristics see
 * the new S; the scheme the paper takes from Trujillo Bueno & Fabiani Bendicho 1995
 * and generalises to 3D with bilinear interpolation).  The blocks of the ordering are
 * the horizontal planes from the top (z = nz - 1) down: per iteration the rays going
 * up (direction cosine along z >= 0) are swept with S^n, then for each plane from the
 * top the rays going down complete J on it (planes above already updated), the plane
 * is updated, and its downward intensities are recomputed with the new S.  Vertices of
 * one plane are updated together (Jacobi within a plane); when every ray crosses a z
 * face first (no coupling inside a plane) this is point Gauss-Seidel.  Periodic ghosts
 * (x, y) read the previous iteration's outgoing intensities for the whole iteration.
 * Arguments, start values, stopping rule (eq. conv per bin), outputs, statuses and
 * rt_ali_bin_stats as for rt_ali_solve; J_out holds the J each vertex was last
 * updated with.  Needs order = RT_SC_LINEAR, interp = RT_INTERP_BILINEAR, a
 * non-periodic z axis, the staged schedule and nx, ny <= 256; else RT_E_UNSUPPORTED
 * before any work.  The first call on a problem allocates its plane buffers
 * (nf * (na/2) * 3 * nx * ny reals).
 */
rt_status rt_ali_solve_gs(rt_problem *p, const rt_ali_opts *opts, void *S_inout, void *J_out,
                          rt_ali_stats *stats, void *stream);

/*
 * Launch shape of the tile-wavefront sweep.  A sweep workgroup takes one 8^3 tile of
 * one octant and bin with `waves` 64-lane waves; with fewer waves than rays per octant
 * (R = na/8) each wave runs several rays in turn.  rt_problem_create picks
 * min(R, 10) waves (as many as fit the device's LDS).
 *
 * rt_problem_set_waves -- use `waves` in [1, min(R, 10)] (RT_E_INVALID outside,
 * RT_E_UNSUPPORTED if the LDS does not fit or for the plane-ordered sweep).  Results
 * change only in the rounding of the sums over the waves.  Host-only call.
 *
 * rt_problem_tune -- time `reps` formal solutions of S (device [nf][cells] in the
 * problem's in_dtype, fields set) for every wave count that fits, keep the fastest, and report it in *waves_out;
 * ms_out (host [10] or NULL) receives the milliseconds per sweep of each count (-1
 * where it does not fit).  The periodic memory the next solve reads is left as it was
 * (a problem with no sweep yet stays cold).  Synchronises the stream.
 */
rt_status rt_problem_set_waves(rt_problem *p, int32_t waves);
rt_status rt_problem_tune(rt_problem *p, const void *S, int32_t reps, int32_t *waves_out, float *ms_out,
                          void *stream);

/*
 * rt_problem_set_wait_limit -- bound of one dependency wait of the persistent schedule
 * (section 3.1: a tile waits for its upwind neighbours), in microseconds of the
 * device's constant-rate clock; the default is 20000.  A wait that runs out makes
 * the call that ran the sweep return RT_E_HIP (the launch still completes; its
 * results are not valid).  For devices shared with other work a longer bound may be
 * needed; 0 makes every wait whose flag is not already set fail (a test of that path
 * needs nothing else).  In a batch the largest bound among a class's members applies.
 * RT_E_INVALID for a negative, non-finite or larger than 1e9 value.  No effect on the
 * staged schedule.  Host-only call.
 */
rt_status rt_problem_set_wait_limit(rt_problem *p, double microseconds);

/*
 * rt_problem_use_graphs -- rt_ali_solve and rt_ali_solve_gs run their iterations in
 * chunks of check_every (the host reads the convergence flags between chunks).  With
 * graphs enabled (the default) a chunk is captured once as a HIP graph on a stream of
 * the problem's own and then replayed on the caller's stream; kernels of converged
 * bins return at once, so a chunk that passes convergence costs little.  The captured
 * launches are those of the eager path, in the same order with the same arguments, so
 * results are bitwise the same either way.  A problem caches two graphs (the full chunk
 * and a shorter last one) keyed by the S and J pointers and the stopping options; the
 * one-time periodic initialisation and any sweep timed by rt_problem_profile run
 * eagerly.  enable = 0 runs every launch from the host.  Host-only call.
 */
rt_status rt_problem_use_graphs(rt_problem *p, int32_t enable);

/* Per-bin iteration counts and last residuals of the most recent rt_ali_solve
 * (host arrays [nf]; either may be NULL).  Synchronises the stream. */
rt_status rt_ali_bin_stats(rt_problem *p, int32_t *iters, double *resid, void *stream);

/*
 * rt_ali_solve_batch -- rt_ali_solve for n independent problems at once (bins and
 * problems do not couple, section 3.1).  Each problem keeps its own grid, rays,
 * bins, boundaries and precision; they may all differ.  Problems of the same sweep
 * precision and waves per workgroup share every launch: per iteration one ghost-value
 * launch, one launch per stage index covering that hyperplane of all of them, one
 * update and one convergence launch.  Problems created with RT_SCHED_PERSISTENT form
 * classes of their own, whose sweep is one persistent launch over the tiles of all
 * their members (listed stage by stage, so every tile's upwind neighbours come
 * first; each member keeps its own completion flags).  A problem with the quadratic upwind intensity
 * runs its own plane-step, update and convergence launches in the same iterations.  A problem that meets the stopping rule (or its
 * max_iter / fixed_iters) leaves the batch at the next check; the others go on.
 * Results per problem are those rt_ali_solve gives for it alone (identical
 * arithmetic).  ctx: the context whose device runs the batch and keeps its errors,
 * or NULL (the current device); every problem must live on that device.  problems:
 * host array [n] of distinct problems with fields set; S_inout, J_out: host arrays
 * [n] of device pointers as for rt_ali_solve (each in its problem's in_dtype); stats,
 * results: host arrays [n] or NULL (per-problem RT_OK / RT_NOT_CONVERGED /
 * RT_E_NONFINITE; stats.seconds = wall time until that problem left the batch).
 * opts apply to every problem.  A dependency wait of a persistent sweep that runs
 * out (rt_problem_set_wait_limit) ends the members of the persistent classes with
 * RT_E_HIP at that check; the others go on.  Returns RT_E_HIP if any member ended so,
 * else RT_E_NONFINITE if any problem hit a non-finite residual, else
 * RT_NOT_CONVERGED if any did not converge, else RT_OK.  Synchronises the stream
 * every check_every iterations.
 */
rt_status rt_ali_solve_batch(rt_context *ctx, rt_problem *const *problems, int32_t n, const rt_ali_opts *opts,
                             void *const *S_inout, void *const *J_out, rt_ali_stats *stats,
                             rt_status *results, void *stream);

/*
 * Serving loop: ALI solves submitted at any time run together in one batch (as in
 * rt_ali_solve_batch) on a worker thread of the server with its own stream on the
 * device of its context (ctx, or with ctx = NULL the device current at
 * rt_server_create); submitted problems must live on that device.  Requests are admitted in arrival
 * order at the batch's convergence checks while the summed rt_problem_bytes of the
 * admitted problems stays within hbm_budget (a request larger than the budget runs
 * alone); the rest wait in the queue.  A problem keeps its device state between
 * requests, so a request with opts.warm_start = 1 or 2 continues from the caller's
 * S or J and the problem's periodic memory (warm starts for later snapshots,
 * section 4).  While a request is queued or running the caller must not use its
 * problem, S or J.  check_every: iterations between checks (0 = 16).
 */
typedef struct rt_server rt_server;

rt_status rt_server_create(rt_context *ctx, size_t hbm_budget, int32_t check_every, rt_server **out);

/* Queue an ALI solve (arguments as for rt_ali_solve); *ticket identifies it.
 * The problem must not be part of another queued or running request.  `stream` is the
 * caller's stream that produced the request's inputs (the problem's fields, S, J): the
 * call records an event on it, and the server's stream waits for that event before
 * any of the request's device work, so work the caller queued on that stream before
 * the call (set_fields, writes to S or J) is complete when the solve reads it.
 * Inputs written on other streams must be complete before the call.  The caller
 * must not touch S or J (or destroy the problem) until rt_server_poll reports the
 * request finished; the library only holds the pointers. */
rt_status rt_server_submit(rt_server *srv, rt_problem *p, const rt_ali_opts *opts, void *S_inout,
                           void *J_out, void *stream, uint64_t *ticket);

/* RT_E_BUSY while the request is queued or running; RT_OK once it has finished,
 * with *result its solve status (RT_OK, RT_NOT_CONVERGED, RT_E_NONFINITE, RT_E_HIP
 * for a persistent-schedule request whose dependency wait ran out (the server goes
 * on), or the error that stopped the server) and *stats its statistics (seconds = time from
 * submission to completion, queueing included).  Either output may be NULL.  A
 * finished ticket can be polled until rt_server_release; unknown tickets give
 * RT_E_INVALID.  Never blocks on the device. */
rt_status rt_server_poll(rt_server *srv, uint64_t ticket, rt_ali_stats *stats, rt_status *result);

/* Forget a finished ticket's record. */
rt_status rt_server_release(rt_server *srv, uint64_t ticket);

/* Counts of queued and running requests, and the summed rt_problem_bytes of the
 * running ones (admission keeps it within hbm_budget unless one request larger than
 * the budget runs alone); any output may be NULL. */
rt_status rt_server_load(rt_server *srv, int32_t *queued, int32_t *running, size_t *running_bytes);

/* Finish every queued and running request, stop the worker and free the server. */
rt_status rt_server_destroy(rt_server *srv);

/* Device outputs in the problem's in_dtype (FP64 sums rounded once at the end when
 * FP32); heating is a host FP64 scalar either way. */
typedef struct {
    void *J;           /* device [nf][cells] or NULL */
    void *H;           /* device [3][nf][cells] or NULL */
    void *K;           /* device [6][nf][cells] (xx yy zz xy xz yz) or NULL */
    void *J_int;       /* device [cells]: sum_nu w_nu J_nu, or NULL */
    void *H_int;       /* device [3][cells] or NULL */
    void *K_int;       /* device [6][cells] or NULL */
    void *f_int;       /* device [6][cells]: K_int/J_int (0 where J_int = 0), or NULL; needs J_int, K_int */
    void *Q_int;       /* device [cells]: sum_nu w_nu Q_nu, or NULL */
    double *heating;   /* host scalar: sum over cells of Q_int dV, or NULL (synchronises) */
} rt_moments_out;

/*
 * rt_moments -- one formal solution on S with moments (section 3.2, eqs.
 * Jsum/Hsum/Ksum), the Eddington tensor f = K/J and the heating rate of section 4:
 * Q_nu = 4 pi eps chi (J - B) where chi min(dx,dy,dz) <= 1, else -4 pi div H (second-order
 * differences, wrapped on periodic axes, one-sided at other faces).  Frequency
 * integrals use w_nu, bins added in order.  Every output pointer may be NULL; f_int
 * needs J_int and K_int.  Periodic ghosts as in rt_formal_solve (the periodic memory
 * advances by one sweep).  Asynchronous unless heating is requested (then the stream
 * is synchronised to return the FP64 sum over cells of Q_int dV).
 */
rt_status rt_moments(rt_problem *p, const void *S, const rt_moments_out *out, void *stream);

/*
 * Sweep-kernel timing, for measuring the formal solution against its roofline.
 * While enabled, the stage launches of one formal solution (the first iteration of
 * each convergence-check interval of rt_ali_solve, and every rt_formal_solve) are
 * bracketed by two HIP events on the call's stream, after the ghost-value pass and
 * after the last stage; the durations are summed when the events have completed,
 * so a launch's share includes the gap to the next launch.  In rt_ali_solve_gs the
 * same first iteration of each interval also times the chain launches of the
 * downward pass that compute a plane and recompute the one above (steps 1 .. nz-1;
 * rays crossing an x or y face first), each by a pair of events that take the start
 * and end of that dispatch itself; the chain_* fields sum those.  Enabling (or disabling) resets the totals.
 */
typedef struct {
    double kernel_ms;       /* summed duration of the timed back-to-back stage launches */
    int64_t launches;       /* number of timed launches */
    int64_t sweeps;         /* number of timed formal solutions */
    double updates;         /* cell*ray*bin updates done by those launches */
    int32_t stages;         /* launches per formal solution */
    double chain_ms;        /* Gauss-Seidel: summed duration of the timed chain launches */
    int64_t chain_launches; /* number of timed chain launches */
    double chain_updates;   /* vertex*ray*bin chain updates they did (each a new and a recomputed intensity) */
} rt_profile;

rt_status rt_problem_profile(rt_problem *p, int32_t enable);
rt_status rt_problem_profile_read(rt_problem *p, rt_profile *out);

/*
 * rt_formal_solve_noalloc -- for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * formal solution of rt_formal_solve on a newly created problem with these fields
 * (periodic ghosts cold: S of the wrapped vertex), computed with the same kernels and
 * launch shape, so J and lambda_star are bitwise those of rt_problem_create +
 * rt_problem_set_fields + rt_formal_solve.  It allocates nothing: its internal
 * state lives in a library-owned device array of 64 MiB per GPU, held until the
 * process ends, and the ray table and tile list are built on the device from kernel
 * arguments.  desc: as for rt_problem_create, with in_dtype RT_DTYPE_F64, the
 * bilinear upwind intensity, the staged schedule (RT_SCHED_PERSISTENT gets
 * RT_E_UNSUPPORTED) and at most 80 rays (n_mu <= 8); chi, B: device FP64
 * [nf][cells] (B for thermal boundaries); S (read), J (written), lambda_star (written
 * or NULL): device FP64 [nf][cells]; I_fixed as in the description.  Problems whose
 * workspace exceeds the 64 MiB (about 64^3 x 48 rays x 1 bin in FP32) return
 * RT_E_UNSUPPORTED, other bad arguments RT_E_INVALID, before any device work.
 * Asynchronous on the stream, on the current device.  Every call on a GPU shares its
 * array and keeps the last call's contents: calls that overlap on one GPU (other
 * streams or host threads before the previous one finished) race, and must be
 * serialised by the caller.
 */
rt_status rt_formal_solve_noalloc(const rt_problem_desc *desc, const void *chi, const void *B, const void *S,
                                  void *J, void *lambda_star, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* RTSC_RT_H */
