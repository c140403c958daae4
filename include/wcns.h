/*
 * wcns.h -- C ABI of the MI355X (gfx950) implementation of the right-hand
 * side of the positivity- and boundedness-preserving incremental-stencil
 * weighted compact nonlinear scheme (PP-WCNS-IS) for Allaire's five-equation
 * gas-liquid model (Wong, Angel, Barad, Kiris, arXiv 2102.05287).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns a wcns_status; no exception crosses the ABI.
 *  - State arrays are DEVICE pointers to float64, structure-of-arrays
 *    [nvar][ny][nx] (x fastest), interior cells only (no ghost layers).
 *      3D: nvar = 7, (a1*rho1, a2*rho2, rho*u, rho*v, rho*w, E, a1),
 *          layout [7][nz][ny][nx]
 *      2D: nvar = 6, (a1*rho1, a2*rho2, rho*u, rho*v, E, a1)
 *      1D: nvar = 5, (a1*rho1, a2*rho2, rho*u, E, a1)           (ny = 1)
 *    This is the conservative vector W of the paper (Sec. 2, Sec. 3).
 *  - The caller owns every state buffer; the context owns its scratch, which
 *    is allocated once in wcns_create.  rhs/step/limit allocate nothing, so
 *    a sequence of calls can be captured into a HIP graph.
 *  - All kernels are enqueued on the context's stream (set at creation or
 *    by wcns_set_stream); calls are asynchronous unless stated otherwise.
 *    Calls on one context must not overlap (they share its scratch).
 *  - Device pointers are checked for NULL only, not for residency or size
 *    (that would cost a runtime query per call): a host pointer or a buffer
 *    shorter than stated is the caller's error and faults the kernel that
 *    touches it.  The Python binding checks every tensor it passes.
 *  - Admissibility is reported lazily (the admissible set G of Sec. 2:
 *    0 <= a1 <= 1, a_k r_k >= 0, rho e - pbar_inf > 0; the limiters of
 *    Sec. 5 exist to keep every stage result inside it).  The kernels count,
 *    with no host synchronisation, every input cell of a call's first stage
 *    and every stage result (cell states after an SSP-RK3 stage) that lies
 *    outside G.  Once a count has been made visible to the host, every later
 *    call that enqueues work on the context (wcns_rhs, wcns_limit,
 *    wcns_max_wavespeed, wcns_ssprk3_step[s], wcns_ssprk3_advance, wcns_run)
 *    returns WCNS_ERR_INADMISSIBLE without enqueuing anything, until
 *    wcns_violations reads and clears the count.  Work already enqueued runs
 *    on (the states it writes are then no longer meaningful).
 */
#ifndef WCNS_H_
#define WCNS_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WCNS_OK = 0,
  WCNS_ERR_ARG = -1,          /* bad argument (null pointer, size < 1, ...)    */
  WCNS_ERR_EOS = -2,          /* fluids violate Lemma 1 / Theorem 1 (Sec. 2):  */
                              /* one phase must have pinf = 0 and the other a  */
                              /* ratio of specific heats >= the gas one        */
  WCNS_ERR_NOMEM = -3,        /* device allocation failed                      */
  WCNS_ERR_HIP = -4,          /* a HIP runtime call failed                     */
  WCNS_ERR_INADMISSIBLE = -5, /* a state lies outside the admissible set G     */
  WCNS_ERR_CFL = -6,          /* non-finite or non-positive time step          */
  WCNS_ERR_TOO_LARGE = -7     /* grid needs more than the allocation-free      */
                              /* entry point's static scratch                  */
} wcns_status;

typedef enum {
  WCNS_BC_PERIODIC = 0,
  WCNS_BC_EXTRAP = 1,         /* constant (zeroth-order) extrapolation         */
  WCNS_BC_REFLECT = 2,        /* mirror state, negate wall-normal momentum     */
  WCNS_BC_DIRICHLET = 3       /* fixed ghost states (grid.dirichlet[_rows])    */
} wcns_bc;

typedef enum { WCNS_FP64 = 0, WCNS_FP32_BULK = 1 } wcns_precision;
typedef enum { WCNS_SCHEME_PPWCNSIS = 0, WCNS_SCHEME_HLLC1 = 1 } wcns_scheme;

/* Fluids (Sec. 2 stiffened gas; Table 1): [0] liquid, [1] ideal gas. */
typedef struct {
  double gamma[2];
  double pinf[2];
} wcns_eos;

/* Uniform Cartesian grid (Sec. 3: cells of size dx = (x1-x0)/nx). */
typedef struct {
  int32_t ndim;               /* 1, 2 or 3 (3D: the direct extension of Sec. 2) */
  int32_t nx, ny;             /* ny = 1 when ndim = 1                          */
  double x0, x1, y0, y1;
  int32_t bc[4];              /* wcns_bc of x-lo, x-hi, y-lo, y-hi             */
  double dirichlet[4][6];     /* host; PRIMITIVE ghost state per side          */
                              /* (a1r1, a2r2, u, [v], p, a1), nvar values, for */
                              /* DIRICHLET sides without a row profile         */
  const double* dirichlet_rows[4];
                              /* host, optional (NULL: dirichlet[side] for the */
                              /* whole side): primitive ghost state of each    */
                              /* boundary row, [n_side][nvar], n_side = ny for */
                              /* x-lo/x-hi and nx for y-lo/y-hi (e.g. the jet  */
                              /* inflow of Sec. 6.7).  The three ghost layers  */
                              /* of a row share its state.  Copied at create;  */
                              /* the caller keeps ownership.                   */
  int32_t nz;                 /* 3D: cells along z (ignored below 3D)          */
  int32_t bc_z[2];            /* 3D: wcns_bc of z-lo, z-hi                     */
  int32_t reserved_z;
  double z0, z1;              /* 3D: z extent                                  */
} wcns_grid;

/* Scheme options; wcns_params_default fills the paper's values. */
typedef struct {
  double eps_arho, eps_alpha, eps_rhoc2;  /* limiter tolerances, Sec. 5.1: 1e-10, 1e-10, 1e-8 */
  double hs_arho, hs_alpha, hs_rhoc2;     /* hard-switch tolerances: 1e-11, 1e-11, 1e-9       */
  double weno_eps;                        /* epsilon of the IS weights (Sec. 4.3); the paper  */
                                          /* gives none; default 1e-40; accepted in           */
                                          /* [1e-200, 1e200] (WCNS_ERR_ARG otherwise), where  */
                                          /* every IS-weight quotient tau_5/(beta + eps) has  */
                                          /* the normal-range operands the kernels' division  */
                                          /* core rounds exactly                              */
  double cfl;                             /* CFL number, <= 0.5 (Sec. 3.3, 5.3); default 0.5  */
  int32_t interp_limiter;                 /* 1: apply Algorithms 1-3 (Sec. 5.1)               */
  int32_t flux_limiter;                   /* 1: apply Algorithms 4-6 (Sec. 5.2)               */
  int32_t scheme;                         /* wcns_scheme                                      */
  int32_t reserved;
} wcns_params;

typedef struct wcns_ctx wcns_ctx;

/* Fill p with the paper's defaults. WCNS_ERR_ARG if p is NULL. */
wcns_status wcns_params_default(wcns_params* p);

/* Create a context for one grid.  Validates the fluids against Lemma 1
 * (WCNS_ERR_EOS), the grid (nx, ny >= 1, ndim in {1,2,3}, bc kinds, reflective
 * sides need >= 3 cells) and the parameters (cfl in (0, 0.5], weno_eps in
 * [1e-200, 1e200], the six tolerances finite and > 0 with eps_alpha and
 * hs_alpha < 1/2, scheme, precision; WCNS_ERR_ARG), checks the
 * Dirichlet ghost states (finite, partial densities >= 0 with a positive sum,
 * 0 <= a1 <= 1, p + pbar_inf > 0, i.e. inside G; else WCNS_ERR_INADMISSIBLE;
 * all before any device call), then allocates all device
 * scratch once (WCNS_ERR_NOMEM).  stream: hipStream_t or NULL for
 * the default stream.  On success *out owns the scratch until wcns_destroy.
 * 3D grids (ndim = 3): FP64 only, sides periodic, extrapolated or
 * reflective (no Dirichlet), nx*ny*nz < 2^29, nz <= 65535 (WCNS_ERR_ARG
 * otherwise); wcns_limit is not available in 3D. */
wcns_status wcns_create(const wcns_grid* grid, const wcns_eos* eos, const wcns_params* params,
                        int32_t precision, void* stream, wcns_ctx** out);

/* Release the context and its scratch (synchronises its stream). */
wcns_status wcns_destroy(wcns_ctx* ctx);

/* Change the stream later calls enqueue on.  Work already enqueued on the
 * previous stream is not waited for: a caller that switches streams orders
 * the two itself (e.g. with an event), since both use the context's scratch.
 * With profiling on, the timings recorded so far are folded first (this
 * synchronises the previous stream). */
wcns_status wcns_set_stream(wcns_ctx* ctx, void* stream);

/* Primitive -> conservative on the device (Sec. 2 mixture EOS):
 * V = (a1r1, a2r2, u, [v], p, a1) SoA -> W, both device [nvar][ny][nx]. */
wcns_status wcns_prim_to_cons(wcns_ctx* ctx, const double* V, double* W);

/* Semi-discrete right-hand side L(W) (Sec. 4.1 flux-difference form with the
 * split fluxes G^{+-} of Sec. 3.2, the WCNS steps of Sec. 4.2, the limiters
 * of Sec. 5).  dt is the forward-Euler step the flux limiter protects: the
 * limiter uses lambda = dt/(dx sigma) with sigma from W (Sec. 3.3).
 * W, dWdt: device [nvar][ny][nx]; must not alias.  Asynchronous. */
wcns_status wcns_rhs(wcns_ctx* ctx, const double* W, double* dWdt, double dt);

/* Stand-alone flux limiter of one sweep direction (Algorithms 4-6 and the
 * hard switch, Sec. 5.2).  dir 0: x-faces, layout [ny][nx+1]; dir 1:
 * y-faces, layout [ny+1][nx]; face (k, line) lies between cells k-1 and k.
 * G_ho, G_lo: device SoA [nvar+1][nfaces]: the high-order reconstructed flux
 * Ghat (nvar components in the state order, alpha slot = fhat_alpha) and, in
 * the last row, uhat; G_lo the same for the first-order HLLC flux.
 * G_out: device SoA [2][nvar][nfaces]: limited G^- then G^+.
 * theta: device [nfaces] (may be NULL): smallest theta applied, 0 if the hard
 * switch fired.  lambda is computed from W and dt as in wcns_rhs. */
wcns_status wcns_limit(wcns_ctx* ctx, int32_t dir, const double* W, const double* G_ho,
                       const double* G_lo, double* G_out, double* theta, double dt);

/* A whole run of a small 1D problem (nx <= 4096; the paper's Sec. 6.2-6.4
 * experiments) with the time loop on the device: SSP-RK3 steps of W (device,
 * in place) from time t0 until t_end or max_steps steps, each step the CFL
 * step of Sec. 3.3 (dt_fixed = 0) or dt_fixed, the last one shortened to land
 * on t_end; every step is the arithmetic of wcns_ssprk3_step, so the result
 * equals stepping with it.  One workgroup runs the loop (one launch per
 * 1024 steps instead of five per stage).  dts (device, optional): dt of step k at
 * dts[k] for k < dts_cap.  Synchronous: *steps_out and *t_out (host) receive
 * the steps taken and the final time.  Cells outside G (the run's input,
 * every stage result) are counted as by the other entry points.
 * WCNS_ERR_ARG for 2D/3D or larger grids, WCNS_ERR_CFL for non-finite times
 * or a negative dt_fixed, and for a run that stopped short of t_end and
 * max_steps because a step would not advance the time (an infinite wave
 * speed; *steps_out and *t_out then give where it stopped). */
wcns_status wcns_run(wcns_ctx* ctx, double* W, double t0, double t_end, double dt_fixed,
                     int64_t max_steps, double* dts, int64_t dts_cap, int64_t* steps_out,
                     double* t_out);

/* Maximum wave speeds max(|u|+c), max(|v|+c) (Sec. 3.3) over the cells and
 * the ghost states of Dirichlet sides (those of the x sides count for the
 * first, of the y sides for the second), i.e. over every state a face flux of
 * that direction sees; the CFL time step and lambda use the same maxima.
 * d_amax: device double[2] (the second entry is 0 in 1D); double[3] in 3D
 * (the third maximum is max(|w|+c)). */
wcns_status wcns_max_wavespeed(wcns_ctx* ctx, const double* W, double* d_amax);

/* One three-stage SSP Runge-Kutta step (TVD-RK3, Sec. 5.3, Sec. 6) in place
 * on W.  dt > 0: that step; dt <= 0: CFL step dt = cfl/(tau_x + tau_y) from
 * the state at the start of the step, computed on the device.  Every stage
 * evaluates sigma/lambda from its own input state.  dt_used: device double*
 * (may be NULL) receives the step taken.  Asynchronous; no host sync. */
wcns_status wcns_ssprk3_step(wcns_ctx* ctx, double* W, double dt, double* dt_used);

/* nsteps such steps (Sec. 5.3) in place on W, each with dt > 0 or, dt <= 0,
 * its own device CFL step; dts: device array of >= nsteps doubles (may be
 * NULL) receiving step k's dt at dts[k].  Bit for bit the same as nsteps
 * calls of wcns_ssprk3_step.  In 2D the node primitives and wave-speed
 * maxima of each step's first stage come from the previous step's last
 * stage (W is not written by anyone else inside the call), which saves one
 * primitive pass per step.  nsteps = 0 does nothing; WCNS_ERR_ARG for
 * nsteps < 0.  Asynchronous; no host sync. */
wcns_status wcns_ssprk3_steps(wcns_ctx* ctx, double* W, int32_t nsteps, double dt, double* dts);

/* Time loop of the paper's runs on the device: up to nsteps SSP-RK3 steps
 * (Sec. 5.3) of W in place, each of size dt > 0 or, dt <= 0, the CFL step
 * of Sec. 3.3 from the state at its start, the last one shortened to end
 * at t_end; the time is kept on the device.  t: device double, the time at
 * the start (in) and after the steps taken (out); steps_taken: device int64
 * (may be NULL), incremented by one per step taken; dts: device array of
 * >= nsteps doubles (may be NULL), the dt of each step slot (0 for a
 * skipped one).  Each step clips its dt to t_end - t when t + dt > t_end; a
 * step that would start at t >= t_end is skipped (its kernels return at
 * once), and so is every later step of the call; so is a step that would
 * not advance t (dt not positive from an infinite wave speed, a NaN, or too
 * small to change t), which leaves t short of t_end.  A caller therefore
 * enqueues chunks without reading t in between, and stops once a chunk
 * took fewer steps than it enqueued; the chunks can be captured in a HIP
 * graph.  The steps taken are the arithmetic of wcns_ssprk3_steps.
 * Asynchronous; no host sync.  WCNS_ERR_CFL for a non-finite dt or t_end. */
wcns_status wcns_ssprk3_advance(wcns_ctx* ctx, double* W, double dt, double t_end, int32_t nsteps,
                                double* t, int64_t* steps_taken, double* dts);

/* Lazy admissibility report (see the conventions above): synchronises the
 * context's stream and returns in *n_bad (host) the number of cells the
 * kernels found outside G since creation or the last clear; clear = 1 then
 * resets the count and lets later calls run again.  Returns
 * WCNS_ERR_INADMISSIBLE when *n_bad > 0, WCNS_OK otherwise. */
wcns_status wcns_violations(wcns_ctx* ctx, int64_t* n_bad, int32_t clear);

/* Count cells outside the admissible set G (Sec. 2): a1 < 0 or a1 > 1,
 * a_k r_k < 0, or rho e - pbar_inf <= 0 (NaN counts as outside).
 * Synchronises the stream; *n_bad is a host pointer. */
wcns_status wcns_check_admissible(wcns_ctx* ctx, const double* W, long long* n_bad);

/* Measurement aid (not needed for the method).  While enabled, every kernel
 * the context launches is timed by a pair of HIP events on the context's
 * stream that the launch itself stamps with the kernel's start and end
 * (hipExtLaunchKernelGGL), so the time excludes the dispatch; a skipped
 * step's kernels count with the time they took to return.
 * wcns_profile_read synchronises the stream and returns,
 * per kernel class, the summed device time in milliseconds and the number of
 * launches since the last reset.  Classes (WCNS_NPROF = 9): 0 node
 * primitives + wave-speed maxima, 1 dt/lambda finalize, 2 x-sweep,
 * 3 y-sweep, 4 tile fixups, 5 other, 6 z-sweep (3D), 7 one-pass stage of the
 * first-order scheme (2D) that reads no U^n (an RHS, the first RK stage),
 * 8 one that combines with U^n (RK stages 2 and 3).  `ms` and `launches`
 * hold WCNS_NPROF entries.  Enabling allocates the event pool (so it is not
 * graph-capturable); disabling releases it. */
#define WCNS_NPROF 9
wcns_status wcns_profile(wcns_ctx* ctx, int32_t enable);
wcns_status wcns_profile_read(wcns_ctx* ctx, double* ms, int64_t* launches, int32_t reset);

/* Verification aid: the kernels divide with the core of gfx950's
 * correctly rounded FP64 division sequence without its range-scaling steps
 * (valid for normal-range operands).  This computes, on the device, both
 * q_ieee[k] = a[k]/b[k] through the compiler's full IEEE sequence and
 * q_core[k] through the kernels' core, for device arrays of n doubles, so a
 * test can check they agree bit for bit over the operand ranges used. */
wcns_status wcns_selftest_division(const double* a, const double* b, double* q_ieee,
                                   double* q_core, int64_t n, void* stream);

/* Measurement aid: issue cost of one FP64 or FP32 operation on this GPU.  Runs
 * `iters` rounds of 8 independent chains of operation `op` per lane over a
 * grid that keeps 8 waves on every SIMD of the device (blocks of 256
 * threads; `blocks` <= 0 picks 32 per compute unit), synchronises, and
 * returns the kernel's device time in *ms (host).  op: 0 FMA, 1 add, 2 mul,
 * 3 IEEE divide (the compiler's sequence), 4 IEEE square root, 5 the
 * kernels' division core; FP32 (the precision form's bulk): 6 FMA, 7 the
 * kernels' quotient (hardware reciprocal and a product), 8 square root.  The ratio of two ops' times at equal iters is
 * their relative issue cost (the roofline of the sweeps weights divides and
 * square roots in FMA slots).  Allocates and frees its own 8-byte-per-thread
 * output; WCNS_ERR_ARG for an unknown op or iters < 1. */
wcns_status wcns_issue_probe(int32_t op, int32_t iters, int32_t blocks, double* ms, void* stream);

/* Verification aid: the kernels divide by a constant b (the HCS divisor
 * 2100 of Sec. 4.1, the grid spacings of the flux difference) through its
 * rounded reciprocal and one FMA correction when that reciprocal is accurate
 * to 2^-55; this runs that path for the n device values a[] and one b:
 * q_core[i], with the compiler's IEEE a[i]/b in q_ieee[i].  WCNS_ERR_ARG when
 * b does not take the path (the kernels then use the division core). */
wcns_status wcns_selftest_division_by(const double* a, double b, double* q_ieee, double* q_core,
                                      int64_t n, void* stream);

/* ------------------------------------------------------------------------
 * Batched form: many independent solves of uneven sizes advanced together.
 * Every phase of a Runge-Kutta stage is one launch over all instances (a
 * device list of (instance, tile) tasks); a whole step is a fixed sequence
 * of launches captured once into a HIP graph and replayed, on the batch's
 * own non-blocking stream.
 * ---------------------------------------------------------------------- */
typedef struct wcns_batch wcns_batch;

/* Create a batch of n solves that share ndim, fluids, options and
 * precision (no Dirichlet sides).  grids[b] is instance b's grid; W[b] its
 * device state [nvar][ny_b][nx_b] (caller-owned, stepped in place).
 * capacity_cells: scratch sized for at least this many cells in total (0:
 * exactly the given instances), so wcns_batch_reset can later rebind other
 * instance sets without allocating.  Errors as wcns_create, plus
 * WCNS_ERR_ARG for n < 1, mixed ndim or a Dirichlet side. */
wcns_status wcns_batch_create(int32_t n, const wcns_grid* grids, const wcns_eos* eos,
                              const wcns_params* params, int32_t precision, double* const* W,
                              int64_t capacity_cells, wcns_batch** out);

/* Rebind the batch to another instance set (same ndim) inside its existing
 * scratch; WCNS_ERR_NOMEM if it does not fit (the bound set stays as it
 * was).  Synchronises the batch stream; the captured graph is rebuilt on the
 * next step.  A reset or configure that fails after that check (a HIP error)
 * leaves no instance set bound: wcns_batch_step and wcns_batch_rhs then
 * return WCNS_ERR_ARG until a reset succeeds. */
wcns_status wcns_batch_reset(wcns_batch* b, int32_t n, const wcns_grid* grids, double* const* W);

/* Schedule: ytile in {2, 4, 8, 16} y-face rows per y-sweep block (32
 * columns, two face rows per wave; default 16); order 0 = instances in the given
 * order (default), 1 = largest instance first, 2 = tiles of an instance kept
 * on one XCD (blocks are dealt round-robin to the 8 XCDs).  Takes effect
 * at the next step (the graph is re-captured). */
wcns_status wcns_batch_configure(wcns_batch* b, int32_t ytile, int32_t order);

/* Enqueue nsteps SSP-RK3 steps of every instance, each with its own CFL
 * time step computed on the device (Sec. 3.3, 5.3).  Asynchronous. */
wcns_status wcns_batch_step(wcns_batch* b, int32_t nsteps);

/* Enqueue one RHS evaluation of every instance into scratch (the states are
 * not changed); used to time schedules.  Asynchronous. */
wcns_status wcns_batch_rhs(wcns_batch* b);

/* Wait for the batch stream; return its handle (hipStream_t) in *stream. */
wcns_status wcns_batch_sync(wcns_batch* b);
wcns_status wcns_batch_stream(wcns_batch* b, void** stream);

/* Per-instance step budgets for continuous batching: instance k takes only
 * steps[k] more steps (>= 0); once its counter reaches 0 every later step
 * skips it (its state stays as it is).  New instances start with an
 * unlimited budget.  wcns_batch_steps_left reads the counters back.  Both
 * synchronise the batch stream; host arrays of n int32. */
wcns_status wcns_batch_set_steps(wcns_batch* b, const int32_t* steps);
wcns_status wcns_batch_steps_left(wcns_batch* b, int32_t* steps);

/* Context-free primitive -> conservative conversion of ncell cells (Sec. 2
 * mixture EOS), V = (a1r1, a2r2, u, [v], p, a1) SoA -> W, device arrays,
 * enqueued on `stream` (hipStream_t or NULL). */
wcns_status wcns_prim_to_cons_n(const wcns_eos* eos, int32_t ndim, int64_t ncell, const double* V,
                                double* W, void* stream);

/* Per-instance admissibility report of the batched form: synchronises the
 * batch stream and writes counts[k] (host int64[n]), the number of cells of
 * instance k found outside G (its input at the first stage of a step call,
 * every stage result) since the instance was bound or the last clear;
 * clear = 1 resets the counts.  Batched calls never refuse work: a server
 * reads these after each tick and retires the instances that failed. */
wcns_status wcns_batch_violations(wcns_batch* b, int64_t* counts, int32_t clear);

/* Host copy of every instance's last time step, dt[n] (synchronises). */
wcns_status wcns_batch_dt(wcns_batch* b, double* dt);

wcns_status wcns_batch_destroy(wcns_batch* b);

/* ------------------------------------------------------------------------
 * Allocation-free right-hand side, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  The arithmetic and kernels of wcns_rhs (same results,
 * bit for bit) without a context: grid, fluids, options and precision are
 * validated as by wcns_create and the scratch (node primitives, y-tile edge
 * fluxes, block maxima, step record) lives in a static device array of
 * WCNS_NOALLOC_SCRATCH_BYTES per GPU, held from the library's load until the
 * process ends.  It needs 8 (5 N + 12 nx ceil((ny+1)/16)) bytes for
 * N = nx*ny cells (1D: 8 * 5 N) plus at most 33 KiB (block maxima, step
 * record) and, for the first-order scheme, a 64 KiB sink: up to ~1.45 M
 * cells in 2D (1024^2 fits); larger grids return WCNS_ERR_TOO_LARGE.  1D and 2D grids without
 * Dirichlet sides (WCNS_ERR_ARG otherwise).  W, dWdt: device [nvar][ny][nx],
 * caller-owned, must not alias; dt as in wcns_rhs.  Calls no allocating
 * routine: the first call on a device looks up the array's address once.
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents (every value a call reads is written by that call first), so
 * calls that overlap on one GPU (other streams, other threads) race.
 * Asynchronous on `stream` (hipStream_t or NULL).  No admissibility report
 * (there is no context to hold one).
 * ---------------------------------------------------------------------- */
#define WCNS_NOALLOC_SCRATCH_BYTES (64u << 20)
wcns_status wcns_rhs_noalloc(const wcns_grid* grid, const wcns_eos* eos, const wcns_params* params,
                             int32_t precision, void* stream, const double* W, double* dWdt,
                             double dt);

/* Human-readable status. */
const char* wcns_status_str(wcns_status s);

#ifdef __cplusplus
}
#endif
#endif /* WCNS_H_ */
