/*
 * claw.h -- C ABI of libclaw, a finite-volume step library for MI355X (gfx950).
 *
 * What it computes (Ketcheson et al., "PyClaw: Accessible, Extensible,
 * Scalable Tools for Wave Propagation Problems"):
 *
 *   one time step for  q_t + f(q)_x + g(q)_y = 0  on a uniform Cartesian grid
 *   (Section 2, eq. conslaw with capacity 1 and no source), in two forms:
 *
 *   CLAW_CLASSIC   -- the Clawpack wave-propagation step: a Riemann solve at
 *                     every interface, waves limited by their upwind
 *                     neighbour, a second-order correction flux
 *                     (Section 2, eq. lwflux: F = F_upwind + F_correction,
 *                     first-order part as fluctuations), and in 2D the
 *                     unsplit transverse corrections from a secondary
 *                     Riemann solver (Section 2.1);
 *   CLAW_SHARPCLAW -- the SharpClaw method of lines: WENO edge values (any
 *                     odd order from 5 to 17), an interface Riemann flux, flux
 *                     differencing (Section 2, eq. fluxdiff), inside the
 *                     stages of an SSP Runge-Kutta method: SSPRK(3,3), or
 *                     the ten-stage fourth-order SSP method (Ketcheson 2008,
 *                     two-register form) that SharpClaw uses by default
 *                     (Section 2.1: WENO in space and SSP RK in time, with
 *                     normal Riemann problems only in 2D; higher WENO
 *                     orders from generated coefficients).
 *
 * Ghost cells carry the boundary conditions (Section 4, "Parallelization");
 * after each step the Courant number is checked and the next step size is
 * chosen (Section 4, the single reduction of the maximum wave speed).
 *
 * Conventions
 * -----------
 *  * Every function returns an int status: CLAW_OK (0) or a negative
 *    CLAW_E_* code; claw_strerror() names it.  Nothing throws across the ABI.
 *  * Arrays are component-major, x fastest: q[k][j][i], k = component
 *    (0..m-1), j = row (0..ny-1), i = column (0..nx-1); ny = 1 in 1D.
 *    State arrays passed in or out are always float64, whatever the
 *    precision the library computes in.
 *  * The caller owns all device memory.  claw_create() receives one device
 *    buffer of at least claw_workspace_bytes() bytes and carves every array
 *    from it; the library never allocates or frees device memory.  The
 *    buffer must stay valid until claw_destroy().  claw_destroy() frees only
 *    host-side objects (the handle, pinned staging, captured graphs).
 *  * Work is enqueued on the handle's HIP stream.  A NULL stream at
 *    claw_create makes the library create a private blocking stream (it
 *    orders with the legacy default stream); graph capture needs a real
 *    stream.  claw_set_state, claw_get_state, claw_totals, claw_step and
 *    the claw_advance calls synchronise the handle's stream before they
 *    return.
 *  * One handle must not be used from two threads at once.  Different
 *    handles are independent.
 *  * Device-side failures (a non-finite Courant number) are reported by the
 *    next call that synchronises.
 */
#ifndef CLAW_H
#define CLAW_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum claw_status {
  CLAW_OK = 0,
  CLAW_E_INVAL = -1,       /* bad argument or unsupported combination */
  CLAW_E_NOMEM = -2,       /* workspace smaller than claw_workspace_bytes() */
  CLAW_E_DEVICE = -3,      /* a HIP runtime call failed */
  CLAW_E_REJECTED = -4,    /* claw_step: Courant number > cfl_max; state unchanged */
  CLAW_E_NONPHYSICAL = -5, /* non-finite Courant number (NaN/Inf in the state) */
  CLAW_E_BUDGET = -6,      /* batch: no free slot */
  CLAW_E_STATE = -7,       /* call order (e.g. stepping before claw_set_state) */
  CLAW_E_MAXSTEPS = -8,    /* claw_advance: max_steps attempts did not reach t_end */
  CLAW_E_TOOBIG = -9       /* claw_step_static: the grid needs more than CLAW_STATIC_SCRATCH_BYTES */
};

enum claw_scheme { CLAW_CLASSIC = 1, CLAW_SHARPCLAW = 2 };
enum claw_riemann {
  CLAW_RP_ADVECTION = 1,  /* q_t + u q_x + v q_y = 0, problem_data = (u, v); m = 1 */
  CLAW_RP_SW_ROE = 2,     /* shallow water, Roe solver (+ Harten-Hyman entropy fix),
                             problem_data = (g); m = 2 (1D) or 3 (2D); classic only */
  CLAW_RP_EULER_HLLE = 3, /* Euler, HLLE flux, problem_data = (gamma); m = 3 (1D) or 4 (2D);
                             SharpClaw only */
  CLAW_RP_ELASTIC_VC = 4, /* 2D linear elasticity, variable coefficients, m = 5,
                             q = (s11, s22, s12, u, v), aux = (rho, lambda, mu); classic, 2D only */
  CLAW_RP_EULER_ROE = 5,  /* Euler, Roe solver (two acoustic, entropy and - in 2D - shear waves)
                             with its transverse solver, problem_data = (gamma); m = 3 (1D) or
                             4 (2D), plus one with a tracer; optional Harten-Hyman entropy fix;
                             classic only */
  CLAW_RP_PSYSTEM = 6     /* nonlinear p-system in a varying medium (Section 7.3, eq. p-system):
                             q = (strain, rho u[, rho v]), m = 2 (1D) or 3 (2D); aux = (K, rho)
                             per cell; stress exp(K strain) - 1; f-wave interface flux (each side
                             in its own material); SharpClaw only */
};
enum claw_source {
  CLAW_SOURCE_NONE = 0,
  CLAW_SOURCE_AXISYMMETRIC = 1  /* CLAW_RP_EULER_ROE in 2D: cylindrical symmetry about y = 0
                                   (x = axial coordinate z, y = radius r > 0), geometric source
                                   -(v/r)(rho, rho u, rho v, E + p) applied after each hyperbolic
                                   step by one step of Heun's method (fractional step) */
};
enum claw_limiter { CLAW_LIM_NONE = 0, CLAW_LIM_MINMOD = 1, CLAW_LIM_MC = 2 };
enum claw_bc { CLAW_BC_EXTRAP = 1, CLAW_BC_PERIODIC = 2, CLAW_BC_WALL = 3, CLAW_BC_DIRICHLET = 4 };
enum claw_integrator {
  CLAW_SSP33 = 1,   /* Shu-Osher SSPRK(3,3): 3 stages (launches), two stage arrays */
  CLAW_SSP104 = 2   /* SSPRK(10,4): 10 stages, SSP coefficient 6, three stage arrays */
};
enum claw_split {
  CLAW_SPLIT_NONE = 0,     /* unsplit 2D step (transverse corrections per `transverse`) */
  CLAW_SPLIT_GODUNOV = 1,  /* classic 2D, dimensionally split (Section 2.1): a 1D wave-propagation
                              sweep along x over dt on every row, then one along y over dt on
                              every column; `transverse` is not used */
  CLAW_SPLIT_STRANG = 2    /* as GODUNOV, but x over dt/2, y over dt, x over dt/2 */
};
enum claw_precision {
  CLAW_FP64 = 1,       /* all arithmetic in float64 */
  CLAW_FP32_KAHAN = 2, /* reconstruction, Riemann and limiter arithmetic in float32; the state is
                          float32 with a float32 compensation term per value (Kahan summation of
                          each update); dt control, Courant reduction and totals in float64 */
  CLAW_FP32 = 3        /* as CLAW_FP32_KAHAN without the compensation (plain float32 updates), to
                          measure what the compensated update gains; classic 2D shallow water
                          (unsplit) and SharpClaw 2D Euler with WENO5 only (else CLAW_E_INVAL) */
};

typedef struct claw_config {
  int ndim;              /* 1 or 2 */
  int num_cells[2];      /* nx, ny (ny ignored in 1D); each >= 4 */
  double lower[2];       /* domain lower corner */
  double upper[2];       /* domain upper corner */
  int scheme;            /* claw_scheme */
  int riemann;           /* claw_riemann */
  int limiter;           /* claw_limiter (classic) */
  int transverse;        /* classic 2D: 0 none, 1 transverse split of the fluctuations,
                            2 "full": fluctuations -/+ the second-order correction term */
  int entropy_fix;       /* shallow water: 1 = Harten-Hyman entropy fix */
  int bc_lower[2];       /* claw_bc at x-lower, y-lower */
  int bc_upper[2];       /* claw_bc at x-upper, y-upper */
  double bc_state[4][8]; /* Dirichlet states: [0] x-lower, [1] x-upper, [2] y-lower, [3] y-upper */
  double cfl_desired;    /* controller target Courant number */
  double cfl_max;        /* steps with a larger Courant number are rejected */
  double dt_initial;     /* first dt; <= 0: cfl_desired / max cell characteristic speed */
  double dt_max;         /* <= 0: unbounded */
  double weno_eps;       /* SharpClaw WENO epsilon (1e-6 if <= 0) */
  int precision;         /* claw_precision */
  double problem_data[8];
  int time_integrator;   /* SharpClaw: claw_integrator (0 = CLAW_SSP33); ignored by classic */
  int weno_order;        /* SharpClaw: odd order 5..17 of the WENO edge values (0 = 5; Section 3.3:
                            generated reconstructions from fifth to seventeenth order); needs
                            (order + 1) / 2 <= num_cells in each dimension.  Ignored by classic.
                            Any other value: CLAW_E_INVAL */
  int tracer;            /* CLAW_RP_EULER_ROE: 1 adds a passive tracer as the last component,
                            advected by the flow (q_t + u phi_x + v phi_y = 0); else 0 */
  int source;            /* claw_source (0 = none) */
  int dimensional_split; /* classic 2D: claw_split (0 = unsplit).  The Courant number of a split
                            step is dt times the largest |speed| / spacing met in any sweep.  Not
                            allowed in 1D, with SharpClaw, or for a batch member (CLAW_E_INVAL) */
} claw_config;

/* Clock and counters of a handle; also the checkpoint record of the
 * controller (state arrays are checkpointed with claw_get_state). */
typedef struct claw_stats {
  long long accepted;    /* accepted steps since the clock was last set */
  long long rejected;    /* rejected attempts */
  double t;              /* simulation time */
  double dt_next;        /* the controller's next dt (0: not yet chosen) */
  double max_courant;    /* largest accepted Courant number */
  double gpu_ms;         /* GPU time of the last claw_advance / claw_advance_graph call, from HIP
                            events recorded on the handle's stream around its launches */
} claw_stats;

/* Kernel tiling.  Results do not depend on it (bit for bit). */
typedef struct claw_tuning {
  int seg_rows;          /* rows per work item of the 2D kernels (>= 1); of the y sweeps of a
                            dimensionally split step.  The rows are split into
                            ceil(ny / seg_rows) segments as evenly as possible */
  int seg_rows_x;        /* rows per work item of the x sweeps of a dimensionally split step
                            (rows are independent there); <= 0: seg_rows.  Ignored otherwise */
  int segs;              /* row segments (work items per column strip) of the 2D kernels;
                            > 0 overrides seg_rows (at most ny).  claw_get_tuning fills both,
                            seg_rows being the longest segment */
  int order;             /* order of the tiles over the workgroups of a launch: 0 strips
                            fastest, 1 segments fastest, 2 and 3 the same with each of the
                            GPU's 8 XCDs (own L2) given a contiguous band of tiles */
} claw_tuning;

typedef struct claw_solver* claw_t;
typedef struct claw_batch* claw_batch_t;

/* Human-readable name of a status code (static storage). */
const char* claw_strerror(int status);

/* Number of equations m and of aux fields for a configuration (0 if invalid). */
int claw_num_eqn(const claw_config* cfg);
int claw_num_aux(const claw_config* cfg);

/* Exact device bytes claw_create needs for cfg (0 if cfg is invalid). */
size_t claw_workspace_bytes(const claw_config* cfg);

/* Validate cfg and build a handle (the solver and solution objects of the
 * paper's interface, Section 3) over the caller's device buffer d_ws
 * (>= claw_workspace_bytes(cfg) bytes, 256-byte aligned, on the current
 * device).  hip_stream: a hipStream_t or NULL.  *out receives the handle. */
int claw_create(const claw_config* cfg, void* d_ws, size_t ws_bytes, void* hip_stream,
                claw_t* out);

/* Copy the state in (a solution's q, Section 3; component first as there).
 * q: float64[m][ny][nx], host (on_device = 0) or device
 * memory.  Resets the compensation terms (FP32 mode).  Does not touch the clock. */
int claw_set_state(claw_t h, const double* q, int on_device);

/* Copy the aux fields in (Section 3: spatially varying coefficients; elasticity: rho, lambda,
 * mu; p-system: K, rho, Section 7.3), float64[na][ny][nx]. */
int claw_set_aux(claw_t h, const double* aux, int on_device);

/* Copy the state out as float64[m][ny][nx] (FP32 mode: value minus
 * compensation, formed in float64). */
int claw_get_state(claw_t h, double* q_out, int on_device);

/* One step of exactly dt (the method of Section 2, eq. fluxdiff, in the
 * configured form of Section 2.1; no controller, no retry).  *courant_out (may be
 * NULL) receives dt * max|wave speed|/spacing over the faces bounding
 * interior cells (SharpClaw: in the first stage).  The step is always
 * applied and the clock advances by dt. */
int claw_step(claw_t h, double dt, double* courant_out);

/* Advance to t_end with the step controller (Section 4: the Courant number
 * is checked after every step and the next step size chosen) on the host (one 8-byte
 * device-to-host read per attempt):
 *   dt_try = min(dt, t_end - t); step; C = dt_try * speed;
 *   C <= cfl_max: accept (t = t_end exactly on the clipped step);
 *   otherwise the state is kept and the attempt counted as rejected;
 *   dt = min(dt_max, dt_try * cfl_desired / C)  (dt_max if C = 0).
 * max_steps bounds the attempts (<= 0: no bound).  st (may be NULL)
 * receives the clock and counters. */
int claw_advance(claw_t h, double t_end, long long max_steps, claw_stats* st);

/* The same controller run on the device: every attempt is one kernel
 * launch (three for SharpClaw) whose last workgroup takes the
 * accept/reject decision and picks the next dt; attempts are replayed from
 * a captured HIP graph of steps_per_graph attempts, and attempts after
 * t_end are skipped on the device.  The host synchronises once per
 * graph launch group.  Same arithmetic and results as claw_advance. */
int claw_advance_graph(claw_t h, double t_end, int steps_per_graph, long long max_steps,
                       claw_stats* st);

/* Conserved totals (Section 2, eq. conslaw: the quantities the finite-volume
 * form conserves): totals[k] = sum over cells of q_k * dx * dy, float64
 * (FP32 mode: of value minus compensation). */
int claw_totals(claw_t h, double* totals);

/* Read / restore the clock (checkpointing; not a passage of the paper). */
int claw_get_clock(claw_t h, claw_stats* st);
int claw_set_clock(claw_t h, const claw_stats* st);

/* Tiling of the 2D kernels (an implementation parameter, not in the paper);
 * results are bitwise independent of it. */
int claw_set_tuning(claw_t h, const claw_tuning* tn);
int claw_get_tuning(claw_t h, claw_tuning* tn);

/* Time one step (without applying it) for each candidate tiling and keep
 * the fastest; *out (may be NULL) receives it.  reps: timed repetitions.
 * Candidates: row segment counts (rows per segment 4..128 and counts that
 * fill whole waves per SIMD), then the four tile orders at the best count;
 * split steps tune the y sweeps' segments first, then seg_rows_x. */
int claw_autotune(claw_t h, int reps, claw_tuning* out);

/* Launch the step's main kernel `reps` times back to back on the handle's
 * stream, without applying the step (classic: the one step kernel writing
 * the spare buffer; SharpClaw: stages 1 and 2, which write only the stage
 * buffers), between two HIP events.  *avg_ms receives the average duration
 * of one launch (SharpClaw: of one stage).  Used to measure the kernels
 * against the HBM roofline.  The state is unchanged. */
int claw_time_kernel(claw_t h, double dt, int reps, double* avg_ms);

/* Release the handle (host objects only). */
int claw_destroy(claw_t h);

/* ---------------------------------------------------------------------------
 * Batching (for serving many small problems; not in the paper, whose
 * controller of Section 4 each member runs): one launch advances every member grid by one attempt, each with
 * its own clock, dt controller and t_end.  Members must be classic 2D
 * handles with the same riemann solver, limiter, transverse mode and
 * precision, created on the same
 * device; each keeps its own workspace.  The batch itself needs
 * claw_batch_workspace_bytes(max_grids) device bytes from the caller.
 * ------------------------------------------------------------------------- */
size_t claw_batch_workspace_bytes(int max_grids);
int claw_batch_create(int max_grids, void* d_ws, size_t ws_bytes, void* hip_stream,
                      claw_batch_t* out);
/* Add a handle (its state must be set) with its own end time; it joins the
 * next launched group.  Synchronises only the member's own stream. */
int claw_batch_add(claw_batch_t b, claw_t h, double t_end);
/* Remove a member.  One that had stopped as of the view leaves without any
 * wait (its clock is the view's; groups still in flight skip it, but may
 * still read its controller: keep its workspace valid until the next
 * claw_batch_wait returns).  Otherwise the batch stream is synchronised. */
int claw_batch_remove(claw_batch_t b, claw_t h);
/* Run `attempts` device-controlled attempts for every member (members
 * that reached t_end idle); *n_active (may be NULL) receives the number of
 * members still short of their t_end.  Waits for every group in flight
 * (= claw_batch_launch + claw_batch_wait). */
int claw_batch_advance(claw_batch_t b, int attempts, int* n_active);
/* Enqueue a group of `attempts` device-controlled attempts for every current
 * member, then an asynchronous copy of the member controllers to pinned host
 * memory; returns without synchronising.  Membership changes made before the
 * call take effect in this group.  At most two groups may be in flight
 * (CLAW_E_STATE otherwise): launching the next group before waiting for the
 * previous one keeps the GPU busy while the host admits and retires. */
int claw_batch_launch(claw_batch_t b, int attempts);
/* Wait for the oldest group in flight (CLAW_E_STATE if none) and make its
 * controller copies the batch's view: claw_batch_finished and
 * claw_batch_remove read it.  *n_active (may be NULL): members of that group
 * still short of their t_end. */
int claw_batch_wait(claw_batch_t b, int* n_active);
/* Members whose controller has stopped (reached t_end or failed) as of the
 * view: up to `cap` handles into out[], count in *n_out.  They stay members
 * until claw_batch_remove. */
int claw_batch_finished(claw_batch_t b, claw_t* out, int cap, int* n_out);
/* Clock of one member (synchronised). */
int claw_batch_member_clock(claw_batch_t b, claw_t h, claw_stats* st);
int claw_batch_destroy(claw_batch_t b);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one step
 * of exactly dt, as claw_step computes it, from a float64 state in device
 * memory to a float64 state in device memory, with no handle and no caller
 * workspace.  Every intermediate -- grid descriptor, controller record,
 * Courant-reduction slots and, as the configuration needs them, the float32
 * state with its compensation, the Runge-Kutta stage buffers, the split
 * step's intermediate states and float32 aux -- lives in one fixed array of
 * CLAW_STATIC_SCRATCH_BYTES inside the library, one copy per device, held
 * from the library's first use on that device until the process ends.  In
 * FP64 the classic step reads d_q_in and writes d_q_out directly.
 *
 *   cfg        configuration as for claw_create (validated the same way)
 *   d_q_in     float64[m][ny][nx] on the current device, read only
 *   d_aux      float64[na][ny][nx] on the current device (NULL if na = 0)
 *   d_q_out    float64[m][ny][nx] on the current device; must not overlap d_q_in
 *   dt         the step size (> 0); the step is always taken
 *   d_courant  one float64 on the current device: receives dt * max|speed| /
 *              spacing over the faces bounding interior cells (SharpClaw: in
 *              the first stage); non-finite for a non-physical state
 *   hip_stream hipStream_t (NULL: the legacy default stream)
 *
 * The call only enqueues work on hip_stream (a fill kernel, the step's
 * kernels, conversions, one device-to-device copy for SharpClaw in FP64): it
 * does not synchronise, allocate or free, and issues no memset or
 * host-to-device copy, so a captured sequence of calls replays as it is.
 * The first call on a device looks up that device's array (do it once
 * outside capture).  All calls on one device share the array: calls that
 * overlap in time on one device (two streams, two threads) race and give
 * wrong results; calls in one stream order are safe.  Each call resets the
 * controller record and reduction slots it uses.
 *
 * Returns CLAW_OK, CLAW_E_INVAL (bad configuration or arguments, missing
 * aux, overlapping buffers), CLAW_E_TOOBIG (claw_static_bytes(cfg) exceeds
 * CLAW_STATIC_SCRATCH_BYTES) or CLAW_E_DEVICE (a launch failed).
 * ------------------------------------------------------------------------- */
#define CLAW_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
/* Bytes of the static array claw_step_static would use for cfg (0 if invalid). */
size_t claw_static_bytes(const claw_config* cfg);
int claw_step_static(const claw_config* cfg, const double* d_q_in, const double* d_aux,
                     double* d_q_out, double dt, double* d_courant, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* CLAW_H */
