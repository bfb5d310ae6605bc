/*
 * hsgn.h -- C ABI of the MI355X (gfx950) library for the semi-implicit IMEX
 * time step of the hyperbolic Serre-Green-Naghdi (hSGN) equations
 * (Macca, Boscheri, Ricchiuto, arXiv 2510.07539).
 *
 * What one step computes (Sec. 3.2, eq. tableau and the efficient form of
 * the remark after it): the two-stage partitioned IMEX Runge-Kutta step
 *   U^(1)   = Stage(U_old = U^n,  U_E = U^n,     tau = gamma dt)
 *   U^{n+1} = Stage(U_old = U~,   U_E = U_E^(2), tau = gamma dt)
 * with gamma = 1 - 1/sqrt(2), U_E^(2) = (1 - c/gamma) U^n + (c/gamma) U^(1),
 * U~ = (1 - (1-gamma)/gamma) U^n + ((1-gamma)/gamma) U^(1), c = 1/(2 gamma).
 * Each Stage is the fully discrete first-order semi-implicit step of
 * Sec. 4.2 (eq. GN_hyp_eq_semi_fully_discrete): explicit Rusanov fluxes of
 * the convective terms on an unlimited linear reconstruction (Sec. 4.1),
 * the exact elimination of the relaxation pair (Sec. 3.1, eq. b1), a
 * tridiagonal (cyclic when periodic) system for the new depth from the
 * linearised pressure (Sec. 3.1, eq. hnew; differenced in conservative
 * pressure form), and back-substitution of momentum, h*eta and h*w.
 * With order = 1 a step is that Stage alone, with tau = dt and no
 * reconstruction (first order in time and space).
 * The time step is CFL dx / max(|u| + sqrt(g h)), capped by the material
 * CFL max|u| dt/dx <= mcfl (Sec. 3.3 eq. MCFL and Sec. 5).
 * With scheme = HSGN_SCHEME_EXPLICIT a step is instead the fully explicit
 * hSGN scheme of Sec. 4.1 (eq. GN_hyp_eq_explicit) with Heun's method,
 *   U1 = U^n + dt L(U^n),  U^{n+1} = (U^n + U1 + dt L(U1)) / 2,
 * L = Rusanov fluxes (speed max(|u| + c) over the face states) on the same
 * reconstruction for h, q u, m u, W u; central differences for the pressure
 * terms a^2 h_x + lambda alpha (h eta)_x; sources h w and
 * -lambda (eta/h - 1).  Its dt is CFL dx / max(|u| + c) (eq. CFL_ex).
 * With scheme = HSGN_SCHEME_SGN a step is the explicit scheme of Sec. 4.4
 * for the standard SGN equations (eq. SGN_standard) with Heun's method:
 * per stage, phi from the tridiagonal (cyclic when periodic) system
 *   h_i phi_i - (H_{i+1/2}(phi_{i+1} - phi_i) - H_{i-1/2}(phi_i - phi_{i-1}))
 *     / (3 dx^2) = -(G_{i+1} - G_{i-1}) / (6 dx^3),
 * H = face mean of h^3, G_j = g h_j^3 (h_{j+1} - 2 h_j + h_{j-1})
 * + (h_j^3 / 2)(u_{j+1} - u_{j-1})^2, then shallow-water Rusanov fluxes
 * with the source h phi.  Its dt follows the semi-implicit rule.
 *
 * State per cell (all FP64, structure of arrays): h (depth), q = h u,
 * m = h eta, W = h w.  Independent instances ("batch") are concatenated:
 * instance j owns cells [offsets[j], offsets[j+1]).  Bed b (bathymetry) is
 * optional per instance.
 *
 * Memory: every pointer named d_* is a device pointer owned by the caller;
 * the library copies from it or into it and never keeps it.  The library
 * owns its own state buffers and workspace, allocated in hsgn_init and freed
 * in hsgn_destroy.  Pointers named h_* are host pointers.
 *
 * Streams: every call is enqueued asynchronously on the HIP stream given to
 * hsgn_init, except hsgn_status, which synchronises that stream.
 *
 * Errors: every int-returning call returns HSGN_OK (0) or a negative code;
 * hsgn_last_error names the failing call.  A context is not thread-safe.
 */
#ifndef HSGN_H
#define HSGN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HSGN_OK 0
#define HSGN_EINVAL (-1)        /* bad argument (sizes, parameters, null)    */
#define HSGN_EHIP (-2)          /* a HIP runtime call failed                 */
#define HSGN_ENONPHYS (-3)      /* some instance produced h <= 0 or NaN      */
#define HSGN_ENONCOERCIVE (-4)  /* some instance produced beta <= 0          */
#define HSGN_ENOMEM (-5)        /* device allocation failed                  */
#define HSGN_EWINDOW (-6)       /* windowed solve could not certify its truncation */

/* Per-instance status bits returned by hsgn_status. A flagged instance is
 * frozen: its later steps use dt = 0 and leave its state unchanged. */
#define HSGN_FLAG_NONPHYS 1     /* h <= 0, or a non-finite value, in a stage */
#define HSGN_FLAG_NONCOERCIVE 2 /* beta <= 0 (coercivity, Sec. 3.1 prop.)  */
#define HSGN_FLAG_WINDOW 4      /* windowed solve: truncation bound > 2^-56  */

typedef enum { HSGN_BC_PERIODIC = 0, HSGN_BC_TRANSMISSIVE = 1 } hsgn_bc;

/* Parameters of one instance, as the paper states the problem. */
typedef struct {
  double g;              /* gravity (9.81)                                  */
  double lambda;         /* relaxation parameter lambda > 0 (eq. hSGN_eq)   */
  double dx;             /* uniform cell width > 0                          */
  double cfl;            /* CFL on max(|u| + sqrt(g h)) (e.g. 0.9)          */
  double mcfl;           /* material CFL cap (0.5; <= 0 disables the cap)   */
  double dt_fixed;       /* > 0: fixed time step; <= 0: adaptive            */
  double t_end;          /* > 0: clamp the last step to t_end, then freeze  */
  int32_t bc;            /* hsgn_bc                                         */
  int32_t has_bathymetry;/* 1: use the bed b of this instance; 0: flat      */
  int32_t order;         /* 2 (or 0): the two-stage IMEX step; 1: the
                            first-order scheme of Sec. 4.2 as printed: one
                            stage with tau = dt and no reconstruction (face
                            values = cell values).  Same for every instance. */
  int32_t scheme;        /* HSGN_SCHEME_SEMI_IMPLICIT (0): the steps above;
                            HSGN_SCHEME_EXPLICIT (1): the fully explicit
                            hSGN scheme of Sec. 4.1 with Heun's method, flat
                            bottom only (has_bathymetry = 0), order 0 or 2;
                            cfl then applies to |u| + c with the hSGN
                            celerity c^2 = g h + (lambda/3)(eta/h)^2
                            (eq. hSGN_c).  HSGN_SCHEME_SGN (2): the
                            standard SGN equations in elliptic-hyperbolic
                            form (Sec. 4.3-4.4) with Heun's method, flat
                            bottom, order 0 or 2, lambda unused, m and W
                            carried unchanged.  Same for every instance.   */
} hsgn_params;

#define HSGN_SCHEME_SEMI_IMPLICIT 0
#define HSGN_SCHEME_EXPLICIT 1
#define HSGN_SCHEME_SGN 2

typedef struct hsgn_ctx hsgn_ctx;

/* Create a context for n_inst instances.
 *  offsets: host, n_inst+1 int64, offsets[0] = 0, each instance >= 4 cells.
 *  params:  host, n_inst entries (copied).
 *  d_b:     device, offsets[n_inst] doubles, or NULL if no instance uses a
 *           bed (copied; instances with has_bathymetry = 0 ignore it: their
 *           bed is 0, also for hsgn_adjoint's initial-state map).
 *  hip_stream: a hipStream_t (NULL = default stream).
 * Allocates the library's state buffers and workspace on the current device.
 * The state is zero until hsgn_set_state.  Returns HSGN_EINVAL, HSGN_ENOMEM
 * or HSGN_EHIP on failure (then *ctx is NULL). */
int hsgn_init(hsgn_ctx** ctx, int32_t n_inst, const int64_t* offsets,
              const hsgn_params* params, const double* d_b, void* hip_stream);

/* Load the state (device arrays of offsets[n_inst] doubles).
 *  d_m: NULL means m = h*h (eta = h, the initial data of Sec. 6.3).
 *  d_W: NULL means W = -h^2 u_x (w = -h u_x, the same initial data), with
 *       the central difference u_x,i = (u_{i+1} - u_{i-1}) / (2 dx) of
 *       u = q/h: periodic instances wrap, transmissive ones take the
 *       boundary cell's own u beyond each end.
 *  d_t: device, n_inst times, or NULL for t = 0.
 * Clears the status flags and step counts, computes the first step's speed
 * bound and plans the solver (synchronises the stream).  Graphs captured by
 * hsgn_run are kept when the new plan has the same launch configuration. */
int hsgn_set_state(hsgn_ctx* ctx, const double* d_h, const double* d_q,
                   const double* d_m, const double* d_W, const double* d_t);

/* Copy the current state out (any pointer may be NULL to skip it).
 * d_t: device, n_inst doubles (time reached per instance). */
int hsgn_get_state(hsgn_ctx* ctx, double* d_h, double* d_q, double* d_m,
                   double* d_W, double* d_t);

/* Copy the last step's dt of every instance (device, n_inst doubles). */
int hsgn_get_dt(hsgn_ctx* ctx, double* d_dt);

/* Advance every instance by nsteps IMEX steps with eager kernel launches. */
int hsgn_step(hsgn_ctx* ctx, int32_t nsteps);

/* Advance by nsteps IMEX steps, replaying a captured HIP graph of `block`
 * steps (block >= 1; odd blocks are rounded up to even); remaining steps run
 * eagerly.  Same results as hsgn_step. */
int hsgn_run(hsgn_ctx* ctx, int32_t nsteps, int32_t block);

/* How the tridiagonal system of each stage is solved.
 *  HSGN_SOLVER_AUTO: an instance that fits one 4096-row window is solved in
 *    one pass, exactly.  A longer instance is cut into windows that solve
 *    their core plus a halo of L rows per side (L from the decay of the
 *    inverse of the depth system at the rest-state coefficients of the
 *    loaded state's deepest cell and speed bound, margin 2); each window
 *    bounds the effect of the truncation on its core and flags the
 *    instance (HSGN_FLAG_WINDOW) if it exceeds 2^-56 of the depth, as it
 *    does for a start far from the relaxation equilibrium (eta far from h),
 *    whose rows couple more strongly than that estimate: such an instance
 *    needs HSGN_SOLVER_EXACT.  When L would exceed a quarter window the
 *    instance uses the exact solver.
 *    Conservation: the sums of h and q telescope only where neighbouring
 *    cells use one new depth.  At a seam between two windows each takes its
 *    neighbour's depth from its own halo row, which differs from the other
 *    window's core value by at most the certified truncation (2^-56 of the
 *    depth at the core edge, 1/rho times that one row further out, rho the
 *    decay per row).  So in windowed mode the momentum sum of a periodic,
 *    flat instance moves per stage and seam by at most
 *    (tau/dx) beta_max h_max 2^-56 (1 + 1/rho), beyond rounding; the exact
 *    solver conserves it to rounding.
 *  HSGN_SOLVER_EXACT: two passes per stage for every instance longer than
 *    2048 cells: tiles reduce to two rows each, a per-instance reduced
 *    system is solved, and the tiles finish (no truncation anywhere).
 *  HSGN_SOLVER_AUTO_SMALL: AUTO with 2048-row windows (256 threads x 8 rows).
 * The plan is made from the state loaded by hsgn_set_state (speed bound
 * and maximum depth per instance); hsgn_set_solver re-plans at once.
 * With scheme = HSGN_SCHEME_SGN the modes plan the phi solve: AUTO and
 * AUTO_SMALL take 4096-row windows (halo from the phi rows' decay at the
 * deepest cell), truncated at their edges with phi = 0 beyond them and
 * certified to 2^-56 of max |phi| (the rows are diagonally dominant by h,
 * so max |phi| <= max |rhs| / min h bounds the replaced values; otherwise
 * HSGN_FLAG_WINDOW); EXACT solves every instance on the two-pass tiling. */
#define HSGN_SOLVER_AUTO 0
#define HSGN_SOLVER_EXACT 1
#define HSGN_SOLVER_AUTO_SMALL 2
int hsgn_set_solver(hsgn_ctx* ctx, int32_t mode);

/* Autotuner: time each solver mode (HSGN_SOLVER_AUTO, HSGN_SOLVER_EXACT,
 * HSGN_SOLVER_AUTO_SMALL) for nsteps eager steps on the loaded state, keep
 * the fastest, and leave the state (with time, status and speed bounds)
 * as it was.  h_ms (host, 3 doubles or NULL): milliseconds per step of each
 * mode, indexed by the mode's value; h_mode (host or NULL): the mode kept.
 * The modes agree with each other to rounding.  Allocates a copy of the
 * state for its duration; synchronises the stream.  Semi-implicit scheme
 * only (else HSGN_EINVAL; the SGN scheme's two forms of the phi solve are
 * chosen with hsgn_set_solver). */
int hsgn_autotune(hsgn_ctx* ctx, int32_t nsteps, double* h_ms, int32_t* h_mode);

/* Per-instance solver modes: h_modes (host, n_inst values of
 * HSGN_SOLVER_AUTO, HSGN_SOLVER_EXACT or HSGN_SOLVER_AUTO_SMALL) choose, for
 * each instance, 4096-row windows, the exact two-pass solve or 2048-row
 * windows (with the same fall-back to the exact solve as the uniform
 * modes).  Instances of each window width go to one launch per stage of the
 * kernel of that width.  Re-plans at once; hsgn_set_solver and hsgn_autotune
 * return to one mode for every instance.  Semi-implicit scheme only. */
int hsgn_set_instance_solvers(hsgn_ctx* ctx, const int32_t* h_modes);

/* Autotuner tables (the tile and schedule choice per class of instances):
 * instances are grouped into classes by the key (N bucket = bit length of
 * n - 1, boundary type, bed flag, halo bucket = bit length of the windowed
 * solve's halo estimate L of the loaded state, as hsgn_plan_info reports
 * it); each class is timed alone,
 * in a context of its own holding a copy of its instances, in each solver
 * mode (hsgn_autotune on that context, nsteps eager steps); each instance
 * then takes its class's fastest mode.  That per-class plan is timed on the
 * whole batch against the three uniform modes, and the fastest of the four
 * is kept.  The loaded state, time, status and speed bounds are left as
 * they were.
 *  max_classes: room in the class arrays; more classes give HSGN_EINVAL;
 *  h_nclass: host, the number of classes;
 *  h_class_of: host, n_inst class indices, or NULL;
 *  h_keys: host, max_classes x 4 ints (N bucket, bc, bed, halo bucket), or NULL;
 *  h_ms: host, max_classes x 3 ms per step, indexed by mode, or NULL;
 *  h_kept: host, max_classes modes, or NULL;
 *  h_whole: host, 5 doubles or NULL: whole-batch ms per step of the three
 *    uniform modes (indexed by mode), of the per-class plan, and the plan
 *    kept (its mode, or -1 for the per-class plan).
 * Allocates the class contexts and a copy of the state for its duration;
 * synchronises the stream. */
int hsgn_autotune_classes(hsgn_ctx* ctx, int32_t nsteps, int32_t max_classes, int32_t* h_nclass,
                          int32_t* h_class_of, int32_t* h_keys, double* h_ms, int32_t* h_kept,
                          double* h_whole);

/* Safety factor of the halo estimates (default 2): the windowed solves size
 * their halos from the decay of the depth rows (the phi rows with the SGN
 * scheme) estimated at `margin` times the coupling of the loaded state's
 * deepest cell (the semi-implicit estimate also at its speed bound).  A
 * smaller factor gives shorter halos, fewer window rows, and more instances
 * flagged: every window still certifies its truncation (HSGN_FLAG_WINDOW,
 * HSGN_EWINDOW).  0 < margin <= 64, else HSGN_EINVAL.  Re-plans at once;
 * the class autotuner's contexts take the same factor. */
int hsgn_set_halo_margin(hsgn_ctx* ctx, double margin);

/* Halo retry, for callers that run with a small halo margin: enable = 1
 * turns it on, 0 (the default) off (else HSGN_EINVAL).  When on, hsgn_step
 * (each call) and hsgn_run (each graph block, and the eager remainder)
 * copy the mutable state first (the four fields, times, speed bounds,
 * status and step counts: 4 doubles per cell, allocated on first use and
 * kept until hsgn_destroy), then read the status flags, which synchronises
 * the stream.  If a windowed solve flagged its truncation
 * (HSGN_FLAG_WINDOW), the copy is restored, the halo margin of every
 * flagged instance doubled (at most 64; the instance keeps its new margin,
 * the others keep theirs), the solver re-planned and the block run again,
 * so every window of the result certifies its truncation as with the
 * default margin.  Other flags, and a window flag at margin 64, are left
 * for hsgn_status.  hsgn_set_halo_margin resets the per-instance margins.
 * No effect with the explicit scheme (no windows).  The windowed solves of
 * hsgn_adjoint do not retry. */
int hsgn_set_halo_retry(hsgn_ctx* ctx, int32_t enable);

/* Current halo margin of every instance (h_margin, host, n_inst doubles, or
 * NULL) and the number of blocks run again by the halo retry since the
 * state was loaded (h_retries, host, or NULL). */
int hsgn_halo_state(hsgn_ctx* ctx, double* h_margin, int32_t* h_retries);

/* Launch of the window stages:
 *  HSGN_LAUNCH_GRID (the default): one workgroup per window, consecutive
 *    windows of an instance dealt to one XCD; the hardware dispatcher
 *    refills a finished workgroup's slot.
 *  HSGN_LAUNCH_PERSISTENT: as many workgroups as are resident at once, each
 *    taking windows from eight work queues (one per XCD, atomic tickets; a
 *    workgroup drains its own XCD's queue first, then the others).  The
 *    kernel resets its queue counters at its end, so graphs replay it as
 *    they are.
 * Both give bitwise the same results (each window is computed the same
 * way).  A change drops the cached hsgn_run graphs.  Contexts of
 * hsgn_step_noalloc have no queues (HSGN_EINVAL for the persistent launch).
 * Two window launches of one context must not overlap: the context's
 * stream orders them (the adjoint's recompute stream has queues of its
 * own). */
#define HSGN_LAUNCH_GRID 0
#define HSGN_LAUNCH_PERSISTENT 1
int hsgn_set_launch(hsgn_ctx* ctx, int32_t launch);

/* Time both launches (nsteps eager steps each, on the current plan and the
 * loaded state), keep the faster, and leave the state, time, status and
 * speed bounds as they were.  h_ms (host, 2 doubles or NULL): milliseconds
 * per step indexed by launch; h_launch (host or NULL): the launch kept.
 * Allocates a copy of the state for its duration; synchronises the stream.
 * Semi-implicit scheme only (else HSGN_EINVAL). */
int hsgn_autotune_launch(hsgn_ctx* ctx, int32_t nsteps, double* h_ms, int32_t* h_launch);

/* Plan of the loaded state (host arrays, any may be NULL): h_mode[j] = 0
 * windowed / 1 exact two-pass; h_halo[j] = halo rows L of instance j's
 * windows (the estimate from the loaded state, also for an instance in the
 * exact mode; 0 before a state is loaded; 1 << 30 where no finite halo
 * would do);
 * h_counts[4] = {windows, two-pass tiles, two-pass instances with more than
 * one tile, window rows (2048 or 4096; -1 when both widths are used)}. */
int hsgn_plan_info(hsgn_ctx* ctx, int32_t* h_mode, int32_t* h_halo, int32_t* h_counts);

/* Kernel kinds timed by hsgn_step_timed. */
#define HSGN_K_DT 0           /* time step per instance                     */
#define HSGN_K_REDUCE1 1      /* stage 1, tile reduction (multi-tile only)   */
#define HSGN_K_RSOLVE1 2      /* stage 1, reduced system across tiles        */
#define HSGN_K_STAGE1 3       /* stage 1, sweep + solve + back-substitution  */
#define HSGN_K_REDUCE2 4
#define HSGN_K_RSOLVE2 5
#define HSGN_K_STAGE2 6
#define HSGN_K_WIN1 7         /* stage 1, windowed single pass               */
#define HSGN_K_WIN2 8         /* stage 2, windowed single pass               */
#define HSGN_K_EX1 9          /* explicit scheme, first Heun stage           */
#define HSGN_K_EX2 10         /* explicit scheme, second Heun stage          */
#define HSGN_K_SGN_ROWS 11    /* SGN: unused (rows are formed in the solve)  */
#define HSGN_K_SGN_SOLVE 12   /* SGN: batched tridiagonal solve for phi      */
#define HSGN_K_SGN_UPDATE 13  /* SGN: flux update with the source h phi      */
#define HSGN_NKERNEL 14

/* Measurement variant of hsgn_step: the same launches, each bracketed by HIP
 * events on the library's stream; synchronises at the end.  h_ms[k]
 * receives the summed milliseconds of kernel kind k over the nsteps steps
 * and h_count[k] its number of launches (host arrays of HSGN_NKERNEL;
 * either may be NULL).  Results are identical to hsgn_step. */
int hsgn_step_timed(hsgn_ctx* ctx, int32_t nsteps, double* h_ms, int32_t* h_count);

/* Discrete adjoint (reverse mode of the IMEX step, hand-written) of the
 * gauge misfit
 *   J_j = (1/2) sum_{s=1..nsteps} sum_{g<n_gauge} (h_j^s(gauge_jg) - target_jsg)^2
 * of every instance j, started from rest with free surface zeta0:
 * h = zeta0 - b, q = 0, m = h^2, W = 0.  Gradients of J_j with respect to
 * zeta0 and to the bed b of instance j (cells of instance j).
 *  nsteps: steps; K: steps between checkpoints (segments are recomputed
 *    from their checkpoint during the reverse sweep, storing U^n and U^(1)
 *    of each step);
 *  d_gauge: device int32 [n_inst][n_gauge], cells relative to the instance;
 *  d_target: device [n_inst][nsteps][n_gauge];
 *  d_zeta0: device, offsets[n_inst] doubles;
 *  d_loss: device [n_inst]; d_grad_zeta0, d_grad_b: device, offsets[n_inst]
 *    doubles or NULL; when both are NULL only the loss is computed (no
 *    reverse sweep, no adjoint workspace).
 * Only for the two-stage semi-implicit step (order 2, scheme 0).  Every
 * instance must use a fixed step (dt_fixed > 0, t_end <= 0), so that
 * the step map is differentiable, and every gauge cell must lie in its
 * instance (else HSGN_EINVAL).  Forward steps use the solver plan made from
 * the initial state (the status flags are cleared first, as by
 * hsgn_set_state); the reverse stages solve the transposed depth system
 * exactly (no truncation).
 * On return the state is the state after nsteps steps and t is reset to 0.
 * If an instance is flagged during the forward pass (HSGN_FLAG_*), it was
 * frozen from that step on and its loss would be that of another map: the
 * call then returns that flag's error code (precedence and message as for
 * hsgn_status) before the reverse sweep, with d_loss written and the
 * gradients not.
 * When the tapes of all segments (8 nsteps doubles per cell) fit the tape
 * budget (hsgn_set_adjoint_tape_bytes), the forward pass writes all of them
 * and no segment is recomputed.  Otherwise it writes the tapes of the last
 * two segments itself (one per tape buffer), and every earlier segment is
 * recomputed from its checkpoint on a second stream of the library while
 * the following segment is swept in reverse.  Both give the same results
 * bit for bit.  The adjoint workspace (22 doubles per cell, the tapes: 8 K
 * doubles per cell per tape buffer, plus 4 (nsteps/K + 1) doubles per cell
 * of checkpoints) is kept until hsgn_destroy.
 * Synchronises the stream twice: after the initial state (to plan) and
 * after the forward pass (to read the status flags). */
int hsgn_adjoint(hsgn_ctx* ctx, int32_t nsteps, int32_t K, int32_t n_gauge,
                 const int32_t* d_gauge, const double* d_target, const double* d_zeta0,
                 double* d_loss, double* d_grad_zeta0, double* d_grad_b);

/* Memory for hsgn_adjoint's tapes, in bytes: when the tapes of every
 * segment fit it, the forward pass tapes them all and nothing is
 * recomputed; 0 always recomputes (two tape buffers).  Negative (the
 * default): half the device memory free at the hsgn_adjoint call (a tape
 * already held by the context counts as free). */
int hsgn_set_adjoint_tape_bytes(hsgn_ctx* ctx, int64_t bytes);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid allocation): the
 * work of hsgn_init + hsgn_set_state + hsgn_step(nsteps) + hsgn_get_state in
 * one call that allocates nothing.  The library's buffers (the U^(1) and
 * stage-output state copies, descriptors, plan lists, per-instance values,
 * reduced rows) are carved from one static device array of about 66 MiB,
 * which every GPU the library runs on holds until the process ends; the
 * kernels are those of hsgn_step and the results are bitwise those of the
 * context path with the same solver mode.
 *  offsets, params, d_b: as for hsgn_init (host, host, device or NULL);
 *    semi-implicit scheme only (scheme 0), order 1 or 2.
 *  d_h, d_q, d_m, d_W: device, offsets[n_inst] doubles each, all required:
 *    the state, advanced in place by nsteps steps.
 *  d_t: device, n_inst times (advanced in place), or NULL for t = 0.
 *  solver: HSGN_SOLVER_AUTO, HSGN_SOLVER_EXACT or HSGN_SOLVER_AUTO_SMALL.
 *  hip_stream: the stream every copy and kernel is enqueued on.
 *  h_flags: host, n_inst int32 status bits after the steps, or NULL.
 *  h_msg: host, HSGN_MSG_LEN chars or NULL: the error message ("" on
 *    success), as hsgn_last_error gives it for a context.
 * Limits: at most HSGN_NOALLOC_MAX_CELLS cells and HSGN_NOALLOC_MAX_INST
 * instances (else HSGN_EINVAL, before anything is enqueued).  Returns as
 * hsgn_status after the steps (a flagged instance: its code).  Synchronises
 * the stream (to plan, and at the end).  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (from several host threads, or
 * on several streams) race and must be serialised by the caller. */
#define HSGN_NOALLOC_MAX_CELLS (1 << 20)
#define HSGN_NOALLOC_MAX_INST 4096
#define HSGN_MSG_LEN 512
int hsgn_step_noalloc(int32_t n_inst, const int64_t* offsets, const hsgn_params* params,
                      const double* d_b, double* d_h, double* d_q, double* d_m, double* d_W,
                      double* d_t, int32_t nsteps, int32_t solver, void* hip_stream,
                      int32_t* h_flags, char* h_msg);

/* Synchronise the stream and copy the per-instance status bits to host
 * (h_flags: n_inst int32, may be NULL).  Returns HSGN_OK if no instance is
 * flagged, else HSGN_ENONPHYS, HSGN_EWINDOW or HSGN_ENONCOERCIVE (in that
 * order of precedence); hsgn_last_error then names the first instance with
 * that flag, the step (counted from the last hsgn_set_state) in which the
 * flag was raised, its time, and how many instances carry the flag. */
int hsgn_status(hsgn_ctx* ctx, int32_t* h_flags);

/* Message describing the last failure of this context ("" if none): the
 * failing call and, for a flagged instance, the instance, the step and the
 * time (see hsgn_status).  The string is owned by the context. */
const char* hsgn_last_error(const hsgn_ctx* ctx);

/* Library version string. */
const char* hsgn_version(void);

/* Free the context and everything it allocated (NULL is a no-op). */
void hsgn_destroy(hsgn_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* HSGN_H */
