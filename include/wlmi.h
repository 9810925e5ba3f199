/*
 * wlmi.h - C ABI of the MI355X BDIM projection solver step.
 *
 * The library computes one time step of the boundary-data-immersion method
 * (BDIM) on a staggered uniform Cartesian grid, as described in the
 * numerical-methods section of Weymouth & Font, "WaterLily.jl: a
 * differentiable and backend-agnostic Julia solver for incompressible viscous
 * flow around dynamic bodies" (arXiv 2407.16032): the limited-QUICK
 * convection-diffusion flux, the BDIM blend of the fluid update with the
 * body's kernel moments mu0/mu1, and the pressure projection solved by
 * geometric multigrid with a Jacobi-PCG smoother, inside an explicit
 * predictor-corrector step with an adaptive CFL time step.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units: grid units, h = 1 cell.  Cell I (0-based padded index, interior
 *   1..n[d], one ghost layer per side; the paper's inside(p)) has its centre
 *   at x = I - 1/2.  Velocity component i at index I sits on the lower
 *   i-face of cell I (x_i = I_i - 1).
 * Layout: every field is a device array of the simulation's precision (float
 *   or double), one array per component, x fastest:
 *     element (i, j, k) at  ((k * py) + j) * px + i,
 *   px >= n[0]+2 (row pitch, a multiple of 64 elements), py = n[1]+2,
 *   pz = n[2]+2 (pz = 1 in 2-D).  wl_field() reports shapes and strides.
 * Memory: the caller allocates ONE device workspace of wl_workspace_bytes()
 *   bytes and owns it; the library never allocates device memory and keeps
 *   only a small host object (plus 64 bytes of pinned host memory for
 *   scalar read-back).  All fields live inside the workspace.
 * Streams: all device work is enqueued on the hipStream_t given at creation.
 *   Calls return after enqueueing, except that the multigrid solve reads one
 *   residual norm per V-cycle back to the host (a stream synchronisation)
 *   and wl_step reads the new time step at its end.
 * Errors: every call returns wl_status; nothing throws across the ABI.
 *   Argument errors are detected before any work is enqueued.  A multigrid
 *   solve that reaches its cycle limit is NOT an error (converged = 0).
 *   wl_last_error() gives a thread-local message for the last failure.
 * Threading: a wl_sim is not thread-safe; distinct sims are independent.
 */
#ifndef WLMI_H
#define WLMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WL_OK = 0,
  WL_ERR_INVALID_ARG = 1,
  WL_ERR_WORKSPACE_TOO_SMALL = 2,
  WL_ERR_HIP = 3,
  WL_ERR_NONFINITE = 4,
  WL_ERR_UNSUPPORTED = 5
} wl_status;

typedef enum { WL_F32 = 0, WL_F64 = 1 } wl_prec;

/* Simulation description (paper, software-design section: Simulation takes
 * the grid size, length/velocity scales, viscosity, boundary conditions, the
 * body, the float type T).  Defaults in brackets are applied when a field is
 * zero. */
typedef struct {
  int ndim;              /* 2 or 3 */
  int64_t n[3];          /* interior cells per axis; n[2] ignored in 2-D.  Each >= 4. */
  double L;              /* characteristic length in cells (the paper's Simulation argument L):
                            wl_sim_time reports t |U| / L [1] */
  double U[3];           /* free-stream velocity (inflow/slip normal faces take U_i) */
  double nu;             /* kinematic viscosity (>= 0) */
  unsigned periodic_mask;/* bit d set -> axis d periodic */
  int convective_exit;   /* 1 -> convective outlet on the +x face (needs U[0] != 0, x not periodic) */
  int prec;              /* wl_prec: field precision; reductions are always FP64 */
  double eps;            /* BDIM kernel half-width in cells [1] */
  double dt0;            /* first time step [0.25] */
  double dt_max;         /* upper bound of the CFL step [10] */
  double cfl_nu_coef;    /* dt = min(dt_max, 1/(max outflux + cfl_nu_coef*nu)) [5] */
  double mg_tol;         /* residual max-norm tolerance of the projection solve [1e-6] */
  int mg_itmax;          /* maximum V-cycles per solve [32] */
  int pcg_iters;         /* PCG smoothing iterations per level [6] */
  int learned_guess;     /* 1 -> plan the buffers of the learned initial guess (3-D only) */
  int adjoint;           /* 1 -> plan the buffers of the discrete adjoint (wl_adj_*) */
  int solver_path;       /* PCG kernels of the 3-D multigrid levels: 0 = automatic (flat
                            vector passes on every level of >= 2^14 cells whose rows hold
                            whole 16-byte vectors), 1 = z-marching tiles on the levels of
                            >= 2^18 cells, 2 = as 0, 3 = the generic grid-stride kernels
                            only.  The levels of <= 4096 cells run the single-workgroup
                            bottom solve in every case.  The arithmetic is the same; sums
                            differ in rounding order only. [0] */
  int reduce_mode;       /* how the flat launches of the large 3-D levels total their
                            per-block partial sums: 0 = automatic (up to 256 blocks the
                            consumer kernels add them; more: a separate totalling launch,
                            in two stages above 16384 partials), 1 = always a separate
                            single-stage launch, 2 = always two stages.  Same arithmetic,
                            sums in a different fixed order. [0] */
  int blend_mode;        /* where a step applies the BDIM blend: 0 = automatic (3-D steps
                            that record nothing for the adjoint blend every face outside
                            the body box inside the flux launch, where the coefficients
                            are body-free, and the box's faces in a launch of their own;
                            the corrector then writes the new velocity over the old one,
                            so WL_FIELD_U0 afterwards holds the predictor's projected
                            velocity), 1 = always a separate pass over every face after
                            the flux launch.  Same arithmetic and the same results. [0] */
  int vcycle_graph;      /* 2 = the coarse part of each multigrid cycle (restriction, the
                            coarse levels' PCG, the bottom solve, prolongation) is captured
                            in a HIP graph (on a stream of the library's own) and
                            replayed on the sim's stream while the partial-sum counts and
                            body boxes it was captured with hold (not while the profiler
                            times those kernels; a capture that fails turns graphs off for
                            the sim); 1 = plain launches; 0 = automatic: as 2 unless the
                            body moves (its box, a launch argument, then changes from step
                            to step), else as 1.  The same kernels with the same
                            arguments.  Graphs, and the one capture stream, are HIP runtime
                            objects the library creates at the first step (no workspace
                            memory); a caller that allows no runtime object creation after
                            wl_sim_create sets 1. [0] */
} wl_sim_desc;

typedef enum {
  WL_BODY_NONE = 0,
  WL_BODY_SPHERE = 1,   /* |x_b| - radius (a circle in 2-D) */
  WL_BODY_BOX = 2,      /* box of half extents half_extent, centred at the body-frame origin */
  WL_BODY_GRID_SDF = 3, /* signed distance sampled on a grid in the body frame (see below) */
  WL_BODY_PLANE = 4     /* half space normal . x_b - radius <= 0 (normal: body frame, unit) */
} wl_body_kind;

/* How a part combines with the body formed by the parts before it (paper,
 * applications section: bodies are combined by the arithmetic of their signed
 * distances).  UNION takes the part nearer to the point (min of d), INTERSECT
 * the farther (max of d), SUBTRACT the body minus the part (max of d and -d_part).
 * The point takes d, n and V of the part that wins, n flipped with d for a
 * subtracted part. */
typedef enum { WL_OP_UNION = 0, WL_OP_INTERSECT = 1, WL_OP_SUBTRACT = 2 } wl_body_op;

/* A body (the paper's AutoBody: a signed-distance function and a coordinate
 * map; software-design section).  One descriptor is one part; parts chain
 * through `next` (at most 8), each combined with those before it by its `op`
 * (ignored on the first).
 *
 * Map of a part from world coordinates x to its body frame x_b:
 *   x_b = S(t) * (Rot(-theta(t)) (x - P(t))) + pivot_offset     (* per axis)
 *   P(t) = center + velocity t + heave_amp sin(2 pi freq t + phase_h) e_h + pivot_offset
 *   theta(t) = pitch_amp sin(2 pi freq t + phase_p) + spin_omega t  (about e_z)
 *   S_a(t) = 1 + scale_amp[a] sin(2 pi freq t + phase_s)
 * with e_h = heave_dir normalised (e_y when heave_dir is zero).  The shape is
 * defined in the body frame around its origin; SDF < 0 inside; shell > 0 makes
 * the part hollow (|SDF| - shell).
 * Measured quantities at a point (paper: every geometric property comes from
 * derivatives of the SDF and of the map): the normal n is the world gradient of
 * the part's SDF through the map, normalised, and d is the SDF divided by that
 * gradient's magnitude (the two agree with the SDF and its normal when the map is
 * rigid, S = 1); the body velocity is V = -J^{-1} dx_b/dt with J = dx_b/dx, the
 * velocity of the material point the map holds fixed (rigid motion: the velocity
 * of P plus the angular velocity times x - P).
 * Gridded SDF: sdf_grid holds grid_n[0] x grid_n[1] (x grid_n[2]) samples (each
 * >= 2), in the simulation's precision, x fastest: sample (i, j, k) at index
 * (k grid_n[1] + j) grid_n[0] + i sits at body-frame point grid_origin +
 * (i, j, k) grid_h.  d is the multilinear interpolant of the samples; the
 * normal is the interpolant, with the same weights, of the samples' gradients by
 * central differences (one-sided on the grid's faces), normalised; outside the
 * sampled box the point is fluid beyond the kernel's reach.  vel_grid (may be
 * NULL) holds ndim components of the same shape, one after the other, whose
 * interpolant is added to the map's velocity.  Both arrays are device pointers,
 * read at creation (and by wl_body_update) into the workspace, so the caller may
 * free them afterwards.
 * The body must stay at least 3 cells away from non-periodic domain faces
 * (checked at every measure of a moving body). */
typedef struct wl_body_desc {
  int kind;                 /* wl_body_kind */
  double center[3];
  double radius;            /* sphere/circle radius; plane offset */
  double half_extent[3];    /* box */
  double heave_amp, pitch_amp, freq, phase_h, phase_p;
  double pivot_offset[3];
  double spin_omega;
  double velocity[3];       /* uniform translation of P */
  double heave_dir[3];      /* direction of the heave (zero: e_y) */
  double scale_amp[3];      /* per-axis amplitude of the map's scale S(t) */
  double phase_s;           /* phase of S(t) */
  double normal[3];         /* plane normal in the body frame */
  double shell;             /* > 0: hollow part of this half thickness */
  const void* sdf_grid;     /* WL_BODY_GRID_SDF: device samples (simulation precision) */
  const void* vel_grid;     /* optional sampled velocity, ndim components */
  int64_t grid_n[3];
  double grid_origin[3];
  double grid_h;
  int op;                   /* wl_body_op: combination with the parts before this one */
  const struct wl_body_desc* next;  /* next part or NULL */
} wl_body_desc;

typedef struct {
  double dt;            /* step just taken */
  double t;             /* time after the step */
  double dt_next;       /* CFL step for the next call */
  int vcycles[2];       /* predictor / corrector multigrid V-cycles */
  double res0_linf[2];  /* residual max-norms of the two solves before their first cycle (FP64) */
  double res_linf[2];   /* final residual max-norms of the two solves (FP64) */
  double res_l2[2];     /* final residual 2-norms over the active cells (FP64 sums) */
  double div_linf;      /* max |div u| over the active cells after the step (FP64) */
  int converged;        /* 1 if both solves met mg_tol */
} wl_step_stats;

typedef struct {
  int vcycles;
  double res0_linf;     /* residual max-norm before the first cycle */
  double res_linf;      /* after the last cycle */
  double res_l2;        /* 2-norm of the final residual over the active cells (FP64 sums) */
  int converged;
} wl_solve_stats;

typedef struct wl_sim wl_sim;

/* Bytes of device workspace needed for (desc, body); 0 on invalid input. */
size_t wl_workspace_bytes(const wl_sim_desc* desc, const wl_body_desc* body);

/* Create a simulation in a caller-owned device workspace (256-byte aligned,
 * at least wl_workspace_bytes bytes) on the given hipStream_t (NULL = the
 * null stream).  Initialises u = U (with boundary conditions), p = 0, t = 0,
 * dt = dt0, and measures the body at t = 0.  body may be NULL (no body). */
wl_status wl_sim_create(const wl_sim_desc* desc, const wl_body_desc* body, void* dev_workspace,
                        size_t bytes, void* hip_stream, wl_sim** out);

/* Release the host object; the workspace stays the caller's. */
wl_status wl_sim_destroy(wl_sim* sim);

/* measure! (paper, performance section): evaluate d, n, V of the body at time
 * t at every velocity point, store mu0 (which is also the fine Poisson
 * coefficient L, with non-periodic boundary faces set to 0), mu1 = mu1(d) n,
 * V, and rebuild the Poisson coefficients and inverse diagonals of every
 * multigrid level. */
wl_status wl_measure_body(wl_sim* sim, double t);

/* One predictor-corrector time step n -> n+1 (numerical-methods section).
 * remeasure != 0 re-runs measure at t_n first when the body moves.  Writes
 * stats if non-NULL.  Returns WL_ERR_NONFINITE if the new time step is not
 * finite (the velocity blew up). */
wl_status wl_step(wl_sim* sim, int remeasure, wl_step_stats* stats);

/* Apply the velocity boundary conditions to the current velocity field
 * (call after writing u through a wl_field view). */
wl_status wl_apply_bc(wl_sim* sim);

/* Convection-diffusion residual R(u) of the current velocity into the
 * scratch field WL_FIELD_F (R on the unknown faces, 0 elsewhere). */
wl_status wl_conv_diff(wl_sim* sim);

/* Projection stage alone on the current velocity with weight w (1 in the
 * predictor, 1/2 in the corrector): z = div u, x0 = p w dt, multigrid solve of
 * A x = z to mg_tol, u_i -= L_i (x[I] - x[I-e_i]), p = x/(w dt), then the
 * boundary conditions. */
wl_status wl_project(wl_sim* sim, double w, wl_solve_stats* stats);

/* Multigrid solve of A x = rhs on the fine level (software-design section:
 * the Poisson coefficients c; numerical-methods section: geometric
 * multigrid).  rhs: device array in the pressure layout, or NULL for the
 * divergence of the current velocity.  x_inout: device array in the pressure
 * layout holding the initial guess, overwritten by the solution; NULL uses
 * the internal WL_FIELD_X.  tol <= 0 or itmax <= 0 take the sim defaults. */
wl_status wl_poisson_solve(wl_sim* sim, const void* rhs, void* x_inout, double tol, int itmax,
                           wl_solve_stats* stats);

/* Pressure and viscous force on the body at the current time (FP64 sums over
 * cell centres; paper, results sections: forces as integrals of the surface
 * stress weighted by the smoothed surface delta K_eps(d)):
 *   F_p = -sum (p - pbar) n K_eps(d),   F_v = sum 2 nu S n K_eps(d),
 * pbar = mean of p over active cells (the pressure's gauge drops out), S the
 * strain rate of u interpolated to the cell centre. */
wl_status wl_forces(wl_sim* sim, double f_pressure[3], double f_viscous[3]);

/* wl_forces for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same force sums,
 * with their per-block partials and totals in a fixed static device array of
 * 11 x 2048 + 16 doubles (about 176 KiB, held by each GPU the library runs on
 * until the process ends) instead of the simulation's workspace.  Allocates
 * nothing (no device, pinned or host memory) and reads the 11 totals back into
 * the simulation's pinned buffer.  The sums are added in a different fixed order
 * than wl_forces, so the two agree to rounding.  Every call on one GPU shares
 * that array: calls that overlap on one GPU (two host threads, or two streams in
 * flight at once) race and must be serialised by the caller.  Synchronises the
 * simulation's stream.  A force grid larger than the array returns
 * WL_ERR_UNSUPPORTED (the grid is at most 2048 blocks, so this does not occur). */
wl_status wl_forces_static(wl_sim* sim, double f_pressure[3], double f_viscous[3]);

enum {
  WL_FIELD_U = 0,     /* velocity, ndim components */
  WL_FIELD_U0 = 1,    /* second velocity buffer: after a step the previous velocity, or
                         the predictor's projected velocity when the step blended in the
                         flux launch (blend_mode) */
  WL_FIELD_F = 2,     /* scratch f~ / R, ndim components (after a blended-in-flux step,
                         valid only within one face of the body box) */
  WL_FIELD_V = 3,     /* body velocity, ndim components */
  WL_FIELD_MU0 = 4,   /* mu0 = fine-level L, ndim components */
  WL_FIELD_MU1 = 5,   /* mu1_ij at component i*ndim + j */
  WL_FIELD_P = 6,     /* pressure */
  WL_FIELD_X = 7,     /* multigrid solution on level `level` */
  WL_FIELD_R = 8,     /* multigrid residual on level `level` */
  WL_FIELD_L = 9,     /* Poisson coefficients on level `level`, ndim components */
  WL_FIELD_ID = 10,   /* inverse diagonal on level `level` (0 on solid cells) */
  WL_FIELD_ADJ_U = 11,/* adjoint of the current velocity, ndim components (desc.adjoint) */
  WL_FIELD_ADJ_P = 12 /* adjoint of the current pressure (desc.adjoint) */
};

/* Zero-copy view of a field inside the workspace.  shape = {components, pz,
 * py, px_used} with px_used = n[0]+2 of that level; strides in elements
 * {component, z, y, x}.  level selects the multigrid level for X, R, L, ID. */
wl_status wl_field(wl_sim* sim, int which, int level, void** dev_ptr, int64_t shape[4],
                   int64_t strides[4]);

/* Number of multigrid levels and the interior size of one of them. */
wl_status wl_levels(wl_sim* sim, int* nlevels, int level, int64_t n_out[3]);

/* Set the clock and the next time step. */
wl_status wl_set_time(wl_sim* sim, double t, double dt_next);
wl_status wl_get_time(wl_sim* sim, double* t, double* dt_next);

/* Convective time t* = t |U| / L of the current clock (the paper's time scale
 * tU/L), with |U| the magnitude of desc.U, taken as 1 when U = 0. */
wl_status wl_sim_time(wl_sim* sim, double* t_star);

/* Replace the body's parameters (same kind) and re-measure at the current time. */
wl_status wl_body_update(wl_sim* sim, const wl_body_desc* body);

/* Index box (padded indices, inclusive; empty if lo[0] > hi[0]) of multigrid
 * level `level` outside of which the coefficients are body-free: L = 1 on the
 * fine level (times 2^(ndim-2) per coarsening) on interior faces, 0 on
 * non-periodic boundary faces, iD from those, and on the fine level mu1 = 0,
 * V = 0.  The kernels evaluate these in closed form there instead of loading
 * them (paper, software-design section: measure! fills the coefficient fields
 * only where the body has an influence).  Valid after the last measure. */
wl_status wl_body_box(wl_sim* sim, int level, int lo[3], int hi[3]);

/* ---------------------------------------------------------------------------
 * Discrete adjoint of the time step (the paper obtains derivatives of the
 * solver by running it on dual numbers, software-design section and the
 * rotating-cylinder example; this is the reverse-mode equivalent, built from
 * the transposes of the step's kernels).  Needs desc.adjoint = 1, no
 * convective exit, and a body whose shape does not move (none, a fixed box,
 * or a sphere/circle that may spin).  Conventions: the time step is frozen
 * to the value the forward used; the QUICK limiter is linearised on the
 * branch the forward took; each multigrid solve counts as the exact solution
 * of A x = z on the active cells with the mean of z removed, so its
 * transpose is one more solve with the same operator (A is symmetric).
 * Adjoint state: ubar (WL_FIELD_ADJ_U) and pbar (WL_FIELD_ADJ_P) belong to
 * the current state; accumulators hold the adjoints of mu0 (with the Poisson
 * coefficient L, which is the same field), mu1 and V over all reversed steps.
 * Scatter transposes use atomics: results agree to rounding, not bitwise.
 * Typical reverse sweep of an objective J = sum_k w_k dir . F(state k):
 *   wl_adj_reset; for k = K .. 1: [set the state to k, wl_adj_forces(w_k)],
 *   set the state to k-1 (u, p, t, frozen dt via wl_set_time), wl_adj_step;
 *   then wl_adj_body_grad.
 * ------------------------------------------------------------------------- */

/* Zero ubar, pbar and the accumulators. */
wl_status wl_adj_reset(wl_sim* sim);

/* Add the gradient of weight * dir . (F_p + F_v) (wl_forces) at the current
 * state: into ubar (viscous term), pbar (pressure term, gauge-free), and, for a
 * sphere, the direct radius derivative through K_eps(d) into the accumulators.
 * value (may be NULL) receives dir . (F_p + F_v).  Synchronises the stream. */
wl_status wl_adj_forces(wl_sim* sim, const double dir[3], double weight, double* value);

/* Reverse of one time step.  On entry the current state (u, p, t) is the
 * state n at the START of the step and dt_next (wl_set_time) its frozen
 * step; ubar/pbar hold the adjoints of the state n+1.  The call recomputes
 * the step forward (remeasuring a spinning body as wl_step does), recording
 * its intermediates, then runs the transposes in reverse order.  On return the
 * current state is n+1 (and dt_next its CFL value), ubar holds the adjoint of
 * u^n, pbar is 0 (p^n does not influence the step), and the mu0/mu1/V
 * accumulators have grown.  tol: residual max-norm of the two adjoint solves
 * (<= 0: desc.mg_tol); adjoint_stats (may be NULL) receives the predictor and
 * corrector adjoint solves' statistics, forward_stats the recomputed step's. */
wl_status wl_adj_step(wl_sim* sim, double tol, wl_step_stats* forward_stats, wl_solve_stats adjoint_stats[2]);

/* wl_adj_step for a rollout whose time steps follow the CFL rule (the step is not
 * frozen): as wl_adj_step, and also the adjoint of the step's dt, which enters
 * through f~ = u0 + dt R - V in both stages and p = x / (w dt),
 *   dt_bar = [<fbar_1, f~_1 - u0 + V> + <fbar_2, f~_2 - u0 + V> - <pbar, p^{n+1}>] / dt,
 * written to *dt_bar (may be NULL).  dt_from_cfl != 0 states that dt_n was
 * min(dt_max, 1/(sigma_max(u^n) + cfl_nu_coef nu)) of the state u^n (not dt0 and not
 * set by the caller): then, when below dt_max, dt_bar (-dt^2) d sigma(I*)/du^n is
 * added to the adjoint of u^n, I* the cell of the largest outflux (the first such cell
 * in x-fastest order), the derivative of the CFL map on its active branch.  The
 * oracle's reference is the complex step of the rollout with the steps live.
 * Synchronises the stream once more than wl_adj_step. */
wl_status wl_adj_step_cfl(wl_sim* sim, double tol, int dt_from_cfl, double* dt_bar, wl_step_stats* forward_stats,
                          wl_solve_stats adjoint_stats[2]);

/* Gradient of the objective with respect to the sphere's radius (at fixed
 * spin rate) and spin rate omega, from the accumulators: mu0 = mu0(d) and
 * mu1 = mu1(d) n with d = |x - c| - R, V = omega e_z x (x - c) where
 * measure sets it, plus the force functionals' direct radius terms.  Sphere
 * bodies only.  Synchronises the stream. */
wl_status wl_adj_body_grad(wl_sim* sim, double* dJ_dradius, double* dJ_dspin);

/* ---------------------------------------------------------------------------
 * Learned multigrid initial guess (an extension of the method, not in the
 * paper): a 3-layer 3x3x3 conv net (3 -> 16 -> 16 -> 1 channels, ReLU, BF16
 * weights and activations, FP32 accumulation on MFMA) maps the previous two
 * pressures and the current divergence, normalised by the mean and RMS
 * deviation of p_{m-1} over active cells, to the pressure change of the next
 * solve; x0 = (p_{m-1} + s * out) w dt replaces the warm start x0 = p w dt.  The
 * multigrid solve to the same tolerance decides whether the guess is used.  Online
 * training: after each guided solve, random crops (64^3 or the grid) of the
 * features and the target (p_m - p_{m-1})/s enter a ring buffer; each solve then
 * runs train_iters Adam steps (FP32 master weights) on ring crops, loss = mean
 * over the crop's inner cells (3 cells from its faces) of the squared
 * mean-removed error.  Needs desc.learned_guess = 1 and ndim = 3.
 * Parameters: a flat FP32 vector of WL_PG_PARAMS values
 *   W1[27][3][16] b1[16] W2[27][16][16] b2[16] W3[27][16][1] b3[1],
 * taps ordered 9 (dz+1) + 3 (dy+1) + (dx+1), out[p] = b + sum W[tap]^T in[p + off].
 * Box arrays (wl_pg_forward / wl_pg_train_step): channels-last on a box of
 * interior n[0] x n[1] x n[2] (each <= 64 and <= the grid) with a one-cell zero
 * halo, point (x, y, z) at ((z (n1+2) + y) (n0+2) + x), x fastest.
 * ------------------------------------------------------------------------- */
#define WL_PG_PARAMS 8673

/* Set the FP32 master parameters (host array of WL_PG_PARAMS), reset Adam. */
wl_status wl_pg_set_weights(wl_sim* sim, const float* host_params);
/* Copy the FP32 master parameters to a host array of WL_PG_PARAMS. */
wl_status wl_pg_get_weights(wl_sim* sim, float* host_params);
/* mode 0: plain warm start; 1: learned guess; 2: learned guess + online training.
 * lr: Adam learning rate; train_iters: Adam steps per solve; crops: crops taken
 * per solve; seed: crop placement / sampling. */
wl_status wl_pg_mode(wl_sim* sim, int mode, double lr, int train_iters, int crops, uint64_t seed);
/* Forward pass on a caller box: x_box device bfloat16 [P][4] (channel 3 = 0),
 * y_out device float [P] (written on the interior). */
wl_status wl_pg_forward(wl_sim* sim, const void* x_box, const int64_t n[3], float* y_out);
/* One training step on a caller box: forward, loss against target (device float
 * [P]) over mask (device uint8 [P]), backward; grad_out (host, WL_PG_PARAMS, may be
 * NULL) receives the FP32 gradient, loss (may be NULL) the loss; apply != 0 then
 * takes the Adam step with the mode's learning rate. */
wl_status wl_pg_train_step(wl_sim* sim, const void* x_box, const float* target, const unsigned char* mask,
                           const int64_t n[3], float* grad_out, double* loss, int apply);
/* Loss of the last training step, training steps and snapshots taken so far, and
 * how many guided solves used the guess out of those that tried it: a guess is
 * used only if its initial residual max-norm is below that of the plain warm
 * start (multigrid stays the fallback and decides).  Any pointer may be NULL. */
wl_status wl_pg_stats(wl_sim* sim, double* last_loss, int64_t* train_steps, int64_t* snapshots,
                      int64_t* guesses_used, int64_t* guesses_tried);

/* Kernel groups timed by the profiler. Fine-level launches are timed per
 * kernel; every launch on a coarser multigrid level counts as WL_K_COARSE. */
enum {
  WL_K_MEASURE = 0,  /* measure: d, n, V -> mu0, mu1, V */
  WL_K_COEF = 1,     /* inverse diagonals and coefficient restriction */
  WL_K_FLUX = 2,     /* convection-diffusion flux and f~ */
  WL_K_BDIM = 3,     /* BDIM blend */
  WL_K_BC = 4,       /* boundary conditions */
  WL_K_EXIT = 5,     /* convective exit plane */
  WL_K_DIVRES = 6,   /* divergence and initial residual */
  WL_K_PCG_A = 7,    /* fine PCG pass A: search direction and sigma = e.Ae (generic form: also A e) */
  WL_K_PCG_B = 8,    /* fine PCG pass B: x and r update */
  WL_K_RESTRICT = 9, /* fine -> first coarse residual restriction */
  WL_K_PROLONG = 10, /* first coarse -> fine prolongation and correction */
  WL_K_PROJECT = 11, /* velocity update u -= L grad x */
  WL_K_CFL = 12,     /* CFL outflux maximum */
  WL_K_FORCES = 13,  /* force integrals */
  WL_K_COARSE = 14,  /* all work on multigrid levels >= 1 */
  WL_K_REDUCE = 15,  /* totals of per-block partial sums (one block, or two stages) */
  WL_K_PG_INFER = 16,/* learned guess: features, conv net, guess */
  WL_K_PG_TRAIN = 17,/* learned guess: snapshots, training steps */
  WL_K_ADJOINT = 18, /* transposes of the step's kernels (adjoint solves count as multigrid) */
  WL_K_COUNT = 19
};

/* Per-kernel timing with HIP events recorded around each launch on the sim's
 * stream.  enable = 1 creates the events (host objects) and zeroes the
 * counters; 0 stops recording.  Timing adds one event pair per launch. */
wl_status wl_profile(wl_sim* sim, int enable);

/* As wl_profile, but only the groups whose bit is set in groups (bit k = group
 * k of the enum above) are timed, so a timed region can carry events around
 * one kernel group without the cost of an event pair per launch of every
 * other group; groups = 0 stops recording. */
wl_status wl_profile_groups(wl_sim* sim, uint32_t groups);

/* Accumulated time (ms) and launch count of one kernel group since the last
 * wl_profile(sim, 1); call after the timed work has completed. */
wl_status wl_profile_read(wl_sim* sim, int kernel, double* total_ms, int64_t* launches);

/* Thread-local message describing the last non-WL_OK status. */
const char* wl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* WLMI_H */
