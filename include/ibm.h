/*
 * ibm.h -- C ABI of the MI355X (gfx950) library for one pressure-based time step
 * of the discrete-forcing immersed boundary method for compressible flow with
 * heat exchange (Riahi, Goncalves da Silva, Meldi: "A Discrete Immersed Boundary
 * Method for the numerical simulation of heat transfer in compressible flows").
 *
 * Problem statement followed by the arguments:
 *   - a body given by Lagrangian markers (Sec. 2.2), with a desired velocity
 *     (Eq. (10)) and an imposed wall temperature (Dirichlet, Sec. 2.2 and
 *     Eqs. (16)-(17)),
 *   - in a perfect gas with Sutherland viscosity (Sec. 2.1, Eqs. (1)-(4)),
 *   - at a given Reynolds, Mach and Prandtl number,
 *   - advanced by the IBM-HT-sonicFoam step of Appendix A on a uniform
 *     Cartesian finite-volume grid,
 *   - returning the flow, the marker forces (Sec. 3.1, Eq. (18)) and the heat
 *     exchanged with the body.
 *
 * Units are non-dimensional: rho_inf = |U_inf| = D = theta_inf = 1,
 * R = 1/(gamma Ma^2), c_v = R/(gamma-1), mu_inf = 1/Re.
 *
 * Conventions for every entry point:
 *   - Return ibm_status; IBM_OK is 0. No C++ exception crosses the ABI.
 *   - On an argument error (IBM_E_ARG, IBM_E_SIZE) nothing is modified and
 *     ibm_last_error() describes the problem.
 *   - All device work is enqueued on the stream given at creation, in order.
 *     Calls that fill host memory (ibm_step_info, totals) synchronise it.
 *   - Device pointers are HIP device addresses owned by the caller; the library
 *     reads them during the call (stream-ordered) and keeps no reference unless
 *     stated. The library never allocates device memory: all of its buffers are
 *     carved from the caller's workspace.
 *   - Cell arrays are structure-of-arrays, x fastest: index i + n0*(j + n1*k).
 *     Vector fields are stored component after component ([dim][N]).
 *     The face array of direction d has n_d+1 faces along d and n_e cells along
 *     the other directions e (face i_d lies between cells i_d-1 and i_d); the dim
 *     face arrays are concatenated, direction 0 first. In a periodic direction
 *     face n_d is the same face as face 0 and holds the same value.
 *   - Field arrays are double (IBM_FP64) or float (IBM_FP32) as the context's
 *     precision says; marker arrays, forces and heat are always double.
 */
#ifndef IBM_H
#define IBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ibm_ctx ibm_ctx;

typedef enum {
  IBM_OK = 0,
  IBM_E_ARG = 1,           /* invalid argument                                   */
  IBM_E_SIZE = 2,          /* workspace or marker capacity too small             */
  IBM_E_HIP = 3,           /* a HIP runtime call failed                           */
  IBM_E_NOT_CONVERGED = 4, /* a CG solve exceeded its iteration limit             */
  IBM_E_NONFINITE = 5,     /* a step produced NaN/Inf or non-positive rho, theta */
  IBM_E_STATE = 6          /* call out of order (e.g. markers never set)         */
} ibm_status;

/* boundary condition of one side of the box (ghost rules per variable):
 *   PERIODIC  wrap (both sides of a direction must be periodic)
 *   INFLOW    u = U_inf and theta = 1 on the face; rho, p zero gradient;
 *             face mass flux rho_P U_inf (rho at the start of the step)
 *   OUTFLOW   zero gradient; p = p_inf on the face
 *   SLIP      no normal velocity, no normal gradient of anything else
 *   SUPERSONIC_INFLOW   rho = 1, u = U_inf, theta = 1 on the face
 *   SUPERSONIC_OUTFLOW  zero gradient of every variable
 * (the two supersonic sides with IBM_SCHEME_DENSITY only)                      */
enum { IBM_PERIODIC = 0, IBM_INFLOW = 1, IBM_OUTFLOW = 2, IBM_SLIP = 3,
       IBM_SUPERSONIC_INFLOW = 4, IBM_SUPERSONIC_OUTFLOW = 5 };
enum { IBM_FP64 = 0, IBM_FP32 = 1 };
/* convected face values: van Leer limited (Sec. 2.2.2) or linear */
enum { IBM_CONV_VANLEER = 0, IBM_CONV_LINEAR = 1 };
enum { IBM_MU_SUTHERLAND = 0, IBM_MU_CONSTANT = 1 };
/* viscous and conductive fluxes: explicit, or their compact face-normal parts
 * (mu_f du/dn, lambda_f dtheta/dn) implicit by backward Euler: after the explicit
 * predictor, rho* u* - dt div(mu_f grad_n u*) = m*(explicit) per component and
 * rho* theta* - dt (gamma/Pr) div(mu_f grad_n theta*) = E*(explicit)/c_v are
 * solved by conjugate gradients (to cg_rtol, from u^n and theta^n); the time step
 * from cfl then follows convection alone. Not with the adjoint. */
enum { IBM_DIFF_EXPLICIT = 0, IBM_DIFF_IMPLICIT = 1 };
/* The step: pressure-based (App. A; the default) or density-based (App. B): the
 * explicit central-upwind step of Kurganov, Noelle and Petrova for rho, rho u,
 * rho e_t (rho, u, theta reconstructed on both sides of a face, van Leer limited
 * with IBM_CONV_VANLEER, the linear average with IBM_CONV_LINEAR), then the
 * viscous and conductive terms explicitly at the intermediate (u**, theta**),
 * then the marker sources of Sec. 2.2 from that result (m += dt f, rho e +=
 * dt q). Its time step adds the sound speed at dt_theta_max to the flow speed.
 * Explicit diffusion and one pass only; no adjoint (IBM_E_ARG). The stored face
 * mass flux is the step's central-upwind density flux. */
enum { IBM_SCHEME_PRESSURE = 0, IBM_SCHEME_DENSITY = 1 };
/* Outer passes (n_outer > 1): App. A step 3 repeated ("until convergence"). Every
 * pass after the first evaluates the predictor's fluxes and cell terms (and the
 * implicit diffusion's face viscosities) at the latest iterate, keeps the step's
 * start as the time derivative's old values, re-spreads the marker sources formed
 * in the first pass (f and q stay fixed within the step) and solves the pressure
 * equation again from the previous pass's solution. The passes are a fixed-point
 * iteration; converged, the step is implicit in every term. It converges where
 * dt |lambda| < 1 for the stiffest explicit mode: use cfl <= 0.25 (at cfl 0.5 an
 * even pass count amplifies the stiffest conduction mode and is unstable). Not
 * with the adjoint. */
/* ibm_set_markers flags: apply the marker check routine of Sec. 3.1 (of the
 * markers that fall in one cell only the one nearest to its centre is used,
 * ties to the lower id), at set-up and after every motion update. */
#define IBM_DEDUPE 1u
/* ibm_set_markers flags: markers without heat exchange (the energy source q of
 * Eq. (17) is zero; the wall temperatures are not used). Not with the adjoint. */
#define IBM_NO_HEAT 2u
/* ibm_step flags: record each step of the call on the tape for the adjoint */
#define IBM_RECORD 1u

typedef struct {
  int32_t dim;              /* 2 or 3                                          */
  int32_t n[3];             /* cells per direction; n[2] = 1 in 2D, each >= 3  */
  double lo[3], hi[3];      /* box; h_d = (hi_d - lo_d)/n_d                    */
  int32_t bc[3][2];         /* IBM_PERIODIC/INFLOW/OUTFLOW/SLIP, [dir][lo,hi]  */
  int32_t precision;        /* IBM_FP64 or IBM_FP32                            */
  int32_t convection;       /* IBM_CONV_VANLEER or IBM_CONV_LINEAR             */
  int32_t viscosity_law;    /* IBM_MU_SUTHERLAND or IBM_MU_CONSTANT            */
  int32_t diffusion;        /* IBM_DIFF_EXPLICIT or IBM_DIFF_IMPLICIT          */
  double Re, Ma, Pr, gamma; /* flow parameters                                 */
  double sutherland_S;      /* Sutherland temperature over T_inf               */
  double U_inf[3];          /* inflow velocity                                 */
  double dt;                /* > 0: time step; <= 0: computed from cfl         */
  double cfl;               /* fraction of the explicit convection+conduction  */
                            /* limit used when dt <= 0 (of convection alone   */
                            /* with IBM_DIFF_IMPLICIT and a flow speed)        */
  double dt_theta_max;      /* largest temperature expected (for the limit)    */
  double dt_u_max;          /* largest body speed expected (for the limit)     */
  double cg_rtol;           /* pressure CG stops at |r| <= cg_rtol |b|         */
  int32_t cg_maxit;         /* pressure CG iteration limit                     */
  int32_t max_markers;      /* capacity for candidate markers                  */
  int32_t n_outer;          /* passes of App. A step 3 per step (0 or 1: one;  */
                            /* at most 64): the outer passes described above  */
  int32_t scheme;           /* IBM_SCHEME_PRESSURE or IBM_SCHEME_DENSITY       */
} ibm_grid_desc;

typedef struct {
  int64_t steps_done;     /* steps completed by the call                      */
  int64_t step;           /* step counter of the state after the call         */
  int32_t cg_iters_last;  /* CG iterations of the last step                   */
  int32_t cg_iters_total; /* CG iterations summed over the call               */
  double cg_residual;     /* |r|/|b| at the end of the last solve              */
  double dt;              /* time step                                        */
  double time;            /* step * dt                                        */
  double mass;            /* sum of rho dV after the call (FP64 reduction)     */
  int32_t diff_iters_total; /* implicit diffusion CG iterations (of the side-  */
                            /* by-side solves) summed over the call            */
  int32_t reserved;
} ibm_step_info;

/* Bytes of device workspace needed for a grid, a marker capacity and a tape
 * of `tape_steps` recorded steps (0: no adjoint). A tape step holds the state in
 * the context's storage type ((dim + 2) N + sum NF words) and the FP64 pressure (N);
 * tape_steps > 0 also adds the adjoint's work buffers (about (9 dim + 12) N +
 * (4 dim + 3) sum NF doubles, (5 dim + 4) sum NF with van Leer convection).
 * Returns 0 for an invalid descriptor. */
size_t ibm_workspace_bytes(const ibm_grid_desc *desc, int32_t max_markers, int32_t tape_steps);

/* Creates a context on the current HIP device. `dev_workspace` (device memory,
 * at least ibm_workspace_bytes(desc, desc->max_markers, tape_steps) bytes,
 * 256-byte aligned) must stay valid until ibm_destroy; `tape_steps` is the
 * capacity used in that size computation.
 * `hip_stream` (hipStream_t, may be NULL for the null stream) orders all work.
 * The state starts as the uniform stream rho = 1, theta = 1, u = U_inf.
 * Environment, read here: IBM_PREDICTOR=plain selects the per-cell predictor
 * instead of the LDS-tiled one. The pressure solve starts from p^n extrapolated
 * in time: 4 p^n - 6 p^{n-1} + 4 p^{n-2} - p^{n-3} after three steps of this
 * context, 3 p^n - 3 p^{n-1} + p^{n-2} after two, 2 p^n - p^{n-1} after one, p^n
 * otherwise (and after ibm_set_state); IBM_CG_START=quadratic caps the order at the
 * three-point form, IBM_CG_START=linear at the two-point form, IBM_CG_START=plain
 * uses p^n always. Every start converges to the same solution within cg_rtol. An
 * IBM_FP32 context solves for the pressure by iterative refinement (FP64 x and
 * residual around an FP32 inner CG) in 3D and with the FP64 CG on its FP32 psi in
 * 2D; IBM_FP32_SOLVE=refine or IBM_FP32_SOLVE=fp64 selects either. In 3D the FP64
 * CG iterates by z-columns (IBM_CG3D=tile: by tiles). */
ibm_status ibm_create_grid(const ibm_grid_desc *desc, void *dev_workspace, size_t bytes,
                           int32_t tape_steps, void *hip_stream, ibm_ctx **out);

/* For callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): ibm_create_grid with the workspace
 * taken from a fixed array of 64 MiB in the library's device memory, one per GPU, held
 * until the process ends. Nothing is allocated on the device or pinned on the host
 * (the context itself is host memory, and without the pinned progress word ibm_step
 * synchronises to follow the CG). Every other entry point works on the context as on
 * one from ibm_create_grid. At most one such context per GPU is alive at a time: a
 * second one on the same device returns IBM_E_STATE until ibm_destroy releases the
 * first (contexts on one array would overwrite each other's buffers). IBM_E_SIZE when
 * ibm_workspace_bytes(desc, desc->max_markers, tape_steps) exceeds 64 MiB (for
 * example 128^2 and 256^2 FP64 grids with a few hundred markers fit, 1024^2 does not);
 * IBM_E_ARG for an invalid descriptor; IBM_E_HIP when the array's address cannot be
 * found. No error message is kept (there is no context). */
ibm_status ibm_create_grid_noalloc(const ibm_grid_desc *desc, int32_t tape_steps,
                                   void *hip_stream, ibm_ctx **out);

/* Releases the host-side context (the workspace stays with the caller). */
void ibm_destroy(ibm_ctx *ctx);

/* Message of the last error of this context ("" if none). */
const char *ibm_last_error(const ibm_ctx *ctx);

/* Time step in use (given, or computed at creation from cfl). */
double ibm_dt(const ibm_ctx *ctx);

/* Sets the state from primitive fields (device, context precision): rho [N],
 * u [dim][N], theta [N]. Conserved state m = rho u, E = rho c_v theta; face
 * mass flux from the momentum (linear interpolation; boundary faces by their
 * rule). Resets the step counter to 0. */
ibm_status ibm_init_primitive(ibm_ctx *ctx, const void *rho, const void *u, const void *theta);

/* Sets the conserved state (device, context precision): rho [N], mom [dim][N],
 * eint = rho e [N], face_flux [sum_d NF_d] or NULL to derive it from mom.
 * `step` sets the step counter (time = step * dt, which drives marker motion). */
ibm_status ibm_set_state(ibm_ctx *ctx, const void *rho, const void *mom, const void *eint,
                         const void *face_flux, int64_t step);

/* Copies the conserved state out (device, context precision). NULL skips. */
ibm_status ibm_get_state(const ibm_ctx *ctx, void *rho, void *mom, void *eint, void *face_flux);

/* Sets the body (Sec. 2.2): n candidate markers with positions X [n][dim],
 * desired velocities U_d [n][dim] (NULL: at rest), wall temperatures T_w [n]
 * (theta_wall / theta_inf) and surface elements dA [n] (NULL: zero); all device
 * double arrays, copied. With IBM_DEDUPE the check routine of Sec. 3.1 selects
 * the markers in use; with IBM_NO_HEAT the markers exchange no heat. Builds the supports (the 3 nearest cells per direction),
 * sorts the (cell, marker) pairs, and solves A eps = 1 (Eqs. (8)-(9)) in FP64.
 * IBM_E_ARG if a support leaves a non-periodic box; IBM_E_SIZE if n exceeds the
 * capacity; IBM_E_NOT_CONVERGED if the eps solve fails. */
ibm_status ibm_set_markers(ibm_ctx *ctx, int32_t n, const double *X, const double *U_d,
                           const double *T_w, const double *dA, uint32_t flags);

/* Prescribed motion (Sec. 5, Eq. (19)): at time t every candidate marker sits at
 * X(0) + amplitude sin(2 pi frequency t) e_axis and moves with the derivative of
 * that law added to its U_d. Step n -> n+1 uses t = (n+1) dt; the markers are
 * re-selected, re-sorted and eps re-solved on the device every step, each solve
 * starting from the candidates' eps of ibm_set_markers (so the markers at a time do
 * not depend on the steps before). Within an ibm_step call, later steps' markers
 * are set up ahead on two more streams of the context, into two marker sets of the
 * workspace, while the current step runs: the next step's into the set it does not
 * use, the step after that's into its own set once its marker kernels are done, so
 * that two set-ups overlap each other and the steps (a context on a caller's
 * workspace; IBM_REBUILD=inline in the environment at creation keeps them on the
 * context's stream, one per step).
 * axis < 0 switches motion off. */
ibm_status ibm_set_motion(ibm_ctx *ctx, int32_t axis, double amplitude, double frequency);

/* Replaces the wall temperatures (device double [n], candidate order). */
ibm_status ibm_set_wall_temperature(ibm_ctx *ctx, const double *T_w);

/* Advances n_steps steps of Appendix A: predictor with f = q = 0; interpolation
 * (Eq. (5)), forcing (Eqs. (10), (17)) and spreading (Eq. (7)); the pressure
 * equation solved by matrix-free CG; correction of the face mass flux, density,
 * momentum and energy. `hist` (device double [n_steps][4] or NULL) receives per
 * step the force of the fluid on the body (Fx, Fy, Fz) and the heat given to
 * the fluid H. `info` (host, may be NULL) is filled after a synchronisation.
 * IBM_E_NOT_CONVERGED: the CG hit cg_maxit (the state is advanced, the call
 * stops after that step). IBM_E_NONFINITE: the step produced NaN/Inf or a
 * non-positive density or temperature; the state is the one before that step (a
 * moving body's markers in use and wall fluxes are then those of a later step).
 * With IBM_RECORD each step is stored on the tape (IBM_E_SIZE when full). */
ibm_status ibm_step(ibm_ctx *ctx, int32_t n_steps, uint32_t flags, double *hist,
                    ibm_step_info *info);

/* Wall fluxes of the last step (Sec. 3.1): per marker in use the force on the
 * body -dV eps_k F_k (device [n_used][dim], may be NULL) and the heat given to
 * the fluid dV eps_k Q_k (device [n_used], may be NULL); totals (host [4]:
 * Fx, Fy, Fz, H, may be NULL; synchronises). */
ibm_status ibm_wall_fluxes(const ibm_ctx *ctx, double *force, double *heat, double *totals);

/* Local wall heat flux of the last step (Sec. 3.1; the heat flux behind a local
 * Nusselt number): per marker in use q_k = H_k / dA'_k (device double [n_used]),
 * H_k = dV eps_k Q_k the heat the marker gives to the fluid (as ibm_wall_fluxes),
 * dA'_k = dA_k (sum of the candidates' dA) / (sum of the used markers' dA): the
 * surface elements given to ibm_set_markers, scaled so that those of the markers
 * in use cover the whole given surface (the check routine drops candidates, whose
 * surface the kept markers then represent). Synchronises. IBM_E_STATE without
 * markers or when the markers in use carry no surface (dA NULL or zero). */
ibm_status ibm_wall_heat_flux(const ibm_ctx *ctx, double *q);

/* Markers in use: their number (host), candidate ids (device int32 [n_used]) and
 * Lagrangian quadrature eps (device double [n_used]); NULL pointers skip. */
ibm_status ibm_markers_in_use(const ibm_ctx *ctx, int32_t *n_used, int32_t *ids, double *eps);

/* Intermediate fields of the last step, for inspection (device, context
 * precision unless noted): 0 rho* (predictor), 1 mom** [dim][N] and 2 E** (the
 * predictor values with the spread forcing added; equal to the predictor values
 * away from the markers), 3 psi, 4 pressure right-hand side (double), 5 pressure
 * solution (double), 6 per-marker rho_L, M (dim), E_L, F (dim), Q
 * (double [n_used][2 dim + 3]). Synchronises. */
ibm_status ibm_get_field(const ibm_ctx *ctx, int32_t which, void *dst);

/* Discrete adjoint of one step recorded by the last ibm_step(..., IBM_RECORD, ...)
 * call (a hand-written reverse of the whole step: correction, pressure CG (the
 * operator is symmetric, so its adjoint is one more CG solve), set-up, forcing and
 * spreading (spreading transposes to interpolation and back), predictor). Not in
 * the paper: it serves gradients of time-averaged Nusselt number and drag with
 * respect to the wall temperatures. With van Leer convection the limiter and the
 * upwind choice are differentiated where they are smooth: the branch the forward
 * took (by the sign of the face mass flux, and whether the limiter is active)
 * is kept, which is the derivative almost everywhere. Requirements: markers at
 * rest and explicit diffusion (IBM_E_ARG otherwise); IBM_E_STATE if tape_index is
 * not a recorded step.
 * In the FP32 form the forward pieces are recomputed in FP32 from the FP32 record
 * and the reverse runs in FP64 (cotangents, transposed stencils, adjoint CG): the
 * gradient along the FP32 trajectory.
 *   tape_index     0 = first step of the recording call
 *   state_bar_in   device double: cotangent of the state after the step, in the
 *                  ibm_set_state layout (rho [N], mom [dim][N], E [N], F [sum NF])
 *   state_bar_out  device double, same layout: cotangent of the state before the
 *                  step (written; must not overlap state_bar_in)
 *   out_bar        host double [4]: cotangents of the step's outputs Fx, Fy, Fz, H
 *                  (the history row of ibm_step)
 *   Tw_bar         device double [n candidate markers]: the step's contribution to
 *                  the gradient with respect to T_w is added (+=)
 * The context's current state is not changed; the step's own buffers are. The
 * host waits for the adjoint pressure solve; the kernels after it are queued on
 * the stream (state_bar_out and Tw_bar are ready when the stream is). Needs a
 * workspace planned with tape_steps > 0. */
ibm_status ibm_adjoint_step(ibm_ctx *ctx, int32_t tape_index, const double *state_bar_in,
                            double *state_bar_out, const double *out_bar, double *Tw_bar);

/* Number of steps on the tape (recorded by the last IBM_RECORD call). */
int32_t ibm_tape_length(const ibm_ctx *ctx);

/* Gradient with respect to the candidate marker positions (not in the paper:
 * shape sensitivities of the same objective as ibm_adjoint_step). An adjoint
 * step adds, for markers at rest, the cotangents of the step's kernel weights
 * w_ck (Sec. 2.2, Eqs. (5)-(7)) and quadrature weights eps_k (Eqs. (8)-(9)) to an
 * accumulator in the workspace. This call turns the accumulation into dJ/dX:
 * one more solve with the Gram matrix A of Eq. (9) (A lambda = eps_bar, the
 * adjoint of A eps = 1) gives w_bar -= lambda_k (W eps)_c + eps_k (W lambda)_c, and
 * the kernel's derivative gives X_bar. The check routine's choice of markers and
 * the support cells are held fixed (the derivative almost everywhere; candidates
 * not in use get 0).
 *   X_bar   device double [n candidates][dim]: dJ/dX is added (+=); NULL clears
 *           the accumulator and starts the accumulation
 * Adjoint steps add to the accumulator only between a NULL call and the next call
 * with X_bar, which reads it and stops the accumulation (so a reverse pass that wants
 * no position gradient pays nothing for it): start such a reverse pass with a NULL
 * call. Synchronises. IBM_E_STATE without a tape workspace or markers, IBM_E_ARG
 * for moving markers, IBM_E_SIZE above 4096 candidates (X_bar given),
 * IBM_E_NOT_CONVERGED if the Gram solve fails. */
ibm_status ibm_shape_gradient(ibm_ctx *ctx, double *X_bar);

/* Kernel timing for measurement. While enabled, ibm_step records HIP events on
 * the context's stream around the launches of each kernel class and, after each
 * step, adds their durations to per-class totals. Classes (IBM_PROF_*): 0
 * predictor, 1 marker work (motion update, interpolation/forcing, spread), 2
 * pressure set-up (with the CG's start), 3 CG iterations (one event pair around
 * each batch of back-to-back iterations; the launch count is the number of
 * iterations that did work, so total / count is the time per iteration, with the
 * launch that detects convergence included in the total), 4 implicit diffusion
 * (face viscosities and the dim + 1 solves, host waits between them included),
 * 5 correction, 6 a moving body's marker set-up for a later step on one of the
 * context's two further streams (it overlaps the steps; class 1 then holds the
 * set-up only where it is on the context's stream: the first step of a call).
 * The events themselves slow a step down; time throughput with timing off.
 * enable != 0 clears the totals and starts timing; 0 stops it. */
enum { IBM_PROF_PREDICTOR = 0, IBM_PROF_MARKERS = 1, IBM_PROF_SETUP = 2, IBM_PROF_CG = 3,
       IBM_PROF_DIFFUSION = 4, IBM_PROF_CORRECT = 5, IBM_PROF_REBUILD = 6,
       IBM_PROF_CLASSES = 8 };
ibm_status ibm_profile(ibm_ctx *ctx, int32_t enable);

/* Per-class totals since timing was enabled: ms [IBM_PROF_CLASSES] (host) summed
 * durations in milliseconds, launches [IBM_PROF_CLASSES] (host) launch counts. */
ibm_status ibm_profile_read(const ibm_ctx *ctx, double *ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* IBM_H */
