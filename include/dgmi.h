/*
 * dgmi -- nodal discontinuous Galerkin right-hand side, SSP-RK3 step and
 * conservative-to-primitive recovery on one AMD MI355X (gfx950).
 *
 * The library evolves a conservation law in flux-conservative form,
 *     d_t U + d_a F^a(U) = S(U)
 * (the conservation-laws section of Kidder et al., arXiv:1609.00098, with the
 * flat metric: lapse 1, zero shift, Euclidean spatial metric), discretised by
 * the strong-form nodal DG scheme (eq. 411) on a periodic box of affine
 * hexahedra (eq. AffineMap) with the local Lax-Friedrichs flux (eq. LLF).
 *
 * Conventions common to every call
 *   - Systems: DGMI_NEWTONIAN_EULER  U = (rho, rho v_x, rho v_y, rho v_z, E)
 *              DGMI_SR_HYDRO         U = (D, S_x, S_y, S_z, tau)
 *              DGMI_SR_MHD           U = (D, S_x, S_y, S_z, tau, B_x, B_y, B_z, Phi)
 *     with the ideal-gas equation of state p = (gamma - 1) rho eps.
 *   - Primitives: prim[5][n] = (rho, v_x, v_y, v_z, p); for MHD the magnetic
 *     field and Phi are read from U.
 *   - All arrays are structure-of-arrays, A[var * n + point], FP64 unless
 *     stated.  Mesh node order: element e = ex + nx*(ey + ny*ez) owns the
 *     contiguous block [off[e], off[e+1]); inside it node
 *     i + (N+1)*(j + (N+1)*k) with i along x fastest, on the GLL nodes.
 *   - Every pointer argument is device memory owned by the caller unless its
 *     name ends in _host.  The library never frees caller memory.
 *   - Calls are asynchronous on `stream` (a hipStream_t passed as void*;
 *     NULL = the default stream) unless stated.
 *   - Every call returns a dgmi_status; nothing aborts and nothing throws
 *     across the ABI.  Invalid arguments return DGMI_EINVAL before any work is
 *     enqueued; dgmi_last_error() then describes the problem (thread-local).
 */
#ifndef DGMI_H
#define DGMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DGMI_OK = 0,
  DGMI_EINVAL = -1,       /* bad argument; nothing was enqueued */
  DGMI_ENOMEM = -2,       /* device allocation failed */
  DGMI_EHIP = -3,         /* a HIP runtime call failed */
  DGMI_ECON2PRIM = -4,    /* a recovery failed (checked variants only) */
  DGMI_EUNSUPPORTED = -5  /* valid request the library does not implement */
} dgmi_status;

enum { DGMI_NEWTONIAN_EULER = 0, DGMI_SR_HYDRO = 1, DGMI_SR_MHD = 2 };

/* Initial pressure for the recovery's Newton iteration. */
enum {
  DGMI_GUESS_INPUT = 0,   /* prim_inout[4][i] on entry */
  DGMI_GUESS_PLAIN = 1,   /* upper end of the bracket (ignores prim_inout on entry) */
  DGMI_GUESS_LEARNED = 2, /* the pressure-guess MLP (needs an MLP handle) */
  DGMI_GUESS_F0 = 3       /* f(0) = (gamma-1) rho eps at zero pressure, the pressure function's value
                             there (closed form; the bracket's top where it is not positive) */
};

/* dgmi_mesh_desc.flags */
#define DGMI_FLAG_PLAIN_GUESS 1   /* dg_rhs / dg_step: seed recoveries from the bracket, not prim_inout */
#define DGMI_FLAG_RECOVER_FIRST 2 /* dg_step: recompute prims of U^n before the first stage */
#define DGMI_FLAG_NO_GRAPH 4      /* mixed degrees: dg_step launches its kernels directly instead of
                                     replaying a captured graph */
#define DGMI_FLAG_AUTOTUNE 8      /* mixed degrees: dgmi_create times every tile option per degree and
                                     keeps the fastest (results do not depend on the choice) */
#define DGMI_FLAG_HLL 16          /* numerical flux HLL (eq. HLL) instead of local Lax-Friedrichs
                                     (eq. LLF), on uniform and mixed-degree meshes (on a face between
                                     unequal degrees at every mortar node) */
#define DGMI_FLAG_ROE 64          /* numerical flux Roe (eq. Roe, with the Roe averages of eq. RoeAverages)
                                     for the Newtonian ideal gas on uniform degrees; not with another
                                     flux flag (DGMI_EINVAL) nor another system, equation of state or
                                     mixed degrees (DGMI_EUNSUPPORTED) */
#define DGMI_FLAG_MARQUINA 128    /* numerical flux Marquina (Marquina subsection), same conditions */
#define DGMI_FLAG_POLYTROPIC 32   /* Newtonian Euler with the polytropic equation of state p = rho^gamma
                                     (K = 1; the adiabatic one of the isentropic vortex test) instead of
                                     the ideal gas; uniform degrees only.  The energy is still evolved;
                                     the standalone con2prim call stays ideal-gas.  Fixed boundary states
                                     take p = rho^gamma. */

typedef struct dgmi_ctx dgmi_ctx;
typedef struct dgmi_mlp dgmi_mlp;

typedef struct {
  int32_t system;         /* DGMI_NEWTONIAN_EULER, DGMI_SR_HYDRO or DGMI_SR_MHD */
  int32_t nx, ny, nz;     /* elements per direction (>= 1 each); a periodic box unless
                             dgmi_set_boundary / dgmi_set_analytic_boundary say otherwise */
  int32_t degree;         /* 1..7: uniform polynomial degree N (N+1 GLL nodes per
                             direction); 0 (or -1): per-element degrees from degrees_host */
  int32_t flags;          /* DGMI_FLAG_* */
  double gamma;           /* ideal-gas adiabatic index, 1 < gamma <= 2 */
  double kappa;           /* divergence-cleaning damping (MHD source -kappa Phi) */
  double lo[3], hi[3];    /* box corners; every element has size (hi-lo)/n_d */
  const int32_t *degrees_host; /* nx*ny*nz degrees in 1..7 when degree == 0 */
} dgmi_mesh_desc;

/* Build a mesh context: GLL nodes, weights and differentiation matrices
 * (eq. for D^{1bar}), neighbour tables, RK scratch.  The table uploads (and,
 * with DGMI_FLAG_AUTOTUNE, the tile timings) run on `stream`, which is
 * synchronised before the call returns; on failure nothing is left allocated
 * and *out is NULL.  The context is bound to the device current at creation.
 *
 * Mixed degrees (degree == 0, degrees_host[e] in 1..7 for element e): the
 * paper defers the coupling of unequal degrees; a face between degrees Na and
 * Nb carries a mortar with the GLL nodes of degree max(Na, Nb).  The lower
 * side is interpolated there in (rho, W v, p [, B, Phi]), one numerical flux
 * (LLF, or HLL with DGMI_FLAG_HLL) is formed per mortar node, the higher side lifts F*.n - F.n at its nodes and
 * the lower side lifts P (F*.n - I F_h.n), P(i,m) = w_m l_i(x_m) / w_i, with
 * I F_h the interpolant of its own nodal fluxes.  dg_step on a non-default
 * stream captures its three stages once per (U, prim_inout) pair and then
 * replays the graph (dt travels in a device scalar); the per-degree kernels
 * run concurrently on the context's own streams.                          */
dgmi_status dgmi_create(const dgmi_mesh_desc *desc, void *stream, dgmi_ctx **out);
dgmi_status dgmi_destroy(dgmi_ctx *ctx);

int64_t dgmi_num_nodes(const dgmi_ctx *ctx);    /* sum over elements of (N_e+1)^3 */
int32_t dgmi_num_vars(const dgmi_ctx *ctx);     /* 5 or 9 */
int64_t dgmi_num_elements(const dgmi_ctx *ctx);
/* Mixed degrees: how the element kernels run, as DGMI_FLAG_AUTOTUNE chose
 * (or the defaults without it): 1 = every degree in one launch, 0 = one
 * launch per degree on the context's streams; -1 for a uniform mesh or a
 * NULL context.  epb_out (int32[8], nullable): elements per workgroup of the
 * per-degree launches, by degree (0 where no element has that degree). */
int32_t dgmi_mixed_launch_mode(const dgmi_ctx *ctx, int32_t *epb_out);
/* off_host[nelem+1]: first node of every element (host copy). */
dgmi_status dgmi_elem_offsets(const dgmi_ctx *ctx, int64_t *off_host);
/* The same nelem+1 offsets as a host array owned by the context (valid until
 * dgmi_destroy; do not free); NULL, with the last error set, for a NULL
 * context. */
const int64_t *dgmi_elem_offsets_host(const dgmi_ctx *ctx);

/* xyz[3][nnodes]: physical coordinates of every node through the affine map
 * x = a + (1 + xbar)(b - a)/2 (eq. AffineMap). */
dgmi_status dgmi_node_coords(const dgmi_ctx *ctx, double *xyz, void *stream);

/* U[nv][n] from prim[5][n] (and mag[4][n] = (B_x, B_y, B_z, Phi) for MHD;
 * ignored otherwise): the definitions of the evolved variables of the
 * conservation-laws section (eq. evolved for MHD). */
dgmi_status dgmi_prim2cons(int32_t system, double gamma, const double *prim, const double *mag, double *U,
                           int64_t n, void *stream);

/* Semi-discrete operator dUdt = L(U) of eq. 411:
 *   L = S - sum_d (2/dx_d) D^(d) F^d - sum_faces (2/dx_d)(1/w_end)(F*.n - F.n),
 * F*.n the LLF flux (HLL with DGMI_FLAG_HLL) with the unit outward normal;
 * across a box face with a fixed exterior state (dgmi_set_boundary) or an
 * analytic one (dgmi_set_analytic_boundary) the exterior is that state.  First recovers the
 * primitives of every node (Newton polished to rounding level, seeded from
 * prim_inout's pressure unless DGMI_FLAG_PLAIN_GUESS), which are written
 * back to prim_inout.  Failed recoveries are counted (dgmi_failures).
 * U[nv][nnodes], prim_inout[5][nnodes], dUdt[nv][nnodes]; dUdt must not
 * alias U or prim_inout. */
dgmi_status dg_rhs(dgmi_ctx *ctx, const double *U, double *prim_inout, double *dUdt, void *stream);

/* The operator alone, for callers that already hold the primitives of U:
 * dUdt = L(U) of eq. 411 with prim[5][nnodes] taken as given (dg_rhs is
 * con2prim followed by this call).  dUdt must not alias U or prim. */
dgmi_status dg_operator(dgmi_ctx *ctx, const double *U, const double *prim, double *dUdt, void *stream);

/* One third-order SSP Runge-Kutta step in place (the RK3-SSP time stepper of
 * the section on initial data, boundary conditions and time steppers), in
 * Shu-Osher form:
 *   U1 = U + dt L(U); U2 = 3/4 U + 1/4 (U1 + dt L(U1));
 *   U <- 1/3 U + 2/3 (U2 + dt L(U2)).
 * prim_inout must hold the primitives of U on entry (or set
 * DGMI_FLAG_RECOVER_FIRST); on exit it holds those of the new U.  Each stage
 * is one kernel that also recovers the primitives of its output.  With a
 * slope limiter set (dgmi_set_limiter), every stage result is limited
 * (as dg_limit does) before its primitives are final.  Advances the
 * context's time by dt. */
dgmi_status dg_step(dgmi_ctx *ctx, double *U, double *prim_inout, double dt, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dg_step
 * with the stage states U^(1), U^(2) and their primitives held in the
 * library's statically allocated device scratch (one 64 MiB array per device,
 * held until the process ends) instead of the context's buffers.  The call
 * allocates nothing; mixed-degree meshes launch their kernels directly (no
 * graph capture).  Results equal dg_step's bit for bit.  Capacity:
 * 2 (nv + 5) nnodes <= 8 Mi doubles (419,430 nodes for NE / SR, 299,593
 * for SRMHD); a larger mesh returns DGMI_EINVAL before any work.  Every call
 * on a device shares its one scratch array, so calls that overlap on one
 * device (on different streams or host threads) race; the context's device
 * must be current (else DGMI_EINVAL). */
dgmi_status dg_step_noalloc(dgmi_ctx *ctx, double *U, double *prim_inout, double dt, void *stream);

/* Checked variants: the same work as dg_rhs / dg_step, then `stream` is
 * synchronised and DGMI_ECON2PRIM is returned if any recovery of this call
 * failed (an unphysical state, or no convergence within the iteration cap;
 * the outputs are still written, failed nodes holding the last iterate).
 * n_failed_host (nullable, host) receives this call's number of failures.
 * The context's failure counter (dgmi_failures) still counts them.  Both
 * synchronise `stream` before and after the work. */
dgmi_status dg_rhs_checked(dgmi_ctx *ctx, const double *U, double *prim_inout, double *dUdt, int64_t *n_failed_host,
                           void *stream);
dgmi_status dg_step_checked(dgmi_ctx *ctx, double *U, double *prim_inout, double dt, int64_t *n_failed_host,
                            void *stream);

/* Box faces with a fixed exterior state (the analytic boundary condition of
 * the section on initial data, boundary conditions and time steppers, for a
 * solution that is constant outside the box; uniform meshes only, mixed
 * degrees return DGMI_EUNSUPPORTED).  direction 0..2 (x, y, z);
 * state_lo_host / state_hi_host (host memory, copied) are the exterior
 * primitives (rho, v_x, v_y, v_z, p) beyond the lower / upper box face, for
 * SRMHD followed by (B_x, B_y, B_z, Phi); both NULL restores periodicity.
 * States must be physical (rho, p > 0; |v| < 1 for the relativistic
 * systems), else DGMI_EINVAL.  Synchronous; affects later dg_rhs, dg_operator,
 * dg_step and dg_limit calls. */
dgmi_status dgmi_set_boundary(dgmi_ctx *ctx, int32_t direction, const double *state_lo_host,
                              const double *state_hi_host);

/* Analytic solutions available as exterior states (uniform meshes). */
enum {
  DGMI_SOLUTION_ISENTROPIC_VORTEX = 1 /* eq. isen_vortex, Newtonian Euler; params: beta, X0, Y0, U, V, W
                                         (gamma from the mesh, p = rho^gamma) */
};

/* Box faces of `direction` (0..2) take the analytic solution as their
 * exterior state (the analytic boundary condition of the section on initial
 * data, boundary conditions and time steppers): before every operator
 * evaluation the solution is evaluated at each boundary face node at the
 * operator's time (the context's time for dg_rhs / dg_operator; t, t + dt,
 * t + dt/2 for the three stages of dg_step).  params_host: nparams (6)
 * doubles, copied.  Newtonian Euler on uniform meshes only, and not with the
 * slope limiter (DGMI_EUNSUPPORTED); synchronous. */
dgmi_status dgmi_set_analytic_boundary(dgmi_ctx *ctx, int32_t direction, int32_t solution, const double *params_host,
                                       int32_t nparams);

/* Time of the state held by the caller (0 at creation; dg_step advances it
 * by dt).  Only analytic boundary states depend on it. */
dgmi_status dgmi_set_time(dgmi_ctx *ctx, double t);
dgmi_status dgmi_get_time(const dgmi_ctx *ctx, double *t_host);

/* Minmod-family slope limiter (high-resolution shock-capturing section,
 * eqs. MinModSol, MinModB and MinMod), uniform meshes only. */
enum {
  DGMI_LIMITER_NONE = 0,
  DGMI_LIMITER_MINMOD = 1, /* neighbour slope estimates with beta = 2 */
  DGMI_LIMITER_MUSCL = 2   /* beta = 1 */
};

/* Select the limiter used by dg_step (after every stage) and dg_limit; M is
 * the minmodB constant (>= 0; 0 gives plain minmod).  Per conserved component
 * of each element: degree 1 limits when a neighbour estimate changes the
 * slope; degree >= 2 limits when the face means fail the generalized
 * troubled-cell test; a limited component becomes mean + limited slopes
 * (the linear part keeps the Legendre modes 1, x, y, z).  Elements holding a
 * node whose primitives cannot be recovered are limited in every
 * component.  Allocates 80 nv bytes per element of device scratch on first
 * use; DGMI_EUNSUPPORTED with analytic boundaries (the limiter's exterior
 * means need fixed states).  On mixed-degree meshes every element is limited
 * with its own degree (its moments, the degree-1 slope test or the
 * troubled-cell test from degree 2, its rewritten nodes) against its
 * neighbours' means, after every RK3 stage and AB3 step. */
dgmi_status dgmi_set_limiter(dgmi_ctx *ctx, int32_t kind, double M);

/* Limit U in place with the selected limiter (DGMI_EINVAL if none).
 * prim_inout: on entry its pressure seeds the recovery of every node; on exit
 * it holds the primitives of the limited U.  Limited element components are
 * counted (dgmi_limited); failed recoveries after limiting are counted
 * (dgmi_failures). */
dgmi_status dg_limit(dgmi_ctx *ctx, double *U, double *prim_inout, void *stream);

/* Number of limited element components since the last call (synchronises
 * `stream`, then resets the counter). */
dgmi_status dgmi_limited(dgmi_ctx *ctx, int64_t *n_limited_host, void *stream);

/* Number of failed recoveries since the last call (synchronises `stream`,
 * then resets the counter).  With a limiter selected, a state is counted
 * after limiting (and fixing): nodes whose recovery fails before the limiter
 * pass are recovered again by it and count only if they still fail. */
dgmi_status dgmi_failures(dgmi_ctx *ctx, int64_t *n_failed_host, void *stream);

/* Atmosphere floors and conserved-variable fixing (relativistic systems;
 * section on the treatment of unphysical conservative variables), read as:
 * D >= D_min; tau_f >= tau_min with tau_f = tau (hydro) or tau - B^2/2
 * (MHD); then the momentum held one part in 1e12 below the largest value for
 * which primitives exist: S^2 <= (1 - 1e-12) tau (tau + 2D) for hydro; for
 * MHD, S scaled along itself to 1 / (1 + 5e-13) of the largest scale at
 * which the pressure function is defined and positive at p = 0 (found by
 * bisection).  Only D, S and tau change; a state meeting every bound is left
 * bit for bit.  A state whose margin 1e-12 S_max^2 is below rounding
 * relative to (tau + D)^2 (very cold, slow flow) can stay unrecoverable.
 *
 * dgmi_set_fixing switches it on for dg_step / dg_limit (both floors > 0;
 * both 0 switches it off; DGMI_EINVAL for Newtonian Euler or other values):
 * after limiting, every node of an element with a limited component is
 * fixed before its primitives are recovered.  The paper limits unphysical
 * cells first; an element holding an unrecoverable node is limited in every
 * component, so fixing acts only where a limiter is selected. */
dgmi_status dgmi_set_fixing(dgmi_ctx *ctx, double D_min, double tau_min);

/* Number of nodes changed by the fixing since the last call (synchronises
 * `stream`, then resets the counter). */
dgmi_status dgmi_fixed(dgmi_ctx *ctx, int64_t *n_fixed_host, void *stream);

/* Pointwise fixing, as above, of n conserved states U (device, SoA: nv rows
 * of n doubles; system DGMI_SR_HYDRO or DGMI_SR_MHD) in place.  n_fixed:
 * optional device int64 to which the number of changed states is added.
 * DGMI_EINVAL for another system, gamma outside (1, 2], floors not finite
 * and > 0, or host pointers. */
dgmi_status dgmi_fix_conserved(int32_t system, double gamma, double D_min, double tau_min, double *U, int64_t n,
                               int64_t *n_fixed, void *stream);

/* Largest characteristic speed of U (section on initial data, boundary
 * conditions and time steppers: the lambda_max of the CFL scaling) over
 * every node, direction and component, written to the device double
 * *lambda_device: |v_d| + c_s (NE), the larger modulus of the acoustic pair
 * (SR), and 1 for SRMHD (its normal field and cleaning scalar move at the
 * light speed).  prim: primitives of U (NE ignores them; SR reads p).
 * Asynchronous; the result is a device value (no host synchronisation). */
dgmi_status dgmi_max_speed(dgmi_ctx *ctx, const double *U, const double *prim, double *lambda_device, void *stream);

/* dt = cfl * dx_min / lambda_max into the device double *dt_device, dx_min the
 * smallest distance between neighbouring GLL nodes on the physical grid
 * (over the degrees present), lambda_max as dgmi_max_speed.  cfl > 0. */
dgmi_status dgmi_stable_dt(dgmi_ctx *ctx, const double *U, const double *prim, double cfl, double *dt_device,
                           void *stream);

/* One step of the third-order Adams-Bashforth method (section on initial
 * data, boundary conditions and time steppers) in place:
 *   U <- U + dt (23/12 L^n - 16/12 L^{n-1} + 5/12 L^{n-2}),  L^k = L(U^k) at t_k,
 * one operator evaluation per step.  The context keeps the last three
 * operator values (24 nv bytes per node, allocated on first use); the first
 * two calls with a given dt are SSP-RK3 steps (dg_step) that start the
 * history, and a call with another dt starts it again.  prim_inout as for
 * dg_step (on exit the primitives of the new U; failures counted); with a
 * slope limiter the new U is limited.  Advances the context's time by dt.
 * Mixed-degree meshes: the operator is their mortar and element pass, the
 * starting steps their RK3 steps. */
dgmi_status dg_step_ab3(dgmi_ctx *ctx, double *U, double *prim_inout, double dt, void *stream);

/* Pointwise recovery of the primitives (conservation-laws section; the
 * relativistic systems solve f(p) = (gamma-1) rho eps(p) - p = 0 by a
 * bracketed Newton iteration on [0, p_hi], p_hi = (gamma-1) tau, or
 * (gamma-1)(tau - B^2/2) for MHD).
 *   U[nv][n] in, prim_inout[5][n] in (pressure guess for DGMI_GUESS_INPUT)
 *   and out.  tol > 0: stop once the backward residual
 *   max(|dD|/D, |dS|_inf/E, |dtau|/E) of the returned primitives is <= tol
 *   (E = tau + D); tol <= 0: polish to rounding level.
 *   iters_out (uint8[n], nullable): pressure-function evaluations used
 *   (the learned and f(0) seeds count their evaluation of f(0));
 *   fail_out (uint8[n], nullable): 1 where no physical state was found
 *   (prims then hold the last iterate); n_failed (device int64, nullable):
 *   incremented by the number of failures.
 *   mlp: trained network for DGMI_GUESS_LEARNED (SR_MHD and SR_HYDRO). */
dgmi_status con2prim(int32_t system, double gamma, const double *U, double *prim_inout, int64_t n, int32_t guess,
                     const dgmi_mlp *mlp, double tol, uint8_t *iters_out, uint8_t *fail_out, int64_t *n_failed,
                     void *stream);

/* Checked recovery: as con2prim, with n_failed (device int64) required; it
 * is set to this call's number of failures, `stream` is synchronised, the
 * count is copied to n_failed_host (nullable, host) and DGMI_ECON2PRIM is
 * returned if it is not zero (the outputs are written either way). */
dgmi_status con2prim_checked(int32_t system, double gamma, const double *U, double *prim_inout, int64_t n,
                             int32_t guess, const dgmi_mlp *mlp, double tol, uint8_t *iters_out, uint8_t *fail_out,
                             int64_t *n_failed, int64_t *n_failed_host, void *stream);

/* ---------------------------------------------------------------------
 * Learned pressure guess: a 5 -> 64 -> 64 -> 1 multilayer perceptron with
 * SiLU activations in FP32 that proposes the recovery's initial pressure
 * (p0 = D exp(y), y the predicted ln(p/D)).  The FP64 bracketed Newton
 * iteration still decides every result.  Inputs are the raw features
 *   x = [ln(tau/D), ln(1 + |S|/D), ln(1 + B^2/D), S.B/(|S||B| + tiny), ln(f(0)/D)]
 * with f the recovery's pressure function (f(0) = (gamma-1) rho eps at zero
 * pressure, the thermal energy left after the kinetic and magnetic parts),
 * in x[5][batch] (float32, device), normalised inside the library with the
 * stored feature means/deviations; targets t[batch] are raw ln(p/D).
 * Parameter vector: 4609 weights W1[64][5] b1[64] W2[64][64] b2[64] W3[64] b3
 * followed by mu[5] sd[5] ymu ysd (4621 floats).
 * ------------------------------------------------------------------- */

/* New network with weights drawn U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from a
 * generator seeded by `seed`; identity normalisation.  The upload runs on
 * `stream`, which is synchronised before the call returns. */
dgmi_status mlp_create(dgmi_mlp **out, uint64_t seed, void *stream);
dgmi_status mlp_destroy(dgmi_mlp *mlp);
/* Copy the 4621-float parameter vector out of / into the network
 * (device to device); mlp_set also resets the optimiser state. */
dgmi_status mlp_get(const dgmi_mlp *mlp, float *params_out, void *stream);
dgmi_status mlp_set(dgmi_mlp *mlp, const float *params_in, void *stream);
/* x_out[5][n] raw features of conserved states U[nv][n] (SR_HYDRO or SR_MHD);
 * when prim[5][n] is given, t_out[n] (nullable) receives the training target
 * ln(p/D). */
dgmi_status mlp_features(int32_t system, double gamma, const double *U, const double *prim, int64_t n, float *x_out,
                         float *t_out, void *stream);
/* Feature matrices are read as x[i * ldx + s] (ldx >= the sample count), so
 * a minibatch is a column slice of a larger [5][ldx] array. */
/* Store the means and standard deviations of x[5][n] and t[n] as the
 * network's normalisation (FP64 accumulation). */
dgmi_status mlp_fit_normalization(dgmi_mlp *mlp, const float *x, int64_t ldx, const float *t, int64_t n, void *stream);
/* y_out[batch]: predicted ln(p/D) for raw features x. */
dgmi_status mlp_forward(const dgmi_mlp *mlp, const float *x, int64_t ldx, int64_t batch, float *y_out, void *stream);
/* Gradient of L = mean over the batch of (y_n - t_n)^2 (normalised units)
 * with respect to the 4609 weights, into grads_out[4609]; loss_out[1]
 * (nullable) receives L.  Deterministic (fixed-order reductions). */
dgmi_status mlp_grad(dgmi_mlp *mlp, const float *x, int64_t ldx, const float *t, int64_t batch, float *grads_out,
                     float *loss_out, void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on that
 * gradient. */
dgmi_status mlp_train_step(dgmi_mlp *mlp, const float *x, int64_t ldx, const float *t, int64_t batch, float lr,
                           float *loss_out, void *stream);
/* Whole training run over x[5][n], t[n]: `epochs` passes of n/batch
 * consecutive minibatches, learning rate cosine-decayed from lr0 to lr1;
 * loss_hist (nullable) receives every step's loss
 * (epochs * (n/batch) floats, device). */
dgmi_status mlp_train(dgmi_mlp *mlp, const float *x, const float *t, int64_t n, int64_t batch, int32_t epochs,
                      float lr0, float lr1, float *loss_hist, void *stream);

const char *dgmi_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
