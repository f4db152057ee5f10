/*
 * dg2p -- explicit DG residual of the quasi-conservative five-equation
 * two-phase model with Allen-Cahn interface terms, on one MI355X (gfx950).
 *
 * Method: Tonicello & Ihme, "A high-order diffused-interface approach for
 * two-phase compressible flow simulations using a Discontinuous Galerkin
 * framework" (arXiv 2306.05002).  The system solved is the one of Section
 * "Five equation model" (phase field phi_1 = alpha with the Allen-Cahn flux
 * a_1 = Gamma (eps grad alpha - alpha (1 - alpha) n), n = grad psi/|grad psi|
 * from the extra level set psi; partial densities with R_l = rho_l^(0) a_l;
 * momentum and energy with f = sum_l R_l, viscous stress, CSF surface
 * tension and gravity; stiffened-gas closure with the mixture rules), in the
 * DG form of Section "Discontinuous Galerkin discretisation": nodal GLL
 * collocation, Lax-Friedrichs fluxes for the convective terms, symmetric
 * interior penalty for every a_l-built flux, and the hat/tilde face fluxes
 * of the quasi-conservative transport of alpha and psi.
 *
 * Layouts (all arrays FP64 unless stated):
 *   element index  e = e_x + N_x (e_y + N_y e_z)   (x fastest)
 *   node index     j = a_x + 4 (a_y + 4 a_z)       (p = 3: 4 GLL nodes per axis)
 *   state          U[f][e][j], f = 0: alpha_1 rho_1, 1: alpha_2 rho_2,
 *                  2..d+1: rho u, d+2: rho E, d+3: alpha, d+4: psi
 *                  (N_f = d + 5 fields)
 *   primitives     P[f][e][j], f = 0: alpha, 1: psi, 2: rho_1, 3: rho_2,
 *                  4..d+3: u, d+4: pressure
 *
 * Conventions
 *   - Pointers marked "device" are device memory owned by the caller; the
 *     library keeps no pointer beyond a call.  Pointers marked "host" are
 *     host memory.  `stream` is a hipStream_t passed as void* (NULL = the
 *     default stream); every device call is stream-ordered and asynchronous.
 *   - The library allocates no device memory: every call that needs scratch
 *     space takes a caller-owned workspace of dg2p_workspace_size() bytes,
 *     256-byte aligned.  A mesh and a workspace must not be used by two
 *     overlapping calls.
 *   - Every function returns a dg2p_status.  Argument errors are reported
 *     synchronously and nothing is launched; dg2p_last_error() gives the
 *     detail (thread-local).  Non-physical states are never fatal inside a
 *     call: they are counted in dg2p_monitors.nonphys.
 *   - The two-phase model is implemented at polynomial order p = 3, and at
 *     p = 4 on quadrilaterals (FP64; no mixed forms, adjoint or kinematic
 *     mode: the paper's order for its wall-bounded runs); the kinematic mode
 *     (dg2p_kin_*, re-initialisation excepted) at p = 3 and p = 1
 *     (DG2P_EUNSUPPORTED else).  Nodes per element n = (p+1)^d, node
 *     j = sum_k a_k (p+1)^k; the layouts below write 4^d for p = 3.
 */
#ifndef DG2P_H
#define DG2P_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg2p_mesh_s* dg2p_mesh; /* opaque, owned by the library */

typedef enum {
  DG2P_OK = 0,
  DG2P_EINVAL = -1,       /* bad argument (null pointer, size, enum value) */
  DG2P_EHIP = -2,         /* a HIP runtime call failed (launch, copy) */
  DG2P_ENONPHYS = -3,     /* reserved for callers: non-physical state seen */
  DG2P_EUNSUPPORTED = -4, /* valid request the library does not implement */
  DG2P_EWORKSPACE = -5    /* workspace missing or misaligned */
} dg2p_status;

typedef enum {
  DG2P_BC_PERIODIC = 0,   /* wrap to the opposite side (both sides of an axis) */
  DG2P_BC_SLIP_WALL = 1,  /* mirror: normal momentum and normal gradients negated */
  DG2P_BC_DIRICHLET = 2,  /* prescribed (q1, q2, rho u, rho E, alpha); interior psi
                             and gradients */
  DG2P_BC_EXTRAPOLATE = 3, /* ghost = interior (state and gradients) */
  DG2P_BC_NO_SLIP = 4,     /* wall with zero velocity: whole momentum negated,
                              normal gradients of alpha and psi negated, the
                              velocity gradient (wall shear) kept */
  DG2P_BC_RIEMANN = 5      /* Riemann-invariant far field with zero velocity
                              and pressure bc_state[0] (Section "Rayleigh-Taylor
                              instability", top boundary): outgoing invariant
                              u.n + 2 xi c from the interior, incoming -2 xi c_far
                              from (u = 0, P = bc_state[0], interior density);
                              interior partial densities, tangential velocity,
                              alpha, psi and gradients */
} dg2p_bc;

typedef enum {
  DG2P_FP64 = 0,       /* every operation in FP64 */
  DG2P_MIXED_FP32 = 1, /* derivative and lift contractions in FP32 with FP32
                          accumulation; closure, mixture sums, fluxes and the
                          RK accumulation in FP64 */
  DG2P_MIXED_BF16 = 2  /* as FP32 but contraction inputs rounded to BF16 */
} dg2p_precision;

typedef enum {
  DG2P_OP_RHS = 0,
  DG2P_OP_RK_STEP = 1,
  DG2P_OP_MAX_DT = 2,
  DG2P_OP_MONITORS = 3,
  DG2P_OP_RHS_VJP = 4,
  DG2P_OP_RK_STEP_VJP = 5,
  DG2P_OP_ADVANCE = 6,
  DG2P_OP_KIN_RHS = 7,   /* kinematic mode (dg2p_kin_workspace_size) */
  DG2P_OP_KIN_RK4 = 8,
  DG2P_OP_KIN_AUX = 9    /* dg2p_kin_max_dt, dg2p_kin_errors */
} dg2p_op;

/* Structured Cartesian grid of dim-dimensional tensor-product elements
 * (the partition of the domain into elements, Section "Discontinuous
 * Galerkin discretisation").  Entries beyond `dim` are ignored. */
typedef struct {
  int dim;                   /* 1, 2 or 3 */
  int order;                 /* polynomial degree p: 3; 4 on quadrilaterals (FP64 two-phase path);
                                1 (kinematic mode only) */
  int n_elem[3];             /* elements per axis, >= 1 */
  double lo[3], hi[3];       /* box corners, hi > lo */
  int bc[3][2];              /* dg2p_bc per axis and side (0 = low, 1 = high) */
  double bc_state[3][2][8];  /* per side: Dirichlet conserved state (first d+4
                                entries: q1, q2, rho u, rho E, alpha); Riemann
                                far-field pressure in entry 0 (must be > 0) */
} dg2p_mesh_desc;

/* Physical and numerical parameters (Section "Five equation model"). */
typedef struct {
  double gamma[2], pinf[2];  /* stiffened-gas gamma_l > 1, P_inf_l */
  double rho0[2];            /* reference densities rho_l^(0) of R_l = rho_l^(0) a_l */
  double Gamma, eps;         /* Allen-Cahn velocity scale and thickness */
  double mu[2];              /* phase viscosities; both 0 disables viscous terms */
  double sigma;              /* surface tension; 0 disables CSF */
  double g[3];               /* gravity */
  double c_ip;               /* interior-penalty constant (eta = c_ip nu (p+1)^2/h) */
  double grad_reg;           /* delta of n = g/sqrt(g.g + delta^2) (e.g. 1e-12) */
  int precision;             /* dg2p_precision */
} dg2p_params;

/* Step monitors (device struct written by dg2p_compute_monitors / dg2p_max_dt). */
typedef struct {
  double max_rate;     /* max_nodes(sum|u_k| + d c)/h_min + (p+1)^2 d nu_max/h_min^2 */
  double dt;           /* cfl / max_rate (written by dg2p_max_dt) */
  double min_alpha, max_alpha;
  double integral[8];  /* sum_j W_j U[f][e][j] per field (diagonal GLL mass) */
  double dev_p, dev_u; /* max |P - p_ref|, max_k |u_k - u_ref_k| */
  long long nonphys;   /* nodes with rho <= 0, xi rho <= 0, (1+xi)P + Pi <= 0 or non-finite */
} dg2p_monitors;

/* Version string of the library. */
const char* dg2p_version(void);

/* Human-readable name of a status code. */
const char* dg2p_status_string(int status);

/* Detail of the last error of the calling thread ("" if none). */
const char* dg2p_last_error(void);

/* Create a mesh handle from a host descriptor.  Validates the descriptor
 * (EINVAL, also for 2^31 or more elements, or more than 2^40 nodes), rejects
 * orders other than 3, 1 and 4, and 4 outside quadrilaterals (EUNSUPPORTED;
 * what each order runs is stated at the top).  Host only, allocates no device
 * memory.  *out is owned by the caller until dg2p_destroy_mesh. */
int dg2p_create_mesh(const dg2p_mesh_desc* desc /*host*/, dg2p_mesh* out /*host*/);

/* Release a mesh handle (NULL is accepted). */
int dg2p_destroy_mesh(dg2p_mesh m);

/* Field count N_f = d + 5, element count E and nodes per element n = (p+1)^d (host outputs). */
int dg2p_layout(dg2p_mesh m, int* n_fields, long long* n_elem, int* nodes_per_elem);

/* Physical GLL node coordinates, host array xyz[d][E][n] (caller-owned). */
int dg2p_node_coords(dg2p_mesh m, double* xyz /*host*/);

/* Diagonal mass-matrix weights W_j = prod_k w_{a_k} J_k of the n nodes of
 * an element (identical for every element), host array W[n]. */
int dg2p_node_weights(dg2p_mesh m, double* W /*host*/);

/* Bytes of device workspace that `op` needs for this mesh and parameters. */
int dg2p_workspace_size(dg2p_mesh m, const dg2p_params* p /*host*/, int op, size_t* bytes /*host*/);

/* Initial-condition map (the stiffened-gas law solved for rho e):
 * U = (alpha rho_1, (1-alpha) rho_2, rho u, xi P + Pi + rho |u|^2/2, alpha, psi).
 * prim, U: device arrays [N_f][E][4^d] (layouts above); may not alias. */
int dg2p_prim_to_cons(dg2p_mesh m, const dg2p_params* p /*host*/, const double* prim /*device*/,
                      double* U /*device*/, void* stream);

/* Reverse of dg2p_prim_to_cons: prim_bar = (dU/dprim)^T U_bar, all primitive
 * fields (alpha, psi, rho_1, rho_2, u, P), overwritten.  Device arrays
 * [N_f][E][4^d], no aliasing. */
int dg2p_prim_to_cons_vjp(dg2p_mesh m, const dg2p_params* p /*host*/, const double* prim /*device*/,
                          const double* U_bar /*device*/, double* prim_bar /*device, out*/, void* stream);

/* Semi-discrete residual R = dU/dt (mass matrix already inverted): volume
 * terms in strong form (equal to the paper's weak form under GLL
 * collocation), Lax-Friedrichs / SIPG / hat-tilde face terms, IIPG viscous
 * stresses, CSF and gravity sources.  U, R: device [N_f][E][4^d], no alias.
 * work: device, dg2p_workspace_size(DG2P_OP_RHS) bytes. */
int dg2p_rhs(dg2p_mesh m, const dg2p_params* p /*host*/, const double* U /*device*/,
             double* R /*device*/, void* work /*device*/, void* stream);

/* Time step dt = cfl / max_rate (rule above, recomputed from U) written to
 * the device scalar *dt; if mon != NULL also mon->max_rate and mon->dt.  A
 * node whose closure fails (NaN sound speed) makes max_rate and dt NaN.
 * work: dg2p_workspace_size(DG2P_OP_MAX_DT) bytes. */
int dg2p_max_dt(dg2p_mesh m, const dg2p_params* p /*host*/, const double* U /*device*/,
                double cfl, double* dt /*device*/, dg2p_monitors* mon /*device, nullable*/,
                void* work /*device*/, void* stream);

/* One Shu-Osher SSP-RK3 step in place, FP64 stage accumulation:
 * U1 = U + dt R(U); U2 = 3/4 U + 1/4 (U1 + dt R(U1)); U <- 1/3 U + 2/3 (U2 + dt R(U2)).
 * dt: device scalar (no host synchronisation).  work: DG2P_OP_RK_STEP bytes. */
int dg2p_rk_step(dg2p_mesh m, const dg2p_params* p /*host*/, double* U /*device, in/out*/,
                 const double* dt /*device*/, void* work /*device*/, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the step of
 * dg2p_rk_step (same kernels, bitwise the same result) with its workspace in
 * a static device array of the library instead of a caller workspace.  That
 * array holds dg2p_noalloc_scratch_bytes() = 64 MiB on every GPU the library
 * runs on, from the first call on that device until the process ends.  The
 * call allocates nothing and calls no hipMalloc / hipFree; meshes whose
 * DG2P_OP_RK_STEP workspace (dg2p_workspace_size) exceeds the array are
 * rejected with DG2P_EWORKSPACE before anything is launched (e.g. the 2D
 * 128 x 128 grid fits: 34 MiB inviscid, 43 MiB viscous).  The calling
 * thread's current device must be the one `stream` belongs to.  Every call on
 * a GPU shares that GPU's array: calls that overlap on one GPU (two streams,
 * two threads) race and give wrong results; calls in stream order are safe.
 * Nothing is carried between calls (every value a call reads from the array,
 * it wrote first).  U, dt: as for dg2p_rk_step. */
int dg2p_rk_step_noalloc(dg2p_mesh m, const dg2p_params* p /*host*/, double* U /*device, in/out*/,
                         const double* dt /*device*/, void* stream);

/* Size in bytes of the static device scratch of dg2p_rk_step_noalloc. */
size_t dg2p_noalloc_scratch_bytes(void);

/* Advance U in place by n_steps SSP-RK3 steps without host synchronisation.
 * Each step's dt is cfl / max_rate of the step's initial state (the rule of
 * dg2p_max_dt), reduced on the device, or *dt_fixed when dt_fixed != NULL
 * (device scalar; a frozen schedule).  Optional device outputs: *t is
 * incremented by every dt taken, *dt_last receives the last dt, *mon the
 * monitors of the final state (p_ref, u_ref as in dg2p_compute_monitors).
 * Produces the same states as n_steps calls of dg2p_rk_step with those dt.
 * work: dg2p_workspace_size(DG2P_OP_ADVANCE) bytes. */
int dg2p_advance(dg2p_mesh m, const dg2p_params* p /*host*/, double* U /*device, in/out*/, int n_steps,
                 double cfl, const double* dt_fixed /*device, nullable*/, double* t /*device, nullable*/,
                 double* dt_last /*device, nullable*/, dg2p_monitors* mon /*device, nullable*/,
                 double p_ref, const double* u_ref /*host, nullable*/, void* work /*device*/, void* stream);

/* dg2p_advance with the monitors of every step (the per-step scalar set of
 * the stepping path): mon_steps[i] (device array of n_steps structs) receives
 * the monitors of the state after step i + 1 -- alpha range, field
 * integrals, non-physical count, max |P - p_ref|, max |u - u_ref| -- and the
 * time-step rate of that state with its dt (the step that would follow;
 * *dt_fixed when given).  The last stage of each step emits the records that
 * are reduced into these monitors and the next dt: inside the next step's
 * first stage on grids of 13 to 1024 element workgroups (p = 3; 13 to 256 at
 * p = 4), by two small kernels per step otherwise and for the last step.  The integrals' summation
 * order differs between the two (rounding-level differences); the rest is
 * exact.  Same states and dt as dg2p_advance.  A NaN anywhere in a state's rate
 * or monitors propagates (the dt of a state with a failed closure is NaN).
 * work: dg2p_workspace_size(DG2P_OP_ADVANCE) bytes. */
int dg2p_advance_monitored(dg2p_mesh m, const dg2p_params* p /*host*/, double* U /*device, in/out*/, int n_steps,
                           double cfl, const double* dt_fixed /*device, nullable*/, double* t /*device, nullable*/,
                           double* dt_last /*device, nullable*/, dg2p_monitors* mon_steps /*device [n_steps]*/,
                           double p_ref, const double* u_ref /*host, nullable*/, void* work /*device*/,
                           void* stream);

/* Vector-Jacobian product of dg2p_rhs (hand-written reverse mode):
 * U_bar = (dR/dU)^T R_bar, overwritten; if param_bar != NULL,
 * param_bar[0] += <R_bar, dR/dsigma> (surface tension).  Non-smooth points:
 * d max(a,b) splits 1/2, 1/2 at ties, d|x|/dx = 0 at 0.  Every boundary
 * kind (the ghost traces are reversed into the boundary element's own
 * values).  FP64 and p = 3 only (DG2P_EUNSUPPORTED otherwise).  U, R_bar,
 * U_bar: device [N_f][E][4^d]; U_bar may not alias.  work: DG2P_OP_RHS_VJP
 * bytes. */
int dg2p_rhs_vjp(dg2p_mesh m, const dg2p_params* p /*host*/, const double* U /*device*/,
                 const double* R_bar /*device*/, double* U_bar /*device, out*/,
                 double* param_bar /*device, nullable, accumulated*/, void* work /*device*/, void* stream);

/* Vector-Jacobian product of one dg2p_rk_step with the (frozen) step *dt:
 * U_n_bar = (dU_{n+1}/dU_n)^T U_np1_bar (overwritten), param_bar[0] +=
 * <U_np1_bar, dU_{n+1}/dsigma>.  Recomputes the two intermediate stages from
 * U_n, then reverses the three stages (three dg2p_rhs_vjp).  Same
 * restrictions as dg2p_rhs_vjp.  work: DG2P_OP_RK_STEP_VJP bytes. */
int dg2p_rk_step_vjp(dg2p_mesh m, const dg2p_params* p /*host*/, const double* U_n /*device*/,
                     const double* dt /*device*/, const double* U_np1_bar /*device*/,
                     double* U_n_bar /*device, out*/, double* param_bar /*device, nullable*/,
                     void* work /*device*/, void* stream);

/* Monitors of a state (all fields of *mon; dt is set to 0.1 / max_rate).  p_ref and u_ref are
 * the reference pressure and velocity of dev_p / dev_u (host values).
 * work: DG2P_OP_MONITORS bytes.  Deterministic (fixed reduction order). */
int dg2p_compute_monitors(dg2p_mesh m, const dg2p_params* p /*host*/, const double* U /*device*/,
                  double p_ref, const double* u_ref /*host, d values*/,
                  dg2p_monitors* mon /*device*/, void* work /*device*/, void* stream);

/* ---- Kinematic mode ----------------------------------------------------------
 * The phase field phi and the level set psi under a prescribed velocity
 * u(x, t) = u0(x) s(t), s = cos(pi t / period) (period > 0) or 1 (Results,
 * "Kinematic tests": linear advection of a droplet, Rider-Kothe vortex).
 * Same discretisation as the alpha and psi rows of dg2p_rhs with the nodal
 * u in place of rho u / rho; the face speed is max |u.m| over both traces
 * (there is no sound speed), which makes the hat/tilde correction the upwind
 * flux.  Classical RK4 in time (the paper's integrator for these tests).
 * Periodic meshes only (EUNSUPPORTED else); FP64; p = 3 or p = 1 (the
 * paper's two orders of the Rider-Kothe study; n = (p+1)^d nodes per element).
 *   state    Phi[2][E][n]: Phi[0] = phi, Phi[1] = psi
 *   velocity u0[d][E][n]: nodal amplitude u0 (device)                        */
typedef struct {
  double Gamma, eps;   /* Allen-Cahn velocity scale and thickness (Gamma >= 0, eps > 0) */
  double c_ip;         /* interior-penalty constant (> 0) */
  double grad_reg;     /* delta of n = g / sqrt(g.g + delta^2) (>= 0) */
  double period;       /* T of s(t) = cos(pi t / T); <= 0: s = 1 */
} dg2p_kin_params;

/* Bytes of device workspace for op DG2P_OP_KIN_RHS, _KIN_RK4 (also
 * dg2p_kin_reinit) or _KIN_AUX. */
int dg2p_kin_workspace_size(dg2p_mesh m, int op, size_t* bytes /*host*/);

/* R = dPhi/dt at time t (host scalar), [2][E][n]; Phi, u0, R device, R may
 * not alias Phi.  work: DG2P_OP_KIN_RHS bytes. */
int dg2p_kin_rhs(dg2p_mesh m, const dg2p_kin_params* kp /*host*/, const double* Phi /*device*/,
                 const double* u0 /*device*/, double t, double* R /*device*/, void* work /*device*/,
                 void* stream);

/* n_steps classical RK4 steps in place from time t0 with the fixed step dt
 * (host scalars; step n starts at t0 + n dt):
 * Phi += dt/6 (k1 + 2 k2 + 2 k3 + k4), k_i = R at t, t + dt/2, t + dt/2, t + dt.
 * work: DG2P_OP_KIN_RK4 bytes. */
int dg2p_kin_rk4(dg2p_mesh m, const dg2p_kin_params* kp /*host*/, double* Phi /*device, in/out*/,
                 const double* u0 /*device*/, int n_steps, double t0, double dt, void* work /*device*/,
                 void* stream);

/* Level-set re-initialisation in place (closing paragraphs of the Section
 * "Discontinuous Galerkin discretisation"): Phi[1] (psi) is replaced by n_iter
 * classical RK4 pseudo-time steps of length dtau of
 *   d psi / d tau = sgn (1 - |grad psi|) + div(nu grad psi)
 * started from psi0 = Phi[0] - 1/2, with sgn = tanh(psi0 / (2 eps |grad psi0|))
 * (|grad psi0| regularised by grad_reg) and the diffusive flux discretised
 * with the symmetric interior penalty (coefficient nu, penalty
 * c_ip nu (p+1)^2 / h).  The source sign is the one that relaxes |grad psi|
 * towards 1.  Phi[0] is unchanged.  p = 3 only.  work: DG2P_OP_KIN_RK4 bytes. */
int dg2p_kin_reinit(dg2p_mesh m, const dg2p_kin_params* kp /*host*/, double* Phi /*device, in/out*/, int n_iter,
                    double nu, double dtau, void* work /*device*/, void* stream);

/* Parameters of dg2p_kin_reinit used for the paper's runs (host outputs; the
 * paper states neither): *nu = h_min / (p+1), one nodal spacing (the
 * viscosity "proportional to the grid size"), and the pseudo step
 * *dtau = cfl h_min / (1 + (p+1)^2 d nu / h_min), the time-step rule of
 * unit-speed transport with that viscosity. */
int dg2p_kin_reinit_params(dg2p_mesh m, double cfl, double* nu /*host*/, double* dtau /*host*/);

/* Time step *dt (device scalar) = cfl h_min / (max_nodes sum_k |u0_k| +
 * (p+1)^2 d Gamma eps / h_min): the rule of dg2p_max_dt without the sound
 * speed.  work: DG2P_OP_KIN_AUX bytes. */
int dg2p_kin_max_dt(dg2p_mesh m, const dg2p_kin_params* kp /*host*/, const double* u0 /*device*/, double cfl,
                    double* dt /*device*/, void* work /*device*/, void* stream);

/* GLL-quadrature integrals for the L1 error and the relative mass error of
 * the Rider-Kothe study: out[0] = int |phi - phi0|, out[1] = int (phi - phi0),
 * out[2] = int phi0 (device array of 3; fixed summation order).  phi, phi0:
 * device [E][n].  work: DG2P_OP_KIN_AUX bytes. */
int dg2p_kin_errors(dg2p_mesh m, const double* phi /*device*/, const double* phi0 /*device*/,
                    double* out /*device*/, void* work /*device*/, void* stream);

/* Velocity amplitude of a 2D kinematic run from a nodal stream function
 * (Results, "Rider-Kothe vortex": the prescribed field is divergence free;
 * this is one representation of it on the mesh): u0 = (dS/dy, -dS/dx), each
 * derivative the element-local derivative of the nodal interpolant of S.
 * The discrete divergence D_x u0_x + D_y u0_y is then zero at every node
 * (the two element-local derivatives commute), and u0.m is continuous across
 * faces (the tangential derivative of the continuous trace of S), so the
 * transport conserves int phi to rounding; the nodally interpolated analytic
 * field conserves it only up to sum_j W_j phi_j (div_h u0)_j.  S: device
 * [E][n]; u0: device [2][E][n], may not alias S.  dim = 2 only (EUNSUPPORTED
 * else); no workspace; p = 3 or 1. */
int dg2p_kin_velocity_from_stream(dg2p_mesh m, const double* S /*device*/, double* u0 /*device, out*/,
                                  void* stream);

/* Kernel kinds of the timing facility. */
typedef enum {
  DG2P_K_INGREDIENTS = 0, /* face-ingredient pass (neighbour interface flux / traction) */
  DG2P_K_STAGE = 1,       /* residual + RK stage combine */
  DG2P_K_RATE = 2,        /* time-step rate reduction, first pass */
  DG2P_K_RATE_FINAL = 3,  /* time-step rate reduction, final pass */
  DG2P_K_MONITOR = 4,     /* monitor reduction */
  DG2P_K_PRIM = 5,        /* initial-condition map */
  DG2P_K_VJP_LOCAL = 6,   /* adjoint: residual VJP (own-element and gather passes) */
  DG2P_K_VJP_GATHER = 7,  /* reserved (timed together with DG2P_K_VJP_LOCAL) */
  DG2P_K_KIN_STAGE = 8    /* kinematic mode: residual + RK4 stage */
} dg2p_kernel_kind;

/* FP64 vector FMA issue rate of the device (a measurement utility, not a hot
 * call): launches a calibration kernel of independent v_fma_f64 chains on
 * `stream` five times, the first to warm up, waits for each (host blocking)
 * and stores the best rate in TFLOP/s into *tflops (the nominal MI355X figure
 * is 78.6: 1024 SIMDs x 16 lanes x 2 flop x 2.4 GHz; a lower rate here means
 * a lower sustained clock).  Allocates no device memory. */
int dg2p_calibrate_fp64_fma(double* tflops /*host*/, void* stream);

/* Benchmark timing.  While enabled, every kernel the library launches is
 * bracketed by a pair of library-owned hipEvents recorded on its stream (at
 * most 8192 launches per enable; enabling resets the record).  The events
 * are created on the first enable (host call, no device allocation).
 * Not thread-safe: for single-threaded benchmark drivers. */
int dg2p_timing_enable(int on);

/* Mean duration (ms) and count of the recorded launches of one kernel kind;
 * synchronises on the recorded events (host blocking). */
int dg2p_timing_read(int kernel, double* mean_ms /*host*/, long long* count /*host*/);

#ifdef __cplusplus
}
#endif

#endif /* DG2P_H */
