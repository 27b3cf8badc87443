/*
 * dgns.h -- C ABI of the MI355X matrix-free DG compressible Navier-Stokes library.
 *
 * The library evaluates the spatial operator of the high-order discontinuous
 * Galerkin discretisation of Fehn, Wall & Kronbichler (arXiv 1806.03095):
 *
 *     dU/dt = L(U) = M^{-1} ( -F_c(U) - F_v(U) + F_rhs(U) )      (Sec. 2.4, eq.
 *                                                                 SpatiallyDiscretizedProblem)
 *
 * with F_c, F_v the convective and viscous weak-form operators of Sec. 2.2.2, eq.
 * (WeakFormulationConservedVariables) -- local Lax-Friedrichs flux, symmetric
 * interior penalty with the penalty of eq. (TauIP_Element) -- evaluated by Gauss
 * quadrature with n_q points per direction (Sec. 2.2.3) and sum factorisation
 * (Sec. 2.3); M the block-diagonal mass matrix on k+1 points, inverted exactly; and
 * a low-storage explicit Runge-Kutta step that calls L once per stage (Sec. 2.4).
 *
 * Conventions (all entry points):
 *  - Every call returns int: DGNS_OK (0) or a negative DGNS_E* code.  On error,
 *    dgns_last_error() returns a message for the calling thread; nothing is thrown
 *    across the ABI and no output is written.
 *  - Solution vectors are DEVICE pointers owned by the caller, float64, contiguous,
 *    laid out [5][n_cells][(k+1)^3]: conserved component (rho, rho u1, rho u2,
 *    rho u3, rho E), cell (i0 + n0*(i1 + n1*i2)), node (a0 + (k+1)*(a1 + (k+1)*a2)
 *    of the tensor-product nodal basis, first coordinate fastest).  They must be
 *    8-byte aligned (a misaligned vector returns DGNS_EINVAL before anything is
 *    launched).  The float32 operator variant keeps this float64 interface.
 *  - The library owns only its context (geometry, metric terms, 1D tables).  It
 *    never frees or retains caller memory.
 *  - Calls are asynchronous on the context's HIP stream unless stated otherwise.
 *    Inputs and outputs must not alias unless stated.  Results are deterministic:
 *    no atomics, fixed summation order.
 *  - One context per stream; a context is not safe for concurrent calls.
 */
#ifndef DGNS_H
#define DGNS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DGNS_OK 0
#define DGNS_EINVAL (-1)         /* bad argument: null pointer, alignment, size, range, alias */
#define DGNS_ENOMEM (-2)         /* device or host allocation failed */
#define DGNS_EHIP (-3)           /* a HIP runtime call failed */
#define DGNS_EUNSUPPORTED (-4)   /* (degree, n_q, precision) has no compiled kernel */
#define DGNS_ENONFINITE (-5)     /* a diagnostic found a NaN or Inf in the state */

#define DGNS_BASIS_LGL 0         /* Legendre-Gauss-Lobatto support points (Sec. 2.2.1) */
#define DGNS_BASIS_GL 1          /* Gauss-Legendre support points */

#define DGNS_FP64 0
#define DGNS_FP32 1              /* operator arithmetic in float32; vectors stay float64 */

#define DGNS_MESH_AFFINE 0       /* uniform box */
#define DGNS_MESH_CHANNEL 1      /* tanh wall-normal stretching in x2 (Sec. 5.3.1) */
#define DGNS_MESH_CURVED 2       /* x_i += a * prod_j sin(2 pi s_j), s the unit-cube coordinate */

#define DGNS_TERM_CONVECTIVE 1u  /* cell + face convective terms */
#define DGNS_TERM_VISCOUS 2u     /* cell + face viscous terms (SIPG) */
#define DGNS_TERM_FORCE 4u       /* body-force right-hand side */
#define DGNS_TERM_ALL 7u

#define DGNS_IC_TAYLOR_GREEN 0   /* Sec. 5.2.1; ic_params = {U0, L, Mach, rho0} */
#define DGNS_IC_CHANNEL 1        /* Sec. 5.3.1; ic_params = {u_max, Mach, power, amp} */
#define DGNS_IC_UNIFORM 2        /* ic_params = {rho, u1, u2, u3, p} */

typedef struct dgns_ctx dgns_ctx;

/* Discretisation and fluid parameters (Sec. 2.1, 2.2). */
typedef struct dgns_params {
    int degree;            /* polynomial degree k, 1..15 */
    int n_q;               /* Gauss points per direction for the flux integrals; compiled
                            * pairs: k = 1..7 with n_q = k+1, the 3/2 rule floor((3k+2)/2)
                            * and 2k+1 for k <= 4; k = 8..15 with n_q = k+1, and the 3/2
                            * rule for k <= 10 (other pairs: DGNS_EUNSUPPORTED) */
    int basis;             /* DGNS_BASIS_* */
    int precision;         /* DGNS_FP64 or DGNS_FP32 */
    double gamma;          /* ratio of specific heats */
    double R;              /* specific gas constant */
    double mu;             /* dynamic viscosity */
    double lambda;         /* thermal conductivity */
    double rho_ref;        /* reference density rho_0 of nu = mu / rho_0 in tau_IP */
    double body_force[3];  /* constant body force f of F_rhs = (0, f, f.u) */
    double wall_T;         /* isothermal wall temperature (non-periodic directions) */
} dgns_params;

/* Structured hexahedral mesh of the box [lo, hi] with n[d] cells per direction.
 * The cell mapping is the degree-k interpolant of the box map at each cell's LGL
 * points (isoparametric).  A direction that is not periodic has walls at both ends. */
typedef struct dgns_box_mesh {
    int n[3];
    double lo[3];
    double hi[3];
    int periodic[3];       /* 1 = periodic, 0 = walls */
    int kind;              /* DGNS_MESH_* */
    double stretch_C;      /* tanh stretching factor C for DGNS_MESH_CHANNEL */
    double deform_amp;     /* warp amplitude a for DGNS_MESH_CURVED */
} dgns_box_mesh;

/* Thread-local text of the last error; never NULL. */
const char* dgns_last_error(void);

/* Builds the mesh, the metric terms at every quadrature point (Sec. 2.2.3, eq.
 * IntegralsReferenceSpace), the penalty tau_IP per face (eq. TauIP_Element), and
 * uploads them.  stream: a hipStream_t (NULL = the default stream).  Synchronous.
 * Fails with DGNS_EINVAL if the mapping folds (det J <= 0 at a quadrature point).
 * Degrees 8..15 stream each cell through the kernels plane by plane (its coefficients
 * and residual no longer fit on chip); they provide the operator, the residual, the
 * inverse mass, the Runge-Kutta step and stage update, the time step, the initial
 * projection, the diagnostics and the kinetic energy (one quadrature plane at a time), and
 * return DGNS_EUNSUPPORTED for a nonzero body force (at creation) and from the channel
 * statistics and adjoint entry points.
 * Device memory owned by the context besides the mesh data: a face buffer of
 * 60 (k+1)^2 doubles per cell, plus 10 n_q (k+1)^2 doubles per cell where the streamed
 * kernels can run (k >= 8; k = 6, n_q = 10 and k = 7, n_q = 11 in float64); DGNS_ENOMEM
 * if that allocation fails. */
int dgns_create(const dgns_params* params, const dgns_box_mesh* mesh, void* stream, dgns_ctx** out);

/* Releases everything the context owns.  Synchronises its stream first.  NULL is a no-op. */
int dgns_destroy(dgns_ctx* ctx);

/* Number of cells, nodes per cell (k+1)^3, and DoFs 5*n_cells*(k+1)^3. */
int dgns_sizes(const dgns_ctx* ctx, int64_t* n_cells, int64_t* nodes_per_cell, int64_t* n_dof);

/* Rebinds the stream used by later calls. */
int dgns_set_stream(dgns_ctx* ctx, void* stream);

/* R = the weak-form right-hand side of eq. (WeakFormulationConservedVariables)
 * tested against every basis function, BEFORE the inverse mass matrix:
 * R = -F_c(U) - F_v(U) + F_rhs(U), restricted to the terms in term_mask
 * (DGNS_TERM_*).  U, R: device, n_dof doubles each, must not alias. */
int dgns_apply_residual(dgns_ctx* ctx, const double* U, double* R, unsigned term_mask);

/* L = M^{-1} R with the exact inverse of the block-diagonal mass matrix on k+1
 * Gauss points (Sec. 2.2.3, 2.3).  R and L may alias (in place is allowed). */
int dgns_apply_inverse_mass(dgns_ctx* ctx, const double* R, double* L);

/* L = M^{-1} (-F_c(U) - F_v(U) + F_rhs(U)), all terms (eq. SpatiallyDiscretizedProblem).
 * t is accepted for time-dependent right-hand sides (none at present). */
int dgns_apply_operator(dgns_ctx* ctx, const double* U, double* L, double t);

/* The explicit low-storage Runge-Kutta scheme of dgns_rk_step, dgns_rk_stage_update and
 * dgns_rk_step_vjp (Sec. 2.4: an s-stage scheme, one L per stage), in the 2N-storage
 * Williamson form  dU <- A_i dU + dt L(U, t + c_i dt);  U <- U + B_i dU,  i = 0..s-1.
 * Default (and after dgns_set_rk_scheme(ctx, 0, NULL, NULL, NULL)): the five-stage,
 * fourth-order scheme of Carpenter & Kennedy (1994).  A, B, c: HOST arrays of `stages`
 * doubles (1 <= stages <= 16), copied; A[0] must be 0; c may be NULL (then computed from
 * A and B).  The paper's own scheme (seven stages, third order) can be set this way
 * when its published coefficients are at hand.  DGNS_EINVAL for a bad argument. */
int dgns_set_rk_scheme(dgns_ctx* ctx, int stages, const double* A, const double* B, const double* c);

/* The scheme in use: *stages, and A, B, c into host arrays of at least *stages doubles
 * (each may be NULL). */
int dgns_get_rk_scheme(const dgns_ctx* ctx, int* stages, double* A, double* B, double* c);

/* One step of the context's 2N Runge-Kutta scheme (dgns_set_rk_scheme), one L per stage.
 * U is updated in place.  work: device scratch of at least 2*n_dof doubles owned
 * by the caller (contents on return are unspecified): dU and a second copy of the
 * state, since stages 1..s-1 fuse the update into the operator kernels and write the
 * new state into the other buffer (U -> work[n_dof:] -> U -> ...; after an odd number
 * of fused stages the result is copied back into U). */
int dgns_rk_step(dgns_ctx* ctx, double* U, double* work, double t, double dt);

/* The vector update of one stage of that scheme on its own (Sec. 2.4; the paper's
 * "RK update" operation): dU <- A_i dU + dt L, then U <- U + B_i dU, for stage
 * i = 0..s-1 (the first stage does not read dU).  U, dU, L: device, n_dof doubles
 * each, pairwise non-overlapping; U and dU are updated in place.  Returns
 * DGNS_EINVAL for a stage outside 0..s-1, a non-finite dt or overlapping vectors. */
int dgns_rk_stage_update(dgns_ctx* ctx, double* U, double* dU, const double* L, int stage, double dt);

/* The time step of eq. (TimeStepRestrictions_Compressible):
 * dt = min(Cr/k^e * h_min/(umax + umax/mach), D/k^f * h_min^2/nu), h_min the
 * minimum vertex distance of the mesh.  Host result, no device work. */
int dgns_compute_dt(const dgns_ctx* ctx, double Cr, double D, double e, double f,
                    double umax, double mach, double* dt);

/* Diagnostics of Sec. 5.2.3 computed on the device, returned to the host
 * (synchronises the stream):
 *   out8[0] = e_k = 1/V int |u|^2/2,      out8[1] = eps = nu/V int grad u : grad u,
 *   out8[2] = -de_k/dt = -1/V int u.(L_m - u L_rho)/rho   (NaN if L is NULL),
 *   out8[3] = int rho,  out8[4..6] = int rho u,  out8[7] = int rho E.
 * e_k, eps and the rate use the n_q rule, the totals the k+1 rule (= 1^T M U).
 * Returns DGNS_ENONFINITE if any of them is not finite (a state that has blown up,
 * Sec. 5.2.2); out8 is then left untouched, as for every other error. */
int dgns_diagnostics(dgns_ctx* ctx, const double* U, const double* L, double* out8);

/* For callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the diagnostics of dgns_diagnostics,
 * computed by the same kernels, written to out8, a DEVICE array of 8 doubles owned by
 * the caller, asynchronously on the context's stream -- no allocation, no host
 * synchronisation.  The per-cell partial sums and their totals live in a static
 * device workspace of the library (18.9 MB per GPU, held until the process ends),
 * which limits the mesh to at most 262144 cells (64^3): larger meshes return
 * DGNS_EINVAL before anything is launched.  Every call on a GPU shares that GPU's
 * workspace, so calls that overlap on one GPU (concurrent streams or threads) race.
 * Non-finite results are not detected here (that needs the host): out8 then holds them
 * as computed.  out8 must not overlap U or L.  L may be NULL (out8[2] = NaN). */
int dgns_diagnostics_noalloc(dgns_ctx* ctx, const double* U, const double* L, double* out8);

/* L2 projection of an initial state onto the DG space: U = M^{-1} (phi_i, U0)
 * with the right-hand side on the n_q rule.  noise: NULL, or device array
 * [3][n_cells][(k+1)^3] of values in [-1,1] used by DGNS_IC_CHANNEL for the
 * velocity perturbation amp * u1(x2) * noise at each node (added after the
 * projection).  U: device output. */
int dgns_project_ic(dgns_ctx* ctx, int ic, const double* ic_params, const double* noise, double* U);

/* ---------------------------------------------------------------- adjoint
 * Hand-written reverse-mode derivatives of the operator above (float64 contexts,
 * degree <= 5).  They differentiate exactly what the forward entry points
 * compute: the Lax-Friedrichs max() takes the derivative of the selected side
 * (the interior one only when it is strictly larger). */

/* Ubar = (dR/dU)^T Rbar for the residual of dgns_apply_residual with the same
 * term_mask.  U, Rbar, Ubar: device, n_dof doubles; Ubar must not overlap U or Rbar. */
int dgns_apply_residual_vjp(dgns_ctx* ctx, const double* U, const double* Rbar, double* Ubar, unsigned term_mask);

/* Ubar = (dL/dU)^T Lbar for L = M^{-1}(-F_c - F_v + F_rhs)(U) (M is symmetric, so
 * Ubar = (dR/dU)^T M^{-1} Lbar).  Uses a context-owned device scratch vector of
 * n_dof doubles, allocated on the first call (DGNS_ENOMEM if that fails). */
int dgns_apply_operator_vjp(dgns_ctx* ctx, const double* U, const double* Lbar, double* Ubar);

/* Reverse of one dgns_rk_step from U_n: Ubar_n = (dU_{n+1}/dU_n)^T Ubar_np1.
 * The stage states are recomputed from U_n.  work: device scratch of at least
 * (s + 4)*n_dof doubles owned by the caller, s the scheme's number of stages (9*n_dof
 * for the default scheme).  Ubar_n may equal Ubar_np1 (in
 * place) but must not otherwise overlap any argument. */
int dgns_rk_step_vjp(dgns_ctx* ctx, const double* U_n, double t, double dt, const double* Ubar_np1,
                     double* Ubar_n, double* work);

/* Profiles of the channel-flow statistics (Sec. 5.3: averages over the homogeneous
 * directions x and z).  At each of the n[1]*n_q wall-normal Gauss points y_{j,p} (cell
 * row j in direction 1, point p of the n_q rule) the averages over the plane of
 * constant y (all cells of row j, all (x, z) Gauss points, weighted by |det J| w) of
 * rho, u, v, w, uu, vv, ww, uv with (u, v, w) = (rho u)/rho.  Time averages and the
 * Reynolds stresses <u'v'> = <uv> - <u><v> are left to the caller.
 * U: device, n_dof doubles.  out: HOST array of n[1]*n_q*9 doubles owned by the
 * caller, rows [y, rho, u, v, w, uu, vv, ww, uv] ordered by j, then p.  Synchronous.
 * Needs planes of constant y: affine or channel mesh, else DGNS_EUNSUPPORTED;
 * DGNS_ENOMEM if the first call cannot allocate its 9*n_q*(n_cells + n[1]) doubles of
 * device buffer (kept for later calls); DGNS_ENONFINITE for a non-finite average. */
int dgns_channel_statistics(dgns_ctx* ctx, const double* U, double* out);

/* Mean wall shear stress of a channel (Sec. 5.3: u_tau = sqrt(tau_w / rho)) over both
 * walls in x_2: at the n_q^2 points of every wall face, mu du_1/dn with n the wall normal
 * into the fluid, from the wall cell's polynomial (du_1/dx_2 = (d(rho u_1)/dx_2 -
 * u_1 drho/dx_2)/rho), averaged with the face weights dA w.  out3: HOST array
 * {tau_w, rho_w (the wall density, same average), wall area}.  Synchronous.  Needs walls
 * in direction 1 (periodic[1] = 0) on an affine or channel mesh, else DGNS_EUNSUPPORTED;
 * DGNS_ENOMEM if the first call cannot allocate its 6 n[0] n[2] doubles (kept). */
int dgns_channel_wall_shear(dgns_ctx* ctx, const double* U, double* out3);

/* Time-averaged channel statistics (Sec. 5.3: averages over x, z and time, sampled by the
 * caller, e.g. every 10th step).  _reset clears the running sums of the context;
 * _sample(U) adds the plane averages of dgns_channel_statistics and the wall shear of
 * dgns_channel_wall_shear of U; _result writes, from the time averages <.> over the
 * samples, u_tau = sqrt(<tau_w> / <rho_w>) and per wall-normal Gauss point (n[1] * n_q rows,
 * ordered as in dgns_channel_statistics) the row
 *   [y, y+ = (y - lo[1]) u_tau / nu, u+ = <u> / u_tau, rms(u)+, rms(v)+, rms(w)+,
 *    <u'v'>+ = (<uv> - <u><v>) / u_tau^2, <rho>],   rms(u) = sqrt(<uu> - <u>^2),
 * into profiles (HOST, n[1] * n_q * 8 doubles), and {u_tau, <tau_w>, <rho_w>, samples}
 * into scalars (HOST, 4 doubles).  _result: DGNS_EINVAL without samples, DGNS_ENONFINITE if
 * the mean wall shear is not positive. */
int dgns_channel_stats_reset(dgns_ctx* ctx);
int dgns_channel_stats_sample(dgns_ctx* ctx, const double* U);
int dgns_channel_stats_result(dgns_ctx* ctx, double* profiles, double* scalars);

/* K = int |u|^2/2 over the domain (n_q rule, u = (rho u)/rho), returned to the
 * host (synchronises the stream); DGNS_ENONFINITE if not finite (ke untouched). */
int dgns_kinetic_energy(dgns_ctx* ctx, const double* U, double* ke);

/* Ubar = dK/dU for K of dgns_kinetic_energy.  Ubar must not overlap U. */
int dgns_kinetic_energy_vjp(dgns_ctx* ctx, const double* U, double* Ubar);

#ifdef __cplusplus
}
#endif

#endif /* DGNS_H */
