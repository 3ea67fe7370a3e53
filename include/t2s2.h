/*
 * t2s2 — D2Q9 T2S2-FDLBM time step on one AMD Instinct MI355X (gfx950).
 *
 * The method is the finite-difference lattice Boltzmann scheme of Chen,
 * Chai, Wang & Shi, "A finite-difference lattice Boltzmann model with
 * second-order accuracy of time and space for incompressible flow"
 * (arXiv 1911.12913):
 *   - BGK collision (eq 2.4) with the D2Q9 equilibrium (eq 3.2) and the
 *     moments of eq 3.3; Guo's force term (eq 3.12);
 *   - the mixed central / second-order upwind gradient (eqs 2.36-2.38) on a
 *     separable stretched Cartesian mesh (eqs 3.9, 3.11), taken in node-index
 *     space with the metric 1/x'(i), x'(i) = (x[i+1] - x[i-1]) / 2;
 *   - the two-stage march of Sec. 2D: half-step characteristic prediction
 *     (eqs 2.33, 2.35, 2.51, 2.52) and full-step update (eqs 2.20, 2.23).
 *     A = 0.5 is T2S2-FDLBM1; A = 0 is Guo's T1S2-FDLBM (Remark I).
 *   - non-equilibrium extrapolation on wall nodes (eq 3.10); periodic axes.
 *
 * Conventions
 *   - Every call returns an int status (T2S2_OK, T2S2_ERR_*).  Nothing throws
 *     across this boundary; t2s2_last_error() returns a message for the last
 *     failure on the calling thread.
 *   - The library never allocates device memory.  State buffers and the
 *     workspace are provided by the caller (device pointers) and must outlive
 *     the context.  Host pointers are read only during the call.
 *   - Device work is enqueued on the bound HIP stream and is asynchronous,
 *     except where a call is marked "synchronises".
 *   - Distributions cross the boundary as deviations from the rest state,
 *     g_q = f~_q - w_q (w_q the D2Q9 weights), FP64, dense layout [9][ny][nx]
 *     with x fastest.  Macroscopic fields are FP64 [ny][nx].
 *   - Lattice speed xi = 1, c_s^2 = 1/3, relaxation time tau = nu / c_s^2.
 */
#ifndef T2S2_H
#define T2S2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define T2S2_OK 0
#define T2S2_ERR_INVALID_ARG 1
#define T2S2_ERR_HIP 2
#define T2S2_ERR_UNSUPPORTED 3
#define T2S2_ERR_NONFINITE 4
#define T2S2_ERR_NOT_BOUND 5

/* Storage of the carried state g = f~ - w.  T2S2_F64 computes in FP64; the
 * reduced forms compute in FP32 with FP64 moment sums.  The state buffers
 * hold g rounded to nearest even, except the FP16 forms, which hold 2^14 g
 * (an exact power-of-two scale, so deviations down to about 4e-9 stay
 * normal FP16 numbers; |g| >= 4 overflows).  T2S2_BF16_SR_DEV and
 * T2S2_F16_SR_DEV hold the bits of T2S2_BF16_DEV and T2S2_F16_DEV, but the
 * step rounds the new interior values it stores stochastically (up in
 * magnitude with probability equal to the fraction of the unit in the last
 * place cut off; random bits from a hash of the node's position and new
 * values, so results do not depend on the launch tiling and are
 * reproducible): increments below half a unit in the last place, lost
 * under rounding to nearest, are kept on average.  Initialisation and wall
 * nodes round to nearest.  The stochastic forms run T2S2_FDLBM1 (any A)
 * only, without the adjoint.  The calls that take or return FP64 fields and
 * distributions convert to and from g. */
#define T2S2_F64 0
#define T2S2_F32_DEV 1
#define T2S2_BF16_DEV 2
#define T2S2_F16_DEV 3
#define T2S2_BF16_SR_DEV 4
#define T2S2_F16_SR_DEV 5

/* Time-marching scheme (Sec. 2A, Sec. 2D).  T2S2_FDLBM1: eq 2.23, the
 * intermediate stage at t + A dt (A = 1/2: T2S2-FDLBM1, A = 0: T1S2).
 * T2S2_FDLBM2: eq 5.23, f~^{n+1} = f~^{+,n} + dt/2 (L(f^n) + L(f^{n+1})) with
 * f^{n+1} predicted by a full-step characteristic update; A is not used.
 * T2S2_FAMILY: the eq 2.13 family with gradient weights btilde and
 * collision weights bbar,
 *   f^{n+1} - B-2 dt Omega(f^{n+1}) = f^n + dt [B-0 Omega(f^n) + B-1 Omega(f*)]
 *                 + dt [B~0 L(f^n) + B~1 L(f*) + B~2 L(f^{n+1})],
 * f* predicted as in T2S2_FDLBM1 (h = A dt), f^{n+1} on the right as in
 * T2S2_FDLBM2; the left side is solved node by node through the moments
 * and the state stays f~ = f - (dt/2) Omega (eq 2.19).  With the collision
 * weights of eqs 2.21 and 5.21, bbar = (1/2, 0, 1/2), this is the explicit
 *   f~^{n+1} = f~^{+,n} + dt [B~0 L(f^n) + B~1 L(f*) + B~2 L(f^{n+1})];
 * btilde = (0, 1, 0) is then T2S2_FDLBM1 and (1/2, 0, 1/2) T2S2_FDLBM2.
 * A B~1 + B~2 = 1/2 and A B-1 + B-2 = 1/2 give second order in time
 * (eq 2.14b). */
#define T2S2_FDLBM1 1
#define T2S2_FDLBM2 2
#define T2S2_FAMILY 3

/* Number of values written by t2s2_diagnostics. */
#define T2S2_NDIAG 6

typedef struct t2s2_config {
  double nu;            /* kinematic viscosity > 0; +INFINITY = no collision */
  double cfl;           /* dt = cfl * (minimum node spacing) / xi (eq 3.1) */
  double dt;            /* if > 0, overrides cfl */
  double eta;           /* upwind weight of the mixed difference, in [0, 1] */
  double A;             /* intermediate stage at t + A dt, in [0, 1] */
  double force[2];      /* body-force acceleration (eq 3.12) */
  double u_wall[4][2];  /* wall velocity: left, right, bottom, top; corner
                           nodes take the left/right value */
  int periodic_x;       /* 1: x periodic with period period_x; 0: walls */
  int periodic_y;
  double period_x;
  double period_y;
  int storage;          /* T2S2_F64, T2S2_F32_DEV, T2S2_BF16_DEV, T2S2_F16_DEV,
                           T2S2_BF16_SR_DEV, T2S2_F16_SR_DEV */
  int scheme;           /* T2S2_FDLBM1 (0 is read as this), T2S2_FDLBM2 or
                           T2S2_FAMILY */
  double btilde[3];     /* T2S2_FAMILY only: (B~0, B~1, B~2), each >= 0,
                           B~0, B~1 <= 1, B~2 <= 1/2, summing to 1 within
                           1e-12 (eq 2.14a); ignored by the other schemes */
  double bbar[3];       /* T2S2_FAMILY only: (B-0, B-1, B-2) in the same
                           ranges; all zero reads as (1/2, 0, 1/2); ignored
                           by the other schemes */
} t2s2_config;

typedef struct t2s2_ctx t2s2_ctx;

/* Create a context for the mesh with node coordinates x[nx], y[ny] (host,
 * strictly increasing; on a walled axis the first and last nodes are walls;
 * on a periodic axis x[nx-1] - x[0] < period).  Validates nx, ny >= 5,
 * 0 < cfl <= 1 (unless dt > 0), nu > 0, 0 <= eta <= 1, 0 <= A <= 1, and
 * computes dt and the stencil coefficients on the host.  T2S2_FDLBM1 with
 * A = 0 (T1S2) runs a single-stencil step kernel (the half step is then the
 * identity); the values are those of the general step.  One population
 * plane (ny * pitch elements of the storage type) must be under 4 GiB
 * (T2S2_ERR_UNSUPPORTED otherwise; FP64 up to about 23000 x 23000 nodes).
 * No device call. */
int t2s2_create(const t2s2_config* cfg, const double* x, int nx, const double* y, int ny,
                t2s2_ctx** out);

/* Bytes of one state buffer: 9 * ny * pitch * sizeof(storage element);
 * pitch = nx rounded up to a multiple of 64. */
size_t t2s2_state_bytes(const t2s2_ctx* ctx);

/* Bytes of the workspace (stencil weights, quadrature weights, reduction
 * partials), 256-byte aligned device memory. */
size_t t2s2_workspace_bytes(const t2s2_ctx* ctx);

/* Attach two state buffers (ping-pong), the workspace and a hipStream_t
 * (NULL = default stream).  Uploads the weight tables; synchronises.  Plans
 * the step's launch from the device's CU count and the step kernel's
 * occupancy; if the environment variable T2S2_BLOCKS is set, its value
 * (rounded down to a multiple of 8, at least 8) replaces the block count, a
 * hook for checking that results do not depend on the tiling. */
int t2s2_bind(t2s2_ctx* ctx, void* state_a, void* state_b, void* workspace, void* stream);

/* f~ = f^eq(rho, u) (Sec. 3), minus the non-equilibrium part of eq 3.5
 * when grad is non-NULL: rho0 w (2 tau + dt)/(2 c_s^2) xi xi : grad u with
 * rho0 = 1.  Device pointers: rho, ux, uy [ny][nx]; grad [4][ny][nx] =
 * du/dx, du/dy, dv/dx, dv/dy.  Writes the current buffer. */
int t2s2_init_macro(t2s2_ctx* ctx, const double* rho, const double* ux, const double* uy,
                    const double* grad);

/* Load an arbitrary state g = f~ - w (device, FP64 [9][ny][nx]) into the
 * current buffer, rounding to the storage type (nearest even). */
int t2s2_init_distributions(t2s2_ctx* ctx, const double* g);

/* Advance nsteps >= 0 time steps (Sec. 2D, eq 2.23); asynchronous. */
int t2s2_step(t2s2_ctx* ctx, int64_t nsteps);

/* Launch plumbing for short steps (small meshes are launch-bound): record
 * steps_per_graph (even, >= 2) consecutive steps of t2s2_step -- the same
 * kernels, the same Sec. 2D step -- into a HIP graph owned by the context,
 * replacing any earlier one.  Needs a non-default bound stream
 * (T2S2_ERR_UNSUPPORTED otherwise).  Nothing executes during the capture.
 * Rebinding the context drops the graph.  The HIP runtime allocates the
 * graph's own resources. */
int t2s2_graph_capture(t2s2_ctx* ctx, int steps_per_graph);

/* Advance nsteps >= 0 steps like t2s2_step, replaying the captured graph for
 * whole multiples of its length and taking the rest (and, when the state
 * sits in the other buffer than at capture, one step first) as plain
 * launches.  Results are bitwise those of t2s2_step.  Asynchronous.
 * T2S2_ERR_NOT_BOUND if no graph was captured. */
int t2s2_graph_step(t2s2_ctx* ctx, int64_t nsteps);

/* Index (0 = state_a, 1 = state_b) of the buffer holding the current state. */
int t2s2_current(const t2s2_ctx* ctx);

/* Number of steps taken since the last init. */
int64_t t2s2_steps_taken(const t2s2_ctx* ctx);

/* Time step dt in use. */
double t2s2_dt(const t2s2_ctx* ctx);

/* Macroscopic fields of eq 3.3 into device arrays [ny][nx]:
 * drho = rho - 1, ux, uy (momentum shifted by dt/2 rho F).  Any may be NULL.
 * Asynchronous. */
int t2s2_moments(t2s2_ctx* ctx, double* drho, double* ux, double* uy);

/* Current state as FP64 deviations g = f~ - w into device memory
 * [9][ny][nx].  Asynchronous. */
int t2s2_read_distributions(t2s2_ctx* ctx, double* g);

/* Global diagnostics of the current state, FP64, deterministic reduction
 * (fixed block partition and order).  J = trapezoid cell measure of the
 * separable mesh.  out[0] = sum J (rho - 1), out[1] = sum J rho |u|^2 / 2,
 * out[2] = max |u|, out[3] = count of nodes with a non-finite population,
 * out[4] = sum J rho ux, out[5] = sum J rho uy.  out is host memory;
 * synchronises.  Returns T2S2_ERR_NONFINITE (after filling out) when
 * out[3] > 0. */
int t2s2_diagnostics(t2s2_ctx* ctx, double out[T2S2_NDIAG]);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops that allow no allocation and no host synchronisation): the values
 * of t2s2_diagnostics for the current state, written to device memory
 * out[T2S2_NDIAG] (FP64, 8-byte aligned) on the bound stream, asynchronous;
 * bitwise those of t2s2_diagnostics (same kernels, same reduction order).
 * The reduction partials live in a static device array of the library
 * (kept per device until the process ends; 32 KiB, enough for the fixed
 * partial grid of any mesh, so no mesh is refused for its size) instead of
 * the workspace; its device address is looked up by t2s2_bind.  No memory
 * is allocated and no HIP call that allocates is made.  No error code for non-finite populations: out[3] counts them.
 * Calls that overlap on one device (several streams or threads) share the
 * array and race; every call overwrites all of the partials it reads.
 * Errors: INVALID_ARG (NULL context, NULL or misaligned out), NOT_BOUND,
 * UNSUPPORTED (device index >= 64), HIP_ERROR. */
int t2s2_diagnostics_noalloc(t2s2_ctx* ctx, double* out);

/* Global relative error of the velocity (eq 3.6) against a reference field
 * u' = (ux_ref, uy_ref): device FP64 arrays [ny][nx] (row-major, no pitch),
 * read only.  out (host, T2S2_NGRE doubles) receives, over all nodes of the
 * current state, u the velocity of the moments (t2s2_moments):
 *   out[0] = sum |u - u'|^2,  out[1] = sum |u'|^2,  out[2] = sum |u|^2,
 *   out[3] = sqrt(out[0] / out[1]), E(u) of eq 3.6 for an analytic u'
 *            (NaN when out[1] = 0),
 *   out[4] = sqrt(out[0] / out[2]), the residual GRE of the cavity
 *            (Sec. 3C) when u' is the velocity at the previous output time
 *            (NaN when out[2] = 0).
 * Deterministic reduction; synchronises.  Non-finite populations make the
 * results non-finite (no error code; t2s2_diagnostics counts them).
 * Errors: INVALID_ARG (NULL pointer), NOT_BOUND, HIP_ERROR. */
#define T2S2_NGRE 5
int t2s2_velocity_error(t2s2_ctx* ctx, const double* ux_ref, const double* uy_ref,
                        double out[T2S2_NGRE]);

/* Host copies of the stencil weights computed at create: the dt-scaled
 * taps of L = -dt xi_a d/dx_a (the mixed difference of eqs 2.36-2.38, eta
 * the upwind weight, times the metric 1/x'(i) of the mesh), per node and
 * sign of xi_a.  wx[8 i + 4 s + k] for x node i: s = 0 (xi_a > 0) taps at
 * offsets -2, -1, 0, +1; s = 1 (xi_a < 0) at -1, 0, +1, +2; zero on wall
 * nodes; central at the first interior node of a walled axis.  wy
 * likewise.  wx, wy: host arrays of 8 nx and 8 ny doubles, either may be
 * NULL.  No device call.  Errors: INVALID_ARG (NULL context). */
int t2s2_stencil_weights(const t2s2_ctx* ctx, double* wx, double* wy);

/* Relaxation parameter omega = dt / tau in use (0 without collision). */
double t2s2_omega(const t2s2_ctx* ctx);

/* ---- Discrete adjoint of the step (unforced flows) --------------------
 * The reverse of the step above, stage by stage, for gradients of a loss of
 * the state with respect to the initial fields and the viscosity.  Adjoint
 * states lambda (dL/dg for g = f~ - w) live in device buffers of
 * t2s2_adjoint_state_bytes() bytes: FP64 for T2S2_F64 storage, FP32
 * otherwise, in the state's pitched [9][ny][pitch] layout. */

/* Bytes of one adjoint state buffer. */
size_t t2s2_adjoint_state_bytes(const t2s2_ctx* ctx);

/* Bytes of the adjoint scratch (recomputed intermediates, partial sums). */
size_t t2s2_adjoint_scratch_bytes(const t2s2_ctx* ctx);

/* Attach the adjoint scratch (device, 256-byte aligned).  Returns
 * T2S2_ERR_UNSUPPORTED for forced flows, for T2S2_FDLBM2 and the family,
 * for the stochastically rounded storage, and when one plane of the
 * adjoint's buffers (ny * pitch elements of its arithmetic type) is not
 * under 4 GiB (16-bit storage above about 1.07 G nodes).  Plans the
 * reverse march from the device's compute units and the kernels' occupancy
 * (blocks of four waves, or eight on small meshes; the environment variable
 * T2S2_ADJ_ROWS=4 or 8, read here, forces the shape); launches nothing. */
int t2s2_bind_adjoint(t2s2_ctx* ctx, void* scratch);

/* lambda = d(<gu, u> + <gv, v>)/dg of the velocity of eq 3.3 at every node,
 * for a state buffer `state` of this context (storage layout).  gu, gv:
 * device FP64 [ny][nx] (either may be NULL).  Asynchronous. */
int t2s2_adjoint_seed_velocity(t2s2_ctx* ctx, const void* state, const double* gu,
                               const double* gv, void* lam);

/* lam_n = (d f~^{n+1} / d f~^n)^T lam_np1 for the step taken from the
 * state `state_n` (storage layout).  If dnu_accum (device, one double) is
 * non-NULL, adds <lam_np1, d f~^{n+1}/d nu> to it, the derivative at a fixed
 * dt through omega = dt / tau = dt c_s^2 / nu (d omega / d nu = -omega / nu;
 * zero without collision).  Summed over the steps of a rollout it is dL/dnu.
 * lam_np1 and lam_n must differ.  Asynchronous; deterministic (fixed
 * reduction order). */
int t2s2_adjoint_step(t2s2_ctx* ctx, const void* state_n, const void* lam_np1, void* lam_n,
                      double* dnu_accum);

/* One step of the bound scheme from the state buffer src into dst (both of
 * t2s2_state_bytes(), storage layout), also storing S, the half-step
 * prediction of eq 2.33, at the interior nodes of s_out
 * (t2s2_adjoint_state_bytes(), the adjoint's type and layout; its other
 * entries are left as they are).  dst is the step's new state, wall nodes
 * included: the state t2s2_step produces (at A = 0 it is formed by the
 * two-stencil kernel, equal to the single-stencil one's to rounding).  The
 * three buffers must differ; the bound state buffers are not touched.  Same
 * scope as the adjoint (unforced, T2S2-FDLBM1 family); needs
 * t2s2_bind_adjoint.  Asynchronous. */
int t2s2_step_save_s(t2s2_ctx* ctx, const void* src, void* dst, void* s_out);

/* t2s2_adjoint_step without its recompute of the step: state_np1 and s_n
 * are dst and s_out of t2s2_step_save_s(ctx, state_n, ...).  Same outputs
 * as t2s2_adjoint_step (lam_n bitwise equal).  For a backward pass that has
 * stored each step's S as it recomputed its segment.  Asynchronous. */
int t2s2_adjoint_step_stored(t2s2_ctx* ctx, const void* state_n, const void* state_np1,
                             const void* s_n, const void* lam_np1, void* lam_n,
                             double* dnu_accum);

/* Gradients of the equilibrium initial state f~ = f^eq(rho, u) (Sec. 3):
 * grho = dL/drho, gux = dL/dux, guy = dL/duy from lam0 = dL/dg^0.  Device
 * FP64 [ny][nx] fields; outputs may be NULL.  Asynchronous. */
int t2s2_adjoint_init_macro(t2s2_ctx* ctx, const void* lam0, const double* rho,
                            const double* ux, const double* uy, double* grho, double* gux,
                            double* guy);

/* Copy an adjoint state to / from dense FP64 [9][ny][nx] device memory. */
int t2s2_adjoint_read(t2s2_ctx* ctx, const void* lam, double* out);
int t2s2_adjoint_load(t2s2_ctx* ctx, const double* in, void* lam);

/* ---- Von Neumann stability maps (Sec. 2C) -----------------------------
 * For each point (omega_i, r_i) -- omega = dt / tau, r = dt / dx on a
 * uniform mesh, xi = 1 -- the largest spectral radius, over a grid of modes
 * k, of the growth matrix G(k) (9 x 9) of a perturbation f' e^{i k.x} about
 * the uniform equilibrium f^eq(rho = 1, u):
 *   T2S2_STAB_PAPER  eq 4.7 for the (B~2, B-2) family (b2tilde, b2bar), with
 *                    the advection symbol applied from the left;
 *   T2S2_STAB_FDLBM1 the exact linearisation of the step of eq 2.23 with
 *                    h = A dt (the step t2s2_step takes for T2S2_FDLBM1);
 *   T2S2_STAB_FDLBM2 the exact linearisation of the eq 5.23 step;
 *   T2S2_STAB_FAMILY the exact linearisation of the T2S2_FAMILY step with
 *                    gradient weights btilde, collision weights bbar and
 *                    h = A dt.
 * S is the symbol of the mixed difference (eq 4.8 with the imaginary unit
 * in its exponentials).  Modes: theta_y = k_y dx in [0, pi] (nk points);
 * theta_x in [0, pi] (nk points) or, with full_kx, in [-pi, pi] (2 nk - 1
 * points), which with theta_y covers every mode up to conjugation.  The
 * radius is ||G^m||^(1/m) at m = 2^squarings (relative error about
 * ln(cond) / m).  omega, r, radius: device FP64 arrays of npoints.
 * Asynchronous on `stream` (a hipStream_t, NULL = default). */
#define T2S2_STAB_PAPER 0
#define T2S2_STAB_FDLBM1 1
#define T2S2_STAB_FDLBM2 2
#define T2S2_STAB_FAMILY 3

typedef struct t2s2_stability_params {
  int model;       /* T2S2_STAB_PAPER, _FDLBM1, _FDLBM2 or _FAMILY */
  double eta;      /* upwind weight, in [0, 1] */
  double A;        /* intermediate stage (_FDLBM1, _FAMILY), in [0, 1] */
  double b2bar;    /* B-2 of eq 4.7 (T2S2_STAB_PAPER) */
  double b2tilde;  /* B~2 of eq 4.7 (T2S2_STAB_PAPER) */
  double u[2];     /* velocity of the uniform state */
  int nk;          /* modes per half axis, 2..257 */
  int full_kx;     /* 1: theta_x in [-pi, pi]; 0: [0, pi] */
  int squarings;   /* 1..60 */
  double btilde[3]; /* T2S2_STAB_FAMILY: (B~0, B~1, B~2), finite (any
                       weights; the step's own ranges are not imposed) */
  double bbar[3];   /* T2S2_STAB_FAMILY: (B-0, B-1, B-2), finite; all zero
                       reads as (1/2, 0, 1/2).  The implicit weight divides
                       by 1 + B-2 omega: a point where that is 0 gets a
                       non-finite radius */
} t2s2_stability_params;

int t2s2_stability_map(const t2s2_stability_params* prm, const double* omega, const double* r,
                       int npoints, double* radius, void* stream);

/* Reference copy for the step's roofline (not part of the method): copies
 * the nine planes of plane_elems elements of elem_bytes (8, 4 or 2) bytes
 * each, [9][plane_elems], from src to dst (device pointers, aligned to
 * elem_bytes, not overlapping), bit for bit, one element per lane and plane,
 * with the step kernel's store policy (non-temporal for 8-byte elements).
 * Its bandwidth, 2 * 9 * plane_elems * elem_bytes bytes per call, is the
 * practical ceiling of a kernel that reads and writes the state once.
 * Asynchronous on `stream` (a hipStream_t, NULL = default); allocates
 * nothing.  INVALID_ARG for NULL, misaligned or overlapping buffers, a
 * non-positive plane_elems or another elem_bytes; HIP_ERROR if the launch
 * fails. */
int t2s2_copy_probe(const void* src, void* dst, int64_t plane_elems, int elem_bytes,
                    void* stream);

void t2s2_destroy(t2s2_ctx* ctx);

/* Message of the last failing call on this thread ("" if none). */
const char* t2s2_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* T2S2_H */
