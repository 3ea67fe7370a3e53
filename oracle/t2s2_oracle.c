/*
 * FP64 CPU ORACLE for the D2Q9 finite-difference lattice Boltzmann step of
 * Chen, Chai, Wang & Shi, "A finite-difference lattice Boltzmann model with
 * second-order accuracy of time and space for incompressible flow"
 * (arXiv 1911.12913).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * statement of what one time step computes.  Only the tests, the smoke check
 * and the benchmark's CPU-baseline leg may build, load or call it; the GPU
 * library never does, and the two share no code.
 *
 * Every stage is a separate loop over materialised full-grid arrays, in the
 * order of the paper's computational sequence (Sec. 2D):
 *
 *   f~ --(eq 2.19 inverted)--> f --(eq 2.34, h)--> fbar^{+,h}        (P)
 *                                --(eq 2.20)------> f~^{+}            (Q)
 *   fbar(t*) = fbar^{+,h} - h xi.grad fbar^{+,h}   (eqs 2.33, 2.35)   (S)
 *   f(t*) from fbar(t*) and f^eq(t*)                (eq 2.32)          (R)
 *   f~^{n+1} = f~^{+} + dt L(f(t*))                 (eqs 2.23, 2.27)
 *
 * with h = A dt (A = 1/2: T2S2-FDLBM1; A = 0: Guo's T1S2-FDLBM, Remark I),
 * BGK collision (eq 2.4), the equilibrium of eq 3.2, moments of eq 3.3,
 * Guo's force term of eq 3.12 and the mixed central / second-order upwind
 * difference of eqs 2.36-2.38.  Wall nodes use non-equilibrium extrapolation
 * (eq 3.10).  The T2S2-FDLBM2 sequence (eq 5.23, Sec. 2D) is scheme 2; the
 * eq 2.13 family with general gradient weights B~ and collision weights B-
 * is step_family.
 *
 * Readings where the paper is silent or garbled (each one is listed with its
 * justification in the design notes of the repository):
 *  - lattice speed xi = 1, c_s^2 = 1/3, tau = nu / c_s^2;
 *  - eta weights the UPWIND part: D = (1-eta) D_central + eta D_upwind
 *    (eq 4.8 and Table 1; eq 2.36 prints the weights swapped);
 *  - the upwind formula's second branch reads f(chi + 2 dchi);
 *  - gradients are taken in node-index space and scaled by the metric
 *    1/x'(i), x'(i) = (x[i+1] - x[i-1]) / 2 (period added across a periodic
 *    seam), the curvilinear form behind eq 2.27's chi;
 *  - at the first interior node next to a wall, the missing upwind point is
 *    a quadratic ghost  f[-1] = 3 f[0] - 3 f[1] + f[2];
 *  - intermediate moments rho* = sum fbar*, rho* u* = sum xi fbar* + (h/2) rho* F
 *    (the h analogue of eq 3.3);
 *  - non-equilibrium extrapolation is applied to f(t*) after it is formed and
 *    to f~^{n+1} after the update, from the nearest interior node along the
 *    wall normal (diagonal at corners); corners belong to the x-walls.
 *
 * Representation: every population array holds  value - offset * w_q.
 * offset = 0 is the paper's absolute f~; offset = 1 carries the departure
 * from the rest state.  Every pointwise map below is an affine combination
 * whose coefficients sum to one and the difference operator annihilates
 * constants, so the offset cancels identically; it only moves FP64 rounding
 * from the scale of w_q to the scale of the flow.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define Q 9

/* D2Q9 velocities and weights in the order printed in Sec. 3. */
static const int EX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                            1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0;

typedef struct {
  int nx, ny;
  int per_x, per_y;
  double *mx, *my;     /* metric 1/x'(i), 1/y'(j); 0 on wall nodes */
  double dt, inv_tau;  /* inv_tau = 0 means no collision (tau -> infinity) */
  double A, eta;
  double Fx, Fy;       /* body-force acceleration */
  double uw[4][2];     /* wall velocity: left, right, bottom, top */
  double offset;
} grid_t;

#define IDX(g, q, i, j) (((size_t)(q) * (g)->ny + (size_t)(j)) * (g)->nx + (size_t)(i))

/* ---------------------------------------------------------------- lattice */

/* Equilibrium eq 3.2 minus offset*w_q, from d = rho - offset and u. */
static double feq_minus_offset(int q, double d, double rho, double ux, double uy) {
  double eu = EX[q] * ux + EY[q] * uy;
  double uu = ux * ux + uy * uy;
  double x = eu / CS2 + (eu * eu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2);
  return W[q] * (d + rho * x);
}

/* Guo force term eq 3.12 with RT = c_s^2. */
static double force_term(int q, double rho, double ux, double uy, double feq_abs,
                         const grid_t* g) {
  (void)rho;
  double fx = g->Fx * (EX[q] - ux) + g->Fy * (EY[q] - uy);
  return fx * feq_abs / CS2;
}

/* Moments of eq 3.3 at one node of an array stored minus offset*w.
 * shift is the half-step force shift (dt/2 for f~, h/2 for fbar(t*), 0 for f). */
static void moments(const grid_t* g, const double* a, int i, int j, double shift,
                    double* d, double* rho, double* ux, double* uy) {
  double s = 0.0, jx = 0.0, jy = 0.0;
  for (int q = 0; q < Q; ++q) {
    double v = a[IDX(g, q, i, j)];
    s += v;
    jx += EX[q] * v;
    jy += EY[q] * v;
  }
  *d = s;
  *rho = s + g->offset;
  *ux = jx / *rho + shift * g->Fx;
  *uy = jy / *rho + shift * g->Fy;
}

/* ------------------------------------------------------------------- mesh */

static int is_wall(const grid_t* g, int i, int j) {
  if (!g->per_x && (i == 0 || i == g->nx - 1)) return 1;
  if (!g->per_y && (j == 0 || j == g->ny - 1)) return 1;
  return 0;
}

/* Wall velocity; x-walls own the corners. */
static void wall_velocity(const grid_t* g, int i, int j, double* ub, double* vb) {
  int side;
  if (!g->per_x && i == 0) side = 0;
  else if (!g->per_x && i == g->nx - 1) side = 1;
  else if (!g->per_y && j == 0) side = 2;
  else side = 3;
  *ub = g->uw[side][0];
  *vb = g->uw[side][1];
}

/* Nearest interior node along the wall normal (diagonal at corners). */
static void fluid_neighbour(const grid_t* g, int i, int j, int* fi, int* fj) {
  *fi = i;
  *fj = j;
  if (!g->per_x) {
    if (i == 0) *fi = 1;
    if (i == g->nx - 1) *fi = g->nx - 2;
  }
  if (!g->per_y) {
    if (j == 0) *fj = 1;
    if (j == g->ny - 1) *fj = g->ny - 2;
  }
}

static void metric(int n, const double* c, int per, double period, double* m) {
  for (int i = 0; i < n; ++i) {
    if (per) {
      double cm = (i == 0) ? c[n - 1] - period : c[i - 1];
      double cp = (i == n - 1) ? c[0] + period : c[i + 1];
      m[i] = 1.0 / ((cp - cm) / 2.0);
    } else if (i == 0 || i == n - 1) {
      m[i] = 0.0;
    } else {
      m[i] = 1.0 / ((c[i + 1] - c[i - 1]) / 2.0);
    }
  }
}

/* ------------------------------------------------------- mixed difference */

/* Value of population q of array a at index k along one axis (the other index
 * fixed).  Periodic axes wrap; on a walled axis the single missing point of an
 * upwind stencil next to the wall is the quadratic ghost value. */
static double along(const grid_t* g, const double* a, int q, int i, int j, int axis,
                    int k) {
  int n = axis == 0 ? g->nx : g->ny;
  int per = axis == 0 ? g->per_x : g->per_y;
  if (per) {
    k = ((k % n) + n) % n;
  } else if (k < 0) {
    return 3.0 * along(g, a, q, i, j, axis, 0) - 3.0 * along(g, a, q, i, j, axis, 1) +
           along(g, a, q, i, j, axis, 2);
  } else if (k > n - 1) {
    return 3.0 * along(g, a, q, i, j, axis, n - 1) -
           3.0 * along(g, a, q, i, j, axis, n - 2) + along(g, a, q, i, j, axis, n - 3);
  }
  return axis == 0 ? a[IDX(g, q, k, j)] : a[IDX(g, q, i, k)];
}

/* Mixed difference d f / d chi (index space, unit spacing) of eqs 2.36-2.38
 * for a population whose velocity component along the axis has sign s. */
static double mixed_index_derivative(const grid_t* g, const double* a, int q, int i,
                                     int j, int axis, int s) {
  int c = axis == 0 ? i : j;
  double fm2 = along(g, a, q, i, j, axis, c - 2);
  double fm1 = along(g, a, q, i, j, axis, c - 1);
  double f0 = along(g, a, q, i, j, axis, c);
  double fp1 = along(g, a, q, i, j, axis, c + 1);
  double fp2 = along(g, a, q, i, j, axis, c + 2);
  double central = (fp1 - fm1) / 2.0;
  double upwind;
  if (s > 0)
    upwind = (3.0 * f0 - 4.0 * fm1 + fm2) / 2.0;
  else
    upwind = -(3.0 * f0 - 4.0 * fp1 + fp2) / 2.0;
  return (1.0 - g->eta) * central + g->eta * upwind;
}

/* Gradient term L(f) = -xi . grad f (eq 2.27), physical derivative by the
 * chain rule d/dx = (1/x'(i)) d/di. */
static double L_term(const grid_t* g, const double* a, int q, int i, int j) {
  double r = 0.0;
  if (EX[q] != 0)
    r -= EX[q] * g->mx[i] * mixed_index_derivative(g, a, q, i, j, 0, EX[q]);
  if (EY[q] != 0)
    r -= EY[q] * g->my[j] * mixed_index_derivative(g, a, q, i, j, 1, EY[q]);
  return r;
}

/* ------------------------------------------------------ pointwise stages */

/* From f~ at every node: physical f (eq 2.19 solved for f), then
 * fbar^{+,hs} = f + (hs/2) Omega_bar (eq 2.34) and f~^+ = f + (dt/2) Omega_bar
 * (eq 2.20).  Either output may be NULL. */
static void collide_all(const grid_t* g, const double* ft, double hs, double* fbp,
                        double* ftp) {
  const double dt = g->dt, it = g->inv_tau;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < g->ny; ++j)
    for (int i = 0; i < g->nx; ++i) {
      double d, rho, ux, uy;
      moments(g, ft, i, j, dt / 2.0, &d, &rho, &ux, &uy);
      for (int q = 0; q < Q; ++q) {
        double feq = feq_minus_offset(q, d, rho, ux, uy);
        double Fq = force_term(q, rho, ux, uy, feq + g->offset * W[q], g);
        double v = ft[IDX(g, q, i, j)];
        /* f~ = f - (dt/2)[-(f - feq) it + F]  =>  f (2 + dt it) = 2 f~ + dt it feq + dt F */
        double f = (2.0 * v + dt * it * feq + dt * Fq) / (2.0 + dt * it);
        double omega_bar = -(f - feq) * it + Fq;
        if (fbp) fbp[IDX(g, q, i, j)] = f + (hs / 2.0) * omega_bar;
        if (ftp) ftp[IDX(g, q, i, j)] = f + (dt / 2.0) * omega_bar;
      }
    }
}

/* Half-step prediction along characteristics, eqs 2.33 and 2.35:
 * fbar(t + hs) = fbar^{+,hs} - hs xi . grad fbar^{+,hs}, at interior nodes. */
static void advect_interior(const grid_t* g, const double* fbp, double hs, double* fb) {
#pragma omp parallel for schedule(static)
  for (int j = 0; j < g->ny; ++j)
    for (int i = 0; i < g->nx; ++i) {
      if (is_wall(g, i, j)) continue;
      for (int q = 0; q < Q; ++q)
        fb[IDX(g, q, i, j)] = fbp[IDX(g, q, i, j)] + hs * L_term(g, fbp, q, i, j);
    }
}

/* Physical f at t + hs from fbar(t + hs), eq 2.32, with moments whose force
 * shift is hs/2, at interior nodes. */
static void unshift_interior(const grid_t* g, const double* fb, double hs, double* fs) {
  const double it = g->inv_tau;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < g->ny; ++j)
    for (int i = 0; i < g->nx; ++i) {
      if (is_wall(g, i, j)) continue;
      double d, rho, ux, uy;
      moments(g, fb, i, j, hs / 2.0, &d, &rho, &ux, &uy);
      for (int q = 0; q < Q; ++q) {
        double feq = feq_minus_offset(q, d, rho, ux, uy);
        double Fq = force_term(q, rho, ux, uy, feq + g->offset * W[q], g);
        /* f = [2 tau fbar + h feq + h tau F] / (2 tau + h), divided through by tau */
        fs[IDX(g, q, i, j)] =
            (2.0 * fb[IDX(g, q, i, j)] + hs * it * feq + hs * Fq) / (2.0 + hs * it);
      }
    }
}

/* Non-equilibrium extrapolation, eq 3.10, on the wall nodes of array a.
 * shift is the force shift of a's momentum (dt/2 for f~, 0 for physical f). */
static void nee_walls(const grid_t* g, double* a, double shift) {
  if (g->per_x && g->per_y) return;
  for (int j = 0; j < g->ny; ++j)
    for (int i = 0; i < g->nx; ++i) {
      if (!is_wall(g, i, j)) continue;
      int fi, fj;
      double d, rho, ux, uy, ub, vb;
      fluid_neighbour(g, i, j, &fi, &fj);
      wall_velocity(g, i, j, &ub, &vb);
      moments(g, a, fi, fj, shift, &d, &rho, &ux, &uy);
      for (int q = 0; q < Q; ++q) {
        double feq_b = feq_minus_offset(q, d, rho, ub, vb);
        double feq_f = feq_minus_offset(q, d, rho, ux, uy);
        a[IDX(g, q, i, j)] = feq_b + (a[IDX(g, q, fi, fj)] - feq_f);
      }
    }
}

/* f~^{n+1} = base + c * dt * L(a) at interior nodes (base is f~^+). */
static void update_interior(const grid_t* g, const double* base, const double* a,
                            double c, double* out) {
#pragma omp parallel for schedule(static)
  for (int j = 0; j < g->ny; ++j)
    for (int i = 0; i < g->nx; ++i) {
      if (is_wall(g, i, j)) continue;
      for (int q = 0; q < Q; ++q)
        out[IDX(g, q, i, j)] = base[IDX(g, q, i, j)] + c * g->dt * L_term(g, a, q, i, j);
    }
}

/* -------------------------------------------------------------- schemes */

/* T2S2-FDLBM1 (and T1S2 at A = 0): Sec. 2D steps (1)-(3), eq 2.23. */
static void step_fdlbm1(const grid_t* g, double* ft, double* P, double* Qp, double* S,
                        double* R) {
  const double h = g->A * g->dt;
  size_t n = (size_t)Q * g->nx * g->ny;
  collide_all(g, ft, h, P, Qp);      /* P = fbar^{+,h}(t_n), Qp = f~^{+,n} */
  memcpy(S, P, n * sizeof(double));  /* wall entries are replaced below */
  advect_interior(g, P, h, S);       /* S = fbar(t*) */
  memcpy(R, S, n * sizeof(double));
  unshift_interior(g, S, h, R);      /* R = f(t*) */
  nee_walls(g, R, 0.0);
  memcpy(ft, Qp, n * sizeof(double));
  update_interior(g, Qp, R, 1.0, ft); /* f~^{n+1} = f~^+ + dt L(f*) */
  nee_walls(g, ft, g->dt / 2.0);
}

/* T2S2-FDLBM2: Sec. 2D steps (1)-(3) of the second sequence, eq 5.23.
 * With h = dt, fbar = f~ and fbar^{+,h} = f~^+. */
static void step_fdlbm2(const grid_t* g, double* ft, double* Fn, double* Qp, double* S,
                        double* R) {
  const double dt = g->dt;
  size_t n = (size_t)Q * g->nx * g->ny;
  /* step (1): f^n from f~^n (eq 2.52 with h = dt, i.e. eq 2.19 solved for f) */
  collide_all(g, ft, 0.0, Fn, Qp); /* fbar^{+,0} = f itself, at every node */
  /* step (2): f~^+ -> fbar(t_{n+1}) -> f(t_{n+1}) */
  memcpy(S, Qp, n * sizeof(double));
  advect_interior(g, Qp, dt, S);
  memcpy(R, S, n * sizeof(double));
  unshift_interior(g, S, dt, R);
  nee_walls(g, R, 0.0);
  /* step (3): f~^{n+1} = f~^+ + dt/2 (L(f^n) + L(f^{n+1})) */
  double* out = ft;
  memcpy(out, Qp, n * sizeof(double));
  update_interior(g, Qp, Fn, 0.5, out);
  /* second half: add dt/2 L(f^{n+1}) at interior nodes */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < g->ny; ++j)
    for (int i = 0; i < g->nx; ++i) {
      if (is_wall(g, i, j)) continue;
      for (int q = 0; q < Q; ++q)
        out[IDX(g, q, i, j)] += 0.5 * dt * L_term(g, R, q, i, j);
    }
  nee_walls(g, out, dt / 2.0);
}

/* Collision term of eq 2.4 with the force of eq 3.12,
 *   Omega_bar(f) = -(f - f^eq) / tau + F,
 * of an array of physical f at every node; f^eq and F from f's own moments
 * (a physical f carries its whole momentum: no force shift). */
static void collision_all(const grid_t* g, const double* a, double* om) {
  const double it = g->inv_tau;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < g->ny; ++j)
    for (int i = 0; i < g->nx; ++i) {
      double d, rho, ux, uy;
      moments(g, a, i, j, 0.0, &d, &rho, &ux, &uy);
      for (int q = 0; q < Q; ++q) {
        double feq = feq_minus_offset(q, d, rho, ux, uy);
        double Fq = force_term(q, rho, ux, uy, feq + g->offset * W[q], g);
        om[IDX(g, q, i, j)] = -(a[IDX(g, q, i, j)] - feq) * it + Fq;
      }
    }
}

/* The implicit collision weight B-2 of eq 2.13, solved node by node.  On
 * entry y holds Y = f^{n+1} - b2 dt Omega_bar(f^{n+1}) at the interior nodes.
 * Omega_bar conserves mass and adds rho F to the momentum, so f^{n+1} has
 * the density of Y and the velocity  u = sum xi Y / rho + b2 dt F; with f^eq
 * and F at (rho, u),
 *   f^{n+1} = [Y + b2 dt (f^eq / tau + F)] / (1 + b2 dt / tau).
 * On exit y holds the state f~^{n+1} = f^{n+1} - (dt/2) Omega_bar(f^{n+1})
 * of eq 2.19 there. */
static void implicit_collision_interior(const grid_t* g, double b2, double* y) {
  const double dt = g->dt, it = g->inv_tau;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < g->ny; ++j)
    for (int i = 0; i < g->nx; ++i) {
      if (is_wall(g, i, j)) continue;
      double d, rho, ux, uy;
      moments(g, y, i, j, b2 * dt, &d, &rho, &ux, &uy);
      for (int q = 0; q < Q; ++q) {
        double feq = feq_minus_offset(q, d, rho, ux, uy);
        double Fq = force_term(q, rho, ux, uy, feq + g->offset * W[q], g);
        double f = (y[IDX(g, q, i, j)] + b2 * dt * (feq * it + Fq)) / (1.0 + b2 * dt * it);
        double omega_bar = -(f - feq) * it + Fq;
        y[IDX(g, q, i, j)] = f - (dt / 2.0) * omega_bar;
      }
    }
}

/* The eq 2.13 family with gradient weights bt = (B~0, B~1, B~2) and
 * collision weights bb = (B-0, B-1, B-2):
 *   f^{n+1} - B-2 dt Omega_bar(f^{n+1})
 *     = f^n + dt [B-0 Omega_bar(f^n) + B-1 Omega_bar(f*)]
 *       + dt [B~0 L(f^n) + B~1 L(f*) + B~2 L(f^{n+1})].
 * Each argument on the right is the paper's own prediction of it: f* by
 * step (1) of the T2S2-FDLBM1 sequence (h = A dt), f^{n+1} by step (2) of
 * the T2S2-FDLBM2 sequence (h = dt), f^n by eq 2.52 at h = 0 (step (1) of
 * the second sequence).  The left side is solved node by node
 * (implicit_collision_interior) and the state stays f~ = f - (dt/2)
 * Omega_bar (eq 2.19).
 * bb = NULL takes the collision weights of eqs 2.21 and 5.21,
 * (1/2, 0, 1/2), in the explicit form of eqs 2.19-2.20 that they allow:
 *   f~^{n+1} = f~^{+,n} + dt [B~0 L(f^n) + B~1 L(f*) + B~2 L(f^{n+1})];
 * bt = (0, 1, 0) is then eq 2.23, (1/2, 0, 1/2) eq 5.23 and (1, 0, 0)
 * eq 2.18.  Om0 and Om1 are used only with bb. */
static void step_family(const grid_t* g, const double bt[3], const double* bb, double* ft,
                        double* P, double* Fn, double* Qp, double* S, double* R1, double* R2,
                        double* Om0, double* Om1) {
  const double h = g->A * g->dt, dt = g->dt;
  size_t n = (size_t)Q * g->nx * g->ny;
  collide_all(g, ft, h, P, Qp);      /* P = fbar^{+,h}(t_n), Qp = f~^{+,n} */
  collide_all(g, ft, 0.0, Fn, NULL); /* f^n */
  /* f(t*) from P along the characteristics, h = A dt */
  memcpy(S, P, n * sizeof(double));
  advect_interior(g, P, h, S);
  memcpy(R1, S, n * sizeof(double));
  unshift_interior(g, S, h, R1);
  nee_walls(g, R1, 0.0);
  /* f(t_{n+1}) from f~^+ along the characteristics, h = dt */
  memcpy(S, Qp, n * sizeof(double));
  advect_interior(g, Qp, dt, S);
  memcpy(R2, S, n * sizeof(double));
  unshift_interior(g, S, dt, R2);
  nee_walls(g, R2, 0.0);
  if (bb) {
    collision_all(g, Fn, Om0); /* Omega_bar(f^n) */
    collision_all(g, R1, Om1); /* Omega_bar(f*) */
  }
  memcpy(ft, Qp, n * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int j = 0; j < g->ny; ++j)
    for (int i = 0; i < g->nx; ++i) {
      if (is_wall(g, i, j)) continue;
      for (int q = 0; q < Q; ++q) {
        size_t k = IDX(g, q, i, j);
        double l = bt[0] * L_term(g, Fn, q, i, j) + bt[1] * L_term(g, R1, q, i, j) +
                   bt[2] * L_term(g, R2, q, i, j);
        if (bb)
          ft[k] = Fn[k] + dt * (bb[0] * Om0[k] + bb[1] * Om1[k]) + dt * l;
        else
          ft[k] = Qp[k] + dt * l;
      }
    }
  if (bb) implicit_collision_interior(g, bb[2], ft);
  nee_walls(g, ft, dt / 2.0);
}

/* ------------------------------------------------------------ public API */

/* Advance phi (= f~ - offset*w, layout [9][ny][nx]) by nsteps.
 * nu_inv_tau: 1/tau (0 = collisionless).  u_wall: [4][2] left,right,bottom,top.
 * scheme: 1 = T2S2-FDLBM1 family (A selects h = A dt), 2 = T2S2-FDLBM2.
 * Returns 0 on success, 1 on bad arguments, 2 on allocation failure. */
static int run_impl(int nx, int ny, const double* x, const double* y, int per_x, int per_y,
                    double period_x, double period_y, double dt, double inv_tau, double A,
                    double eta, double Fx, double Fy, const double* u_wall, double offset,
                    int scheme, const double* bt, const double* bb, double* phi,
                    long nsteps) {
  if (nx < 5 || ny < 5 || dt <= 0.0 || inv_tau < 0.0 || !phi || !x || !y) return 1;
  if (scheme != 1 && scheme != 2 && !(scheme == 3 && bt)) return 1;
  grid_t g;
  memset(&g, 0, sizeof g);
  g.nx = nx;
  g.ny = ny;
  g.per_x = per_x;
  g.per_y = per_y;
  g.dt = dt;
  g.inv_tau = inv_tau;
  g.A = A;
  g.eta = eta;
  g.Fx = Fx;
  g.Fy = Fy;
  g.offset = offset;
  if (u_wall)
    for (int s = 0; s < 4; ++s) {
      g.uw[s][0] = u_wall[2 * s];
      g.uw[s][1] = u_wall[2 * s + 1];
    }
  size_t n = (size_t)Q * nx * ny;
  g.mx = (double*)malloc(nx * sizeof(double));
  g.my = (double*)malloc(ny * sizeof(double));
  double* P = (double*)malloc(n * sizeof(double));
  double* Qp = (double*)malloc(n * sizeof(double));
  double* S = (double*)malloc(n * sizeof(double));
  double* R = (double*)malloc(n * sizeof(double));
  double* Fn = scheme == 3 ? (double*)malloc(n * sizeof(double)) : NULL;
  double* R2 = scheme == 3 ? (double*)malloc(n * sizeof(double)) : NULL;
  double* Om0 = bb ? (double*)malloc(n * sizeof(double)) : NULL;
  double* Om1 = bb ? (double*)malloc(n * sizeof(double)) : NULL;
  int rc = 0;
  if (!g.mx || !g.my || !P || !Qp || !S || !R || (scheme == 3 && (!Fn || !R2)) ||
      (bb && (!Om0 || !Om1))) {
    rc = 2;
  } else {
    metric(nx, x, per_x, period_x, g.mx);
    metric(ny, y, per_y, period_y, g.my);
    for (long s = 0; s < nsteps; ++s) {
      if (scheme == 1)
        step_fdlbm1(&g, phi, P, Qp, S, R);
      else if (scheme == 2)
        step_fdlbm2(&g, phi, P, Qp, S, R);
      else
        step_family(&g, bt, bb, phi, P, Fn, Qp, S, R, R2, Om0, Om1);
    }
  }
  free(g.mx);
  free(g.my);
  free(P);
  free(Qp);
  free(S);
  free(R);
  free(Fn);
  free(R2);
  free(Om0);
  free(Om1);
  return rc;
}

int oracle_run(int nx, int ny, const double* x, const double* y, int per_x, int per_y,
               double period_x, double period_y, double dt, double inv_tau, double A,
               double eta, double Fx, double Fy, const double* u_wall, double offset,
               int scheme, double* phi, long nsteps) {
  if (scheme != 1 && scheme != 2) return 1;
  return run_impl(nx, ny, x, y, per_x, per_y, period_x, period_y, dt, inv_tau, A, eta, Fx, Fy,
                  u_wall, offset, scheme, NULL, NULL, phi, nsteps);
}

/* The eq 2.13 family (step_family) with gradient weights bt[3] and
 * collision weights bb[3] (NULL: (1/2, 0, 1/2) in the explicit form). */
int oracle_run_family(int nx, int ny, const double* x, const double* y, int per_x, int per_y,
                      double period_x, double period_y, double dt, double inv_tau, double A,
                      double eta, double Fx, double Fy, const double* u_wall, double offset,
                      const double* bt, const double* bb, double* phi, long nsteps) {
  if (!bt) return 1;
  return run_impl(nx, ny, x, y, per_x, per_y, period_x, period_y, dt, inv_tau, A, eta, Fx, Fy,
                  u_wall, offset, 3, bt, bb, phi, nsteps);
}

/* Initial populations (Sec. 3): f~ = f^eq(rho, u), optionally minus the
 * non-equilibrium part of eq 3.5,  rho0 w (2 tau + dt) / (2 c_s^2) xi xi : grad u,
 * (the printed coefficient "tau(2+dt)" read as 2 tau + dt).  grad may be NULL;
 * else it holds four [ny][nx] planes du/dx, du/dy, dv/dx, dv/dy.  rho0 = 1. */
int oracle_init(int nx, int ny, const double* rho, const double* ux, const double* uy,
                const double* grad, double tau, double dt, double offset, double* phi) {
  if (nx < 1 || ny < 1 || !rho || !ux || !uy || !phi) return 1;
  size_t plane = (size_t)nx * ny;
  for (size_t p = 0; p < plane; ++p) {
    double r = rho[p];
    for (int q = 0; q < Q; ++q) {
      double v = feq_minus_offset(q, r - offset, r, ux[p], uy[p]);
      if (grad) {
        double dudx = grad[p], dudy = grad[plane + p];
        double dvdx = grad[2 * plane + p], dvdy = grad[3 * plane + p];
        /* xi_a xi_b d_a u_b */
        double contr = EX[q] * EX[q] * dudx + EX[q] * EY[q] * (dudy + dvdx) +
                       EY[q] * EY[q] * dvdy;
        v -= 1.0 * W[q] * (2.0 * tau + dt) / (2.0 * CS2) * contr;
      }
      phi[q * plane + p] = v;
    }
  }
  return 0;
}

/* Macroscopic fields of phi with the eq 3.3 force shift dt/2:
 * drho = rho - offset, ux, uy on [ny][nx]. */
int oracle_moments(int nx, int ny, const double* phi, double offset, double dt, double Fx,
                   double Fy, double* drho, double* ux, double* uy) {
  if (nx < 1 || ny < 1 || !phi) return 1;
  size_t plane = (size_t)nx * ny;
  for (size_t p = 0; p < plane; ++p) {
    double s = 0.0, jx = 0.0, jy = 0.0;
    for (int q = 0; q < Q; ++q) {
      double v = phi[q * plane + p];
      s += v;
      jx += EX[q] * v;
      jy += EY[q] * v;
    }
    double r = s + offset;
    drho[p] = s;
    ux[p] = jx / r + dt / 2.0 * Fx;
    uy[p] = jy / r + dt / 2.0 * Fy;
  }
  return 0;
}

/* Thread count of the OpenMP stage loops; returns the count now in effect. */
int oracle_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
}
