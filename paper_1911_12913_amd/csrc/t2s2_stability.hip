// Von Neumann stability maps of the T2S2-FDLBM (Sec. 2C, eqs 4.1-4.8).
//
// For each (omega, r) point of a map, the largest spectral radius over a
// grid of modes k of the growth matrix G(k) (9 x 9, complex) of a
// perturbation f' e^{i k.x} about the uniform equilibrium f^eq(1, u):
//   model 0 (eq 4.7): G = lhs^{-1} rhs for the (B~2, B-2) family, with
//     lhs = (1 + w B-2) I + w (1/2 - 2 B-2) Gamma + rS (B~2 I + (1/2 - B~2) Gamma)
//     rhs = (1 - w (1 - B-2)) I + w (3/2 - 2 B-2) Gamma
//           - rS ((1 - B~2) I - (1/2 - B~2) Gamma);
//   model 1: the exact linearisation of the implemented eq 2.23 step (h = A
//     dt):  G = J_Q - rS J_R (I - A rS) J_P;
//   model 2: the exact linearisation of the eq 5.23 step:
//     G = J_Q - (rS/2) (J_f + J_R1 (I - rS) J_Q);
//   model 3: the exact linearisation of the eq 2.13 family step:
//     G = J_Q - rS (b0 J_f + b1 J_R (I - A rS) J_P + b2 J_R1 (I - rS) J_Q);
//     with collision weights (B-0, B-1, B-2) other than (1/2, 0, 1/2)
//     (dt Omega(f) = w (Gamma - I) f, unforced):
//     Y = J_f + w (Gamma - I) (B-0 J_f + B-1 J_R (I - A rS) J_P)
//         - rS (b0 J_f + b1 J_R (I - A rS) J_P + b2 J_R1 (I - rS) J_Q),
//     G = (aY I + aE Gamma) Y with aY = (1 + w/2) / (1 + B-2 w) and
//     aE = w (B-2 - 1/2) / (1 + B-2 w): the implicit weight solved (Gamma
//     is a projection, Gamma^2 = Gamma: f^eq keeps the moments it is built
//     from) and the state taken as f~ = f - (dt/2) Omega(f) (eq 2.19);
// with Gamma = d f^eq / d f, J_X = c_Xg I + c_Xe Gamma, and S the symbol of
// dx xi_q . D of the mixed difference (eq 4.8, imaginary unit restored in
// the exponentials).  The advection symbol multiplies from the left (it
// acts on the population it advects).
//
// One wave per map point walks the k grid; the matrices live in LDS.  The
// spectral radius is lim ||G^m||^(1/m), taken at m = 2^J by J normalised
// squarings (the log of each normalisation is accumulated), in FP64.
#include <hip/hip_runtime.h>

#include <cmath>

#include "t2s2_device.h"
#include "t2s2_internal.h"

namespace t2s2 {
namespace {

struct cplx {
  double re, im;
};
__device__ inline cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline cplx cmul(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ inline cplx cscale(cplx a, double s) { return {a.re * s, a.im * s}; }
__device__ inline double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }
__device__ inline cplx cdiv(cplx a, cplx b) {
  const double d = cabs2(b);
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

constexpr int kN = 9, kN2 = 81;

// Gamma_ij = d f^eq_i / d f_j at rho = 1, velocity u (eq 3.2, c_s^2 = 1/3):
// f^eq depends on f through rho = sum f and m = sum xi f.
__device__ inline double gamma_ij(int i, int j, double ux, double uy) {
  const double exi = ex_of(i), eyi = ey_of(i), wi = w_of(i);
  const double eu = exi * ux + eyi * uy, uu = ux * ux + uy * uy;
  const double d_rho = wi * (1.0 - 4.5 * eu * eu + 1.5 * uu);
  const double d_mx = wi * (3.0 * exi + 9.0 * eu * exi - 3.0 * ux);
  const double d_my = wi * (3.0 * eyi + 9.0 * eu * eyi - 3.0 * uy);
  return d_rho + d_mx * ex_of(j) + d_my * ey_of(j);
}

// dx * symbol of xi_q . D, mixed difference with upwind weight eta.
__device__ inline cplx symbol_q(int q, double thx, double thy, double eta) {
  cplx s{0.0, 0.0};
  const double th[2] = {thx * ex_of(q), thy * ey_of(q)};
  for (int a = 0; a < 2; ++a) {
    const double t = th[a];
    s.im += (1.0 - eta) * sin(t);
    s.re += 0.5 * eta * (3.0 - 4.0 * cos(t) + cos(2.0 * t));
    s.im += 0.5 * eta * (4.0 * sin(t) - sin(2.0 * t));
  }
  return s;
}

// One pass over the (up to two) matrix elements e = lane, lane + 64 of a
// 9 x 9 matrix.
template <typename F>
__device__ inline void for_elems(int lane, F f) {
  f(lane / kN, lane % kN);
  if (lane + 64 < kN2) f((lane + 64) / kN, (lane + 64) % kN);
}

__global__ __launch_bounds__(64) void stability_kernel(StabArgs a, const double* omega_p,
                                                        const double* r_p, double* radius) {
  __shared__ double gam[kN2];
  __shared__ cplx X[kN2], T[kN2], T2[kN2], U[kN2];
  __shared__ cplx sym[kN];
  const int lane = threadIdx.x;
  const int point = blockIdx.x;
  for (int e = lane; e < kN2; e += 64) gam[e] = gamma_ij(e / kN, e % kN, a.ux, a.uy);
  const double w = omega_p[point], r = r_p[point];
  // collision-map coefficients
  const double A = a.A;
  const double cPg = (2 - A * w) / (2 + w), cPe = (1 + A) * w / (2 + w);
  const double cQg = (2 - w) / (2 + w), cQe = 2 * w / (2 + w);
  const double cRs = a.model == 2 ? 2 / (2 + w) : 2 / (2 + A * w);
  const double cRe = a.model == 2 ? w / (2 + w) : A * w / (2 + A * w);
  const double cFg = 2 / (2 + w), cFe = w / (2 + w);  // f from f~ (A = 0); R at h = dt
  __syncthreads();

  double best = 0.0;
  const int nk = a.nkx * a.nky;
  for (int kk = 0; kk < nk; ++kk) {
    const double thx = a.thx0 + (kk / a.nky) * a.dthx;
    const double thy = (kk % a.nky) * a.dthy;
    if (lane < kN) sym[lane] = symbol_q(lane, thx, thy, a.eta);
    __syncthreads();

    if (a.model == 0) {
      // lhs in X, rhs in T; Gauss-Jordan with partial pivoting: T <- X^-1 T.
      const double b2 = a.b2bar, bt = a.b2tilde;
      for_elems(lane, [&](int i, int j) {
        const double d = i == j ? 1.0 : 0.0, g = gam[i * kN + j];
        const cplx rs = cscale(sym[i], r);
        X[i * kN + j] = cadd({(1 + w * b2) * d + w * (0.5 - 2 * b2) * g, 0.0},
                             cscale(rs, bt * d + (0.5 - bt) * g));
        T[i * kN + j] = csub({(1 - w * (1 - b2)) * d + w * (1.5 - 2 * b2) * g, 0.0},
                             cscale(rs, (1 - bt) * d - (0.5 - bt) * g));
      });
      __syncthreads();
      for (int c = 0; c < kN; ++c) {
        int piv = c;
        double pmax = cabs2(X[c * kN + c]);
        for (int i = c + 1; i < kN; ++i) {
          const double v = cabs2(X[i * kN + c]);
          if (v > pmax) {
            pmax = v;
            piv = i;
          }
        }
        __syncthreads();
        if (lane < kN && piv != c) {
          const cplx x0 = X[c * kN + lane], t0 = T[c * kN + lane];
          X[c * kN + lane] = X[piv * kN + lane];
          T[c * kN + lane] = T[piv * kN + lane];
          X[piv * kN + lane] = x0;
          T[piv * kN + lane] = t0;
        }
        __syncthreads();
        const cplx p = X[c * kN + c];
        __syncthreads();
        if (lane < kN) {
          X[c * kN + lane] = cdiv(X[c * kN + lane], p);
          T[c * kN + lane] = cdiv(T[c * kN + lane], p);
        }
        __syncthreads();
        cplx fac[2], xr[2], tr[2];
        int n = 0;
        for_elems(lane, [&](int i, int j) {
          fac[n] = X[i * kN + c];
          xr[n] = X[c * kN + j];
          tr[n] = T[c * kN + j];
          ++n;
        });
        __syncthreads();
        n = 0;
        for_elems(lane, [&](int i, int j) {
          if (i != c) {
            X[i * kN + j] = csub(X[i * kN + j], cmul(fac[n], xr[n]));
            T[i * kN + j] = csub(T[i * kN + j], cmul(fac[n], tr[n]));
          }
          ++n;
        });
        __syncthreads();
      }
      // G in T; copy to X
      for_elems(lane, [&](int i, int j) { X[i * kN + j] = T[i * kN + j]; });
      __syncthreads();
    } else if (a.model == 3) {
      // T = (I - A rS) J_P, T2 = (I - rS) J_Q; then
      // X = J_Q - rS (b0 J_f + b1 J_R T + b2 J_R1 T2), J_R1 = cFg I + cFe Gamma.
      for_elems(lane, [&](int i, int j) {
        const double d = i == j ? 1.0 : 0.0, g = gam[i * kN + j];
        T[i * kN + j] = cscale(csub({1.0, 0.0}, cscale(sym[i], A * r)), cPg * d + cPe * g);
        T2[i * kN + j] = cscale(csub({1.0, 0.0}, cscale(sym[i], r)), cQg * d + cQe * g);
      });
      __syncthreads();
      for_elems(lane, [&](int i, int j) {
        cplx m1{0.0, 0.0}, m2{0.0, 0.0};
        for (int k = 0; k < kN; ++k) {
          const double dk = i == k ? 1.0 : 0.0, gk = gam[i * kN + k];
          m1 = cadd(m1, cscale(T[k * kN + j], cRs * dk + cRe * gk));
          m2 = cadd(m2, cscale(T2[k * kN + j], cFg * dk + cFe * gk));
        }
        const double d = i == j ? 1.0 : 0.0, g = gam[i * kN + j];
        cplx m = cadd(cscale(m1, a.bt[1]), cscale(m2, a.bt[2]));
        m = cadd(m, {a.bt[0] * (cFg * d + cFe * g), 0.0});
        // The base: J_Q, or J_f with the collision weights' terms added below.
        const double base = a.gen_bb ? cFg * d + cFe * g : cQg * d + cQe * g;
        X[i * kN + j] = csub({base, 0.0}, cmul(cscale(sym[i], r), m));
        U[i * kN + j] = m1;  // J_R (I - A rS) J_P, the Jacobian of f*
      });
      __syncthreads();
      if (a.gen_bb) {
        // X += w (Gamma - I) (B-0 J_f + B-1 U)
        for_elems(lane, [&](int i, int j) {
          cplx acc{0.0, 0.0};
          for (int k = 0; k < kN; ++k) {
            const double gik = gam[i * kN + k] - (i == k ? 1.0 : 0.0);
            const double jf = cFg * (k == j ? 1.0 : 0.0) + cFe * gam[k * kN + j];
            acc = cadd(acc, cscale(cadd({a.bb[0] * jf, 0.0}, cscale(U[k * kN + j], a.bb[1])), gik));
          }
          X[i * kN + j] = cadd(X[i * kN + j], cscale(acc, w));
        });
        __syncthreads();
        // G = (aY I + aE Gamma) X
        const double aY = (1 + 0.5 * w) / (1 + a.bb[2] * w);
        const double aE = w * (a.bb[2] - 0.5) / (1 + a.bb[2] * w);
        for_elems(lane, [&](int i, int j) {
          cplx acc{0.0, 0.0};
          for (int k = 0; k < kN; ++k)
            acc = cadd(acc, cscale(X[k * kN + j], aY * (i == k ? 1.0 : 0.0) + aE * gam[i * kN + k]));
          T[i * kN + j] = acc;
        });
        __syncthreads();
        for_elems(lane, [&](int i, int j) { X[i * kN + j] = T[i * kN + j]; });
        __syncthreads();
      }
    } else {
      // T = (I - c rS) J, with (c, J) = (A, J_P) for model 1 and (1, J_Q) for model 2.
      const double cs = a.model == 1 ? A : 1.0;
      const double jg = a.model == 1 ? cPg : cQg, je = a.model == 1 ? cPe : cQe;
      for_elems(lane, [&](int i, int j) {
        const double J = jg * (i == j ? 1.0 : 0.0) + je * gam[i * kN + j];
        const cplx f = csub({1.0, 0.0}, cscale(sym[i], cs * r));
        T[i * kN + j] = cscale(f, J);
      });
      __syncthreads();
      // X = J_Q - c2 rS (J_extra + J_R T)
      for_elems(lane, [&](int i, int j) {
        cplx m{0.0, 0.0};
        for (int k = 0; k < kN; ++k) {
          const double jr = cRs * (i == k ? 1.0 : 0.0) + cRe * gam[i * kN + k];
          m = cadd(m, cscale(T[k * kN + j], jr));
        }
        const double d = i == j ? 1.0 : 0.0, g = gam[i * kN + j];
        if (a.model == 2) m = cadd(m, {cFg * d + cFe * g, 0.0});
        const double c2 = a.model == 2 ? 0.5 * r : r;
        X[i * kN + j] = csub({cQg * d + cQe * g, 0.0}, cmul(cscale(sym[i], c2), m));
      });
      __syncthreads();
    }

    // Spectral radius by normalised squaring.
    double c2 = 0.0;
    for_elems(lane, [&](int i, int j) { c2 = fmax(c2, cabs2(X[i * kN + j])); });
    c2 = wave_max(c2);
    double ell = 0.5 * log(c2);  // log ||G||_max
    bool zero = !(c2 > 0.0);
    {
      const double inv = zero ? 0.0 : 1.0 / sqrt(c2);
      for_elems(lane, [&](int i, int j) { X[i * kN + j] = cscale(X[i * kN + j], inv); });
    }
    __syncthreads();
    for (int s = 0; s < a.squarings && !zero; ++s) {
      cplx v[2];
      int n = 0;
      double m2 = 0.0;
      for_elems(lane, [&](int i, int j) {
        cplx acc{0.0, 0.0};
        for (int k = 0; k < kN; ++k) acc = cadd(acc, cmul(X[i * kN + k], X[k * kN + j]));
        v[n++] = acc;
        m2 = fmax(m2, cabs2(acc));
      });
      m2 = wave_max(m2);
      __syncthreads();
      zero = !(m2 > 0.0);
      const double inv = zero ? 0.0 : 1.0 / sqrt(m2);
      n = 0;
      for_elems(lane, [&](int i, int j) { X[i * kN + j] = cscale(v[n++], inv); });
      ell = 2.0 * ell + (zero ? 0.0 : 0.5 * log(m2));
      __syncthreads();
    }
    const double rho = zero ? 0.0 : exp(ldexp(ell, -a.squarings));
    best = fmax(best, rho);
  }
  if (lane == 0) radius[point] = best;
}

}  // namespace

hipError_t launch_stability(const StabArgs& a, const double* omega, const double* r, int npoints,
                            double* radius, hipStream_t s) {
  hipLaunchKernelGGL(stability_kernel, dim3(npoints), dim3(64), 0, s, a, omega, r, radius);
  return hipGetLastError();
}

}  // namespace t2s2
