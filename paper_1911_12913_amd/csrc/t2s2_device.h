// Device helpers shared by the step and adjoint kernels: the D2Q9 lattice,
// storage conversions, the equilibrium and its neighbours.  Internal linkage
// (anonymous namespace) in every translation unit that includes it.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "t2s2_internal.h"

namespace t2s2 {
namespace {

__host__ __device__ constexpr int ex_of(int q) {
  return (q == 1 || q == 5 || q == 8) ? 1 : ((q == 3 || q == 6 || q == 7) ? -1 : 0);
}
__host__ __device__ constexpr int ey_of(int q) {
  return (q == 2 || q == 5 || q == 6) ? 1 : ((q == 4 || q == 7 || q == 8) ? -1 : 0);
}
__host__ __device__ constexpr double w_of(int q) {
  return q == 0 ? 4.0 / 9.0 : (q < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
}

template <typename S>
struct Cvt;
template <>
struct Cvt<double> {
  using R = double;
  __device__ static double ld(double v) { return v; }
  __device__ static double st(double v) { return v; }
};
template <>
struct Cvt<float> {
  using R = float;
  __device__ static float ld(float v) { return v; }
  __device__ static float st(float v) { return v; }
};
// BF16 as raw bits: widening is a 16-bit shift; narrowing rounds to nearest
// even, with gfx950's conversion instruction (v_cvt_pk_bf16_f32).
struct Bf16 {
  unsigned short bits;
};
template <>
struct Cvt<Bf16> {
  using R = float;
  __device__ static float ld(Bf16 v) { return __uint_as_float(static_cast<unsigned>(v.bits) << 16); }
  __device__ static Bf16 st(float v) {
    return Bf16{__builtin_bit_cast(unsigned short, static_cast<__bf16>(v))};
  }
};
// FP16 holds the deviation times 2^14 (kF16Scale): the multiplications by
// a power of two are exact, and deviations down to about 4e-9 stay normal
// FP16 numbers (unscaled, everything below 6.1e-5 would be subnormal, with
// an absolute spacing of 6e-8, and below 3e-8 zero).  A stored value
// overflows only for |g| >= 4, far outside a physical state
// (-w_q < g_q < rho - w_q).
constexpr float kF16Scale = 16384.0f;
template <>
struct Cvt<_Float16> {
  using R = float;
  __device__ static float ld(_Float16 v) { return static_cast<float>(v) * (1.0f / kF16Scale); }
  __device__ static _Float16 st(float v) { return static_cast<_Float16>(v * kF16Scale); }  // RNE
};

// The stochastically rounded 16-bit forms: the same bits as Bf16 and
// _Float16 storage (FP16 with the 2^14 scale), read the same way; the new
// interior values a step stores are rounded stochastically (round_node_sr
// below), every other store (initialisation, wall nodes) to nearest even.
struct Bf16Sr {
  unsigned short bits;
};
struct F16Sr {
  _Float16 v;
};
template <>
struct Cvt<Bf16Sr> {
  using R = float;
  __device__ static float ld(Bf16Sr v) { return Cvt<Bf16>::ld(Bf16{v.bits}); }
  __device__ static Bf16Sr st(float v) { return Bf16Sr{Cvt<Bf16>::st(v).bits}; }
};
template <>
struct Cvt<F16Sr> {
  using R = float;
  __device__ static float ld(F16Sr v) { return Cvt<_Float16>::ld(v.v); }
  __device__ static F16Sr st(float v) { return F16Sr{Cvt<_Float16>::st(v)}; }
};
template <typename S>
constexpr bool kStochastic = std::is_same<S, Bf16Sr>::value || std::is_same<S, F16Sr>::value;
// BF16 bits, either rounding.
template <typename S>
constexpr bool kBf16Bits = std::is_same<S, Bf16>::value || std::is_same<S, Bf16Sr>::value;

// Storage code of a storage type.
template <typename S>
constexpr int kStorageOf = std::is_same<S, double>::value   ? kF64
                           : std::is_same<S, float>::value  ? kF32
                           : std::is_same<S, Bf16>::value   ? kBF16
                           : std::is_same<S, _Float16>::value ? kF16
                           : std::is_same<S, Bf16Sr>::value ? kBF16Sr
                                                            : kF16Sr;

// 32-bit integer mixing function (the "lowbias32" hash published by
// C. Wellons): every output bit depends on every input bit.
__device__ inline unsigned mix32(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// Stochastic rounding of the nine new values v of one node to 16 bits:
// value x rounds up in magnitude with probability (x - x_down) / (x_up -
// x_down), so the stored value is x on average and increments smaller than
// half a unit in the last place are kept on average instead of lost, as
// they are under rounding to nearest.  The random bits come from a counter
// generator that needs no step counter: mix32 of the node's position (pos) and of the nine values'
// FP32 bits, then a linear congruential sequence (multiplier 1664525,
// increment 1013904223, on the low 24 bits of the state) whose upper 16
// bits serve one value each.  They depend only on the node and the values,
// so results do not depend on the launch's tiling, graph replays give the
// values of plain launches, and a state that does not change rounds the
// same way again.  BF16: add 16 random bits to the FP32 bits and cut them;
// FP16: the same with 13 bits on 2^14 x, then an exact conversion (in the
// normal FP16 range; below it, 2^14 |x| < 6.1e-5, the conversion rounds to
// nearest).  Non-finite values keep their class (canonical NaNs, Inf).
template <typename S>
__device__ inline void round_node_sr(const float v[kQ], unsigned pos, S out[kQ]) {
  constexpr bool kBf = std::is_same<S, Bf16Sr>::value;
  unsigned b[kQ];
  unsigned fold = pos;
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    b[q] = __float_as_uint(kBf ? v[q] : v[q] * kF16Scale);
    fold += b[q];
  }
  unsigned st = mix32(fold);
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    st = __umul24(st, 1664525u) + 1013904223u;
    if constexpr (kBf) {
      out[q] = Bf16Sr{static_cast<unsigned short>((b[q] + (st >> 16)) >> 16)};
    } else {
      const float t = __uint_as_float((b[q] + (st >> 19)) & ~0x1FFFu);
      out[q] = F16Sr{static_cast<_Float16>(t)};
    }
  }
}

// The nine planes of a row of a [9][ny][pitch] buffer, loaded or stored at
// a 32-bit byte offset (the same for every plane) in the global
// instructions' scalar-base form: a 64-bit plane base in SGPRs plus the
// 32-bit offset in a VGPR.  The base walks from plane to plane in the
// global address space and is made opaque to the optimiser at each step
// (the asm emits nothing); otherwise the optimiser folds the plane offsets
// into one 64-bit vector address addition per plane, or keeps nine bases
// live in SGPRs.  Elements move as their bits.  base must be wave-uniform.
template <int N>
struct BitsOf;
template <>
struct BitsOf<2> {
  using T = unsigned short;
};
template <>
struct BitsOf<4> {
  using T = unsigned int;
};
template <>
struct BitsOf<8> {
  using T = unsigned long long;
};
template <typename T>
__device__ inline void load_planes(const T* base, unsigned long long plane_bytes, unsigned boff,
                                   T (&out)[kQ]) {
  using B = typename BitsOf<sizeof(T)>::T;
  auto b = (const __attribute__((address_space(1))) char*)(base);
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    asm volatile("" : "+s"(b));
    out[q] = __builtin_bit_cast(T, *(const __attribute__((address_space(1))) B*)(b + boff));
    b += plane_bytes;
  }
}
// The same walk for loads at several offsets per plane: plane_base makes
// the (wave-uniform) base opaque, next_plane steps it by one plane, and
// load_at reads one element at a 32-bit byte offset from it.
using GlobalBytes = const __attribute__((address_space(1))) char*;
template <typename T>
__device__ inline GlobalBytes plane_base(const T* base) {
  auto b = (GlobalBytes)(base);
  asm volatile("" : "+s"(b));
  return b;
}
__device__ inline GlobalBytes next_plane(GlobalBytes b, unsigned long long plane_bytes) {
  b += plane_bytes;
  asm volatile("" : "+s"(b));
  return b;
}
template <typename T>
__device__ inline T load_at(GlobalBytes b, unsigned off) {
  using B = typename BitsOf<sizeof(T)>::T;
  return __builtin_bit_cast(T, *(const __attribute__((address_space(1))) B*)(b + off));
}

// kNonTemporal: streaming stores, for data the launch does not read again.
template <bool kNonTemporal, typename T>
__device__ inline void store_planes(T* base, unsigned long long plane_bytes, unsigned boff,
                                    const T (&v)[kQ]) {
  using B = typename BitsOf<sizeof(T)>::T;
  auto b = (__attribute__((address_space(1))) char*)(base);
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    asm volatile("" : "+s"(b));
    auto p = (__attribute__((address_space(1))) B*)(b + boff);
    if constexpr (kNonTemporal)
      __builtin_nontemporal_store(__builtin_bit_cast(B, v[q]), p);
    else
      *p = __builtin_bit_cast(B, v[q]);
    b += plane_bytes;
  }
}

// Value of the neighbouring lane l-1 (from_below) or l+1 (from_above) of a
// wave64, through DPP wave shifts (two 32-bit moves for a double).  Every
// lane of the wave must hold a defined value.  bound_ctrl makes the edge
// lane (no source lane) read 0, so the move does not depend on the old
// destination value and needs no zero-fill before it.
__device__ inline int dpp_shr1(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ inline int dpp_shl1(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
__device__ inline double from_below(double v) {
  return __hiloint2double(dpp_shr1(__double2hiint(v)), dpp_shr1(__double2loint(v)));
}
__device__ inline double from_above(double v) {
  return __hiloint2double(dpp_shl1(__double2hiint(v)), dpp_shl1(__double2loint(v)));
}
__device__ inline float from_below(float v) { return __int_as_float(dpp_shr1(__float_as_int(v))); }
__device__ inline float from_above(float v) { return __int_as_float(dpp_shl1(__float_as_int(v))); }

// Sum (or max) over the 64 lanes of a wave by a butterfly of lane exchanges
// (__shfl_xor); every lane ends with the same result (a + b = b + a), formed
// in the same order on every run.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, kLanes);
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v = fmax(v, __shfl_xor(v, m, kLanes));
  return v;
}

__device__ inline int wrap(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}
__device__ inline int clampi(int i, int lo, int hi) { return i < lo ? lo : (i > hi ? hi : i); }

// 1/x from the hardware reciprocal estimate refined by two Newton steps
// (each squares the relative error), for the one division per node.
__device__ inline double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// f^eq_q - w_q = w_q (drho + rho X_q),  X_q = 3 e + 9/2 e^2 - 3/2 |u|^2,
// e = xi_q . u  (eq 3.2 with c_s^2 = 1/3).
template <typename Real>
__device__ inline void feq_dev(double drho, double rho, double ux, double uy, Real out[kQ]) {
  const Real d = static_cast<Real>(drho), r = static_cast<Real>(rho);
  const Real x = static_cast<Real>(ux), y = static_cast<Real>(uy);
  const Real uu = Real(1.5) * (x * x + y * y);
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const Real e = Real(ex_of(q)) * x + Real(ey_of(q)) * y;
    const Real X = e * (Real(3) + Real(4.5) * e) - uu;
    out[q] = Real(w_of(q)) * (d + r * X);
  }
}

// Guo force term (eq 3.12): F_q = (F . (xi_q - u)) f^eq_q / c_s^2.
template <typename Real>
__device__ inline void force_terms(double Fx, double Fy, double ux, double uy,
                                   const Real feq[kQ], Real out[kQ]) {
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const Real fu = static_cast<Real>(Fx * (ex_of(q) - ux) + Fy * (ey_of(q) - uy));
    out[q] = Real(3) * fu * (Real(w_of(q)) + feq[q]);
  }
}

// Moment sums in FP64, in a fixed order: the three populations moving in
// +x, in -x, in +y and in -y are summed first, and the mass reuses the x
// groups (14 additions).
template <typename Real>
__device__ inline void moment_sums(const Real a[kQ], double& s, double& jx, double& jy) {
  double v[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) v[q] = static_cast<double>(a[q]);
  const double xp = v[1] + v[5] + v[8], xm = v[3] + v[6] + v[7];
  const double yp = v[2] + v[5] + v[6], ym = v[4] + v[7] + v[8];
  jx = xp - xm;
  jy = yp - ym;
  s = (v[0] + (v[2] + v[4])) + (xp + xm);
}

// Lattice-weight class of direction q: 0 rest, 1 axis, 2 diagonal.
__host__ __device__ constexpr int wclass(int q) { return q == 0 ? 0 : (q < 5 ? 1 : 2); }

// Density and velocity of eq 3.3 (without the force shift) from the FP64
// moment sums.  FP64 arithmetic divides in FP64.  FP32 arithmetic rounds
// the sums to FP32 and multiplies by the hardware reciprocal of rho refined
// by one Newton step.
__device__ inline void velocity(double s, double jx, double jy, double& r, double& x, double& y) {
  r = 1.0 + s;
  const double ir = recip(r);
  x = jx * ir;
  y = jy * ir;
}
__device__ inline void velocity(double s, double jx, double jy, float& r, float& x, float& y) {
  r = 1.0f + static_cast<float>(s);
  float ir = __builtin_amdgcn_rcpf(r);
  ir = __builtin_fmaf(__builtin_fmaf(-r, ir, 1.0f), ir, ir);
  x = static_cast<float>(jx) * ir;
  y = static_cast<float>(jy) * ir;
}

// Brackets X_q of the equilibrium, f^eq_q - w_q = w_q (drho + rho X_q) with
// X_q = 3 e_q + 9/2 e_q^2 - 3/2 |u|^2 and e_q = xi_q . u (eq 3.2, c_s^2 =
// 1/3).  Opposite directions share 9/2 e^2 - 3/2 |u|^2.
template <typename Real>
__device__ inline void eq_brackets(Real x, Real y, Real X[kQ]) {
  const Real uu = Real(1.5) * (x * x + y * y);
  X[0] = -uu;
  auto pair = [&](Real e, int qp, int qm) {
    const Real T = (Real(4.5) * e) * e - uu;
    X[qp] = T + Real(3) * e;
    X[qm] = T - Real(3) * e;
  };
  pair(x, 1, 3);
  pair(y, 2, 4);
  pair(x + y, 5, 7);
  pair(y - x, 6, 8);
}

// f^eq(rho, u_b) - f^eq(rho, u_f) (the non-equilibrium extrapolation shift
// of eq 3.10, with rho taken at the fluid node).
template <typename Real>
__device__ inline void nee_shift(double rho, double uxf, double uyf, double uxb, double uyb,
                                 Real out[kQ]) {
  const Real r = static_cast<Real>(rho);
  const Real xf = static_cast<Real>(uxf), yf = static_cast<Real>(uyf);
  const Real xb = static_cast<Real>(uxb), yb = static_cast<Real>(uyb);
  const Real uuf = Real(1.5) * (xf * xf + yf * yf), uub = Real(1.5) * (xb * xb + yb * yb);
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const Real ef = Real(ex_of(q)) * xf + Real(ey_of(q)) * yf;
    const Real eb = Real(ex_of(q)) * xb + Real(ey_of(q)) * yb;
    const Real Xf = ef * (Real(3) + Real(4.5) * ef) - uuf;
    const Real Xb = eb * (Real(3) + Real(4.5) * eb) - uub;
    out[q] = Real(w_of(q)) * r * (Xb - Xf);
  }
}

// f^eq(rho, u_b) - f^eq(rho, u_f) of eq 3.10 for q >= 1 from the brackets
// Xf of the fluid node's velocity (eq_brackets) and Xb of the wall's
// (StepParams::xb): w_q rho (Xb_q - Xf_q).  out[0] is not formed.
template <typename Real>
__device__ inline void nee_shift_x(Real rho, const Real (&Xf)[kQ], const Real* Xb, Real out[kQ]) {
  const Real r1 = Real(w_of(1)) * rho, r2 = Real(w_of(5)) * rho;
#pragma unroll
  for (int q = 1; q < kQ; ++q) out[q] = (wclass(q) == 1 ? r1 : r2) * (Xb[q] - Xf[q]);
}

// The wall whose node (i + dx, j + dy) is extrapolated from the fluid node
// (i, j) next to it (dx, dy in -1..1, not both 0; a corner counts as its x
// wall): 0 for x = 0, 1 for x = nx-1, 2 for y = 0, 3 for y = ny-1.
__host__ __device__ constexpr int wall_side_of(int dx, int dy) {
  return dx < 0 ? 0 : (dx > 0 ? 1 : (dy < 0 ? 2 : 3));
}
template <typename Real>
__device__ inline const Real* wall_brackets(const StepParams& p, int side);
template <>
__device__ inline const double* wall_brackets<double>(const StepParams& p, int side) {
  return p.xb[side];
}
template <>
__device__ inline const float* wall_brackets<float>(const StepParams& p, int side) {
  return p.xb32[side];
}

__device__ inline void wall_velocity(const StepParams& p, int c, int r, double& ub,
                                     double& vb) {
  int side;
  if (!p.per_x && c == 0)
    side = 0;
  else if (!p.per_x && c == p.nx - 1)
    side = 1;
  else if (!p.per_y && r == 0)
    side = 2;
  else
    side = 3;
  ub = p.uw[side][0];
  vb = p.uw[side][1];
}

template <typename Real>
__device__ inline const StepParams::Coef<Real>& coef(const StepParams& p);
template <>
__device__ inline const StepParams::Coef<double>& coef<double>(const StepParams& p) {
  return p.c64;
}
template <>
__device__ inline const StepParams::Coef<float>& coef<float>(const StepParams& p) {
  return p.c32;
}

template <typename Real>
__device__ inline const Real* weights_x(const StepParams& p);
template <>
__device__ inline const double* weights_x<double>(const StepParams& p) {
  return p.wx;
}
template <>
__device__ inline const float* weights_x<float>(const StepParams& p) {
  return p.wx32;
}
template <typename Real>
__device__ inline const Real* weights_y(const StepParams& p);
template <>
__device__ inline const double* weights_y<double>(const StepParams& p) {
  return p.wy;
}
template <>
__device__ inline const float* weights_y<float>(const StepParams& p) {
  return p.wy32;
}

}  // namespace
}  // namespace t2s2
