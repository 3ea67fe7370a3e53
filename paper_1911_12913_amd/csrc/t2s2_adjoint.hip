// Discrete adjoint of the fused T2S2-FDLBM step (unforced flows).
//
// The forward step, stage by stage (g = f~^n - w, all populations as
// deviations from the rest state):
//   [1] P = cPg g + cPe (feq(g) - w),  Q = cQg g + cQe (feq(g) - w)   all nodes
//   [2] S = P + A L(P)                                          interior nodes
//   [3] R = cRs S + cRe (feq(S) - w)                            interior nodes
//   [4] R_b = R_f + feq(rho_f, u_b) - feq(rho_f, u_f), moments of S_f   walls
//   [5] o = Q + L(R)                                            interior nodes
//   [6] o_b = o_f + feq(rho_f, u_b) - feq(rho_f, u_f), moments of o_f   walls
// with L the dt-scaled mixed-difference operator -dt xi . grad.  The
// adjoint runs [6]..[1] in reverse with the transposed stencil (a gather
// over the nodes whose stencil reads this one, with their weights) and the
// transposed moment Jacobians of the equilibrium.  S comes from the fused
// step run with a side output that stores it (again from state_n, or stored
// by the caller's earlier such run); [6'] (walled domains only; otherwise
// the output adjoint is lam_{n+1} itself) writes mu on the frame of wall
// nodes and their interior neighbours, where alone it differs from
// lam_{n+1}; [5'] .. [1'] then run in one kernel that marches down strips of
// the mesh like the forward step, holding lamS in an LDS ring, so neither
// lamR nor lamS goes to memory.  The wall-to-fluid scatter of [4] and [6] is
// gathered at the fluid node, so no atomics are needed and the result is
// deterministic.  d/d omega of the step (omega = dt / tau) enters only
// through the pointwise coefficients; its inner products with the adjoints
// are reduced in a fixed block order.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdlib>

#include "t2s2_device.h"
#include "t2s2_internal.h"

namespace t2s2 {
namespace {

// The reverse march takes blocks of eight waves when a block of four would
// have fewer than this many strip-rows.
constexpr long long kAdjRows8Below = 64;

template <typename Real>
__device__ inline const Real* wtab_x(const AdjParams& a);
template <>
__device__ inline const double* wtab_x<double>(const AdjParams& a) {
  return a.wx;
}
template <>
__device__ inline const float* wtab_x<float>(const AdjParams& a) {
  return a.wx32;
}
template <typename Real>
__device__ inline const Real* wtab_y(const AdjParams& a);
template <>
__device__ inline const double* wtab_y<double>(const AdjParams& a) {
  return a.wy;
}
template <>
__device__ inline const float* wtab_y<float>(const AdjParams& a) {
  return a.wy32;
}

__device__ inline bool interior(const AdjParams& a, int x, int y) {
  return (a.per_x || (x >= 1 && x <= a.nx - 2)) && (a.per_y || (y >= 1 && y <= a.ny - 2));
}

// Neighbour along an axis; -1 when it falls outside a walled axis.
__device__ inline int along(int i, int off, int n, int per) {
  const int j = i + off;
  if (per) return j < 0 ? j + n : (j >= n ? j - n : j);
  return (j < 0 || j >= n) ? -1 : j;
}

// Offset of tap k for velocity sign class s (0: positive, 1: negative).
__device__ inline int tap_offset(int s, int k) { return s == 0 ? k - 2 : k - 1; }

// The moment algebra of the reverse stages runs in the arithmetic type T of
// the forward step (FP64 for FP64 storage, FP32 otherwise); the moment sums
// themselves are FP64 in both, as in the forward step.

// 1/x: FP64 from the hardware estimate and two Newton steps, FP32 from the
// estimate and one.
__device__ inline double inv(double x) { return recip(x); }
__device__ inline float inv(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(__builtin_fmaf(-x, r, 1.0f), r, r);
}

// X_q(u) = 3 e + 9/2 e^2 - 3/2 |u|^2 and dX_q/du = (3 + 9 e) xi_q - 3 u.
template <typename T>
__device__ inline T Xq(int q, T ux, T uy) {
  const T e = T(ex_of(q)) * ux + T(ey_of(q)) * uy;
  return e * (T(3) + T(4.5) * e) - T(1.5) * (ux * ux + uy * uy);
}

// Moments of a node (unforced: u = sum xi g / rho) from FP64 sums, as in
// the forward step: d = rho - 1 (the sum itself, rounded to T), rho, u.
template <typename V, typename T>
__device__ inline void node_rho_u(const V v[kQ], T& d, T& rho, T& ux, T& uy) {
  double s, jx, jy;
  moment_sums(v, s, jx, jy);
  velocity(s, jx, jy, rho, ux, uy);
  d = static_cast<T>(s);
}

// f^eq_q - w_q = w_q (d + rho X_q) in the arithmetic type.
template <typename T>
__device__ inline void feq_of(T d, T rho, T ux, T uy, T out[kQ]) {
#pragma unroll
  for (int q = 0; q < kQ; ++q) out[q] = T(w_of(q)) * (d + rho * Xq(q, ux, uy));
}

// Transpose of d(sum_q mu_q F_q)/dg for a pointwise map whose dependence on
// g goes only through (rho, u): given a = dF/drho . mu and b = dF/du . mu,
// the gradient is a + b . (xi_q - u) / rho.
template <typename T, typename Real>
__device__ inline void through_moments(T rho, T ux, T uy, T a, T bx, T by, Real out[kQ],
                                       bool accumulate) {
  const T ir = inv(rho);
  const T cx = bx * ir, cy = by * ir;
  const T base = a - (cx * ux + cy * uy);
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const T g = base + T(ex_of(q)) * cx + T(ey_of(q)) * cy;
    out[q] = accumulate ? out[q] + static_cast<Real>(g) : static_cast<Real>(g);
  }
}

// (a, b) for F = feq(rho, u) - w:  dF_q = w_q [(1 + X_q) drho + rho dX_q].
template <typename T, typename Real>
__device__ inline void feq_ab(T rho, T ux, T uy, const Real mu[kQ], T& a, T& bx, T& by) {
  a = T(0);
  bx = T(0);
  by = T(0);
  T m3 = T(0);  // sum of w_q mu_q, times 3 u below
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const T m = static_cast<T>(mu[q]) * T(w_of(q));
    const T e = T(ex_of(q)) * ux + T(ey_of(q)) * uy;
    a += m * (T(1) + Xq(q, ux, uy));
    const T k = m * (T(3) + T(9) * e);
    if (ex_of(q) != 0) bx += T(ex_of(q)) * k;
    if (ey_of(q) != 0) by += T(ey_of(q)) * k;
    m3 += m;
  }
  bx = rho * (bx - T(3) * ux * m3);
  by = rho * (by - T(3) * uy * m3);
}

// (a, b) for the extrapolation shift F = feq(rho, u_b) - feq(rho, u):
//   dF_q = w_q [(X_q(u_b) - X_q(u)) drho - rho dX_q(u)].
template <typename T, typename Real>
__device__ inline void shift_ab(T rho, T ux, T uy, T ub, T vb, const Real mu[kQ], T& a, T& bx,
                                T& by) {
  a = T(0);
  bx = T(0);
  by = T(0);
  T m3 = T(0);
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const T m = static_cast<T>(mu[q]) * T(w_of(q));
    const T e = T(ex_of(q)) * ux + T(ey_of(q)) * uy;
    a += m * (Xq(q, ub, vb) - Xq(q, ux, uy));
    const T k = m * (T(3) + T(9) * e);
    if (ex_of(q) != 0) bx -= T(ex_of(q)) * k;
    if (ey_of(q) != 0) by -= T(ey_of(q)) * k;
    m3 += m;
  }
  bx = rho * (bx + T(3) * ux * m3);
  by = rho * (by + T(3) * uy * m3);
}

__device__ inline void wall_vel(const AdjParams& a, int c, int r, double& ub, double& vb) {
  int side;
  if (!a.per_x && c == 0)
    side = 0;
  else if (!a.per_x && c == a.nx - 1)
    side = 1;
  else if (!a.per_y && r == 0)
    side = 2;
  else
    side = 3;
  ub = a.uw[side][0];
  vb = a.uw[side][1];
}

// Calls fn(bx, by) for every wall node whose nearest interior node is
// (x, y) (the node itself must be interior).
template <typename Fn>
__device__ inline void for_wall_dependents(const AdjParams& a, int x, int y, Fn fn) {
  const bool xl = !a.per_x && x == 1, xr = !a.per_x && x == a.nx - 2;
  const bool yb = !a.per_y && y == 1, yt = !a.per_y && y == a.ny - 2;
  if (!(xl || xr || yb || yt)) return;
  for (int dy = -1; dy <= 1; ++dy) {
    if ((dy == -1 && !yb) || (dy == 1 && !yt)) continue;
    for (int dx = -1; dx <= 1; ++dx) {
      if ((dx == -1 && !xl) || (dx == 1 && !xr)) continue;
      if (dx == 0 && dy == 0) continue;
      fn(x + dx, y + dy);
    }
  }
}

#define NODE_LOOP(a)                                                                      \
  for (long long node = blockIdx.x * 256LL + threadIdx.x,                                 \
                 nn = static_cast<long long>((a).nx) * (a).ny;                            \
       node < nn; node += 256LL * gridDim.x)

template <typename T>
__device__ inline void load9(const T* base, long long plane, long long off, T v[kQ]) {
#pragma unroll
  for (int q = 0; q < kQ; ++q) v[q] = base[q * plane + off];
}

// ---- [6'] mu = adjoint of the interior output including the wall rows
// extrapolated from it; zero on walls.  Only the frame of a walled domain
// differs from lam: the wall nodes and the interior nodes next to a wall
// (the two outermost rows and columns of each walled axis).  This kernel
// writes mu there; the reverse march reads mu on the frame and lam
// everywhere else.
template <typename Store>
__global__ __launch_bounds__(256) void adj_out_walls(AdjParams a, const Store* next,
                                                      const typename Cvt<Store>::R* lam) {
  using Real = typename Cvt<Store>::R;
  Real* mu = static_cast<Real*>(a.mu);
  const int nx = a.nx, ny = a.ny;
  // Rows 0, 1, ny-2, ny-1 (walled y), then columns 0, 1, nx-2, nx-1 of
  // the other rows (walled x).
  const long long nrow = a.per_y ? 0 : 4LL * nx;
  const int r_lo = a.per_y ? 0 : 2, r_hi = a.per_y ? ny : ny - 2;
  const long long nframe = nrow + (a.per_x ? 0 : 4LL * (r_hi - r_lo));
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < nframe; i += 256LL * gridDim.x) {
    int x, y;
    if (i < nrow) {
      const int k = static_cast<int>(i / nx);
      x = static_cast<int>(i % nx);
      y = k < 2 ? k : ny - 4 + k;
    } else {
      const long long j = i - nrow;
      const int k = static_cast<int>(j % 4);
      y = r_lo + static_cast<int>(j / 4);
      x = k < 2 ? k : nx - 4 + k;
    }
    const long long off = static_cast<long long>(y) * a.pitch + x;
    Real m[kQ];
    if (!interior(a, x, y)) {
#pragma unroll
      for (int q = 0; q < kQ; ++q) mu[q * a.plane + off] = Real(0);
      continue;
    }
    load9(lam, a.plane, off, m);
    bool first = true;
    Real d = 0, rho = 1, ux = 0, uy = 0;
    for_wall_dependents(a, x, y, [&](int bx, int by) {
      if (first) {
        Real o[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) o[q] = Cvt<Store>::ld(next[q * a.plane + off]);
        node_rho_u(o, d, rho, ux, uy);
        first = false;
      }
      const long long boff = static_cast<long long>(by) * a.pitch + bx;
      Real lb[kQ];
      load9(lam, a.plane, boff, lb);
      double ub, vb;
      wall_vel(a, bx, by, ub, vb);
      Real sa, sbx, sby;
      shift_ab(rho, ux, uy, static_cast<Real>(ub), static_cast<Real>(vb), lb, sa, sbx, sby);
#pragma unroll
      for (int q = 0; q < kQ; ++q) m[q] += lb[q];
      through_moments(rho, ux, uy, sa, sbx, sby, m, true);
    });
#pragma unroll
    for (int q = 0; q < kQ; ++q) mu[q * a.plane + off] = m[q];
  }
}

// ---- [5'] .. [1'] in one march down strips of the mesh, with the layout
// of the fused forward step: 64-lane strips with 56 output columns, kRows
// waves (4, or 8 on small meshes), one row each per iteration.
//   Phase A, row r = p0 + t: lamR = L^T mu (population 0 none) gathered
//   from the interior nodes whose stencil reads (c, r) -- x taps as
//   products w(source) mu(source) formed at the source lane and shifted
//   in, y taps from the rows around -- then the transpose of the R stage
//   and of the wall extrapolation of R ([4']: x-wall nodes' lamR from the
//   neighbouring lane, y-wall rows' gathered on the fly, corners have none);
//   lamS (zero off the interior) goes to an LDS ring of 2 kRows rows.
//   Phase B, row o = p0 - 2 + t: lamP = [interior] lamS + A L^T lamS from
//   the ring, lamQ = mu, and lam_n through the P and Q stages.
// The d/d omega partials sum over the nodes each lane outputs, once each.
// Waves per SIMD that the registers of a march variant are budgeted for.
// The wall paths hold it at two in FP64 and three in FP32; a periodic grid
// compiles without them but holds the next phase's loads in registers, so
// its FP64 blocks fit two per CU and its FP32 four-row ones four.
template <typename Store, int kRows, bool kWalls>
constexpr int adj_waves_per_simd() {
  constexpr bool f32 = sizeof(typename Cvt<Store>::R) == 4;
  return kWalls ? (f32 && kRows == 4 ? 3 : 2) : (f32 ? 4 : 2);
}

template <typename Store, int kRows, bool kWalls>
__global__ __launch_bounds__(kLanes * kRows, (adj_waves_per_simd<Store, kRows, kWalls>())) void adj_strip(AdjParams a, const Store* g,
                                                 const typename Cvt<Store>::R* lam,
                                                 const typename Cvt<Store>::R* muf,
                                                 typename Cvt<Store>::R* lam_out, double* partial,
                                                 int nstrips) {
  using Real = typename Cvt<Store>::R;
  constexpr int kThreads = kLanes * kRows;
  constexpr int kSlots = 2 * kRows;  // rows p0-4 .. p0+kRows-1 in use, a power of two
  __shared__ Real ring[kSlots * kQ * kLanes];  // lamS: [slot][q][lane]
  __shared__ double red[kThreads];
  const int lane = threadIdx.x & (kLanes - 1);
  const int t = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
  const int nx = a.nx, ny = a.ny;
  // A periodic grid (no walled axis) compiles without the wall paths.
  const bool per_x = !kWalls || a.per_x, per_y = !kWalls || a.per_y;
  const long long plane = a.plane;
  // Plane strides in bytes; every plane of the Real and Store buffers is
  // under 4 GiB (checked when the adjoint is bound), so in-plane byte
  // offsets fit 32 bits.
  const unsigned long long pbr = static_cast<unsigned long long>(plane) * sizeof(Real);
  const unsigned long long pbs = static_cast<unsigned long long>(plane) * sizeof(Store);
  const Real* S = static_cast<const Real*>(a.S);
  const Real* WX = wtab_x<Real>(a);
  const Real* WY = wtab_y<Real>(a);
  const Real A = static_cast<Real>(a.A);
  double dw = 0.0;
  for (int i = threadIdx.x; i < kSlots * kQ * kLanes; i += kThreads) ring[i] = Real(0);

  // y weight of tap k, sign class sc, of the stencil at source row yi
  // (wave-uniform: read through the constant address space so it becomes a
  // scalar load, which the vector-memory counter does not wait for).
  // mu at (c, y): from the frame buffer on the frame of a walled domain (the
  // two outermost rows or columns of a walled axis), from lam elsewhere.
  auto frame_row = [&](int y) { return !per_y && (y <= 1 || y >= ny - 2); };
  auto frame_col = [&](int c) { return !per_x && (c <= 1 || c >= nx - 2); };
  using CReal = const __attribute__((address_space(4))) Real*;
  auto ywt = [&](int yi, int sc, int k) {
    const int idx = __builtin_amdgcn_readfirstlane(yi * kWeightsPerNode + sc * kTaps + k);
    return ((CReal)(WY))[idx];
  };

  // lamR of population q at (c, y) from the rows around (y taps only, over
  // interior source rows), for the wall rows (the interior rows' y taps are
  // loaded with the rest of phase A's loads below).  y is a row inside the
  // grid; the caller zeroes wall columns.  In FP32 every tap loads (from row
  // y when its source row is not interior, with weight 0), so the four loads
  // issue together; FP64 skips those loads, which keeps its registers within
  // two waves per SIMD.
  auto lamR_y = [&](int q, int c, int y) {
    const Real* mcol = frame_col(c) ? muf : lam;
    Real acc = Real(0);
    if (ey_of(q) == 0) return acc;
    const int s = ey_of(q) > 0 ? 0 : 1;
#pragma unroll
    for (int k = 0; k < kTaps; ++k) {
      const int yi = along(y, -tap_offset(s, k), ny, per_y);
      const bool rok = yi >= 0 && (per_y || (yi >= 1 && yi <= ny - 2));
      if constexpr (sizeof(Real) == 8) {
        if (rok)
          acc += WY[yi * kWeightsPerNode + s * kTaps + k] *
                 (frame_row(yi) ? muf : mcol)[q * plane + static_cast<long long>(yi) * a.pitch + c];
      } else {
        const int yc = rok ? yi : y;
        const Real w = rok ? WY[yc * kWeightsPerNode + s * kTaps + k] : Real(0);
        acc += w * (frame_row(yc) ? muf : mcol)[q * plane + static_cast<long long>(yc) * a.pitch + c];
      }
    }
    return acc;
  };

  const long long total = static_cast<long long>(nstrips) * ny;
  long long beg = total * blockIdx.x / gridDim.x;
  const long long end = total * (blockIdx.x + 1) / gridDim.x;
  while (beg < end) {  // uniform per block
    const int strip = static_cast<int>(beg / ny);
    const int y0 = static_cast<int>(beg % ny);
    const int y1 = static_cast<int>(min(static_cast<long long>(ny), y0 + (end - beg)));
    beg += y1 - y0;
    const int x0 = strip * kStripOut;
    const int x1 = min(x0 + kStripOut, nx);
    const int c0 = x0 - kHalo + lane;  // this lane's column, unwrapped
    const bool in_x = per_x || (c0 >= 0 && c0 < nx);
    const int c = per_x ? wrap(c0, nx) : clampi(c0, 0, nx - 1);
    const bool col_int = in_x && (per_x || (c0 >= 1 && c0 <= nx - 2));
    const bool lane_o = lane >= kHalo && lane < kLanes - kHalo && c0 < x1;
    const bool xl = !per_x && c0 == 1, xr = !per_x && c0 == nx - 2;
    const Real* mcol = frame_col(c) ? muf : lam;  // mu of this lane's column off the frame rows
    Real wx[kWeightsPerNode];
#pragma unroll
    for (int k = 0; k < kWeightsPerNode; ++k) wx[k] = in_x ? WX[c * kWeightsPerNode + k] : Real(0);
    __syncthreads();  // ring zero-fill / previous piece complete

    const int niter = (y1 - y0 + 3 + kRows) / kRows;
    // Periodic grids: each phase's loads are issued one phase ahead of
    // their use, into registers -- phase A's during phase B of the previous
    // iteration, phase B's during phase A -- so their latency overlaps the
    // other phase's arithmetic instead of stalling the wave at every phase
    // (the rows wrap, so every load is in the grid, also those of rows past
    // the piece, which go unused).  Without a frame, mu is lam everywhere,
    // at a wave-uniform base, so the loads walk the planes from a scalar
    // base with 32-bit row offsets.
    // Phase A of row r: lam of populations 1..8 at (c, r) (the centre tap
    // of the y-moving ones too), their other three y taps, S at (c, r) and
    // the row's y weights.
    Real a_lc[kQ], a_yt[kQ][kTaps], a_sv[kQ], a_wy[2][kTaps];
    // Phase B of row o: the state and lam at (c, o), the y weights at o.
    Store b_gs[kQ];
    Real b_lq[kQ], b_wy[2][kTaps];
    auto issue_a = [&](int r0) {
      const int r = wrap(r0, ny);
      const unsigned rb = static_cast<unsigned>(static_cast<long long>(r) * a.pitch + c) *
                          static_cast<unsigned>(sizeof(Real));
      unsigned tb[2][kTaps];
#pragma unroll
      for (int sc = 0; sc < 2; ++sc) {
#pragma unroll
        for (int k = 0; k < kTaps; ++k) {
          const int yi = along(r, -tap_offset(sc, k), ny, true);
          tb[sc][k] = static_cast<unsigned>(static_cast<long long>(yi) * a.pitch + c) *
                      static_cast<unsigned>(sizeof(Real));
          a_wy[sc][k] = ywt(yi, sc, k);
        }
      }
      GlobalBytes b = plane_base(lam);
#pragma unroll
      for (int q = 1; q < kQ; ++q) {
        b = next_plane(b, pbr);
        a_lc[q] = load_at<Real>(b, rb);
        if (ey_of(q) != 0) {
          const int sq = ey_of(q) > 0 ? 0 : 1;
#pragma unroll
          for (int k = 0; k < kTaps; ++k)
            if (tap_offset(sq, k) != 0) a_yt[q][k] = load_at<Real>(b, tb[sq][k]);
        }
      }
      load_planes(S, pbr, rb, a_sv);
    };
    auto issue_b = [&](int o0) {
      const int o = wrap(o0, ny);
      const unsigned ooff = static_cast<unsigned>(static_cast<long long>(o) * a.pitch + c);
      load_planes(g, pbs, ooff * static_cast<unsigned>(sizeof(Store)), b_gs);
      load_planes(lam, pbr, ooff * static_cast<unsigned>(sizeof(Real)), b_lq);
#pragma unroll
      for (int sc = 0; sc < 2; ++sc) {
#pragma unroll
        for (int k = 0; k < kTaps; ++k)
          b_wy[sc][k] = ywt(along(o, -tap_offset(sc, k), ny, true), sc, k);
      }
    };
    if constexpr (!kWalls) issue_a(y0 - 2 + t);
    for (int it = 0; it < niter; ++it) {
      const int p0 = y0 - 2 + kRows * it;
      if constexpr (!kWalls) issue_b(p0 - 2 + t);

      // ---- phase A: lamS of row r
      {
        const int r0 = p0 + t;
        const bool in_y = per_y || (r0 >= 0 && r0 < ny);
        Real ls[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) ls[q] = Real(0);
        if (in_y) {  // uniform per wave
          const int r = per_y ? wrap(r0, ny) : r0;
          const bool row_int = per_y || (r >= 1 && r <= ny - 2);
          const bool nin = col_int && row_int;
          const long long roff = static_cast<long long>(r) * a.pitch + c;
          // Every load of the phase, issued together before any of it is
          // used (a load followed at once by its use waits out the whole
          // memory latency, once per population): mu at (c, r) for the
          // x-moving populations, the y taps of L^T mu (from row r, with
          // weight 0, where the source row is not interior) and S at (c, r).
          // 20% faster at 513^2, 30% at 4096^2, the same values.
          Real mvx[kQ], myt[kQ][kTaps], wys[2][kTaps], sv[kQ];
          if constexpr (!kWalls) {
            // Issued by issue_a one phase earlier.
#pragma unroll
            for (int q = 1; q < kQ; ++q) {
              mvx[q] = ex_of(q) != 0 ? a_lc[q] : Real(0);
              if (ey_of(q) != 0) {
                const int s = ey_of(q) > 0 ? 0 : 1;
#pragma unroll
                for (int k = 0; k < kTaps; ++k)
                  myt[q][k] = tap_offset(s, k) == 0 ? a_lc[q] : a_yt[q][k];
              }
            }
#pragma unroll
            for (int sc = 0; sc < 2; ++sc) {
#pragma unroll
              for (int k = 0; k < kTaps; ++k) wys[sc][k] = a_wy[sc][k];
            }
#pragma unroll
            for (int q = 0; q < kQ; ++q) sv[q] = a_sv[q];
          } else {
            int ysrc[2][kTaps];
#pragma unroll
            for (int sc = 0; sc < 2; ++sc) {
#pragma unroll
              for (int k = 0; k < kTaps; ++k) {
                const int yi = along(r, -tap_offset(sc, k), ny, per_y);
                const bool rok = yi >= 0 && (per_y || (yi >= 1 && yi <= ny - 2));
                ysrc[sc][k] = rok ? yi : r;
                wys[sc][k] = rok ? ywt(yi, sc, k) : Real(0);
              }
            }
            const Real* mr = frame_row(r) ? muf : mcol;
#pragma unroll
            for (int q = 1; q < kQ; ++q) {
              mvx[q] = ex_of(q) != 0 ? mr[q * plane + roff] : Real(0);
              if (ey_of(q) != 0) {
                const int s = ey_of(q) > 0 ? 0 : 1;
#pragma unroll
                for (int k = 0; k < kTaps; ++k) {
                  const int ys = ysrc[s][k];
                  myt[q][k] = (frame_row(ys) ? muf : mcol)[q * plane + static_cast<long long>(ys) * a.pitch + c];
                }
              }
            }
            const unsigned rb = static_cast<unsigned>(roff) * static_cast<unsigned>(sizeof(Real));
            load_planes(S, pbr, rb, sv);
          }
          Real lr[kQ];
          lr[0] = Real(0);
#pragma unroll
          for (int q = 1; q < kQ; ++q) {
            // x part: sources (c - o_k, r), o_k the tap offset
            Real acc = Real(0);
            if (ex_of(q) != 0) {
              const Real mv = mvx[q];
              const Real m = nin ? mv : Real(0);
              if (ex_of(q) > 0) {  // o = -2, -1, 0, +1
                acc = from_above(from_above(wx[0] * m)) + from_above(wx[1] * m) + wx[2] * m +
                      from_below(wx[3] * m);
              } else {  // o = -1, 0, +1, +2
                acc = from_above(wx[4] * m) + wx[5] * m + from_below(wx[6] * m) +
                      from_below(from_below(wx[7] * m));
              }
            }
            Real lyv = Real(0);
            if (ey_of(q) != 0) {
#pragma unroll
              for (int k = 0; k < kTaps; ++k) lyv += wys[ey_of(q) > 0 ? 0 : 1][k] * myt[q][k];
            }
            const Real ly = row_int ? lyv : Real(0);
            lr[q] = acc + (col_int ? ly : Real(0));
          }
          // lamR of the x-wall neighbour (its own lane computed it above)
          Real lw[kQ];
          lw[0] = Real(0);
          if (!per_x) {
#pragma unroll
            for (int q = 1; q < kQ; ++q) {
              const Real lo = from_below(lr[q]), hi = from_above(lr[q]);
              lw[q] = xl ? lo : hi;
            }
          }
          if (nin) {
            Real d, rho, ux, uy;
            node_rho_u(sv, d, rho, ux, uy);
            auto add_wall = [&](int bx, int by, const Real lb[kQ]) {
              double ub, vb;
              wall_vel(a, bx, by, ub, vb);
              Real sa, sbx, sby;
              shift_ab(rho, ux, uy, static_cast<Real>(ub), static_cast<Real>(vb), lb, sa, sbx,
                       sby);
#pragma unroll
              for (int q = 0; q < kQ; ++q) lr[q] += lb[q];
              through_moments(rho, ux, uy, sa, sbx, sby, ls, true);
            };
            if (xl) add_wall(0, r, lw);
            if (xr) add_wall(nx - 1, r, lw);
            if (!per_y && (r == 1 || r == ny - 2)) {
              const int by = r == 1 ? 0 : ny - 1;
              Real lb[kQ];
              lb[0] = Real(0);
#pragma unroll
              for (int q = 1; q < kQ; ++q) lb[q] = lamR_y(q, c, by);
              add_wall(c, by, lb);
            }
            Real feq[kQ];
            feq_of(d, rho, ux, uy, feq);
            Real fa, fbx, fby;
            feq_ab(rho, ux, uy, lr, fa, fbx, fby);
            Real jt[kQ];
            const Real cRe = static_cast<Real>(a.cRe);
            through_moments(rho, ux, uy, cRe * fa, cRe * fbx, cRe * fby, jt, false);
            const bool own = lane_o && r0 >= y0 && r0 < y1;
            Real dn = Real(0);  // this node's <lamR, d R / d cRs>
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
              ls[q] += static_cast<Real>(a.cRs) * lr[q] + jt[q];
              dn += lr[q] * (sv[q] - feq[q]);
            }
            if (own) dw += a.dcRs * static_cast<double>(dn);
          }
        }
        Real* slot = ring + (r0 & (kSlots - 1)) * kQ * kLanes;
#pragma unroll
        for (int q = 0; q < kQ; ++q) slot[q * kLanes + lane] = ls[q];
      }
      if constexpr (!kWalls) issue_a(p0 + kRows + t);  // phase A of the next iteration
      __syncthreads();

      // ---- phase B: lam_n of row o
      {
        const int o = p0 - 2 + t;
        if (o >= y0 && o < y1) {  // uniform per wave
          const bool nin = col_int && (per_y || (o >= 1 && o <= ny - 2));
          // This row's state and mu: on walled grids loaded here, before the
          // ring taps, so their latency overlaps them; on periodic grids
          // issued at the start of the iteration.
          const long long ooff = static_cast<long long>(o) * a.pitch + c;
          const unsigned ob = static_cast<unsigned>(ooff) * static_cast<unsigned>(sizeof(Real));
          Real v[kQ], lq[kQ];
          // y weights of the taps (zero where the source row is outside a
          // walled axis; the ring holds zero off the interior).
          Real wyo[2][kTaps];
          if constexpr (!kWalls) {
            // Issued by issue_b at the start of the iteration.
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
              v[q] = Cvt<Store>::ld(b_gs[q]);
              lq[q] = b_lq[q];
            }
#pragma unroll
            for (int sc = 0; sc < 2; ++sc) {
#pragma unroll
              for (int k = 0; k < kTaps; ++k) wyo[sc][k] = b_wy[sc][k];
            }
          } else {
            {
              Store gs[kQ];
              load_planes(g, pbs, static_cast<unsigned>(ooff) * static_cast<unsigned>(sizeof(Store)), gs);
#pragma unroll
              for (int q = 0; q < kQ; ++q) v[q] = Cvt<Store>::ld(gs[q]);
            }
            load9(frame_row(o) ? muf : mcol, plane, ooff, lq);
#pragma unroll
            for (int sc = 0; sc < 2; ++sc) {
#pragma unroll
              for (int k = 0; k < kTaps; ++k) {
                const int yi = along(o, -tap_offset(sc, k), ny, per_y);
                wyo[sc][k] = yi >= 0 ? ywt(yi, sc, k) : Real(0);
              }
            }
          }
          const Real* cen = ring + (o & (kSlots - 1)) * kQ * kLanes + lane;
          Real lp[kQ];
#pragma unroll
          for (int q = 0; q < kQ; ++q) {
            const Real l = cen[q * kLanes];
            Real acc = Real(0);
            if (ex_of(q) > 0)
              acc = from_above(from_above(wx[0] * l)) + from_above(wx[1] * l) + wx[2] * l +
                    from_below(wx[3] * l);
            if (ex_of(q) < 0)
              acc = from_above(wx[4] * l) + wx[5] * l + from_below(wx[6] * l) +
                    from_below(from_below(wx[7] * l));
            if (ey_of(q) != 0) {
              const int s = ey_of(q) > 0 ? 0 : 1;
#pragma unroll
              for (int k = 0; k < kTaps; ++k) {
                const int yu = o - tap_offset(s, k);  // unwrapped source row
                acc += wyo[s][k] * ring[(yu & (kSlots - 1)) * kQ * kLanes + q * kLanes + lane];
              }
            }
            lp[q] = (nin ? l : Real(0)) + (q == 0 ? Real(0) : A * acc);
          }
          Real d, rho, ux, uy;
          node_rho_u(v, d, rho, ux, uy);
          Real feq[kQ], mix[kQ];
          feq_of(d, rho, ux, uy, feq);
#pragma unroll
          for (int q = 0; q < kQ; ++q)
            mix[q] = static_cast<Real>(a.cPe) * lp[q] + static_cast<Real>(a.cQe) * lq[q];
          Real fa, fbx, fby;
          feq_ab(rho, ux, uy, mix, fa, fbx, fby);
          Real out[kQ];
          through_moments(rho, ux, uy, fa, fbx, fby, out, false);
          Real dp = Real(0), dq = Real(0);  // this node's <lamP, g - feq>, <lamQ, g - feq>
#pragma unroll
          for (int q = 0; q < kQ; ++q) {
            out[q] += static_cast<Real>(a.cPg) * lp[q] + static_cast<Real>(a.cQg) * lq[q];
            const Real neq = v[q] - feq[q];
            dp += lp[q] * neq;
            dq += lq[q] * neq;
          }
          if (lane_o) store_planes<false>(lam_out, pbr, ob, out);
          if (lane_o) dw += a.dcPg * static_cast<double>(dp) + a.dcQg * static_cast<double>(dq);
        }
      }
      __syncthreads();
    }
  }
  red[threadIdx.x] = dw;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// accum += scale * (the sum of the n block partials of d/d omega), by one
// wave: lane l adds partials l, l + 64, ... in that order, then the lanes
// are summed by the butterfly; the same order on every run.  scale is
// d omega / d nu, so accum gathers d/d nu.  (One thread walking the
// partials one at a time waited out a cache round trip per partial.)
__global__ __launch_bounds__(64) void adj_accumulate(const double* partial, int n,
                                                      double scale, double* accum) {
  double s = 0.0;
  for (int b = threadIdx.x; b < n; b += kLanes) s += partial[b];
  s = wave_sum(s);
  if (threadIdx.x == 0) *accum += s * scale;
}

// ---- seed: lam = d(<gu, u> + <gv, v>)/dg at every node.
template <typename Store>
__global__ __launch_bounds__(256) void adj_seed_velocity(AdjParams a, const Store* g,
                                                          const double* gu, const double* gv,
                                                          typename Cvt<Store>::R* lam) {
  using Real = typename Cvt<Store>::R;
  NODE_LOOP(a) {
    const int x = static_cast<int>(node % a.nx), y = static_cast<int>(node / a.nx);
    const long long off = static_cast<long long>(y) * a.pitch + x;
    Real v[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) v[q] = Cvt<Store>::ld(g[q * a.plane + off]);
    Real d, rho, ux, uy;
    node_rho_u(v, d, rho, ux, uy);
    Real out[kQ];
    through_moments(rho, ux, uy, Real(0), static_cast<Real>(gu ? gu[node] : 0.0),
                    static_cast<Real>(gv ? gv[node] : 0.0), out, false);
#pragma unroll
    for (int q = 0; q < kQ; ++q) lam[q * a.plane + off] = out[q];
  }
}

// ---- gradient of the equilibrium initial state f~ = feq(rho, u).
template <typename Real>
__global__ __launch_bounds__(256) void adj_init_macro(AdjParams a, const Real* lam,
                                                       const double* rho, const double* ux,
                                                       const double* uy, double* grho,
                                                       double* gux, double* guy) {
  NODE_LOOP(a) {
    const int x = static_cast<int>(node % a.nx), y = static_cast<int>(node / a.nx);
    const long long off = static_cast<long long>(y) * a.pitch + x;
    Real l[kQ];
    load9(lam, a.plane, off, l);
    double fa, fbx, fby;
    feq_ab(rho[node], ux[node], uy[node], l, fa, fbx, fby);
    if (grho) grho[node] = fa;
    if (gux) gux[node] = fbx;
    if (guy) guy[node] = fby;
  }
}

template <typename Real>
__global__ __launch_bounds__(256) void adj_convert(AdjParams a, const Real* lam, double* dense,
                                                    const double* dense_in, Real* lam_out) {
  NODE_LOOP(a) {
    const int x = static_cast<int>(node % a.nx), y = static_cast<int>(node / a.nx);
    const long long off = static_cast<long long>(y) * a.pitch + x;
    const long long n = static_cast<long long>(a.nx) * a.ny;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      if (dense) dense[q * n + node] = static_cast<double>(lam[q * a.plane + off]);
      if (lam_out) lam_out[q * a.plane + off] = static_cast<Real>(dense_in[q * n + node]);
    }
  }
}

int adj_grid(const AdjParams& a) {
  long long g = (static_cast<long long>(a.nx) * a.ny + 255) / 256;
  return static_cast<int>(g < 1 ? 1 : (g > kDiagBlocks ? kDiagBlocks : g));
}

// The reverse stages of the step from state_n, given its S (a.S) and the
// new state (a.next, whose moments the walls' adjoint needs at the fluid
// nodes).
template <typename Store>
hipError_t adjoint_reverse_t(const AdjParams& a, const void* state_n, const void* lam_np1,
                             void* lam_n, double* partial, double* accum, hipStream_t s) {
  using Real = typename Cvt<Store>::R;
  const bool walls = !a.per_x || !a.per_y;
  const Real* mu = static_cast<const Real*>(lam_np1);
  const Store* g = static_cast<const Store*>(state_n);
  // mu on the frame of a walled domain; without walls mu is lam_np1 itself.
  const Real* muf = mu;
  if (walls) {
    const long long nframe = 4LL * (a.nx + a.ny);
    const int fg = static_cast<int>(std::min<long long>(kDiagBlocks, (nframe + 255) / 256));
    hipLaunchKernelGGL(adj_out_walls<Store>, dim3(fg), dim3(256), 0, s, a,
                       static_cast<const Store*>(a.next), mu);
    muf = static_cast<const Real*>(a.mu);
  }
  const int nstrips = (a.nx + kStripOut - 1) / kStripOut;
  const bool rows8 = a.march_rows8 != 0;
  const int Gs = a.march_grid;
  Real* lo = static_cast<Real*>(lam_n);
  if (rows8 && walls)
    hipLaunchKernelGGL((adj_strip<Store, 8, true>), dim3(Gs), dim3(kLanes * 8), 0, s, a, g, mu,
                       muf, lo, partial, nstrips);
  else if (rows8)
    hipLaunchKernelGGL((adj_strip<Store, 8, false>), dim3(Gs), dim3(kLanes * 8), 0, s, a, g, mu,
                       muf, lo, partial, nstrips);
  else if (walls)
    hipLaunchKernelGGL((adj_strip<Store, 4, true>), dim3(Gs), dim3(kLanes * 4), 0, s, a, g, mu,
                       muf, lo, partial, nstrips);
  else
    hipLaunchKernelGGL((adj_strip<Store, 4, false>), dim3(Gs), dim3(kLanes * 4), 0, s, a, g, mu,
                       muf, lo, partial, nstrips);
  if (accum)
    hipLaunchKernelGGL(adj_accumulate, dim3(1), dim3(64), 0, s, partial, Gs,
                       a.dnu_per_domega, accum);
  return hipGetLastError();
}

// The step again from state_n into the scratch state, storing S into the
// scratch as it goes, then the reverse stages.
template <typename Store>
hipError_t adjoint_step_t(int storage, const AdjParams& a, const StepParams& sp, int step_grid,
                          const void* state_n, const void* lam_np1, void* lam_n,
                          double* partial, double* accum, hipStream_t s) {
  StepParams fwd = sp;
  fwd.src = state_n;
  fwd.dst = a.next;
  fwd.save_s = a.S;
  hipError_t e = launch_step_save_s(storage, fwd, step_grid, s);
  if (e != hipSuccess) return e;
  return adjoint_reverse_t<Store>(a, state_n, lam_np1, lam_n, partial, accum, s);
}

template <typename Store, int kRows, bool kWalls>
hipError_t march_blocks_per_cu(int& n) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, adj_strip<Store, kRows, kWalls>,
                                                      kLanes * kRows, 0);
}

// Blocks of the reverse march: as many as are resident at once on the
// device (two waves per SIMD with walls, three or four on periodic grids,
// see adj_waves_per_simd).  Small meshes, where a four-wave block would
// march fewer than kAdjRows8Below strip-rows, take eight-wave blocks: a
// block then marches twice the rows and fewer of its rows are the two-row
// halos above and below its range.  The plan is fixed per context, so the
// order of the d/d omega reduction is too.
template <typename Store>
hipError_t plan_march_t(AdjParams& a, int cus) {
  const bool walls = !a.per_x || !a.per_y;
  int n4 = 0, n8 = 0;
  hipError_t e = walls ? march_blocks_per_cu<Store, 4, true>(n4)
                       : march_blocks_per_cu<Store, 4, false>(n4);
  if (e == hipSuccess)
    e = walls ? march_blocks_per_cu<Store, 8, true>(n8) : march_blocks_per_cu<Store, 8, false>(n8);
  if (e != hipSuccess) return e;
  auto grid = [&](int per_cu) {
    const long long g = static_cast<long long>(std::max(per_cu, 1)) * std::max(cus, 1);
    return static_cast<int>(std::min<long long>(g, kAdjMaxBlocks));
  };
  const int g4 = grid(n4);
  const long long nstrips = (a.nx + kStripOut - 1) / kStripOut;
  a.march_rows8 = nstrips * a.ny < kAdjRows8Below * g4 ? 1 : 0;
  // T2S2_ADJ_ROWS=4 or 8 forces the block shape (tests compare the two).
  if (const char* env = std::getenv("T2S2_ADJ_ROWS")) {
    if (env[0] == '4' && env[1] == 0) a.march_rows8 = 0;
    if (env[0] == '8' && env[1] == 0) a.march_rows8 = 1;
  }
  a.march_grid = a.march_rows8 ? grid(n8) : g4;
  return hipSuccess;
}

}  // namespace

#define T2S2_ADJ_DISPATCH(storage, CALL)                   \
  switch (storage) {                                       \
    case kF64: { using Store = double; CALL; } break;      \
    case kF32: { using Store = float; CALL; } break;       \
    case kBF16: { using Store = Bf16; CALL; } break;       \
    case kF16: { using Store = _Float16; CALL; } break;    \
    default: return hipErrorInvalidValue;                  \
  }

size_t adjoint_real_bytes(int storage) { return storage == kF64 ? 8 : 4; }

hipError_t plan_adjoint_march(int storage, AdjParams& a, int cus) {
  T2S2_ADJ_DISPATCH(storage, return plan_march_t<Store>(a, cus));
  return hipSuccess;
}

hipError_t launch_adjoint_step(int storage, const AdjParams& a, const StepParams& sp,
                               int step_grid, const void* state_n, const void* lam_np1,
                               void* lam_n, double* partial, double* accum, hipStream_t s) {
  T2S2_ADJ_DISPATCH(storage, return adjoint_step_t<Store>(storage, a, sp, step_grid, state_n,
                                                          lam_np1, lam_n, partial, accum, s));
  return hipSuccess;
}

hipError_t launch_adjoint_step_stored(int storage, const AdjParams& a, const void* state_n,
                                      const void* state_np1, const void* s_n,
                                      const void* lam_np1, void* lam_n, double* partial,
                                      double* accum, hipStream_t s) {
  AdjParams b = a;
  b.S = const_cast<void*>(s_n);
  b.next = const_cast<void*>(state_np1);
  T2S2_ADJ_DISPATCH(storage,
                    return adjoint_reverse_t<Store>(b, state_n, lam_np1, lam_n, partial, accum, s));
  return hipSuccess;
}

hipError_t launch_adjoint_seed(int storage, const AdjParams& a, const void* state,
                               const double* gu, const double* gv, void* lam, hipStream_t s) {
  T2S2_ADJ_DISPATCH(storage,
                    hipLaunchKernelGGL(adj_seed_velocity<Store>, dim3(adj_grid(a)), dim3(256), 0,
                                       s, a, static_cast<const Store*>(state), gu, gv,
                                       static_cast<typename Cvt<Store>::R*>(lam)));
  return hipGetLastError();
}

hipError_t launch_adjoint_init(int storage, const AdjParams& a, const void* lam,
                               const double* rho, const double* ux, const double* uy,
                               double* grho, double* gux, double* guy, hipStream_t s) {
  if (storage == kF64)
    hipLaunchKernelGGL(adj_init_macro<double>, dim3(adj_grid(a)), dim3(256), 0, s, a,
                       static_cast<const double*>(lam), rho, ux, uy, grho, gux, guy);
  else
    hipLaunchKernelGGL(adj_init_macro<float>, dim3(adj_grid(a)), dim3(256), 0, s, a,
                       static_cast<const float*>(lam), rho, ux, uy, grho, gux, guy);
  return hipGetLastError();
}

hipError_t launch_adjoint_convert(int storage, const AdjParams& a, const void* lam,
                                  double* dense, const double* dense_in, void* lam_out,
                                  hipStream_t s) {
  if (storage == kF64)
    hipLaunchKernelGGL(adj_convert<double>, dim3(adj_grid(a)), dim3(256), 0, s, a,
                       static_cast<const double*>(lam), dense, dense_in,
                       static_cast<double*>(lam_out));
  else
    hipLaunchKernelGGL(adj_convert<float>, dim3(adj_grid(a)), dim3(256), 0, s, a,
                       static_cast<const float*>(lam), dense, dense_in,
                       static_cast<float*>(lam_out));
  return hipGetLastError();
}

}  // namespace t2s2
