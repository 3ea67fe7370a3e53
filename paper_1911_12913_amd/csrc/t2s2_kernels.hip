// HIP kernels of the D2Q9 T2S2-FDLBM step for gfx950 (wave64).
//
// The fused step kernel computes one full time step f~^n -> f~^{n+1} of the
// paper's Sec. 2D sequence in a single pass over HBM:
//   P = fbar^{+,h}(f~)                 pointwise (eqs 2.34, 2.51)
//   Q = f~^{+}(f~)                     pointwise (eq 2.20)
//   S = P - h xi . grad_m P            half-step characteristic (eqs 2.33, 2.35)
//   R = f(t*) from S                   pointwise with new moments (eqs 2.32, 2.52)
//   f~^{n+1} = Q - dt xi . grad_m R    (eq 2.23)
// with non-equilibrium extrapolation (eq 3.10) on wall nodes, for R (the
// stencil reads it) and for the new state, both written by the lane of the
// wall node's nearest interior node.  All populations are carried as
// deviations g = f~ - w.
//
// Work decomposition: a block owns a strip of 64 columns (56 outputs plus a
// 4-column halo each side, the reach of the two chained radius-2 stencils)
// and a segment of rows, and marches down the segment.  Each of its four
// waves handles one row per iteration.  P and R rows live in LDS ring
// buffers of 8 rows; Q stays in registers for one iteration.  Every value is
// read from HBM once per strip and written once.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "t2s2_device.h"
#include "t2s2_internal.h"

namespace t2s2 {
namespace {

// ---------------------------------------------------------------------------
// Fused step.
// ---------------------------------------------------------------------------
// The row weights are the same for the whole wave: read them through the
// constant address space at a wave-uniform index so they become scalar loads
// (counted by lgkmcnt).  A vector load here would be waited for with the
// in-order vmcnt counter and so drain the row prefetches in flight.
template <typename Real>
__device__ inline void row_weights(const Real* table, int row, Real out[kWeightsPerNode]) {
  using CPtr = const __attribute__((address_space(4))) Real*;
  const int r = __builtin_amdgcn_readfirstlane(row);
  CPtr w = (CPtr)(table) + r * kWeightsPerNode;
#pragma unroll
  for (int k = 0; k < kWeightsPerNode; ++k) out[k] = w[k];
}


// Element at a 32-bit byte offset from a plane base: the row offset is
// formed once per row in 32 bits and shared by the nine planes.  Every
// population plane is under 4 GiB (checked when the context is created).
template <typename T>
__device__ inline const T* at_byte(const T* base, unsigned boff) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + boff);
}
template <typename T>
__device__ inline T* at_byte(T* base, unsigned boff) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + boff);
}

// The nine new values of one interior node at byte offset boff of each
// plane: rounded to nearest even, or, for the stochastic forms, by
// round_node_sr with the node's offset as its position.  FP64 rows (448
// bytes per wave) go out as non-temporal (streaming) stores: the state is
// not read again in this launch, and they reach HBM faster than write-back
// stores.  The narrower FP32 and 16-bit rows (224 and 112 bytes, not
// line-aligned) merge better in L2 and use ordinary stores (measured: FP32
// 5% faster so).
template <typename Store>
__device__ inline void store_node(Store* dst, long long plane, unsigned boff,
                                  const typename Cvt<Store>::R (&out)[kQ]) {
  constexpr bool kNt = std::is_same<Store, double>::value;
  Store r[kQ];
  if constexpr (kStochastic<Store>) {
    round_node_sr(out, boff, r);
  } else {
#pragma unroll
    for (int q = 0; q < kQ; ++q) r[q] = Cvt<Store>::st(out[q]);
  }
  store_planes<kNt>(dst, plane * sizeof(Store), boff, r);
}

// Row index brought into [0, n) by whole periods; the rows a piece touches
// lie within a few rows of the grid, so this loops at most a few times.
__device__ inline int wrap_near(int i, int n) {
  while (i < 0) i += n;
  while (i >= n) i -= n;
  return i;
}

// acc + sum_k w[k] v(lane + offset_k) for the 4 taps of the mixed difference
// along x: offsets (-2,-1,0,+1) for a positive velocity component (sx = 0),
// (-1,0,+1,+2) for a negative one (sx = 1); the neighbours come from the
// centre values of the other lanes.
template <int sx, typename Real>
__device__ inline Real x_taps(const Real* w, Real centre, Real acc) {
  const Real m1 = from_below(centre), p1 = from_above(centre);
  if (sx == 0) {
    const Real m2 = from_below(m1);
    acc += w[0] * m2;
    acc += w[1] * m1;
    acc += w[2] * centre;
    acc += w[3] * p1;
  } else {
    const Real p2 = from_above(p1);
    acc += w[4] * m1;
    acc += w[5] * centre;
    acc += w[6] * p1;
    acc += w[7] * p2;
  }
  return acc;
}

// Guo force term (eq 3.12) of direction q from E = (f^eq_q - w_q) / w_q:
// F_q = 3 (F . (xi_q - u)) f^eq_q with f^eq_q = w_q (1 + E).
template <typename Real>
__device__ inline Real force_term(int q, const StepParams& p, Real ux, Real uy, Real E) {
  const Real fu = static_cast<Real>(p.Fx) * (Real(ex_of(q)) - ux) +
                  static_cast<Real>(p.Fy) * (Real(ey_of(q)) - uy);
  return Real(3.0 * w_of(q)) * fu * (Real(1) + E);
}

// Wall nodes of the new state (eq 3.10),
//   f~_b = f~_f + f^eq(rho_f, u_b) - f^eq(rho_f, u_f),
// from the moments of the stored new state at the nearest interior node f
// (diagonal at the corners), u_f with the force shift of eq 3.3.  Run by a
// strip's threads after its piece [y0, y1) has been marched and the block
// has passed a barrier: the sources are the nodes next to a wall among the
// piece's outputs (columns [x0, x1)), which this block has just stored, so
// the loads see them (the coherence point is L2; the buffer was not read
// earlier in the launch).  Each wall node has exactly one source node, and
// each source node is output by exactly one piece.
template <typename Store>
__device__ inline void piece_walls(const StepParams& p, Store* dst, int x0, int x1, int y0,
                                   int y1, int tid, int nthreads) {
  using Real = typename Cvt<Store>::R;
  const int nx = p.nx, ny = p.ny;
  // Interior output columns and rows of this strip-piece.
  const int cx0 = p.per_x ? x0 : max(x0, 1), cx1 = p.per_x ? x1 : min(x1, nx - 1);
  const int ry0 = p.per_y ? y0 : max(y0, 1), ry1 = p.per_y ? y1 : min(y1, ny - 1);
  if (cx0 >= cx1 || ry0 >= ry1) return;
  // Sources: (a) the rows next to the bottom and top walls, every column;
  // (b) the columns next to the left and right walls, the other rows.
  const bool rb = !p.per_y && ry0 <= 1 && 1 < ry1;
  const bool rt = !p.per_y && ry0 <= ny - 2 && ny - 2 < ry1;
  const bool cl = !p.per_x && cx0 <= 1 && 1 < cx1;
  const bool cr = !p.per_x && cx0 <= nx - 2 && nx - 2 < cx1;
  const int ncol = cx1 - cx0;
  const int nrow_a = (rb ? 1 : 0) + (rt ? 1 : 0);
  const int nrows_b = (ry1 - ry0) - nrow_a;  // rows not already in (a)
  const int nsrc = nrow_a * ncol + ((cl ? 1 : 0) + (cr ? 1 : 0)) * nrows_b;
#pragma unroll 1
  for (int k = tid; k < nsrc; k += nthreads) {
    int i, j;
    if (k < nrow_a * ncol) {
      j = (k < ncol && rb) ? 1 : ny - 2;
      i = cx0 + k % ncol;
    } else {
      const int kb = k - nrow_a * ncol;
      i = (kb < nrows_b && cl) ? 1 : nx - 2;
      // The (kb mod nrows_b)-th row of [ry0, ry1) other than rows 1 and
      // ny - 2 when those are in (a): row 1 is then ry0, row ny - 2 is ry1 - 1.
      j = ry0 + (rb ? 1 : 0) + kb % nrows_b;
    }
    const long long fb = static_cast<long long>(j) * p.pitch + i;
    Real v[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) v[q] = Cvt<Store>::ld(dst[q * p.plane + fb]);
    double s, jx, jy;
    moment_sums(v, s, jx, jy);
    const double rho = 1.0 + s;
    const double ir = recip(rho);
    const double ux = jx * ir + p.half_dt * p.Fx;
    const double uy = jy * ir + p.half_dt * p.Fy;
    const bool wl = !p.per_x && i == 1, wr = !p.per_x && i == nx - 2;
    const bool wb = !p.per_y && j == 1, wt = !p.per_y && j == ny - 2;
#pragma unroll 1
    for (int dy = -1; dy <= 1; ++dy) {
      if ((dy == -1 && !wb) || (dy == 1 && !wt)) continue;
#pragma unroll 1
      for (int dx = -1; dx <= 1; ++dx) {
        if ((dx == -1 && !wl) || (dx == 1 && !wr)) continue;
        if (dx == 0 && dy == 0) continue;
        double ub, vb;
        wall_velocity(p, i + dx, j + dy, ub, vb);
        Real sh[kQ];
        nee_shift(rho, ux, uy, ub, vb, sh);
        const long long wo = static_cast<long long>(j + dy) * p.pitch + (i + dx);
#pragma unroll
        for (int q = 0; q < kQ; ++q) dst[q * p.plane + wo] = Cvt<Store>::st(v[q] + sh[q]);
      }
    }
  }
}

// Resident waves per SIMD the register allocation must allow: the FP64 rings
// (68 KB per block) admit two blocks per CU; the FP32 rings admit four, which
// the FP32 / FP16 variants without a force reach without spilling (the force
// variants, the walled FP16 ones, and BF16 with its conversions, settle for
// three).
// T2S2-FDLBM2's first ring (106 KB in FP64, 53 KB in FP32) admits one and
// three blocks per CU; in FP64 on periodic meshes it holds Q alone, as
// FDLBM1's holds P, and admits two blocks.
// The family's ring (140 KB in FP64, 70 KB in FP32) admits one and two.
template <typename Store, bool kForce, bool kWalls, int kScheme>
constexpr int kMinWaves =
    sizeof(typename Cvt<Store>::R) == 8
        ? ((kScheme == 1 || (kScheme == 2 && !kWalls)) ? 2 : 1)
        : (kScheme >= 3 ? 2
                        : (((kScheme == 2 && (kWalls || std::is_same<Store, float>::value)) ||
                            kForce || kBf16Bits<Store> ||
                            kStochastic<Store> || (kWalls && !std::is_same<Store, float>::value))
                               ? 3
                               : 4));

// T2S2-FDLBM2 on a periodic mesh keeps each row's f^n in the registers of
// the wave that loaded the row, instead of in the first LDS ring: the
// waves take the phase-2 rows in the order that makes each one's phase-2
// row a row it loaded (in this iteration for waves 0 and 1, in the previous
// one for waves 2 and 3), and the ring holds Q alone.  At 4096^2: FP64
// 643 -> 503 us per step (two blocks per CU, where forming f^n again from
// a reload of the row fetched the rows twice from HBM), BF16 261 -> 232
// us; FP32 storage keeps the ring (365 against 374 us).  Walled meshes keep
// f^n in the ring: eq 3.10 reads it at wall nodes that another wave loaded.
template <typename Store, bool kWalls, int kScheme>
constexpr bool kFnRegsOf = kScheme == 2 && !kWalls && !std::is_same<Store, float>::value;

// Planes of the first LDS ring: P for T2S2-FDLBM1 (and T1S2); for
// T2S2-FDLBM2, Q = f~^+ (the field the prediction advects) and, for the
// eight moving directions, the physical f^n (not with kFnRegsOf); for the
// family, P, Q and the eight moving directions of f^n.
template <int kScheme, bool kFnRegs>
constexpr int kPPlanes =
    kScheme == 1 ? kQ : (kScheme == 2 ? (kFnRegs ? kQ : 2 * kQ - 1) : 3 * kQ - 1);

// The fused step, templated on the storage type, the presence of a body
// force, of walls, on the scheme, and on kSaveS (the discrete adjoint's
// recompute: also store S = fbar(t*) at the interior nodes, into
// p.save_s in the arithmetic type, [9][ny][pitch]):
//   kScheme 1: T2S2-FDLBM1 family (eq 2.23; A = 0 is T1S2);
//   kScheme 2: T2S2-FDLBM2 (eq 5.23): f~^{n+1} = Q + dt/2 (L(f^n) + L(f^{n+1}))
//     with f^{n+1} predicted by S = Q + dt L(Q) and unshifted with h = dt;
//     L is linear, so the two gradients are taken as one, of T = f^n + R;
//   kScheme 3: the eq 2.13 family, f~^{n+1} = Q + dt L(T) with
//     T = b0 f^n + b1 f* + b2 f^{n+1}, f* predicted as in scheme 1 and
//     f^{n+1} as in scheme 2;
//   kScheme 4: the family with collision weights other than (1/2, 0, 1/2)
//     (p.gen_bbar; host scheme 3): the base is Q2 = f^n + B-0 dt Omega(f^n)
//     and V = B-1 dt Omega(f*) is added, and the new state is formed from
//     Y = Q2 + V + dt L(T) by solving the implicit weight B-2 through Y's
//     moments.  V of a node is formed in phase 2 from that node's f* and
//     used by phase 3 of the same wave, in registers: the waves take the
//     phase-2 rows in the order that makes each one's phase-2 row the row it
//     outputs (in the same iteration for waves 2 and 3, in the next for
//     waves 0 and 1).
template <typename Store, bool kForce, bool kWalls, int kScheme, bool kSaveS = false>
__global__ __launch_bounds__(step_threads(kStorageOf<Store>, kScheme), (kMinWaves<Store, kForce, kWalls, kScheme>)) void step_kernel(
    StepParams p) {
  using Real = typename Cvt<Store>::R;
  // T2S2-FDLBM2, FP64, periodic: f^n of the phase-2 row from a reload.
  constexpr bool kFnRegs = kFnRegsOf<Store, kWalls, kScheme>;
  constexpr int kNP = kPPlanes<kScheme, kFnRegs>;
  constexpr int kSB = strips_per_block(kStorageOf<Store>, kScheme);
  constexpr int kThreads = step_threads(kStorageOf<Store>, kScheme);
  constexpr int kSizeP = kRing * kNP * kLanes, kSizeR = kRing * (kQ - 1) * kLanes;
  constexpr int kSizeT = kWalls ? (kQ - 1) * kLanes : 1;
  __shared__ Real ringP_all[kSB * kSizeP];  // per strip: [slot][plane][lane]
  __shared__ Real ringR_all[kSB * kSizeR];  // per strip: [slot][q-1][lane]
  // R of the top wall row ny-1, kept out of the ring: it is written (eq 3.10)
  // by the wave that computes row ny-2, in the same phase in which the ring
  // slot of row ny-1 still holds row ny-9 for the output row ny-7.
  __shared__ Real topR_all[kSB * kSizeT];

  const int lane = threadIdx.x & (kLanes - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
  const int half = kSB == 1 ? 0 : wave / kRowsPerIter;  // which of the block's strips
  const int t = kSB == 1 ? wave : wave % kRowsPerIter;  // which row of an iteration
  Real* const ringP = ringP_all + half * kSizeP;
  Real* const ringR = ringR_all + half * kSizeR;
  Real* const topR = topR_all + half * kSizeT;
  const int nx = p.nx, ny = p.ny;
  const Store* __restrict__ src = static_cast<const Store*>(p.src);
  Store* __restrict__ dst = static_cast<Store*>(p.dst);
  const long long plane = p.plane;

  for (int i = threadIdx.x; i < kSB * kSizeP; i += kThreads) ringP_all[i] = Real(0);
  for (int i = threadIdx.x; i < kSB * kSizeR; i += kThreads) ringR_all[i] = Real(0);
  if (kWalls)
    for (int i = threadIdx.x; i < kSB * kSizeT; i += kThreads) topR_all[i] = Real(0);

  // Work: a unit is kSB neighbouring strips, marched side by side by the
  // block's kSB groups of four waves (a strip past the last column computes
  // in its own rings and stores nothing).  The rows are cut into bands of
  // p.band rows; the unit-rows are ordered band by band, unit by unit within
  // a band, row by row within a unit, and this order is cut into nblocks
  // equal ranges (one per block, so every block does the same work).  With
  // the band height equal to one block's share, a block owns one unit of one
  // band, and the blocks of neighbouring units start on the same row and
  // march in step: the cache lines that two strips share (the halo columns)
  // are fetched from HBM once and found in L1 or L2 by the other strip.  A
  // range may run over a unit or band boundary; each piece is marched
  // separately.  XCD-aware order: the grid is a multiple of 8 and blocks are
  // dealt round-robin to the 8 XCDs, so block b runs on XCD b % 8; each XCD
  // gets a contiguous run of ranges, i.e. neighbouring units of a band share
  // one L2.
  const int G = gridDim.x;
  const int L = (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8;
  if (L >= p.nblocks) return;  // padding block: whole block, before any barrier
  const long long total = static_cast<long long>(p.nunits) * ny;
  const long long band_pieces = static_cast<long long>(p.nunits) * p.band;
  long long beg = total * L / p.nblocks;
  const long long end = total * (L + 1) / p.nblocks;

  while (beg < end) {  // uniform per block
    const int b = static_cast<int>(beg / band_pieces);
    const long long rem = beg - b * band_pieces;
    const int r0 = b * p.band;
    const int hb = min(p.band, ny - r0);  // the last band may be shorter
    const int strip = static_cast<int>(rem / hb) * kSB + half;
    const int y0 = r0 + static_cast<int>(rem % hb);
    const int y1 = static_cast<int>(min(static_cast<long long>(r0 + hb), y0 + (end - beg)));
    beg += y1 - y0;

    const int x0 = strip * kStripOut;
    const int x1 = min(x0 + kStripOut, nx);
    // This lane's column; loads and weights use the wrapped (periodic) or
    // clamped (walled) column so every ring entry holds finite data.
    const int c = x0 - kHalo + lane;
    const int cm = p.per_x ? wrap(c, nx) : clampi(c, 0, nx - 1);
    Real wxr[kWeightsPerNode];
    {
      const Real* wx = weights_x<Real>(p);
#pragma unroll
      for (int k = 0; k < kWeightsPerNode; ++k) wxr[k] = wx[cm * kWeightsPerNode + k];
    }
    const bool col_interior = p.per_x || (c >= 1 && c <= nx - 2);
    const bool lane_r = lane >= 2 && lane < kLanes - 2;
    const bool lane_o = lane >= kHalo && lane < kLanes - kHalo && c < x1;
    const bool src_xl = !p.per_x && c == 1;
    const bool src_xr = !p.per_x && c == nx - 2;

    // Q of the rows of the previous and of this iteration, alternating
    // between two register arrays over the iteration pair.
    Real qA[kQ], qB[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) qA[q] = qB[q] = Real(0);
    // A value each wave forms for its own phase-2 rows, of this and of the
    // previous iteration: the family's V = B-1 dt Omega(f*) (kScheme 4,
    // formed in phase 2 for phase 3), or f^n (kFnRegs, formed in phase 1
    // for phase 2).
    Real vA[kQ], vB[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) vA[q] = vB[q] = Real(0);
    constexpr bool kFamily = kScheme >= 3;
    constexpr bool gen_bbar = kScheme == 4;

    // Iterations come in pairs (one per prefetch buffer); a trailing extra
    // iteration only reloads clamped rows and stores nothing (its rows fail
    // the row checks below).
    const int niter = ((y1 - y0 + kRowsPerIter - 1) / kRowsPerIter + 3) & ~1;

    // Row loads run two iterations ahead in two register buffers, so two
    // iterations of loads are in flight while the stencil phases compute.
    Store gA[kQ], gB[kQ];
    const int pitch = static_cast<int>(p.pitch);
    // Rows y0-4 .. y1+3 are needed; prefetches past the last one repeat it
    // (found in cache instead of fetched from HBM).
    auto load_row = [&](int pr, Store (&gb)[kQ]) {
      const int pc = min(pr, y1 + kHalo - 1);
      const int prm = p.per_y ? wrap_near(pc, ny) : clampi(pc, 0, ny - 1);
      const unsigned boff =
          (static_cast<unsigned>(prm) * static_cast<unsigned>(pitch) + static_cast<unsigned>(cm)) *
          static_cast<unsigned>(sizeof(Store));
      load_planes(src, plane * sizeof(Store), boff, gb);
    };
    load_row(y0 - kHalo + t, gA);
    load_row(y0 - kHalo + kRowsPerIter + t, gB);
    __syncthreads();  // ring zero-fill / previous piece complete

    auto iteration = [&](const int it, Store (&gb)[kQ], Real (&qnew)[kQ], const Real (&qold)[kQ],
                         Real (&vnew)[kQ], const Real (&vold)[kQ]) {
      const int p0 = y0 - kHalo + kRowsPerIter * it;

      // ---- phase 1: P (to LDS) and Q (registers) of row p0 + t; for
      // T2S2-FDLBM2 Q and f^n to LDS (P's coefficients then give f^n), or
      // f^n to registers (kFnRegs).
      {
        const int pr = p0 + t;
        Real g[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) g[q] = Cvt<Store>::ld(gb[q]);
        // Unconditional (rows are clamped or wrapped into the grid): the
        // buffers then stay in fixed registers with their loads in flight.
        load_row(pr + 2 * kRowsPerIter, gb);
        double s, jx, jy;
        moment_sums(g, s, jx, jy);
        Real rho, ux, uy;
        velocity(s, jx, jy, rho, ux, uy);
        if (kForce) {
          ux += static_cast<Real>(p.half_dt * p.Fx);
          uy += static_cast<Real>(p.half_dt * p.Fy);
        }
        const Real d = static_cast<Real>(s);
        Real X[kQ];
        eq_brackets(ux, uy, X);
        const auto& k = coef<Real>(p);
        Real* slotP = ringP + (pr & (kRing - 1)) * kNP * kLanes;
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          // E = (f^eq_q - w_q) / w_q; P and Q take their f^eq coefficient
          // times w_q per weight class.
          const Real E = d + rho * X[q];
          Real Pq = k.cPg * g[q] + k.kP[wclass(q)] * E;
          Real Qq = k.cQg * g[q] + k.kQ[wclass(q)] * E;
          Real Fq = Real(0);
          if (kForce) {
            Fq = force_term(q, p, ux, uy, E);
            Pq += static_cast<Real>(p.cPF) * Fq;
            Qq += static_cast<Real>(p.cQF) * Fq;
          }
          slotP[q * kLanes + lane] = kScheme == 2 ? Qq : Pq;
          if (kScheme == 2 && !kFnRegs && q > 0) slotP[(kQ + q - 1) * kLanes + lane] = Pq;
          if constexpr (kFnRegs) vnew[q] = Pq;
          if (kFamily) {
            slotP[(kQ + q) * kLanes + lane] = Qq;
            if (q > 0) {
              Real Uq = k.cU * g[q] + k.kU[wclass(q)] * E;  // f^n
              if (kForce) Uq += static_cast<Real>(p.cUF) * Fq;
              slotP[(2 * kQ + q - 1) * kLanes + lane] = Uq;
            }
          }
          qnew[q] = Qq;
          if constexpr (gen_bbar) {  // Q2 = f^n + B-0 dt Omega(f^n)
            Real Q2 = k.cQ2g * g[q] + k.kQ2[wclass(q)] * E;
            if (kForce) Q2 += static_cast<Real>(p.cQ2F) * Fq;
            qnew[q] = Q2;
          }
        }
      }
      __syncthreads();

      // ---- phase 2: S and R of row p0 - 2 + t (interior nodes), R (or the
      // scheme's combination T) to LDS.  The whole wave computes (the x taps
      // take neighbouring lanes' centre values); only interior lanes 2..61
      // store.
      {
        const int r = p0 - 2 + (gen_bbar || kFnRegs ? (t + 2) % kRowsPerIter : t);
        const bool row_ok =
            r >= y0 - 2 && r < y1 + 2 && (p.per_y || (r >= 1 && r <= ny - 2));
        if (row_ok) {
          const int rm = p.per_y ? wrap_near(r, ny) : r;
          Real wyr[kWeightsPerNode];
          row_weights(weights_y<Real>(p), rm, wyr);
          // One base pointer per ring row r-2 .. r+2 at this lane.
          const Real* rb[5];
#pragma unroll
          for (int o = 0; o < 5; ++o)
            rb[o] = ringP + ((r + o - 2) & (kRing - 1)) * kNP * kLanes + lane;
          const auto& k = coef<Real>(p);
          // A prediction along the characteristics from ring planes
          // [base, base + 9): S = centre + fac L(centre); then f at the
          // predicted time, R = cs S + ke E (+ cf F), from S's moments with
          // force shift hf.  With want_v, also V = B-1 dt Omega(R) (all
          // nine directions; R[0] stays 0, the rest direction has no
          // gradient).
          auto predict = [&](int base, Real fac, Real cs, const Real* ke, double cf, double hf,
                             Real (&S)[kQ], Real (&R)[kQ], Real& rho, Real& ux, Real& uy,
                             Real (&X)[kQ], bool want_v, Real (&V)[kQ]) {
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
              const int pq = (base + q) * kLanes;
              const Real centre = rb[2][pq];
              Real acc = Real(0);
              if (ex_of(q) > 0) acc = x_taps<0>(wxr, centre, acc);
              if (ex_of(q) < 0) acc = x_taps<1>(wxr, centre, acc);
              if (ey_of(q) != 0) {
                const int sy = ey_of(q) > 0 ? 0 : 1;
#pragma unroll
                for (int k2 = 0; k2 < kTaps; ++k2) acc += wyr[sy * kTaps + k2] * rb[k2 + sy][pq];
              }
              S[q] = q == 0 ? centre : centre + fac * acc;
            }
            double s, jx, jy;
            moment_sums(S, s, jx, jy);
            velocity(s, jx, jy, rho, ux, uy);
            if (kForce) {
              ux += static_cast<Real>(hf * p.Fx);
              uy += static_cast<Real>(hf * p.Fy);
            }
            const Real d = static_cast<Real>(s);
            eq_brackets(ux, uy, X);
            R[0] = Real(0);
#pragma unroll
            for (int q = 1; q < kQ; ++q) {
              const Real E = d + rho * X[q];
              Real Rq = cs * S[q] + ke[wclass(q)] * E;
              if (kForce) Rq += static_cast<Real>(cf) * force_term(q, p, ux, uy, E);
              R[q] = Rq;
            }
            if (want_v) {
              // Omega(f*) dt = w (f^eq* - f*) + dt F*, in deviations from w.
#pragma unroll
              for (int q = 0; q < kQ; ++q) {
                const Real E = d + rho * X[q];
                Real Fq = Real(0);
                if (kForce) Fq = force_term(q, p, ux, uy, E);
                Real Rq = cs * S[q] + ke[wclass(q)] * E;
                if (kForce) Rq += static_cast<Real>(cf) * Fq;
                Real Vq = k.kV[wclass(q)] * E - k.cV * Rq;
                if (kForce) Vq += static_cast<Real>(p.cVF) * Fq;
                V[q] = Vq;
              }
            }
          };
          Real S[kQ], R[kQ], X[kQ], rho, ux, uy;
          predict(0, k.A, k.cRs, k.kR, p.cRF, p.half_h, S, R, rho, ux, uy, X, gen_bbar, vnew);
          if (kSaveS && lane_o && col_interior && r >= y0 && r < y1) {
            Real* sv = static_cast<Real*>(p.save_s);
            const unsigned boff =
                (static_cast<unsigned>(r) * static_cast<unsigned>(pitch) + static_cast<unsigned>(c)) *
                static_cast<unsigned>(sizeof(Real));
#pragma unroll
            for (int q = 0; q < kQ; ++q) *at_byte(sv + q * plane, boff) = S[q];
          }
          // The family's second prediction: f^{n+1} from Q with h = dt.
          Real R2[kQ], X2[kQ], rho2 = Real(1), ux2 = Real(0), uy2 = Real(0);
#pragma unroll
          for (int q = 0; q < kQ; ++q) R2[q] = X2[q] = Real(0);
          if constexpr (kFamily) {
            Real S2[kQ];
            predict(kQ, Real(1), k.cU, k.kU, p.cUF, p.half_dt, S2, R2, rho2, ux2, uy2, X2, false,
                    S2);
          }
          // f^n of this node (kFnRegs): formed in phase 1 of this iteration
          // by waves 0 and 1, of the previous one by waves 2 and 3.
          Real fn[kQ];
#pragma unroll
          for (int q = 0; q < kQ; ++q) fn[q] = Real(0);
          if constexpr (kFnRegs) {
#pragma unroll
            for (int q = 1; q < kQ; ++q) fn[q] = t < 2 ? vnew[q] : vold[q];
          }
          // T, the field whose gradient the full step takes: R (scheme 1),
          // f^n + R (scheme 2, halved in phase 3), b0 f^n + b1 R + b2 R2
          // (scheme 3); f^n of (row, ln) from the ring (from fn with
          // kFnRegs, where (row, ln) is always this node).
          auto t_of = [&](int q, int row, int ln, Real r1, Real r2) {
            const Real* slot = ringP + (row & (kRing - 1)) * kNP * kLanes + ln;
            if (kScheme == 2) return r1 + (kFnRegs ? fn[q] : slot[(kQ + q - 1) * kLanes]);
            if (kFamily)
              return k.b[0] * slot[(2 * kQ + q - 1) * kLanes] + k.b[1] * r1 + k.b[2] * r2;
            return r1;
          };
          if (lane_r && col_interior) {
            Real* slotR = ringR + (r & (kRing - 1)) * (kQ - 1) * kLanes;
#pragma unroll
            for (int q = 1; q < kQ; ++q) slotR[(q - 1) * kLanes + lane] = t_of(q, r, lane, R[q], R2[q]);
            // Wall nodes whose nearest interior node is this one (eq 3.10
            // on f(t*) and f(t_{n+1}); corners take the diagonal
            // neighbour).  Physical f carries no force shift:
            // u_f = sum xi R / rho = u*.
            const bool src_yb = !p.per_y && r == 1;
            const bool src_yt = !p.per_y && r == ny - 2;
            if (kWalls && (src_xl || src_xr || src_yb || src_yt)) {
              for (int dy = -1; dy <= 1; ++dy) {
                if ((dy == -1 && !src_yb) || (dy == 1 && !src_yt)) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                  if ((dx == -1 && !src_xl) || (dx == 1 && !src_xr)) continue;
                  if (dx == 0 && dy == 0) continue;
                  // The shift from the brackets of u_f, formed above, and
                  // of the wall's velocity.
                  const Real* Xb = wall_brackets<Real>(p, wall_side_of(dx, dy));
                  Real sh[kQ], sh2[kQ];
                  nee_shift_x(rho, X, Xb, sh);
#pragma unroll
                  for (int q = 0; q < kQ; ++q) sh2[q] = Real(0);
                  if constexpr (kFamily) nee_shift_x(rho2, X2, Xb, sh2);
                  Real* slotW = dy == 1 ? topR : ringR + ((r + dy) & (kRing - 1)) * (kQ - 1) * kLanes;
#pragma unroll
                  for (int q = 1; q < kQ; ++q)
                    slotW[(q - 1) * kLanes + lane + dx] =
                        t_of(q, r + dy, lane + dx, R[q] + sh[q], R2[q] + sh2[q]);
                }
              }
            }
          }
        }
      }
      __syncthreads();

      // ---- phase 3: f~^{n+1} of row p0 - 4 + t (whole wave computes,
      // interior output lanes store).
      {
        const int o = p0 - 4 + t;
        const bool row_ok = o >= y0 && o < y1 && (p.per_y || (o >= 1 && o <= ny - 2));
        if (row_ok) {
          Real wyr[kWeightsPerNode];
          row_weights(weights_y<Real>(p), o, wyr);
          const Real* rb[5];
#pragma unroll
          for (int k = 0; k < 5; ++k) {
            rb[k] = ringR + ((o + k - 2) & (kRing - 1)) * (kQ - 1) * kLanes + lane;
            if (kWalls && !p.per_y && o + k - 2 == ny - 1) rb[k] = topR + lane;
          }
          Real out[kQ];
          // V of this row: formed in this iteration's phase 2 by waves 2
          // and 3, in the previous one's by waves 0 and 1.
          const bool v_now = t >= 2;
          out[0] = qold[0];
          if constexpr (gen_bbar) out[0] += v_now ? vnew[0] : vold[0];
#pragma unroll
          for (int q = 1; q < kQ; ++q) {
            const int pq = (q - 1) * kLanes;
            const Real centre = rb[2][pq];
            Real acc = kScheme == 2 ? Real(0) : qold[q];
            if constexpr (gen_bbar) acc += v_now ? vnew[q] : vold[q];
            if (ex_of(q) > 0) acc = x_taps<0>(wxr, centre, acc);
            if (ex_of(q) < 0) acc = x_taps<1>(wxr, centre, acc);
            if (ey_of(q) != 0) {
              const int sy = ey_of(q) > 0 ? 0 : 1;
#pragma unroll
              for (int k = 0; k < kTaps; ++k) acc += wyr[sy * kTaps + k] * rb[k + sy][pq];
            }
            out[q] = kScheme == 2 ? qold[q] + Real(0.5) * acc : acc;
          }
          if constexpr (gen_bbar) {
            // The implicit weight: f^{n+1} has Y's density and Y's momentum
            // plus B-2 dt rho F; the state is f~ = aY Y + aE (f^eq - w) + aF F
            // at that (rho, u).
            const auto& k = coef<Real>(p);
            double s, jx, jy;
            moment_sums(out, s, jx, jy);
            Real rho, ux, uy;
            velocity(s, jx, jy, rho, ux, uy);
            if (kForce) {
              ux += static_cast<Real>(p.b2dt * p.Fx);
              uy += static_cast<Real>(p.b2dt * p.Fy);
            }
            const Real d = static_cast<Real>(s);
            Real X[kQ];
            eq_brackets(ux, uy, X);
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
              const Real E = d + rho * X[q];
              Real o = k.aY * out[q] + k.kA[wclass(q)] * E;
              if (kForce) o += static_cast<Real>(p.aF) * force_term(q, p, ux, uy, E);
              out[q] = o;
            }
          }
          if (lane_o && col_interior) {
            const unsigned boff =
                (static_cast<unsigned>(o) * static_cast<unsigned>(pitch) + static_cast<unsigned>(c)) *
                static_cast<unsigned>(sizeof(Store));
            store_node(dst, plane, boff, out);
          }
        }
      }
    };

    for (int it = 0; it < niter; it += 2) {
      iteration(it, gA, qA, qB, vA, vB);
      iteration(it + 1, gB, qB, qA, vB, vA);
    }
    __syncthreads();  // the next piece reuses the rings; the piece's stores are visible
    if (kWalls) piece_walls(p, dst, x0, x1, y0, y1, threadIdx.x % kBlockThreads, kBlockThreads);
  }
}

// ---------------------------------------------------------------------------
// Tile step for small meshes (T2S2-FDLBM1 family).  A block of eight waves
// takes one strip (56 output columns) and kTileRows output rows as a whole
// tile instead of marching down a range of rows: it loads the tile's rows
// y0-4 .. y0+kTileRows+3 at once, forms P of all of them (LDS) and Q of its
// output rows (registers), then S and R of rows y0-2 .. y0+kTileRows+1
// (LDS), then the new state: three phases and two barriers, where a march
// over a few rows runs four pipelined iterations of three phases each.  Each
// node takes the expressions of step_kernel.  Wave w forms P of tile rows w
// and w+8 (rows counted from y0-4) and keeps Q of the one that is an output
// row (w+8 for w < 4, w otherwise), which it outputs in phase 3.  kSaveS
// also stores S at the interior nodes, as in step_kernel.
// ---------------------------------------------------------------------------
constexpr int kTileRows = 8;
constexpr int kTileWaves = 8;
constexpr int kTileIn = kTileRows + 2 * kHalo;   // rows of P
constexpr int kTileMid = kTileRows + kHalo;      // rows of R

template <typename Store, bool kForce, bool kWalls, bool kSaveS = false>
__global__ __launch_bounds__(kTileWaves * kLanes) void tile_step_kernel(StepParams p) {
  using Real = typename Cvt<Store>::R;
  __shared__ Real tP[kTileIn * kQ * kLanes];           // [row][q][lane]
  __shared__ Real tR[kTileMid * (kQ - 1) * kLanes];    // [row][q-1][lane]
  const int lane = threadIdx.x & (kLanes - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
  const int nx = p.nx, ny = p.ny;
  const Store* __restrict__ src = static_cast<const Store*>(p.src);
  Store* __restrict__ dst = static_cast<Store*>(p.dst);
  const long long plane = p.plane;
  const int pitch = static_cast<int>(p.pitch);
  const int ntiles = (ny + kTileRows - 1) / kTileRows;
  const int strip = blockIdx.x / ntiles;
  const int y0 = (blockIdx.x % ntiles) * kTileRows;
  const int y1 = min(y0 + kTileRows, ny);
  if (strip >= p.nstrips) return;  // whole block, before any barrier

  for (int i = threadIdx.x; i < kTileMid * (kQ - 1) * kLanes; i += kTileWaves * kLanes)
    tR[i] = Real(0);

  const int x0 = strip * kStripOut;
  const int x1 = min(x0 + kStripOut, nx);
  const int c = x0 - kHalo + lane;
  const int cm = p.per_x ? wrap(c, nx) : clampi(c, 0, nx - 1);
  Real wxr[kWeightsPerNode];
  {
    const Real* wx = weights_x<Real>(p);
#pragma unroll
    for (int k = 0; k < kWeightsPerNode; ++k) wxr[k] = wx[cm * kWeightsPerNode + k];
  }
  const bool col_interior = p.per_x || (c >= 1 && c <= nx - 2);
  const bool lane_r = lane >= 2 && lane < kLanes - 2;
  const bool lane_o = lane >= kHalo && lane < kLanes - kHalo && c < x1;
  const bool src_xl = !p.per_x && c == 1;
  const bool src_xr = !p.per_x && c == nx - 2;
  const auto& k = coef<Real>(p);

  // ---- phase 1: P of tile rows w and w + 8, Q of the wave's output row.
  const int jout = w < kHalo ? w + kTileWaves : w;
  Real qout[kQ];
  {
    Store gr[2][kQ];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int pr = y0 - kHalo + w + kTileWaves * h;
      const int prm = p.per_y ? wrap_near(pr, ny) : clampi(pr, 0, ny - 1);
      const unsigned boff =
          (static_cast<unsigned>(prm) * static_cast<unsigned>(pitch) + static_cast<unsigned>(cm)) *
          static_cast<unsigned>(sizeof(Store));
      load_planes(src, plane * sizeof(Store), boff, gr[h]);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = w + kTileWaves * h;
      Real g[kQ];
#pragma unroll
      for (int q = 0; q < kQ; ++q) g[q] = Cvt<Store>::ld(gr[h][q]);
      double s, jx, jy;
      moment_sums(g, s, jx, jy);
      Real rho, ux, uy;
      velocity(s, jx, jy, rho, ux, uy);
      if (kForce) {
        ux += static_cast<Real>(p.half_dt * p.Fx);
        uy += static_cast<Real>(p.half_dt * p.Fy);
      }
      const Real d = static_cast<Real>(s);
      Real X[kQ];
      eq_brackets(ux, uy, X);
      Real* row = tP + j * kQ * kLanes;
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const Real E = d + rho * X[q];
        Real Pq = k.cPg * g[q] + k.kP[wclass(q)] * E;
        Real Qq = k.cQg * g[q] + k.kQ[wclass(q)] * E;
        if (kForce) {
          const Real Fq = force_term(q, p, ux, uy, E);
          Pq += static_cast<Real>(p.cPF) * Fq;
          Qq += static_cast<Real>(p.cQF) * Fq;
        }
        row[q * kLanes + lane] = Pq;
        if (j == jout) qout[q] = Qq;
      }
    }
  }
  __syncthreads();

  // ---- phase 2: S and R of rows y0 - 2 + m, m = w and w + 8 (m < 12).
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int m = w + kTileWaves * h;
    if (m >= kTileMid) break;  // uniform per wave
    const int r = y0 - 2 + m;
    if (!(p.per_y || (r >= 1 && r <= ny - 2))) continue;
    const int rm = p.per_y ? wrap_near(r, ny) : r;
    Real wyr[kWeightsPerNode];
    row_weights(weights_y<Real>(p), rm, wyr);
    const Real* rb[5];
#pragma unroll
    for (int o = 0; o < 5; ++o) rb[o] = tP + (m + o) * kQ * kLanes + lane;
    Real S[kQ], R[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int pq = q * kLanes;
      const Real centre = rb[2][pq];
      Real acc = Real(0);
      if (ex_of(q) > 0) acc = x_taps<0>(wxr, centre, acc);
      if (ex_of(q) < 0) acc = x_taps<1>(wxr, centre, acc);
      if (ey_of(q) != 0) {
        const int sy = ey_of(q) > 0 ? 0 : 1;
#pragma unroll
        for (int k2 = 0; k2 < kTaps; ++k2) acc += wyr[sy * kTaps + k2] * rb[k2 + sy][pq];
      }
      S[q] = q == 0 ? centre : centre + k.A * acc;
    }
    if (kSaveS && lane_o && col_interior && r >= y0 && r < y1) {
      Real* sv = static_cast<Real*>(p.save_s);
      const unsigned boff =
          (static_cast<unsigned>(r) * static_cast<unsigned>(pitch) + static_cast<unsigned>(c)) *
          static_cast<unsigned>(sizeof(Real));
#pragma unroll
      for (int q = 0; q < kQ; ++q) *at_byte(sv + q * plane, boff) = S[q];
    }
    double s, jx, jy;
    moment_sums(S, s, jx, jy);
    Real rho, ux, uy;
    velocity(s, jx, jy, rho, ux, uy);
    if (kForce) {
      ux += static_cast<Real>(p.half_h * p.Fx);
      uy += static_cast<Real>(p.half_h * p.Fy);
    }
    const Real d = static_cast<Real>(s);
    Real X[kQ];
    eq_brackets(ux, uy, X);
    R[0] = Real(0);
#pragma unroll
    for (int q = 1; q < kQ; ++q) {
      const Real E = d + rho * X[q];
      Real Rq = k.cRs * S[q] + k.kR[wclass(q)] * E;
      if (kForce) Rq += static_cast<Real>(p.cRF) * force_term(q, p, ux, uy, E);
      R[q] = Rq;
    }
    if (lane_r && col_interior) {
      Real* slot = tR + m * (kQ - 1) * kLanes;
#pragma unroll
      for (int q = 1; q < kQ; ++q) slot[(q - 1) * kLanes + lane] = R[q];
      // Wall nodes whose nearest interior node is this one (eq 3.10 on
      // f(t*); corners take the diagonal neighbour); a wall row past the
      // tile's last R row is read by none of its outputs.
      const bool src_yb = !p.per_y && r == 1;
      const bool src_yt = !p.per_y && r == ny - 2;
      if (kWalls && (src_xl || src_xr || src_yb || src_yt)) {
        for (int dy = -1; dy <= 1; ++dy) {
          if ((dy == -1 && !src_yb) || (dy == 1 && !src_yt)) continue;
          if (m + dy < 0 || m + dy >= kTileMid) continue;
          for (int dx = -1; dx <= 1; ++dx) {
            if ((dx == -1 && !src_xl) || (dx == 1 && !src_xr)) continue;
            if (dx == 0 && dy == 0) continue;
            Real sh[kQ];
            nee_shift_x(rho, X, wall_brackets<Real>(p, wall_side_of(dx, dy)), sh);
            Real* slotW = tR + (m + dy) * (kQ - 1) * kLanes;
#pragma unroll
            for (int q = 1; q < kQ; ++q) slotW[(q - 1) * kLanes + lane + dx] = R[q] + sh[q];
          }
        }
      }
    }
  }
  __syncthreads();

  // ---- phase 3: the new state of the wave's output row o (R rows o-2..o+2
  // are tile rows jout-4 .. jout).
  {
    const int o = y0 - kHalo + jout;
    if (o < y1 && (p.per_y || (o >= 1 && o <= ny - 2))) {
      Real wyr[kWeightsPerNode];
      row_weights(weights_y<Real>(p), o, wyr);
      const Real* rb[5];
#pragma unroll
      for (int k2 = 0; k2 < 5; ++k2) rb[k2] = tR + (jout - kHalo + k2) * (kQ - 1) * kLanes + lane;
      Real out[kQ];
      out[0] = qout[0];
#pragma unroll
      for (int q = 1; q < kQ; ++q) {
        const int pq = (q - 1) * kLanes;
        const Real centre = rb[2][pq];
        Real acc = qout[q];
        if (ex_of(q) > 0) acc = x_taps<0>(wxr, centre, acc);
        if (ex_of(q) < 0) acc = x_taps<1>(wxr, centre, acc);
        if (ey_of(q) != 0) {
          const int sy = ey_of(q) > 0 ? 0 : 1;
#pragma unroll
          for (int k2 = 0; k2 < kTaps; ++k2) acc += wyr[sy * kTaps + k2] * rb[k2 + sy][pq];
        }
        out[q] = acc;
      }
      if (lane_o && col_interior) {
        const unsigned boff =
            (static_cast<unsigned>(o) * static_cast<unsigned>(pitch) + static_cast<unsigned>(c)) *
            static_cast<unsigned>(sizeof(Store));
        store_node(dst, plane, boff, out);
      }
    }
  }
  if (kWalls) {
    __syncthreads();  // the tile's stores are visible to the block
    piece_walls(p, dst, x0, x1, y0, y1, threadIdx.x, kTileWaves * kLanes);
  }
}

// ---------------------------------------------------------------------------
// Single-stencil step: the scheme at A = 0, Guo's T1S2-FDLBM (Remark I).
// With h = 0 the half-step prediction is the identity (S = P) and the mid-step
// map returns its input (R = S), so the step is
//   f~^{n+1} = Q - dt xi . grad_m R,  R = P = [2 f~ + w f^eq + dt F] / (2 + w),
// R being the physical f^n (eqs 2.18-2.20).  R is pointwise, so one pass
// forms R and Q of a row, puts R in an LDS ring, and takes the stencil of the
// row four above.  Strips are those of step_kernel (56 outputs; the stencil
// uses 2 of the 4 halo columns each side), marched from 2 rows above the
// piece instead of 4.  Wall nodes of R take eq 3.10 from their
// nearest interior node, written by that node's lane; the new state's wall
// nodes are set after each piece (piece_walls), as in step_kernel.  Each
// output takes
// the same expressions in the same order as step_kernel at A = 0 (where
// S = P + 0 L(P) and R = 1 S + 0 E reproduce P).
//
// Ring hazards, with rows p0..p0+3 loaded in an iteration and one barrier per
// iteration between its two phases: phase 1 writes rows p0..p0+3 and, for
// eq 3.10, wall rows p0-1 and p0+4; phase 2 reads rows p0-6..p0+1.  Over 16
// slots the rows written in phase 1 of the next iteration (p0+3..p0+8) share
// no slot with the rows still being read in phase 2 of this one.
// ---------------------------------------------------------------------------
template <typename Store, bool kForce, bool kWalls>
__global__ __launch_bounds__(step_threads(kStorageOf<Store>, 0), (kMinWaves<Store, kForce, kWalls, 1>)) void single_step_kernel(
    StepParams p) {
  using Real = typename Cvt<Store>::R;
  constexpr int kSB = strips_per_block(kStorageOf<Store>, 0);
  constexpr int kThreads = step_threads(kStorageOf<Store>, 0);
  constexpr int kSizeR = kRing1 * (kQ - 1) * kLanes;
  __shared__ Real ringR_all[kSB * kSizeR];  // per strip: [slot][q-1][lane]

  const int lane = threadIdx.x & (kLanes - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
  const int half = kSB == 1 ? 0 : wave / kRowsPerIter;
  const int t = kSB == 1 ? wave : wave % kRowsPerIter;
  Real* const ringR = ringR_all + half * kSizeR;
  const int nx = p.nx, ny = p.ny;
  const Store* __restrict__ src = static_cast<const Store*>(p.src);
  Store* __restrict__ dst = static_cast<Store*>(p.dst);
  const long long plane = p.plane;

  for (int i = threadIdx.x; i < kSB * kSizeR; i += kThreads) ringR_all[i] = Real(0);

  // Work order and XCD-aware block map as in step_kernel.
  const int G = gridDim.x;
  const int L = (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8;
  if (L >= p.nblocks) return;  // padding block: whole block, before any barrier
  const long long total = static_cast<long long>(p.nunits) * ny;
  const long long band_pieces = static_cast<long long>(p.nunits) * p.band;
  long long beg = total * L / p.nblocks;
  const long long end = total * (L + 1) / p.nblocks;

  while (beg < end) {  // uniform per block
    const int b = static_cast<int>(beg / band_pieces);
    const long long rem = beg - b * band_pieces;
    const int r0 = b * p.band;
    const int hb = min(p.band, ny - r0);
    const int strip = static_cast<int>(rem / hb) * kSB + half;
    const int y0 = r0 + static_cast<int>(rem % hb);
    const int y1 = static_cast<int>(min(static_cast<long long>(r0 + hb), y0 + (end - beg)));
    beg += y1 - y0;

    const int x0 = strip * kStripOut;
    const int x1 = min(x0 + kStripOut, nx);
    const int c = x0 - kHalo + lane;
    const int cm = p.per_x ? wrap(c, nx) : clampi(c, 0, nx - 1);
    Real wxr[kWeightsPerNode];
    {
      const Real* wx = weights_x<Real>(p);
#pragma unroll
      for (int k = 0; k < kWeightsPerNode; ++k) wxr[k] = wx[cm * kWeightsPerNode + k];
    }
    const bool col_interior = p.per_x || (c >= 1 && c <= nx - 2);
    const bool lane_o = lane >= kHalo && lane < kLanes - kHalo && c < x1;
    const bool src_xl = !p.per_x && c == 1;
    const bool src_xr = !p.per_x && c == nx - 2;

    Real qA[kQ], qB[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) qA[q] = qB[q] = Real(0);

    // Rows y0-2 .. y1+1 are needed, four per iteration from ybase = y0 - 2;
    // iteration it outputs the rows loaded in iteration it - 1 (so Q stays
    // in the registers of the wave that formed it).  Prefetches past the
    // last needed row repeat that row, which the cache still holds.
    const int ybase = y0 - kHalo1;
    const int ylast = y1 + kHalo1 - 1;
    const int niter = ((y1 - y0 + 1) / kRowsPerIter + 3) & ~1;

    Store gA[kQ], gB[kQ];
    const int pitch = static_cast<int>(p.pitch);
    auto load_row = [&](int pr, Store (&gb)[kQ]) {
      const int pc = min(pr, ylast);
      const int prm = p.per_y ? wrap_near(pc, ny) : clampi(pc, 0, ny - 1);
      const unsigned boff =
          (static_cast<unsigned>(prm) * static_cast<unsigned>(pitch) + static_cast<unsigned>(cm)) *
          static_cast<unsigned>(sizeof(Store));
      load_planes(src, plane * sizeof(Store), boff, gb);
    };
    load_row(ybase + t, gA);
    load_row(ybase + kRowsPerIter + t, gB);
    __syncthreads();  // ring zero-fill / previous piece complete

    auto iteration = [&](const int it, Store (&gb)[kQ], Real (&qnew)[kQ], const Real (&qold)[kQ]) {
      const int p0 = ybase + kRowsPerIter * it;

      // ---- phase 1: R (to LDS) and Q (registers) of row p0 + t.
      {
        const int pr = p0 + t;
        Real g[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) g[q] = Cvt<Store>::ld(gb[q]);
        load_row(pr + 2 * kRowsPerIter, gb);
        double s, jx, jy;
        moment_sums(g, s, jx, jy);
        Real rho, ux, uy;
        velocity(s, jx, jy, rho, ux, uy);
        if (kForce) {
          ux += static_cast<Real>(p.half_dt * p.Fx);
          uy += static_cast<Real>(p.half_dt * p.Fy);
        }
        const Real d = static_cast<Real>(s);
        Real X[kQ];
        eq_brackets(ux, uy, X);
        const auto& k = coef<Real>(p);
        Real R[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          const Real E = d + rho * X[q];
          Real Rq = k.cPg * g[q] + k.kP[wclass(q)] * E;
          Real Qq = k.cQg * g[q] + k.kQ[wclass(q)] * E;
          if (kForce) {
            const Real Fq = force_term(q, p, ux, uy, E);
            Rq += static_cast<Real>(p.cPF) * Fq;
            Qq += static_cast<Real>(p.cQF) * Fq;
          }
          R[q] = Rq;
          qnew[q] = Qq;
        }
        const bool row_int = p.per_y || (pr >= 1 && pr <= ny - 2);
        if (row_int && col_interior) {
          Real* slot = ringR + (pr & (kRing1 - 1)) * (kQ - 1) * kLanes;
#pragma unroll
          for (int q = 1; q < kQ; ++q) slot[(q - 1) * kLanes + lane] = R[q];
          // Wall nodes whose nearest interior node is this one (eq 3.10;
          // corners take the diagonal neighbour), from the moments of R.
          const bool src_yb = !p.per_y && pr == 1;
          const bool src_yt = !p.per_y && pr == ny - 2;
          if (kWalls && (src_xl || src_xr || src_yb || src_yt)) {
            double s2, jx2, jy2;
            moment_sums(R, s2, jx2, jy2);
            Real rho2, ux2, uy2;
            velocity(s2, jx2, jy2, rho2, ux2, uy2);
            Real X2[kQ];
            eq_brackets(ux2, uy2, X2);
            for (int dy = -1; dy <= 1; ++dy) {
              if ((dy == -1 && !src_yb) || (dy == 1 && !src_yt)) continue;
              for (int dx = -1; dx <= 1; ++dx) {
                if ((dx == -1 && !src_xl) || (dx == 1 && !src_xr)) continue;
                if (dx == 0 && dy == 0) continue;
                // A source in the strip's edge lane has its wall node outside
                // the strip; no output of this strip reads it.
                if (lane + dx < 0 || lane + dx >= kLanes) continue;
                Real sh[kQ];
                nee_shift_x(rho2, X2, wall_brackets<Real>(p, wall_side_of(dx, dy)), sh);
                Real* slotW = ringR + ((pr + dy) & (kRing1 - 1)) * (kQ - 1) * kLanes;
#pragma unroll
                for (int q = 1; q < kQ; ++q) slotW[(q - 1) * kLanes + lane + dx] = R[q] + sh[q];
              }
            }
          }
        }
      }
      __syncthreads();

      // ---- phase 2: f~^{n+1} of row p0 - 4 + t (whole wave computes,
      // interior output lanes store).
      {
        const int o = p0 - kRowsPerIter + t;
        const bool row_ok = o >= y0 && o < y1 && (p.per_y || (o >= 1 && o <= ny - 2));
        if (row_ok) {
          Real wyr[kWeightsPerNode];
          row_weights(weights_y<Real>(p), o, wyr);
          const Real* rb[5];
#pragma unroll
          for (int k = 0; k < 5; ++k)
            rb[k] = ringR + ((o + k - 2) & (kRing1 - 1)) * (kQ - 1) * kLanes + lane;
          Real out[kQ];
          out[0] = qold[0];
#pragma unroll
          for (int q = 1; q < kQ; ++q) {
            const int pq = (q - 1) * kLanes;
            const Real centre = rb[2][pq];
            Real acc = qold[q];
            if (ex_of(q) > 0) acc = x_taps<0>(wxr, centre, acc);
            if (ex_of(q) < 0) acc = x_taps<1>(wxr, centre, acc);
            if (ey_of(q) != 0) {
              const int sy = ey_of(q) > 0 ? 0 : 1;
#pragma unroll
              for (int k = 0; k < kTaps; ++k) acc += wyr[sy * kTaps + k] * rb[k + sy][pq];
            }
            out[q] = acc;
          }
          if (lane_o && col_interior) {
            const unsigned boff =
                (static_cast<unsigned>(o) * static_cast<unsigned>(pitch) + static_cast<unsigned>(c)) *
                static_cast<unsigned>(sizeof(Store));
            store_node(dst, plane, boff, out);
          }
        }
      }
    };

    for (int it = 0; it < niter; it += 2) {
      iteration(it, gA, qA, qB);
      iteration(it + 1, gB, qB, qA);
    }
    __syncthreads();  // the next piece reuses the ring; the piece's stores are visible
    if (kWalls) piece_walls(p, dst, x0, x1, y0, y1, threadIdx.x % kBlockThreads, kBlockThreads);
  }
}

// ---------------------------------------------------------------------------
// Auxiliary kernels: node-parallel, grid-stride.
// ---------------------------------------------------------------------------
template <typename Store>
__global__ __launch_bounds__(256) void init_macro_kernel(AuxParams a, Store* state,
                                                         const double* rho, const double* ux,
                                                         const double* uy, const double* grad) {
  const long long n = static_cast<long long>(a.nx) * a.ny;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    const int x = static_cast<int>(i % a.nx), y = static_cast<int>(i / a.nx);
    const double r = rho[i];
    double feq[kQ];
    feq_dev<double>(r - 1.0, r, ux[i], uy[i], feq);
    if (grad) {
      // eq 3.5 with rho0 = 1: rho0 w (2 tau + dt)/(2 c_s^2) xi_a xi_b d_a u_b
      const double dudx = grad[i], dudy = grad[n + i], dvdx = grad[2 * n + i],
                   dvdy = grad[3 * n + i];
      const double k = (2.0 * a.tau + a.dt) * 1.5;
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const double cx = ex_of(q), cy = ey_of(q);
        const double contr = cx * cx * dudx + cx * cy * (dudy + dvdx) + cy * cy * dvdy;
        feq[q] -= w_of(q) * k * contr;
      }
    }
    const long long base = static_cast<long long>(y) * a.pitch + x;
#pragma unroll
    for (int q = 0; q < kQ; ++q) state[q * a.plane + base] = Cvt<Store>::st(feq[q]);
  }
}

template <typename Store>
__global__ __launch_bounds__(256) void load_dist_kernel(AuxParams a, Store* state,
                                                        const double* g) {
  const long long n = static_cast<long long>(a.nx) * a.ny;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n * kQ; i += 256LL * gridDim.x) {
    const long long q = i / n, j = i % n;
    const int x = static_cast<int>(j % a.nx), y = static_cast<int>(j / a.nx);
    state[q * a.plane + static_cast<long long>(y) * a.pitch + x] =
        Cvt<Store>::st(static_cast<typename Cvt<Store>::R>(g[i]));
  }
}

template <typename Store>
__global__ __launch_bounds__(256) void read_dist_kernel(AuxParams a, const Store* state,
                                                        double* g) {
  const long long n = static_cast<long long>(a.nx) * a.ny;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n * kQ; i += 256LL * gridDim.x) {
    const long long q = i / n, j = i % n;
    const int x = static_cast<int>(j % a.nx), y = static_cast<int>(j / a.nx);
    g[i] = static_cast<double>(
        Cvt<Store>::ld(state[q * a.plane + static_cast<long long>(y) * a.pitch + x]));
  }
}

template <typename Store>
__device__ inline void node_moments(const AuxParams& a, const Store* state, int x, int y,
                                    double& s, double& ux, double& uy, bool& finite) {
  const long long base = static_cast<long long>(y) * a.pitch + x;
  double v[kQ];
  finite = true;
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    v[q] = static_cast<double>(Cvt<Store>::ld(state[q * a.plane + base]));
    finite = finite && isfinite(v[q]);
  }
  double jx, jy;
  moment_sums(v, s, jx, jy);
  const double rho = 1.0 + s;
  ux = jx / rho + a.half_dt * a.Fx;
  uy = jy / rho + a.half_dt * a.Fy;
}

template <typename Store>
__global__ __launch_bounds__(256) void moments_kernel(AuxParams a, const Store* state,
                                                      double* drho, double* ux, double* uy) {
  const long long n = static_cast<long long>(a.nx) * a.ny;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    const int x = static_cast<int>(i % a.nx), y = static_cast<int>(i / a.nx);
    double s, u, v;
    bool fin;
    node_moments(a, state, x, y, s, u, v, fin);
    if (drho) drho[i] = s;
    if (ux) ux[i] = u;
    if (uy) uy[i] = v;
  }
}

// Deterministic two-pass reduction: fixed grid of kDiagBlocks blocks, each
// thread accumulates a fixed grid-stride subset, each wave reduces its lanes
// with wave_sum / wave_max, the block adds its four wave results in wave
// order, and one final block reduces the partials in a fixed order.
template <typename Store>
__global__ __launch_bounds__(256) void diag_partial_kernel(AuxParams a, const Store* state,
                                                           double* partials) {
  __shared__ double red[kDiagSlots][256 / kLanes];
  double acc[kDiagSlots] = {0, 0, 0, 0, 0, 0, 0, 0};
  const long long n = static_cast<long long>(a.nx) * a.ny;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    const int x = static_cast<int>(i % a.nx), y = static_cast<int>(i / a.nx);
    double s, u, v;
    bool fin;
    node_moments(a, state, x, y, s, u, v, fin);
    const double J = a.jx[x] * a.jy[y];
    const double rho = 1.0 + s;
    if (fin) {
      acc[0] += J * s;
      acc[1] += J * rho * 0.5 * (u * u + v * v);
      acc[2] = fmax(acc[2], sqrt(u * u + v * v));
      acc[4] += J * rho * u;
      acc[5] += J * rho * v;
    } else {
      acc[3] += 1.0;
    }
  }
  const int lane = threadIdx.x & (kLanes - 1), wave = threadIdx.x / kLanes;
#pragma unroll
  for (int k = 0; k < kDiagSlots; ++k) {
    const double v = k == 2 ? wave_max(acc[k]) : wave_sum(acc[k]);
    if (lane == 0) red[k][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < kDiagSlots) {
    const int k = threadIdx.x;
    double v = red[k][0];
    for (int w = 1; w < 256 / kLanes; ++w) v = k == 2 ? fmax(v, red[k][w]) : v + red[k][w];
    partials[blockIdx.x * kDiagSlots + k] = v;
  }
}

// Final pass: wave w reduces slots w, w + 4; lane l takes the partials of
// blocks l, l + 64, ... in that order, then the butterfly combines the
// lanes.  The loads of a lane are independent, so they are in flight
// together (a walk over the blocks one at a time waited out a cache round
// trip per block).
// The first nout slots go to result.
__global__ __launch_bounds__(256) void diag_final_kernel(const double* partials, int nblocks,
                                                         double* result, int nout) {
  const int lane = threadIdx.x & (kLanes - 1), wave = threadIdx.x / kLanes;
  for (int k = wave; k < kDiagSlots; k += 256 / kLanes) {  // uniform per wave
    double acc = 0.0;
    for (int b = lane; b < nblocks; b += kLanes) {
      const double v = partials[b * kDiagSlots + k];
      acc = (k == 2) ? fmax(acc, v) : acc + v;
    }
    acc = k == 2 ? wave_max(acc) : wave_sum(acc);
    if (lane == 0 && k < nout) result[k] = acc;
  }
}

// Sums for the global relative error of the velocity against a reference
// field (eq 3.6, and the residual form of Sec. 3C): slot 0 sum |u - u'|^2,
// slot 1 sum |u'|^2, slot 3 sum |u|^2, over all nodes, the other slots
// zero (slot 2 is a max in the final pass).  Same fixed partition and order
// as the diagnostics.
template <typename Store>
__global__ __launch_bounds__(256) void gre_partial_kernel(AuxParams a, const Store* state,
                                                          const double* uref,
                                                          const double* vref,
                                                          double* partials) {
  __shared__ double red[3][256 / kLanes];
  double acc[3] = {0.0, 0.0, 0.0};
  const long long n = static_cast<long long>(a.nx) * a.ny;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    const int x = static_cast<int>(i % a.nx), y = static_cast<int>(i / a.nx);
    double s, u, v;
    bool fin;
    node_moments(a, state, x, y, s, u, v, fin);
    const double ur = uref[i], vr = vref[i];
    const double du = u - ur, dv = v - vr;
    acc[0] += du * du + dv * dv;
    acc[1] += ur * ur + vr * vr;
    acc[2] += u * u + v * v;
  }
  const int lane = threadIdx.x & (kLanes - 1), wave = threadIdx.x / kLanes;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double v = wave_sum(acc[k]);
    if (lane == 0) red[k][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < kDiagSlots) {
    const int k = threadIdx.x;
    double v[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      v[j] = red[j][0];
      for (int w = 1; w < 256 / kLanes; ++w) v[j] += red[j][w];
    }
    partials[blockIdx.x * kDiagSlots + k] =
        k == 0 ? v[0] : (k == 1 ? v[1] : (k == 3 ? v[2] : 0.0));
  }
}

template <typename Store, int kScheme>
void launch_fused(const StepParams& p, dim3 g, dim3 b, hipStream_t s, bool walls) {
  if (p.has_force) {
    if (walls)
      hipLaunchKernelGGL((step_kernel<Store, true, true, kScheme>), g, b, 0, s, p);
    else
      hipLaunchKernelGGL((step_kernel<Store, true, false, kScheme>), g, b, 0, s, p);
  } else {
    if (walls)
      hipLaunchKernelGGL((step_kernel<Store, false, true, kScheme>), g, b, 0, s, p);
    else
      hipLaunchKernelGGL((step_kernel<Store, false, false, kScheme>), g, b, 0, s, p);
  }
}

template <typename Store>
void launch_single(const StepParams& p, dim3 g, dim3 b, hipStream_t s, bool walls) {
  if (p.has_force) {
    if (walls)
      hipLaunchKernelGGL((single_step_kernel<Store, true, true>), g, b, 0, s, p);
    else
      hipLaunchKernelGGL((single_step_kernel<Store, true, false>), g, b, 0, s, p);
  } else {
    if (walls)
      hipLaunchKernelGGL((single_step_kernel<Store, false, true>), g, b, 0, s, p);
    else
      hipLaunchKernelGGL((single_step_kernel<Store, false, false>), g, b, 0, s, p);
  }
}

template <typename Store>
void launch_tile(const StepParams& p, hipStream_t s, bool walls) {
  const dim3 g(p.nstrips * ((p.ny + kTileRows - 1) / kTileRows)), b(kTileWaves * kLanes);
  if (p.has_force) {
    if (walls)
      hipLaunchKernelGGL((tile_step_kernel<Store, true, true>), g, b, 0, s, p);
    else
      hipLaunchKernelGGL((tile_step_kernel<Store, true, false>), g, b, 0, s, p);
  } else {
    if (walls)
      hipLaunchKernelGGL((tile_step_kernel<Store, false, true>), g, b, 0, s, p);
    else
      hipLaunchKernelGGL((tile_step_kernel<Store, false, false>), g, b, 0, s, p);
  }
}

template <typename Store>
hipError_t launch_step_t(const StepParams& p, int grid, hipStream_t s) {
  const dim3 g(grid), b(step_threads(kStorageOf<Store>, p.single ? 0 : p.scheme));
  const bool walls = !p.per_x || !p.per_y;
  if (p.tile)
    launch_tile<Store>(p, s, walls);
  else if (p.single)
    launch_single<Store>(p, g, b, s, walls);
  else if (p.scheme == 1)
    launch_fused<Store, 1>(p, g, b, s, walls);
  else if constexpr (kStochastic<Store>)
    return hipErrorInvalidValue;  // the stochastic forms run scheme 1 only
  else if (p.scheme == 2)
    launch_fused<Store, 2>(p, g, b, s, walls);
  else if (p.gen_bbar)
    launch_fused<Store, 4>(p, g, b, s, walls);
  else
    launch_fused<Store, 3>(p, g, b, s, walls);
  return hipGetLastError();
}

int aux_grid(long long n) {
  long long g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return static_cast<int>(g);
}

}  // namespace

size_t storage_bytes(int storage) {
  switch (storage) {
    case kF64: return 8;
    case kF32: return 4;
    case kBF16: return 2;
    case kF16: return 2;
    case kBF16Sr: return 2;
    case kF16Sr: return 2;
    default: return 0;
  }
}

#define T2S2_DISPATCH(storage, CALL)                                  \
  switch (storage) {                                                  \
    case kF64: { using Store = double; CALL; } break;                 \
    case kF32: { using Store = float; CALL; } break;                  \
    case kBF16: { using Store = Bf16; CALL; } break;                  \
    case kF16: { using Store = _Float16; CALL; } break;               \
    case kBF16Sr: { using Store = Bf16Sr; CALL; } break;              \
    case kF16Sr: { using Store = F16Sr; CALL; } break;                \
    default: return hipErrorInvalidValue;                             \
  }

template <typename Store, int kScheme>
int occupancy_s(bool force, bool walls) {
  int n = 0;
  hipError_t e;
  if (force)
    e = walls ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &n, step_kernel<Store, true, true, kScheme>, step_threads(kStorageOf<Store>, kScheme), 0)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &n, step_kernel<Store, true, false, kScheme>, step_threads(kStorageOf<Store>, kScheme), 0);
  else
    e = walls ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &n, step_kernel<Store, false, true, kScheme>, step_threads(kStorageOf<Store>, kScheme), 0)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &n, step_kernel<Store, false, false, kScheme>, step_threads(kStorageOf<Store>, kScheme), 0);
  return e == hipSuccess ? n : -1;
}

template <typename Store>
int occupancy_single(bool force, bool walls) {
  int n = 0;
  const int threads = step_threads(kStorageOf<Store>, 0);
  hipError_t e;
  if (force)
    e = walls ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, single_step_kernel<Store, true, true>, threads, 0)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, single_step_kernel<Store, true, false>, threads, 0);
  else
    e = walls ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, single_step_kernel<Store, false, true>, threads, 0)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, single_step_kernel<Store, false, false>, threads, 0);
  return e == hipSuccess ? n : -1;
}

template <typename Store>
int occupancy_t(bool force, bool walls, int scheme) {
  if (scheme == 0) return occupancy_single<Store>(force, walls);
  if (scheme == 1) return occupancy_s<Store, 1>(force, walls);
  if constexpr (kStochastic<Store>) {
    return -1;  // scheme 1 only
  } else {
    if (scheme == 2) return occupancy_s<Store, 2>(force, walls);
    if (scheme == 4) return occupancy_s<Store, 4>(force, walls);
    return occupancy_s<Store, 3>(force, walls);
  }
}

int step_blocks_per_cu(int storage, bool force, bool walls, int scheme) {
  switch (storage) {
    case kF64: return occupancy_t<double>(force, walls, scheme);
    case kF32: return occupancy_t<float>(force, walls, scheme);
    case kBF16: return occupancy_t<Bf16>(force, walls, scheme);
    case kF16: return occupancy_t<_Float16>(force, walls, scheme);
    case kBF16Sr: return occupancy_t<Bf16Sr>(force, walls, scheme);
    case kF16Sr: return occupancy_t<F16Sr>(force, walls, scheme);
    default: return -1;
  }
}

hipError_t launch_step(int storage, const StepParams& p, int grid, hipStream_t s) {
  T2S2_DISPATCH(storage, return launch_step_t<Store>(p, grid, s));
  return hipSuccess;
}

// The adjoint's recompute: the unforced T2S2-FDLBM1-family step from p.src
// into p.dst, storing S into p.save_s as well.  The new state's wall nodes
// are not set (the adjoint reads it at interior nodes only).
template <typename Store>
hipError_t launch_step_save_s_t(const StepParams& p, int grid, hipStream_t s) {
  const dim3 g(grid), b(step_threads(kStorageOf<Store>, 1));
  if (p.tile) {
    const dim3 gt(p.nstrips * ((p.ny + kTileRows - 1) / kTileRows)), bt(kTileWaves * kLanes);
    if (!p.per_x || !p.per_y)
      hipLaunchKernelGGL((tile_step_kernel<Store, false, true, true>), gt, bt, 0, s, p);
    else
      hipLaunchKernelGGL((tile_step_kernel<Store, false, false, true>), gt, bt, 0, s, p);
    return hipGetLastError();
  }
  if (!p.per_x || !p.per_y)
    hipLaunchKernelGGL((step_kernel<Store, false, true, 1, true>), g, b, 0, s, p);
  else
    hipLaunchKernelGGL((step_kernel<Store, false, false, 1, true>), g, b, 0, s, p);
  return hipGetLastError();
}

hipError_t launch_step_save_s(int storage, const StepParams& p, int grid, hipStream_t s) {
  if (p.has_force || p.scheme != 1 || p.single || !p.save_s) return hipErrorInvalidValue;
  // The adjoint covers the storage forms rounded to nearest.
  switch (storage) {
    case kF64: return launch_step_save_s_t<double>(p, grid, s);
    case kF32: return launch_step_save_s_t<float>(p, grid, s);
    case kBF16: return launch_step_save_s_t<Bf16>(p, grid, s);
    case kF16: return launch_step_save_s_t<_Float16>(p, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_init_macro(int storage, const AuxParams& a, void* state, const double* rho,
                             const double* ux, const double* uy, const double* grad,
                             hipStream_t s) {
  const int grid = aux_grid(static_cast<long long>(a.nx) * a.ny);
  T2S2_DISPATCH(storage,
                hipLaunchKernelGGL(init_macro_kernel<Store>, dim3(grid), dim3(256), 0, s, a,
                                   static_cast<Store*>(state), rho, ux, uy, grad));
  return hipGetLastError();
}

hipError_t launch_load_dist(int storage, const AuxParams& a, void* state, const double* g,
                            hipStream_t s) {
  const int grid = aux_grid(static_cast<long long>(a.nx) * a.ny * kQ);
  T2S2_DISPATCH(storage, hipLaunchKernelGGL(load_dist_kernel<Store>, dim3(grid), dim3(256), 0,
                                            s, a, static_cast<Store*>(state), g));
  return hipGetLastError();
}

hipError_t launch_read_dist(int storage, const AuxParams& a, const void* state, double* g,
                            hipStream_t s) {
  const int grid = aux_grid(static_cast<long long>(a.nx) * a.ny * kQ);
  T2S2_DISPATCH(storage, hipLaunchKernelGGL(read_dist_kernel<Store>, dim3(grid), dim3(256), 0,
                                            s, a, static_cast<const Store*>(state), g));
  return hipGetLastError();
}

hipError_t launch_moments(int storage, const AuxParams& a, const void* state, double* drho,
                          double* ux, double* uy, hipStream_t s) {
  const int grid = aux_grid(static_cast<long long>(a.nx) * a.ny);
  T2S2_DISPATCH(storage, hipLaunchKernelGGL(moments_kernel<Store>, dim3(grid), dim3(256), 0, s,
                                            a, static_cast<const Store*>(state), drho, ux, uy));
  return hipGetLastError();
}

hipError_t launch_diagnostics(int storage, const AuxParams& a, const void* state,
                              double* partials, double* result, int nout, hipStream_t s) {
  T2S2_DISPATCH(storage,
                hipLaunchKernelGGL(diag_partial_kernel<Store>, dim3(kDiagBlocks), dim3(256), 0,
                                   s, a, static_cast<const Store*>(state), partials));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(256), 0, s, partials, kDiagBlocks, result,
                     nout);
  return hipGetLastError();
}

hipError_t launch_velocity_error(int storage, const AuxParams& a, const void* state,
                                 const double* uref, const double* vref, double* partials,
                                 double* result, hipStream_t s) {
  T2S2_DISPATCH(storage,
                hipLaunchKernelGGL(gre_partial_kernel<Store>, dim3(kDiagBlocks), dim3(256), 0,
                                   s, a, static_cast<const Store*>(state), uref, vref, partials));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(256), 0, s, partials, kDiagBlocks, result,
                     kDiagSlots);
  return hipGetLastError();
}

}  // namespace t2s2
