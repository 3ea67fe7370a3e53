// Internal declarations shared by the t2s2 host code and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace t2s2 {

// D2Q9 velocities in the order printed in Sec. 3 of the paper.
constexpr int kQ = 9;

// Strip geometry of the fused step: one 64-lane wave covers 64 consecutive
// columns; the outer 4 on each side are halo (the output depends on f~ up to
// 4 nodes away along each axis), so a strip produces 56 output columns.
constexpr int kLanes = 64;
constexpr int kHalo = 4;
constexpr int kStripOut = kLanes - 2 * kHalo;
// The single-stencil step that the scheme reduces to at A = 0 (Guo's T1S2,
// Remark I: the half-step prediction is the identity) reaches 2 nodes along
// each axis.  It keeps the 56-column strips (the FP64 row stores of a strip
// then start on a 64-byte boundary and fill whole 64-byte segments; 60-column
// strips measured 17% slower), but needs only 2 halo rows, and its LDS ring
// holds 16 rows (rows p0..p0+3 written while rows p0-6..p0+1 are read, so one
// barrier per iteration suffices).
constexpr int kHalo1 = 2;
constexpr int kRing1 = 16;
// The tile kernel (small meshes) takes 8 output rows per block; it replaces
// the march when a march block would hold fewer unit-rows than this (the
// crossover measured on cavities from 65^2 to 2049^2, all storages).
constexpr int kTileMaxMarchRows = 24;
// Rows advanced per iteration of the y-march = waves per block.
constexpr int kRowsPerIter = 4;
constexpr int kBlockThreads = kLanes * kRowsPerIter;
// LDS ring depth in rows (P rows [p0-4, p0+4), R rows [p0-6, p0+2)).
constexpr int kRing = 8;

// Stencil weights per node and sign of the velocity component: 4 taps.
// sign > 0: offsets (-2, -1, 0, +1); sign < 0: offsets (-1, 0, +1, +2).
constexpr int kTaps = 4;
constexpr int kWeightsPerNode = 2 * kTaps;

// Storage codes (match include/t2s2.h).  kBF16Sr and kF16Sr hold the bits
// of kBF16 and kF16; the step rounds its new interior values stochastically.
enum Storage { kF64 = 0, kF32 = 1, kBF16 = 2, kF16 = 3, kBF16Sr = 4, kF16Sr = 5 };

// Strips marched side by side by one block of the fused step.  Two for the
// FP32-storage T2S2-FDLBM1 family: the cache lines the two strips share
// are then loaded by one CU in the same iteration, and two such blocks
// still fit on a CU.  One otherwise: FP64 rings fit only once per CU in a
// two-strip block, and a single block per CU stalls the whole CU at every
// barrier; T2S2-FDLBM2's wider rings do not fit twice.
// Scheme code 0 here is the single-stencil (A = 0) step, which takes two
// strips per FP32 block as well.
__host__ __device__ constexpr int strips_per_block(int storage, int scheme) {
  return ((scheme == 1 || scheme == 0) && storage == kF32) ? 2 : 1;
}
__host__ __device__ constexpr int step_threads(int storage, int scheme) {
  return kBlockThreads * strips_per_block(storage, scheme);
}

struct StepParams {
  const void* src;
  void* dst;
  int nx, ny;
  long long pitch;  // elements per row
  long long plane;  // elements per population plane (ny * pitch)
  int per_x, per_y;
  int nstrips;  // strips of kStripOut output columns
  int nunits;   // groups of strips_per_block(storage, scheme) neighbouring strips
  int nblocks;  // equal ranges of the nunits * ny unit-rows, one per block
  int band;     // rows per band of the band-major strip-row order
  int scheme;   // 1: T2S2-FDLBM1 family (eq 2.23); 2: T2S2-FDLBM2 (eq 5.23);
                // 3: the eq 2.13 family with gradient weights b
  int single;   // scheme 1 at A = 0 (T1S2): the single-stencil kernel
  int tile;     // small mesh, scheme 1 with A > 0: the tile kernel, one block
                // per strip and kTileRows rows (grid nstrips * row tiles)
  void* save_s; // adjoint recompute only: S in the arithmetic type, else NULL
  const double* wx;   // [nx][2][4] dt-scaled x weights (FP64)
  const double* wy;   // [ny][2][4]
  const float* wx32;  // same in FP32
  const float* wy32;
  double A;
  double cPg, cPe, cPF;  // P = cPg g + cPe (feq - w) + cPF F
  double cQg, cQe, cQF;  // Q = cQg g + cQe (feq - w) + cQF F
  double cRs, cRe, cRF;  // R = cRs S + cRe (feq* - w) + cRF F*
  double cUg, cUe, cUF;  // f at h = dt: cUg X + cUe (feq(X) - w) + cUF F(X)
  double b[3];           // gradient weights of L(f^n), L(f*), L(f^{n+1})
  // Collision weights of the family other than (1/2, 0, 1/2) (gen_bbar):
  //   Q2 = f^n + B-0 dt Omega(f^n) = cQ2g g + cQ2e (feq - w) + cQ2F F
  //     (the base of the update, in place of Q),
  //   V  = B-1 dt Omega(f*) = cV ((feq* - w) - (f* - w)) + cVF F*,
  //   and the new state from Y = Q2 + V + dt L(T), the implicit weight
  //   solved through Y's moments (velocity shift b2dt = B-2 dt):
  //   f~ = aY Y + aE (feq - w) + aF F.
  int gen_bbar;
  double bbar[3];
  double cQ2g, cQ2e, cQ2F, cV, cVF, aY, aE, aF, b2dt;
  double half_dt, half_h;
  double Fx, Fy;
  double uw[4][2];
  // Brackets X_q(u_b) = 3 e + 9/2 e^2 - 3/2 |u_b|^2 (e = xi_q . u_b) of each
  // wall's velocity, for the extrapolation of eq 3.10 (sides: x = 0,
  // x = nx-1, y = 0, y = ny-1), FP64 and FP32.
  double xb[4][kQ];
  float xb32[4][kQ];
  int has_force;
  // The coefficients in the arithmetic type of the kernel: cPg, cQg, cRs,
  // A, cU = cUg, and per lattice-weight class c (rest, axis, diagonal) the
  // products kP[c] = cPe w_c, kQ[c] = cQe w_c, kR[c] = cRe w_c,
  // kU[c] = cUe w_c, which multiply E = drho + rho X of f^eq - w = w E;
  // the family's weights b.
  template <typename Real>
  struct Coef {
    Real cPg, cQg, cRs, A, cU;
    Real kP[3], kQ[3], kR[3], kU[3];
    Real b[3];
    // gen_bbar: cQ2g, cV, aY and per weight class kQ2[c] = cQ2e w_c,
    // kV[c] = cV w_c, kA[c] = aE w_c.
    Real cQ2g, cV, aY;
    Real kQ2[3], kV[3], kA[3];
  };
  Coef<double> c64;
  Coef<float> c32;
};

struct AuxParams {
  int nx, ny;
  long long pitch, plane;
  double tau, dt;       // for the eq 3.5 correction
  double half_dt, Fx, Fy;
  const double* jx;     // trapezoid measure [nx]
  const double* jy;     // [ny]
};

// Von Neumann stability maps (t2s2_stability.hip).
struct StabArgs {
  int model;  // 0: eq 4.7; 1: eq 2.23 step, exact; 2: eq 5.23 step, exact;
              // 3: the eq 2.13 family step with gradient weights bt and
              //    collision weights bb (gen_bb: other than (1/2, 0, 1/2)), exact
  double eta, A, b2bar, b2tilde, ux, uy;
  double bt[3];
  double bb[3];
  int gen_bb;
  int nkx, nky;             // k grid: theta_x = thx0 + i dthx, theta_y = j dthy
  double thx0, dthx, dthy;
  int squarings;
};
hipError_t launch_stability(const StabArgs& a, const double* omega, const double* r, int npoints,
                            double* radius, hipStream_t s);

// Adjoint of the step (t2s2_adjoint.hip).  Real-typed buffers (FP64 for
// T2S2_F64 storage, FP32 otherwise) share the state's pitched layout.
struct AdjParams {
  int nx, ny;
  long long pitch, plane;
  int per_x, per_y;
  const double* wx;
  const double* wy;
  const float* wx32;
  const float* wy32;
  double A;
  double cPg, cPe, cQg, cQe, cRs, cRe;
  double dcPg, dcQg, dcRs;  // d/d omega of cPg, cQg, cRs
  double dnu_per_domega;    // d omega / d nu = -omega / nu at a fixed dt (0 without collision)
  double uw[4][2];
  void* S;     // S, from the recompute of the step
  void* mu;    // adjoint of the interior output (= adjoint of Q); walled domains
  void* next;  // f~^{n+1} recomputed (storage type)
  // Plan of the reverse march (plan_adjoint_march): eight-wave blocks or
  // four, and the block count (at most kAdjMaxBlocks).
  int march_rows8;
  int march_grid;
};

constexpr int kDiagBlocks = 512;
constexpr int kDiagSlots = 8;
// Blocks of the reverse march of the adjoint (one d/d omega partial each).
constexpr int kAdjMaxBlocks = 1024;

// Launchers (t2s2_kernels.hip).  Return hipError_t of the launch.
hipError_t launch_step(int storage, const StepParams& p, int grid, hipStream_t s);
hipError_t launch_step_save_s(int storage, const StepParams& p, int grid, hipStream_t s);
// Resident step-kernel blocks per CU for this variant (-1 on error); scheme
// 0 is the single-stencil (A = 0) kernel, 4 the family (scheme 3) with
// collision weights other than (1/2, 0, 1/2).
int step_blocks_per_cu(int storage, bool force, bool walls, int scheme);
hipError_t launch_init_macro(int storage, const AuxParams& a, void* state, const double* rho,
                             const double* ux, const double* uy, const double* grad,
                             hipStream_t s);
hipError_t launch_load_dist(int storage, const AuxParams& a, void* state, const double* g,
                            hipStream_t s);
hipError_t launch_read_dist(int storage, const AuxParams& a, const void* state, double* g,
                            hipStream_t s);
hipError_t launch_moments(int storage, const AuxParams& a, const void* state, double* drho,
                          double* ux, double* uy, hipStream_t s);
// kDiagBlocks * kDiagSlots partials; the first nout of the kDiagSlots
// results go to result.
hipError_t launch_diagnostics(int storage, const AuxParams& a, const void* state,
                              double* partials, double* result, int nout, hipStream_t s);
hipError_t launch_velocity_error(int storage, const AuxParams& a, const void* state,
                                 const double* uref, const double* vref, double* partials,
                                 double* result, hipStream_t s);

size_t storage_bytes(int storage);

// Reference copy of nine planes of `plane` elements of elem_bytes (8, 4 or
// 2) bytes (t2s2_probe.hip).
hipError_t launch_copy_probe(const void* src, void* dst, long long plane, int elem_bytes,
                             hipStream_t s);

// Adjoint launchers (t2s2_adjoint.hip).
size_t adjoint_real_bytes(int storage);
// Sets a.march_rows8 and a.march_grid for this mesh, storage and device
// (cus compute units): as many blocks as fit on the device at once.
hipError_t plan_adjoint_march(int storage, AdjParams& a, int cus);
hipError_t launch_adjoint_step(int storage, const AdjParams& a, const StepParams& sp,
                               int step_grid, const void* state_n, const void* lam_np1,
                               void* lam_n, double* partial, double* accum, hipStream_t s);
// The reverse stages alone, given S of the step from state_n and the new
// state state_np1 (from launch_step_save_s).
hipError_t launch_adjoint_step_stored(int storage, const AdjParams& a, const void* state_n,
                                      const void* state_np1, const void* s_n,
                                      const void* lam_np1, void* lam_n, double* partial,
                                      double* accum, hipStream_t s);
hipError_t launch_adjoint_seed(int storage, const AdjParams& a, const void* state,
                               const double* gu, const double* gv, void* lam, hipStream_t s);
hipError_t launch_adjoint_init(int storage, const AdjParams& a, const void* lam,
                               const double* rho, const double* ux, const double* uy,
                               double* grho, double* gux, double* guy, hipStream_t s);
hipError_t launch_adjoint_convert(int storage, const AdjParams& a, const void* lam,
                                  double* dense, const double* dense_in, void* lam_out,
                                  hipStream_t s);

}  // namespace t2s2
