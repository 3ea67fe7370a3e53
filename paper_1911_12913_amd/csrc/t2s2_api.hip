// C-ABI of the t2s2 library (declared in include/t2s2.h): argument checks,
// time step and stencil coefficients on the host, launch plan, ping-pong
// state.  The library allocates no device memory: the caller provides the
// two state buffers and the workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/t2s2.h"
#include "t2s2_internal.h"

using namespace t2s2;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(T2S2_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

// Metric 1/x'(i) with x'(i) = (x[i+1] - x[i-1]) / 2 (period added across a
// periodic seam); zero on wall nodes, which are never differentiated.
std::vector<double> metric(const std::vector<double>& c, bool per, double period) {
  const int n = static_cast<int>(c.size());
  std::vector<double> m(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double cm, cp;
    if (per) {
      cm = i == 0 ? c[n - 1] - period : c[i - 1];
      cp = i == n - 1 ? c[0] + period : c[i + 1];
    } else {
      if (i == 0 || i == n - 1) continue;
      cm = c[i - 1];
      cp = c[i + 1];
    }
    m[i] = 2.0 / (cp - cm);
  }
  return m;
}

// Trapezoid measure of each node (diagnostics).
std::vector<double> measure(const std::vector<double>& c, bool per, double period) {
  const int n = static_cast<int>(c.size());
  std::vector<double> J(n);
  for (int i = 0; i < n; ++i) {
    if (per) {
      const double cm = i == 0 ? c[n - 1] - period : c[i - 1];
      const double cp = i == n - 1 ? c[0] + period : c[i + 1];
      J[i] = 0.5 * (cp - cm);
    } else if (i == 0) {
      J[i] = 0.5 * (c[1] - c[0]);
    } else if (i == n - 1) {
      J[i] = 0.5 * (c[n - 1] - c[n - 2]);
    } else {
      J[i] = 0.5 * (c[i + 1] - c[i - 1]);
    }
  }
  return J;
}

// dt-scaled stencil weights of -xi_a d/dx_a per node: for each sign of the
// velocity component, the 4 taps of the mixed difference (eqs 2.36-2.38 with
// eta the upwind weight) times the metric.  sign > 0 taps at offsets
// (-2,-1,0,+1), sign < 0 at (-1,0,+1,+2).  At the first interior node of a
// walled axis the upwind point outside the domain is replaced by quadratic
// extrapolation, which turns that upwind difference into the central one.
std::vector<double> stencil_weights(const std::vector<double>& m, bool per, double eta,
                                    double dt) {
  const int n = static_cast<int>(m.size());
  std::vector<double> w(static_cast<size_t>(n) * kWeightsPerNode, 0.0);
  const double up_pos[kTaps] = {eta / 2.0, -(1.0 + 3.0 * eta) / 2.0, 3.0 * eta / 2.0,
                                (1.0 - eta) / 2.0};
  const double up_neg[kTaps] = {-(1.0 - eta) / 2.0, -3.0 * eta / 2.0, (1.0 + 3.0 * eta) / 2.0,
                                -eta / 2.0};
  const double cen_pos[kTaps] = {0.0, -0.5, 0.0, 0.5};
  const double cen_neg[kTaps] = {-0.5, 0.0, 0.5, 0.0};
  for (int i = 0; i < n; ++i) {
    if (!per && (i == 0 || i == n - 1)) continue;
    const double* ap = (!per && i == 1) ? cen_pos : up_pos;
    const double* an = (!per && i == n - 2) ? cen_neg : up_neg;
    for (int k = 0; k < kTaps; ++k) {
      w[static_cast<size_t>(i) * kWeightsPerNode + k] = -dt * m[i] * ap[k];
      w[static_cast<size_t>(i) * kWeightsPerNode + kTaps + k] = dt * m[i] * an[k];
    }
  }
  return w;
}

bool check_axis(const double* c, int n, int per, double period, std::string& why) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(c[i])) {
      why = "non-finite coordinate";
      return false;
    }
  for (int i = 1; i < n; ++i)
    if (!(c[i] > c[i - 1])) {
      why = "coordinates must be strictly increasing";
      return false;
    }
  if (per && !(std::isfinite(period) && period > c[n - 1] - c[0])) {
    why = "period must exceed the coordinate span";
    return false;
  }
  return true;
}

// Strip plan of the step kernel that p selects: strips of 56 output columns
// grouped into units of the kernel's strips per block.  The block count is
// set at bind time (plan_blocks).
void plan_strips(StepParams& p, int storage) {
  p.nstrips = (p.nx + kStripOut - 1) / kStripOut;
  const int spb = strips_per_block(storage, p.single ? 0 : p.scheme);
  p.nunits = (p.nstrips + spb - 1) / spb;
  p.nblocks = 8;
  p.band = p.ny;
}

// Band height of the march's split of nunits x ny unit-rows over nb blocks:
// one block's share, so that away from the last band a block owns one unit
// of one band.
int band_of(long long nunits, int ny, long long nb) {
  const long long rows = nunits * ny;
  return static_cast<int>(std::min<long long>(ny, std::max<long long>(1, (rows + nb - 1) / nb)));
}

// Work of the busiest block under that split, in unit-rows: the rows of its
// range plus kPieceWork for each piece the range is cut into at unit and
// band ends (a piece refills the march's pipeline: it loads the four rows
// above and below its range again and runs its leading and trailing
// iterations).  The ranges and pieces are enumerated as the step kernels
// cut them.  A last band of a few rows cuts each range that covers it into
// one piece per unit: on a 4060^2 grid in FP64 the default 512 blocks leave
// a last band of 7 rows and 74 pieces in the busiest range.
constexpr long long kPieceWork = 4;  // fitted to step times at 1101^2 - 4060^2
long long busiest_block_work(long long nunits, int ny, long long nb) {
  const int band = band_of(nunits, ny, nb);
  const long long total = nunits * ny, band_rows = nunits * band;
  long long worst = 0;
  for (long long L = 0; L < nb; ++L) {
    long long beg = total * L / nb;
    const long long end = total * (L + 1) / nb;
    long long work = end - beg;
    while (beg < end) {
      const long long b = beg / band_rows, rem = beg - b * band_rows;
      const long long r0 = b * band, hb = std::min<long long>(band, ny - r0);
      const long long y0 = r0 + rem % hb;
      const long long y1 = std::min(r0 + hb, y0 + (end - beg));
      beg += y1 - y0;
      work += kPieceWork;
    }
    worst = std::max(worst, work);
  }
  return worst;
}

// One block per resident slot (CUs x blocks per CU), so every block runs in
// a single wave of the grid with an equal share of the unit-rows (a unit is
// the block's group of neighbouring strips), as long as a share keeps at
// least 8 unit-rows.  Smaller meshes, where a block's march is a few
// latency-bound iterations, use one block per CU (equal work on every CU)
// while a share keeps at least 4 unit-rows, and below that one block per 4
// unit-rows.  A multiple of 8 for the XCD-aware block order.  Where that
// count cuts the ranges into many pieces, a count up to a quarter smaller
// whose busiest block does at least 3% less work (busiest_block_work) is
// taken instead: a step lasts as long as its busiest block, since with
// fewer blocks than slots each block marches at about the same rate.
// Returns the grid size, or -1 if the kernel cannot be resident.
int plan_blocks(StepParams& p, int storage, int cus) {
  const bool walls = !p.per_x || !p.per_y;
  // Kernel scheme codes: 0 the single-stencil step, 4 the family with
  // collision weights other than (1/2, 0, 1/2).
  const int kscheme = p.single ? 0 : (p.scheme == 3 && p.gen_bbar ? 4 : p.scheme);
  const int per_cu = step_blocks_per_cu(storage, p.has_force != 0, walls, kscheme);
  if (per_cu < 1) return -1;
  const long long rows = static_cast<long long>(p.nunits) * p.ny;
  const long long slots = static_cast<long long>(cus) * per_cu;
  long long nb = rows >= 8 * slots ? slots : (rows >= 4LL * cus ? cus : rows / 4);
  const char* forced = std::getenv("T2S2_BLOCKS");
  if (forced) nb = std::atoll(forced);
  nb = std::max<long long>(8, nb / 8 * 8);
  nb = std::min<long long>(nb, std::max<long long>(8, rows / 8 * 8));
  if (!forced) {
    const long long w0 = busiest_block_work(p.nunits, p.ny, nb);
    long long best = nb, wbest = w0;
    for (long long c = nb - 8; c >= std::max<long long>(8, nb - nb / 4); c -= 8) {
      const long long w = busiest_block_work(p.nunits, p.ny, c);
      if (w < wbest) {
        wbest = w;
        best = c;
      }
    }
    if (wbest * 100 < w0 * 97) nb = best;
  }
  p.nblocks = static_cast<int>(nb);
  // The blocks of neighbouring units in a band march the same rows at the
  // same time, so the halo lines they share are fetched once.
  p.band = band_of(p.nunits, p.ny, nb);
  return static_cast<int>(nb);
}

}  // namespace

// Reduction partials of t2s2_diagnostics_noalloc: a file-scope device array
// (one copy per device, held until the process ends) instead of workspace
// memory.  In host code `scratch` names a host-side stand-in, not device
// memory; its device address comes from hipGetSymbolAddress, once per device
// (scratch_address), and only that address reaches the kernels.
constexpr int kNoAllocDoubles = kDiagBlocks * kDiagSlots;  // 32 KiB
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on device dev, which must be current; looked
// up on the first call for that device (t2s2_bind) and kept.
hipError_t scratch_address(int dev, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}
}  // namespace

struct t2s2_ctx {
  t2s2_config cfg;
  int device = -1;  // device current at bind
  int nx = 0, ny = 0;
  long long pitch = 0;
  double dt = 0, tau = 0, omega = 0;
  std::vector<double> wx, wy, jx, jy;
  std::vector<float> wx32, wy32;
  size_t off_wx = 0, off_wy = 0, off_wx32 = 0, off_wy32 = 0, off_jx = 0, off_jy = 0,
         off_part = 0, off_res = 0, ws_bytes = 0;
  void* state[2] = {nullptr, nullptr};
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  bool bound = false;
  int cur = 0;
  int64_t steps = 0;
  StepParams sp{};
  AuxParams ap{};
  int grid = 0;
  // The two-stencil kernels' plan of the same step (their own occupancy),
  // for the adjoint's recompute, which stores S, formed only by step_kernel
  // and tile_step_kernel; equal to sp unless sp.single.
  StepParams sp_gen{};
  int grid_gen = 0;
  // adjoint
  AdjParams adj{};
  bool adj_bound = false;
  double* adj_partial = nullptr;
  size_t adj_state_bytes = 0;
  // captured multi-step graph
  hipGraphExec_t graph = nullptr;
  int graph_steps = 0;
  int graph_cur = 0;  // buffer holding the state when the graph starts
  ~t2s2_ctx() {
    if (graph) (void)hipGraphExecDestroy(graph);
  }
};

namespace {
void drop_graph(t2s2_ctx* c) {
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  c->graph = nullptr;
  c->graph_steps = 0;
}
}  // namespace

extern "C" {

const char* t2s2_last_error(void) { return g_last_error.c_str(); }

int t2s2_create(const t2s2_config* cfg, const double* x, int nx, const double* y, int ny,
                t2s2_ctx** out) {
  g_last_error.clear();
  if (!out) return fail(T2S2_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!cfg || !x || !y) return fail(T2S2_ERR_INVALID_ARG, "NULL config or coordinates");
  if (nx < 5 || ny < 5) return fail(T2S2_ERR_INVALID_ARG, "nx and ny must be >= 5");
  if (nx > (1 << 20) || ny > (1 << 20) || static_cast<long long>(nx) * ny > (1LL << 31))
    return fail(T2S2_ERR_INVALID_ARG, "mesh too large");
  std::string why;
  if (!check_axis(x, nx, cfg->periodic_x, cfg->period_x, why))
    return fail(T2S2_ERR_INVALID_ARG, "x: " + why);
  if (!check_axis(y, ny, cfg->periodic_y, cfg->period_y, why))
    return fail(T2S2_ERR_INVALID_ARG, "y: " + why);
  if (!(cfg->nu > 0.0)) return fail(T2S2_ERR_INVALID_ARG, "nu must be > 0 (or +INFINITY)");
  if (!(cfg->dt > 0.0) && !(cfg->cfl > 0.0 && cfg->cfl <= 1.0))
    return fail(T2S2_ERR_INVALID_ARG, "cfl must be in (0, 1] when dt <= 0");
  if (cfg->dt > 0.0 && !std::isfinite(cfg->dt)) return fail(T2S2_ERR_INVALID_ARG, "dt not finite");
  if (!(cfg->eta >= 0.0 && cfg->eta <= 1.0)) return fail(T2S2_ERR_INVALID_ARG, "eta not in [0,1]");
  if (!(cfg->A >= 0.0 && cfg->A <= 1.0)) return fail(T2S2_ERR_INVALID_ARG, "A not in [0,1]");
  if (cfg->storage < T2S2_F64 || cfg->storage > T2S2_F16_SR_DEV)
    return fail(T2S2_ERR_INVALID_ARG, "unknown storage");
  if (cfg->scheme != 0 && cfg->scheme != T2S2_FDLBM1 && cfg->scheme != T2S2_FDLBM2 &&
      cfg->scheme != T2S2_FAMILY)
    return fail(T2S2_ERR_INVALID_ARG, "unknown scheme");
  if ((cfg->storage == T2S2_BF16_SR_DEV || cfg->storage == T2S2_F16_SR_DEV) &&
      cfg->scheme != 0 && cfg->scheme != T2S2_FDLBM1)
    return fail(T2S2_ERR_UNSUPPORTED, "stochastically rounded storage runs T2S2_FDLBM1 only");
  if (cfg->scheme == T2S2_FAMILY) {
    const double* b = cfg->btilde;
    for (int k = 0; k < 3; ++k)
      if (!(b[k] >= 0.0 && b[k] <= (k == 2 ? 0.5 : 1.0)))
        return fail(T2S2_ERR_INVALID_ARG, "btilde: B~0, B~1 in [0,1], B~2 in [0,1/2]");
    if (!(std::fabs(b[0] + b[1] + b[2] - 1.0) <= 1e-12))
      return fail(T2S2_ERR_INVALID_ARG, "btilde must sum to 1 (eq 2.14a)");
    const double* bb = cfg->bbar;
    if (!(bb[0] == 0.0 && bb[1] == 0.0 && bb[2] == 0.0)) {
      for (int k = 0; k < 3; ++k)
        if (!(bb[k] >= 0.0 && bb[k] <= (k == 2 ? 0.5 : 1.0)))
          return fail(T2S2_ERR_INVALID_ARG, "bbar: B-0, B-1 in [0,1], B-2 in [0,1/2]");
      if (!(std::fabs(bb[0] + bb[1] + bb[2] - 1.0) <= 1e-12))
        return fail(T2S2_ERR_INVALID_ARG, "bbar must sum to 1 (eq 2.14a)");
    }
  }
  // The step kernel addresses a population plane with 32-bit byte offsets.
  if (static_cast<long long>(ny) * ((nx + 63) / 64 * 64) *
          static_cast<long long>(storage_bytes(cfg->storage)) >= (1LL << 32))
    return fail(T2S2_ERR_UNSUPPORTED, "one population plane (ny * pitch elements) must be under 4 GiB");
  if (!std::isfinite(cfg->force[0]) || !std::isfinite(cfg->force[1]))
    return fail(T2S2_ERR_INVALID_ARG, "force not finite");
  for (int s = 0; s < 4; ++s)
    if (!std::isfinite(cfg->u_wall[s][0]) || !std::isfinite(cfg->u_wall[s][1]))
      return fail(T2S2_ERR_INVALID_ARG, "wall velocity not finite");

  t2s2_ctx* c = new t2s2_ctx();
  c->cfg = *cfg;
  c->nx = nx;
  c->ny = ny;
  c->pitch = (nx + 63) / 64 * 64;
  std::vector<double> xs(x, x + nx), ys(y, y + ny);

  // eq 3.1 with xi = 1 and dx = the smallest node spacing over both axes.
  double dmin = INFINITY;
  for (int i = 1; i < nx; ++i) dmin = std::fmin(dmin, xs[i] - xs[i - 1]);
  for (int i = 1; i < ny; ++i) dmin = std::fmin(dmin, ys[i] - ys[i - 1]);
  if (cfg->periodic_x) dmin = std::fmin(dmin, xs[0] + cfg->period_x - xs[nx - 1]);
  if (cfg->periodic_y) dmin = std::fmin(dmin, ys[0] + cfg->period_y - ys[ny - 1]);
  c->dt = cfg->dt > 0.0 ? cfg->dt : cfg->cfl * dmin;
  c->tau = 3.0 * cfg->nu;
  c->omega = std::isinf(cfg->nu) ? 0.0 : c->dt / c->tau;

  const int scheme = cfg->scheme == T2S2_FDLBM2 ? 2 : (cfg->scheme == T2S2_FAMILY ? 3 : 1);
  c->cfg.scheme = scheme;
  // T2S2-FDLBM2 predicts with a full step (h = dt, A = 1 in the maps below)
  // and needs the physical f^n, which is P at A = 0.
  const double A = scheme == 2 ? 1.0 : cfg->A, Ap = scheme == 2 ? 0.0 : A;
  const double w = c->omega, dt = c->dt;
  StepParams& p = c->sp;
  p.scheme = scheme;
  // At A = 0 the half step is the identity and one stencil remains (T1S2).
  p.single = (scheme == 1 && A == 0.0) ? 1 : 0;
  p.nx = nx;
  p.ny = ny;
  p.pitch = c->pitch;
  p.plane = c->pitch * ny;
  p.per_x = cfg->periodic_x ? 1 : 0;
  p.per_y = cfg->periodic_y ? 1 : 0;
  p.A = A;
  // Closed forms of the pointwise maps in terms of w = dt / tau:
  //   P = fbar^{+,h} = [(2 - A w) f~ + (1 + A) w f^eq + (1 + A) dt F] / (2 + w)
  //   Q = f~^+       = [(2 - w) f~ + 2 w f^eq + 2 dt F] / (2 + w)
  //   R = f(t*)      = [2 S + A w f^eq* + A dt F*] / (2 + A w)
  p.cPg = (2.0 - Ap * w) / (2.0 + w);
  p.cPe = (1.0 + Ap) * w / (2.0 + w);
  p.cPF = (1.0 + Ap) * dt / (2.0 + w);
  p.cQg = (2.0 - w) / (2.0 + w);
  p.cQe = 2.0 * w / (2.0 + w);
  p.cQF = 2.0 * dt / (2.0 + w);
  p.cRs = 2.0 / (2.0 + A * w);
  p.cRe = A * w / (2.0 + A * w);
  p.cRF = A * dt / (2.0 + A * w);
  // The family (scheme 3) also takes f at h = dt from f~ or from fbar(t_{n+1}):
  //   U = [2 X + w f^eq + dt F] / (2 + w)  (f^n from f~^n, f^{n+1} from S2),
  // and weighs the three gradients by btilde.
  p.cUg = 2.0 / (2.0 + w);
  p.cUe = w / (2.0 + w);
  p.cUF = dt / (2.0 + w);
  for (int k = 0; k < 3; ++k) p.b[k] = scheme == 3 ? cfg->btilde[k] : (k == 1 ? 1.0 : 0.0);
  // Collision weights of the family (all zero: (1/2, 0, 1/2)).  Other than
  // (1/2, 0, 1/2), with w = dt / tau and Omega(f) dt = w (f^eq - f) + dt F:
  //   Q2 = f^n + B-0 dt Omega(f^n), f^n = cUg f~ + cUe f^eq + cUF F:
  //     cQ2g = (1 - B-0 w) cUg, cQ2e = (1 - B-0 w) cUe + B-0 w,
  //     cQ2F = (1 - B-0 w) cUF + B-0 dt;
  //   V = B-1 dt Omega(f*): cV = B-1 w, cVF = B-1 dt;
  //   f^{n+1} = [Y + B-2 (w f^eq + dt F)] / (1 + B-2 w) and
  //   f~ = f^{n+1} + (w/2) (f^{n+1} - f^eq) - (dt/2) F (eq 2.19):
  //     aY = (1 + w/2) / (1 + B-2 w), aE = w (B-2 - 1/2) / (1 + B-2 w),
  //     aF = dt (B-2 - 1/2) / (1 + B-2 w).
  {
    const double* bb = cfg->bbar;
    const bool zero = bb[0] == 0.0 && bb[1] == 0.0 && bb[2] == 0.0;
    const double b0 = zero ? 0.5 : bb[0], b1 = zero ? 0.0 : bb[1], b2 = zero ? 0.5 : bb[2];
    p.gen_bbar = (scheme == 3 && !(b0 == 0.5 && b1 == 0.0 && b2 == 0.5)) ? 1 : 0;
    p.bbar[0] = b0;
    p.bbar[1] = b1;
    p.bbar[2] = b2;
    p.cQ2g = (1.0 - b0 * w) * p.cUg;
    p.cQ2e = (1.0 - b0 * w) * p.cUe + b0 * w;
    p.cQ2F = (1.0 - b0 * w) * p.cUF + b0 * dt;
    p.cV = b1 * w;
    p.cVF = b1 * dt;
    p.aY = (1.0 + 0.5 * w) / (1.0 + b2 * w);
    p.aE = w * (b2 - 0.5) / (1.0 + b2 * w);
    p.aF = dt * (b2 - 0.5) / (1.0 + b2 * w);
    p.b2dt = b2 * dt;
    c->cfg.bbar[0] = b0;
    c->cfg.bbar[1] = b1;
    c->cfg.bbar[2] = b2;
  }
  {
    const double wc[3] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0};
    p.c64.cPg = p.cPg;
    p.c64.cQg = p.cQg;
    p.c64.cRs = p.cRs;
    p.c64.A = A;
    p.c64.cU = p.cUg;
    for (int k = 0; k < 3; ++k) {
      p.c64.kP[k] = p.cPe * wc[k];
      p.c64.kQ[k] = p.cQe * wc[k];
      p.c64.kR[k] = p.cRe * wc[k];
      p.c64.kU[k] = p.cUe * wc[k];
      p.c64.b[k] = p.b[k];
      p.c64.kQ2[k] = p.cQ2e * wc[k];
      p.c64.kV[k] = p.cV * wc[k];
      p.c64.kA[k] = p.aE * wc[k];
    }
    p.c64.cQ2g = p.cQ2g;
    p.c64.cV = p.cV;
    p.c64.aY = p.aY;
    p.c32.cPg = static_cast<float>(p.c64.cPg);
    p.c32.cQg = static_cast<float>(p.c64.cQg);
    p.c32.cRs = static_cast<float>(p.c64.cRs);
    p.c32.A = static_cast<float>(A);
    p.c32.cU = static_cast<float>(p.c64.cU);
    for (int k = 0; k < 3; ++k) {
      p.c32.kP[k] = static_cast<float>(p.c64.kP[k]);
      p.c32.kQ[k] = static_cast<float>(p.c64.kQ[k]);
      p.c32.kR[k] = static_cast<float>(p.c64.kR[k]);
      p.c32.kU[k] = static_cast<float>(p.c64.kU[k]);
      p.c32.b[k] = static_cast<float>(p.c64.b[k]);
      p.c32.kQ2[k] = static_cast<float>(p.c64.kQ2[k]);
      p.c32.kV[k] = static_cast<float>(p.c64.kV[k]);
      p.c32.kA[k] = static_cast<float>(p.c64.kA[k]);
    }
    p.c32.cQ2g = static_cast<float>(p.c64.cQ2g);
    p.c32.cV = static_cast<float>(p.c64.cV);
    p.c32.aY = static_cast<float>(p.c64.aY);
  }
  p.half_dt = 0.5 * dt;
  p.half_h = 0.5 * A * dt;
  p.Fx = cfg->force[0];
  p.Fy = cfg->force[1];
  p.has_force = (cfg->force[0] != 0.0 || cfg->force[1] != 0.0) ? 1 : 0;
  for (int s = 0; s < 4; ++s) {
    p.uw[s][0] = cfg->u_wall[s][0];
    p.uw[s][1] = cfg->u_wall[s][1];
    // D2Q9 velocities in the paper's order (Sec. 3).
    static const int ex[kQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static const int ey[kQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const double ux = p.uw[s][0], uy = p.uw[s][1], uu = 1.5 * (ux * ux + uy * uy);
    for (int q = 0; q < kQ; ++q) {
      const double e = ex[q] * ux + ey[q] * uy;
      p.xb[s][q] = e * (3.0 + 4.5 * e) - uu;
      p.xb32[s][q] = static_cast<float>(p.xb[s][q]);
    }
  }

  c->wx = stencil_weights(metric(xs, cfg->periodic_x, cfg->period_x), cfg->periodic_x, cfg->eta, dt);
  c->wy = stencil_weights(metric(ys, cfg->periodic_y, cfg->period_y), cfg->periodic_y, cfg->eta, dt);
  c->wx32.assign(c->wx.begin(), c->wx.end());
  c->wy32.assign(c->wy.begin(), c->wy.end());
  c->jx = measure(xs, cfg->periodic_x, cfg->period_x);
  c->jy = measure(ys, cfg->periodic_y, cfg->period_y);

  // Launch plans; the block counts are set at bind time from the device's
  // CU count and the kernels' occupancy.
  plan_strips(p, cfg->storage);
  c->grid = 8;
  c->sp_gen = p;
  c->sp_gen.single = 0;
  plan_strips(c->sp_gen, cfg->storage);
  c->grid_gen = 8;

  size_t off = 0;
  c->off_wx = off;
  off = align256(off + c->wx.size() * sizeof(double));
  c->off_wy = off;
  off = align256(off + c->wy.size() * sizeof(double));
  c->off_wx32 = off;
  off = align256(off + c->wx32.size() * sizeof(float));
  c->off_wy32 = off;
  off = align256(off + c->wy32.size() * sizeof(float));
  c->off_jx = off;
  off = align256(off + c->jx.size() * sizeof(double));
  c->off_jy = off;
  off = align256(off + c->jy.size() * sizeof(double));
  c->off_part = off;
  off = align256(off + static_cast<size_t>(kDiagBlocks) * kDiagSlots * sizeof(double));
  c->off_res = off;
  off = align256(off + kDiagSlots * sizeof(double));
  c->ws_bytes = off;

  AuxParams& a = c->ap;
  a.nx = nx;
  a.ny = ny;
  a.pitch = c->pitch;
  a.plane = c->pitch * ny;
  a.tau = c->tau;
  a.dt = dt;
  a.half_dt = 0.5 * dt;
  a.Fx = cfg->force[0];
  a.Fy = cfg->force[1];
  *out = c;
  return T2S2_OK;
}

size_t t2s2_state_bytes(const t2s2_ctx* c) {
  if (!c) return 0;
  return static_cast<size_t>(kQ) * c->ny * c->pitch * storage_bytes(c->cfg.storage);
}

size_t t2s2_workspace_bytes(const t2s2_ctx* c) { return c ? c->ws_bytes : 0; }

int t2s2_bind(t2s2_ctx* c, void* state_a, void* state_b, void* workspace, void* stream) {
  g_last_error.clear();
  if (!c) return fail(T2S2_ERR_INVALID_ARG, "NULL context");
  if (!state_a || !state_b || !workspace || state_a == state_b)
    return fail(T2S2_ERR_INVALID_ARG, "need two distinct state buffers and a workspace");
  if ((reinterpret_cast<uintptr_t>(state_a) | reinterpret_cast<uintptr_t>(state_b) |
       reinterpret_cast<uintptr_t>(workspace)) & 255)
    return fail(T2S2_ERR_INVALID_ARG, "buffers must be 256-byte aligned");
  drop_graph(c);  // a captured graph holds the previous buffer addresses
  c->state[0] = state_a;
  c->state[1] = state_b;
  c->ws = static_cast<char*>(workspace);
  c->stream = static_cast<hipStream_t>(stream);
  hipError_t e;
  struct {
    size_t off;
    const void* src;
    size_t bytes;
  } up[] = {{c->off_wx, c->wx.data(), c->wx.size() * sizeof(double)},
            {c->off_wy, c->wy.data(), c->wy.size() * sizeof(double)},
            {c->off_wx32, c->wx32.data(), c->wx32.size() * sizeof(float)},
            {c->off_wy32, c->wy32.data(), c->wy32.size() * sizeof(float)},
            {c->off_jx, c->jx.data(), c->jx.size() * sizeof(double)},
            {c->off_jy, c->jy.data(), c->jy.size() * sizeof(double)}};
  for (auto& u : up) {
    e = hipMemcpyAsync(c->ws + u.off, u.src, u.bytes, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(e, "bind: upload");
  }
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "bind: synchronize");
  c->sp.wx = reinterpret_cast<const double*>(c->ws + c->off_wx);
  c->sp.wy = reinterpret_cast<const double*>(c->ws + c->off_wy);
  c->sp.wx32 = reinterpret_cast<const float*>(c->ws + c->off_wx32);
  c->sp.wy32 = reinterpret_cast<const float*>(c->ws + c->off_wy32);
  c->ap.jx = reinterpret_cast<const double*>(c->ws + c->off_jx);
  c->ap.jy = reinterpret_cast<const double*>(c->ws + c->off_jy);
  c->sp_gen.wx = c->sp.wx;
  c->sp_gen.wy = c->sp.wy;
  c->sp_gen.wx32 = c->sp.wx32;
  c->sp_gen.wy32 = c->sp.wy32;
  int dev = 0, cus = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "bind: device query");
  c->device = dev;
  // The no-allocation diagnostics' scratch: its device address is looked up
  // here, at set-up with the device current, so that the entry point itself
  // (possibly under graph capture) makes no such call.
  if (dev < kMaxDevices) {
    double* scratch_dev = nullptr;
    e = scratch_address(dev, &scratch_dev);
    if (e != hipSuccess) return hip_fail(e, "bind: scratch address");
  }
  c->grid = plan_blocks(c->sp, c->cfg.storage, cus);
  c->grid_gen = c->sp.single ? plan_blocks(c->sp_gen, c->cfg.storage, cus) : c->grid;
  // Small meshes take the tile kernel (scheme 1, A > 0), when a march would
  // leave each block fewer than kTileMaxMarchRows unit-rows; not when the
  // block count is forced (T2S2_BLOCKS), which selects the march.
  c->sp.tile = 0;
  if (c->sp.scheme == 1 && !c->sp.single && !std::getenv("T2S2_BLOCKS") &&
      static_cast<long long>(c->sp.nunits) * c->ny < static_cast<long long>(kTileMaxMarchRows) * c->grid)
    c->sp.tile = 1;
  if (!c->sp.single) c->sp_gen = c->sp;
  if (c->grid < 1 || c->grid_gen < 1) return fail(T2S2_ERR_HIP, "bind: step kernel cannot be resident");
  c->bound = true;
  c->cur = 0;
  c->steps = 0;
  return T2S2_OK;
}

int t2s2_init_macro(t2s2_ctx* c, const double* rho, const double* ux, const double* uy,
                    const double* grad) {
  g_last_error.clear();
  if (!c) return fail(T2S2_ERR_INVALID_ARG, "NULL context");
  if (!c->bound) return fail(T2S2_ERR_NOT_BOUND, "context not bound");
  if (!rho || !ux || !uy) return fail(T2S2_ERR_INVALID_ARG, "NULL field");
  if (grad && std::isinf(c->cfg.nu))
    return fail(T2S2_ERR_INVALID_ARG, "eq 3.5 correction needs a finite tau");
  hipError_t e = launch_init_macro(c->cfg.storage, c->ap, c->state[c->cur], rho, ux, uy, grad,
                                   c->stream);
  if (e != hipSuccess) return hip_fail(e, "init_macro");
  c->steps = 0;
  return T2S2_OK;
}

int t2s2_init_distributions(t2s2_ctx* c, const double* g) {
  g_last_error.clear();
  if (!c) return fail(T2S2_ERR_INVALID_ARG, "NULL context");
  if (!c->bound) return fail(T2S2_ERR_NOT_BOUND, "context not bound");
  if (!g) return fail(T2S2_ERR_INVALID_ARG, "NULL distributions");
  hipError_t e = launch_load_dist(c->cfg.storage, c->ap, c->state[c->cur], g, c->stream);
  if (e != hipSuccess) return hip_fail(e, "init_distributions");
  c->steps = 0;
  return T2S2_OK;
}

int t2s2_step(t2s2_ctx* c, int64_t nsteps) {
  g_last_error.clear();
  if (!c) return fail(T2S2_ERR_INVALID_ARG, "NULL context");
  if (!c->bound) return fail(T2S2_ERR_NOT_BOUND, "context not bound");
  if (nsteps < 0) return fail(T2S2_ERR_INVALID_ARG, "nsteps < 0");
  for (int64_t k = 0; k < nsteps; ++k) {
    c->sp.src = c->state[c->cur];
    c->sp.dst = c->state[1 - c->cur];
    hipError_t e = launch_step(c->cfg.storage, c->sp, c->grid, c->stream);
    if (e != hipSuccess) return hip_fail(e, "step");
    c->cur = 1 - c->cur;
    ++c->steps;
  }
  return T2S2_OK;
}

int t2s2_graph_capture(t2s2_ctx* c, int steps_per_graph) {
  g_last_error.clear();
  if (!c) return fail(T2S2_ERR_INVALID_ARG, "NULL context");
  if (!c->bound) return fail(T2S2_ERR_NOT_BOUND, "context not bound");
  if (steps_per_graph < 2 || (steps_per_graph & 1))
    return fail(T2S2_ERR_INVALID_ARG, "steps_per_graph must be even and >= 2");
  if (c->stream == nullptr)
    return fail(T2S2_ERR_UNSUPPORTED, "graph capture needs a non-default stream");
  drop_graph(c);
  hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return hip_fail(e, "graph capture: begin");
  // Record the launches of steps_per_graph steps; nothing executes, so the
  // host-side buffer index is advanced on a copy only.
  int cur = c->cur;
  hipError_t le = hipSuccess;
  for (int k = 0; k < steps_per_graph && le == hipSuccess; ++k) {
    StepParams sp = c->sp;
    sp.src = c->state[cur];
    sp.dst = c->state[1 - cur];
    le = launch_step(c->cfg.storage, sp, c->grid, c->stream);
    cur = 1 - cur;
  }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(c->stream, &g);
  if (le != hipSuccess || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(le != hipSuccess ? le : e, "graph capture: launches");
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(e, "graph capture: instantiate");
  c->graph = exec;
  c->graph_steps = steps_per_graph;
  c->graph_cur = c->cur;
  return T2S2_OK;
}

int t2s2_graph_step(t2s2_ctx* c, int64_t nsteps) {
  g_last_error.clear();
  if (!c) return fail(T2S2_ERR_INVALID_ARG, "NULL context");
  if (!c->bound) return fail(T2S2_ERR_NOT_BOUND, "context not bound");
  if (!c->graph) return fail(T2S2_ERR_NOT_BOUND, "no graph captured");
  if (nsteps < 0) return fail(T2S2_ERR_INVALID_ARG, "nsteps < 0");
  int64_t left = nsteps;
  int rc = T2S2_OK;
  // The graph reads the buffer that held the state at capture; an odd
  // number of plain steps since then is evened out with one plain step.
  if (left > 0 && c->cur != c->graph_cur) {
    if ((rc = t2s2_step(c, 1)) != T2S2_OK) return rc;
    --left;
  }
  while (left >= c->graph_steps) {
    hipError_t e = hipGraphLaunch(c->graph, c->stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    c->steps += c->graph_steps;  // an even count leaves c->cur unchanged
    left -= c->graph_steps;
  }
  return left > 0 ? t2s2_step(c, left) : T2S2_OK;
}

int t2s2_current(const t2s2_ctx* c) { return c ? c->cur : -1; }

int64_t t2s2_steps_taken(const t2s2_ctx* c) { return c ? c->steps : -1; }

double t2s2_dt(const t2s2_ctx* c) { return c ? c->dt : 0.0; }

int t2s2_moments(t2s2_ctx* c, double* drho, double* ux, double* uy) {
  g_last_error.clear();
  if (!c) return fail(T2S2_ERR_INVALID_ARG, "NULL context");
  if (!c->bound) return fail(T2S2_ERR_NOT_BOUND, "context not bound");
  hipError_t e =
      launch_moments(c->cfg.storage, c->ap, c->state[c->cur], drho, ux, uy, c->stream);
  if (e != hipSuccess) return hip_fail(e, "moments");
  return T2S2_OK;
}

int t2s2_read_distributions(t2s2_ctx* c, double* g) {
  g_last_error.clear();
  if (!c) return fail(T2S2_ERR_INVALID_ARG, "NULL context");
  if (!c->bound) return fail(T2S2_ERR_NOT_BOUND, "context not bound");
  if (!g) return fail(T2S2_ERR_INVALID_ARG, "NULL output");
  hipError_t e = launch_read_dist(c->cfg.storage, c->ap, c->state[c->cur], g, c->stream);
  if (e != hipSuccess) return hip_fail(e, "read_distributions");
  return T2S2_OK;
}

int t2s2_diagnostics(t2s2_ctx* c, double out[T2S2_NDIAG]) {
  g_last_error.clear();
  if (!c) return fail(T2S2_ERR_INVALID_ARG, "NULL context");
  if (!c->bound) return fail(T2S2_ERR_NOT_BOUND, "context not bound");
  if (!out) return fail(T2S2_ERR_INVALID_ARG, "NULL output");
  double* part = reinterpret_cast<double*>(c->ws + c->off_part);
  double* res = reinterpret_cast<double*>(c->ws + c->off_res);
  hipError_t e = launch_diagnostics(c->cfg.storage, c->ap, c->state[c->cur], part, res,
                                    kDiagSlots, c->stream);
  if (e != hipSuccess) return hip_fail(e, "diagnostics");
  double host[kDiagSlots];
  e = hipMemcpyAsync(host, res, sizeof(host), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return hip_fail(e, "diagnostics: copy");
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "diagnostics: synchronize");
  for (int k = 0; k < T2S2_NDIAG; ++k) out[k] = host[k];
  if (host[3] > 0.0) return fail(T2S2_ERR_NONFINITE, "non-finite populations in the state");
  return T2S2_OK;
}

int t2s2_diagnostics_noalloc(t2s2_ctx* c, double* out) {
  g_last_error.clear();
  if (!c) return fail(T2S2_ERR_INVALID_ARG, "NULL context");
  if (!c->bound) return fail(T2S2_ERR_NOT_BOUND, "context not bound");
  if (!out || (reinterpret_cast<uintptr_t>(out) & 7))
    return fail(T2S2_ERR_INVALID_ARG, "out must be an 8-byte aligned device pointer");
  // The partials take kDiagBlocks * kDiagSlots doubles for any mesh (a
  // fixed grid of partial blocks), which the array holds.
  static_assert(kDiagBlocks * kDiagSlots <= kNoAllocDoubles, "scratch too small");
  if (c->device < 0 || c->device >= kMaxDevices)
    return fail(T2S2_ERR_UNSUPPORTED, "device index beyond the scratch table");
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "diagnostics_noalloc: device query");
  if (cur != c->device && (e = hipSetDevice(c->device)) != hipSuccess)
    return hip_fail(e, "diagnostics_noalloc: set device");
  double* part = nullptr;
  e = scratch_address(c->device, &part);
  if (e == hipSuccess)
    e = launch_diagnostics(c->cfg.storage, c->ap, c->state[c->cur], part, out, T2S2_NDIAG,
                           c->stream);
  if (cur != c->device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return hip_fail(e, "diagnostics_noalloc");
  return T2S2_OK;
}

int t2s2_velocity_error(t2s2_ctx* c, const double* ux_ref, const double* uy_ref,
                        double out[T2S2_NGRE]) {
  g_last_error.clear();
  if (!c) return fail(T2S2_ERR_INVALID_ARG, "NULL context");
  if (!c->bound) return fail(T2S2_ERR_NOT_BOUND, "context not bound");
  if (!ux_ref || !uy_ref || !out) return fail(T2S2_ERR_INVALID_ARG, "NULL reference or output");
  double* part = reinterpret_cast<double*>(c->ws + c->off_part);
  double* res = reinterpret_cast<double*>(c->ws + c->off_res);
  hipError_t e = launch_velocity_error(c->cfg.storage, c->ap, c->state[c->cur], ux_ref, uy_ref,
                                       part, res, c->stream);
  if (e != hipSuccess) return hip_fail(e, "velocity_error");
  double host[kDiagSlots];
  e = hipMemcpyAsync(host, res, sizeof(host), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return hip_fail(e, "velocity_error: copy");
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "velocity_error: synchronize");
  out[0] = host[0];
  out[1] = host[1];
  out[2] = host[3];
  // E(u) of eq 3.6 (normalised by the reference) and the residual form of
  // Sec. 3C (normalised by the current field).
  out[3] = host[1] > 0.0 ? std::sqrt(host[0] / host[1]) : NAN;
  out[4] = host[3] > 0.0 ? std::sqrt(host[0] / host[3]) : NAN;
  return T2S2_OK;
}

int t2s2_stencil_weights(const t2s2_ctx* c, double* wx, double* wy) {
  g_last_error.clear();
  if (!c) return fail(T2S2_ERR_INVALID_ARG, "NULL context");
  if (wx) std::copy(c->wx.begin(), c->wx.end(), wx);
  if (wy) std::copy(c->wy.begin(), c->wy.end(), wy);
  return T2S2_OK;
}

double t2s2_omega(const t2s2_ctx* c) { return c ? c->omega : 0.0; }

size_t t2s2_adjoint_state_bytes(const t2s2_ctx* c) {
  if (!c) return 0;
  return static_cast<size_t>(kQ) * c->sp.plane * adjoint_real_bytes(c->cfg.storage);
}

size_t t2s2_adjoint_scratch_bytes(const t2s2_ctx* c) {
  if (!c) return 0;
  return 2 * align256(t2s2_adjoint_state_bytes(c)) + align256(t2s2_state_bytes(c)) +
         align256(kAdjMaxBlocks * sizeof(double));
}

int t2s2_bind_adjoint(t2s2_ctx* c, void* scratch) {
  g_last_error.clear();
  if (!c) return fail(T2S2_ERR_INVALID_ARG, "NULL context");
  if (!c->bound) return fail(T2S2_ERR_NOT_BOUND, "context not bound");
  if (c->sp.has_force) return fail(T2S2_ERR_UNSUPPORTED, "the adjoint covers unforced flows");
  if (c->sp.scheme != 1) return fail(T2S2_ERR_UNSUPPORTED, "the adjoint covers T2S2-FDLBM1 / T1S2");
  if (c->cfg.storage == T2S2_BF16_SR_DEV || c->cfg.storage == T2S2_F16_SR_DEV)
    return fail(T2S2_ERR_UNSUPPORTED, "the adjoint covers the storage forms rounded to nearest");
  if (!scratch || (reinterpret_cast<uintptr_t>(scratch) & 255))
    return fail(T2S2_ERR_INVALID_ARG, "scratch must be a 256-byte aligned device pointer");
  // The adjoint kernels address a plane of its arithmetic-type buffers
  // (twice the storage's bytes for the 16-bit forms) with 32-bit byte offsets.
  if (static_cast<long long>(c->sp.plane) * static_cast<long long>(adjoint_real_bytes(c->cfg.storage)) >=
      (1LL << 32))
    return fail(T2S2_ERR_UNSUPPORTED, "one plane of the adjoint's buffers must be under 4 GiB");
  AdjParams& a = c->adj;
  a.nx = c->nx;
  a.ny = c->ny;
  a.pitch = c->pitch;
  a.plane = c->sp.plane;
  a.per_x = c->sp.per_x;
  a.per_y = c->sp.per_y;
  a.wx = c->sp.wx;
  a.wy = c->sp.wy;
  a.wx32 = c->sp.wx32;
  a.wy32 = c->sp.wy32;
  const double A = c->cfg.A, w = c->omega;
  a.A = A;
  a.cPg = c->sp.cPg;
  a.cPe = c->sp.cPe;
  a.cQg = c->sp.cQg;
  a.cQe = c->sp.cQe;
  a.cRs = c->sp.cRs;
  a.cRe = c->sp.cRe;
  // d/d omega of (2 - A w)/(2 + w), (2 - w)/(2 + w) and 2/(2 + A w); the
  // equilibrium coefficients are one minus these.
  a.dcPg = -2.0 * (1.0 + A) / ((2.0 + w) * (2.0 + w));
  a.dcQg = -4.0 / ((2.0 + w) * (2.0 + w));
  a.dcRs = -2.0 * A / ((2.0 + A * w) * (2.0 + A * w));
  // omega = dt / tau = dt c_s^2 / nu at a fixed dt: d omega / d nu = -omega / nu.
  a.dnu_per_domega = std::isinf(c->cfg.nu) ? 0.0 : -w / c->cfg.nu;
  for (int k = 0; k < 4; ++k) {
    a.uw[k][0] = c->sp.uw[k][0];
    a.uw[k][1] = c->sp.uw[k][1];
  }
  char* p = static_cast<char*>(scratch);
  const size_t ab = align256(t2s2_adjoint_state_bytes(c));
  a.S = p;
  a.mu = p + ab;
  a.next = p + 2 * ab;
  c->adj_partial = reinterpret_cast<double*>(p + 2 * ab + align256(t2s2_state_bytes(c)));
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = plan_adjoint_march(c->cfg.storage, a, cus);
  if (e != hipSuccess) return hip_fail(e, "bind_adjoint: march plan");
  c->adj_bound = true;
  return T2S2_OK;
}

static int adj_ready(t2s2_ctx* c) {
  if (!c) return fail(T2S2_ERR_INVALID_ARG, "NULL context");
  if (!c->bound || !c->adj_bound) return fail(T2S2_ERR_NOT_BOUND, "adjoint scratch not bound");
  return T2S2_OK;
}

int t2s2_adjoint_seed_velocity(t2s2_ctx* c, const void* state, const double* gu,
                               const double* gv, void* lam) {
  g_last_error.clear();
  if (int rc = adj_ready(c)) return rc;
  if (!state || !lam) return fail(T2S2_ERR_INVALID_ARG, "NULL state or adjoint");
  hipError_t e = launch_adjoint_seed(c->cfg.storage, c->adj, state, gu, gv, lam, c->stream);
  if (e != hipSuccess) return hip_fail(e, "adjoint_seed_velocity");
  return T2S2_OK;
}

int t2s2_adjoint_step(t2s2_ctx* c, const void* state_n, const void* lam_np1, void* lam_n,
                      double* dnu_accum) {
  g_last_error.clear();
  if (int rc = adj_ready(c)) return rc;
  if (!state_n || !lam_np1 || !lam_n || lam_np1 == lam_n)
    return fail(T2S2_ERR_INVALID_ARG, "need a state and two distinct adjoint buffers");
  hipError_t e = launch_adjoint_step(c->cfg.storage, c->adj, c->sp_gen, c->grid_gen, state_n, lam_np1,
                                     lam_n, c->adj_partial, dnu_accum, c->stream);
  if (e != hipSuccess) return hip_fail(e, "adjoint_step");
  return T2S2_OK;
}

int t2s2_step_save_s(t2s2_ctx* c, const void* src, void* dst, void* s_out) {
  g_last_error.clear();
  if (int rc = adj_ready(c)) return rc;
  if (!src || !dst || !s_out || src == dst || dst == s_out || src == s_out)
    return fail(T2S2_ERR_INVALID_ARG, "need three distinct buffers");
  StepParams fwd = c->sp_gen;
  fwd.src = src;
  fwd.dst = dst;
  fwd.save_s = s_out;
  hipError_t e = launch_step_save_s(c->cfg.storage, fwd, c->grid_gen, c->stream);
  if (e != hipSuccess) return hip_fail(e, "step_save_s");
  return T2S2_OK;
}

int t2s2_adjoint_step_stored(t2s2_ctx* c, const void* state_n, const void* state_np1,
                             const void* s_n, const void* lam_np1, void* lam_n,
                             double* dnu_accum) {
  g_last_error.clear();
  if (int rc = adj_ready(c)) return rc;
  if (!state_n || !state_np1 || !s_n || !lam_np1 || !lam_n || lam_np1 == lam_n)
    return fail(T2S2_ERR_INVALID_ARG, "need the stored step and two distinct adjoint buffers");
  hipError_t e = launch_adjoint_step_stored(c->cfg.storage, c->adj, state_n, state_np1, s_n,
                                            lam_np1, lam_n, c->adj_partial, dnu_accum,
                                            c->stream);
  if (e != hipSuccess) return hip_fail(e, "adjoint_step_stored");
  return T2S2_OK;
}

int t2s2_adjoint_init_macro(t2s2_ctx* c, const void* lam0, const double* rho, const double* ux,
                            const double* uy, double* grho, double* gux, double* guy) {
  g_last_error.clear();
  if (int rc = adj_ready(c)) return rc;
  if (!lam0 || !rho || !ux || !uy) return fail(T2S2_ERR_INVALID_ARG, "NULL input");
  hipError_t e = launch_adjoint_init(c->cfg.storage, c->adj, lam0, rho, ux, uy, grho, gux, guy,
                                     c->stream);
  if (e != hipSuccess) return hip_fail(e, "adjoint_init_macro");
  return T2S2_OK;
}

int t2s2_adjoint_read(t2s2_ctx* c, const void* lam, double* out) {
  g_last_error.clear();
  if (int rc = adj_ready(c)) return rc;
  if (!lam || !out) return fail(T2S2_ERR_INVALID_ARG, "NULL buffer");
  hipError_t e = launch_adjoint_convert(c->cfg.storage, c->adj, lam, out, nullptr, nullptr,
                                        c->stream);
  if (e != hipSuccess) return hip_fail(e, "adjoint_read");
  return T2S2_OK;
}

int t2s2_adjoint_load(t2s2_ctx* c, const double* in, void* lam) {
  g_last_error.clear();
  if (int rc = adj_ready(c)) return rc;
  if (!lam || !in) return fail(T2S2_ERR_INVALID_ARG, "NULL buffer");
  hipError_t e = launch_adjoint_convert(c->cfg.storage, c->adj, nullptr, nullptr, in, lam,
                                        c->stream);
  if (e != hipSuccess) return hip_fail(e, "adjoint_load");
  return T2S2_OK;
}

int t2s2_copy_probe(const void* src, void* dst, int64_t plane_elems, int elem_bytes,
                    void* stream) {
  g_last_error.clear();
  if (!src || !dst) return fail(T2S2_ERR_INVALID_ARG, "NULL buffer");
  if (plane_elems <= 0) return fail(T2S2_ERR_INVALID_ARG, "plane_elems must be > 0");
  if (elem_bytes != 8 && elem_bytes != 4 && elem_bytes != 2)
    return fail(T2S2_ERR_INVALID_ARG, "elem_bytes must be 8, 4 or 2");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) %
      static_cast<uintptr_t>(elem_bytes))
    return fail(T2S2_ERR_INVALID_ARG, "buffers must be aligned to elem_bytes");
  const uintptr_t bytes = static_cast<uintptr_t>(kQ) * static_cast<uintptr_t>(plane_elems) *
                          static_cast<uintptr_t>(elem_bytes);
  const uintptr_t a = reinterpret_cast<uintptr_t>(src), b = reinterpret_cast<uintptr_t>(dst);
  if (a < b + bytes && b < a + bytes) return fail(T2S2_ERR_INVALID_ARG, "buffers overlap");
  hipError_t e = launch_copy_probe(src, dst, static_cast<long long>(plane_elems), elem_bytes,
                                   static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "copy_probe");
  return T2S2_OK;
}

int t2s2_stability_map(const t2s2_stability_params* prm, const double* omega, const double* r,
                       int npoints, double* radius, void* stream) {
  g_last_error.clear();
  if (!prm) return fail(T2S2_ERR_INVALID_ARG, "NULL parameters");
  if (prm->model < T2S2_STAB_PAPER || prm->model > T2S2_STAB_FAMILY)
    return fail(T2S2_ERR_INVALID_ARG, "unknown stability model");
  if (!(prm->eta >= 0.0 && prm->eta <= 1.0)) return fail(T2S2_ERR_INVALID_ARG, "eta not in [0,1]");
  if (!(prm->A >= 0.0 && prm->A <= 1.0)) return fail(T2S2_ERR_INVALID_ARG, "A not in [0,1]");
  if (!std::isfinite(prm->b2bar) || !std::isfinite(prm->b2tilde) || !std::isfinite(prm->u[0]) ||
      !std::isfinite(prm->u[1]))
    return fail(T2S2_ERR_INVALID_ARG, "non-finite parameter");
  if (prm->model == T2S2_STAB_FAMILY && !(std::isfinite(prm->btilde[0]) &&
                                          std::isfinite(prm->btilde[1]) &&
                                          std::isfinite(prm->btilde[2])))
    return fail(T2S2_ERR_INVALID_ARG, "non-finite btilde");
  if (prm->model == T2S2_STAB_FAMILY && !(std::isfinite(prm->bbar[0]) &&
                                          std::isfinite(prm->bbar[1]) &&
                                          std::isfinite(prm->bbar[2])))
    return fail(T2S2_ERR_INVALID_ARG, "non-finite bbar");
  if (prm->nk < 2 || prm->nk > 257) return fail(T2S2_ERR_INVALID_ARG, "nk not in [2, 257]");
  if (prm->squarings < 1 || prm->squarings > 60)
    return fail(T2S2_ERR_INVALID_ARG, "squarings not in [1, 60]");
  if (npoints < 0) return fail(T2S2_ERR_INVALID_ARG, "npoints < 0");
  if (npoints == 0) return T2S2_OK;
  if (!omega || !r || !radius) return fail(T2S2_ERR_INVALID_ARG, "NULL array");
  StabArgs a{};
  a.model = prm->model;
  a.eta = prm->eta;
  a.A = prm->A;
  a.b2bar = prm->b2bar;
  a.b2tilde = prm->b2tilde;
  a.ux = prm->u[0];
  a.uy = prm->u[1];
  const double pi = 3.14159265358979323846;
  a.nky = prm->nk;
  a.dthy = pi / (prm->nk - 1);
  a.dthx = a.dthy;
  a.nkx = prm->full_kx ? 2 * prm->nk - 1 : prm->nk;
  a.thx0 = prm->full_kx ? -pi : 0.0;
  a.squarings = prm->squarings;
  for (int k = 0; k < 3; ++k) a.bt[k] = prm->model == T2S2_STAB_FAMILY ? prm->btilde[k] : 0.0;
  {
    const double* bb = prm->bbar;
    const bool zero = bb[0] == 0.0 && bb[1] == 0.0 && bb[2] == 0.0;
    a.bb[0] = zero ? 0.5 : bb[0];
    a.bb[1] = zero ? 0.0 : bb[1];
    a.bb[2] = zero ? 0.5 : bb[2];
    a.gen_bb = prm->model == T2S2_STAB_FAMILY &&
               !(a.bb[0] == 0.5 && a.bb[1] == 0.0 && a.bb[2] == 0.5);
  }
  hipError_t e = launch_stability(a, omega, r, npoints, radius, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "stability map");
  return T2S2_OK;
}

void t2s2_destroy(t2s2_ctx* c) { delete c; }

}  // extern "C"
