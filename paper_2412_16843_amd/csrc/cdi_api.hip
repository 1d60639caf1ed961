// Host side of the C ABI: parameter validation, multigrid hierarchy and
// workspace layout, tile lists spanning every instance of a batch, and the
// stream-ordered launch sequence of one RK4 step (4 stage evaluations, 4
// variable-density projections by multigrid-preconditioned flexible CG).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "../../include/cdi.h"
#include "host_util.h"
#include "persistent_kernels.h"
#include "net_internal.h"

using namespace cdi;

namespace {
thread_local std::string g_err;
}  // namespace

cdi_status cdi_host::fail(cdi_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

namespace {

using cdi_host::fail;

constexpr double RK_C[4] = {0.0, 0.5, 0.5, 1.0};
constexpr double RK_B[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};

struct Resolved {
  cdi_params p;
  double h, dt, rtol;
  int maxit, nlev, lc;
  int lg;                   // first level done by the one-block coarse kernel (<= lc)
  int lnx[kMaxLevels], lny[kMaxLevels];
};

double cfl_dt(const cdi_params& p, double h) {
  const double cfl = p.cfl > 0 ? p.cfl : 0.2;
  double m = INFINITY;
  const double uw = std::max(std::fabs(p.u_wall_bot), std::fabs(p.u_wall_top));
  if (uw > 0) m = std::min(m, h / uw);
  const double nu = std::max(p.mu1 / p.rho1, p.mu2 / p.rho2);
  if (nu > 0) m = std::min(m, h * h / nu);
  if (p.sigma > 0) m = std::min(m, std::sqrt((p.rho1 + p.rho2) * h * h * h / (4.0 * M_PI * p.sigma)));
  if (p.gamma * p.eps > 0) m = std::min(m, h * h / (p.gamma * p.eps));
  return cfl * m;
}

cdi_status resolve(const cdi_params* in, Resolved& r) {
  if (!in) return fail(CDI_ERR_ARG, "params is NULL");
  const cdi_params& p = *in;
  if (p.abi_version != CDI_ABI_VERSION)
    return fail(CDI_ERR_ARG, "abi_version %d != %d", p.abi_version, CDI_ABI_VERSION);
  if (p.nx < 8 || p.ny < 8 || (p.nx & 1) || (p.ny & 1))
    return fail(CDI_ERR_SHAPE, "nx=%d ny=%d: both must be even and >= 8", p.nx, p.ny);
  if ((long long)p.nx * (p.ny + 1) >= (1LL << 31))
    return fail(CDI_ERR_SHAPE, "nx=%d ny=%d: more than 2^31 - 1 cells", p.nx, p.ny);
  if (!(p.lx > 0) || !(p.ly > 0)) return fail(CDI_ERR_ARG, "lx, ly must be > 0");
  const double hx = p.lx / p.nx, hy = p.ly / p.ny;
  if (std::fabs(hx - hy) > 1e-12 * hx) return fail(CDI_ERR_SHAPE, "lx/nx=%g != ly/ny=%g", hx, hy);
  if (!(p.eps > 0)) return fail(CDI_ERR_ARG, "eps must be > 0");
  if (!(p.gamma > 0)) return fail(CDI_ERR_ARG, "gamma must be > 0");
  if (!(p.gamma_factor >= 0)) return fail(CDI_ERR_ARG, "gamma_factor must be >= 0");
  if (!(p.sigma >= 0)) return fail(CDI_ERR_ARG, "sigma must be >= 0");
  if (!(p.theta_eq > 0 && p.theta_eq < M_PI)) return fail(CDI_ERR_ARG, "theta_eq must be in (0, pi)");
  if (!(p.rho1 > 0 && p.rho2 > 0)) return fail(CDI_ERR_ARG, "densities must be > 0");
  if (!(p.mu1 >= 0 && p.mu2 >= 0)) return fail(CDI_ERR_ARG, "viscosities must be >= 0");
  if (!(p.beta1 > 0 && p.beta2 > 0)) return fail(CDI_ERR_ARG, "beta1, beta2 must be > 0");
  if (!std::isfinite(p.u_wall_bot) || !std::isfinite(p.u_wall_top))
    return fail(CDI_ERR_ARG, "wall speeds must be finite");
  if (p.dt < 0 || !std::isfinite(p.dt)) return fail(CDI_ERR_ARG, "dt must be >= 0");
  if (p.cfl < 0) return fail(CDI_ERR_ARG, "cfl must be >= 0");
  if (p.slip_model < CDI_SLIP_1A || p.slip_model > CDI_SLIP_4B) return fail(CDI_ERR_ARG, "bad slip_model");
  if (p.precision != CDI_FP64 && p.precision != CDI_MIXED) return fail(CDI_ERR_ARG, "bad precision");
  if (p.guess < CDI_GUESS_ZERO || p.guess > CDI_GUESS_LEARNED) return fail(CDI_ERR_ARG, "bad guess");
  if (p.poisson_rtol < 0 || p.poisson_maxit < 0 || p.mg_smooth < 0) return fail(CDI_ERR_ARG, "bad solver limits");
  if (p.mg_smooth > 2) return fail(CDI_ERR_ARG, "mg_smooth: 1 or 2 sweep pairs are supported");
  r.p = p;
  r.h = hx;
  r.dt = p.dt > 0 ? p.dt : cfl_dt(p, hx);
  if (!(r.dt > 0) || !std::isfinite(r.dt)) return fail(CDI_ERR_ARG, "time step could not be determined");
  r.rtol = p.poisson_rtol > 0 ? p.poisson_rtol : 1e-10;
  r.maxit = p.poisson_maxit > 0 ? p.poisson_maxit : 200;
  // multigrid hierarchy: halve both directions while both stay even and the
  // level has more than 64 cells
  int nx = p.nx, ny = p.ny, l = 0;
  r.lnx[0] = nx; r.lny[0] = ny;
  while ((nx % 2 == 0) && (ny % 2 == 0) && nx * ny > 64 && l + 1 < kMaxLevels) {
    nx /= 2; ny /= 2; ++l;
    r.lnx[l] = nx; r.lny[l] = ny;
  }
  r.nlev = l + 1;
  if ((long)r.lnx[r.nlev - 1] * r.lny[r.nlev - 1] > kCoarseCells)
    return fail(CDI_ERR_SHAPE, "coarsest multigrid grid %dx%d exceeds %d cells", r.lnx[r.nlev - 1],
                r.lny[r.nlev - 1], kCoarseCells);
  r.lc = r.nlev - 1;
  for (int k = 0; k < r.nlev; ++k)
    if ((long)r.lnx[k] * r.lny[k] <= kCoarseCells) { r.lc = k; break; }
  r.lg = r.lc;
  long cells = 0, yfaces = 0;   // LDS footprint of the single-block coarse cycle
  for (int k = r.lc; k < r.nlev; ++k) {
    cells += (long)r.lnx[k] * r.lny[k];
    yfaces += (long)(r.lny[k] + 1) * r.lnx[k];
  }
  if (cells > kCLX || yfaces > kCLY)
    return fail(CDI_ERR_SHAPE, "coarse multigrid levels too large for one block");
  if (r.nlev - r.lc > kMaxCoarseLevels)
    return fail(CDI_ERR_SHAPE, "more than %d coarse multigrid levels", kMaxCoarseLevels);
  return CDI_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int ceil_div(int a, int b) { return (a + b - 1) / b; }

struct Layout {
  size_t inst_bytes;        // per instance (sum over instances in `offs`)
};

// Doubles of one instance's step state: phi, u, p and the 8 pressure-history
// fields (ny * nx each) and v ((ny + 1) * nx).
size_t snap_doubles(int nx, int ny) { return (4 + 4 * kHistDepth) * (size_t)nx * ny + (size_t)nx; }

// Carve one instance's arrays out of `base` (device) starting at offset `off`;
// with base == nullptr only the size is computed.
size_t carve(const Resolved& R, int ntiles_cell, int ntiles_mg0, char* base, size_t off, Inst* I) {
  const int nx = R.p.nx, ny = R.p.ny;
  const size_t nc = (size_t)nx * ny, nf = (size_t)(ny + 1) * nx;
  const bool mixed = R.p.precision == CDI_MIXED;
  const size_t S = mixed ? sizeof(float) : sizeof(double);
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? (void*)(base + off) : nullptr;
    off = align256(off + bytes);
    return p;
  };
  Inst tmp;
  Inst& D = I ? *I : tmp;
  D.phi_a = (double*)take(nc * 8);
  D.phi_b = (double*)take(nc * 8);
  D.us = (double*)take(nc * 8);
  D.vs = (double*)take(nf * 8);
  D.mx = (double*)take(nc * 8);
  D.my = (double*)take(nf * 8);
  D.ustar = (double*)take(nc * 8);
  D.vstar = (double*)take(nf * 8);
  D.acc_phi = (double*)take(nc * 8);
  D.acc_mx = (double*)take(nc * 8);
  D.acc_my = (double*)take(nf * 8);
  D.nhx = take(nc * S);
  D.nhy = take(nc * S);
  D.muc = take(nc * S);
  D.wall = (double*)take((size_t)10 * nx * 8);
  D.uY = (double*)take((size_t)2 * nx * 8);
  D.uslip = (double*)take((size_t)2 * nx * 8);
  D.ax0 = (double*)take(nc * 8);
  D.ay0 = (double*)take(nf * 8);
  D.b = (double*)take(nc * 8);
  D.x = (double*)take(nc * 8);
  D.rr = (double*)take(nc * 8);
  D.rr2 = (double*)take(nc * 8);
  D.d0 = (double*)take(nc * 8);
  D.d1 = (double*)take(nc * 8);
  D.q = (double*)take(nc * 8);
  D.zf = (double*)take(nc * 8);
  D.snap = (double*)take(snap_doubles(nx, ny) * 8);
  D.mg_t = take(nc * S);
  D.mg_r0 = take(nc * S);
  for (int d = 0; d < kHistDepth; ++d)
    for (int k = 0; k < 4; ++k) D.hp[d][k] = (double*)take(nc * 8);
  D.part = (double*)take((size_t)8 * std::max(ntiles_cell, ntiles_mg0) * 8);
  D.pcg = (PcgScalars*)take(sizeof(PcgScalars));
  D.counters = (unsigned*)take(sizeof(unsigned) * 8 * kCounterStride);
  for (int l = 0; l < R.nlev; ++l) {
    Level& L = D.lev[l];
    L.nx = R.lnx[l];
    L.ny = R.lny[l];
    const size_t lc = (size_t)L.nx * L.ny, lf = (size_t)(L.ny + 1) * L.nx;
    if (l == 0 && !mixed) {
      L.ax = D.ax0.p;
      L.ay = D.ay0.p;
    } else {
      L.ax = take(lc * S);
      L.ay = take(lf * S);
    }
    L.r = (l == 0) ? nullptr : take(lc * S);
    L.z = take(lc * S);
    L.zo = (l == 0) ? nullptr : take(lc * S);
  }
  const size_t ncs = (size_t)R.lnx[R.nlev - 1] * R.lny[R.nlev - 1];
  // constant operator coefficients (uniform density): computed once; the dense
  // coarsest inverse is then worth its set-up.  With a variable density the
  // coarsest grid is solved by the coarsest CG instead of re-inverting it
  // at every projection.
  D.coef_const = R.p.rho1 == R.p.rho2 ? 1 : 0;
  D.cdense = (ncs <= (size_t)kDenseMax && D.coef_const) ? 1 : 0;
  D.cinv = D.cdense ? (double*)take(ncs * ncs * 8) : nullptr;
  return off;
}

struct Batch {
  int n;
  std::vector<Resolved> R;
  std::vector<Inst> inst;               // host copies
  // tile lists (host), concatenated into one device array
  std::vector<Tile> cell;               // level-0 cell tiles of every instance
  std::vector<Tile> wide;               // level-0 wide tiles of every instance
  std::vector<Tile> strip;              // level-0 strips of the FP64 stage kernel
  int strip_rows = sr::SH;              // rows of a strip
  std::vector<std::vector<Tile>> mg;    // per level: multigrid tiles of instances with level < lc
  int max_lc = 0, max_nlev = 0, max_lg = 0;
  size_t shared_bytes = 0;
};

void build_wide(Batch& B, int rows) {
  B.wide.clear();
  const int wy = rows * TY;
  for (int k = 0; k < B.n; ++k) {
    const Resolved& R = B.R[k];
    Inst& I = B.inst[k];
    I.first_wide = (int)B.wide.size();
    int lw = 0;
    for (int j0 = 0; j0 < R.p.ny; j0 += wy)
      for (int i0 = 0; i0 < R.p.nx; i0 += TX) B.wide.push_back(Tile{k, i0, j0, 0, lw++, 0, nullptr});
    I.nwide = lw;
  }
}

// Multigrid tiles of the tiled kernels: levels below each instance's lg.
void build_mg(Batch& B) {
  B.max_lg = 0;
  for (int k = 0; k < B.n; ++k) B.max_lg = std::max(B.max_lg, B.R[k].lg);
  B.mg.assign(std::max(B.max_lc, 1), {});
  for (int k = 0; k < B.n; ++k) {
    const Resolved& R = B.R[k];
    Inst& I = B.inst[k];
    I.lg = R.lg;
    for (int l = 0; l < R.lg; ++l) {
      Level& L = I.lev[l];
      L.first_tile = (int)B.mg[l].size();
      int loc = 0;
      for (int j0 = 0; j0 < L.ny; j0 += FY)
        for (int i0 = 0; i0 < L.nx; i0 += FX) B.mg[l].push_back(Tile{k, i0, j0, l, loc++, 0, nullptr});
      L.ntiles = loc;
    }
    for (int l = R.lg; l < R.nlev; ++l) { I.lev[l].first_tile = 0; I.lev[l].ntiles = 0; }
  }
}

int strip_tiles(const Resolved& R, int rows) { return ceil_div(R.p.nx, sr::TW) * ceil_div(R.p.ny, rows); }

// Rows of the stage kernel's strips: the tallest of 64, 32, 16 that still
// gives every CU several strips (each strip's first chunk recomputes a few
// halo rows, so taller strips do less work, but fewer of them fill the GPU
// less evenly).
constexpr int kStripRows[3] = {64, 32, 16};
constexpr long kStripBlocksMin = 256L * 3 * 3;   // CUs x resident strips x rounds
int strip_rows(const std::vector<Resolved>& Rs) {
  for (int r : kStripRows) {
    long n = 0;
    for (const Resolved& R : Rs) n += strip_tiles(R, r);
    if (n >= kStripBlocksMin) return r;
  }
  return kStripRows[2];
}

// Strips of the FP64 stage kernel: TW columns x `rows` rows.
void build_strips(Batch& B, int rows) {
  B.strip.clear();
  B.strip_rows = rows;
  for (int k = 0; k < B.n; ++k) {
    const Resolved& R = B.R[k];
    int local = 0;
    for (int j0 = 0; j0 < R.p.ny; j0 += rows)
      for (int i0 = 0; i0 < R.p.nx; i0 += sr::TW) B.strip.push_back(Tile{k, i0, j0, 0, local++, 0, nullptr});
  }
}

void build_tiles(Batch& B, int wide_rows) {
  B.cell.clear();
  B.max_lc = 0;
  B.max_nlev = 0;
  for (int k = 0; k < B.n; ++k) {
    B.max_lc = std::max(B.max_lc, B.R[k].lc);
    B.max_nlev = std::max(B.max_nlev, B.R[k].nlev);
  }
  for (int k = 0; k < B.n; ++k) {
    const Resolved& R = B.R[k];
    Inst& I = B.inst[k];
    I.first_tile = (int)B.cell.size();
    int local = 0;
    for (int j0 = 0; j0 < R.p.ny; j0 += TY)
      for (int i0 = 0; i0 < R.p.nx; i0 += TX) B.cell.push_back(Tile{k, i0, j0, 0, local++, 0, nullptr});
    I.ntiles = local;
  }
  build_strips(B, strip_rows(B.R));
  build_mg(B);
  build_wide(B, wide_rows);
}

// Coarse-kernel start level for a threshold: the first level with at most
// `cells` cells (never below lc: those levels live in the kernel's LDS).
void set_lg(Resolved& R, long cells) {
  R.lg = R.lc;
  for (int k = 0; k < R.lc; ++k)
    if ((long)R.lnx[k] * R.lny[k] <= cells) { R.lg = k; break; }
}

// Workgroups of a launch are dispatched to the XCDs round robin (block b on
// XCD b % kXcds), each XCD with its own L2.  Reorder a tile list so that every
// XCD receives one contiguous band of tiles: neighbouring tiles, whose halos
// overlap, then share an L2 instead of fetching the same rows from HBM twice.
constexpr size_t kXcds = 8;
constexpr long kDefaultCoarseCells = 4096;
constexpr long kTuneCoarse[3] = {1024, 4096, 16384};   // coarse-kernel thresholds tried by cdi_tune

std::vector<Tile> xcd_order(const std::vector<Tile>& t) {
  const size_t n = t.size();
  std::vector<Tile> out(n);
  size_t src = 0;
  for (size_t x = 0; x < kXcds && x < n; ++x) {
    const size_t cnt = (n - x + kXcds - 1) / kXcds;   // blocks x, x + 8, x + 16, ...
    for (size_t k = 0; k < cnt; ++k) out[x + k * kXcds] = t[src + k];
    src += cnt;
  }
  return out;
}

int mg0_tiles(const Resolved& R) { return ceil_div(R.p.nx, FX) * ceil_div(R.p.ny, FY); }
int cell_tiles(const Resolved& R) { return ceil_div(R.p.nx, TX) * ceil_div(R.p.ny, TY); }

size_t batch_bytes(const std::vector<Resolved>& Rs, Batch* B, char* base) {
  const int n = (int)Rs.size();
  // shared header: instances, diag outputs, tile lists
  size_t ntile_cell = 0, ntile_mg = 0, ntile_wide = 0, ntile_strip = 0;
  for (auto& R : Rs) {
    ntile_cell += cell_tiles(R);
    ntile_strip += strip_tiles(R, kStripRows[2]);   // room for the shortest strips
    ntile_wide += (size_t)cell_tiles(R);   // room for the shortest wide tile (1 row)
    int nx = R.p.nx, ny = R.p.ny;
    for (int l = 0; l < R.lc; ++l) { ntile_mg += (size_t)ceil_div(nx, FX) * ceil_div(ny, FY); nx /= 2; ny /= 2; }
  }
  size_t off = 0;
  off = align256(off + sizeof(Inst) * n);
  off = align256(off + sizeof(DiagOut) * n);
  off = align256(off + sizeof(PcgScalars) * n);
  off = align256(off + sizeof(Tile) * (2 * ntile_cell + ntile_wide + ntile_mg + ntile_strip + 1));
  for (int k = 0; k < n; ++k)
    off = carve(Rs[k], cell_tiles(Rs[k]), mg0_tiles(Rs[k]), base, off, B ? &B->inst[k] : nullptr);
  (void)B;
  return off;
}

void fill_inst(const Resolved& R, const cdi_fields& f, Inst& I) {
  const cdi_params& p = R.p;
  I.nx = p.nx; I.ny = p.ny;
  I.nlev = R.nlev; I.lc = R.lc; I.lg = R.lg;
  {
    int a = 0, b = 0;
    for (int m = 0; m <= kMaxCoarseLevels; ++m) {
      I.cpre_x[m] = a;
      I.cpre_y[m] = b;
      const int l = R.lc + m;
      if (m < kMaxCoarseLevels && l < R.nlev) {
        a += R.lnx[l] * R.lny[l];
        b += (R.lny[l] + 1) * R.lnx[l];
      }
    }
  }
  I.nu = p.mg_smooth > 0 ? p.mg_smooth : 1;
  I.nu_c = I.nu + 1;
  I.slip_model = p.slip_model;
  I.mixed = p.precision == CDI_MIXED;
  I.h = R.h; I.inv_h = 1.0 / R.h;
  I.eps = p.eps; I.inv_eps = 1.0 / p.eps; I.gamma = p.gamma; I.sigma = p.sigma; I.cos_eq = std::cos(p.theta_eq);
  I.gamma_factor = p.gamma_factor;
  I.rho1 = p.rho1; I.rho2 = p.rho2; I.mu1 = p.mu1; I.mu2 = p.mu2;
  I.beta1 = p.beta1; I.beta2 = p.beta2;
  I.uw_bot = p.u_wall_bot; I.uw_top = p.u_wall_top;
  I.dt = R.dt;
  I.phi = f.phi; I.u = f.u; I.v = f.v; I.p = f.p;
}

}  // namespace

struct cdi_ctx {
  Batch B;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  Inst* d_inst = nullptr;
  DiagOut* d_diag = nullptr;
  PcgScalars* d_pcg_all = nullptr;   // gather area of the batch's CG scalars
  Tile* d_cell = nullptr;          // level-0 tiles, XCD-banded order (tiled launches)
  Tile* d_cell_inst = nullptr;     // level-0 tiles, instance by instance (persistent launch)
  Tile* d_wide = nullptr;          // level-0 wide tiles, XCD-banded order
  Tile* d_strip = nullptr;         // level-0 strips of the stage kernel, XCD-banded order
  std::vector<Tile*> d_mg;
  bool mixed = false;
  bool uniform_rho = true;
  bool dyn_gamma = false;         // an instance recomputes gamma every step
  bool coef_ready = false;
  double t = 0.0;
  long step = 0;
  std::vector<double> mass0;
  PcgScalars* h_pcg = nullptr;   // pinned
  int pred_iters = 4;
  int pred_stage[4] = {0, 0, 0, 0};   // per RK stage: CG iterations of its last solve
  int wide_rows = 4;             // rows per thread of the wide-tile kernels (1 or 4)
  int nu = 1;                    // red-black sweep pairs of the V-cycle
  int wide_rows_pick = 4;        // autotuner: faster tiled shape so far
  long coarse_cells = 4096;      // coarse kernel takes every level with at most this many cells
  long coarse_cells_pick = 4096;
  int nu_pick = 1;
  std::vector<int> last_iters;
  std::vector<double> last_relres;
  std::vector<int> last_conv;
  int guess = CDI_GUESS_PREV;
  double rtol = 1e-10;
  int maxit = 200;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  cdi_net* net = nullptr;        // learned initial guess (borrowed)
  int hist_steps = 0;            // steps recorded in the per-stage pressure history
  int extrap_order = kHistDepth - 1;   // highest time-extrapolation order of the guess
  int launch = CDI_LAUNCH_TILED; // how cdi_step enqueues a step
  // graph launch: captured step with a fixed CG budget per solve
  hipStream_t gstream = nullptr;   // capture / replay stream (the caller's may be the null stream)
  hipEvent_t gev0 = nullptr, gev1 = nullptr;
  // one captured step per pressure-history ring slot (step mod 4): a step's
  // launches carry the slot it writes
  hipGraph_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
  hipGraphExec_t gexec[4] = {nullptr, nullptr, nullptr, nullptr};
  int graph_budget = 0;            // CG iterations per solve in the captured steps
  int graph_slack = 0;             // consecutive steps that needed at most budget - 2
  long graph_replays = 0, graph_misses = 0;
  // measurement hook: events around every launch of one kernel family
  std::string timed;
  std::vector<hipEvent_t> tev;
  int tev_used = 0;
  hipEvent_t kev0 = nullptr, kev1 = nullptr;   // events of the launch being measured
  double timed_ms = 0.0;
  long timed_launches = 0;
};

// ---------------------------------------------------------------- launches
namespace {

constexpr int kTimedPairs = 512;

// Call f with the rows-per-thread of the wide-tile kernels as a constant.
template <typename F>
void with_rows(int rows, F&& f) {
  if (rows == kWideRows[1]) f(std::integral_constant<int, kWideRows[1]>{});
  else f(std::integral_constant<int, kWideRows[0]>{});
}

hipError_t timing_flush(cdi_ctx* c) {
  if (c->tev_used == 0) return hipSuccess;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return e;
  for (int k = 0; k < c->tev_used; ++k) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, c->tev[2 * k], c->tev[2 * k + 1]);
    if (e != hipSuccess) return e;
    c->timed_ms += ms;
  }
  c->timed_launches += c->tev_used;
  c->tev_used = 0;
  return hipSuccess;
}

// Launch `body` and, when `name` is the kernel family being measured,
// bracket it with events on the context stream.
template <typename F>
void timed(cdi_ctx* c, const char* name, F&& body, bool single = true) {
  if (c->timed.empty() || c->timed != name) { body(); return; }
  if (c->tev_used == kTimedPairs) (void)timing_flush(c);
  hipEvent_t e0 = c->tev[2 * c->tev_used], e1 = c->tev[2 * c->tev_used + 1];
  if (single) {
    // one kernel: its own begin / end timestamps (the launch carries the events)
    c->kev0 = e0;
    c->kev1 = e1;
    body();
    c->kev0 = c->kev1 = nullptr;
  } else {
    (void)hipEventRecord(e0, c->stream);
    body();
    (void)hipEventRecord(e1, c->stream);
  }
  c->tev_used += 1;
}

// Launch on the context stream; while a kernel family is being measured the
// launch records the kernel's start and end in the family's event pair.
#define CDI_LAUNCH(c, kern, grid, block, ...)                                          \
  hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, (c)->stream, (c)->kev0,     \
                        (c)->kev1, 0, __VA_ARGS__)

// The stage operator of every instance (phase preparation fused in): the
// strip kernel in FP64; in mixed precision the 64 x 4 tile kernel, whose
// lower register count keeps more waves resident.
template <typename S>
void launch_stage(cdi_ctx* c, int k, int src, int dst, double c_next, double b_k, int write_wall) {
  const Batch& B = c->B;
  if constexpr (std::is_same<S, double>::value)
    CDI_LAUNCH(c, k_stage_strip<double>, (unsigned)B.strip.size(), kNT, c->d_strip, c->d_inst, k,
               src, dst, c_next, b_k, write_wall, B.strip_rows);
  else
    CDI_LAUNCH(c, k_stage_fused<float>, (unsigned)B.cell.size(), kNT, c->d_cell, c->d_inst, k, src,
               dst, c_next, b_k, write_wall);
}

// V-cycle z = M r over every instance.  update: the first kernel applies the
// CG step (d from buffer dpar) and the stopping test; rsel: residual buffer
// holding the V-cycle's input.
template <typename S>
void launch_vcycle(cdi_ctx* c, int update, int dpar, int rsel) {
  Batch& B = c->B;
  for (int l = 0; l < B.max_lg; ++l)
    if (!B.mg[l].empty())
      timed(c, (l == 0 && update) ? "mg_down" : "mg_down_other", [&] {
        const unsigned nb = (unsigned)B.mg[l].size();
        if (c->nu == 2 && l == 0)
          CDI_LAUNCH(c, (k_mg_down<S, 2, true>), nb, kNT, c->d_mg[l], c->d_inst, l, update, dpar, rsel);
        else if (c->nu == 2)
          CDI_LAUNCH(c, (k_mg_down<S, 2, false>), nb, kNT, c->d_mg[l], c->d_inst, l, update, dpar, rsel);
        else if (l == 0)
          CDI_LAUNCH(c, (k_mg_down<S, 1, true>), nb, kNT, c->d_mg[l], c->d_inst, l, update, dpar, rsel);
        else
          CDI_LAUNCH(c, (k_mg_down<S, 1, false>), nb, kNT, c->d_mg[l], c->d_inst, l, update, dpar, rsel);
      });
  timed(c, "mg_coarse", [&] {
    CDI_LAUNCH(c, k_mg_coarse<S>, (unsigned)B.n, kCoarseNT, c->d_inst, update, dpar, rsel);
  });
  for (int l = B.max_lg - 1; l >= 0; --l)
    if (!B.mg[l].empty())
      timed(c, l == 0 ? "mg_up" : "mg_up_other", [&] {
        const unsigned nb = (unsigned)B.mg[l].size();
        if (c->nu == 2 && l == 0)
          CDI_LAUNCH(c, (k_mg_up<S, 2, true>), nb, kNT, c->d_mg[l], c->d_inst, l, rsel);
        else if (c->nu == 2)
          CDI_LAUNCH(c, (k_mg_up<S, 2, false>), nb, kNT, c->d_mg[l], c->d_inst, l, rsel);
        else if (l == 0)
          CDI_LAUNCH(c, (k_mg_up<S, 1, true>), nb, kNT, c->d_mg[l], c->d_inst, l, rsel);
        else
          CDI_LAUNCH(c, (k_mg_up<S, 1, false>), nb, kNT, c->d_mg[l], c->d_inst, l, rsel);
      });
}

// Coarse-level operator coefficients of every instance from the level-0 ones.
// Instances of uniform density keep constant coefficients: once they have
// been formed (c->coef_ready) only the variable-density instances recompute
// theirs, and the dense coarsest inverse (uniform density only) is formed
// once.
template <typename S>
void launch_coef(cdi_ctx* c) {
  const int only_variable = c->coef_ready ? 1 : 0;
  // the tiled levels 1 .. lg-1 one launch per level, then every level from
  // lg in one launch (one block per instance)
  for (int l = 1; l < c->B.max_lg; ++l) {
    int maxc = 0;
    for (int k = 0; k < c->B.n; ++k)
      if (c->B.R[k].nlev > l && c->B.R[k].lg > l)
        maxc = std::max(maxc, c->B.R[k].lnx[l] * (c->B.R[k].lny[l] + 1));
    const dim3 grid((unsigned)std::max(1, std::min(1024, ceil_div(maxc, kNT))), (unsigned)c->B.n);
    timed(c, "mg_coef", [&] { CDI_LAUNCH(c, k_mg_coef<S>, grid, kNT, c->d_inst, l, only_variable); });
  }
  if (c->B.max_nlev > 1)
    timed(c, "mg_coef", [&] {
      CDI_LAUNCH(c, k_mg_coef_small<S>, (unsigned)c->B.n, kCoarseNT, c->d_inst, only_variable);
    });
  if (!only_variable)
    timed(c, "mg_coef", [&] { CDI_LAUNCH(c, k_coarse_inv<S>, (unsigned)c->B.n, kCoarseNT, c->d_inst); });
}

// Enqueue the copy of every instance's CG scalars into the pinned host array
// (one copy for a single instance, else a gather kernel and one copy).
cdi_status pcg_to_host(cdi_ctx* c) {
  const int n = c->B.n;
  if (n == 1) {
    HIPCHK(hipMemcpyAsync(c->h_pcg, c->B.inst[0].pcg, sizeof(PcgScalars), hipMemcpyDeviceToHost,
                          c->stream));
    return CDI_OK;
  }
  k_gather_pcg<<<(unsigned)ceil_div(n, 64), 64, 0, c->stream>>>(c->d_inst, n, c->d_pcg_all);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->h_pcg, c->d_pcg_all, sizeof(PcgScalars) * n, hipMemcpyDeviceToHost,
                        c->stream));
  return CDI_OK;
}

// True if a solve of the batch met a NaN or Inf (host copies of the CG
// scalars must be current).
bool any_nonfinite(const cdi_ctx* c) {
  for (int k = 0; k < c->B.n; ++k)
    if (c->h_pcg[k].nonfinite) return true;
  return false;
}

// Pressure-history ring slot the current step writes (the step number mod
// the history depth); the guess reads the slots before it.
int hist_slot(const cdi_ctx* c) { return (int)(c->step & (kHistDepth - 1)); }

// Flexible-CG loop after the right-hand side is in place.  Returns NOCONV
// if an instance stopped at maxit.
template <typename S>
cdi_status solve_loop(cdi_ctx* c, int guess, int stage) {
  Batch& B = c->B;
  const unsigned nwide = (unsigned)B.wide.size();
  if (!c->uniform_rho || !c->coef_ready) {
    launch_coef<S>(c);
    c->coef_ready = true;
  }
  timed(c, "pcg_init", [&] {
    with_rows(c->wide_rows, [&](auto R) {
      CDI_LAUNCH(c, k_pcg_init<decltype(R)::value>, nwide, kNT, c->d_wide, c->d_inst, guess, stage,
                 hist_slot(c));
    });
  });
  // z0 = M r0 (residual in buffer 0)
  launch_vcycle<S>(c, 0, 0, 0);
  // the host first checks after the predicted count (the last solve's):
  // with a steady count that is the one wait per solve; an over-estimate
  // costs only early-exit launches
  int it = 0;
  // (each RK stage keeps its own count: the four stages' solves differ,
  // while one stage's count changes slowly from step to step)
  int& pred = c->pred_stage[stage & 3];
  int next_check = std::max(1, pred > 0 ? pred : c->pred_iters);
  bool all_done = false;
  while (it < c->maxit) {
    const int par = it & 1;
    timed(c, "pcg_spmv", [&] {
      with_rows(c->wide_rows, [&](auto R) {
        CDI_LAUNCH(c, k_pcg_spmv<decltype(R)::value>, nwide, kNT, c->d_wide, c->d_inst, par, par);
      });
    });
    launch_vcycle<S>(c, 1, par, par ^ 1);
    ++it;
    if (it >= next_check || it >= c->maxit) {
      cdi_status cs = pcg_to_host(c);
      if (cs != CDI_OK) return cs;
      HIPCHK(hipStreamSynchronize(c->stream));
      all_done = true;
      for (int k = 0; k < B.n; ++k) all_done = all_done && c->h_pcg[k].done;
      if (all_done) break;
      next_check = it + 1;
    }
  }
  if (!all_done) {
    cdi_status cs = pcg_to_host(c);
    if (cs != CDI_OK) return cs;
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  // the solution mean needs its own pass only for a solve that ended before
  // any CG update (the update kernels sum x as they go); the host copies of
  // the CG scalars say whether any instance did
  bool need_xmean = false;
  for (int k = 0; k < B.n; ++k) need_xmean = need_xmean || c->h_pcg[k].iters == 0;
  if (need_xmean)
    timed(c, "pcg_xmean", [&] {
      with_rows(c->wide_rows, [&](auto R) {
        CDI_LAUNCH(c, k_pcg_xmean<decltype(R)::value>, nwide, kNT, c->d_wide, c->d_inst);
      });
    });
  int maxi = 0;
  bool noconv = false;
  for (int k = 0; k < B.n; ++k) {
    c->last_iters[k] = c->h_pcg[k].iters;
    c->last_relres[k] = c->h_pcg[k].relres;
    c->last_conv[k] = c->h_pcg[k].converged;
    maxi = std::max(maxi, c->h_pcg[k].iters);
    if (!c->h_pcg[k].converged) noconv = true;
  }
  c->pred_iters = std::max(1, maxi);
  pred = std::max(1, maxi);
  HIPCHK(hipGetLastError());
  if (any_nonfinite(c)) return fail(CDI_ERR_NONFINITE, "non-finite value in the pressure solve");
  if (noconv) return fail(CDI_ERR_NOCONV, "pressure solve did not reach rtol within maxit");
  return CDI_OK;
}

// Initial-guess mode of k_pcg_init: 0 zero, 1 previous pressure, 2 fitted
// network output.
int guess_mode(const cdi_ctx* c) {
  if (c->guess == CDI_GUESS_ZERO) return 0;
  return (c->guess == CDI_GUESS_LEARNED && c->net) ? 2 : 1;
}

// Network inference for the initial guess of instance 0's next solve (the
// right-hand side and its statistics come from k_rhs / k_solve_setup).
void learned_guess(cdi_ctx* c, int src, int base, int stage) {
  const Inst& I = c->B.inst[0];
  const double* phi = src == 0 ? I.phi : (src == 1 ? I.phi_a : I.phi_b);
  const unsigned g = (unsigned)std::min(1024, ceil_div(I.nx * I.ny, kNT));
  timed(c, "net", [&] {
    CDI_LAUNCH(c, k_features, g, kNT, c->d_inst, 0, phi, nullptr, cdinet::features(c->net), nullptr);
    cdinet::forward(c->net);
    CDI_LAUNCH(c, k_guess_apply, g, kNT, c->d_inst, cdinet::output(c->net));
    with_rows(c->wide_rows, [&](auto R) {
      k_guess_fit<decltype(R)::value><<<(unsigned)c->B.wide.size(), kNT, 0, c->stream>>>(
          c->d_wide, c->d_inst, base, stage, hist_slot(c));
    });
  }, false);
}

template <typename S>
cdi_status run_step(cdi_ctx* c) {
  Batch& B = c->B;
  const unsigned ncell = (unsigned)B.cell.size();
  const unsigned nwide = (unsigned)B.wide.size();
  cdi_status st = CDI_OK;
  if (c->dyn_gamma) k_gamma_step<<<ncell, kNT, 0, c->stream>>>(c->d_cell, c->d_inst);
  for (int k = 0; k < 4; ++k) {
    const int src = k == 0 ? 0 : (k == 2 ? 2 : 1);
    const int dst = (k == 0 || k == 2) ? 1 : 2;
    // phase preparation and stage operator in one launch; per-instance dt:
    // c_next and tau are passed as multiples of the instance dt
    timed(c, "stage", [&] {
      launch_stage<S>(c, k, src, dst, k < 3 ? RK_C[k + 1] : 1.0, RK_B[k], k == 3);
    });
    const double tfac = k < 3 ? RK_C[k + 1] : 1.0;
    timed(c, "rhs", [&] {
      with_rows(c->wide_rows, [&](auto R) {
        CDI_LAUNCH(c, (k_rhs<S, decltype(R)::value>), nwide, kNT, c->d_wide, c->d_inst, dst, tfac,
                                                                   c->rtol, c->maxit);
      });
    });
    // the learned guess is fitted on top of the plain guess of this solve
    if (c->guess == CDI_GUESS_LEARNED && c->net)
      learned_guess(c, dst, c->hist_steps >= 1 ? history_mode(c->hist_steps, c->extrap_order) : 1, k);
    // previous-pressure guess: the same stage of the previous step (linear
    // extrapolation once two steps exist), else the last pressure
    int gm = guess_mode(c);
    if (gm == 1 && c->hist_steps >= 1) gm = history_mode(c->hist_steps, c->extrap_order);
    cdi_status s = solve_loop<S>(c, gm, k);
    if (s == CDI_ERR_NOCONV) st = s;
    else if (s != CDI_OK) return s;
    timed(c, "project", [&] {
      with_rows(c->wide_rows, [&](auto R) {
        CDI_LAUNCH(c, k_project<decltype(R)::value>, nwide, kNT, c->d_wide, c->d_inst, tfac, k == 3, dst, k,
                   hist_slot(c));
      });
    });
  }
  c->hist_steps += 1;
  // the graph launch sizes its fixed budget from the step's largest count
  c->pred_iters = *std::max_element(c->pred_stage, c->pred_stage + 4);
  HIPCHK(hipGetLastError());
  return st;
}

// ------------------------------------------------------------ graph launch
// The same launches as solve_loop with exactly `budget` CG iterations and no
// host polling: once an instance's solve has converged, its remaining
// iteration kernels return at once, so the result is bitwise that of the
// stream path.  k_graph_mark records an instance whose solve needed more.
template <typename S>
void enqueue_solve_fixed(cdi_ctx* c, int guess, int stage, int budget) {
  Batch& B = c->B;
  const unsigned nwide = (unsigned)B.wide.size();
  if (!c->uniform_rho) launch_coef<S>(c);
  with_rows(c->wide_rows, [&](auto R) {
    k_pcg_init<decltype(R)::value><<<nwide, kNT, 0, c->stream>>>(c->d_wide, c->d_inst, guess, stage,
                                                                 hist_slot(c));
  });
  launch_vcycle<S>(c, 0, 0, 0);
  for (int it = 0; it < budget; ++it) {
    const int par = it & 1;
    with_rows(c->wide_rows, [&](auto R) {
      k_pcg_spmv<decltype(R)::value><<<nwide, kNT, 0, c->stream>>>(c->d_wide, c->d_inst, par, par);
    });
    launch_vcycle<S>(c, 1, par, par ^ 1);
  }
  with_rows(c->wide_rows, [&](auto R) {
    k_pcg_xmean<decltype(R)::value><<<nwide, kNT, 0, c->stream>>>(c->d_wide, c->d_inst);
  });
  k_graph_mark<<<(unsigned)ceil_div(B.n, 64), 64, 0, c->stream>>>(c->d_inst, B.n, 0);
}

// Copy every instance's step state (fields and per-stage pressure history)
// to (save) or from its snapshot area.
// (k_snapshot: phi, u, p, the history hp[d][stage] and v one after another.)
cdi_status snapshot(cdi_ctx* c, bool save) {
  size_t most = 0;
  for (int k = 0; k < c->B.n; ++k) {
    const Inst& I = c->B.inst[k];
    const size_t need = (4 + 4 * kHistDepth) * (size_t)I.nx * I.ny + I.nx;
    if (need > snap_doubles(I.nx, I.ny)) return fail(CDI_ERR_STATE, "snapshot layout exceeds its area");
    most = std::max(most, need);
  }
  const dim3 grid((unsigned)std::min<size_t>(1024, (most + kNT - 1) / kNT), (unsigned)c->B.n);
  k_snapshot<<<grid, kNT, 0, c->stream>>>(c->d_inst, save ? 1 : 0);
  HIPCHK(hipGetLastError());
  return CDI_OK;
}

// Upload the run-time tile lists (wide tiles, multigrid tiles below lg) and
// the instance descriptors into their fixed slots.
cdi_status upload_shape(cdi_ctx* c) {
  Batch& B = c->B;
  // the wide and multigrid tiles carry their instance's CG-scalar address
  auto with_pcg = [&](std::vector<Tile> v) {
    for (Tile& t : v) t.pcg = B.inst[t.inst].pcg;   // gptr copy
    return v;
  };
  const std::vector<Tile> w = with_pcg(xcd_order(B.wide));
  HIPCHK(hipMemcpyAsync(c->d_wide, w.data(), sizeof(Tile) * w.size(), hipMemcpyHostToDevice, c->stream));
  std::vector<std::vector<Tile>> lv(B.max_lg);
  for (int l = 0; l < B.max_lg; ++l) {
    lv[l] = with_pcg(xcd_order(B.mg[l]));
    if (!lv[l].empty())
      HIPCHK(hipMemcpyAsync(c->d_mg[l], lv[l].data(), sizeof(Tile) * lv[l].size(),
                            hipMemcpyHostToDevice, c->stream));
  }
  HIPCHK(hipMemcpyAsync(c->d_inst, B.inst.data(), sizeof(Inst) * B.n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));   // the host lists go out of scope
  return CDI_OK;
}

void graph_drop_slot(cdi_ctx* c, int ph) {
  if (c->gexec[ph]) (void)hipGraphExecDestroy(c->gexec[ph]);
  if (c->graph[ph]) (void)hipGraphDestroy(c->graph[ph]);
  c->gexec[ph] = nullptr;
  c->graph[ph] = nullptr;
}

void graph_drop(cdi_ctx* c) {
  for (int ph = 0; ph < 4; ++ph) graph_drop_slot(c, ph);
  c->graph_budget = 0;
}

// Capture one RK4 step (snapshot, 4 stages with fixed-budget solves, copy of
// the CG scalars to pinned memory) on the context's capture stream, for the
// history ring slot of the current step.  A new budget drops the steps
// captured for the other slots.
template <typename S>
cdi_status graph_capture(cdi_ctx* c, int budget) {
  const int ph = hist_slot(c);
  if (budget != c->graph_budget) graph_drop(c);
  else graph_drop_slot(c, ph);
  Batch& B = c->B;
  const unsigned ncell = (unsigned)B.cell.size();
  const unsigned nwide = (unsigned)B.wide.size();
  hipStream_t user = c->stream;
  const std::string timed0 = c->timed;
  c->timed.clear();
  c->stream = c->gstream;
  auto body = [&]() -> cdi_status {
    cdi_status st = snapshot(c, true);
    if (st != CDI_OK) return st;
    k_graph_mark<<<(unsigned)ceil_div(B.n, 64), 64, 0, c->stream>>>(c->d_inst, B.n, 1);
    if (c->dyn_gamma) k_gamma_step<<<ncell, kNT, 0, c->stream>>>(c->d_cell, c->d_inst);
    // the full history of the extrapolation order exists (run_graph_step)
    const int gm = c->guess == CDI_GUESS_ZERO ? 0 : history_mode(c->extrap_order + 1, c->extrap_order);
    for (int k = 0; k < 4; ++k) {
      const int src = k == 0 ? 0 : (k == 2 ? 2 : 1);
      const int dst = (k == 0 || k == 2) ? 1 : 2;
      const double tfac = k < 3 ? RK_C[k + 1] : 1.0;
      launch_stage<S>(c, k, src, dst, tfac, RK_B[k], k == 3);
      with_rows(c->wide_rows, [&](auto R) {
        k_rhs<S, decltype(R)::value><<<nwide, kNT, 0, c->stream>>>(c->d_wide, c->d_inst, dst, tfac,
                                                                   c->rtol, c->maxit);
      });
      enqueue_solve_fixed<S>(c, gm, k, budget);
      with_rows(c->wide_rows, [&](auto R) {
        k_project<decltype(R)::value><<<nwide, kNT, 0, c->stream>>>(c->d_wide, c->d_inst, tfac, k == 3, dst, k,
                                                                    hist_slot(c));
      });
    }
    return pcg_to_host(c);
  };
  hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
  cdi_status st = e == hipSuccess ? body() : fail(CDI_ERR_DEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  hipGraph_t g = nullptr;
  if (e == hipSuccess) {
    hipError_t e2 = hipStreamEndCapture(c->stream, &g);
    if (st == CDI_OK && e2 != hipSuccess) st = fail(CDI_ERR_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e2));
    if (st == CDI_OK && (e2 = hipGetLastError()) != hipSuccess)
      st = fail(CDI_ERR_DEVICE, "capture: %s", hipGetErrorString(e2));
  }
  c->stream = user;
  c->timed = timed0;
  if (st != CDI_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  c->graph[ph] = g;
  e = hipGraphInstantiate(&c->gexec[ph], g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    graph_drop(c);
    return fail(CDI_ERR_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  if (c->graph_budget != budget) c->graph_slack = 0;
  c->graph_budget = budget;
  return CDI_OK;
}

// One step through the captured graph.  The first two steps (before the
// pressure history exists) and any step whose budget turned out too small run
// on the stream path; the latter from the restored snapshot.
template <typename S>
cdi_status run_graph_step(cdi_ctx* c) {
  if (c->hist_steps < c->extrap_order + 1) return run_step<S>(c);
  Batch& B = c->B;
  if (!c->gstream) {
    HIPCHK(hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&c->gev0, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->gev1, hipEventDisableTiming));
  }
  if (!c->uniform_rho || !c->coef_ready) {
    // coefficients of a uniform density are set up once, outside the graph
    if (c->uniform_rho) { launch_coef<S>(c); c->coef_ready = true; }
  }
  const int want = std::min(c->maxit, c->pred_iters + 1);
  const int ph = hist_slot(c);
  const bool rebudget = c->graph_budget == 0 || want > c->graph_budget ||
                        (c->graph_slack >= 50 && want < c->graph_budget);
  if (rebudget || !c->gexec[ph]) {
    cdi_status st = graph_capture<S>(c, rebudget ? want : c->graph_budget);
    if (st != CDI_OK) return st;
  }
  // order the replay after the caller's work and the caller's later work after it
  HIPCHK(hipEventRecord(c->gev0, c->stream));
  HIPCHK(hipStreamWaitEvent(c->gstream, c->gev0, 0));
  HIPCHK(hipGraphLaunch(c->gexec[ph], c->gstream));
  HIPCHK(hipEventRecord(c->gev1, c->gstream));
  HIPCHK(hipStreamWaitEvent(c->stream, c->gev1, 0));
  HIPCHK(hipEventSynchronize(c->gev1));
  c->graph_replays += 1;
  bool miss = false;
  int maxi = 0;
  for (int k = 0; k < B.n; ++k) {
    miss = miss || c->h_pcg[k].miss;
    maxi = std::max(maxi, c->h_pcg[k].step_iters);
  }
  if (miss) {
    // budget too small: back to the step's start, redo it on the stream path
    c->graph_misses += 1;
    cdi_status st = snapshot(c, false);
    if (st != CDI_OK) return st;
    c->pred_iters = std::max(c->pred_iters, c->graph_budget + 2);
    return run_step<S>(c);
  }
  bool noconv = false;
  for (int k = 0; k < B.n; ++k) {
    c->last_iters[k] = c->h_pcg[k].iters;
    c->last_relres[k] = c->h_pcg[k].relres;
    c->last_conv[k] = c->h_pcg[k].converged;
    if (!c->h_pcg[k].converged) noconv = true;
  }
  c->pred_iters = std::max(1, maxi);
  c->graph_slack = maxi + 2 <= c->graph_budget ? c->graph_slack + 1 : 0;
  c->hist_steps += 1;
  if (any_nonfinite(c)) return fail(CDI_ERR_NONFINITE, "non-finite value in the pressure solve");
  if (noconv) return fail(CDI_ERR_NOCONV, "pressure solve did not reach rtol within maxit");
  return CDI_OK;
}

// Steps of the persistent launch per kernel: bounds the duration of one
// launch; the per-stage history carries over between launches.
constexpr int kPersistChunk = 32;

template <typename S>
cdi_status run_persistent(cdi_ctx* c, int nsteps) {
  Batch& B = c->B;
  const int gm = c->guess == CDI_GUESS_ZERO ? 0 : 1;
  for (int done = 0; done < nsteps; done += kPersistChunk) {
    const int m = std::min(kPersistChunk, nsteps - done);
    timed(c, "persistent", [&] {
      CDI_LAUNCH(c, k_step_persistent<S>, (unsigned)B.n, PNT, c->d_cell_inst, c->d_inst, m,
                 (int)((c->step + done) & 3), c->hist_steps, gm, c->extrap_order, c->rtol, c->maxit,
                 (int)(done > 0));
    });
    HIPCHK(hipGetLastError());
    c->hist_steps += m;
  }
  {
    cdi_status cs = pcg_to_host(c);
    if (cs != CDI_OK) return cs;
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  bool noconv = false;
  int maxi = 0;
  for (int k = 0; k < B.n; ++k) {
    c->last_iters[k] = c->h_pcg[k].iters;
    c->last_relres[k] = c->h_pcg[k].relres;
    c->last_conv[k] = c->h_pcg[k].converged;
    maxi = std::max(maxi, c->h_pcg[k].max_iters);
    if (c->h_pcg[k].nfail) noconv = true;
  }
  c->pred_iters = std::max(1, maxi);
  if (any_nonfinite(c)) return fail(CDI_ERR_NONFINITE, "non-finite value in the pressure solve");
  if (noconv) return fail(CDI_ERR_NOCONV, "pressure solve did not reach rtol within maxit");
  return CDI_OK;
}

}  // namespace

// ================================================================ C ABI
extern "C" {

const char* cdi_last_error(void) { return g_err.c_str(); }

double cdi_default_dt(const cdi_params* params) {
  Resolved R;
  if (resolve(params, R) != CDI_OK) return -1.0;
  return R.dt;
}

size_t cdi_workspace_bytes(const cdi_params* params, int32_t n) {
  if (!params || n < 1) { fail(CDI_ERR_ARG, "bad arguments"); return 0; }
  std::vector<Resolved> Rs(n);
  for (int k = 0; k < n; ++k)
    if (resolve(params + k, Rs[k]) != CDI_OK) return 0;
  return batch_bytes(Rs, nullptr, nullptr);
}

cdi_status cdi_init_batch(const cdi_params* params, int32_t n, const cdi_fields* fields,
                          void* workspace, size_t workspace_bytes, void* hip_stream, cdi_ctx** out) {
  if (!out) return fail(CDI_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!params || !fields || n < 1) return fail(CDI_ERR_ARG, "params/fields NULL or n < 1");
  if (!workspace) return fail(CDI_ERR_ARG, "workspace is NULL");
  if (((uintptr_t)workspace) & 255) return fail(CDI_ERR_ARG, "workspace must be 256-byte aligned");
  std::vector<Resolved> Rs(n);
  for (int k = 0; k < n; ++k) {
    cdi_status s = resolve(params + k, Rs[k]);
    if (s != CDI_OK) return s;
    if (!fields[k].phi || !fields[k].u || !fields[k].v || !fields[k].p)
      return fail(CDI_ERR_ARG, "instance %d: a field pointer is NULL", k);
    if (Rs[k].p.precision != Rs[0].p.precision)
      return fail(CDI_ERR_ARG, "all instances of a batch must use the same precision");
    if (std::max(1, Rs[k].p.mg_smooth) != std::max(1, Rs[0].p.mg_smooth))
      return fail(CDI_ERR_ARG, "all instances of a batch must use the same mg_smooth");
  }
  const size_t need = batch_bytes(Rs, nullptr, nullptr);
  if (workspace_bytes < need)
    return fail(CDI_ERR_ARG, "workspace too small: %zu < %zu bytes", workspace_bytes, need);

  cdi_ctx* c = new cdi_ctx();
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)workspace;
  Batch& B = c->B;
  B.n = n;
  B.R = Rs;
  B.inst.assign(n, Inst{});
  c->mixed = Rs[0].p.precision == CDI_MIXED;
  c->nu = std::max(1, Rs[0].p.mg_smooth);
  c->guess = Rs[0].p.guess;
  c->rtol = Rs[0].rtol;
  c->maxit = Rs[0].maxit;
  for (int k = 0; k < n; ++k) {
    fill_inst(Rs[k], fields[k], B.inst[k]);
    if (Rs[k].p.rho1 != Rs[k].p.rho2) c->uniform_rho = false;
    if (Rs[k].p.gamma_factor > 0) c->dyn_gamma = true;
  }
  batch_bytes(Rs, &B, c->ws);
  // wide tiles: 4 rows per thread once the batch has enough cells to fill
  // the GPU with the taller tiles (cdi_tune measures instead of guessing)
  long cells = 0;
  for (int k = 0; k < n; ++k) cells += (long)Rs[k].p.nx * Rs[k].p.ny;
  c->wide_rows = cells >= (1L << 18) ? 4 : 1;
  c->coarse_cells = kDefaultCoarseCells;
  for (int k = 0; k < n; ++k) set_lg(B.R[k], c->coarse_cells);
  build_tiles(B, c->wide_rows);
  // shared header
  size_t off = 0;
  c->d_inst = (Inst*)(c->ws + off);
  off = align256(off + sizeof(Inst) * n);
  c->d_diag = (DiagOut*)(c->ws + off);
  off = align256(off + sizeof(DiagOut) * n);
  c->d_pcg_all = (PcgScalars*)(c->ws + off);
  off = align256(off + sizeof(PcgScalars) * n);
  Tile* tl = (Tile*)(c->ws + off);
  // fixed slots: level-0 cell tiles (XCD-banded order, tiled launches; then
  // instance order, persistent launch), the wide tiles (room for 1 row per
  // thread), the multigrid tiles of every level below lc (the coarse-kernel
  // start level lg <= lc and the wide shape change at run time)
  std::vector<Tile> all = xcd_order(B.cell);
  c->d_cell = tl;
  size_t pos = all.size();
  c->d_cell_inst = tl + pos;
  all.insert(all.end(), B.cell.begin(), B.cell.end());
  pos += B.cell.size();
  c->d_wide = tl + pos;
  pos += B.cell.size();
  c->d_mg.assign(std::max(B.max_lc, 1), nullptr);
  for (int l = 0; l < B.max_lc; ++l) {
    c->d_mg[l] = tl + pos;
    for (int k = 0; k < n; ++k)
      if (l < Rs[k].lc)
        pos += (size_t)ceil_div(Rs[k].lnx[l], FX) * ceil_div(Rs[k].lny[l], FY);
  }
  c->d_strip = tl + pos;
  {
    const std::vector<Tile> sv = xcd_order(B.strip);
    all.resize(pos, Tile{});
    all.insert(all.end(), sv.begin(), sv.end());
  }
  c->h_pcg = nullptr;
  hipError_t e = hipHostMalloc((void**)&c->h_pcg, sizeof(PcgScalars) * n, hipHostMallocDefault);
  if (e != hipSuccess) { delete c; return fail(CDI_ERR_DEVICE, "hipHostMalloc: %s", hipGetErrorString(e)); }
  c->last_iters.assign(n, 0);
  c->last_relres.assign(n, 0.0);
  c->last_conv.assign(n, 1);
  c->mass0.assign(n, 0.0);
  auto cleanup_fail = [&](hipError_t err, const char* what) {
    (void)hipHostFree(c->h_pcg);
    delete c;
    return fail(CDI_ERR_DEVICE, "%s: %s", what, hipGetErrorString(err));
  };
  if ((e = hipMemcpyAsync(c->d_inst, B.inst.data(), sizeof(Inst) * n, hipMemcpyHostToDevice, c->stream)) != hipSuccess)
    return cleanup_fail(e, "copy instances");
  if ((e = hipMemcpyAsync(tl, all.data(), sizeof(Tile) * all.size(), hipMemcpyHostToDevice, c->stream)) != hipSuccess)
    return cleanup_fail(e, "copy tiles");
  {
    cdi_status us = upload_shape(c);
    if (us != CDI_OK) {
      (void)hipHostFree(c->h_pcg);
      delete c;
      return us;
    }
  }
  // zero the whole per-instance workspace once (walls of v-type arrays,
  // counters, flags); every later write stays inside the domain
  const size_t hdr = (size_t)((char*)B.inst[0].phi_a.p - c->ws);
  if ((e = hipMemsetAsync(c->ws + hdr, 0, need - hdr, c->stream)) != hipSuccess)
    return cleanup_fail(e, "clear workspace");
  k_gamma_init<<<(unsigned)ceil_div(n, 64), 64, 0, c->stream>>>(c->d_inst, n);
  if ((e = hipGetLastError()) != hipSuccess) return cleanup_fail(e, "gamma init");
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return cleanup_fail(e, "init sync");
  if ((e = hipEventCreate(&c->ev0)) != hipSuccess) return cleanup_fail(e, "event");
  if ((e = hipEventCreate(&c->ev1)) != hipSuccess) return cleanup_fail(e, "event");
  // initial diagnostics: mass0
  *out = c;
  for (int k = 0; k < n; ++k) {
    cdi_diag d;
    cdi_status s = cdi_diagnostics(c, k, &d);
    if (s != CDI_OK) { cdi_destroy(c); *out = nullptr; return s; }
    c->mass0[k] = d.mass;
  }
  return CDI_OK;
}

cdi_status cdi_init(const cdi_params* params, const cdi_fields* fields, void* workspace,
                    size_t workspace_bytes, void* hip_stream, cdi_ctx** out) {
  return cdi_init_batch(params, 1, fields, workspace, workspace_bytes, hip_stream, out);
}

cdi_status cdi_step(cdi_ctx* c, int32_t nsteps) {
  if (!c) return fail(CDI_ERR_ARG, "ctx is NULL");
  if (nsteps < 0) return fail(CDI_ERR_ARG, "nsteps < 0");
  cdi_status st = CDI_OK;
  if (c->launch == CDI_LAUNCH_PERSISTENT && nsteps > 0) {
    if (c->guess == CDI_GUESS_LEARNED && c->net)
      return fail(CDI_ERR_STATE, "the learned guess needs the tiled launch");
    st = c->mixed ? run_persistent<float>(c, nsteps) : run_persistent<double>(c, nsteps);
    if (st != CDI_OK && st != CDI_ERR_NOCONV) return st;
    c->t += nsteps * c->B.R[0].dt;
    c->step += nsteps;
    return st;
  }
  const bool graph = c->launch == CDI_LAUNCH_GRAPH;
  if (graph && c->guess == CDI_GUESS_LEARNED && c->net)
    return fail(CDI_ERR_STATE, "the learned guess needs the tiled launch");
  for (int s = 0; s < nsteps; ++s) {
    cdi_status r = graph ? (c->mixed ? run_graph_step<float>(c) : run_graph_step<double>(c))
                         : (c->mixed ? run_step<float>(c) : run_step<double>(c));
    if (r == CDI_ERR_NOCONV) st = r;
    else if (r != CDI_OK) return r;
    c->t += c->B.R[0].dt;
    c->step += 1;
  }
  return st;
}

cdi_status cdi_step_concurrent(cdi_ctx* const* ctxs, int32_t n, int32_t nsteps) {
  if (!ctxs || n < 1) return fail(CDI_ERR_ARG, "ctxs is NULL or n < 1");
  if (nsteps < 0) return fail(CDI_ERR_ARG, "nsteps < 0");
  for (int k = 0; k < n; ++k) {
    if (!ctxs[k]) return fail(CDI_ERR_ARG, "ctxs[%d] is NULL", k);
    for (int m = 0; m < k; ++m)
      if (ctxs[m] == ctxs[k]) return fail(CDI_ERR_ARG, "ctxs[%d] repeats ctxs[%d]", k, m);
  }
  // one host thread per further context; each keeps its own error message,
  // handed back to the caller's thread for the first failing context
  // a worker thread starts on device 0: give it the device of its
  // context's stream (the caller's device for the null stream)
  int dev0 = 0;
  hipError_t e = hipGetDevice(&dev0);
  if (e != hipSuccess) return fail(CDI_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  std::vector<int> dev(n, dev0);
  for (int k = 0; k < n; ++k)
    if (ctxs[k]->stream) {
      hipDevice_t d;
      e = hipStreamGetDevice(ctxs[k]->stream, &d);
      if (e != hipSuccess) return fail(CDI_ERR_DEVICE, "hipStreamGetDevice: %s", hipGetErrorString(e));
      dev[k] = (int)d;
    }
  std::vector<cdi_status> st(n, CDI_OK);
  std::vector<std::string> msg(n);
  auto run = [&](int k) {
    if (k > 0) {
      hipError_t he = hipSetDevice(dev[k]);
      if (he != hipSuccess) {
        st[k] = CDI_ERR_DEVICE;
        msg[k] = std::string("hipSetDevice: ") + hipGetErrorString(he);
        return;
      }
    }
    st[k] = cdi_step(ctxs[k], nsteps);
    if (st[k] != CDI_OK) msg[k] = g_err;
  };
  std::vector<std::thread> th;
  th.reserve(n - 1);
  for (int k = 1; k < n; ++k) th.emplace_back(run, k);
  run(0);
  for (auto& t : th) t.join();
  cdi_status out = CDI_OK;
  for (int k = 0; k < n; ++k)
    if (st[k] != CDI_OK && st[k] != CDI_ERR_NOCONV) {
      g_err = msg[k];
      return st[k];
    } else if (st[k] == CDI_ERR_NOCONV && out == CDI_OK) {
      out = st[k];
      g_err = msg[k];
    }
  return out;
}

cdi_status cdi_solve_pressure(cdi_ctx* c, const double* b, double* p, cdi_solve_info* info) {
  if (!c) return fail(CDI_ERR_ARG, "ctx is NULL");
  if (!p) return fail(CDI_ERR_ARG, "p is NULL");
  Batch& B = c->B;
  if (B.n != 1) return fail(CDI_ERR_STATE, "standalone solve needs a single-instance context");
  const unsigned ncell = (unsigned)B.cell.size();
  // the solve uses the caller p as guess buffer: point the instance at it
  Inst I = B.inst[0];
  double* saved_p = I.p;
  I.p = p;
  HIPCHK(hipMemcpyAsync(c->d_inst, &I, sizeof(Inst), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipEventRecord(c->ev0, c->stream));
  if (c->mixed)
    k_solve_setup<float><<<ncell, kNT, 0, c->stream>>>(c->d_cell, c->d_inst, b, c->rtol, c->maxit);
  else
    k_solve_setup<double><<<ncell, kNT, 0, c->stream>>>(c->d_cell, c->d_inst, b, c->rtol, c->maxit);
  c->coef_ready = false;
  if (c->guess == CDI_GUESS_LEARNED && c->net) learned_guess(c, 0, 1, 0);
  const int guess = guess_mode(c);
  cdi_status s = c->mixed ? solve_loop<float>(c, guess, 0) : solve_loop<double>(c, guess, 0);
  c->coef_ready = false;   // coefficients now follow the caller phase field
  k_solve_out<<<ncell, kNT, 0, c->stream>>>(c->d_cell, c->d_inst, p);
  HIPCHK(hipEventRecord(c->ev1, c->stream));
  I.p = saved_p;
  HIPCHK(hipMemcpyAsync(c->d_inst, &I, sizeof(Inst), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (info) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    info->iterations = c->last_iters[0];
    info->converged = c->last_conv[0];
    info->guess_used = guess ? ((c->guess == CDI_GUESS_LEARNED && c->net) ? CDI_GUESS_LEARNED
                                                                       : CDI_GUESS_PREV)
                             : CDI_GUESS_ZERO;
    info->relres = c->last_relres[0];
    info->bnorm = c->h_pcg[0].fnorm;
    info->ms = ms;
  }
  return s;
}

cdi_status cdi_eval_rhs(cdi_ctx* c, double* l_phi, double* l_mx, double* l_my, double* u_y,
                        double* u_slip) {
  if (!c) return fail(CDI_ERR_ARG, "ctx is NULL");
  if (!l_phi || !l_mx || !l_my) return fail(CDI_ERR_ARG, "output pointer is NULL");
  Batch& B = c->B;
  const unsigned ncell = (unsigned)B.cell.size();
  const Inst& I = B.inst[0];
  const size_t nc = (size_t)I.nx * I.ny;
  // the regularisation velocity of a step that would start from this state
  if (c->dyn_gamma) k_gamma_step<<<ncell, kNT, 0, c->stream>>>(c->d_cell, c->d_inst);
  if (c->mixed)
    launch_stage<float>(c, -1, 0, 0, 0.0, 0.0, 1);
  else
    launch_stage<double>(c, -1, 0, 0, 0.0, 0.0, 1);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(l_phi, I.acc_phi, nc * 8, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(l_mx, I.acc_mx, nc * 8, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemsetAsync(l_my, 0, (size_t)(I.ny + 1) * I.nx * 8, c->stream));
  HIPCHK(hipMemcpyAsync(l_my + I.nx, I.acc_my + I.nx, (size_t)(I.ny - 1) * I.nx * 8,
                        hipMemcpyDeviceToDevice, c->stream));
  if (u_y) HIPCHK(hipMemcpyAsync(u_y, I.uY, (size_t)2 * I.nx * 8, hipMemcpyDeviceToDevice, c->stream));
  if (u_slip) HIPCHK(hipMemcpyAsync(u_slip, I.uslip, (size_t)2 * I.nx * 8, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return CDI_OK;
}

cdi_status cdi_cg_iterations(cdi_ctx* c, int64_t* per_instance) {
  if (!c || !per_instance) return fail(CDI_ERR_ARG, "NULL argument");
  cdi_status st = pcg_to_host(c);
  if (st != CDI_OK) return st;
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int k = 0; k < c->B.n; ++k) per_instance[k] = c->h_pcg[k].iters_total;
  return CDI_OK;
}

cdi_status cdi_diagnostics(cdi_ctx* c, int32_t idx, cdi_diag* out) {
  if (!c || !out) return fail(CDI_ERR_ARG, "NULL argument");
  Batch& B = c->B;
  if (idx < 0 || idx >= B.n) return fail(CDI_ERR_ARG, "instance %d out of range", idx);
  const unsigned ncell = (unsigned)B.cell.size();
  if (c->mixed) k_phase_prep<float, 1><<<ncell, kNT, 0, c->stream>>>(c->d_cell, c->d_inst, 0);
  else k_phase_prep<double, 1><<<ncell, kNT, 0, c->stream>>>(c->d_cell, c->d_inst, 0);
  k_wall<<<(unsigned)B.n, kNT, 0, c->stream>>>(c->d_inst);
  k_diag<<<ncell, kNT, 0, c->stream>>>(c->d_cell, c->d_inst, c->d_diag);
  k_contact<<<dim3((unsigned)B.n, 2), kNT, 0, c->stream>>>(c->d_inst, c->d_diag);
  HIPCHK(hipGetLastError());
  const Inst& I = B.inst[idx];
  DiagOut d;
  std::vector<double> w((size_t)4 * I.nx + I.nx);
  HIPCHK(hipMemcpyAsync(&d, c->d_diag + idx, sizeof d, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(w.data(), I.uY, (size_t)2 * I.nx * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(w.data() + 2 * I.nx, I.uslip, (size_t)2 * I.nx * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(w.data() + 4 * I.nx, I.wall, (size_t)I.nx * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  std::memset(out, 0, sizeof *out);
  out->t = c->t;
  out->step = c->step;
  out->mass = d.mass;
  out->mass0 = c->mass0[idx];
  out->phi_min = d.phi_min;
  out->phi_max = d.phi_max;
  out->max_div = d.max_div;
  out->ke = d.ke;
  out->nonfinite = d.nonfinite > 0 ? 1 : 0;
  for (int wl = 0; wl < 2; ++wl) {
    double mu = 0.0, ms = 0.0;
    for (int i = 0; i < I.nx; ++i) {
      mu = std::max(mu, std::fabs(w[(size_t)wl * I.nx + i]));
      ms = std::max(ms, std::fabs(w[(size_t)2 * I.nx + wl * I.nx + i]));
    }
    out->max_uY[wl] = mu;
    out->max_uslip[wl] = ms;
  }
  out->last_iters = c->last_iters[idx];
  out->last_relres = c->last_relres[idx];
  for (int wl = 0; wl < 2; ++wl) {
    out->n_contact[wl] = d.n_contact[wl];
    for (int m = 0; m < kMaxContacts; ++m) out->contact_x[2 * wl + m] = d.contact_x[wl][m];
    out->wetted_len[wl] = d.wetted_len[wl];
    out->theta_est[wl] = d.theta_est[wl];
  }
  return out->nonfinite ? fail(CDI_ERR_NONFINITE, "non-finite value in the state") : CDI_OK;
}

cdi_status cdi_timing_enable(cdi_ctx* c, const char* kernel) {
  if (!c) return fail(CDI_ERR_ARG, "ctx is NULL");
  static const char* known[] = {"phase_prep", "stage", "rhs", "pcg_init", "mg_down",
                                "mg_down_other", "mg_coarse", "mg_up", "mg_up_other", "mg_coef",
                                "pcg_spmv", "pcg_xmean", "project", "net", "persistent"};
  HIPCHK(hipStreamSynchronize(c->stream));
  c->tev_used = 0;
  c->timed_ms = 0.0;
  c->timed_launches = 0;
  if (!kernel) { c->timed.clear(); return CDI_OK; }
  bool ok = false;
  for (const char* k : known) ok = ok || std::strcmp(k, kernel) == 0;
  if (!ok) return fail(CDI_ERR_ARG, "unknown kernel family '%s'", kernel);
  if (c->tev.empty()) {
    c->tev.assign(2 * kTimedPairs, nullptr);
    for (auto& e : c->tev) HIPCHK(hipEventCreate(&e));
  }
  c->timed = kernel;
  return CDI_OK;
}

cdi_status cdi_timing_read(cdi_ctx* c, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches) return fail(CDI_ERR_ARG, "NULL argument");
  HIPCHK(timing_flush(c));
  *total_ms = c->timed_ms;
  *launches = c->timed_launches;
  return CDI_OK;
}

// Switch the run-time launch shape: rows per thread of the wide-tile kernels
// and the coarse kernel's start level (first level with at most
// `coarse_cells` cells); rebuilds and uploads the affected tile lists.
static cdi_status apply_shape(cdi_ctx* c, int rows, long coarse_cells, int nu) {
  if (rows == c->wide_rows && coarse_cells == c->coarse_cells && nu == c->nu) return CDI_OK;
  graph_drop(c);   // the captured step holds the old launch grids
  Batch& B = c->B;
  HIPCHK(hipStreamSynchronize(c->stream));
  build_wide(B, rows);
  for (int k = 0; k < B.n; ++k) set_lg(B.R[k], coarse_cells);
  build_mg(B);
  for (int k = 0; k < B.n; ++k) {
    B.inst[k].nu = nu;
    B.inst[k].nu_c = nu + 1;
  }
  c->wide_rows = rows;
  c->coarse_cells = coarse_cells;
  c->nu = nu;
  return upload_shape(c);
}

// Rows of the stage kernel's strips (16, 32 or 64): rebuild and upload the
// strip list (its slot holds the 16-row count, the largest).
static cdi_status apply_strip_rows(cdi_ctx* c, int rows) {
  if (rows == c->B.strip_rows) return CDI_OK;
  graph_drop(c);
  HIPCHK(hipStreamSynchronize(c->stream));
  build_strips(c->B, rows);
  const std::vector<Tile> sv = xcd_order(c->B.strip);
  HIPCHK(hipMemcpyAsync(c->d_strip, sv.data(), sizeof(Tile) * sv.size(), hipMemcpyHostToDevice,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return CDI_OK;
}

static cdi_status apply_wide_rows(cdi_ctx* c, int rows) {
  return apply_shape(c, rows, c->coarse_cells, c->nu);
}

cdi_status cdi_set_mg_smooth(cdi_ctx* c, int32_t nu) {
  if (!c) return fail(CDI_ERR_ARG, "ctx is NULL");
  if (nu < 1 || nu > 2) return fail(CDI_ERR_ARG, "mg_smooth must be 1 or 2");
  return apply_shape(c, c->wide_rows, c->coarse_cells, nu);
}

cdi_status cdi_get_mg_smooth(cdi_ctx* c, int32_t* nu) {
  if (!c || !nu) return fail(CDI_ERR_ARG, "NULL argument");
  *nu = c->nu;
  return CDI_OK;
}

cdi_status cdi_set_extrapolation(cdi_ctx* c, int32_t order) {
  if (!c) return fail(CDI_ERR_ARG, "ctx is NULL");
  if (order < 0 || order > kHistDepth - 1)
    return fail(CDI_ERR_ARG, "extrapolation order must be in [0, %d]", kHistDepth - 1);
  if (order != c->extrap_order) graph_drop(c);   // a captured step holds its guess mode
  c->extrap_order = order;
  return CDI_OK;
}

cdi_status cdi_get_extrapolation(cdi_ctx* c, int32_t* order) {
  if (!c || !order) return fail(CDI_ERR_ARG, "NULL argument");
  *order = c->extrap_order;
  return CDI_OK;
}

cdi_status cdi_set_coarse_cells(cdi_ctx* c, int32_t cells) {
  if (!c) return fail(CDI_ERR_ARG, "ctx is NULL");
  if (cells < kCoarseCells || cells > (1 << 20))
    return fail(CDI_ERR_ARG, "coarse_cells must be in [%d, %d]", kCoarseCells, 1 << 20);
  return apply_shape(c, c->wide_rows, cells, c->nu);
}

cdi_status cdi_get_coarse_cells(cdi_ctx* c, int32_t* cells) {
  if (!c || !cells) return fail(CDI_ERR_ARG, "NULL argument");
  *cells = (int32_t)c->coarse_cells;
  return CDI_OK;
}

cdi_status cdi_set_strip_rows(cdi_ctx* c, int32_t rows) {
  if (!c) return fail(CDI_ERR_ARG, "ctx is NULL");
  if (rows != kStripRows[0] && rows != kStripRows[1] && rows != kStripRows[2])
    return fail(CDI_ERR_ARG, "strip rows must be %d, %d or %d", kStripRows[2], kStripRows[1],
                kStripRows[0]);
  return apply_strip_rows(c, rows);
}

cdi_status cdi_get_strip_rows(cdi_ctx* c, int32_t* rows) {
  if (!c || !rows) return fail(CDI_ERR_ARG, "NULL argument");
  *rows = c->B.strip_rows;
  return CDI_OK;
}

cdi_status cdi_set_tile_rows(cdi_ctx* c, int32_t rows) {
  if (!c) return fail(CDI_ERR_ARG, "ctx is NULL");
  if (rows != kWideRows[0] && rows != kWideRows[1])
    return fail(CDI_ERR_ARG, "rows must be %d or %d", kWideRows[0], kWideRows[1]);
  return apply_wide_rows(c, rows);
}

cdi_status cdi_get_tile_rows(cdi_ctx* c, int32_t* rows) {
  if (!c || !rows) return fail(CDI_ERR_ARG, "NULL argument");
  *rows = c->wide_rows;
  return CDI_OK;
}

// Device state a step reads besides its scratch: the caller fields and the
// per-stage pressure history (FP64), per instance.
static size_t tune_bytes(const cdi_ctx* c) {
  size_t b = 0;
  for (int k = 0; k < c->B.n; ++k)
    b += align256(snap_doubles(c->B.R[k].p.nx, c->B.R[k].p.ny) * sizeof(double));
  return b;
}

size_t cdi_tune_bytes(const cdi_ctx* c) { return c ? tune_bytes(c) : 0; }

static cdi_status tune_copy(cdi_ctx* c, char* scratch, bool save) {
  size_t off = 0;
  for (int k = 0; k < c->B.n; ++k) {
    const Inst& I = c->B.inst[k];
    const size_t n = (size_t)I.nx * I.ny, nf = n + I.nx;
    double* bufs[3 + 4 * kHistDepth] = {I.phi, I.u, I.p};
    for (int d = 0; d < kHistDepth; ++d)
      for (int s = 0; s < 4; ++s) bufs[3 + 4 * d + s] = I.hp[d][s];
    double* base = (double*)(scratch + off);
    size_t pos = 0;
    for (double* b : bufs) {
      void* dst = save ? (void*)(base + pos) : (void*)b;
      const void* src = save ? (const void*)b : (const void*)(base + pos);
      HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      pos += n;
    }
    if (pos + nf > snap_doubles(I.nx, I.ny)) return fail(CDI_ERR_STATE, "saved state exceeds its area");
    void* dst = save ? (void*)(base + pos) : (void*)I.v;
    const void* src = save ? (const void*)I.v : (const void*)(base + pos);
    HIPCHK(hipMemcpyAsync(dst, src, nf * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    off += align256(snap_doubles(I.nx, I.ny) * sizeof(double));
  }
  return CDI_OK;
}

// Host-side state a step advances (restored after every tuning candidate).
struct HostSnap {
  double t = 0.0;
  long step = 0;
  int hist = 0, pred = 0;
  int pred_stage[4] = {0, 0, 0, 0};
  std::vector<int> iters, conv;
  std::vector<double> relres;
  std::string timed;
  explicit HostSnap(const cdi_ctx* c)
      : t(c->t), step(c->step), hist(c->hist_steps), pred(c->pred_iters), iters(c->last_iters),
        conv(c->last_conv), relres(c->last_relres), timed(c->timed) {
    std::copy(c->pred_stage, c->pred_stage + 4, pred_stage);
  }
  // time, step and the iteration predictor (between candidates)
  void rewind(cdi_ctx* c) const {
    c->t = t; c->step = step; c->hist_steps = hist; c->pred_iters = pred;
    std::copy(pred_stage, pred_stage + 4, c->pred_stage);
  }
  // everything (at the end)
  void restore(cdi_ctx* c) const {
    rewind(c);
    c->last_iters = iters; c->last_conv = conv; c->last_relres = relres;
    c->timed = timed;
  }
};

constexpr long kPersistTuneCells = 16384;

cdi_status cdi_tune(cdi_ctx* c, int32_t trial_steps, void* scratch, size_t scratch_bytes,
                    cdi_tune_info* out) {
  if (!c || !scratch) return fail(CDI_ERR_ARG, "NULL argument");
  if (trial_steps < 1) return fail(CDI_ERR_ARG, "trial_steps must be >= 1");
  if (scratch_bytes < tune_bytes(c))
    return fail(CDI_ERR_ARG, "scratch too small: %zu < %zu bytes", scratch_bytes, tune_bytes(c));
  char* sc = (char*)scratch;
  HIPCHK(hipStreamSynchronize(c->stream));
  cdi_status st = tune_copy(c, sc, true);
  if (st != CDI_OK) return st;
  const HostSnap snap(c);
  c->timed.clear();
  c->wide_rows_pick = c->wide_rows;
  c->coarse_cells_pick = c->coarse_cells;
  c->nu_pick = c->nu;
  // candidates: tiled for every (sweep pairs, rows, coarse cells), then
  // persistent (with the fastest tiled sweep count) and graph (with the
  // fastest tiled shape)
  struct Cand { int launch, rows; long coarse; int nu; int slot; };
  std::vector<Cand> cands;
  for (int v = 0; v < 2; ++v)
    for (int r = 0; r < 2; ++r)
      for (int q = 0; q < 3; ++q)
        cands.push_back({CDI_LAUNCH_TILED, kWideRows[r], kTuneCoarse[q], v + 1, v * 6 + r * 3 + q});
  cands.push_back({CDI_LAUNCH_PERSISTENT, 0, 0, 0, 12});
  cands.push_back({CDI_LAUNCH_GRAPH, 0, 0, 0, 13});
  double best = INFINITY, best_tiled = INFINITY;
  Cand pick{c->launch, c->wide_rows, c->coarse_cells, c->nu, -1};
  cdi_tune_info info{};
  for (int q = 0; q < 14; ++q) info.ms_per_step[q] = -1.0;
  // one block per instance: timed only where an instance fits a CU's reach
  // (beyond 16384 cells a step takes several times the tiled one, up to
  // seconds on the largest grids)
  long max_cells = 0;
  for (int k = 0; k < c->B.n; ++k) max_cells = std::max(max_cells, (long)c->B.R[k].p.nx * c->B.R[k].p.ny);
  for (Cand& cd : cands) {
    const bool learned = c->guess == CDI_GUESS_LEARNED && c->net;
    if (cd.launch != CDI_LAUNCH_TILED && learned) continue;
    if (cd.launch == CDI_LAUNCH_PERSISTENT && (max_cells > kPersistTuneCells || c->dyn_gamma))
      continue;
    if (cd.launch != CDI_LAUNCH_TILED) {   // the fastest tiled shape
      cd.rows = c->wide_rows_pick;
      cd.coarse = c->coarse_cells_pick;
      cd.nu = c->nu_pick;
    }
    if ((st = apply_shape(c, cd.rows, cd.coarse, cd.nu)) != CDI_OK) break;
    c->launch = cd.launch;
    // warm-up: code load, iteration predictor; the graph form captures its
    // step once the pressure history exists
    cdi_status r = cdi_step(c, cd.launch == CDI_LAUNCH_GRAPH ? 3 : 1);
    if (r == CDI_OK || r == CDI_ERR_NOCONV) {
      HIPCHK(hipEventRecord(c->ev0, c->stream));
      r = cdi_step(c, trial_steps);
      HIPCHK(hipEventRecord(c->ev1, c->stream));
      HIPCHK(hipEventSynchronize(c->ev1));
    }
    if (r != CDI_OK && r != CDI_ERR_NOCONV) { st = r; break; }
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    const double per = ms / trial_steps;
    info.ms_per_step[cd.slot] = per;
    info.ncand += 1;
    if (per < best) { best = per; pick = cd; }
    if (cd.launch == CDI_LAUNCH_TILED && per < best_tiled) {
      best_tiled = per;
      c->wide_rows_pick = cd.rows;
      c->coarse_cells_pick = cd.coarse;
      c->nu_pick = cd.nu;
    }
    // back to the saved state for the next candidate
    cdi_status rs = tune_copy(c, sc, false);
    if (rs != CDI_OK) return rs;
    snap.rewind(c);
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  snap.restore(c);
  if (st != CDI_OK) {
    (void)tune_copy(c, sc, false);
    (void)hipStreamSynchronize(c->stream);
    return st;
  }
  if ((st = apply_shape(c, pick.rows, pick.coarse, pick.nu)) != CDI_OK) return st;
  c->launch = pick.launch;
  info.launch = pick.launch;
  info.tile_rows = pick.rows;
  info.coarse_cells = (int32_t)pick.coarse;
  info.mg_smooth = pick.nu;
  if (out) *out = info;
  return CDI_OK;
}

cdi_status cdi_tune_concurrent(cdi_ctx* const* ctxs, int32_t n, int32_t trial_steps,
                               void* const* scratch, const size_t* scratch_bytes,
                               cdi_tune_info* out) {
  if (!ctxs || n < 1 || !scratch || !scratch_bytes) return fail(CDI_ERR_ARG, "NULL argument or n < 1");
  if (trial_steps < 1) return fail(CDI_ERR_ARG, "trial_steps must be >= 1");
  for (int k = 0; k < n; ++k) {
    if (!ctxs[k] || !scratch[k]) return fail(CDI_ERR_ARG, "ctxs[%d] or scratch[%d] is NULL", k, k);
    for (int m = 0; m < k; ++m)
      if (ctxs[m] == ctxs[k]) return fail(CDI_ERR_ARG, "ctxs[%d] repeats ctxs[%d]", k, m);
    if (scratch_bytes[k] < tune_bytes(ctxs[k]))
      return fail(CDI_ERR_ARG, "scratch[%d] too small: %zu < %zu bytes", k, scratch_bytes[k],
                  tune_bytes(ctxs[k]));
  }
  auto sync_all = [&]() -> cdi_status {
    for (int k = 0; k < n; ++k) HIPCHK(hipStreamSynchronize(ctxs[k]->stream));
    return CDI_OK;
  };
  cdi_status st = sync_all();
  if (st != CDI_OK) return st;
  std::vector<HostSnap> snaps;
  snaps.reserve(n);
  for (int k = 0; k < n; ++k) {
    if ((st = tune_copy(ctxs[k], (char*)scratch[k], true)) != CDI_OK) return st;
    snaps.emplace_back(ctxs[k]);
    ctxs[k]->timed.clear();
  }
  cdi_tune_info info{};
  for (int q = 0; q < 14; ++q) info.ms_per_step[q] = -1.0;
  double best = INFINITY;
  int pick_rows = ctxs[0]->wide_rows, pick_nu = ctxs[0]->nu;
  long pick_coarse = ctxs[0]->coarse_cells;
  for (int v = 0; v < 2 && st == CDI_OK; ++v)
    for (int r = 0; r < 2 && st == CDI_OK; ++r)
      for (int q = 0; q < 3 && st == CDI_OK; ++q) {
        const int rows = kWideRows[r], nu = v + 1;
        const long coarse = kTuneCoarse[q];
        for (int k = 0; k < n && st == CDI_OK; ++k) {
          st = apply_shape(ctxs[k], rows, coarse, nu);
          ctxs[k]->launch = CDI_LAUNCH_TILED;
        }
        if (st != CDI_OK) break;
        // warm-up step (code load, iteration predictor), then the timed steps
        cdi_status r1 = cdi_step_concurrent(ctxs, n, 1);
        if (r1 != CDI_OK && r1 != CDI_ERR_NOCONV) { st = r1; break; }
        if ((st = sync_all()) != CDI_OK) break;
        const auto t0 = std::chrono::steady_clock::now();
        r1 = cdi_step_concurrent(ctxs, n, trial_steps);
        if (r1 != CDI_OK && r1 != CDI_ERR_NOCONV) { st = r1; break; }
        if ((st = sync_all()) != CDI_OK) break;
        const double per =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() /
            trial_steps;
        info.ms_per_step[v * 6 + r * 3 + q] = per;
        info.ncand += 1;
        if (per < best) { best = per; pick_rows = rows; pick_coarse = coarse; pick_nu = nu; }
        for (int k = 0; k < n && st == CDI_OK; ++k) {
          st = tune_copy(ctxs[k], (char*)scratch[k], false);
          snaps[k].rewind(ctxs[k]);
        }
      }
  // then the stage kernel's strip height with that shape: the block-count
  // rule that picks it for a context alone does not see the other contexts
  // sharing the GPU
  std::vector<int> strip0(n);
  for (int k = 0; k < n; ++k) strip0[k] = ctxs[k]->B.strip_rows;
  int pick_strip = -1;
  for (int k = 0; k < n && st == CDI_OK; ++k) st = apply_shape(ctxs[k], pick_rows, pick_coarse, pick_nu);
  for (int si = 0; si < 3 && st == CDI_OK; ++si) {
    const int rows = kStripRows[si];
    for (int k = 0; k < n && st == CDI_OK; ++k) st = apply_strip_rows(ctxs[k], rows);
    if (st != CDI_OK) break;
    cdi_status r1 = cdi_step_concurrent(ctxs, n, 1);
    if (r1 != CDI_OK && r1 != CDI_ERR_NOCONV) { st = r1; break; }
    if ((st = sync_all()) != CDI_OK) break;
    const auto t0 = std::chrono::steady_clock::now();
    r1 = cdi_step_concurrent(ctxs, n, trial_steps);
    if (r1 != CDI_OK && r1 != CDI_ERR_NOCONV) { st = r1; break; }
    if ((st = sync_all()) != CDI_OK) break;
    const double per =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() /
        trial_steps;
    info.ncand += 1;
    if (pick_strip < 0 || per < best) { best = per; pick_strip = rows; }
    for (int k = 0; k < n && st == CDI_OK; ++k) {
      st = tune_copy(ctxs[k], (char*)scratch[k], false);
      snaps[k].rewind(ctxs[k]);
    }
  }
  for (int k = 0; k < n; ++k) {
    if (st != CDI_OK) {
      (void)tune_copy(ctxs[k], (char*)scratch[k], false);
      (void)apply_strip_rows(ctxs[k], strip0[k]);
    }
    snaps[k].restore(ctxs[k]);
  }
  cdi_status ss = sync_all();
  if (st != CDI_OK) return st;
  if (ss != CDI_OK) return ss;
  for (int k = 0; k < n; ++k) {
    if ((st = apply_shape(ctxs[k], pick_rows, pick_coarse, pick_nu)) != CDI_OK) return st;
    if ((st = apply_strip_rows(ctxs[k], pick_strip)) != CDI_OK) return st;
    ctxs[k]->launch = CDI_LAUNCH_TILED;
  }
  info.launch = CDI_LAUNCH_TILED;
  info.tile_rows = pick_rows;
  info.coarse_cells = (int32_t)pick_coarse;
  info.mg_smooth = pick_nu;
  info.strip_rows = pick_strip;
  if (out) *out = info;
  return CDI_OK;
}

cdi_status cdi_set_launch(cdi_ctx* c, int32_t mode) {
  if (!c) return fail(CDI_ERR_ARG, "ctx is NULL");
  if (mode != CDI_LAUNCH_TILED && mode != CDI_LAUNCH_PERSISTENT && mode != CDI_LAUNCH_GRAPH)
    return fail(CDI_ERR_ARG, "bad launch mode %d", mode);
  if (mode == CDI_LAUNCH_PERSISTENT && c->dyn_gamma)
    return fail(CDI_ERR_ARG, "the persistent launch keeps gamma fixed (gamma_factor > 0)");
  c->launch = mode;
  return CDI_OK;
}

cdi_status cdi_graph_stats(cdi_ctx* c, int64_t* replays, int64_t* redone, int32_t* budget) {
  if (!c || !replays || !redone || !budget) return fail(CDI_ERR_ARG, "NULL argument");
  *replays = c->graph_replays;
  *redone = c->graph_misses;
  *budget = c->graph_budget;
  return CDI_OK;
}

cdi_status cdi_get_launch(cdi_ctx* c, int32_t* mode) {
  if (!c || !mode) return fail(CDI_ERR_ARG, "NULL argument");
  *mode = c->launch;
  return CDI_OK;
}

cdi_status cdi_set_guess(cdi_ctx* c, int32_t guess) {
  if (!c) return fail(CDI_ERR_ARG, "ctx is NULL");
  if (guess < CDI_GUESS_ZERO || guess > CDI_GUESS_LEARNED) return fail(CDI_ERR_ARG, "bad guess");
  if (guess != c->guess) graph_drop(c);   // the captured step holds the guess mode
  c->guess = guess;
  return CDI_OK;
}

cdi_status cdi_guess_attach(cdi_ctx* c, cdi_net* net) {
  if (!c) return fail(CDI_ERR_ARG, "ctx is NULL");
  if (!net) { c->net = nullptr; return CDI_OK; }
  if (c->B.n != 1) return fail(CDI_ERR_STATE, "the learned guess needs a single-instance context");
  const Inst& I = c->B.inst[0];
  if (cdinet::batch(net) != 1 || cdinet::height(net) != I.ny || cdinet::width(net) != I.nx)
    return fail(CDI_ERR_SHAPE, "network shape must be batch 1, h = ny, w = nx");
  if (cdinet::stream_of(net) != c->stream) return fail(CDI_ERR_ARG, "network and context must share the stream");
  c->net = net;
  return CDI_OK;
}

cdi_status cdi_guess_features(cdi_ctx* c, int32_t idx, float* features, float* target) {
  if (!c || !features) return fail(CDI_ERR_ARG, "NULL argument");
  if (idx < 0 || idx >= c->B.n) return fail(CDI_ERR_ARG, "instance out of range");
  const Inst& I = c->B.inst[idx];
  const unsigned g = (unsigned)std::min(1024, ceil_div(I.nx * I.ny, kNT));
  k_features<<<g, kNT, 0, c->stream>>>(c->d_inst, idx, I.phi, I.p, features, target);
  if (target) k_target_unit_rms<<<1, kNT, 0, c->stream>>>(target, (size_t)I.nx * I.ny);
  HIPCHK(hipGetLastError());
  return CDI_OK;
}

void cdi_destroy(cdi_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  graph_drop(c);
  if (c->gstream) {
    (void)hipStreamSynchronize(c->gstream);
    (void)hipStreamDestroy(c->gstream);
  }
  if (c->gev0) (void)hipEventDestroy(c->gev0);
  if (c->gev1) (void)hipEventDestroy(c->gev1);
  if (c->h_pcg) (void)hipHostFree(c->h_pcg);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  for (auto e : c->tev) if (e) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"

// ============================================== allocation-free stage operator
// cdi_eval_rhs_noalloc: the stage operator of cdi_eval_rhs with its scratch
// (instance descriptor, tile list, CG scalars, reduction partials and
// counters) in a file-scope device array instead of a caller workspace, and
// no context.  The stage kernel (strip kernel in FP64, tile kernel in mixed
// precision) forms n, mu_c and the wall extrapolations in LDS.
namespace {

constexpr int kMaxDevices = 64;

// Scratch layout of one call (offsets in bytes from the array's device
// address); with base == nullptr only the size is computed.
struct NoAllocLayout {
  size_t inst, pcg, counters, part, tiles, uY, uslip, total;
};

NoAllocLayout noalloc_layout(const Resolved& R) {
  const size_t nt = (size_t)cell_tiles(R);
  NoAllocLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = align256(off + bytes); return o; };
  L.inst = take(sizeof(Inst));
  L.pcg = take(sizeof(PcgScalars));
  L.counters = take(sizeof(unsigned) * 8 * kCounterStride);
  L.part = take(sizeof(double) * 8 * nt);
  L.tiles = take(sizeof(Tile) * (nt + (size_t)strip_tiles(R, kStripRows[2])));
  L.uY = take(sizeof(double) * 2 * (size_t)R.p.nx);
  L.uslip = take(sizeof(double) * 2 * (size_t)R.p.nx);
  L.total = off;
  return L;
}

std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

}  // namespace

// The scratch array.  Host code never passes this name to a kernel or a copy:
// it uses the device address that hipGetSymbolAddress returns for the
// current device (each GPU holds its own copy of the array).
static __device__ __align__(256) char scratch[CDI_NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of `scratch` on the current device, looked up once per device.
cdi_status scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(CDI_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(CDI_ERR_DEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(CDI_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return CDI_OK;
}

// One launch that prepares a call in the scratch: the instance descriptor
// (passed by value), its CG scalars' regularisation velocity, the level-0
// cell tile list followed by the strip list of the stage kernel, cleared
// arrival counters (their reductions start from zero), and the two wall rows
// of L_my, which the stage kernel leaves alone.
__global__ void k_noalloc_setup(Inst I, Inst* __restrict__ dst, Tile* __restrict__ tiles,
                                int ntx, int ntiles, int ntxs, int nstrips, int srows,
                                unsigned* __restrict__ counters,
                                int ncounters, double* __restrict__ l_my) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g == 0) {
    *dst = I;
    I.pcg->gamma_step = I.gamma;
  }
  if (g < ntiles) tiles[g] = Tile{0, (g % ntx) * TX, (g / ntx) * TY, 0, g, 0, nullptr};
  if (g < nstrips)
    tiles[ntiles + g] = Tile{0, (g % ntxs) * sr::TW, (g / ntxs) * srows, 0, g, 0, nullptr};
  if (g < ncounters) counters[g] = 0u;
  if (g < I.nx) {
    l_my[g] = 0.0;
    l_my[(size_t)I.ny * I.nx + g] = 0.0;
  }
}

}  // namespace

extern "C" {

cdi_status cdi_eval_rhs_noalloc(const cdi_params* params, const cdi_fields* fields,
                                double* l_phi, double* l_mx, double* l_my, double* u_y,
                                double* u_slip, void* hip_stream) {
  Resolved R;
  cdi_status s = resolve(params, R);
  if (s != CDI_OK) return s;
  if (!fields || !fields->phi || !fields->u || !fields->v)
    return fail(CDI_ERR_ARG, "fields (phi, u, v) must be non-NULL");
  if (!l_phi || !l_mx || !l_my) return fail(CDI_ERR_ARG, "output pointer is NULL");
  const NoAllocLayout Lo = noalloc_layout(R);
  if (Lo.total > (size_t)CDI_NOALLOC_SCRATCH_BYTES)
    return fail(CDI_ERR_SHAPE,
                "grid %dx%d needs %zu bytes of scratch, more than the %zu bytes of the "
                "allocation-free entry point", R.p.nx, R.p.ny, Lo.total,
                (size_t)CDI_NOALLOC_SCRATCH_BYTES);
  void* base_v = nullptr;
  s = scratch_address(&base_v);
  if (s != CDI_OK) return s;
  char* base = (char*)base_v;
  hipStream_t st = (hipStream_t)hip_stream;
  Inst I{};
  fill_inst(R, *fields, I);
  const int ntx = ceil_div(R.p.nx, TX), ntiles = cell_tiles(R);
  const int srows = strip_rows({R});
  const int ntxs = ceil_div(R.p.nx, sr::TW), nstrips = strip_tiles(R, srows);
  I.first_tile = 0;
  I.ntiles = ntiles;
  I.pcg = (PcgScalars*)(base + Lo.pcg);
  I.counters = (unsigned*)(base + Lo.counters);
  I.part = (double*)(base + Lo.part);
  I.uY = u_y ? u_y : (double*)(base + Lo.uY);
  I.uslip = u_slip ? u_slip : (double*)(base + Lo.uslip);
  I.acc_phi = l_phi;
  I.acc_mx = l_mx;
  I.acc_my = l_my;
  Inst* d_inst = (Inst*)(base + Lo.inst);
  Tile* d_tiles = (Tile*)(base + Lo.tiles);
  const int ncount = 8 * kCounterStride;
  const int nset = std::max(std::max(std::max(ntiles, nstrips), ncount), R.p.nx);
  k_noalloc_setup<<<(unsigned)ceil_div(nset, kNT), kNT, 0, st>>>(
      I, d_inst, d_tiles, ntx, ntiles, ntxs, nstrips, srows, I.counters, ncount, l_my);
  if (R.p.gamma_factor > 0)
    k_gamma_step<<<(unsigned)ntiles, kNT, 0, st>>>(d_tiles, d_inst);
  if (R.p.precision == CDI_MIXED)
    k_stage_fused<float><<<(unsigned)ntiles, kNT, 0, st>>>(d_tiles, d_inst, -1, 0, 0, 0.0, 0.0, 1);
  else
    k_stage_strip<double><<<(unsigned)nstrips, kNT, 0, st>>>(d_tiles + ntiles, d_inst, -1, 0, 0,
                                                              0.0, 0.0, 1, srows);
  HIPCHK(hipGetLastError());
  return CDI_OK;
}

}  // extern "C"
