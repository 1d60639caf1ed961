// Stage kernels of the CDI + GNBC step: phase-field preparation, the fused
// CDI-flux / momentum / surface-tension / GNBC stage operator with its RK4
// update, the projection right-hand side and the projection itself.
//
// S is the stencil precision (double on the FP64 path, float on the mixed
// path).  The phase field, its RK accumulation, the flux differences of the
// phi update and every reduction stay in FP64 on both paths.
#pragma once
#include <type_traits>

#include "cdi_dev.h"

namespace cdi {

// tile of the cell kernels: TX x TY cells, one cell per thread
constexpr int TX = 64, TY = 4;
static_assert(TX * TY == kNT, "cell tile must match the block size");
// wide tile of the pointwise / 5-point CG kernels: TX x (WR * TY) cells, WR
// rows per thread (fewer blocks, fewer per-block reductions and shorter
// halos on large grids; WR = 1 keeps more, shorter blocks for small ones)
constexpr int kWideRows[2] = {1, 4};
__device__ __forceinline__ int wide_tx() { return threadIdx.x % TX; }
__device__ __forceinline__ int wide_ty(int r) { return threadIdx.x / TX + r * TY; }

// ---------------------------------------------------------------- wall GNBC
// Contact-line slip u^Y at wall corner i (Sec. 2 eq. u_slip_Y; Sec. 3 Models
// 1A..4B).  Wall quantities are linear extrapolations per column (Sec. 4)
// averaged to the corner; n points into the fluid, tau = +x on both walls.
// W: the wall's 5 quantities, quantity q of column c at W[q * ws + c]; the
// corner lies between columns im (west) and i (east).
__device__ __forceinline__ double slip_uY_w(const Inst& I, const double* W, int ws, int wall,
                                            int im, int i, double& phc_out, double& beta_out) {
  const double sgn = wall == 0 ? 1.0 : -1.0;
  double phc = 0.5 * (W[im] + W[i]);
  phc = fmin(fmax(phc, 0.0), 1.0);
  const double psc = 0.5 * (W[ws + im] + W[ws + i]);
  const double dpn = sgn * 0.5 * (W[2 * ws + im] + W[2 * ws + i]);
  const double kac = 0.5 * (W[3 * ws + im] + W[3 * ws + i]);
  const double dphn = sgn * 0.5 * (W[4 * ws + im] + W[4 * ws + i]);
  const double dpt = (W[ws + i] - W[ws + im]) * I.inv_h;
  const double dpht = (W[i] - W[im]) * I.inv_h;
  const double g = phc * (1.0 - phc);
  const double beta = I.beta2 + (I.beta1 - I.beta2) * phc;
  const double ce = I.cos_eq;
  const double corr = 1.0 + kac * psc;
  const double pre = -6.0 * I.sigma / beta;
  const double eps = I.eps;
  double uY;
  switch (I.slip_model) {
    case 0:  uY = pre * (eps * dphn + g * ce) * dpht; break;                                   // 1A
    case 1:  uY = pre * (eps * dphn + eps * sqrt(dphn * dphn + dpht * dpht) * ce) * dpht; break; // 1B
    case 2:  uY = pre * (g * dpn + g * ce) * g / eps * dpt; break;                             // 2A
    case 3:  uY = pre * (g * dpn + g * sqrt(dpn * dpn + dpt * dpt) * ce) * g / eps * dpt; break; // 2B
    case 4:  uY = pre * (eps * dphn + g * corr * ce) * dpht; break;                            // 3A
    case 5:  uY = pre * (eps * dphn + eps * sqrt(dphn * dphn + dpht * dpht) * corr * ce) * dpht; break; // 3B
    case 7:  uY = pre * (g * dpn + g * sqrt(dpn * dpn + dpt * dpt) * corr * ce) * g / eps * dpt; break; // 4B
    default: uY = pre * (g * dpn + g * corr * ce) * g / eps * dpt; break;                     // 4A
  }
  phc_out = phc;
  beta_out = beta;
  return uY;
}

// u^Y at wall corner i from the instance's wall arrays (I.wall).
__device__ __forceinline__ double slip_uY(const Inst& I, int wall, int i, double& phc_out,
                                          double& beta_out) {
  const int nx = I.nx;
  return slip_uY_w(I, I.wall + (size_t)wall * 5 * nx, nx, wall, wrap(i - 1, nx), i, phc_out,
                   beta_out);
}

// Robin form of the slip condition: u_wall - U = (mu/beta) du/dn + u^Y with
// du/dn = 2 (u_row - u_wall)/h along the inward normal.  Returns the wall
// shear stress mu du/dy at the corner between wall columns im and i of W
// (layout of slip_uY_w).
__device__ __forceinline__ double gnbc_corner_w(const Inst& I, const double* W, int ws, int wall,
                                                int im, int i, double urow, double& uY,
                                                double& uslip) {
  double phc, beta;
  uY = slip_uY_w(I, W, ws, wall, im, i, phc, beta);
  const double U = wall == 0 ? I.uw_bot : I.uw_top;
  const double muw = I.mu2 + (I.mu1 - I.mu2) * phc;
  const double lam = 2.0 * muw / (beta * I.h);
  const double uw = (U + uY + lam * urow) / (1.0 + lam);
  uslip = uw - U;
  return wall == 0 ? 2.0 * muw * (urow - uw) * I.inv_h : 2.0 * muw * (uw - urow) * I.inv_h;
}

__device__ __forceinline__ double gnbc_corner(const Inst& I, int wall, int i, double urow,
                                              double& uY, double& uslip) {
  const int nx = I.nx;
  return gnbc_corner_w(I, I.wall + (size_t)wall * 5 * nx, nx, wall, wrap(i - 1, nx), i, urow, uY,
                       uslip);
}

// Stencil views of an LDS region: at(dr, dc) is the value dr rows above and
// dc columns right of the centre cell.  FlatView: a region of row pitch RX;
// RingView: rows j-3..j+3 of a ring of row buffers (row offsets per row).
template <typename T, int RX>
struct FlatView {
  const T* c;
  __device__ __forceinline__ T at(int dr, int dc) const { return c[dr * RX + dc]; }
};
template <typename T>
struct RingView {
  const T* base;
  int off[7];
  __device__ __forceinline__ T at(int dr, int dc) const { return base[off[dr + 3] + dc]; }
};

// ------------------------------------------------------------ phase prep
// n = G/(|G| + dN), psi, kappa, mu_c (Sec. 2, eqs. CDI, psi, curvature,
// chemical potential) with one-sided rows at the walls (Sec. 4); the wall
// rows also publish the extrapolated wall quantities of the slip models.
// src: 0 caller phi, 1 phi_a, 2 phi_b.
constexpr int PRY = TY + 6, PRX = TX + 2;   // rows j0-3 .. j0+TY+2, cols i0-1 .. i0+TX
// LDS of one phase-preparation tile of TX x (WR * TY) cells
template <typename S, int WR = 1>
struct PrepLds {
  double phi[(WR * TY + 6) * PRX];
  S psi[(WR * TY + 6) * PRX];
};

// n = G/(|G| + dN) and mu_c at the centre cell of the views (grid row j) from
// the FP64 phase field P and psi Q (one-sided rows at the walls, Sec. 4).
// INTERIOR: the caller guarantees 0 < j < ny - 1 (central rows only).
template <typename S, bool INTERIOR = false, typename VP, typename VQ>
__device__ __forceinline__ void prep_point_v(const Inst& I, const VP& P, const VQ& Q, int j,
                                             S& onx, S& ony, S& omu) {
  const int ny = I.ny;
  const bool bot = !INTERIOR && j == 0, top = !INTERIOR && j == ny - 1;
  const S inv2h = (S)(0.5 * I.inv_h), inv_h2 = (S)(I.inv_h * I.inv_h);
  // normal from phi
  const S gx = ((S)P.at(0, 1) - (S)P.at(0, -1)) * inv2h;
  S gy;
  if (bot) gy = (S(-3) * (S)P.at(0, 0) + S(4) * (S)P.at(1, 0) - (S)P.at(2, 0)) * inv2h;
  else if (top) gy = (S(3) * (S)P.at(0, 0) - S(4) * (S)P.at(-1, 0) + (S)P.at(-2, 0)) * inv2h;
  else gy = ((S)P.at(1, 0) - (S)P.at(-1, 0)) * inv2h;
  const S mag = sqrt(gx * gx + gy * gy) + (S)kDeltaN;
  // psi derivatives, curvature, chemical potential
  const S q0 = Q.at(0, 0), qe = Q.at(0, 1), qw = Q.at(0, -1);
  const S px = (qe - qw) * inv2h;
  S py, d2y;
  if (bot) {
    py = (S(-3) * q0 + S(4) * Q.at(1, 0) - Q.at(2, 0)) * inv2h;
    d2y = (S(2) * q0 - S(5) * Q.at(1, 0) + S(4) * Q.at(2, 0) - Q.at(3, 0)) * inv_h2;
  } else if (top) {
    py = (S(3) * q0 - S(4) * Q.at(-1, 0) + Q.at(-2, 0)) * inv2h;
    d2y = (S(2) * q0 - S(5) * Q.at(-1, 0) + S(4) * Q.at(-2, 0) - Q.at(-3, 0)) * inv_h2;
  } else {
    py = (Q.at(1, 0) - Q.at(-1, 0)) * inv2h;
    d2y = (Q.at(1, 0) - S(2) * q0 + Q.at(-1, 0)) * inv_h2;
  }
  const S lap = (qe - S(2) * q0 + qw) * inv_h2 + d2y;
  const S ph = (S)P.at(0, 0);
  const S g = ph * (S(1) - ph);
  const S grad2 = px * px + py * py;
  const S rmag = S(1) / mag;
  onx = gx * rmag;
  ony = gy * rmag;
  omu = S(6) * (S)I.sigma * (g * (S(1) - S(2) * ph) * (S(1) - grad2) * (S)I.inv_eps - g * lap);
}

// prep_point_v on a flat LDS region of row pitch RX, centre cell index c.
template <typename S, int RX>
__device__ __forceinline__ void prep_point(const Inst& I, const double* s_phi, const S* s_psi,
                                           int c, int j, S& onx, S& ony, S& omu) {
  prep_point_v<S>(I, FlatView<double, RX>{s_phi + c}, FlatView<S, RX>{s_psi + c}, j, onx, ony,
                  omu);
}

// Wall quantities of the slip models for the column of a wall-row cell (the
// centre of the views, grid row j = 0 or ny - 1): phi, psi, d psi/dy, kappa
// and d phi/dy of the wall row and the next row, linearly extrapolated to the
// wall per column (Sec. 4), in FP64.
template <typename S, typename VP, typename VQ>
__device__ __forceinline__ void prep_wall_v(const Inst& I, const VP& P, const VQ& Q, int j,
                                            double out[5]) {
  const int ny = I.ny;
  const int dj = j == 0 ? 1 : -1;          // second cell row from the wall
  double vals[2][5];
  for (int r = 0; r < 2; ++r) {
    const int o = r == 0 ? 0 : dj, jj = j + o;   // row offset of this cell from the centre
    const double i2h = 0.5 * I.inv_h, ih2 = I.inv_h * I.inv_h;
    const double p0 = (double)Q.at(o, 0);
    double pyd, d2y;
    if (jj == 0) {
      pyd = (-3.0 * p0 + 4.0 * (double)Q.at(o + 1, 0) - (double)Q.at(o + 2, 0)) * i2h;
      d2y = (2.0 * p0 - 5.0 * (double)Q.at(o + 1, 0) + 4.0 * (double)Q.at(o + 2, 0) -
             (double)Q.at(o + 3, 0)) * ih2;
    } else if (jj == ny - 1) {
      pyd = (3.0 * p0 - 4.0 * (double)Q.at(o - 1, 0) + (double)Q.at(o - 2, 0)) * i2h;
      d2y = (2.0 * p0 - 5.0 * (double)Q.at(o - 1, 0) + 4.0 * (double)Q.at(o - 2, 0) -
             (double)Q.at(o - 3, 0)) * ih2;
    } else {
      pyd = ((double)Q.at(o + 1, 0) - (double)Q.at(o - 1, 0)) * i2h;
      d2y = ((double)Q.at(o + 1, 0) - 2.0 * p0 + (double)Q.at(o - 1, 0)) * ih2;
    }
    const double pxd = ((double)Q.at(o, 1) - (double)Q.at(o, -1)) * i2h;
    const double lapd = ((double)Q.at(o, 1) - 2.0 * p0 + (double)Q.at(o, -1)) * ih2 + d2y;
    const double phd = P.at(o, 0);
    const double kap = (1.0 - 2.0 * phd) * (1.0 - pxd * pxd - pyd * pyd) / I.eps - lapd;
    double phy;
    if (jj == 0) phy = (-3.0 * phd + 4.0 * P.at(o + 1, 0) - P.at(o + 2, 0)) * i2h;
    else if (jj == ny - 1) phy = (3.0 * phd - 4.0 * P.at(o - 1, 0) + P.at(o - 2, 0)) * i2h;
    else phy = (P.at(o + 1, 0) - P.at(o - 1, 0)) * i2h;
    vals[r][0] = phd; vals[r][1] = p0; vals[r][2] = pyd; vals[r][3] = kap; vals[r][4] = phy;
  }
  for (int qk = 0; qk < 5; ++qk) out[qk] = 0.5 * (3.0 * vals[0][qk] - vals[1][qk]);
}

template <typename S, int RX>
__device__ __forceinline__ void prep_wall(const Inst& I, const double* s_phi, const S* s_psi,
                                          int c, int j, double out[5]) {
  prep_wall_v<S>(I, FlatView<double, RX>{s_phi + c}, FlatView<S, RX>{s_psi + c}, j, out);
}

// Cell (ty, tx) of a phase-preparation tile whose LDS region has RY rows.
template <typename S, int RY>
__device__ __forceinline__ void phase_prep_cell(const Tile& t, const Inst& I,
                                                const double* s_phi, const S* s_psi, int tx,
                                                int ty) {
  constexpr int RX = PRX;
  const int nx = I.nx, ny = I.ny;
  const int i = t.i0 + tx, j = t.j0 + ty;
  if (i >= nx || j >= ny) return;
  const int c = (ty + 3) * RX + (tx + 1);
  S vnx, vny, vmu;
  prep_point<S, RX>(I, s_phi, s_psi, c, j, vnx, vny, vmu);
  const size_t o = (size_t)j * nx + i;
  (gas<S>(I.nhx))[o] = vnx;
  (gas<S>(I.nhy))[o] = vny;
  (gas<S>(I.muc))[o] = vmu;
  // wall rows: extrapolate phi, psi, d psi/dy, kappa, d phi/dy to the wall (per column)
  if (j == 0 || j == ny - 1) {
    double w[5];
    prep_wall<S, RX>(I, s_phi, s_psi, c, j, w);
    double* W = I.wall + (size_t)(j == 0 ? 0 : 1) * 5 * nx;
    for (int qk = 0; qk < 5; ++qk) W[qk * nx + i] = w[qk];
  }
}

// One tile of the phase preparation (TX x WR*TY cells, WR rows per thread),
// run by kNT threads (tid in [0, kNT)).  Contains one block barrier: every
// thread of the block calls it, with active = false for threads that have no
// tile in this pass over the tiles.
template <typename S, int WR = 1>
__device__ __forceinline__ void phase_prep_tile(const Tile& t, const Inst& I, int src,
                                                PrepLds<S, WR>& L, int tid, bool active) {
  constexpr int RY = WR * TY + 6, RX = PRX;
  constexpr int NPT = (RY * RX + kNT - 1) / kNT;
  double* s_phi = L.phi;
  S* s_psi = L.psi;
  const int nx = I.nx, ny = I.ny;
  const double* __restrict__ phi = src == 0 ? I.phi : (src == 1 ? I.phi_a : I.phi_b);
  // every load of the thread's region cells first, then psi from FP64 phi
  double fv[NPT];
#pragma unroll
  for (int e = 0; e < NPT; ++e) {
    const int k = tid + e * kNT;
    const int rj = k / RX, ri = k - rj * RX;
    const int j = t.j0 - 3 + rj;
    fv[e] = 0.0;
    if (active && k < RY * RX && j >= 0 && j < ny)
      fv[e] = phi[(size_t)j * nx + wrap_any(t.i0 - 1 + ri, nx)];
  }
#pragma unroll
  for (int e = 0; e < NPT; ++e) {
    const int k = tid + e * kNT;
    if (!active || k >= RY * RX) continue;
    const int j = t.j0 - 3 + k / RX;
    double ps = 0.0;
    if (j >= 0 && j < ny) {
      const double c = fmin(fmax(fv[e], 0.0), 1.0);
      ps = I.eps * cdi_log((c + kDeltaPsi) / (1.0 - c + kDeltaPsi));
    }
    s_phi[k] = fv[e];
    s_psi[k] = (S)ps;
  }
  __syncthreads();
  if (!active) return;
#pragma unroll
  for (int row = 0; row < WR; ++row)
    phase_prep_cell<S, RY>(t, I, s_phi, s_psi, tid % TX, tid / TX + row * TY);
}

template <typename S, int WR>
__global__ void __launch_bounds__(kNT) k_phase_prep(const Tile* __restrict__ tiles,
                                                     const Inst* __restrict__ insts, int src) {
  __shared__ PrepLds<S, WR> L;
  const Tile t = tiles[blockIdx.x];
  phase_prep_tile<S, WR>(t, insts[t.inst], src, L, threadIdx.x, true);
}



// ------------------------------------------------------------ stage operator
// One RK4 stage: CDI face fluxes F = u phi_f - gamma[eps dphi/h - phi_f(1-phi_f) n_f]
// (eq. CDI; wall y-faces F = 0 by the no-flux and no-penetration BCs), the
// phase-field right-hand side -div F accumulated in FP64, the mass flux
// m = rho2 u + (rho1-rho2) F (consistent transport, eq. NS_momentum), the
// momentum right-hand side (advection of m u, variable-viscosity stress with
// the GNBC wall stress, EB surface tension mu_c grad phi at the faces), then
// the RK4 combination and the stage (rho u)*.
//
// k: stage index 0..3 (k < 0: evaluate the operator only); src/dst:
// phase-field buffers (0 caller, 1 phi_a, 2 phi_b); c_next = RK c_{k+1}
// (multiplied by each instance's dt), b_k the RK4 weight of stage k.
namespace st {
constexpr int CY = TY + 3, CX = TX + 3;   // cells: rows j0-2..j0+TY, cols i0-2..i0+TX
constexpr int UY = TY + 2, UX = TX + 2;   // u/v: rows j0-1..j0+TY, cols i0-1..i0+TX
constexpr int XY = TY + 1, XX = TX + 2;   // x-faces: rows j0-1..j0+TY-1, cols i0-1..i0+TX
constexpr int YY = TY + 2, YX = TX + 1;   // y-faces: rows j0-1..j0+TY, cols i0-1..i0+TX-1
constexpr int CRY = TY + 1, CRX = TX + 1; // corners: rows j0..j0+TY, cols i0..i0+TX
constexpr int PY = TY + 5, PX = TX + 5;   // fused prep: phi rows j0-3..j0+TY+1, cols i0-3..i0+TX+1
constexpr int WX = TX + 2;                // fused prep: wall columns i0-1..i0+TX
}  // namespace st

template <typename S>
struct StageLds {
  S phi[st::CY * st::CX], nx[st::CY * st::CX], ny[st::CY * st::CX], mc[st::CY * st::CX];
  S u[st::UY * st::UX], v[st::UY * st::UX];
  union {
    struct {
      S fx[st::XY * st::XX], mx[st::XY * st::XX];
      S fy[st::YY * st::YX], my[st::YY * st::YX];
      S txy[st::CRY * st::CRX];
    } f;
    // fused phase preparation: the FP64 phase field and psi of the region
    // the tile's n and mu_c need, dead once those are formed
    struct {
      double phi[st::PY * st::PX];
      S psi[st::PY * st::PX];
    } p;
  } x;
};

// One tile of the stage operator, run by kNT threads (tid in [0, kNT)).
// Contains two block barriers: every thread of the block calls it, with
// active = false for threads that have no tile in this pass over the tiles.
// Fused = true (tiled kernel k_stage_fused): n and mu_c of the tile and its
// halo, and the wall extrapolations of its columns, are formed here from the
// phase field (the arithmetic of the phase preparation, prep_point and
// prep_wall) instead of being read from the arrays k_phase_prep writes;
// s_wall holds the wall quantities (5 x WX doubles).
template <typename S, bool Fused = false>
__device__ __forceinline__ void stage_tile(const Tile& t, const Inst& I, int k, int src, int dst,
                                           double c_next, double b_k, int write_wall,
                                           StageLds<S>& L, int tid, bool active,
                                           double* s_wall = nullptr) {
  using namespace st;
  S* s_phi = L.phi; S* s_nx = L.nx; S* s_ny = L.ny; S* s_mc = L.mc;
  S* s_u = L.u; S* s_v = L.v;
  S* s_fx = L.x.f.fx; S* s_mx = L.x.f.mx;
  S* s_fy = L.x.f.fy; S* s_my = L.x.f.my;
  S* s_txy = L.x.f.txy;
  const int nx = I.nx, ny = I.ny;
  const int i0 = t.i0, j0 = t.j0;
  const CDI_GLOBAL double* __restrict__ phs = src == 0 ? I.phi : (src == 1 ? I.phi_a : I.phi_b);
  const CDI_GLOBAL double* __restrict__ us = k <= 0 ? I.u : I.us;
  const CDI_GLOBAL double* __restrict__ vs = k <= 0 ? I.v : I.vs;
  const S* __restrict__ gnx = gas<const S>(I.nhx);
  const S* __restrict__ gny = gas<const S>(I.nhy);
  const S* __restrict__ gmc = gas<const S>(I.muc);

  // operands of this thread's RK update, fetched now so that their latency
  // hides behind the LDS phases (own cell; west and south base densities)
  const int ctx = tid % TX, cty = tid / TX;
  const int ci = i0 + ctx, cj = j0 + cty;
  const bool own = active && ci < nx && cj < ny;
  const size_t co_ = own ? (size_t)cj * nx + ci : 0;
  double pre_acc[3] = {0.0, 0.0, 0.0}, pre_phn = 0.0, pre_phw = 0.0, pre_phs = 0.0;
  double pre_u = 0.0, pre_v = 0.0;
  if (own && k >= 0) {
    const double* __restrict__ phn0 = I.phi;
    if (k > 0) { pre_acc[0] = I.acc_phi[co_]; pre_acc[1] = I.acc_mx[co_]; pre_acc[2] = I.acc_my[co_]; }
    pre_phn = phn0[co_];
    pre_phw = phn0[(size_t)cj * nx + wrap(ci - 1, nx)];
    if (cj >= 1) pre_phs = phn0[co_ - nx];
    pre_u = I.u[co_];
    pre_v = I.v[co_];
  }
  // halo regions: every load of the thread first, then the LDS stores
  if constexpr (Fused) {
    // phase field of rows j0-3..j0+TY+1, columns i0-3..i0+TX+1 (FP64), psi
    // from it, then n and mu_c on the stage region and the wall quantities
    constexpr int NP = (PY * PX + kNT - 1) / kNT, NU = (UY * UX + kNT - 1) / kNT;
    double fv[NP];
    S vu[NU][2];
#pragma unroll
    for (int e = 0; e < NP; ++e) {
      const int q = tid + e * kNT;
      const int rj = q / PX, ri = q - rj * PX;
      const int j = j0 - 3 + rj;
      fv[e] = 0.0;
      if (active && q < PY * PX && j >= 0 && j < ny)
        fv[e] = phs[(size_t)j * nx + wrap_any(i0 - 3 + ri, nx)];
    }
#pragma unroll
    for (int e = 0; e < NU; ++e) {
      const int q = tid + e * kNT;
      const int rj = q / UX, ri = q - rj * UX;
      const int j = j0 - 1 + rj;
      vu[e][0] = vu[e][1] = S(0);
      if (active && q < UY * UX) {
        const size_t o = (size_t)j * nx + wrap_any(i0 - 1 + ri, nx);
        if (j >= 0 && j < ny) vu[e][0] = (S)us[o];
        if (j >= 0 && j <= ny) vu[e][1] = (S)vs[o];
      }
    }
    double* p_phi = L.x.p.phi;
    S* p_psi = L.x.p.psi;
#pragma unroll
    for (int e = 0; e < NP; ++e) {
      const int q = tid + e * kNT;
      if (!active || q >= PY * PX) continue;
      const int j = j0 - 3 + q / PX;
      double ps = 0.0;
      if (j >= 0 && j < ny) {
        const double cl = fmin(fmax(fv[e], 0.0), 1.0);
        ps = I.eps * cdi_log((cl + kDeltaPsi) / (1.0 - cl + kDeltaPsi));
      }
      p_phi[q] = fv[e];
      p_psi[q] = (S)ps;
    }
#pragma unroll
    for (int e = 0; e < NU; ++e) {
      const int q = tid + e * kNT;
      if (active && q < UY * UX) { s_u[q] = vu[e][0]; s_v[q] = vu[e][1]; }
    }
    __syncthreads();
    for (int q = tid; active && q < CY * CX; q += kNT) {
      const int rj = q / CX, ri = q - rj * CX;
      const int j = j0 - 2 + rj;
      S a0 = S(0), a1 = S(0), a2 = S(0), a3 = S(0);
      if (j >= 0 && j < ny) {
        const int c = (rj + 1) * PX + (ri + 1);   // the cell in the phi region
        a0 = (S)p_phi[c];
        prep_point<S, PX>(I, p_phi, p_psi, c, j, a1, a2, a3);
      }
      s_phi[q] = a0; s_nx[q] = a1; s_ny[q] = a2; s_mc[q] = a3;
    }
    // wall quantities of columns i0-1..i0+TX for the wall this tile touches
    // (the bottom one when j0 = 0, the top one when its corner rows reach ny)
    if (j0 == 0 || j0 + TY >= ny) {
      const int jw = j0 == 0 ? 0 : ny - 1;
      for (int lc = tid; active && lc < WX; lc += kNT) {
        double w[5];
        prep_wall<S, PX>(I, p_phi, p_psi, (jw - (j0 - 3)) * PX + (lc + 2), jw, w);
        for (int qk = 0; qk < 5; ++qk) s_wall[qk * WX + lc] = w[qk];
      }
    }
    __syncthreads();   // the flux arrays below reuse the phi / psi region
  } else {
    constexpr int NC = (CY * CX + kNT - 1) / kNT, NU = (UY * UX + kNT - 1) / kNT;
    S va[NC][4];
    S vu[NU][2];
#pragma unroll
    for (int e = 0; e < NC; ++e) {
      const int q = tid + e * kNT;
      const int rj = q / CX, ri = q - rj * CX;
      const int j = j0 - 2 + rj;
      va[e][0] = va[e][1] = va[e][2] = va[e][3] = S(0);
      if (active && q < CY * CX && j >= 0 && j < ny) {
        const size_t o = (size_t)j * nx + wrap_any(i0 - 2 + ri, nx);
        va[e][0] = (S)phs[o]; va[e][1] = gnx[o]; va[e][2] = gny[o]; va[e][3] = gmc[o];
      }
    }
#pragma unroll
    for (int e = 0; e < NU; ++e) {
      const int q = tid + e * kNT;
      const int rj = q / UX, ri = q - rj * UX;
      const int j = j0 - 1 + rj;
      vu[e][0] = vu[e][1] = S(0);
      if (active && q < UY * UX) {
        const size_t o = (size_t)j * nx + wrap_any(i0 - 1 + ri, nx);
        if (j >= 0 && j < ny) vu[e][0] = (S)us[o];
        if (j >= 0 && j <= ny) vu[e][1] = (S)vs[o];
      }
    }
#pragma unroll
    for (int e = 0; e < NC; ++e) {
      const int q = tid + e * kNT;
      if (active && q < CY * CX) {
        s_phi[q] = va[e][0]; s_nx[q] = va[e][1]; s_ny[q] = va[e][2]; s_mc[q] = va[e][3];
      }
    }
#pragma unroll
    for (int e = 0; e < NU; ++e) {
      const int q = tid + e * kNT;
      if (active && q < UY * UX) { s_u[q] = vu[e][0]; s_v[q] = vu[e][1]; }
    }
    __syncthreads();
  }
  const S gam = (S)I.pcg->gamma_step, eps = (S)I.eps, inv_h = (S)I.inv_h;
  const S drho = (S)(I.rho1 - I.rho2), rho2 = (S)I.rho2;
  // x-face fluxes (each face computed once per block by this one code path)
  for (int q = tid; active && q < XY * XX; q += kNT) {
    const int rj = q / XX, ri = q - rj * XX;
    const int j = j0 - 1 + rj;
    S F = 0, m = 0;
    if (j >= 0 && j < ny) {
      const int cR = (rj + 1) * CX + (ri + 1);   // cell i  (face i between cells i-1 and i)
      const int cL = cR - 1;
      const S pl = s_phi[cL], pr = s_phi[cR];
      const S pf = S(0.5) * (pl + pr);
      const S nf = S(0.5) * (s_nx[cL] + s_nx[cR]);
      const S R = gam * (eps * (pr - pl) * inv_h - pf * (S(1) - pf) * nf);
      const S u = s_u[rj * UX + ri];
      F = u * pf - R;
      m = rho2 * u + drho * F;
    }
    s_fx[q] = F; s_mx[q] = m;
  }
  // y-face fluxes; wall faces carry no flux
  for (int q = tid; active && q < YY * YX; q += kNT) {
    const int rj = q / YX, ri = q - rj * YX;
    const int f = j0 - 1 + rj;   // y-face index
    S F = 0, m = 0;
    if (f >= 1 && f <= ny - 1) {
      const int cT = (rj + 1) * CX + (ri + 1);   // cell row f
      const int cB = cT - CX;                     // cell row f-1
      const S pb = s_phi[cB], pt = s_phi[cT];
      const S pf = S(0.5) * (pb + pt);
      const S nf = S(0.5) * (s_ny[cB] + s_ny[cT]);
      const S R = gam * (eps * (pt - pb) * inv_h - pf * (S(1) - pf) * nf);
      const S v = s_v[rj * UX + ri];
      F = v * pf - R;
      m = rho2 * v + drho * F;
    }
    s_fy[q] = F; s_my[q] = m;
  }
  // corner shear stress: interior corners mu4 (du/dy + dv/dx); wall corners GNBC
  {
    const S mud = (S)(I.mu1 - I.mu2), mu2 = (S)I.mu2;
    for (int q = tid; active && q < CRY * CRX; q += kNT) {
      const int rj = q / CRX, ri = q - rj * CRX;
      const int jc = j0 + rj, ic = i0 + ri;
      S tau = 0;
      if (jc >= 1 && jc <= ny - 1) {
        const int cT = (rj + 2) * CX + (ri + 2);   // cell (jc, ic)
        const int cB = cT - CX;
        const S mu4 = S(0.25) * ((mud * s_phi[cB] + mu2) + (mud * s_phi[cB - 1] + mu2) +
                                 (mud * s_phi[cT] + mu2) + (mud * s_phi[cT - 1] + mu2));
        const int uo = (rj + 1) * UX + (ri + 1);   // u[jc, ic]
        const S dudy = (s_u[uo] - s_u[uo - UX]) * inv_h;
        const S dvdx = (s_v[uo] - s_v[uo - 1]) * inv_h;  // v[jc, ic] - v[jc, ic-1]
        tau = mu4 * (dudy + dvdx);
      } else if ((jc == 0 || jc == ny) && ic <= nx) {
        const int wall = jc == 0 ? 0 : 1;
        const int ii = wrap(ic, nx);
        const int urow = wall == 0 ? 0 : ny - 1;
        const double ur = (double)s_u[(urow - (j0 - 1)) * UX + (ri + 1)];
        double uY, usl;
        if constexpr (Fused)   // wall columns ic - 1 and ic are local columns ri and ri + 1
          tau = (S)gnbc_corner_w(I, s_wall, WX, wall, ri, ri + 1, ur, uY, usl);
        else
          tau = (S)gnbc_corner(I, wall, ii, ur, uY, usl);
        if (write_wall && ri < TX && ic < nx) {
          I.uY[wall * nx + ic] = uY;
          I.uslip[wall * nx + ic] = usl;
        }
      }
      s_txy[q] = tau;
    }
  }
  __syncthreads();

  if (!active) return;
  const int tx = tid % TX, ty = tid / TX;
  const int i = i0 + tx, j = j0 + ty;
  if (i >= nx || j >= ny) return;
  const size_t o = (size_t)j * nx + i;
  const double* __restrict__ phn = I.phi;   // base phase field of the step
  CDI_GLOBAL double* __restrict__ pdst = dst == 0 ? I.phi : (dst == 1 ? I.phi_a : I.phi_b);

  // ---- phase field: L_phi = -div F, face values differenced in FP64
  const int fxo = (ty + 1) * XX + (tx + 1);   // x-face i at row j
  const int fyo = (ty + 1) * YX + (tx + 1);   // y-face j at column i
  const double Lphi = -(((double)s_fx[fxo + 1] - (double)s_fx[fxo]) +
                        ((double)s_fy[fyo + YX] - (double)s_fy[fyo])) * I.inv_h;

  const int cc = (ty + 2) * CX + (tx + 2);   // cell (j, i) in the cell region
  const int uo = (ty + 1) * UX + (tx + 1);   // u[j,i] / v[j,i]
  const S mud = (S)(I.mu1 - I.mu2), mu2 = (S)I.mu2;

  // ---- x-momentum at u[j, i]
  S Lmx;
  {
    const S fcE = S(0.5) * (s_mx[fxo] + s_mx[fxo + 1]) * S(0.5) * (s_u[uo] + s_u[uo + 1]);
    const S fcW = S(0.5) * (s_mx[fxo - 1] + s_mx[fxo]) * S(0.5) * (s_u[uo - 1] + s_u[uo]);
    // corner (i, j+1) and (i, j): y-faces j+1 / j, columns i-1, i
    const int jt = j + 1;
    const S fcN = (jt >= ny) ? S(0)
        : S(0.5) * (s_my[fyo + YX - 1] + s_my[fyo + YX]) * S(0.5) * (s_u[uo] + s_u[uo + UX]);
    const S fcS = (j == 0) ? S(0)
        : S(0.5) * (s_my[fyo - 1] + s_my[fyo]) * S(0.5) * (s_u[uo - UX] + s_u[uo]);
    const S muE = mud * s_phi[cc] + mu2, muW = mud * s_phi[cc - 1] + mu2;
    const S txxE = S(2) * muE * (s_u[uo + 1] - s_u[uo]) * inv_h;
    const S txxW = S(2) * muW * (s_u[uo] - s_u[uo - 1]) * inv_h;
    const int co = ty * CRX + tx;   // corner (i, j)
    const S tN = s_txy[co + CRX], tS = s_txy[co];
    const S st = S(0.5) * (s_mc[cc - 1] + s_mc[cc]) * (s_phi[cc] - s_phi[cc - 1]) * inv_h;
    Lmx = -((fcE - fcW) + (fcN - fcS)) * inv_h + (txxE - txxW) * inv_h + (tN - tS) * inv_h + st;
  }
  // ---- y-momentum at interior v[j, i]
  S Lmy = 0;
  if (j >= 1) {
    const S gN = S(0.5) * (s_my[fyo] + s_my[fyo + YX]) * S(0.5) * (s_v[uo] + s_v[uo + UX]);
    const S gS = S(0.5) * (s_my[fyo - YX] + s_my[fyo]) * S(0.5) * (s_v[uo - UX] + s_v[uo]);
    // corners (i+1, j) and (i, j): x-faces i+1 / i, rows j-1, j
    const S fcE = S(0.5) * (s_mx[fxo + 1 - XX] + s_mx[fxo + 1]) * S(0.5) * (s_v[uo] + s_v[uo + 1]);
    const S fcW = S(0.5) * (s_mx[fxo - XX] + s_mx[fxo]) * S(0.5) * (s_v[uo - 1] + s_v[uo]);
    const S muN = mud * s_phi[cc] + mu2, muS = mud * s_phi[cc - CX] + mu2;
    const S tyyN = S(2) * muN * (s_v[uo + UX] - s_v[uo]) * inv_h;
    const S tyyS = S(2) * muS * (s_v[uo] - s_v[uo - UX]) * inv_h;
    const int co = ty * CRX + tx;
    const S tE = s_txy[co + 1], tW = s_txy[co];
    const S st = S(0.5) * (s_mc[cc - CX] + s_mc[cc]) * (s_phi[cc] - s_phi[cc - CX]) * inv_h;
    Lmy = -((fcE - fcW) + (gN - gS)) * inv_h + (tyyN - tyyS) * inv_h + (tE - tW) * inv_h + st;
  }

  if (k < 0) {   // operator evaluation only: publish L_phi, L_mx, L_my
    I.acc_phi[o] = Lphi;
    I.acc_mx[o] = (double)Lmx;
    I.acc_my[o] = (double)Lmy;
    return;
  }
  // ---- RK4 accumulation and next stage (operands prefetched above)
  (void)phn;
  double ap, am, an;
  if (k == 0) {
    ap = b_k * Lphi; am = b_k * (double)Lmx; an = b_k * (double)Lmy;
  } else {
    ap = pre_acc[0] + b_k * Lphi;
    am = pre_acc[1] + b_k * (double)Lmx;
    an = pre_acc[2] + b_k * (double)Lmy;
  }
  const double cn = c_next * I.dt;   // RK c_{k+1} dt of this instance
  const double r1 = I.rho1, r2 = I.rho2;
  const double rl = (r1 - r2) * pre_phw + r2;
  const double rc = (r1 - r2) * pre_phn + r2;
  const double rfx0 = 0.5 * (rl + rc);
  const double mx0 = rfx0 * pre_u;
  if (k < 3) {
    I.acc_phi[o] = ap; I.acc_mx[o] = am;
    pdst[o] = pre_phn + cn * Lphi;
    I.mx[o] = mx0 + cn * (double)Lmx;
  } else {
    pdst[o] = pre_phn + I.dt * ap;
    I.mx[o] = mx0 + I.dt * am;
  }
  if (j >= 1) {
    const double rb = (r1 - r2) * pre_phs + r2;
    const double rfy0 = 0.5 * (rb + rc);
    const double my0 = rfy0 * pre_v;
    if (k < 3) {
      I.acc_my[o] = an;
      I.my[o] = my0 + cn * (double)Lmy;
    } else {
      I.my[o] = my0 + I.dt * an;
    }
  }
}

// The stage kernel of the tiled launch, with the phase preparation fused in:
// one launch per RK stage instead of two, and no n, mu_c and wall arrays
// written and read back through memory (the persistent kernel runs the
// preparation and the stage as two passes over its tiles).
template <typename S>
__global__ void __launch_bounds__(kNT) k_stage_fused(const Tile* __restrict__ tiles,
                                                      const Inst* __restrict__ insts, int k,
                                                      int src, int dst, double c_next, double b_k,
                                                      int write_wall) {
  __shared__ StageLds<S> L;
  __shared__ double s_wall[5 * st::WX];
  const Tile t = tiles[blockIdx.x];
  stage_tile<S, true>(t, insts[t.inst], k, src, dst, c_next, b_k, write_wall, L, threadIdx.x, true,
                      s_wall);
}

// ------------------------------------------------------------ stage strip
// The stage operator over a strip of TW columns and up to sh rows, advanced
// NW rows (one chunk) at a time, with the phase preparation fused in.  Each
// of the NW waves of a block works on whole rows: lane l holds grid column
// i0 - 3 + l of every quantity (the phase field and psi of columns
// i0-3..i0+TW+1, n, mu_c, u, v, fluxes and corner stresses of the columns
// each needs), so that row indices are wave-uniform and every phase is one
// row per wave.  Rows that a chunk shares with the next (phase field, psi,
// u, v, n, mu_c, face fluxes and corner stresses) stay in rings of LDS rows:
// psi, n and mu_c of a cell, its faces and corners are each formed once per
// strip (apart from the first chunk's halo rows and ~8 % of halo columns).
// The arithmetic of every face, corner and cell is that of stage_tile.
namespace sr {
constexpr int NW = kNT / 64;       // waves of a block = rows of a chunk
constexpr int TW = 64 - 5;         // owned columns of a strip
constexpr int RW = 66;             // LDS row pitch: lane l at entry 1 + l, one pad entry each side
constexpr int SH = 32;             // rows of a strip in the tile lists
// Rows of each ring, for the chunk of rows jc..jc+NW-1 (the next chunk's
// phase-field, u and v rows are stored while this chunk's update still runs,
// without a barrier; fluxes, corners, n and mu_c of the next chunk are formed
// after its first barrier):
//   phi      rows jc-3..jc+NW+1 prepared, jc-1..jc+NW-1 read by the update,
//            next rows jc+NW+2..jc+2NW+1 arriving                -> 2NW+3
//   psi      shares the phase field's ring rows
//   u, v     rows jc-1..jc+NW in use, next jc+NW+1..jc+2NW arriving -> 2NW+2
//   n, mu_c  rows jc-2..jc+NW                                     -> NW+3
//   x-faces  rows jc-1..jc+NW-1 -> NW+1;  y-faces rows jc-1..jc+NW -> NW+2;
//   corners  rows jc..jc+NW     -> NW+1
constexpr int RP = 2 * NW + 3, RU = 2 * NW + 2, RC = NW + 3;
constexpr int RFX = NW + 1, RFY = NW + 2, RCO = NW + 1;
}  // namespace sr

template <typename S>
struct StripLds {
  double phi[sr::RP * sr::RW];   // phase field and psi share their ring rows
  S psi[sr::RP * sr::RW];
  S u[sr::RU * sr::RW], v[sr::RU * sr::RW];
  S nx[sr::RC * sr::RW], ny[sr::RC * sr::RW], mc[sr::RC * sr::RW];
  S fx[sr::RFX * sr::RW], mx[sr::RFX * sr::RW];
  S fy[sr::RFY * sr::RW], my[sr::RFY * sr::RW];
  S txy[sr::RCO * sr::RW];
  double wall[5 * sr::RW];   // wall quantities of the wall this chunk touches
};

// Position of one wave's rows in a ring of R rows: b is the LDS offset of
// row j = jc + w (this chunk's row of the wave); at<d>() the offset of row
// j + d, advance() moves to the next chunk.  All wave-uniform (scalar).
template <int R>
struct RingPos {
  int b;
  template <int d>
  __device__ __forceinline__ int at() const {
    static_assert(d > -R && d < R, "ring offset out of range");
    constexpr int span = R * sr::RW, dd = d * sr::RW;
    const int x = b + dd;
    if constexpr (d >= 0) return x >= span ? x - span : x;
    else return x < 0 ? x + span : x;
  }
  __device__ __forceinline__ void advance() {
    constexpr int span = R * sr::RW;
    b += sr::NW * sr::RW;
    if (b >= span) b -= span;
  }
};

// Tiles: one per strip (i0 a multiple of TW, j0 a multiple of sh).  Other
// arguments as k_stage_fused.  Element offsets are 32-bit (global accesses
// then take a scalar base and a 32-bit vector offset): the host keeps every
// level-0 array of an instance below 2^31 elements.
template <typename S>
__global__ void __launch_bounds__(kNT) k_stage_strip(const Tile* __restrict__ tiles,
                                                      const Inst* __restrict__ insts, int k,
                                                      int src, int dst, double c_next, double b_k,
                                                      int write_wall, int sh) {
  using sr::NW; using sr::TW; using sr::RW;
  using sr::RP; using sr::RU; using sr::RC;
  using sr::RFX; using sr::RFY; using sr::RCO;
  __shared__ StripLds<S> L;
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  const int nx = I.nx, ny = I.ny;
  const int i0 = t.i0, js = t.j0;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave = row of a chunk
  const int l = threadIdx.x & 63;                                   // lane = column i0 - 3 + l
  const int e = 1 + l;                                              // LDS entry of the lane
  const int nch = (min(sh, ny - js) + NW - 1) / NW;
  const CDI_GLOBAL double* __restrict__ phs = src == 0 ? I.phi : (src == 1 ? I.phi_a : I.phi_b);
  const CDI_GLOBAL double* __restrict__ us = k <= 0 ? I.u : I.us;
  const CDI_GLOBAL double* __restrict__ vs = k <= 0 ? I.v : I.vs;
  CDI_GLOBAL double* __restrict__ pdst = dst == 0 ? I.phi : (dst == 1 ? I.phi_a : I.phi_b);
  const int gcol = wrap_any(i0 - 3 + l, nx);   // periodic column of the lane
  // LDS row offset of grid row j of a ring of n rows whose lowest row is js - low
  auto ring = [&](int j, int low, unsigned n) { return (int)((unsigned)(j - js + low + (int)n) % n) * RW; };
  auto rp = [&](int j) { return ring(j, 3, RP); };
  auto ru = [&](int j) { return ring(j, 1, RU); };
  auto rc = [&](int j) { return ring(j, 2, RC); };
  auto rfx = [&](int j) { return ring(j, 1, RFX); };
  auto rfy = [&](int j) { return ring(j, 1, RFY); };
  auto rco = [&](int j) { return ring(j, 0, RCO); };
  // Row helpers take a compile-time tag: with IN (std::true_type) the caller
  // guarantees an interior row (the chunk's rows and everything they reach
  // lie strictly between the walls), so the row-range tests and the
  // one-sided wall branches are compiled out.
  auto load_phi = [&](auto in, int j) {
    constexpr bool IN = decltype(in)::value;
    return (IN || (j >= 0 && j < ny)) ? phs[(unsigned)(j * nx + gcol)] : 0.0;
  };
  auto store_phi = [&](auto in, int off, int j, double f) {   // phase field and psi of row j at offset off
    constexpr bool IN = decltype(in)::value;
    double ps = 0.0;
    if (IN || (j >= 0 && j < ny)) {
      const double cl = fmin(fmax(f, 0.0), 1.0);
      ps = I.eps * cdi_log((cl + kDeltaPsi) / (1.0 - cl + kDeltaPsi));
    }
    L.phi[off + e] = f;
    L.psi[off + e] = (S)ps;
  };
  auto load_u = [&](auto in, int j) {
    constexpr bool IN = decltype(in)::value;
    return (IN || (j >= 0 && j < ny)) ? (S)us[(unsigned)(j * nx + gcol)] : S(0);
  };
  auto load_v = [&](auto in, int j) {
    constexpr bool IN = decltype(in)::value;
    return (IN || (j >= 0 && j <= ny)) ? (S)vs[(unsigned)(j * nx + gcol)] : S(0);
  };
  const std::false_type edge{};
  const std::true_type inner{};
  const S gam = (S)I.pcg->gamma_step, eps = (S)I.eps, inv_h = (S)I.inv_h;
  const S drho = (S)(I.rho1 - I.rho2), rho2 = (S)I.rho2;
  const S mud = (S)(I.mu1 - I.mu2), mu2 = (S)I.mu2;
  const int i = i0 - 3 + l;   // grid column of the lane (unwrapped)
  const bool ocol = l >= 3 && l < 3 + TW && i < nx;   // the lane owns its column

  // one cell's n and mu_c (grid row jr, ring offsets of rows jr-3..jr+3)
  auto prep_row = [&](auto in, int jr, const int (&po)[7], int co) {
    constexpr bool IN = decltype(in)::value;
    S a1 = S(0), a2 = S(0), a3 = S(0);
    if (IN || (jr >= 0 && jr < ny)) {
      RingView<double> P{L.phi, {}};
      RingView<S> Q{L.psi, {}};
#pragma unroll
      for (int d = 0; d < 7; ++d) { P.off[d] = po[d] + e; Q.off[d] = po[d] + e; }
      prep_point_v<S, IN>(I, P, Q, jr, a1, a2, a3);
    }
    L.nx[co + e] = a1; L.ny[co + e] = a2; L.mc[co + e] = a3;
  };
  // x-face flux of row jr (face i between cells i-1 and i)
  auto xface = [&](auto in, int jr, int op, int oc, int ou, int of) {
    constexpr bool IN = decltype(in)::value;
    S F = 0, m = 0;
    if (IN || (jr >= 0 && jr < ny)) {
      const double* ph = L.phi + op + e;
      const S* nr = L.nx + oc + e;
      const S pl = (S)ph[-1], pr = (S)ph[0];
      const S pfc = S(0.5) * (pl + pr);
      const S nf = S(0.5) * (nr[-1] + nr[0]);
      const S R = gam * (eps * (pr - pl) * inv_h - pfc * (S(1) - pfc) * nf);
      const S u = L.u[ou + e];
      F = u * pfc - R;
      m = rho2 * u + drho * F;
    }
    L.fx[of + e] = F; L.mx[of + e] = m;
  };
  // y-face flux of face row f (between cell rows f-1 and f); wall faces carry no flux
  auto yface = [&](auto in, int f, int opb, int opt, int ocb, int oct, int ou, int of) {
    constexpr bool IN = decltype(in)::value;
    S F = 0, m = 0;
    if (IN || (f >= 1 && f <= ny - 1)) {
      const S pb = (S)L.phi[opb + e], pt = (S)L.phi[opt + e];
      const S pfc = S(0.5) * (pb + pt);
      const S nf = S(0.5) * (L.ny[ocb + e] + L.ny[oct + e]);
      const S R = gam * (eps * (pt - pb) * inv_h - pfc * (S(1) - pfc) * nf);
      const S v = L.v[ou + e];
      F = v * pfc - R;
      m = rho2 * v + drho * F;
    }
    L.fy[of + e] = F; L.my[of + e] = m;
  };
  // corner shear stress at (row jcr, column i): interior mu4 (du/dy + dv/dx); walls GNBC
  auto corner = [&](auto in, int jcr, int opb, int opt, int oub, int out, int oco) {
    constexpr bool IN = decltype(in)::value;
    S tau = 0;
    if (IN || (jcr >= 1 && jcr <= ny - 1)) {
      const double* pT = L.phi + opt + e;   // cell (jcr, i)
      const double* pB = L.phi + opb + e;
      const S mu4 = S(0.25) * ((mud * (S)pB[0] + mu2) + (mud * (S)pB[-1] + mu2) +
                               (mud * (S)pT[0] + mu2) + (mud * (S)pT[-1] + mu2));
      const S dudy = (L.u[out + e] - L.u[oub + e]) * inv_h;
      const S dvdx = (L.v[out + e] - L.v[out + e - 1]) * inv_h;
      tau = mu4 * (dudy + dvdx);
    } else if constexpr (!IN) {
      if ((jcr == 0 || jcr == ny) && i <= nx) {
        const int wall = jcr == 0 ? 0 : 1;
        const int urow = wall == 0 ? 0 : ny - 1;
        const double ur = (double)L.u[ru(urow) + e];
        double uY, usl;
        tau = (S)gnbc_corner_w(I, L.wall, RW, wall, e - 1, e, ur, uY, usl);
        if (write_wall && ocol) {
          I.uY[wall * nx + i] = uY;
          I.uslip[wall * nx + i] = usl;
        }
      }
    }
    L.txy[oco + e] = tau;
  };

  // Loads run a chunk ahead of their use: the operands of the RK update (own
  // cell; west and south base densities) of the next chunk, and the phase
  // field, u and v rows of the chunk after it.
  struct Pre { double acc[3], phn, phw, phs, u, v; };
  auto load_pre = [&](auto in, int j, Pre& p) {
    constexpr bool IN = decltype(in)::value;
    p.acc[0] = p.acc[1] = p.acc[2] = p.phn = p.phw = p.phs = p.u = p.v = 0.0;
    if (ocol && (IN || j < ny) && k >= 0) {
      const unsigned o = (unsigned)(j * nx + i);
      const CDI_GLOBAL double* __restrict__ phn0 = I.phi;
      if (k > 0) { p.acc[0] = I.acc_phi[o]; p.acc[1] = I.acc_mx[o]; p.acc[2] = I.acc_my[o]; }
      p.phn = phn0[o];
      p.phw = phn0[(unsigned)(j * nx + wrap(i - 1, nx))];
      if (IN || j >= 1) p.phs = phn0[o - nx];
      p.u = I.u[o];
      p.v = I.v[o];
    }
  };
  Pre cur, nxt;
  load_pre(edge, js + w, cur);
  // first chunk: phase field rows js-3..js+NW+1, u / v rows js-1..js+NW
  {
    double f[2];
    S a[2], b[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int rf = w + q * NW, ru_ = w + q * NW;
      f[q] = rf < NW + 5 ? load_phi(edge, js - 3 + rf) : 0.0;
      a[q] = b[q] = S(0);
      if (ru_ < NW + 2) { a[q] = load_u(edge, js - 1 + ru_); b[q] = load_v(edge, js - 1 + ru_); }
    }
    const double f2 = w == 0 ? load_phi(edge, js - 3 + 2 * NW) : 0.0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int rf = w + q * NW, ru_ = w + q * NW;
      if (rf < NW + 5) store_phi(edge, rp(js - 3 + rf), js - 3 + rf, f[q]);
      if (ru_ < NW + 2) { L.u[ru(js - 1 + ru_) + e] = a[q]; L.v[ru(js - 1 + ru_) + e] = b[q]; }
    }
    static_assert(NW + 5 <= 3 * NW, "first-chunk rows: at most three per wave");
    if (w == 0 && 2 * NW < NW + 5) store_phi(edge, rp(js - 3 + 2 * NW), js - 3 + 2 * NW, f2);
  }
  double r1phi = 0.0, r2phi = 0.0;   // phase-field row of the next chunk / the one after
  S r1u = S(0), r1v = S(0), r2u = S(0), r2v = S(0);
  if (nch > 1) {
    r1phi = load_phi(edge, js + NW + 2 + w);
    r1u = load_u(edge, js + NW + 1 + w);
    r1v = load_v(edge, js + NW + 1 + w);
  }
  // ring positions of row js + w (row jc + w of each chunk as the strip advances)
  RingPos<RP> P{(w + 3) * RW};
  RingPos<RU> U{(w + 1) * RW};
  RingPos<RC> C{(w + 2) * RW};
  RingPos<RFX> FXr{(w + 1) * RW};
  RingPos<RFY> FYr{(w + 1) * RW};
  RingPos<RCO> COr{w * RW};

  // One chunk.  IN: an interior chunk -- not the first of the strip, and
  // every row it prepares, reads, loads ahead or stores (rows jc .. jc +
  // 3 NW + 1) lies strictly between the walls.
  auto chunk = [&](auto in, int c) {
    constexpr bool IN = decltype(in)::value;
    const int jc = js + c * NW;
    const int j = jc + w;
    const bool own = ocol && (IN || j < ny);
    const unsigned o = own ? (unsigned)(j * nx + i) : 0u;
    __syncthreads();   // this chunk's phase-field, psi, u and v rows are in the rings

    // n and mu_c of the rows new to this chunk (row j + 1 of each wave; the
    // first chunk also rows jc-2..jc); wall quantities at a wall
    if constexpr (!IN) {
      if (c == 0) {
        for (int r = w; r < 3; r += NW) {
          const int jr = jc - 2 + r;
          int po[7];
#pragma unroll
          for (int d = 0; d < 7; ++d) po[d] = rp(jr + d - 3);
          prep_row(edge, jr, po, rc(jr));
        }
      }
    }
    {
      const int jr = j + 1;
      int po[7];
      po[2] = P.at<0>(); po[3] = P.at<1>(); po[4] = P.at<2>();
      if (!IN && (jr == 0 || jr >= ny - 1)) {   // one-sided wall rows reach three rows out
        po[0] = P.at<-2>(); po[1] = P.at<-1>(); po[5] = P.at<3>(); po[6] = P.at<4>();
      } else {
        po[0] = po[1] = po[5] = po[6] = 0;
      }
      prep_row(in, jr, po, C.at<1>());
    }
    if constexpr (!IN) {
      // the wall whose corner row is new to this chunk (bottom: row 0 of the
      // first chunk of the first strip; top: row ny)
      const int cra = c == 0 ? jc : jc + 1;
      const bool bot = cra == 0, top = cra <= ny && ny <= jc + NW;
      if (w == NW - 1 && (bot || top)) {
        const int jw = bot ? 0 : ny - 1;
        RingView<double> PV{L.phi, {}};
        RingView<S> QV{L.psi, {}};
#pragma unroll
        for (int d = 0; d < 7; ++d) {
          PV.off[d] = rp(jw + d - 3) + e;
          QV.off[d] = PV.off[d];
        }
        double wq[5];
        prep_wall_v<S>(I, PV, QV, jw, wq);
        for (int qk = 0; qk < 5; ++qk) L.wall[qk * RW + e] = wq[qk];
      }
    }
    __syncthreads();

    // loads for the chunks ahead
    const bool more = c + 1 < nch;
    const int jn = jc + NW;
    if (more) load_pre(in, jn + w, nxt);
    if (c + 2 < nch) {
      r2phi = load_phi(in, jn + NW + 2 + w);
      r2u = load_u(in, jn + NW + 1 + w);
      r2v = load_v(in, jn + NW + 1 + w);
    }

    // fluxes and corner stresses new to this chunk: x-faces of row j, y-faces
    // of face row j + 1, corners of row j + 1 (the first chunk also x-faces of
    // row jc - 1, y-faces of rows jc - 1 and jc, corners of row jc)
    if constexpr (!IN) {
      if (c == 0 && w < 2) {
        if (w == 0) xface(edge, jc - 1, rp(jc - 1), rc(jc - 1), ru(jc - 1), rfx(jc - 1));
        const int f = jc - 1 + w;
        yface(edge, f, rp(f - 1), rp(f), rc(f - 1), rc(f), ru(f), rfy(f));
        if (w == 1) corner(edge, jc, rp(jc - 1), rp(jc), ru(jc - 1), ru(jc), rco(jc));
      }
    }
    xface(in, j, P.at<0>(), C.at<0>(), U.at<0>(), FXr.at<0>());
    yface(in, j + 1, P.at<0>(), P.at<1>(), C.at<0>(), C.at<1>(), U.at<1>(), FYr.at<1>());
    corner(in, j + 1, P.at<0>(), P.at<1>(), U.at<0>(), U.at<1>(), COr.at<1>());
    __syncthreads();

    if (own) {
      const double* phr = L.phi + P.at<0>() + e;    // cell (j, i)
      const double* phb = L.phi + P.at<-1>() + e;   // cell (j-1, i)
      const S* mcr = L.mc + C.at<0>() + e;
      const S* mcb = L.mc + C.at<-1>() + e;
      const S* U0 = L.u + U.at<0>() + e;
      const S* UN = L.u + U.at<1>() + e;
      const S* US = L.u + U.at<-1>() + e;
      const S* V0 = L.v + U.at<0>() + e;
      const S* VN = L.v + U.at<1>() + e;
      const S* VS = L.v + U.at<-1>() + e;
      const S* FX = L.fx + FXr.at<0>() + e;
      const S* MX = L.mx + FXr.at<0>() + e;
      const S* MXS = L.mx + FXr.at<-1>() + e;
      const S* FY = L.fy + FYr.at<0>() + e;
      const S* FYN = L.fy + FYr.at<1>() + e;
      const S* MY = L.my + FYr.at<0>() + e;
      const S* MYN = L.my + FYr.at<1>() + e;
      const S* MYS = L.my + FYr.at<-1>() + e;
      const S* TS = L.txy + COr.at<0>() + e;   // corner (j, i)
      const S* TN = L.txy + COr.at<1>() + e;   // corner (j+1, i)
      // ---- phase field: L_phi = -div F, face values differenced in FP64
      const double Lphi = -(((double)FX[1] - (double)FX[0]) + ((double)FYN[0] - (double)FY[0])) *
                          I.inv_h;
      // ---- x-momentum at u[j, i]
      S Lmx;
      {
        const S fcE = S(0.5) * (MX[0] + MX[1]) * S(0.5) * (U0[0] + U0[1]);
        const S fcW = S(0.5) * (MX[-1] + MX[0]) * S(0.5) * (U0[-1] + U0[0]);
        const S fcN = (!IN && j + 1 >= ny) ? S(0) : S(0.5) * (MYN[-1] + MYN[0]) * S(0.5) * (U0[0] + UN[0]);
        const S fcS = (!IN && j == 0) ? S(0) : S(0.5) * (MY[-1] + MY[0]) * S(0.5) * (US[0] + U0[0]);
        const S muE = mud * (S)phr[0] + mu2, muW = mud * (S)phr[-1] + mu2;
        const S txxE = S(2) * muE * (U0[1] - U0[0]) * inv_h;
        const S txxW = S(2) * muW * (U0[0] - U0[-1]) * inv_h;
        const S tN = TN[0], tS = TS[0];
        const S st = S(0.5) * (mcr[-1] + mcr[0]) * ((S)phr[0] - (S)phr[-1]) * inv_h;
        Lmx = -((fcE - fcW) + (fcN - fcS)) * inv_h + (txxE - txxW) * inv_h + (tN - tS) * inv_h + st;
      }
      // ---- y-momentum at interior v[j, i]
      S Lmy = 0;
      if (IN || j >= 1) {
        const S gN = S(0.5) * (MY[0] + MYN[0]) * S(0.5) * (V0[0] + VN[0]);
        const S gS = S(0.5) * (MYS[0] + MY[0]) * S(0.5) * (VS[0] + V0[0]);
        const S fcE = S(0.5) * (MXS[1] + MX[1]) * S(0.5) * (V0[0] + V0[1]);
        const S fcW = S(0.5) * (MXS[0] + MX[0]) * S(0.5) * (V0[-1] + V0[0]);
        const S muN = mud * (S)phr[0] + mu2, muS = mud * (S)phb[0] + mu2;
        const S tyyN = S(2) * muN * (VN[0] - V0[0]) * inv_h;
        const S tyyS = S(2) * muS * (V0[0] - VS[0]) * inv_h;
        const S tE = TS[1], tW = TS[0];
        const S st = S(0.5) * (mcb[0] + mcr[0]) * ((S)phr[0] - (S)phb[0]) * inv_h;
        Lmy = -((fcE - fcW) + (gN - gS)) * inv_h + (tyyN - tyyS) * inv_h + (tE - tW) * inv_h + st;
      }
      if (k < 0) {   // operator evaluation only: publish L_phi, L_mx, L_my
        I.acc_phi[o] = Lphi;
        I.acc_mx[o] = (double)Lmx;
        I.acc_my[o] = (double)Lmy;
      } else {
        // ---- RK4 accumulation and next stage
        double ap, am, an;
        if (k == 0) {
          ap = b_k * Lphi; am = b_k * (double)Lmx; an = b_k * (double)Lmy;
        } else {
          ap = cur.acc[0] + b_k * Lphi;
          am = cur.acc[1] + b_k * (double)Lmx;
          an = cur.acc[2] + b_k * (double)Lmy;
        }
        const double cn = c_next * I.dt;   // RK c_{k+1} dt of this instance
        const double r1 = I.rho1, r2 = I.rho2;
        const double rl = (r1 - r2) * cur.phw + r2;
        const double rcn = (r1 - r2) * cur.phn + r2;
        const double mx0 = 0.5 * (rl + rcn) * cur.u;
        if (k < 3) {
          I.acc_phi[o] = ap; I.acc_mx[o] = am;
          pdst[o] = cur.phn + cn * Lphi;
          I.mx[o] = mx0 + cn * (double)Lmx;
        } else {
          pdst[o] = cur.phn + I.dt * ap;
          I.mx[o] = mx0 + I.dt * am;
        }
        if (IN || j >= 1) {
          const double rb = (r1 - r2) * cur.phs + r2;
          const double my0 = 0.5 * (rb + rcn) * cur.v;
          if (k < 3) {
            I.acc_my[o] = an;
            I.my[o] = my0 + cn * (double)Lmy;
          } else {
            I.my[o] = my0 + I.dt * an;
          }
        }
      }
    }
    // the next chunk's rows into the rings (slots this chunk's update does not read)
    if (more) {
      store_phi(in, P.at<NW + 2>(), jn + 2 + w, r1phi);
      L.u[U.at<NW + 1>() + e] = r1u;
      L.v[U.at<NW + 1>() + e] = r1v;
    }
    cur = nxt;
    r1phi = r2phi; r1u = r2u; r1v = r2v;
    P.advance(); U.advance(); C.advance(); FXr.advance(); FYr.advance(); COr.advance();
  };

  for (int c = 0; c < nch; ++c) {
    if (c >= 1 && js + c * NW + 3 * NW + 3 <= ny - 1) chunk(inner, c);
    else chunk(edge, c);
  }
}

}  // namespace cdi
