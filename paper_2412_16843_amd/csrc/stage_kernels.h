// Stage kernels of the CDI + GNBC step: phase-field preparation, the fused
// CDI-flux / momentum / surface-tension / GNBC stage operator with its RK4
// update, the projection right-hand side and the projection itself.
//
// S is the stencil precision (double on the FP64 path, float on the mixed
// path).  The phase field, its RK accumulation, the flux differences of the
// phi update and every reduction stay in FP64 on both paths.
#pragma once
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

template <typename T>
__device__ __forceinline__ T ddy_cell(const T* q, int stride, int j, int ny, T inv2h) {
  // q points at the cell; stride = LDS row pitch
  if (j == 0) return (T(-3) * q[0] + T(4) * q[stride] - q[2 * stride]) * inv2h;
  if (j == ny - 1) return (T(3) * q[0] - T(4) * q[-stride] + q[-2 * stride]) * inv2h;
  return (q[stride] - q[-stride]) * inv2h;
}
template <typename T>
__device__ __forceinline__ T d2dy2_cell(const T* q, int stride, int j, int ny, T inv_h2) {
  if (j == 0) return (T(2) * q[0] - T(5) * q[stride] + T(4) * q[2 * stride] - q[3 * stride]) * inv_h2;
  if (j == ny - 1) return (T(2) * q[0] - T(5) * q[-stride] + T(4) * q[-2 * stride] - q[-3 * stride]) * inv_h2;
  return (q[stride] - T(2) * q[0] + q[-stride]) * inv_h2;
}

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

// n = G/(|G| + dN) and mu_c at the cell of LDS index c (row pitch RX) in
// grid row j, from the FP64 phase field and psi (one-sided rows at the
// walls, Sec. 4).
template <typename S, int RX>
__device__ __forceinline__ void prep_point(const Inst& I, const double* s_phi, const S* s_psi,
                                           int c, int j, S& onx, S& ony, S& omu) {
  const int ny = I.ny;
  const S inv2h = (S)(0.5 * I.inv_h), inv_h2 = (S)(I.inv_h * I.inv_h);
  const S eps = (S)I.eps;
  // normal from phi
  const S gx = ((S)s_phi[c + 1] - (S)s_phi[c - 1]) * inv2h;
  S gy;
  {
    if (j == 0) gy = (S(-3) * (S)s_phi[c] + S(4) * (S)s_phi[c + RX] - (S)s_phi[c + 2 * RX]) * inv2h;
    else if (j == ny - 1) gy = (S(3) * (S)s_phi[c] - S(4) * (S)s_phi[c - RX] + (S)s_phi[c - 2 * RX]) * inv2h;
    else gy = ((S)s_phi[c + RX] - (S)s_phi[c - RX]) * inv2h;
  }
  const S mag = sqrt(gx * gx + gy * gy) + (S)kDeltaN;
  // psi derivatives, curvature, chemical potential
  const S* q = s_psi + c;
  const S px = (q[1] - q[-1]) * inv2h;
  const S py = ddy_cell<S>(q, RX, j, ny, inv2h);
  const S lap = (q[1] - S(2) * q[0] + q[-1]) * inv_h2 + d2dy2_cell<S>(q, RX, j, ny, inv_h2);
  const S ph = (S)s_phi[c];
  const S g = ph * (S(1) - ph);
  const S grad2 = px * px + py * py;
  onx = gx / mag;
  ony = gy / mag;
  omu = S(6) * (S)I.sigma * (g * (S(1) - S(2) * ph) * (S(1) - grad2) / eps - g * lap);
}

// Wall quantities of the slip models for the column of a wall-row cell (LDS
// index c, row pitch RX, grid row j = 0 or ny - 1): phi, psi, d psi/dy,
// kappa and d phi/dy of the wall row and the next row, linearly
// extrapolated to the wall per column (Sec. 4), in FP64.
template <typename S, int RX>
__device__ __forceinline__ void prep_wall(const Inst& I, const double* s_phi, const S* s_psi,
                                          int c, int j, double out[5]) {
  const int ny = I.ny;
  const int dj = j == 0 ? 1 : -1;          // second cell row from the wall
  const int c2 = c + dj * RX;
  const int j2 = j + dj;
  double vals[2][5];
  for (int r = 0; r < 2; ++r) {
    const int cc = r == 0 ? c : c2, jj = r == 0 ? j : j2;
    // FP64 wall quantities from the psi tile
    const S* qs = s_psi + cc;
    const double i2h = 0.5 * I.inv_h, ih2 = I.inv_h * I.inv_h;
    const double p0 = (double)qs[0];
    double pyd, d2y;
    if (jj == 0) {
      pyd = (-3.0 * p0 + 4.0 * (double)qs[RX] - (double)qs[2 * RX]) * i2h;
      d2y = (2.0 * p0 - 5.0 * (double)qs[RX] + 4.0 * (double)qs[2 * RX] - (double)qs[3 * RX]) * ih2;
    } else if (jj == ny - 1) {
      pyd = (3.0 * p0 - 4.0 * (double)qs[-RX] + (double)qs[-2 * RX]) * i2h;
      d2y = (2.0 * p0 - 5.0 * (double)qs[-RX] + 4.0 * (double)qs[-2 * RX] - (double)qs[-3 * RX]) * ih2;
    } else {
      pyd = ((double)qs[RX] - (double)qs[-RX]) * i2h;
      d2y = ((double)qs[RX] - 2.0 * p0 + (double)qs[-RX]) * ih2;
    }
    const double pxd = ((double)qs[1] - (double)qs[-1]) * i2h;
    const double lapd = ((double)qs[1] - 2.0 * p0 + (double)qs[-1]) * ih2 + d2y;
    const double phd = s_phi[cc];
    const double kap = (1.0 - 2.0 * phd) * (1.0 - pxd * pxd - pyd * pyd) / I.eps - lapd;
    double phy;
    if (jj == 0) phy = (-3.0 * phd + 4.0 * s_phi[cc + RX] - s_phi[cc + 2 * RX]) * i2h;
    else if (jj == ny - 1) phy = (3.0 * phd - 4.0 * s_phi[cc - RX] + s_phi[cc - 2 * RX]) * i2h;
    else phy = (s_phi[cc + RX] - s_phi[cc - RX]) * i2h;
    vals[r][0] = phd; vals[r][1] = p0; vals[r][2] = pyd; vals[r][3] = kap; vals[r][4] = phy;
  }
  for (int qk = 0; qk < 5; ++qk) out[qk] = 0.5 * (3.0 * vals[0][qk] - vals[1][qk]);
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
  ((S*)I.nhx)[o] = vnx;
  ((S*)I.nhy)[o] = vny;
  ((S*)I.muc)[o] = vmu;
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
      ps = I.eps * log((c + kDeltaPsi) / (1.0 - c + kDeltaPsi));
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
  const double* __restrict__ phs = src == 0 ? I.phi : (src == 1 ? I.phi_a : I.phi_b);
  const double* __restrict__ us = k <= 0 ? I.u : I.us;
  const double* __restrict__ vs = k <= 0 ? I.v : I.vs;
  const S* __restrict__ gnx = (const S*)I.nhx;
  const S* __restrict__ gny = (const S*)I.nhy;
  const S* __restrict__ gmc = (const S*)I.muc;

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
        ps = I.eps * log((cl + kDeltaPsi) / (1.0 - cl + kDeltaPsi));
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
  double* __restrict__ pdst = dst == 0 ? I.phi : (dst == 1 ? I.phi_a : I.phi_b);

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

}  // namespace cdi
