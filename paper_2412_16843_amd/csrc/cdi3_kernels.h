// Device side of the three-dimensional CDI + GNBC step (gfx950).
//
// Grid (x fastest): cells (k, j, i) at ((i+1/2) h, (j+1/2) h, (k+1/2) h),
// x and z periodic, walls at y = 0 and y = ny h.  u on x-faces, w on
// z-faces (nz ny nx); v on y-faces (nz (ny+1) nx, rows 0 and ny on the walls).
// Shear stresses live on edges: xy-edges and yz-edges in the v layout (rows 0
// and ny on the walls, where the GNBC gives them), xz-edges in the cell
// layout.  The arithmetic is that of the two-dimensional kernels face by face
// with the z terms added (Sec. 2, 4 of the paper); the wall model carries the
// slip as a vector in the wall plane and the in-plane curvature kappa_p of
// the curvature correction (Sec. 2, slip BC; Sec. 3.1.2).
//
// One thread per cell, face or edge; neighbours come from global memory
// (L2).  Element offsets are 32-bit: the host keeps nz (ny+1) nx < 2^31.
#pragma once
#include <hip/hip_runtime.h>

#include "cdi_dev.h"

namespace cdi3 {

constexpr int kNT3 = 256;
constexpr int kMaxLev3 = 12;
constexpr int kCoarseMax3 = 1024;   // cells of the coarsest level (one block)
constexpr int kCoarseSweeps3 = 40;  // red-black sweep pairs of the coarsest solve
constexpr double kDeltaT = 1e-12;   // regularises |t_q| where psi has no tangential gradient

// device scalars of a solve / step
enum { S_GAMMA = 0, S_BMEAN, S_FF, S_RR, S_RZ, S_RZOLD, S_DQ, S_ALPHA, S_ZQ, S_XMEAN, S_RELRES,
       S_VMAX, S_NSCAL };

struct Lev3 {
  int nx, ny, nz;
  cdi::gptr<double> ax;   // x-faces, cell layout
  cdi::gptr<double> ay;   // y-faces, v layout (wall rows 0)
  cdi::gptr<double> az;   // z-faces, cell layout
  cdi::gptr<double> r;    // right-hand side of the level
  cdi::gptr<double> x;    // correction of the level
};

struct Ctx3 {
  int nx, ny, nz, slip_model;
  double h, inv_h, eps, inv_eps, sigma, cos_eq;
  double rho1, rho2, mu1, mu2, beta1, beta2;
  double uwb, uwt, wwb, wwt;   // wall speeds: x bottom / top, z bottom / top
  double dt;
  cdi::gptr<double> phi, u, v, w, p;                     // caller state
  cdi::gptr<double> phi_a, phi_b, us, vs, ws;            // stage phase field and velocity
  cdi::gptr<double> acc_phi, acc_mx, acc_my, acc_mz;      // RK accumulators (acc_my: v layout)
  cdi::gptr<double> mx, my, mz;                            // next-stage momentum (my: v layout)
  cdi::gptr<double> psi, nxv, nyv, nzv, muc, kap_p;
  cdi::gptr<double> wall;                                    // [2][5][nz][nx]: phi, psi, psi_y, kappa_p, phi_y
  cdi::gptr<double> Fx, Fy, Fz, fmx, fmy, fmz;           // face fluxes and mass fluxes (Fy, fmy: v layout)
  cdi::gptr<double> txy, tyz, txz;                         // edge stresses
  cdi::gptr<double> uYx, uYz, slx, slz;                   // [2][nz][nx] Young slip and total slip
  cdi::gptr<double> b, x, r, z, d, q;
  cdi::gptr<double> part;                                    // block partials
  cdi::gptr<double> scal;                                    // S_* scalars
  cdi::gptr<double> hp[4][4];   // [slot][RK stage] mean-free pressure of the last four steps
                                // (ring: step n writes slot n mod 4)
  int nlev;
  Lev3 lev[kMaxLev3];
};

__device__ __forceinline__ int wrap3(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }
__device__ __forceinline__ unsigned ic3(int nx, int ny, int k, int j, int i) {
  return (unsigned)((k * ny + j) * nx + i);
}
__device__ __forceinline__ unsigned iv3(int nx, int ny, int k, int j, int i) {
  return (unsigned)((k * (ny + 1) + j) * nx + i);
}

// n / d for 0 <= n < 2^31 and d >= 1: the quotient from the hardware
// reciprocal refined by one Newton step (relative error far below 2^-31, so
// off by at most one) and one exact integer correction -- a few operations
// instead of the long integer division sequence.
__device__ __forceinline__ int quot3(int n, int d) {
  const double dd = (double)d;
  double r = __builtin_amdgcn_rcp(dd);
  r = fma(fma(-dd, r, 1.0), r, r);
  int q = (int)((double)n * r);
  const int rem = n - q * d;
  q += (rem >= d) - (rem < 0);
  return q;
}

// (k, j, i) of flat index g over nz x rows x nx (the host keeps the product
// below 2^31); false beyond the grid.
__device__ __forceinline__ bool unflat3(long g, int nx, int rows, int nz, int& k, int& j, int& i) {
  if (g >= (long)nx * rows * nz) return false;
  const int gi = (int)g;
  const int t = quot3(gi, nx);
  i = gi - t * nx;
  k = quot3(t, rows);
  j = t - k * rows;
  return true;
}

// block sum of up to 2 values into part[blockIdx.x] and part[gridDim.x + blockIdx.x]
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double* __restrict__ part) {
  __shared__ double sh[NV][kNT3 / 64];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = v[q];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) sh[q][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double s = 0.0;
      for (int wv = 0; wv < kNT3 / 64; ++wv) s += sh[q][wv];
      part[(size_t)q * gridDim.x + blockIdx.x] = s;
    }
  }
}

// ------------------------------------------------------------ phase fields
__global__ void __launch_bounds__(kNT3) k3_psi(const Ctx3* __restrict__ C, int src) {
  const long g = (long)blockIdx.x * kNT3 + threadIdx.x;
  const int n = C->nx * C->ny * C->nz;
  if (g >= n) return;
  const CDI_GLOBAL double* ph = src == 0 ? C->phi : (src == 1 ? C->phi_a : C->phi_b);
  const double cl = fmin(fmax(ph[g], 0.0), 1.0);
  C->psi[g] = C->eps * cdi::cdi_log((cl + cdi::kDeltaPsi) / (1.0 - cl + cdi::kDeltaPsi));
}

// d/dy of q at row j of a column (one-sided second order on the wall rows)
__device__ __forceinline__ double ddy3(const double* q, int s, int j, int ny, double i2h) {
  if (j == 0) return (-3.0 * q[0] + 4.0 * q[s] - q[2 * s]) * i2h;
  if (j == ny - 1) return (3.0 * q[0] - 4.0 * q[-s] + q[-2 * s]) * i2h;
  return (q[s] - q[-s]) * i2h;
}
__device__ __forceinline__ double d2dy3(const double* q, int s, int j, int ny, double ih2) {
  if (j == 0) return (2.0 * q[0] - 5.0 * q[s] + 4.0 * q[2 * s] - q[3 * s]) * ih2;
  if (j == ny - 1) return (2.0 * q[0] - 5.0 * q[-s] + 4.0 * q[-2 * s] - q[-3 * s]) * ih2;
  return (q[s] - 2.0 * q[0] + q[-s]) * ih2;
}

// n = G/(|G| + dN) and mu_c at every cell (eqs. CDI, chemical potential).
__global__ void __launch_bounds__(kNT3) k3_prep(const Ctx3* __restrict__ C, int src) {
  const int nx = C->nx, ny = C->ny, nz = C->nz;
  int k, j, i;
  if (!unflat3((long)blockIdx.x * kNT3 + threadIdx.x, nx, ny, nz, k, j, i)) return;
  const CDI_GLOBAL double* ph = src == 0 ? C->phi : (src == 1 ? C->phi_a : C->phi_b);
  const double* ps = C->psi;
  const unsigned c = ic3(nx, ny, k, j, i);
  const unsigned ce = ic3(nx, ny, k, j, wrap3(i + 1, nx)), cw = ic3(nx, ny, k, j, wrap3(i - 1, nx));
  const unsigned cf = ic3(nx, ny, wrap3(k + 1, nz), j, i), cb = ic3(nx, ny, wrap3(k - 1, nz), j, i);
  const double i2h = 0.5 * C->inv_h, ih2 = C->inv_h * C->inv_h;
  const double gx = (ph[ce] - ph[cw]) * i2h;
  const double gz = (ph[cf] - ph[cb]) * i2h;
  const double gy = ddy3(ph + c, nx, j, ny, i2h);
  const double mag = sqrt(gx * gx + gy * gy + gz * gz) + cdi::kDeltaN;
  const double rm = 1.0 / mag;
  C->nxv[c] = gx * rm;
  C->nyv[c] = gy * rm;
  C->nzv[c] = gz * rm;
  const double px = (ps[ce] - ps[cw]) * i2h, pz = (ps[cf] - ps[cb]) * i2h;
  const double py = ddy3(ps + c, nx, j, ny, i2h);
  const double lap = (ps[ce] - 2.0 * ps[c] + ps[cw]) * ih2 + d2dy3(ps + c, nx, j, ny, ih2) +
                     (ps[cf] - 2.0 * ps[c] + ps[cb]) * ih2;
  const double f = ph[c];
  const double g = f * (1.0 - f);
  C->muc[c] = 6.0 * C->sigma *
              (g * (1.0 - 2.0 * f) * (1.0 - px * px - py * py - pz * pz) * C->inv_eps - g * lap);
}

// kappa_p at cell (k, j, i): the energy-based curvature plus the normal
// curvature term of psi along the contact line t_q = (-psi_z, 0, psi_x)/|.|.
__device__ __forceinline__ double kappa_p_at(const Ctx3* __restrict__ C, const double* ph,
                                             int k, int j, int i) {
  const int nx = C->nx, ny = C->ny, nz = C->nz;
  const double* ps = C->psi;
  const unsigned c = ic3(nx, ny, k, j, i);
  const int ie = wrap3(i + 1, nx), iw = wrap3(i - 1, nx);
  const int kf = wrap3(k + 1, nz), kb = wrap3(k - 1, nz);
  const unsigned ce = ic3(nx, ny, k, j, ie), cw = ic3(nx, ny, k, j, iw);
  const unsigned cf = ic3(nx, ny, kf, j, i), cb = ic3(nx, ny, kb, j, i);
  const double i2h = 0.5 * C->inv_h, ih2 = C->inv_h * C->inv_h;
  const double px = (ps[ce] - ps[cw]) * i2h, pz = (ps[cf] - ps[cb]) * i2h;
  const double py = ddy3(ps + c, nx, j, ny, i2h);
  const double pxx = (ps[ce] - 2.0 * ps[c] + ps[cw]) * ih2;
  const double pzz = (ps[cf] - 2.0 * ps[c] + ps[cb]) * ih2;
  const double lap = pxx + d2dy3(ps + c, nx, j, ny, ih2) + pzz;
  const double pxz = (ps[ic3(nx, ny, kf, j, ie)] - ps[ic3(nx, ny, kf, j, iw)] -
                      ps[ic3(nx, ny, kb, j, ie)] + ps[ic3(nx, ny, kb, j, iw)]) * (0.25 * ih2);
  const double f = ph[c];
  const double kap = (1.0 - 2.0 * f) * (1.0 - px * px - py * py - pz * pz) * C->inv_eps - lap;
  return kap + (pz * pz * pxx - 2.0 * px * pz * pxz + px * px * pzz) /
                   (px * px + pz * pz + kDeltaT * kDeltaT);
}

__global__ void __launch_bounds__(kNT3) k3_kappa_p(const Ctx3* __restrict__ C, int src,
                                                   double* __restrict__ out) {
  int k, j, i;
  if (!unflat3((long)blockIdx.x * kNT3 + threadIdx.x, C->nx, C->ny, C->nz, k, j, i)) return;
  const CDI_GLOBAL double* ph = src == 0 ? C->phi : (src == 1 ? C->phi_a : C->phi_b);
  out[ic3(C->nx, C->ny, k, j, i)] = kappa_p_at(C, ph, k, j, i);
}

// Wall quantities per (wall, k, i) column: phi, psi, d psi/dy, kappa_p and
// d phi/dy of the wall row and the next, linearly extrapolated to the wall.
__global__ void __launch_bounds__(kNT3) k3_wall(const Ctx3* __restrict__ C, int src) {
  const int nx = C->nx, ny = C->ny, nz = C->nz;
  const long g = (long)blockIdx.x * kNT3 + threadIdx.x;
  if (g >= 2L * nz * nx) return;
  const int i = (int)(g % nx), k = (int)((g / nx) % nz), wall = (int)(g / ((long)nx * nz));
  const CDI_GLOBAL double* ph = src == 0 ? C->phi : (src == 1 ? C->phi_a : C->phi_b);
  const double i2h = 0.5 * C->inv_h;
  double val[2][5];
  for (int r = 0; r < 2; ++r) {
    const int jj = wall == 0 ? r : ny - 1 - r;
    const unsigned c = ic3(nx, ny, k, jj, i);
    val[r][0] = ph[c];
    val[r][1] = C->psi[c];
    val[r][2] = ddy3(C->psi + c, nx, jj, ny, i2h);
    val[r][3] = kappa_p_at(C, ph, k, jj, i);
    val[r][4] = ddy3(ph + c, nx, jj, ny, i2h);
  }
  for (int q = 0; q < 5; ++q)
    C->wall[((size_t)(wall * 5 + q) * nz + k) * nx + i] = 0.5 * (3.0 * val[0][q] - val[1][q]);
}

// ------------------------------------------------------------ wall slip
// Young slip of one tangential component at an edge between wall columns a
// (minus side) and b (plus side) of wall `wall`; o_a, o_b: the central
// differences of the wall quantities along the other tangential direction at
// a and b (phi and psi).  Models 1A..4B (Sec. 3), in the form of the
// two-dimensional kernel with |grad| over all three components.
__device__ __forceinline__ double slip_edge(const Ctx3* __restrict__ C, int wall, unsigned a,
                                            unsigned b, double ophi, double opsi,
                                            double& phc_out, double& beta_out) {
  const int nx = C->nx, nz = C->nz;
  const double* W = C->wall + (size_t)wall * 5 * nz * nx;
  const size_t ws = (size_t)nz * nx;
  const double sgn = wall == 0 ? 1.0 : -1.0;
  double phc = 0.5 * (W[a] + W[b]);
  phc = fmin(fmax(phc, 0.0), 1.0);
  const double psc = 0.5 * (W[ws + a] + W[ws + b]);
  const double dpn = sgn * 0.5 * (W[2 * ws + a] + W[2 * ws + b]);
  const double kac = 0.5 * (W[3 * ws + a] + W[3 * ws + b]);
  const double dphn = sgn * 0.5 * (W[4 * ws + a] + W[4 * ws + b]);
  const double dpt = (W[ws + b] - W[ws + a]) * C->inv_h;
  const double dpht = (W[b] - W[a]) * C->inv_h;
  const double g = phc * (1.0 - phc);
  const double beta = C->beta2 + (C->beta1 - C->beta2) * phc;
  const double ce = C->cos_eq;
  const double corr = 1.0 + kac * psc;
  const double pre = -6.0 * C->sigma / beta;
  const double eps = C->eps;
  const double gphi = sqrt(dphn * dphn + dpht * dpht + ophi * ophi);
  const double gpsi = sqrt(dpn * dpn + dpt * dpt + opsi * opsi);
  double uY;
  switch (C->slip_model) {
    case 0:  uY = pre * (eps * dphn + g * ce) * dpht; break;                          // 1A
    case 1:  uY = pre * (eps * dphn + eps * gphi * ce) * dpht; break;                 // 1B
    case 2:  uY = pre * (g * dpn + g * ce) * g / eps * dpt; break;                    // 2A
    case 3:  uY = pre * (g * dpn + g * gpsi * ce) * g / eps * dpt; break;             // 2B
    case 4:  uY = pre * (eps * dphn + g * corr * ce) * dpht; break;                   // 3A
    case 5:  uY = pre * (eps * dphn + eps * gphi * corr * ce) * dpht; break;          // 3B
    case 7:  uY = pre * (g * dpn + g * gpsi * corr * ce) * g / eps * dpt; break;      // 4B
    default: uY = pre * (g * dpn + g * corr * ce) * g / eps * dpt; break;             // 4A
  }
  phc_out = phc;
  beta_out = beta;
  return uY;
}

// ------------------------------------------------------------ fluxes
// CDI face fluxes F = u phi_f - gamma[eps dphi/dn - phi_f(1 - phi_f) n_f] and
// mass fluxes m = rho2 u + (rho1 - rho2) F on the x-, y- and z-faces of the
// cell (west, south, back); the thread of the last row also clears the top
// wall face.  src / k as in k3_stage.
__global__ void __launch_bounds__(kNT3) k3_flux(const Ctx3* __restrict__ C, int src, int kst) {
  const int nx = C->nx, ny = C->ny, nz = C->nz;
  int k, j, i;
  if (!unflat3((long)blockIdx.x * kNT3 + threadIdx.x, nx, ny, nz, k, j, i)) return;
  const CDI_GLOBAL double* ph = src == 0 ? C->phi : (src == 1 ? C->phi_a : C->phi_b);
  const CDI_GLOBAL double* uu = kst <= 0 ? C->u : C->us;
  const CDI_GLOBAL double* vv = kst <= 0 ? C->v : C->vs;
  const CDI_GLOBAL double* ww = kst <= 0 ? C->w : C->ws;
  const double gam = C->scal[S_GAMMA], eps = C->eps, inv_h = C->inv_h;
  const double drho = C->rho1 - C->rho2, rho2 = C->rho2;
  const unsigned c = ic3(nx, ny, k, j, i);
  const double pc = ph[c];
  {
    const unsigned cw = ic3(nx, ny, k, j, wrap3(i - 1, nx));
    const double pl = ph[cw];
    const double pf = 0.5 * (pl + pc);
    const double nf = 0.5 * (C->nxv[cw] + C->nxv[c]);
    const double F = uu[c] * pf - gam * (eps * (pc - pl) * inv_h - pf * (1.0 - pf) * nf);
    C->Fx[c] = F;
    C->fmx[c] = rho2 * uu[c] + drho * F;
  }
  {
    const unsigned cb = ic3(nx, ny, wrap3(k - 1, nz), j, i);
    const double pl = ph[cb];
    const double pf = 0.5 * (pl + pc);
    const double nf = 0.5 * (C->nzv[cb] + C->nzv[c]);
    const double F = ww[c] * pf - gam * (eps * (pc - pl) * inv_h - pf * (1.0 - pf) * nf);
    C->Fz[c] = F;
    C->fmz[c] = rho2 * ww[c] + drho * F;
  }
  const unsigned fv = iv3(nx, ny, k, j, i);
  if (j == 0) {
    C->Fy[fv] = 0.0;
    C->fmy[fv] = 0.0;
  } else {
    const unsigned cs = c - nx;
    const double pl = ph[cs];
    const double pf = 0.5 * (pl + pc);
    const double nf = 0.5 * (C->nyv[cs] + C->nyv[c]);
    const double F = vv[fv] * pf - gam * (eps * (pc - pl) * inv_h - pf * (1.0 - pf) * nf);
    C->Fy[fv] = F;
    C->fmy[fv] = rho2 * vv[fv] + drho * F;
  }
  if (j == ny - 1) {
    C->Fy[fv + nx] = 0.0;
    C->fmy[fv + nx] = 0.0;
  }
}

// ------------------------------------------------------------ edge stresses
// Thread (k, j, i), j = 0..ny: the xy-edge (i h, j h, (k+1/2) h) and the
// yz-edge ((i+1/2) h, j h, k h) stresses (GNBC on the wall rows, also
// publishing the slip), and for j < ny the xz-edge (i h, (j+1/2) h, k h).
__global__ void __launch_bounds__(kNT3) k3_edges(const Ctx3* __restrict__ C, int src, int kst,
                                                 int write_wall) {
  const int nx = C->nx, ny = C->ny, nz = C->nz;
  int k, j, i;
  if (!unflat3((long)blockIdx.x * kNT3 + threadIdx.x, nx, ny + 1, nz, k, j, i)) return;
  const CDI_GLOBAL double* ph = src == 0 ? C->phi : (src == 1 ? C->phi_a : C->phi_b);
  const CDI_GLOBAL double* uu = kst <= 0 ? C->u : C->us;
  const CDI_GLOBAL double* vv = kst <= 0 ? C->v : C->vs;
  const CDI_GLOBAL double* ww = kst <= 0 ? C->w : C->ws;
  const double mud = C->mu1 - C->mu2, mu2 = C->mu2, inv_h = C->inv_h;
  const int iw = wrap3(i - 1, nx), kb = wrap3(k - 1, nz);
  const unsigned e = iv3(nx, ny, k, j, i);
  if (j >= 1 && j <= ny - 1) {
    const unsigned c = ic3(nx, ny, k, j, i), cs = c - nx;
    const unsigned cw = ic3(nx, ny, k, j, iw), csw = cw - nx;
    const double mu4 = 0.25 * ((mud * ph[cs] + mu2) + (mud * ph[csw] + mu2) + (mud * ph[c] + mu2) +
                               (mud * ph[cw] + mu2));
    const double dudy = (uu[c] - uu[cs]) * inv_h;
    const double dvdx = (vv[e] - vv[iv3(nx, ny, k, j, iw)]) * inv_h;
    C->txy[e] = mu4 * (dudy + dvdx);
    const unsigned cbk = ic3(nx, ny, kb, j, i), cbs = cbk - nx;
    const double mu4z = 0.25 * ((mud * ph[cs] + mu2) + (mud * ph[cbs] + mu2) + (mud * ph[c] + mu2) +
                                (mud * ph[cbk] + mu2));
    const double dwdy = (ww[c] - ww[cs]) * inv_h;
    const double dvdz = (vv[e] - vv[iv3(nx, ny, kb, j, i)]) * inv_h;
    C->tyz[e] = mu4z * (dwdy + dvdz);
  } else {
    const int wall = j == 0 ? 0 : 1;
    const int urow = wall == 0 ? 0 : ny - 1;
    const double sgt = wall == 0 ? 1.0 : -1.0;   // tau = sgt * 2 mu (row - wall)/h
    const double* W = C->wall + (size_t)wall * 5 * nz * nx;
    const size_t wsz = (size_t)nz * nx;
    const double i2h = 0.5 * inv_h;
    const int ie = wrap3(i + 1, nx), kf = wrap3(k + 1, nz);
    // x-slip at the xy-edge between columns (k, i-1) and (k, i)
    {
      const unsigned a = (unsigned)(k * nx + iw), b = (unsigned)(k * nx + i);
      const double oa_phi = (W[kf * nx + iw] - W[kb * nx + iw]) * i2h;
      const double ob_phi = (W[kf * nx + i] - W[kb * nx + i]) * i2h;
      const double oa_psi = (W[wsz + kf * nx + iw] - W[wsz + kb * nx + iw]) * i2h;
      const double ob_psi = (W[wsz + kf * nx + i] - W[wsz + kb * nx + i]) * i2h;
      double phc, beta;
      const double uY = slip_edge(C, wall, a, b, 0.5 * (oa_phi + ob_phi), 0.5 * (oa_psi + ob_psi),
                                  phc, beta);
      const double U = wall == 0 ? C->uwb : C->uwt;
      const double muw = C->mu2 + (C->mu1 - C->mu2) * phc;
      const double lam = 2.0 * muw / (beta * C->h);
      const double row = uu[ic3(nx, ny, k, urow, i)];
      const double uw = (U + uY + lam * row) / (1.0 + lam);
      C->txy[e] = wall == 0 ? 2.0 * muw * (row - uw) * inv_h : 2.0 * muw * (uw - row) * inv_h;
      if (write_wall) {
        C->uYx[(size_t)wall * wsz + b] = uY;
        C->slx[(size_t)wall * wsz + b] = uw - U;
      }
    }
    // z-slip at the yz-edge between columns (k-1, i) and (k, i)
    {
      const unsigned a = (unsigned)(kb * nx + i), b = (unsigned)(k * nx + i);
      const double oa_phi = (W[kb * nx + ie] - W[kb * nx + iw]) * i2h;
      const double ob_phi = (W[k * nx + ie] - W[k * nx + iw]) * i2h;
      const double oa_psi = (W[wsz + kb * nx + ie] - W[wsz + kb * nx + iw]) * i2h;
      const double ob_psi = (W[wsz + k * nx + ie] - W[wsz + k * nx + iw]) * i2h;
      double phc, beta;
      const double uY = slip_edge(C, wall, a, b, 0.5 * (oa_phi + ob_phi), 0.5 * (oa_psi + ob_psi),
                                  phc, beta);
      const double U = wall == 0 ? C->wwb : C->wwt;
      const double muw = C->mu2 + (C->mu1 - C->mu2) * phc;
      const double lam = 2.0 * muw / (beta * C->h);
      const double row = ww[ic3(nx, ny, k, urow, i)];
      const double uw = (U + uY + lam * row) / (1.0 + lam);
      C->tyz[e] = wall == 0 ? 2.0 * muw * (row - uw) * inv_h : 2.0 * muw * (uw - row) * inv_h;
      if (write_wall) {
        C->uYz[(size_t)wall * wsz + b] = uY;
        C->slz[(size_t)wall * wsz + b] = uw - U;
      }
    }
    (void)sgt;
  }
  if (j < ny) {
    const unsigned c = ic3(nx, ny, k, j, i), cw = ic3(nx, ny, k, j, iw);
    const unsigned cbk = ic3(nx, ny, kb, j, i), cbw = ic3(nx, ny, kb, j, iw);
    const double mu4 = 0.25 * ((mud * ph[c] + mu2) + (mud * ph[cw] + mu2) + (mud * ph[cbk] + mu2) +
                               (mud * ph[cbw] + mu2));
    const double dudz = (uu[c] - uu[cbk]) * inv_h;
    const double dwdx = (ww[c] - ww[cw]) * inv_h;
    C->txz[c] = mu4 * (dudz + dwdx);
  }
}

// ------------------------------------------------------------ momentum + RK4
// L_phi, L_mx, L_my, L_mz at cell (k, j, i) (u, v, w of the cell's west,
// south and back faces), then the RK4 combination as in two dimensions.
// kst: stage 0..3 (< 0: evaluate only, into the accumulators); src, dst:
// phase-field buffers; c_next: RK c_{k+1} as a multiple of dt; b_k the RK4
// weight of the stage.
__global__ void __launch_bounds__(kNT3) k3_mom(const Ctx3* __restrict__ C, int kst, int src,
                                               int dst, double c_next, double b_k) {
  const int nx = C->nx, ny = C->ny, nz = C->nz;
  int k, j, i;
  if (!unflat3((long)blockIdx.x * kNT3 + threadIdx.x, nx, ny, nz, k, j, i)) return;
  const CDI_GLOBAL double* ph = src == 0 ? C->phi : (src == 1 ? C->phi_a : C->phi_b);
  const CDI_GLOBAL double* uu = kst <= 0 ? C->u : C->us;
  const CDI_GLOBAL double* vv = kst <= 0 ? C->v : C->vs;
  const CDI_GLOBAL double* ww = kst <= 0 ? C->w : C->ws;
  const double mud = C->mu1 - C->mu2, mu2 = C->mu2, inv_h = C->inv_h;
  const int ie = wrap3(i + 1, nx), iw = wrap3(i - 1, nx);
  const int kf = wrap3(k + 1, nz), kb = wrap3(k - 1, nz);
  const unsigned c = ic3(nx, ny, k, j, i);
  const unsigned ce = ic3(nx, ny, k, j, ie), cw = ic3(nx, ny, k, j, iw);
  const unsigned cf = ic3(nx, ny, kf, j, i), cb = ic3(nx, ny, kb, j, i);
  const unsigned e = iv3(nx, ny, k, j, i), en = e + nx;
  const double* Fx = C->Fx; const double* Fy = C->Fy; const double* Fz = C->Fz;
  const double* mx = C->fmx; const double* my = C->fmy; const double* mz = C->fmz;
  const double* muc = C->muc;
  auto mu = [&](unsigned o) { return mud * ph[o] + mu2; };

  const double Lphi = -((Fx[ce] - Fx[c]) + (Fy[en] - Fy[e]) + (Fz[cf] - Fz[c])) * inv_h;

  // ---- x-momentum at u (west x-face of the cell)
  double Lmx;
  {
    const double fcE = 0.5 * (mx[c] + mx[ce]) * 0.5 * (uu[c] + uu[ce]);
    const double fcW = 0.5 * (mx[cw] + mx[c]) * 0.5 * (uu[cw] + uu[c]);
    const double fyS = j == 0 ? 0.0
        : 0.5 * (my[iv3(nx, ny, k, j, iw)] + my[e]) * 0.5 * (uu[c - nx] + uu[c]);
    const double fyN = j + 1 >= ny ? 0.0
        : 0.5 * (my[iv3(nx, ny, k, j + 1, iw)] + my[en]) * 0.5 * (uu[c] + uu[c + nx]);
    const double fzB = 0.5 * (mz[cw] + mz[c]) * 0.5 * (uu[cb] + uu[c]);
    const double fzF = 0.5 * (mz[ic3(nx, ny, kf, j, iw)] + mz[cf]) * 0.5 * (uu[c] + uu[cf]);
    const double txxE = 2.0 * mu(c) * (uu[ce] - uu[c]) * inv_h;
    const double txxW = 2.0 * mu(cw) * (uu[c] - uu[cw]) * inv_h;
    const double st = 0.5 * (muc[cw] + muc[c]) * (ph[c] - ph[cw]) * inv_h;
    Lmx = -((fcE - fcW) + (fyN - fyS) + (fzF - fzB)) * inv_h + (txxE - txxW) * inv_h +
          (C->txy[en] - C->txy[e]) * inv_h + (C->txz[cf] - C->txz[c]) * inv_h + st;
  }
  // ---- y-momentum at interior v (south y-face of the cell)
  double Lmy = 0.0;
  if (j >= 1) {
    const unsigned cs = c - nx;
    const unsigned ee = iv3(nx, ny, k, j, ie), ew = iv3(nx, ny, k, j, iw);
    const unsigned ef = iv3(nx, ny, kf, j, i), eb = iv3(nx, ny, kb, j, i);
    const double fxE = 0.5 * (mx[ce - nx] + mx[ce]) * 0.5 * (vv[e] + vv[ee]);
    const double fxW = 0.5 * (mx[cs] + mx[c]) * 0.5 * (vv[ew] + vv[e]);
    const double gN = 0.5 * (my[e] + my[en]) * 0.5 * (vv[e] + vv[en]);
    const double gS = 0.5 * (my[e - nx] + my[e]) * 0.5 * (vv[e - nx] + vv[e]);
    const double fzB = 0.5 * (mz[cs] + mz[c]) * 0.5 * (vv[eb] + vv[e]);
    const double fzF = 0.5 * (mz[cf - nx] + mz[cf]) * 0.5 * (vv[e] + vv[ef]);
    const double tyyN = 2.0 * mu(c) * (vv[en] - vv[e]) * inv_h;
    const double tyyS = 2.0 * mu(cs) * (vv[e] - vv[e - nx]) * inv_h;
    const double st = 0.5 * (muc[cs] + muc[c]) * (ph[c] - ph[cs]) * inv_h;
    Lmy = -((fxE - fxW) + (gN - gS) + (fzF - fzB)) * inv_h + (tyyN - tyyS) * inv_h +
          (C->txy[ee] - C->txy[e]) * inv_h + (C->tyz[ef] - C->tyz[e]) * inv_h + st;
  }
  // ---- z-momentum at w (back z-face of the cell)
  double Lmz;
  {
    const unsigned cbe = ic3(nx, ny, kb, j, ie);
    const double fxE = 0.5 * (mx[cbe] + mx[ce]) * 0.5 * (ww[c] + ww[ce]);
    const double fxW = 0.5 * (mx[cb] + mx[c]) * 0.5 * (ww[cw] + ww[c]);
    const double fyS = j == 0 ? 0.0
        : 0.5 * (my[iv3(nx, ny, kb, j, i)] + my[e]) * 0.5 * (ww[c - nx] + ww[c]);
    const double fyN = j + 1 >= ny ? 0.0
        : 0.5 * (my[iv3(nx, ny, kb, j + 1, i)] + my[en]) * 0.5 * (ww[c] + ww[c + nx]);
    const double gF = 0.5 * (mz[c] + mz[cf]) * 0.5 * (ww[c] + ww[cf]);
    const double gB = 0.5 * (mz[cb] + mz[c]) * 0.5 * (ww[cb] + ww[c]);
    const double tzzF = 2.0 * mu(c) * (ww[cf] - ww[c]) * inv_h;
    const double tzzB = 2.0 * mu(cb) * (ww[c] - ww[cb]) * inv_h;
    const double st = 0.5 * (muc[cb] + muc[c]) * (ph[c] - ph[cb]) * inv_h;
    Lmz = -((fxE - fxW) + (fyN - fyS) + (gF - gB)) * inv_h + (tzzF - tzzB) * inv_h +
          (C->txz[ce] - C->txz[c]) * inv_h + (C->tyz[en] - C->tyz[e]) * inv_h + st;
  }
  if (kst < 0) {
    C->acc_phi[c] = Lphi;
    C->acc_mx[c] = Lmx;
    C->acc_mz[c] = Lmz;
    if (j >= 1) C->acc_my[e] = Lmy;
    return;
  }
  CDI_GLOBAL double* pdst = dst == 1 ? C->phi_a : C->phi_b;
  const double* p0 = C->phi;
  const double r1 = C->rho1, r2 = C->rho2;
  const double rc = (r1 - r2) * p0[c] + r2;
  const double mx0 = 0.5 * ((r1 - r2) * p0[cw] + r2 + rc) * C->u[c];
  const double mz0 = 0.5 * ((r1 - r2) * p0[cb] + r2 + rc) * C->w[c];
  const double cn = c_next * C->dt;
  double ap, am, az, an = 0.0;
  if (kst == 0) {
    ap = b_k * Lphi; am = b_k * Lmx; az = b_k * Lmz; an = b_k * Lmy;
  } else {
    ap = C->acc_phi[c] + b_k * Lphi;
    am = C->acc_mx[c] + b_k * Lmx;
    az = C->acc_mz[c] + b_k * Lmz;
    if (j >= 1) an = C->acc_my[e] + b_k * Lmy;
  }
  if (kst < 3) {
    C->acc_phi[c] = ap; C->acc_mx[c] = am; C->acc_mz[c] = az;
    pdst[c] = p0[c] + cn * Lphi;
    C->mx[c] = mx0 + cn * Lmx;
    C->mz[c] = mz0 + cn * Lmz;
  } else {
    pdst[c] = p0[c] + C->dt * ap;
    C->mx[c] = mx0 + C->dt * am;
    C->mz[c] = mz0 + C->dt * az;
  }
  if (j >= 1) {
    const double my0 = 0.5 * ((r1 - r2) * p0[c - nx] + r2 + rc) * C->v[e];
    if (kst < 3) {
      C->acc_my[e] = an;
      C->my[e] = my0 + cn * Lmy;
    } else {
      C->my[e] = my0 + C->dt * an;
    }
  }
}

// ------------------------------------------------------------ projection
// u* = m / rho_f(phi_next) on the cell's west, south, back faces, b =
// div(u*) / (tau dt) and the face coefficients 1/(rho_f h^2); partial sums
// of b.  src: the phase-field buffer of the stage result.
__global__ void __launch_bounds__(kNT3) k3_rhs(const Ctx3* __restrict__ C, int src, double tau) {
  const int nx = C->nx, ny = C->ny, nz = C->nz;
  int k, j, i;
  const bool in = unflat3((long)blockIdx.x * kNT3 + threadIdx.x, nx, ny, nz, k, j, i);
  double s[1] = {0.0};
  if (in) {
    const CDI_GLOBAL double* ph = src == 1 ? C->phi_a : C->phi_b;
    const double r1 = C->rho1, r2 = C->rho2;
    auto rho = [&](unsigned o) { return (r1 - r2) * ph[o] + r2; };
    const unsigned c = ic3(nx, ny, k, j, i);
    const unsigned ce = ic3(nx, ny, k, j, wrap3(i + 1, nx)), cw = ic3(nx, ny, k, j, wrap3(i - 1, nx));
    const unsigned cf = ic3(nx, ny, wrap3(k + 1, nz), j, i), cb = ic3(nx, ny, wrap3(k - 1, nz), j, i);
    const unsigned e = iv3(nx, ny, k, j, i);
    const double rc = rho(c);
    const double rfw = 0.5 * (rho(cw) + rc), rfe = 0.5 * (rc + rho(ce));
    const double rfb = 0.5 * (rho(cb) + rc), rff = 0.5 * (rc + rho(cf));
    const double uw = C->mx[c] / rfw, ue = C->mx[ce] / rfe;
    const double wb = C->mz[c] / rfb, wf = C->mz[cf] / rff;
    double vs = 0.0, vn = 0.0, rfs = 0.0;
    if (j >= 1) { rfs = 0.5 * (rho(c - nx) + rc); vs = C->my[e] / rfs; }
    if (j + 1 <= ny - 1) vn = C->my[e + nx] / (0.5 * (rc + rho(c + nx)));
    const double b = ((ue - uw) + (vn - vs) + (wf - wb)) * C->inv_h / (tau * C->dt);
    C->us[c] = uw;
    C->ws[c] = wb;
    if (j >= 1) C->vs[e] = vs;
    C->b[c] = b;
    const double ih2 = C->inv_h * C->inv_h;
    const Lev3& L0 = C->lev[0];
    L0.ax[c] = ih2 / rfw;
    L0.az[c] = ih2 / rfb;
    L0.ay[e] = j >= 1 ? ih2 / rfs : 0.0;
    if (j == ny - 1) L0.ay[e + nx] = 0.0;
    s[0] = b;
  }
  block_partials<1>(s, C->part);
}

// K x at cell (k, j, i) of a level: sum over non-wall faces of a_f (x - x_nb)
__device__ __forceinline__ double applyK3(const Lev3& L, const double* __restrict__ x, int k, int j,
                                          int i, double& diag, double& offs) {
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const unsigned c = ic3(nx, ny, k, j, i);
  const unsigned ce = ic3(nx, ny, k, j, wrap3(i + 1, nx)), cw = ic3(nx, ny, k, j, wrap3(i - 1, nx));
  const unsigned cf = ic3(nx, ny, wrap3(k + 1, nz), j, i), cb = ic3(nx, ny, wrap3(k - 1, nz), j, i);
  const unsigned e = iv3(nx, ny, k, j, i);
  const double aw = L.ax[c], ae = L.ax[ce], ab = L.az[c], af = L.az[cf];
  const double as = L.ay[e], an = L.ay[e + nx];   // 0 on wall faces
  double s = aw * x[cw] + ae * x[ce] + ab * x[cb] + af * x[cf];
  if (j >= 1) s += as * x[c - nx];
  if (j + 1 < ny) s += an * x[c + nx];
  diag = aw + ae + ab + af + as + an;
  offs = s;
  return diag * x[c] - s;
}

// Initial guess x0 of a solve into C->x: the state's pressure (q < 0), or
// the polynomial extrapolation in time of order q (0..3) of the same RK
// stage's pressure through the last q + 1 steps, slot[0] the newest (0: the
// last step's pressure, 1: 2 p1 - p2, 2: 3 p1 - 3 p2 + p3, 3: 4 p1 - 6 p2 +
// 4 p3 - p4).  Only the starting point of the solve depends on it.
struct Guess3 {
  int stage, q;
  int slot[4];
};
__global__ void __launch_bounds__(kNT3) k3_guess(const Ctx3* __restrict__ C, Guess3 g) {
  const long n = (long)C->nx * C->ny * C->nz;
  const long c = (long)blockIdx.x * kNT3 + threadIdx.x;
  if (c >= n) return;
  if (g.q < 0) {
    C->x[c] = C->p[c];
    return;
  }
  const double p1 = C->hp[g.slot[0]][g.stage][c];
  double x = p1;
  if (g.q == 1) {
    x = 2.0 * p1 - C->hp[g.slot[1]][g.stage][c];
  } else if (g.q == 2) {
    x = 3.0 * (p1 - C->hp[g.slot[1]][g.stage][c]) + C->hp[g.slot[2]][g.stage][c];
  } else if (g.q == 3) {
    const double p2 = C->hp[g.slot[1]][g.stage][c], p3 = C->hp[g.slot[2]][g.stage][c];
    x = 4.0 * (p1 + p3) - 6.0 * p2 - C->hp[g.slot[3]][g.stage][c];
  }
  C->x[c] = x;
}

// r0 = f - K x0 with f = -(b - mean b); guess != 0: x0 is in C->x (k3_guess),
// else x0 = 0.  Partial sums of f^2, r^2.
__global__ void __launch_bounds__(kNT3) k3_pcg_init(const Ctx3* __restrict__ C, int guess) {
  const Lev3& L = C->lev[0];
  int k, j, i;
  const bool in = unflat3((long)blockIdx.x * kNT3 + threadIdx.x, L.nx, L.ny, L.nz, k, j, i);
  double s[2] = {0.0, 0.0};
  if (in) {
    const unsigned c = ic3(L.nx, L.ny, k, j, i);
    const double f = -(C->b[c] - C->scal[S_BMEAN]);
    double r = f;
    if (guess) {
      double dg, of;
      r = f - applyK3(L, C->x, k, j, i, dg, of);
    } else {
      C->x[c] = 0.0;
    }
    C->r[c] = r;
    s[0] = f * f;
    s[1] = r * r;
  }
  block_partials<2>(s, C->part);
}

// q = K d; partial sums of (d, q).
__global__ void __launch_bounds__(kNT3) k3_spmv(const Ctx3* __restrict__ C) {
  const Lev3& L = C->lev[0];
  int k, j, i;
  const bool in = unflat3((long)blockIdx.x * kNT3 + threadIdx.x, L.nx, L.ny, L.nz, k, j, i);
  double s[1] = {0.0};
  if (in) {
    const unsigned c = ic3(L.nx, L.ny, k, j, i);
    double dg, of;
    const double q = applyK3(L, C->d, k, j, i, dg, of);
    C->q[c] = q;
    s[0] = C->d[c] * q;
  }
  block_partials<1>(s, C->part);
}

// x += alpha d, r -= alpha q (alpha = (r, z)/(d, q)); partial sums of r^2.
__global__ void __launch_bounds__(kNT3) k3_update(const Ctx3* __restrict__ C) {
  const long g = (long)blockIdx.x * kNT3 + threadIdx.x;
  const long n = (long)C->nx * C->ny * C->nz;
  double s[1] = {0.0};
  if (g < n) {
    const double alpha = C->scal[S_ALPHA];
    C->x[g] += alpha * C->d[g];
    const double r = C->r[g] - alpha * C->q[g];
    C->r[g] = r;
    s[0] = r * r;
  }
  block_partials<1>(s, C->part);
}

// partial sums of (r, z) and (q, z)
__global__ void __launch_bounds__(kNT3) k3_dot_rz(const Ctx3* __restrict__ C) {
  const long g = (long)blockIdx.x * kNT3 + threadIdx.x;
  const long n = (long)C->nx * C->ny * C->nz;
  double s[2] = {0.0, 0.0};
  if (g < n) {
    s[0] = C->r[g] * C->z[g];
    s[1] = C->q[g] * C->z[g];
  }
  block_partials<2>(s, C->part);
}

// d = z + beta d with the flexible (Polak-Ribiere) beta = (z, r - r_old) /
// (z_old, r_old) = -alpha (z, q) / (z_old, r_old), since r - r_old = -alpha q;
// d = z on the first iteration.
__global__ void __launch_bounds__(kNT3) k3_dir(const Ctx3* __restrict__ C, int first) {
  const long g = (long)blockIdx.x * kNT3 + threadIdx.x;
  const long n = (long)C->nx * C->ny * C->nz;
  if (g >= n) return;
  const double beta = first ? 0.0 : -C->scal[S_ALPHA] * C->scal[S_ZQ] / C->scal[S_RZOLD];
  C->d[g] = C->z[g] + beta * C->d[g];
}

// block maxima of |u|, |v|, |w| over the faces (the step's gamma)
__global__ void __launch_bounds__(kNT3) k3_absmax(const Ctx3* __restrict__ C) {
  const int nx = C->nx, ny = C->ny, nz = C->nz;
  int k, j, i;
  const bool in = unflat3((long)blockIdx.x * kNT3 + threadIdx.x, nx, ny, nz, k, j, i);
  double m = 0.0;
  if (in) {
    const unsigned c = ic3(nx, ny, k, j, i);
    m = fmax(fmax(fabs(C->u[c]), fabs(C->w[c])), fabs(C->v[iv3(nx, ny, k, j, i)]));
  }
  __shared__ double sm[kNT3 / 64];
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = sm[0];
    for (int wv = 1; wv < kNT3 / 64; ++wv) v = fmax(v, sm[wv]);
    C->part[blockIdx.x] = v;
  }
}

// gamma of the step = min(gamma, factor * max |u|) from nb block maxima
__global__ void __launch_bounds__(1024) k3_gamma(const Ctx3* __restrict__ C, int nb, double gamma,
                                                 double factor) {
  __shared__ double sm[16];
  double m = 0.0;
  for (int t = threadIdx.x; t < nb; t += 1024) m = fmax(m, C->part[t]);
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = sm[0];
    for (int wv = 1; wv < 16; ++wv) v = fmax(v, sm[wv]);
    C->scal[S_VMAX] = v;
    C->scal[S_GAMMA] = factor > 0.0 ? fmin(gamma, factor * v) : gamma;
  }
}

// partial sums of x (for the mean-free pressure)
__global__ void __launch_bounds__(kNT3) k3_sum_x(const Ctx3* __restrict__ C) {
  const long g = (long)blockIdx.x * kNT3 + threadIdx.x;
  const long n = (long)C->nx * C->ny * C->nz;
  double s[1] = {0.0};
  if (g < n) s[0] = C->x[g];
  block_partials<1>(s, C->part);
}

// One block: sum nb partials (one or two sums) in a fixed order and derive
// the scalars.  what: 0 b -> S_BMEAN; 1 (f^2, r^2) -> S_FF, S_RR, S_RELRES;
// 2 (d, q) -> S_DQ, S_ALPHA = S_RZ / S_DQ; 3 r^2 -> S_RR, S_RELRES;
// 4 ((r, z), (q, z)) -> S_RZOLD <- S_RZ, S_RZ, S_ZQ; 5 x -> S_XMEAN.
__global__ void __launch_bounds__(1024) k3_finalize(const Ctx3* __restrict__ C, int nb, int what) {
  __shared__ double sh[2][1024 / 64];
  const int nv = (what == 1 || what == 4) ? 2 : 1;
  double acc[2] = {0.0, 0.0};
  for (int q = 0; q < nv; ++q)
    for (int t = threadIdx.x; t < nb; t += 1024) acc[q] += C->part[(size_t)q * nb + t];
  for (int q = 0; q < 2; ++q) {
    double s = acc[q];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) sh[q][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double t[2] = {0.0, 0.0};
  for (int q = 0; q < 2; ++q)
    for (int wv = 0; wv < 16; ++wv) t[q] += sh[q][wv];
  double* S = C->scal;
  const double n = (double)C->nx * C->ny * C->nz;
  switch (what) {
    case 0: S[S_BMEAN] = t[0] / n; break;
    case 1:
      S[S_FF] = t[0]; S[S_RR] = t[1];
      S[S_RELRES] = t[0] > 0.0 ? sqrt(t[1] / t[0]) : 0.0;
      if (!isfinite(t[0]) || !isfinite(t[1])) S[S_RELRES] = NAN;
      break;
    case 2: S[S_DQ] = t[0]; S[S_ALPHA] = S[S_RZ] / t[0]; break;
    case 3:
      S[S_RR] = t[0];
      S[S_RELRES] = S[S_FF] > 0.0 ? sqrt(t[0] / S[S_FF]) : 0.0;
      if (!isfinite(t[0])) S[S_RELRES] = NAN;
      break;
    case 4: S[S_RZOLD] = S[S_RZ]; S[S_RZ] = t[0]; S[S_ZQ] = t[1]; break;
    default: S[S_XMEAN] = t[0] / n; break;
  }
}

// u = u* - tau grad p / rho_f on every face (v on interior y-faces); p = x -
// mean(x) is stored as the state's pressure and, with hslot >= 0, as RK stage
// `stage`'s entry hp[hslot] of the pressure history.  final: the new state
// (caller u, v, w; phi copied from phi_b), else the next stage's velocity (in
// place).
__global__ void __launch_bounds__(kNT3) k3_project(const Ctx3* __restrict__ C, int src, double tau,
                                                   int final_stage, int hslot, int stage) {
  const int nx = C->nx, ny = C->ny, nz = C->nz;
  int k, j, i;
  if (!unflat3((long)blockIdx.x * kNT3 + threadIdx.x, nx, ny, nz, k, j, i)) return;
  const CDI_GLOBAL double* ph = src == 1 ? C->phi_a : C->phi_b;
  const double r1 = C->rho1, r2 = C->rho2;
  auto rho = [&](unsigned o) { return (r1 - r2) * ph[o] + r2; };
  const double xm = C->scal[S_XMEAN];
  const unsigned c = ic3(nx, ny, k, j, i);
  const unsigned cw = ic3(nx, ny, k, j, wrap3(i - 1, nx)), cb = ic3(nx, ny, wrap3(k - 1, nz), j, i);
  const unsigned e = iv3(nx, ny, k, j, i);
  const double pc = C->x[c] - xm;
  const double fac = tau * C->dt * C->inv_h;
  const double rc = rho(c);
  const double un = C->us[c] - fac * (pc - (C->x[cw] - xm)) / (0.5 * (rho(cw) + rc));
  const double wn = C->ws[c] - fac * (pc - (C->x[cb] - xm)) / (0.5 * (rho(cb) + rc));
  double vn = 0.0;
  if (j >= 1) vn = C->vs[e] - fac * (pc - (C->x[c - nx] - xm)) / (0.5 * (rho(c - nx) + rc));
  CDI_GLOBAL double* uo = final_stage ? C->u : C->us;
  CDI_GLOBAL double* vo = final_stage ? C->v : C->vs;
  CDI_GLOBAL double* wo = final_stage ? C->w : C->ws;
  uo[c] = un;
  wo[c] = wn;
  vo[e] = vn;                       // row 0: the wall (v = 0)
  if (j == ny - 1) vo[e + nx] = 0.0;
  C->p[c] = pc;
  if (hslot >= 0) C->hp[hslot][stage][c] = pc;
  if (final_stage) C->phi[c] = ph[c];
}

// ------------------------------------------------------------ multigrid
// Coarse coefficients of level l + 1 from level l: each coarse face takes the
// mean of the four fine faces it covers, divided by 4 (h doubles).
__global__ void __launch_bounds__(kNT3) k3_mg_coef(const Ctx3* __restrict__ C, int l) {
  const Lev3& F = C->lev[l];
  const Lev3& G = C->lev[l + 1];
  int k, j, i;
  if (!unflat3((long)blockIdx.x * kNT3 + threadIdx.x, G.nx, G.ny + 1, G.nz, k, j, i)) return;
  const int fi = 2 * i, fj = 2 * j, fk = 2 * k;
  const double q = 0.25 * 0.25;
  if (j < G.ny) {
    const unsigned c = ic3(G.nx, G.ny, k, j, i);
    G.ax[c] = q * (F.ax[ic3(F.nx, F.ny, fk, fj, fi)] + F.ax[ic3(F.nx, F.ny, fk, fj + 1, fi)] +
                   F.ax[ic3(F.nx, F.ny, fk + 1, fj, fi)] + F.ax[ic3(F.nx, F.ny, fk + 1, fj + 1, fi)]);
    G.az[c] = q * (F.az[ic3(F.nx, F.ny, fk, fj, fi)] + F.az[ic3(F.nx, F.ny, fk, fj + 1, fi)] +
                   F.az[ic3(F.nx, F.ny, fk, fj, fi + 1)] + F.az[ic3(F.nx, F.ny, fk, fj + 1, fi + 1)]);
  }
  const unsigned e = iv3(G.nx, G.ny, k, j, i);
  if (j == 0 || j == G.ny) {
    G.ay[e] = 0.0;
  } else {
    G.ay[e] = q * (F.ay[iv3(F.nx, F.ny, fk, fj, fi)] + F.ay[iv3(F.nx, F.ny, fk, fj, fi + 1)] +
                   F.ay[iv3(F.nx, F.ny, fk + 1, fj, fi)] + F.ay[iv3(F.nx, F.ny, fk + 1, fj, fi + 1)]);
  }
}

// One red-black Gauss-Seidel half-sweep on level l: cells of colour
// (i + j + k) & 1 == color take x = (r + sum a x_nb) / sum a.  One thread per
// pair of cells (2m, 2m + 1) of a row (the level's nx is even), updating the
// one of the colour; zero: the first half-sweep from x = 0 (the colour cell
// r / D, the other cell of the pair 0).
__global__ void __launch_bounds__(kNT3) k3_mg_smooth(const Ctx3* __restrict__ C, int l, int color,
                                                     int zero) {
  const Lev3& L = C->lev[l];
  const int hx = L.nx >> 1;
  const long t = (long)blockIdx.x * kNT3 + threadIdx.x;
  if (t >= (long)hx * L.ny * L.nz) return;
  const int row = quot3((int)t, hx);
  const int m = (int)t - row * hx;
  const int k = quot3(row, L.ny), j = row - k * L.ny;
  const int i = 2 * m + ((j + k + color) & 1);
  const unsigned c = ic3(L.nx, L.ny, k, j, i);
  if (zero) {
    const unsigned e = iv3(L.nx, L.ny, k, j, i);
    const double D = L.ax[c] + L.ax[ic3(L.nx, L.ny, k, j, wrap3(i + 1, L.nx))] + L.az[c] +
                     L.az[ic3(L.nx, L.ny, wrap3(k + 1, L.nz), j, i)] + L.ay[e] + L.ay[e + L.nx];
    L.x[c] = L.r[c] / D;
    L.x[c ^ 1u] = 0.0;   // the other cell of the pair (row offsets are even)
    return;
  }
  double D, s;
  (void)applyK3(L, L.x, k, j, i, D, s);
  L.x[c] = (L.r[c] + s) / D;
}

// r_{l+1} = mean over the 8 children of (r - K x) on level l.
__global__ void __launch_bounds__(kNT3) k3_mg_restrict(const Ctx3* __restrict__ C, int l) {
  const Lev3& F = C->lev[l];
  const Lev3& G = C->lev[l + 1];
  int k, j, i;
  if (!unflat3((long)blockIdx.x * kNT3 + threadIdx.x, G.nx, G.ny, G.nz, k, j, i)) return;
  double s = 0.0;
  for (int dk = 0; dk < 2; ++dk)
    for (int dj = 0; dj < 2; ++dj)
      for (int di = 0; di < 2; ++di) {
        const int fk = 2 * k + dk, fj = 2 * j + dj, fi = 2 * i + di;
        double D, o;
        const double kx = applyK3(F, F.x, fk, fj, fi, D, o);
        s += F.r[ic3(F.nx, F.ny, fk, fj, fi)] - kx;
      }
  G.r[ic3(G.nx, G.ny, k, j, i)] = 0.125 * s;
}

// x_l += P x_{l+1}: trilinear interpolation between cell centres (weights
// 3/4 and 1/4 per direction), periodic in x and z, reflected at the walls.
__global__ void __launch_bounds__(kNT3) k3_mg_prolong(const Ctx3* __restrict__ C, int l) {
  const Lev3& F = C->lev[l];
  const Lev3& G = C->lev[l + 1];
  int k, j, i;
  if (!unflat3((long)blockIdx.x * kNT3 + threadIdx.x, F.nx, F.ny, F.nz, k, j, i)) return;
  const int I = i >> 1, J = j >> 1, K = k >> 1;
  const int I2 = wrap3(I + ((i & 1) ? 1 : -1), G.nx);
  const int K2 = wrap3(K + ((k & 1) ? 1 : -1), G.nz);
  int J2 = J + ((j & 1) ? 1 : -1);
  if (J2 < 0 || J2 >= G.ny) J2 = J;
  const int is[2] = {I, I2}, js[2] = {J, J2}, ks[2] = {K, K2};
  const double wgt[2] = {0.75, 0.25};
  double s = 0.0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int cc = 0; cc < 2; ++cc)
        s += wgt[a] * wgt[b] * wgt[cc] * G.x[ic3(G.nx, G.ny, ks[a], js[b], is[cc])];
  F.x[ic3(F.nx, F.ny, k, j, i)] += s;
}

// The coarsest level in one block (at most kCoarseMax3 cells, one per
// thread): 2 kCoarseSweeps3 + 1 red-black half-sweeps from zero, red first
// and last (a palindromic sequence keeps the preconditioner symmetric).  Each
// thread keeps its cell's six face coefficients, neighbour indices and
// right-hand side in registers; the correction lives in LDS.
__global__ void __launch_bounds__(kCoarseMax3) k3_mg_coarse(const Ctx3* __restrict__ C, int l) {
  __shared__ double sx[kCoarseMax3];
  const Lev3& L = C->lev[l];
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const int n = nx * ny * nz;
  const int t = threadIdx.x;
  const bool in = t < n;
  double a[6] = {0, 0, 0, 0, 0, 0}, D = 1.0, rr = 0.0;
  int nb[6] = {0, 0, 0, 0, 0, 0};
  int color = 0;
  if (in) {
    const int i = t % nx, j = (t / nx) % ny, k = t / (nx * ny);
    color = (i + j + k) & 1;
    const unsigned e = iv3(nx, ny, k, j, i);
    nb[0] = (int)ic3(nx, ny, k, j, wrap3(i - 1, nx));
    nb[1] = (int)ic3(nx, ny, k, j, wrap3(i + 1, nx));
    nb[2] = (int)ic3(nx, ny, wrap3(k - 1, nz), j, i);
    nb[3] = (int)ic3(nx, ny, wrap3(k + 1, nz), j, i);
    nb[4] = j >= 1 ? t - nx : t;          // wall faces carry a zero coefficient
    nb[5] = j + 1 < ny ? t + nx : t;
    a[0] = L.ax[t]; a[1] = L.ax[nb[1]]; a[2] = L.az[t]; a[3] = L.az[nb[3]];
    a[4] = L.ay[e]; a[5] = L.ay[e + nx];
    D = a[0] + a[1] + a[2] + a[3] + a[4] + a[5];
    rr = L.r[t];
  }
  sx[t] = 0.0;
  __syncthreads();
  for (int it = 0; it < 2 * kCoarseSweeps3 + 1; ++it) {
    if (in && color == (it & 1)) {
      const double s = a[0] * sx[nb[0]] + a[1] * sx[nb[1]] + a[2] * sx[nb[2]] + a[3] * sx[nb[3]] +
                       a[4] * sx[nb[4]] + a[5] * sx[nb[5]];
      sx[t] = D > 0.0 ? (rr + s) / D : 0.0;
    }
    __syncthreads();
  }
  if (in) L.x[t] = sx[t];
}

// ------------------------------------------------------------ diagnostics
// partials: mass, ke, max |div| (as sums of per-block maxima are wrong, the
// maxima use a second array); one block per 256 cells.
__global__ void __launch_bounds__(kNT3) k3_diag(const Ctx3* __restrict__ C,
                                                double* __restrict__ out) {
  const int nx = C->nx, ny = C->ny, nz = C->nz;
  int k, j, i;
  const bool in = unflat3((long)blockIdx.x * kNT3 + threadIdx.x, nx, ny, nz, k, j, i);
  double s[2] = {0.0, 0.0};
  double mx[3] = {-INFINITY, -INFINITY, -INFINITY};   // max phi, -min phi, max |div|
  if (in) {
    const double r1 = C->rho1, r2 = C->rho2;
    const unsigned c = ic3(nx, ny, k, j, i);
    const unsigned ce = ic3(nx, ny, k, j, wrap3(i + 1, nx)), cw = ic3(nx, ny, k, j, wrap3(i - 1, nx));
    const unsigned cf = ic3(nx, ny, wrap3(k + 1, nz), j, i), cb = ic3(nx, ny, wrap3(k - 1, nz), j, i);
    const unsigned e = iv3(nx, ny, k, j, i);
    const double f = C->phi[c];
    auto rho = [&](unsigned o) { return (r1 - r2) * C->phi[o] + r2; };
    const double rc = rho(c);
    s[0] = f;
    double ke = 0.5 * (rho(cw) + rc) * C->u[c] * C->u[c] + 0.5 * (rho(cb) + rc) * C->w[c] * C->w[c];
    if (j >= 1) ke += 0.5 * (rho(c - nx) + rc) * C->v[e] * C->v[e];
    s[1] = ke;
    const double div = ((C->u[ce] - C->u[c]) + (C->v[e + nx] - C->v[e]) + (C->w[cf] - C->w[c])) *
                       C->inv_h;
    mx[0] = f; mx[1] = -f; mx[2] = fabs(div);
  }
  block_partials<2>(s, out);
  __shared__ double sm[3][kNT3 / 64];
  for (int q = 0; q < 3; ++q) {
    double v = mx[q];
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) sm[q][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) {
      double v = sm[q][0];
      for (int wv = 1; wv < kNT3 / 64; ++wv) v = fmax(v, sm[q][wv]);
      out[(size_t)(2 + q) * gridDim.x + blockIdx.x] = v;
    }
}

}  // namespace cdi3
