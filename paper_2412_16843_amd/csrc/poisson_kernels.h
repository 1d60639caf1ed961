// Variable-density pressure projection: right-hand side, flexible CG with a
// geometric multigrid V-cycle preconditioner, and the velocity correction.
//
// Operator (the paper leaves the pressure coupling to its references; this
// is the plain second-order staggered reading): K p = sum over a cell's
// non-wall faces of a_f (p - p_nb), a_f = 1/(rho_f h^2), rho_f the mean of the
// two adjacent cell densities, x periodic.  K is the negative of the
// Laplacian-like operator A; the projection solves A p = div(u*)/tau - mean,
// i.e. K p = f with f = -(b - mean(b)).
//
// Multigrid: cell-centred, bilinear prolongation P (Neumann reflection at the
// walls), restriction R = P^T / 4, coarse coefficients averaged from the two
// fine faces covering each coarse face and scaled by 1/4 (h doubles), one
// red-black Gauss-Seidel sweep before (red, black) and after (black, red)
// the coarse correction so that the V-cycle is symmetric; the coarsest grid
// is solved by CG inside one block.  Levels at or below kCoarseCells cells
// run inside a single-block kernel; finer levels use LDS-tiled kernels whose
// tiles span every instance of a batch.
#pragma once
#include "stage_kernels.h"

namespace cdi {

constexpr int kCoarseCells = 4096;
constexpr int kCoarseNT = 512;
constexpr int FX = 32, FY = 16;            // fine tile of the multigrid kernels
static_assert(FX * FY == 2 * kNT, "MG tile = 2 cells per thread");

// ------------------------------------------------------------ projection RHS
// u* = (rho u)* / rho_f(phi_next) on the faces of every cell, b = div(u*)/tau
// (tau given as a multiple of the instance time step),
// the FP64 face coefficients of the pressure operator (and their S copy for
// the V-cycle), and the instance's sum of b.  Resets the CG state.
template <typename S>
__global__ void __launch_bounds__(kNT) k_rhs(const Tile* __restrict__ tiles,
                                              const Inst* __restrict__ insts, int src, double tau,
                                              double rtol, int maxit) {
  __shared__ double sh[kNT / 64];
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  const int nx = I.nx, ny = I.ny;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int i = t.i0 + tx, j = t.j0 + ty;
  const double* __restrict__ ph = src == 0 ? I.phi : (src == 1 ? I.phi_a : I.phi_b);
  double bsum[1] = {0.0};
  if (i < nx && j < ny) {
    const size_t o = (size_t)j * nx + i;
    const int ie = wrap(i + 1, nx), iw = wrap(i - 1, nx);
    const double r1 = I.rho1, r2 = I.rho2;
    const double rc = (r1 - r2) * ph[o] + r2;
    const double rw = (r1 - r2) * ph[(size_t)j * nx + iw] + r2;
    const double re = (r1 - r2) * ph[(size_t)j * nx + ie] + r2;
    const double rfw = 0.5 * (rw + rc), rfe = 0.5 * (rc + re);
    const double uw = I.mx[o] / rfw;
    const double ue = I.mx[(size_t)j * nx + ie] / rfe;
    double vs = 0.0, vn = 0.0, rfs = 0.0, rfn = 0.0;
    if (j >= 1) {
      const double rs = (r1 - r2) * ph[o - nx] + r2;
      rfs = 0.5 * (rs + rc);
      vs = I.my[o] / rfs;
    }
    if (j + 1 <= ny - 1) {
      const double rn = (r1 - r2) * ph[o + nx] + r2;
      rfn = 0.5 * (rc + rn);
      vn = I.my[o + nx] / rfn;
    }
    const double b = ((ue - uw) + (vn - vs)) * I.inv_h / (tau * I.dt);
    I.ustar[o] = uw;
    I.vstar[o] = vs;
    I.b[o] = b;
    bsum[0] = b;
    const double ih2 = I.inv_h * I.inv_h;
    const double ax = ih2 / rfw;
    const double ay = j >= 1 ? ih2 / rfs : 0.0;
    I.ax0[o] = ax;
    I.ay0[o] = ay;
    if (I.mixed) {
      ((S*)I.lev[0].ax)[o] = (S)ax;
      ((S*)I.lev[0].ay)[o] = (S)ay;
    }
  }
  block_sum<1>(bsum, sh);
  if (threadIdx.x == 0) I.part[t.local] = bsum[0];
  if (arrive_last(&I.pcg->counter[0], I.ntiles)) {
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int k = 0; k < I.ntiles; ++k) s += ld_agent(&I.part[k]);
      PcgScalars* P = I.pcg;
      P->bmean = s / ((double)nx * ny);
      P->done = 0; P->iters = 0; P->first = 1; P->converged = 0; P->pad = 0;
      P->rtol = rtol; P->maxit = maxit;
    }
  }
}

// K x on a cell from FP64 neighbours (x periodic, wall faces omitted)
__device__ __forceinline__ double apply_K(const Inst& I, const double* __restrict__ x, int j, int i) {
  const int nx = I.nx, ny = I.ny;
  const size_t o = (size_t)j * nx + i;
  const int ie = wrap(i + 1, nx), iw = wrap(i - 1, nx);
  const double xc = x[o];
  const double aw = I.ax0[o], ae = I.ax0[(size_t)j * nx + ie];
  double s = aw * (xc - x[(size_t)j * nx + iw]) + ae * (xc - x[(size_t)j * nx + ie]);
  if (j >= 1) s += I.ay0[o] * (xc - x[o - nx]);
  if (j + 1 < ny) s += I.ay0[o + nx] * (xc - x[o + nx]);
  return s;
}

// f = -(b - mean b); x0 = guess (previous pressure) or 0; r = f - K x0.
__global__ void __launch_bounds__(kNT) k_pcg_init(const Tile* __restrict__ tiles,
                                                  const Inst* __restrict__ insts, int guess) {
  __shared__ double sh[2 * kNT / 64];
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  const int nx = I.nx, ny = I.ny;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int i = t.i0 + tx, j = t.j0 + ty;
  double s[2] = {0.0, 0.0};
  if (i < nx && j < ny) {
    const size_t o = (size_t)j * nx + i;
    const double f = -(I.b[o] - I.pcg->bmean);
    double r = f;
    if (guess) {
      r = f - apply_K(I, I.p, j, i);
      I.x[o] = I.p[o];
    } else {
      I.x[o] = 0.0;
    }
    I.rr[o] = r;
    s[0] = f * f;
    s[1] = r * r;
  }
  block_sum<2>(s, sh);
  if (threadIdx.x == 0) {
    I.part[t.local] = s[0];
    I.part[I.ntiles + t.local] = s[1];
  }
  if (arrive_last(&I.pcg->counter[1], I.ntiles)) {
    if (threadIdx.x == 0) {
      double ff = 0.0, rr = 0.0;
      for (int k = 0; k < I.ntiles; ++k) ff += ld_agent(&I.part[k]);
      for (int k = 0; k < I.ntiles; ++k) rr += ld_agent(&I.part[I.ntiles + k]);
      PcgScalars* P = I.pcg;
      P->fnorm = sqrt(ff);
      P->rr = rr;
      if (ff == 0.0) {          // b = 0: the mean-free solution is p = 0
        P->relres = 0.0; P->done = 1; P->converged = 1; P->pad = 1;
      } else {
        P->relres = sqrt(rr) / P->fnorm;
        if (P->relres <= P->rtol) { P->done = 1; P->converged = 1; }
      }
    }
  }
}

// d = z + beta d_old (d = z on the first iteration), q = K d, (d, r), (d, q);
// last block: alpha = (d, r)/(d, q).
__global__ void __launch_bounds__(kNT) k_pcg_spmv(const Tile* __restrict__ tiles,
                                                  const Inst* __restrict__ insts, int parity) {
  __shared__ double sh[2 * kNT / 64];
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (I.pcg->done) return;
  const int nx = I.nx, ny = I.ny;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int i = t.i0 + tx, j = t.j0 + ty;
  const double* __restrict__ dold = parity ? I.d0 : I.d1;
  double* __restrict__ dnew = parity ? I.d1 : I.d0;
  const double* __restrict__ z = I.zf;
  const bool first = I.pcg->first != 0;
  const double beta = first ? 0.0 : I.pcg->beta;
  double s[2] = {0.0, 0.0};
  if (i < nx && j < ny) {
    const size_t o = (size_t)j * nx + i;
    auto dval = [&](size_t idx) { return first ? z[idx] : z[idx] + beta * dold[idx]; };
    const int ie = wrap(i + 1, nx), iw = wrap(i - 1, nx);
    const double dc = dval(o);
    double q = I.ax0[o] * (dc - dval((size_t)j * nx + iw)) +
               I.ax0[(size_t)j * nx + ie] * (dc - dval((size_t)j * nx + ie));
    if (j >= 1) q += I.ay0[o] * (dc - dval(o - nx));
    if (j + 1 < ny) q += I.ay0[o + nx] * (dc - dval(o + nx));
    dnew[o] = dc;
    I.q[o] = q;
    s[0] = dc * I.rr[o];
    s[1] = dc * q;
  }
  block_sum<2>(s, sh);
  if (threadIdx.x == 0) {
    I.part[t.local] = s[0];
    I.part[I.ntiles + t.local] = s[1];
  }
  if (arrive_last(&I.pcg->counter[2], I.ntiles)) {
    if (threadIdx.x == 0) {
      double dr = 0.0, dq = 0.0;
      for (int k = 0; k < I.ntiles; ++k) dr += ld_agent(&I.part[k]);
      for (int k = 0; k < I.ntiles; ++k) dq += ld_agent(&I.part[I.ntiles + k]);
      PcgScalars* P = I.pcg;
      P->dr = dr; P->dq = dq;
      P->alpha = dq != 0.0 ? dr / dq : 0.0;
      P->first = 0;
    }
  }
}

// x += alpha d, r -= alpha q; last block: relres = ||r|| / ||f||, stop test.
__global__ void __launch_bounds__(kNT) k_pcg_update(const Tile* __restrict__ tiles,
                                                    const Inst* __restrict__ insts, int parity) {
  __shared__ double sh[2 * kNT / 64];
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (I.pcg->done) return;
  const int nx = I.nx, ny = I.ny;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int i = t.i0 + tx, j = t.j0 + ty;
  const double* __restrict__ d = parity ? I.d1 : I.d0;
  const double alpha = I.pcg->alpha;
  double s[2] = {0.0, 0.0};
  if (i < nx && j < ny) {
    const size_t o = (size_t)j * nx + i;
    const double x = I.x[o] + alpha * d[o];
    const double r = I.rr[o] - alpha * I.q[o];
    I.x[o] = x;
    I.rr[o] = r;
    s[0] = r * r;
    s[1] = x;
  }
  block_sum<2>(s, sh);
  if (threadIdx.x == 0) {
    I.part[t.local] = s[0];
    I.part[I.ntiles + t.local] = s[1];
  }
  if (arrive_last(&I.pcg->counter[3], I.ntiles)) {
    if (threadIdx.x == 0) {
      double rr = 0.0, sx = 0.0;
      for (int k = 0; k < I.ntiles; ++k) rr += ld_agent(&I.part[k]);
      for (int k = 0; k < I.ntiles; ++k) sx += ld_agent(&I.part[I.ntiles + k]);
      PcgScalars* P = I.pcg;
      P->rr = rr;
      P->xmean = sx / ((double)nx * ny);
      P->iters += 1;
      P->relres = sqrt(rr) / P->fnorm;
      if (P->relres <= P->rtol) { P->done = 1; P->converged = 1; }
      else if (P->iters >= P->maxit) { P->done = 1; }
    }
  }
}

// Mean of the solution when the solve ended before any CG update.
__global__ void __launch_bounds__(kNT) k_pcg_xmean(const Tile* __restrict__ tiles,
                                                   const Inst* __restrict__ insts) {
  __shared__ double sh[kNT / 64];
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  const int nx = I.nx, ny = I.ny;
  if (I.pcg->iters > 0) return;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int i = t.i0 + tx, j = t.j0 + ty;
  double s[1] = {0.0};
  if (i < nx && j < ny) s[0] = I.x[(size_t)j * nx + i];
  block_sum<1>(s, sh);
  if (threadIdx.x == 0) I.part[t.local] = s[0];
  if (arrive_last(&I.pcg->counter[6], I.ntiles)) {
    if (threadIdx.x == 0) {
      double sx = 0.0;
      for (int k = 0; k < I.ntiles; ++k) sx += ld_agent(&I.part[k]);
      I.pcg->xmean = sx / ((double)nx * ny);
    }
  }
}

// u = u* - tau grad(p)/rho_f on interior faces (tau a multiple of the
// instance time step); the pressure is stored
// mean-free.  final_stage: the result is the new state (caller fields) and
// the new phase field is copied from phi_next.
__global__ void __launch_bounds__(kNT) k_project(const Tile* __restrict__ tiles,
                                                 const Inst* __restrict__ insts, double tau,
                                                 int final_stage, int src) {
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  const int nx = I.nx, ny = I.ny;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int i = t.i0 + tx, j = t.j0 + ty;
  if (i >= nx || j >= ny) return;
  const size_t o = (size_t)j * nx + i;
  const bool zero = I.pcg->pad != 0;
  const double* __restrict__ x = I.x;
  const double xc = zero ? 0.0 : x[o];
  const double xw = zero ? 0.0 : x[(size_t)j * nx + wrap(i - 1, nx)];
  const double scale = tau * I.dt * I.h;   // tau grad(p)/rho_f = tau (p_c - p_w) h a_f
  double* __restrict__ uo = final_stage ? I.u : I.us;
  double* __restrict__ vo = final_stage ? I.v : I.vs;
  uo[o] = I.ustar[o] - scale * (xc - xw) * I.ax0[o];
  if (j >= 1) {
    const double xs = zero ? 0.0 : x[o - nx];
    vo[o] = I.vstar[o] - scale * (xc - xs) * I.ay0[o];
  } else {
    vo[o] = 0.0;
  }
  I.p[o] = xc - (zero ? 0.0 : I.pcg->xmean);
  if (final_stage) {
    const double* __restrict__ ph = src == 1 ? I.phi_a : I.phi_b;
    I.phi[o] = ph[o];
  }
}

// ================================================================ multigrid
template <typename S>
__device__ __forceinline__ S ldS(const void* p, size_t o) { return ((const S*)p)[o]; }

// Pre-smoothing from z = 0 (red z = r/D, black Gauss-Seidel), residual
// r - K z and restriction R = P^T/4 to the next level, on one fine tile.
// Level 0 reads the FP64 CG residual.
template <typename S>
__global__ void __launch_bounds__(kNT) k_mg_down(const Tile* __restrict__ tiles,
                                                  const Inst* __restrict__ insts, int level) {
  constexpr int H = 3;
  constexpr int RY = FY + 2 * H, RX = FX + 2 * H;       // 22 x 38 (r, z)
  constexpr int PY = FY + 2, PX = FX + 2;                // residual, halo 1
  __shared__ S s_r[RY * RX], s_z[RY * RX];
  __shared__ S s_ax[RY * (RX + 1)], s_ay[(RY + 1) * RX];
  __shared__ S s_rp[PY * PX];
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (I.pcg->done) return;
  const Level& L = I.lev[level];
  const int nx = L.nx, ny = L.ny;
  const int i0 = t.i0, j0 = t.j0;
  // loads (rows outside the grid hold zeros and are never used as cells)
  for (int k = threadIdx.x; k < RY * (RX + 1); k += kNT) {
    const int rj = k / (RX + 1), ri = k - rj * (RX + 1);
    const int j = j0 - H + rj, i = wrap(i0 - H + ri, nx);
    s_ax[k] = (j >= 0 && j < ny) ? ldS<S>(L.ax, (size_t)j * nx + i) : S(0);
  }
  for (int k = threadIdx.x; k < (RY + 1) * RX; k += kNT) {
    const int rj = k / RX, ri = k - rj * RX;
    const int j = j0 - H + rj, i = wrap(i0 - H + ri, nx);
    s_ay[k] = (j >= 0 && j <= ny) ? ldS<S>(L.ay, (size_t)j * nx + i) : S(0);
  }
  for (int k = threadIdx.x; k < RY * RX; k += kNT) {
    const int rj = k / RX, ri = k - rj * RX;
    const int j = j0 - H + rj, i = wrap(i0 - H + ri, nx);
    S r = 0;
    if (j >= 0 && j < ny) {
      const size_t o = (size_t)j * nx + i;
      r = level == 0 ? (S)I.rr[o] : ldS<S>(L.r, o);
    }
    s_r[k] = r;
  }
  __syncthreads();
  auto diag = [&](int rj, int ri) {
    return s_ax[rj * (RX + 1) + ri] + s_ax[rj * (RX + 1) + ri + 1] + s_ay[rj * RX + ri] +
           s_ay[(rj + 1) * RX + ri];
  };
  auto valid = [&](int rj) { const int j = j0 - H + rj; return j >= 0 && j < ny; };
  // red cells: z = r / D over the whole region
  for (int k = threadIdx.x; k < RY * RX; k += kNT) {
    const int rj = k / RX, ri = k - rj * RX;
    const int j = j0 - H + rj, i = i0 - H + ri;
    S z = 0;
    if (valid(rj) && ((i + j) & 1) == 0) z = s_r[k] / diag(rj, ri);
    s_z[k] = z;
  }
  __syncthreads();
  // black cells: Gauss-Seidel with the red neighbours (halo 2)
  for (int k = threadIdx.x; k < RY * RX; k += kNT) {
    const int rj = k / RX, ri = k - rj * RX;
    if (rj < 1 || rj >= RY - 1 || ri < 1 || ri >= RX - 1) continue;
    const int j = j0 - H + rj, i = i0 - H + ri;
    if (!valid(rj) || ((i + j) & 1) == 0) continue;
    const S aw = s_ax[rj * (RX + 1) + ri], ae = s_ax[rj * (RX + 1) + ri + 1];
    const S as = s_ay[rj * RX + ri], an = s_ay[(rj + 1) * RX + ri];
    const S nb = aw * s_z[k - 1] + ae * s_z[k + 1] + as * s_z[k - RX] + an * s_z[k + RX];
    s_z[k] = (s_r[k] + nb) / (aw + ae + as + an);
  }
  __syncthreads();
  // store the smoothed z on the tile
  for (int k = threadIdx.x; k < FX * FY; k += kNT) {
    const int ty = k / FX, tx = k - ty * FX;
    const int j = j0 + ty, i = i0 + tx;
    if (j < ny && i < nx) ((S*)L.z)[(size_t)j * nx + i] = s_z[(ty + H) * RX + (tx + H)];
  }
  // residual r - K z on the tile + halo 1
  for (int k = threadIdx.x; k < PY * PX; k += kNT) {
    const int pj = k / PX, pi = k - pj * PX;
    const int rj = pj + H - 1, ri = pi + H - 1;
    const int c = rj * RX + ri;
    S rp = 0;
    if (valid(rj)) {
      const S aw = s_ax[rj * (RX + 1) + ri], ae = s_ax[rj * (RX + 1) + ri + 1];
      const S as = s_ay[rj * RX + ri], an = s_ay[(rj + 1) * RX + ri];
      const S zc = s_z[c];
      rp = s_r[c] - (aw * (zc - s_z[c - 1]) + ae * (zc - s_z[c + 1]) + as * (zc - s_z[c - RX]) +
                     an * (zc - s_z[c + RX]));
    }
    s_rp[k] = rp;
  }
  __syncthreads();
  // restriction to the coarse tile
  const Level& C = I.lev[level + 1];
  const int I0 = i0 / 2, J0 = j0 / 2;
  for (int k = threadIdx.x; k < (FX / 2) * (FY / 2); k += kNT) {
    const int cy = k / (FX / 2), cx = k - cy * (FX / 2);
    const int J = J0 + cy, Ic = I0 + cx;
    if (J >= C.ny || Ic >= C.nx) continue;
    S wy[4] = {S(0.25), S(0.75), S(0.75), S(0.25)};
    if (J == 0) { wy[0] = S(0); wy[1] = S(1); }
    if (J == C.ny - 1) { wy[3] = S(0); wy[2] = S(1); }
    const S wx[4] = {S(0.25), S(0.75), S(0.75), S(0.25)};
    S acc = 0;
    for (int dy = 0; dy < 4; ++dy) {
      if (wy[dy] == S(0)) continue;
      const int pj = 2 * cy + dy;          // fine row 2J-1+dy -> halo-1 region row
      S row = 0;
      for (int dx = 0; dx < 4; ++dx) row += wx[dx] * s_rp[pj * PX + 2 * cx + dx];
      acc += wy[dy] * row;
    }
    ((S*)C.r)[(size_t)J * C.nx + Ic] = S(0.25) * acc;
  }
}

// Bilinear prolongation of the coarse correction at fine cell (j, i).
template <typename S>
__device__ __forceinline__ S prolong(const S* e, int cnx, int cny, int j, int i) {
  const int J = j >> 1, Ic = i >> 1;
  const int I2 = (i & 1) ? wrap(Ic + 1, cnx) : wrap(Ic - 1, cnx);
  int J2 = (j & 1) ? J + 1 : J - 1;
  if (J2 < 0 || J2 >= cny) J2 = J;
  const S a = e[(size_t)J * cnx + Ic], b = e[(size_t)J * cnx + I2];
  const S c = e[(size_t)J2 * cnx + Ic], d = e[(size_t)J2 * cnx + I2];
  return S(0.5625) * a + S(0.1875) * b + S(0.1875) * c + S(0.0625) * d;
}

// z += P e, then post-smoothing (black, then red).  Level 0 writes the FP64
// preconditioned residual and the partial (z, q) of the flexible-CG beta.
template <typename S>
__global__ void __launch_bounds__(kNT) k_mg_up(const Tile* __restrict__ tiles,
                                                const Inst* __restrict__ insts, int level) {
  constexpr int H = 2;
  constexpr int RY = FY + 2 * H, RX = FX + 2 * H;       // 20 x 36
  __shared__ S s_r[RY * RX], s_z[RY * RX];
  __shared__ S s_ax[RY * (RX + 1)], s_ay[(RY + 1) * RX];
  __shared__ double sh[kNT / 64];
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (I.pcg->done) return;
  const Level& L = I.lev[level];
  const Level& C = I.lev[level + 1];
  const int nx = L.nx, ny = L.ny;
  const int i0 = t.i0, j0 = t.j0;
  for (int k = threadIdx.x; k < RY * (RX + 1); k += kNT) {
    const int rj = k / (RX + 1), ri = k - rj * (RX + 1);
    const int j = j0 - H + rj, i = wrap(i0 - H + ri, nx);
    s_ax[k] = (j >= 0 && j < ny) ? ldS<S>(L.ax, (size_t)j * nx + i) : S(0);
  }
  for (int k = threadIdx.x; k < (RY + 1) * RX; k += kNT) {
    const int rj = k / RX, ri = k - rj * RX;
    const int j = j0 - H + rj, i = wrap(i0 - H + ri, nx);
    s_ay[k] = (j >= 0 && j <= ny) ? ldS<S>(L.ay, (size_t)j * nx + i) : S(0);
  }
  const S* e = (const S*)C.z;
  for (int k = threadIdx.x; k < RY * RX; k += kNT) {
    const int rj = k / RX, ri = k - rj * RX;
    const int j = j0 - H + rj, i = wrap(i0 - H + ri, nx);
    S r = 0, z = 0;
    if (j >= 0 && j < ny) {
      const size_t o = (size_t)j * nx + i;
      r = level == 0 ? (S)I.rr[o] : ldS<S>(L.r, o);
      z = ldS<S>(L.z, o) + prolong<S>(e, C.nx, C.ny, j, i);
    }
    s_r[k] = r;
    s_z[k] = z;
  }
  __syncthreads();
  auto valid = [&](int rj) { const int j = j0 - H + rj; return j >= 0 && j < ny; };
  auto gs = [&](int k, int rj, int ri) {
    const S aw = s_ax[rj * (RX + 1) + ri], ae = s_ax[rj * (RX + 1) + ri + 1];
    const S as = s_ay[rj * RX + ri], an = s_ay[(rj + 1) * RX + ri];
    const S nb = aw * s_z[k - 1] + ae * s_z[k + 1] + as * s_z[k - RX] + an * s_z[k + RX];
    return (s_r[k] + nb) / (aw + ae + as + an);
  };
  // black sweep on the tile + halo 1
  for (int k = threadIdx.x; k < RY * RX; k += kNT) {
    const int rj = k / RX, ri = k - rj * RX;
    if (rj < 1 || rj >= RY - 1 || ri < 1 || ri >= RX - 1) continue;
    const int j = j0 - H + rj, i = i0 - H + ri;
    if (!valid(rj) || ((i + j) & 1) == 0) continue;
    s_z[k] = gs(k, rj, ri);
  }
  __syncthreads();
  // red sweep on the tile
  for (int k = threadIdx.x; k < RY * RX; k += kNT) {
    const int rj = k / RX, ri = k - rj * RX;
    if (rj < H || rj >= RY - H || ri < H || ri >= RX - H) continue;
    const int j = j0 - H + rj, i = i0 - H + ri;
    if (!valid(rj) || ((i + j) & 1) != 0) continue;
    s_z[k] = gs(k, rj, ri);
  }
  __syncthreads();
  double zq[1] = {0.0};
  for (int k = threadIdx.x; k < FX * FY; k += kNT) {
    const int ty = k / FX, tx = k - ty * FX;
    const int j = j0 + ty, i = i0 + tx;
    if (j < ny && i < nx) {
      const size_t o = (size_t)j * nx + i;
      const S z = s_z[(ty + H) * RX + (tx + H)];
      if (level == 0) {
        I.zf[o] = (double)z;
        zq[0] += (double)z * I.q[o];
      } else {
        ((S*)L.z)[o] = z;
      }
    }
  }
  if (level != 0) return;   // uniform per launch: every thread of the block returns here
  block_sum<1>(zq, sh);
  if (threadIdx.x == 0) I.part[t.local] = zq[0];
  if (arrive_last(&I.pcg->counter[4], L.ntiles)) {
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int k = 0; k < L.ntiles; ++k) s += ld_agent(&I.part[k]);
      PcgScalars* P = I.pcg;
      P->zq = s;
      // flexible CG: the new direction is K-orthogonalised against the last one
      P->beta = P->first ? 0.0 : (P->dq != 0.0 ? -s / P->dq : 0.0);
    }
  }
}

// ------------------------------------------------ single-block coarse cycle
template <typename S>
struct CoarseAcc {
  const Inst& I;
  int level;
  __device__ S r(size_t o) const {
    return (level == 0) ? (S)I.rr[o] : ((const S*)I.lev[level].r)[o];
  }
};

// One red-black half sweep on a whole level (cells of parity `color`).
template <typename S>
__device__ void coarse_half_sweep(const Inst& I, int level, int color, bool from_zero) {
  const Level& L = I.lev[level];
  const int nx = L.nx, ny = L.ny;
  const S* ax = (const S*)L.ax;
  const S* ay = (const S*)L.ay;
  S* z = (S*)L.z;
  CoarseAcc<S> R{I, level};
  for (int c = threadIdx.x; c < nx * ny; c += kCoarseNT) {
    const int j = c / nx, i = c - j * nx;
    if (((i + j) & 1) != color) continue;
    const int ie = wrap(i + 1, nx), iw = wrap(i - 1, nx);
    const S aw = ax[c], ae = ax[(size_t)j * nx + ie];
    const S as = ay[c], an = ay[c + nx];
    const S D = aw + ae + as + an;
    if (from_zero) { z[c] = R.r(c) / D; continue; }
    S nb = aw * z[(size_t)j * nx + iw] + ae * z[(size_t)j * nx + ie];
    if (j >= 1) nb += as * z[c - nx];
    if (j + 1 < ny) nb += an * z[c + nx];
    z[c] = (R.r(c) + nb) / D;
  }
}

template <typename S>
__global__ void __launch_bounds__(kCoarseNT) k_mg_coarse(const Inst* __restrict__ insts) {
  __shared__ double sh[4 * kCoarseNT / 64];
  __shared__ double s_sc[4];
  const Inst& I = insts[blockIdx.x];
  if (I.pcg->done) return;
  const int lc = I.lc, nl = I.nlev;
  // ---- down: smooth, residual (kept in the coarse workspace), restrict
  for (int l = lc; l < nl - 1; ++l) {
    const Level& L = I.lev[l];
    const Level& C = I.lev[l + 1];
    const int nx = L.nx, ny = L.ny;
    coarse_half_sweep<S>(I, l, 0, true);
    // black cells need z = 0 before the GS update reads them as neighbours of nothing:
    // every black cell's neighbours are red, so no initialisation is required.
    __syncthreads();
    coarse_half_sweep<S>(I, l, 1, false);
    __syncthreads();
    const S* ax = (const S*)L.ax;
    const S* ay = (const S*)L.ay;
    const S* z = (const S*)L.z;
    double* rp = I.coarse_ws;
    CoarseAcc<S> R{I, l};
    for (int c = threadIdx.x; c < nx * ny; c += kCoarseNT) {
      const int j = c / nx, i = c - j * nx;
      const int ie = wrap(i + 1, nx), iw = wrap(i - 1, nx);
      const S zc = z[c];
      S kz = ax[c] * (zc - z[(size_t)j * nx + iw]) + ax[(size_t)j * nx + ie] * (zc - z[(size_t)j * nx + ie]);
      if (j >= 1) kz += ay[c] * (zc - z[c - nx]);
      if (j + 1 < ny) kz += ay[c + nx] * (zc - z[c + nx]);
      rp[c] = (double)(R.r(c) - kz);
    }
    __syncthreads();
    S* rc = (S*)C.r;
    for (int c = threadIdx.x; c < C.nx * C.ny; c += kCoarseNT) {
      const int J = c / C.nx, Ic = c - J * C.nx;
      double wy[4] = {0.25, 0.75, 0.75, 0.25};
      if (J == 0) { wy[0] = 0.0; wy[1] = 1.0; }
      if (J == C.ny - 1) { wy[3] = 0.0; wy[2] = 1.0; }
      const double wx[4] = {0.25, 0.75, 0.75, 0.25};
      double acc = 0.0;
      for (int dy = 0; dy < 4; ++dy) {
        if (wy[dy] == 0.0) continue;
        const int j = 2 * J - 1 + dy;
        double row = 0.0;
        for (int dx = 0; dx < 4; ++dx) {
          const int i = wrap(2 * Ic - 1 + dx, nx);
          row += wx[dx] * rp[(size_t)j * nx + i];
        }
        acc += wy[dy] * row;
      }
      rc[c] = (S)(0.25 * acc);
    }
    __syncthreads();
  }
  // ---- coarsest level: CG on the (singular, mean-free) system, FP64
  {
    const Level& L = I.lev[nl - 1];
    const int nx = L.nx, ny = L.ny, n = nx * ny;
    const S* ax = (const S*)L.ax;
    const S* ay = (const S*)L.ay;
    double* xw = I.coarse_ws;
    double* rw = xw + n;
    double* pw = rw + n;
    double* qw = pw + n;
    CoarseAcc<S> R{I, nl - 1};
    double m[1] = {0.0};
    for (int c = threadIdx.x; c < n; c += kCoarseNT) m[0] += (double)R.r(c);
    block_sum<1, kCoarseNT>(m, sh);
    if (threadIdx.x == 0) s_sc[0] = m[0] / n;
    __syncthreads();
    const double mean = s_sc[0];
    double rr[1] = {0.0};
    for (int c = threadIdx.x; c < n; c += kCoarseNT) {
      const double r = (double)R.r(c) - mean;
      xw[c] = 0.0; rw[c] = r; pw[c] = r;
      rr[0] += r * r;
    }
    block_sum<1, kCoarseNT>(rr, sh);
    if (threadIdx.x == 0) s_sc[1] = rr[0];
    __syncthreads();
    double rho = s_sc[1];
    const double rho0 = rho;
    const int maxit = 2 * n;
    for (int it = 0; it < maxit && rho > 1e-24 * rho0 && rho > 0.0; ++it) {
      double pq[1] = {0.0};
      for (int c = threadIdx.x; c < n; c += kCoarseNT) {
        const int j = c / nx, i = c - j * nx;
        const int ie = wrap(i + 1, nx), iw = wrap(i - 1, nx);
        const double pc = pw[c];
        double q = (double)ax[c] * (pc - pw[(size_t)j * nx + iw]) +
                   (double)ax[(size_t)j * nx + ie] * (pc - pw[(size_t)j * nx + ie]);
        if (j >= 1) q += (double)ay[c] * (pc - pw[c - nx]);
        if (j + 1 < ny) q += (double)ay[c + nx] * (pc - pw[c + nx]);
        qw[c] = q;
        pq[0] += pc * q;
      }
      block_sum<1, kCoarseNT>(pq, sh);
      if (threadIdx.x == 0) s_sc[2] = pq[0];
      __syncthreads();
      const double alpha = s_sc[2] > 0.0 ? rho / s_sc[2] : 0.0;
      double rn[1] = {0.0};
      for (int c = threadIdx.x; c < n; c += kCoarseNT) {
        xw[c] += alpha * pw[c];
        const double r = rw[c] - alpha * qw[c];
        rw[c] = r;
        rn[0] += r * r;
      }
      block_sum<1, kCoarseNT>(rn, sh);
      if (threadIdx.x == 0) s_sc[3] = rn[0];
      __syncthreads();
      const double rho_new = s_sc[3];
      const double beta = rho_new / rho;
      for (int c = threadIdx.x; c < n; c += kCoarseNT) pw[c] = rw[c] + beta * pw[c];
      rho = rho_new;
      __syncthreads();
      if (alpha == 0.0) break;
    }
    S* z = (S*)L.z;
    for (int c = threadIdx.x; c < n; c += kCoarseNT) z[c] = (S)xw[c];
    __syncthreads();
  }
  // ---- up: prolong, post-smooth (black, red)
  for (int l = nl - 2; l >= lc; --l) {
    const Level& L = I.lev[l];
    const Level& C = I.lev[l + 1];
    const int nx = L.nx, ny = L.ny;
    S* z = (S*)L.z;
    const S* e = (const S*)C.z;
    for (int c = threadIdx.x; c < nx * ny; c += kCoarseNT) {
      const int j = c / nx, i = c - j * nx;
      z[c] += prolong<S>(e, C.nx, C.ny, j, i);
    }
    __syncthreads();
    coarse_half_sweep<S>(I, l, 1, false);
    __syncthreads();
    coarse_half_sweep<S>(I, l, 0, false);
    __syncthreads();
  }
  // ---- whole V-cycle in this block: publish z and beta
  if (lc == 0) {
    const Level& L = I.lev[0];
    const int n = L.nx * L.ny;
    const S* z = (const S*)L.z;
    double zq[1] = {0.0};
    for (int c = threadIdx.x; c < n; c += kCoarseNT) {
      const double zz = (double)z[c];
      I.zf[c] = zz;
      zq[0] += zz * I.q[c];
    }
    block_sum<1, kCoarseNT>(zq, sh);
    if (threadIdx.x == 0) {
      PcgScalars* P = I.pcg;
      P->zq = zq[0];
      P->beta = P->first ? 0.0 : (P->dq != 0.0 ? -zq[0] / P->dq : 0.0);
    }
  }
}

// Coarse-level coefficients: average of the two fine faces covering each
// coarse face, times 1/4 (the spacing doubles).  One launch per level.
template <typename S>
__global__ void __launch_bounds__(kNT) k_mg_coef(const Inst* __restrict__ insts, int ninst,
                                                  int level) {
  // grid-stride over (instance, coarse face)
  for (int inst = 0; inst < ninst; ++inst) {
    const Inst& I = insts[inst];
    if (level >= I.nlev) continue;
    const Level& F = I.lev[level - 1];
    const Level& C = I.lev[level];
    const int n = C.nx * (C.ny + 1);
    for (int c = blockIdx.x * kNT + threadIdx.x; c < n; c += gridDim.x * kNT) {
      const int J = c / C.nx, Ic = c - J * C.nx;
      const S* fax = (const S*)F.ax;
      const S* fay = (const S*)F.ay;
      if (J < C.ny) {
        const S a = fax[(size_t)(2 * J) * F.nx + 2 * Ic] + fax[(size_t)(2 * J + 1) * F.nx + 2 * Ic];
        ((S*)C.ax)[(size_t)J * C.nx + Ic] = S(0.125) * a;
      }
      S b = 0;
      if (J >= 1 && J < C.ny)
        b = S(0.125) * (fay[(size_t)(2 * J) * F.nx + 2 * Ic] + fay[(size_t)(2 * J) * F.nx + 2 * Ic + 1]);
      ((S*)C.ay)[(size_t)J * C.nx + Ic] = b;
    }
  }
}

}  // namespace cdi
