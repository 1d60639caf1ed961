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
// the coarse correction so that the V-cycle is symmetric.  Levels at or
// below kCoarseCells cells live in the LDS of one block per instance; the
// coarsest grid is solved exactly (dense inverse of K + s 11^T/n, or CG when
// it is larger than kDenseMax).  Finer levels use LDS-tiled kernels whose
// tiles span every instance of a batch.
//
// One flexible-CG iteration is: k_pcg_spmv (d, q = K d, alpha) then the
// V-cycle, whose first kernel also applies x += alpha d, r -= alpha q and
// takes the stopping test, and whose last kernel forms beta.
#pragma once
#include "stage_kernels.h"

namespace cdi {

constexpr int kCoarseCells = 1024;   // levels at or below this size run in one block
constexpr int kCoarseNT = 1024;
static_assert(kCoarseCells <= kCoarseNT, "a coarse right-hand side is loaded one value per thread");
constexpr int kDenseMax = 64;        // coarsest grids up to this size use a dense inverse
// relative residual of the coarsest CG otherwise: as the coarsest solve of a
// preconditioner it need not be exact (the flexible outer CG keeps its own
// tolerance).  On the 64-instance ensemble 1e-8, 1e-6, 1e-4, 1e-2 and 1e-1
// took the same outer iterations (21.0 per step over the first 50 steps from
// rest, 8.0 per step after), and 1e-1 the least time.
constexpr double kCoarseCgRtol = 1e-1;
constexpr int kCLX = 1376;           // LDS cells of all coarse levels (<= 1024 * 4/3)
constexpr int kCLY = 2432;           // LDS y-faces of all coarse levels
constexpr int kWideOwn = 4;          // cells per thread of the wide coarse level (2 per colour)
constexpr int kWideCells = kWideOwn * kCoarseNT;   // its maximum size
constexpr int FX = 32, FY = 16;            // fine tile of the multigrid kernels
static_assert(FX * FY == 2 * kNT, "MG tile = 2 cells per thread");

// ------------------------------------------------------------ projection RHS
// u* = (rho u)* / rho_f(phi_next) on the faces of every cell, b = div(u*)/tau
// (tau given as a multiple of the instance time step), the FP64 face
// coefficients of the pressure operator (and their S copy for the V-cycle),
// and the instance's mean of b.  Resets the CG state.
// Right-hand side and operator coefficients at cell (j, i): the values it
// reads (load) and the arithmetic and stores (store), split so that a thread
// can issue the loads of all its cells first; rhs_cell does both; returns b.
struct RhsIn {
  double pc, pw, pe, ps, pn;   // phase field: cell, west, east, south, north
  double mxo, mxe, myo, myn;   // (rho u)* on the west/east x-faces, south/north y-faces
};

__device__ __forceinline__ RhsIn rhs_load(const Inst& I, const double* __restrict__ ph, int j,
                                          int i) {
  const int nx = I.nx, ny = I.ny;
  const unsigned o = (unsigned)(j * nx) + i;
  const int ie = wrap(i + 1, nx), iw = wrap(i - 1, nx);
  RhsIn v;
  v.pc = ph[o];
  v.pw = ph[(unsigned)(j * nx) + iw];
  v.pe = ph[(unsigned)(j * nx) + ie];
  v.mxo = I.mx[o];
  v.mxe = I.mx[(unsigned)(j * nx) + ie];
  v.ps = v.myo = v.pn = v.myn = 0.0;
  if (j >= 1) { v.ps = ph[o - nx]; v.myo = I.my[o]; }
  if (j + 1 <= ny - 1) { v.pn = ph[o + nx]; v.myn = I.my[o + nx]; }
  return v;
}

// Arithmetic of the right-hand side: every face value is the face's momentum
// times the reciprocal of its density rho_f = (rho_a + rho_b)/2, and the
// same reciprocal times 1/h^2 is the face's operator coefficient.  A face is
// shared by two cells; k_rhs forms each reciprocal once and hands it to the
// neighbour (the per-cell form below forms both and gets the same bits).
__device__ __forceinline__ double rho_of(const Inst& I, double phi) {
  return (I.rho1 - I.rho2) * phi + I.rho2;
}
__device__ __forceinline__ double inv_face_rho(double ra, double rb) {
  return 1.0 / (0.5 * (ra + rb));
}
// b from the four face velocities
__device__ __forceinline__ double rhs_div(const Inst& I, double uw, double ue, double vs, double vn,
                                          double tau) {
  return ((ue - uw) + (vn - vs)) * I.inv_h / (tau * I.dt);
}

template <typename S>
__device__ __forceinline__ double rhs_store(const Inst& I, const RhsIn& v, int j, int i,
                                            double tau) {
  const int nx = I.nx, ny = I.ny;
  const unsigned o = (unsigned)(j * nx) + i;
  const double rc = rho_of(I, v.pc);
  const double irw = inv_face_rho(rho_of(I, v.pw), rc);
  const double ire = inv_face_rho(rc, rho_of(I, v.pe));
  const double irs = j >= 1 ? inv_face_rho(rho_of(I, v.ps), rc) : 0.0;
  const double irn = j + 1 <= ny - 1 ? inv_face_rho(rc, rho_of(I, v.pn)) : 0.0;
  const double uw = v.mxo * irw, ue = v.mxe * ire;
  const double vs = j >= 1 ? v.myo * irs : 0.0;
  const double vn = j + 1 <= ny - 1 ? v.myn * irn : 0.0;
  const double b = rhs_div(I, uw, ue, vs, vn, tau);
  I.ustar[o] = uw;
  I.vstar[o] = vs;
  I.b[o] = b;
  const double ih2 = I.inv_h * I.inv_h;
  const double ax = ih2 * irw;
  const double ay = j >= 1 ? ih2 * irs : 0.0;
  I.ax0[o] = ax;
  I.ay0[o] = ay;
  if (I.mixed) {
    (gas<S>(I.lev[0].ax))[o] = (S)ax;
    (gas<S>(I.lev[0].ay))[o] = (S)ay;
  }
  return b;
}

template <typename S>
__device__ __forceinline__ double rhs_cell(const Inst& I, const double* __restrict__ ph, int j,
                                           int i, double tau) {
  return rhs_store<S>(I, rhs_load(I, ph, j, i), j, i, tau);
}

// Wide-tile form: a wave holds TX = 64 consecutive cells of a row and each
// thread WR consecutive rows, so the east face's reciprocal density comes
// from the next lane (formed directly at the wave's last lane and where the
// row wraps) and the north face's from the thread's next row (formed
// directly for its last row): two divisions per cell instead of four.
template <typename S, int WR>
__global__ void __launch_bounds__(kNT) k_rhs(const Tile* __restrict__ tiles,
                                              const Inst* __restrict__ insts, int src, double tau,
                                              double rtol, int maxit) {
  static_assert(TX == 64, "one wave per row of the tile");
  __shared__ double sh[2 * kNT / 64];
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  const int nx = I.nx, ny = I.ny;
  const CDI_GLOBAL double* __restrict__ ph = src == 0 ? I.phi : (src == 1 ? I.phi_a : I.phi_b);
  const int lane = (int)threadIdx.x % TX;
  const int i = t.i0 + lane;
  const int jb = t.j0 + ((int)threadIdx.x / TX) * WR;   // the thread's first row
  const bool col = i < nx;
  const int ie = wrap(i + 1, nx), iw = wrap(i - 1, nx);
  // every global read first: phi of column i on rows jb-1 .. jb+WR, phi of
  // the west and east columns, the x-momentum on the west and east faces and
  // the y-momentum on the south faces of rows jb .. jb+WR
  double pc[WR + 2], pw[WR], pe[WR], mxo[WR], mxe[WR], myo[WR + 1];
#pragma unroll
  for (int k = 0; k < WR + 2; ++k) {
    const int j = jb - 1 + k;
    pc[k] = (col && j >= 0 && j < ny) ? ph[(unsigned)(j * nx) + i] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < WR; ++r) {
    const int j = jb + r;
    const bool in = col && j < ny;
    pw[r] = in ? ph[(unsigned)(j * nx) + iw] : 0.0;
    pe[r] = in ? ph[(unsigned)(j * nx) + ie] : 0.0;
    mxo[r] = in ? I.mx[(unsigned)(j * nx) + i] : 0.0;
    mxe[r] = in ? I.mx[(unsigned)(j * nx) + ie] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < WR + 1; ++r) {
    const int j = jb + r;
    myo[r] = (col && j >= 1 && j < ny) ? I.my[(unsigned)(j * nx) + i] : 0.0;
  }
  double rho[WR + 2], irw[WR], irs[WR + 1];
#pragma unroll
  for (int k = 0; k < WR + 2; ++k) rho[k] = rho_of(I, pc[k]);
#pragma unroll
  for (int r = 0; r < WR; ++r) irw[r] = inv_face_rho(rho_of(I, pw[r]), rho[r + 1]);
#pragma unroll
  for (int r = 0; r < WR + 1; ++r) {   // south face of row jb + r (r = WR: north of the last row)
    const int j = jb + r;
    irs[r] = (j >= 1 && j < ny) ? inv_face_rho(rho[r], rho[r + 1]) : 0.0;
  }
  const double ih2 = I.inv_h * I.inv_h;
  const bool own_e = lane + 1 < TX && i + 1 < nx;   // the east face is the next lane's west face
  double bsum[2] = {0.0, 0.0};
#pragma unroll
  for (int r = 0; r < WR; ++r) {
    const int j = jb + r;
    double ire = __shfl_down(irw[r], 1, TX);
    if (!own_e) ire = inv_face_rho(rho[r + 1], rho_of(I, pe[r]));
    if (col && j < ny) {
      const unsigned o = (unsigned)(j * nx) + i;
      const double uw = mxo[r] * irw[r], ue = mxe[r] * ire;
      const double vs = j >= 1 ? myo[r] * irs[r] : 0.0;
      const double vn = j + 1 <= ny - 1 ? myo[r + 1] * irs[r + 1] : 0.0;
      const double b = rhs_div(I, uw, ue, vs, vn, tau);
      I.ustar[o] = uw;
      I.vstar[o] = vs;
      I.b[o] = b;
      const double ax = ih2 * irw[r];
      const double ay = j >= 1 ? ih2 * irs[r] : 0.0;
      I.ax0[o] = ax;
      I.ay0[o] = ay;
      if (I.mixed) {
        (gas<S>(I.lev[0].ax))[o] = (S)ax;
        (gas<S>(I.lev[0].ay))[o] = (S)ay;
      }
      bsum[0] += b;
      bsum[1] += b * b;
    }
  }
  block_sum<2>(bsum, sh);
  if (threadIdx.x == 0) {
    st_agent(&I.part[t.local], bsum[0]);
    st_agent(&I.part[I.nwide + t.local], bsum[1]);
  }
  if (arrive_last(I.counters + 0 * kCounterStride, I.nwide, t.local)) {
    double ss[2];
    sum_partials_n<2>(I.part, I.nwide, I.nwide, ss, sh);
    const double s = ss[0], s2 = ss[1];
    if (threadIdx.x == 0) {
      PcgScalars* P = I.pcg;
      const double n = (double)nx * ny;
      P->bmean = s / n;
      P->brms = sqrt(fmax(s2 / n - P->bmean * P->bmean, 0.0));
      P->done = 0; P->iters = 0; P->first = 1; P->converged = 0; P->zero_rhs = 0;
      P->nonfinite = 0;
      P->rtol = rtol; P->maxit = maxit;
    }
  }
}

// K x on a cell from FP64 neighbours (x periodic, wall faces omitted)
__device__ __forceinline__ double apply_K(const Inst& I, const double* __restrict__ x, int j, int i) {
  const int nx = I.nx, ny = I.ny;
  const unsigned o = (unsigned)(j * nx) + i;
  const int ie = wrap(i + 1, nx), iw = wrap(i - 1, nx);
  const double xc = x[o];
  const double aw = I.ax0[o], ae = I.ax0[(unsigned)(j * nx) + ie];
  double s = aw * (xc - x[(unsigned)(j * nx) + iw]) + ae * (xc - x[(unsigned)(j * nx) + ie]);
  if (j >= 1) s += I.ay0[o] * (xc - x[o - nx]);
  if (j + 1 < ny) s += I.ay0[o + nx] * (xc - x[o + nx]);
  return s;
}

// Initial guess of a solve, value at cell o (r0 = f - K x0 with f = -(b -
// mean b)).  guess 1: the caller's / last pressure p; 3..6: the same RK
// stage's pressure extrapolated in time from the last 1..4 steps (constant,
// linear, quadratic, cubic polynomial through equally spaced values: weights
// 1; 2, -1; 3, -3, 1; 4, -6, 4, -1); 2: the learned guess, the fitted
// combination gscale * base + gscale2 * g of a base of mode gbase (one of the
// above) and the network output g held in zf.  The history is a ring of
// kHistDepth slots: step s writes slot s mod kHistDepth (hw, the slot the
// current step writes), so the pressure d + 1 steps back is in slot
// hw - 1 - d and no step moves the older entries.
// The arrays and scalars a guess reads, gathered once per thread (uniform
// values: one batch of scalar reads instead of one per cell and case).
struct GuessSrc {
  const CDI_GLOBAL double* p;      // last pressure
  const CDI_GLOBAL double* h[4];   // the stage's pressure d + 1 steps back (ring slot hw - 1 - d)
  const CDI_GLOBAL double* zf;     // network output (learned guess)
  double gscale, gscale2;
  int gbase;
};

__device__ __forceinline__ GuessSrc guess_src(const Inst& I, int stage, int hw) {
  static_assert(kHistDepth == 4, "ring slots are taken mod 4");
  GuessSrc g;
  const int s = stage >= 0 ? stage : 0;   // no history outside a time step
  g.p = I.p;
#pragma unroll
  for (int d = 0; d < 4; ++d) g.h[d] = I.hp[(hw + 3 - d) & 3][s];
  g.zf = I.zf;
  g.gscale = I.pcg->gscale;
  g.gscale2 = I.pcg->gscale2;
  g.gbase = I.pcg->gbase;
  return g;
}

__device__ __forceinline__ double base_guess(const GuessSrc& G, int guess, unsigned o) {
  switch (guess) {
    case 1: return G.p[o];
    case 3: return G.h[0][o];
    case 4: return 2.0 * G.h[0][o] - G.h[1][o];
    case 5: return 3.0 * (G.h[0][o] - G.h[1][o]) + G.h[2][o];
    case 6: return 4.0 * (G.h[0][o] + G.h[2][o]) - 6.0 * G.h[1][o] - G.h[3][o];
    default: return 0.0;
  }
}

__device__ __forceinline__ double guess_value(const GuessSrc& G, int guess, unsigned o) {
  if (guess == 2) {
    const double b = G.gscale * base_guess(G, G.gbase, o);
    const double c = G.gscale2;   // 0 when the network output was dropped
    return c != 0.0 ? b + c * G.zf[o] : b;
  }
  return base_guess(G, guess, o);
}

// f = -(b - mean b), x0 and r0 = f - K x0 at cell (j, i).
__device__ __forceinline__ void pcg_init_cell(const Inst& I, const GuessSrc& G, int guess, int j,
                                              int i, double bmean, double& f, double& r) {
  const int nx = I.nx, ny = I.ny;
  const unsigned o = (unsigned)(j * nx) + i;
  f = -(I.b[o] - bmean);
  r = f;
  if (guess) {
    const int ie = wrap(i + 1, nx), iw = wrap(i - 1, nx);
    const double xc = guess_value(G, guess, o);
    double kx = I.ax0[o] * (xc - guess_value(G, guess, (unsigned)(j * nx) + iw)) +
                I.ax0[(unsigned)(j * nx) + ie] * (xc - guess_value(G, guess, (unsigned)(j * nx) + ie));
    if (j >= 1) kx += I.ay0[o] * (xc - guess_value(G, guess, o - nx));
    if (j + 1 < ny) kx += I.ay0[o + nx] * (xc - guess_value(G, guess, o + nx));
    r = f - kx;
    I.x[o] = xc;
  } else {
    I.x[o] = 0.0;
  }
  I.rr[o] = r;
}

// Wide-tile form: the guess over the tile and a one-cell halo is formed once
// into LDS, then r0 = f - K x0 on the tile (same arithmetic as pcg_init_cell).
template <int WR>
__global__ void __launch_bounds__(kNT) k_pcg_init(const Tile* __restrict__ tiles,
                                                  const Inst* __restrict__ insts, int guess,
                                                  int stage, int hw) {
  constexpr int RY = WR * TY + 2, RX = TX + 2;
  __shared__ double s_x[RY * RX];
  __shared__ double sh[2 * kNT / 64];
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  const int nx = I.nx, ny = I.ny;
  const double bmean = I.pcg->bmean;
  const GuessSrc G = guess_src(I, stage, hw);
  if (guess) {
    // the guess over the tile and its halo: all reads of the thread first
    constexpr int NG = (RY * RX + kNT - 1) / kNT;
    double gv[NG];
#pragma unroll
    for (int e = 0; e < NG; ++e) {
      const int k = threadIdx.x + e * kNT;
      const int rj = k / RX, ri = k - rj * RX;
      const int j = t.j0 - 1 + rj;
      gv[e] = (k < RY * RX && j >= 0 && j < ny)
                  ? guess_value(G, guess, (unsigned)(j * nx) + wrap_any(t.i0 - 1 + ri, nx))
                  : 0.0;
    }
#pragma unroll
    for (int e = 0; e < NG; ++e) {
      const int k = threadIdx.x + e * kNT;
      if (k < RY * RX) s_x[k] = gv[e];
    }
    __syncthreads();
  }
  double s[2] = {0.0, 0.0};
  // every global read of the thread's rows first, then arithmetic and stores
  double bv[WR], aw[WR], ae[WR], as[WR], an[WR];
#pragma unroll
  for (int r = 0; r < WR; ++r) {
    const int i = t.i0 + wide_tx(), j = t.j0 + wide_ty(r);
    bv[r] = aw[r] = ae[r] = as[r] = an[r] = 0.0;
    if (i < nx && j < ny) {
      const unsigned o = (unsigned)(j * nx) + i;
      bv[r] = I.b[o];
      if (guess) {
        aw[r] = I.ax0[o];
        ae[r] = I.ax0[(unsigned)(j * nx) + wrap(i + 1, nx)];
        if (j >= 1) as[r] = I.ay0[o];
        if (j + 1 < ny) an[r] = I.ay0[o + nx];
      }
    }
  }
  double xo[WR], ro[WR];
#pragma unroll
  for (int r = 0; r < WR; ++r) {
    const int tx = wide_tx(), ty = wide_ty(r);
    const int i = t.i0 + tx, j = t.j0 + ty;
    xo[r] = ro[r] = 0.0;
    if (i < nx && j < ny) {
      const double f = -(bv[r] - bmean);
      double rv = f, xc = 0.0;
      if (guess) {
        const int c = (ty + 1) * RX + tx + 1;
        xc = s_x[c];
        double kx = aw[r] * (xc - s_x[c - 1]) + ae[r] * (xc - s_x[c + 1]);
        if (j >= 1) kx += as[r] * (xc - s_x[c - RX]);
        if (j + 1 < ny) kx += an[r] * (xc - s_x[c + RX]);
        rv = f - kx;
      }
      xo[r] = xc;
      ro[r] = rv;
      s[0] += f * f;
      s[1] += rv * rv;
    }
  }
#pragma unroll
  for (int r = 0; r < WR; ++r) {
    const int i = t.i0 + wide_tx(), j = t.j0 + wide_ty(r);
    if (i < nx && j < ny) {
      const unsigned o = (unsigned)(j * nx) + i;
      I.x[o] = xo[r];
      I.rr[o] = ro[r];
    }
  }
  block_sum<2>(s, sh);
  if (threadIdx.x == 0) {
    st_agent(&I.part[t.local], s[0]);
    st_agent(&I.part[I.nwide + t.local], s[1]);
  }
  if (arrive_last(I.counters + 1 * kCounterStride, I.nwide, t.local)) {
    double ss[2];
    sum_partials_n<2>(I.part, I.nwide, I.nwide, ss, sh);
    const double ff = ss[0], rr = ss[1];
    if (threadIdx.x == 0) {
      PcgScalars* P = I.pcg;
      P->fnorm = sqrt(ff);
      P->rr = rr;
      if (!isfinite(ff) || !isfinite(rr)) {   // NaN / Inf in b or the guess: stop
        P->relres = NAN; P->done = 1; P->converged = 0; P->nonfinite = 1;
      } else if (ff == 0.0) {   // b = 0: the mean-free solution is p = 0
        P->relres = 0.0; P->done = 1; P->converged = 1; P->zero_rhs = 1;
      } else {
        P->relres = sqrt(rr) / P->fnorm;
        if (P->relres <= P->rtol) { P->done = 1; P->converged = 1; }
      }
    }
  }
}

// d = z + beta d_old (d = z on the first iteration), q = K d, (d, r), (d, q);
// last block: alpha = (d, r)/(d, q).
// Wide-tile form: d over the tile and a one-cell halo is formed once into
// LDS; q = K d on the tile from it.
template <int WR>
__global__ void __launch_bounds__(kNT) k_pcg_spmv(const Tile* __restrict__ tiles,
                                                  const Inst* __restrict__ insts, int parity,
                                                  int rsel) {
  constexpr int RY = WR * TY + 2, RX = TX + 2;
  __shared__ double s_d[RY * RX];
  __shared__ double sh[2 * kNT / 64];
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  const int done = t.pcg->done;
  const int nx = I.nx, ny = I.ny;
  scalars_ready(done, nx, ny, I.zf.p, I.d0.p, I.d1.p);
  if (done) return;
  const CDI_GLOBAL double* __restrict__ dold = parity ? I.d0 : I.d1;
  CDI_GLOBAL double* __restrict__ dnew = parity ? I.d1 : I.d0;
  const double* __restrict__ z = I.zf;
  const CDI_GLOBAL double* __restrict__ rv = rsel ? I.rr2 : I.rr;
  const bool first = t.pcg->first != 0;
  const double beta = first ? 0.0 : t.pcg->beta;
  // every global read of the thread first: d over the tile and its halo,
  // then the coefficients and r of its own rows
  constexpr int ND = (RY * RX + kNT - 1) / kNT;
  double zl[ND], dl[ND];
#pragma unroll
  for (int e = 0; e < ND; ++e) {
    const int k = threadIdx.x + e * kNT;
    const int rj = k / RX, ri = k - rj * RX;
    const int j = t.j0 - 1 + rj;
    zl[e] = dl[e] = 0.0;
    if (k < RY * RX && j >= 0 && j < ny) {
      const unsigned o = (unsigned)(j * nx) + wrap_any(t.i0 - 1 + ri, nx);
      zl[e] = z[o];
      if (!first) dl[e] = dold[o];
    }
  }
  double s[2] = {0.0, 0.0};
  double aw[WR], ae[WR], as[WR], an[WR], rr[WR];
#pragma unroll
  for (int r = 0; r < WR; ++r) {
    const int i = t.i0 + wide_tx(), j = t.j0 + wide_ty(r);
    aw[r] = ae[r] = as[r] = an[r] = rr[r] = 0.0;
    if (i < nx && j < ny) {
      const unsigned o = (unsigned)(j * nx) + i;
      aw[r] = I.ax0[o];
      ae[r] = I.ax0[(unsigned)(j * nx) + wrap(i + 1, nx)];
      if (j >= 1) as[r] = I.ay0[o];
      if (j + 1 < ny) an[r] = I.ay0[o + nx];
      rr[r] = rv[o];
    }
  }
#pragma unroll
  for (int e = 0; e < ND; ++e) {
    const int k = threadIdx.x + e * kNT;
    if (k < RY * RX) s_d[k] = first ? zl[e] : zl[e] + beta * dl[e];
  }
  __syncthreads();
  double dco[WR], qo[WR];
#pragma unroll
  for (int r = 0; r < WR; ++r) {
    const int tx = wide_tx(), ty = wide_ty(r);
    const int i = t.i0 + tx, j = t.j0 + ty;
    dco[r] = qo[r] = 0.0;
    if (i < nx && j < ny) {
      const int c = (ty + 1) * RX + tx + 1;
      const double dc = s_d[c];
      double q = aw[r] * (dc - s_d[c - 1]) + ae[r] * (dc - s_d[c + 1]);
      if (j >= 1) q += as[r] * (dc - s_d[c - RX]);
      if (j + 1 < ny) q += an[r] * (dc - s_d[c + RX]);
      dco[r] = dc;
      qo[r] = q;
      s[0] += dc * rr[r];
      s[1] += dc * q;
    }
  }
#pragma unroll
  for (int r = 0; r < WR; ++r) {
    const int i = t.i0 + wide_tx(), j = t.j0 + wide_ty(r);
    if (i < nx && j < ny) {
      const unsigned o = (unsigned)(j * nx) + i;
      dnew[o] = dco[r];
      I.q[o] = qo[r];
    }
  }
  block_sum<2>(s, sh);
  if (threadIdx.x == 0) {
    st_agent(&I.part[t.local], s[0]);
    st_agent(&I.part[I.nwide + t.local], s[1]);
  }
  if (arrive_last(I.counters + 2 * kCounterStride, I.nwide, t.local)) {
    double ss[2];
    sum_partials_n<2>(I.part, I.nwide, I.nwide, ss, sh);
    const double dr = ss[0], dq = ss[1];
    if (threadIdx.x == 0) {
      PcgScalars* P = I.pcg;
      P->dr = dr; P->dq = dq;
      P->alpha = dq != 0.0 ? dr / dq : 0.0;
      P->first = 0;
    }
  }
}

// Galerkin fit of the initial guess on span{p, g}: p the previous pressure,
// g the network's guess (in zf).  The coefficients (a, c) solve the 2x2
// normal equations of min ||x0 - x*||_K over x0 = a p + c g, so the fitted
// guess is never worse, in that norm, than the previous pressure or zero.
template <int WR>
__global__ void __launch_bounds__(kNT) k_guess_fit(const Tile* __restrict__ tiles,
                                                   const Inst* __restrict__ insts, int base,
                                                   int stage, int hw) {
  __shared__ double sh[5 * kNT / 64];
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  const int nx = I.nx, ny = I.ny;
  const GuessSrc G = guess_src(I, stage, hw);
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // pKp, pKg, gKg, p.f, g.f
  for (int r = 0; r < WR; ++r) {
    const int i = t.i0 + wide_tx(), j = t.j0 + wide_ty(r);
    if (i < nx && j < ny) {
      const unsigned o = (unsigned)(j * nx) + i;
      const double f = -(I.b[o] - I.pcg->bmean);
      const int ie = wrap(i + 1, nx), iw = wrap(i - 1, nx);
      const double pv = base_guess(G, base, o), gv = I.zf[o];
      // K applied to the base (apply_K's terms, with base values)
      double kp = I.ax0[o] * (pv - base_guess(G, base, (unsigned)(j * nx) + iw)) +
                  I.ax0[(unsigned)(j * nx) + ie] * (pv - base_guess(G, base, (unsigned)(j * nx) + ie));
      if (j >= 1) kp += I.ay0[o] * (pv - base_guess(G, base, o - nx));
      if (j + 1 < ny) kp += I.ay0[o + nx] * (pv - base_guess(G, base, o + nx));
      const double kg = apply_K(I, I.zf, j, i);
      s[0] += pv * kp; s[1] += pv * kg; s[2] += gv * kg; s[3] += pv * f; s[4] += gv * f;
    }
  }
  block_sum<5>(s, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 5; ++k) st_agent(&I.part[k * I.nwide + t.local], s[k]);
  if (arrive_last(I.counters + 7 * kCounterStride, I.nwide, t.local)) {
    double m[5];
    sum_partials_n<5>(I.part, I.nwide, I.nwide, m, sh);
    if (threadIdx.x == 0) {
      double a = 0.0, c = 0.0;
      const double det = m[0] * m[2] - m[1] * m[1];
      bool finite = true;
      for (int k = 0; k < 5; ++k) finite = finite && isfinite(m[k]);
      if (!finite) {   // a non-finite network output (e.g. garbage weights): the base alone
        a = 1.0;
      } else if (m[0] > 0.0 && m[2] > 0.0 && det > 1e-12 * m[0] * m[2]) {
        a = (m[3] * m[2] - m[4] * m[1]) / det;
        c = (m[4] * m[0] - m[3] * m[1]) / det;
      } else if (m[2] > 0.0) {
        c = m[4] / m[2];
      } else if (m[0] > 0.0) {
        a = m[3] / m[0];
      }
      I.pcg->gscale = a;
      I.pcg->gscale2 = c;
      I.pcg->gbase = base;
    }
  }
}

// Stopping test after the update x += alpha d, r -= alpha q (run by the
// last block of the kernel that applied it).
__device__ __forceinline__ void pcg_stop_test(PcgScalars* P, double rr, double sx, double n) {
  P->rr = rr;
  P->xmean = sx / n;
  P->iters += 1;
  P->iters_total += 1;
  P->relres = sqrt(rr) / P->fnorm;
  if (!isfinite(rr)) { P->done = 1; P->nonfinite = 1; }
  else if (P->relres <= P->rtol) { P->done = 1; P->converged = 1; }
  else if (P->iters >= P->maxit) { P->done = 1; }
}

// Mean of the solution when the solve ended before any CG update.
template <int WR>
__global__ void __launch_bounds__(kNT) k_pcg_xmean(const Tile* __restrict__ tiles,
                                                   const Inst* __restrict__ insts) {
  __shared__ double sh[kNT / 64];
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  const int nx = I.nx, ny = I.ny;
  if (I.pcg->iters > 0) return;
  double s[1] = {0.0};
  for (int r = 0; r < WR; ++r) {
    const int i = t.i0 + wide_tx(), j = t.j0 + wide_ty(r);
    if (i < nx && j < ny) s[0] += I.x[(unsigned)(j * nx) + i];
  }
  block_sum<1>(s, sh);
  if (threadIdx.x == 0) st_agent(&I.part[t.local], s[0]);
  if (arrive_last(I.counters + 6 * kCounterStride, I.nwide, t.local)) {
    const double sx = sum_partials(I.part, I.nwide, sh);
    if (threadIdx.x == 0) I.pcg->xmean = sx / ((double)nx * ny);
  }
}

// u = u* - tau grad(p)/rho_f on interior faces (tau a multiple of the
// instance time step); the pressure is stored mean-free.  final_stage: the
// result is the new state (caller fields) and the new phase field is copied
// from phi_next.
// Projection at cell (j, i), split into the reads (project_load) and the
// arithmetic and stores (project_store) like the right-hand side.
struct ProjIn {
  double xc, xw, xs;       // pressure iterate: cell, west, south
  double us, vs, ax, ay;   // u*, v*, face coefficients
  double ph;               // next phase field (final stage)
};

__device__ __forceinline__ ProjIn project_load(const Inst& I, int final_stage,
                                               const double* __restrict__ ph, int stage,
                                               bool zero, int j, int i) {
  const int nx = I.nx;
  const unsigned o = (unsigned)(j * nx) + i;
  ProjIn v;
  v.xc = zero ? 0.0 : I.x[o];
  v.xw = zero ? 0.0 : I.x[(unsigned)(j * nx) + wrap(i - 1, nx)];
  v.xs = (zero || j < 1) ? 0.0 : I.x[o - nx];
  v.us = I.ustar[o];
  v.ax = I.ax0[o];
  v.vs = j >= 1 ? I.vstar[o] : 0.0;
  v.ay = j >= 1 ? I.ay0[o] : 0.0;
  v.ph = final_stage ? ph[o] : 0.0;
  return v;
}

__device__ __forceinline__ void project_store(const Inst& I, const ProjIn& v, double tau,
                                              int final_stage, int stage, int hw, bool zero,
                                              double xmean, int j, int i) {
  const int nx = I.nx;
  const unsigned o = (unsigned)(j * nx) + i;
  const double scale = tau * I.dt * I.h;   // tau grad(p)/rho_f = tau (p_c - p_w) h a_f
  CDI_GLOBAL double* __restrict__ uo = final_stage ? I.u : I.us;
  CDI_GLOBAL double* __restrict__ vo = final_stage ? I.v : I.vs;
  uo[o] = v.us - scale * (v.xc - v.xw) * v.ax;
  vo[o] = j >= 1 ? v.vs - scale * (v.xc - v.xs) * v.ay : 0.0;
  const double pn = v.xc - (zero ? 0.0 : xmean);
  I.p[o] = pn;
  // pressure history of this RK stage (for the next steps' guesses): the
  // ring slot of this step
  if (stage >= 0) I.hp[hw][stage][o] = pn;
  if (final_stage) I.phi[o] = v.ph;
}

__device__ __forceinline__ void project_cell(const Inst& I, double tau, int final_stage,
                                             const double* __restrict__ ph, int stage, int hw,
                                             bool zero, double xmean, int j, int i) {
  project_store(I, project_load(I, final_stage, ph, stage, zero, j, i), tau, final_stage, stage,
                hw, zero, xmean, j, i);
}

template <int WR>
__global__ void __launch_bounds__(kNT) k_project(const Tile* __restrict__ tiles,
                                                 const Inst* __restrict__ insts, double tau,
                                                 int final_stage, int src, int stage, int hw) {
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  const int nx = I.nx, ny = I.ny;
  const CDI_GLOBAL double* __restrict__ ph = src == 1 ? I.phi_a : I.phi_b;
  // the CG scalars through the tile's address, read with the instance's
  // fields in one batch (not again in every row's branch)
  const int zero_rhs = t.pcg->zero_rhs;
  const double xmean = t.pcg->xmean;
  scalars_ready(nx, ny, zero_rhs, I.x.p, I.ustar.p, I.vstar.p, I.ax0.p, I.ay0.p);
  const bool zero = zero_rhs != 0;
  ProjIn v[WR];
#pragma unroll
  for (int r = 0; r < WR; ++r) {
    const int i = t.i0 + wide_tx(), j = t.j0 + wide_ty(r);
    if (i < nx && j < ny) v[r] = project_load(I, final_stage, ph, stage, zero, j, i);
  }
#pragma unroll
  for (int r = 0; r < WR; ++r) {
    const int i = t.i0 + wide_tx(), j = t.j0 + wide_ty(r);
    if (i < nx && j < ny) project_store(I, v[r], tau, final_stage, stage, hw, zero, xmean, j, i);
  }
}

// ================================================================ multigrid
template <typename S>
__device__ __forceinline__ S ldS(const void* p, unsigned o) { return ((const S*)p)[o]; }

// One red-black Gauss-Seidel half-sweep (m >= 1) on an LDS region of RY x RX cells
// (coefficients s_ax with RX + 1 per row, s_ay with RX per row and RY + 1
// rows): the cells of colour `color` ((rj + ri) & 1) in rows and columns
// [m, RY - m) x [m, RX - m), 0 on rows outside the grid.  A cell of one colour
// reads only cells of the other, so each thread issues the LDS reads of all
// its cells before the first of its writes.
// Reciprocal of a smoother's diagonal: the hardware estimate refined by
// Newton steps (within an ulp or two of the quotient; the smoother is a
// preconditioner, so its rounding changes only the CG path, never the
// converged solution) instead of the longer correctly rounded division.
__device__ __forceinline__ double mg_rcp(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  return fma(fma(-d, r, 1.0), r, r);
}
__device__ __forceinline__ float mg_rcp(float d) {
  const float r = __builtin_amdgcn_rcpf(d);
  return fmaf(fmaf(-d, r, 1.0f), r, r);
}

template <typename S, int RY, int RX, typename ValidF>
__device__ __forceinline__ void lds_half_sweep(S* s_z, const S* s_r, const S* s_ax, const S* s_ay,
                                               int m, int color, const ValidF& valid) {
  // Thread layout: thread tid takes colour cell hx of region row m + hy (tid
  // = hy HX + hx, hy < CR) and, element by element, the same cell CR rows
  // further down, so the index arithmetic is done once; a row's colour parity
  // changes by CR each element (a compile-time amount).
  constexpr int HX = RX / 2;
  constexpr int CR = kNT / HX;
  constexpr int NC = (RY - 2 + CR - 1) / CR;   // rows m .. RY - m - 1, m >= 1
  const int hy = (int)threadIdx.x / HX, hx = (int)threadIdx.x - hy * HX;
  const bool tact = hy < CR;
  const int p0 = (hy + m + color) & 1;
  S val[NC];
  int kk[NC];
  bool act[NC];
#pragma unroll
  for (int e = 0; e < NC; ++e) {
    const int rj = m + hy + e * CR;
    const int ri = 2 * hx + (p0 ^ ((e * CR) & 1));
    act[e] = tact && rj < RY - m && ri >= m && ri < RX - m;
    kk[e] = rj * RX + ri;
    val[e] = S(0);
    if (act[e] && valid(rj)) {
      const int k = kk[e];
      const S aw = s_ax[rj * (RX + 1) + ri], ae = s_ax[rj * (RX + 1) + ri + 1];
      const S as = s_ay[rj * RX + ri], an = s_ay[(rj + 1) * RX + ri];
      const S nb = aw * s_z[k - 1] + ae * s_z[k + 1] + as * s_z[k - RX] + an * s_z[k + RX];
      val[e] = (s_r[k] + nb) * mg_rcp(aw + ae + as + an);
    }
  }
#pragma unroll
  for (int e = 0; e < NC; ++e)
    if (act[e]) s_z[kk[e]] = val[e];
}

// Pre-smoothing from z = 0 (red z = r/D, black Gauss-Seidel), residual
// r - K z and restriction R = P^T/4 to the next level, on one fine tile.
// Level 0 (L0, which must equal level == 0) reads the FP64 CG residual; with
// `update` it first applies the CG step x += alpha d, r -= alpha q (d from
// buffer `parity`) and takes the stopping test.
template <typename S, int NU, bool L0>
__global__ void __launch_bounds__(kNT) k_mg_down(const Tile* __restrict__ tiles,
                                                  const Inst* __restrict__ insts, int level,
                                                  int update, int parity, int rsel) {
  // NU red-black pairs; every half-sweep after the first (pointwise) one
  // shrinks the valid region by one cell, the residual needs a 2-cell halo
  constexpr int H = 2 * NU + 1;
  constexpr int RY = FY + 2 * H, RX = FX + 2 * H;       // 22 x 38 (r, z) for NU = 1
  constexpr int PY = FY + 2, PX = FX + 2;                // residual, halo 1
  __shared__ S s_r[RY * RX], s_z[RY * RX];
  __shared__ S s_ax[RY * (RX + 1)], s_ay[(RY + 1) * RX];
  __shared__ double sh[2 * kNT / 64];
  // the residual for the restriction replaces the right-hand side once every
  // read of it is done (one LDS array less: 4 blocks per CU instead of 3 at
  // V(2,2) FP64)
  static_assert(PY * PX <= RY * RX, "residual fits the right-hand-side array");
  S* const s_rp = s_r;
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  const Level& L = I.lev[level];
  // the done flag (its address is in the tile) and the level's scalars are
  // read together
  const int done = t.pcg->done;
  const int nx = L.nx, ny = L.ny;
  if constexpr (L0) scalars_ready(done, nx, ny, L.ax.p, L.ay.p, I.rr.p, I.rr2.p);
  else scalars_ready(done, nx, ny, L.ax.p, L.ay.p, L.r.p);
  if (done) return;
  const int i0 = t.i0, j0 = t.j0;
  const bool upd = update && L0;   // L0: level == 0 (the launch's every tile)
  const double alpha = upd ? t.pcg->alpha : 0.0;
  // level-0 residual: read the previous buffer when updating, write the current one
  const double* __restrict__ rin = (upd ? (rsel ? I.rr : I.rr2) : (rsel ? I.rr2 : I.rr));
  CDI_GLOBAL double* __restrict__ rout = rsel ? I.rr2 : I.rr;
  // Every global read of the thread (coefficients, right-hand side and, with
  // the CG update, q, x, d) is issued before the first LDS store, so a block
  // waits for one memory latency, not one per loop trip.  Rows outside the
  // grid hold zeros and are never used as cells.
  // Thread layout of the region loops: thread tid holds column cx of region
  // row cy (tid = cy RX + cx, cy < CR); its element e is the cell (cy + e CR,
  // cx), so the index arithmetic is done once and the elements step by
  // constant strides.  The x-faces' last column (RX) is one more value per
  // row, taken by threads tid < RY.
  constexpr int CR = kNT / RX;
  constexpr int NE = (RY + CR - 1) / CR;            // region rows
  constexpr int NEY = (RY + 1 + CR - 1) / CR;       // y-face rows
  static_assert(RY <= kNT, "one thread per row for the last x-face column");
  const int tid = threadIdx.x;
  const int cy = tid / RX, cx = tid - cy * RX;
  const bool tact = cy < CR;
  const int gi = wrap_any(i0 - H + cx, nx);          // grid column of the thread
  const bool ocx = cx >= H && cx < H + FX && i0 - H + cx < nx;   // the column is on the tile
  S axl[NE], ayl[NEY], axe = S(0);
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int rj = cy + e * CR, j = j0 - H + rj;
    axl[e] = (tact && rj < RY && j >= 0 && j < ny) ? ldS<S>(L.ax, (unsigned)(j * nx) + gi) : S(0);
  }
  if (tid < RY) {
    const int j = j0 - H + tid;
    if (j >= 0 && j < ny) axe = ldS<S>(L.ax, (unsigned)(j * nx) + wrap_any(i0 - H + RX, nx));
  }
#pragma unroll
  for (int e = 0; e < NEY; ++e) {
    const int rj = cy + e * CR, j = j0 - H + rj;
    ayl[e] = (tact && rj <= RY && j >= 0 && j <= ny) ? ldS<S>(L.ay, (unsigned)(j * nx) + gi) : S(0);
  }
  const CDI_GLOBAL double* __restrict__ dvec = parity ? I.d1 : I.d0;
  const double* __restrict__ qv = I.q;
  double* __restrict__ xv = I.x;
  double rl[NE], ql[NE], xl[NE], dl[NE];
  unsigned ol[NE];
  bool inl[NE], own[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int rj = cy + e * CR, j = j0 - H + rj;
    inl[e] = tact && rj < RY && j >= 0 && j < ny;
    own[e] = upd && inl[e] && ocx && rj >= H && rj < H + FY;
    ol[e] = inl[e] ? (unsigned)(j * nx) + gi : 0;
    if constexpr (L0) rl[e] = inl[e] ? rin[ol[e]] : 0.0;
    else rl[e] = inl[e] ? (double)ldS<S>(L.r, ol[e]) : 0.0;
    ql[e] = (upd && inl[e]) ? qv[ol[e]] : 0.0;
    xl[e] = own[e] ? xv[ol[e]] : 0.0;
    dl[e] = own[e] ? dvec[ol[e]] : 0.0;
  }
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int rj = cy + e * CR;
    if (tact && rj < RY) s_ax[rj * (RX + 1) + cx] = axl[e];
  }
  if (tid < RY) s_ax[tid * (RX + 1) + RX] = axe;
#pragma unroll
  for (int e = 0; e < NEY; ++e) {
    const int rj = cy + e * CR;
    if (tact && rj <= RY) s_ay[rj * RX + cx] = ayl[e];
  }
  // residual over the region; with the CG update (level 0) the new residual
  // r - alpha q is formed once per cell from a single read of r and q, and
  // on the tile itself x += alpha d, r is stored, ||r||^2 and sum(x) summed
  double red[2] = {0.0, 0.0};
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int rj = cy + e * CR;
    if (!tact || rj >= RY) continue;
    const int k = rj * RX + cx;
    if (!upd) {
      s_r[k] = (S)rl[e];
      continue;
    }
    const double rv = rl[e] - alpha * ql[e];
    s_r[k] = inl[e] ? (S)rv : S(0);
    if (own[e]) {
      const double x = xl[e] + alpha * dl[e];
      xl[e] = x;
      rl[e] = rv;
      red[0] += rv * rv;
      red[1] += x;
    }
  }
  if (upd) {
#pragma unroll
    for (int e = 0; e < NE; ++e)
      if (own[e]) {
        xv[ol[e]] = xl[e];
        rout[ol[e]] = rl[e];
      }
    block_sum<2>(red, sh);
    if (threadIdx.x == 0) {
      st_agent(&I.part[t.local], red[0]);
      st_agent(&I.part[L.ntiles + t.local], red[1]);
    }
  }
  __syncthreads();
  auto diag = [&](int rj, int ri) {
    return s_ax[rj * (RX + 1) + ri] + s_ax[rj * (RX + 1) + ri + 1] + s_ay[rj * RX + ri] +
           s_ay[(rj + 1) * RX + ri];
  };
  auto valid = [&](int rj) { const int j = j0 - H + rj; return j >= 0 && j < ny; };
  // The region's colour is (rj + ri) & 1 (i0, j0 even): the sweeps visit
  // only cells of their colour, RX/2 per row, so no lane idles on the other
  // colour.
  static_assert(RX % 2 == 0, "colour-compact sweeps need an even region width");
  constexpr int HX = RX / 2;
  // red cells: z = r / D over the whole region (0 on rows outside the grid).
  // Black cells need no start value: the first black half-sweep reads only
  // red neighbours, and every later read stays inside the part of the region
  // that an earlier half-sweep has written.
  {
    constexpr int CRH = kNT / HX;
    const int hy = tid / HX, hx = tid - hy * HX;
#pragma unroll
    for (int e = 0; e < (RY + CRH - 1) / CRH; ++e) {
      const int rj = hy + e * CRH, ri = 2 * hx + (rj & 1);
      if (hy < CRH && rj < RY)
        s_z[rj * RX + ri] = valid(rj) ? s_r[rj * RX + ri] * mg_rcp(diag(rj, ri)) : S(0);
    }
  }
  __syncthreads();
  // then Gauss-Seidel half-sweeps black, red, black, ... (half-sweep sw on
  // the region shrunk by sw cells; 0 on rows outside the grid)
#pragma unroll
  for (int sw = 1; sw < 2 * NU; ++sw) {
    lds_half_sweep<S, RY, RX>(s_z, s_r, s_ax, s_ay, sw, sw & 1 /* 1 black, 0 red */, valid);
    __syncthreads();
  }
  // store the smoothed z on the tile
  for (int k = threadIdx.x; k < FX * FY; k += kNT) {
    const int ty = k / FX, tx = k - ty * FX;
    const int j = j0 + ty, i = i0 + tx;
    if (j < ny && i < nx) (gas<S>(L.z))[(unsigned)(j * nx) + i] = s_z[(ty + H) * RX + (tx + H)];
  }
  // residual r - K z on the tile + halo 1: into registers, then (after every
  // thread's reads of s_r) into s_rp = s_r
  constexpr int CRP = kNT / PX;
  constexpr int NR = (PY + CRP - 1) / CRP;
  const int py = tid / PX, px = tid - py * PX;
  S rpl[NR];
#pragma unroll
  for (int e = 0; e < NR; ++e) {
    const int pj = py + e * CRP;
    S rp = 0;
    if (py < CRP && pj < PY) {
      const int rj = pj + H - 1, ri = px + H - 1;
      const int c = rj * RX + ri;
      if (valid(rj)) {
        const S aw = s_ax[rj * (RX + 1) + ri], ae = s_ax[rj * (RX + 1) + ri + 1];
        const S as = s_ay[rj * RX + ri], an = s_ay[(rj + 1) * RX + ri];
        const S zc = s_z[c];
        rp = s_r[c] - (aw * (zc - s_z[c - 1]) + ae * (zc - s_z[c + 1]) +
                       as * (zc - s_z[c - RX]) + an * (zc - s_z[c + RX]));
      }
    }
    rpl[e] = rp;
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < NR; ++e) {
    const int pj = py + e * CRP;
    if (py < CRP && pj < PY) s_rp[pj * PX + px] = rpl[e];
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
    (gas<S>(C.r))[(unsigned)(J * C.nx) + Ic] = S(0.25) * acc;
  }
  if (upd && arrive_last(I.counters + 3 * kCounterStride, L.ntiles, t.local)) {
    double ss[2];
    sum_partials_n<2>(I.part, L.ntiles, L.ntiles, ss, sh);
    const double rr = ss[0], sx = ss[1];
    if (threadIdx.x == 0) pcg_stop_test(I.pcg, rr, sx, (double)nx * ny);
  }
}

// Bilinear prolongation of the coarse correction at fine cell (j, i).
template <typename S>
__device__ __forceinline__ S prolong(const S* e, int cnx, int cny, int j, int i) {
  const int J = j >> 1, Ic = i >> 1;
  const int I2 = (i & 1) ? wrap(Ic + 1, cnx) : wrap(Ic - 1, cnx);
  int J2 = (j & 1) ? J + 1 : J - 1;
  if (J2 < 0 || J2 >= cny) J2 = J;
  const S a = e[(unsigned)(J * cnx) + Ic], b = e[(unsigned)(J * cnx) + I2];
  const S c = e[(unsigned)(J2 * cnx) + Ic], d = e[(unsigned)(J2 * cnx) + I2];
  return S(0.5625) * a + S(0.1875) * b + S(0.1875) * c + S(0.0625) * d;
}

// z += P e, then post-smoothing (black, then red).  Level 0 writes the FP64
// preconditioned residual and forms the flexible-CG beta; a coarser level
// writes its result to zo, never to z: the blocks of one launch read the
// pre-smoothed z of their neighbours' cells in their halos, and a block may
// start after its neighbour has finished.
template <typename S, int NU, bool L0>
__global__ void __launch_bounds__(kNT) k_mg_up(const Tile* __restrict__ tiles,
                                                const Inst* __restrict__ insts, int level,
                                                int rsel) {
  constexpr int H = 2 * NU;
  constexpr int RY = FY + 2 * H, RX = FX + 2 * H;       // 20 x 36 for NU = 1
  // coarse correction around the region: rows and columns (j0-H)/2-1 ..
  // (j0-H)/2+RY/2 (i0, j0 and H are even), columns wrapped on load
  constexpr int EY = RY / 2 + 2, EX = RX / 2 + 2;
  __shared__ S s_r[RY * RX], s_z[RY * RX];
  __shared__ S s_ax[RY * (RX + 1)], s_ay[(RY + 1) * RX];
  __shared__ double sh[kNT / 64];
  // the staged coarse correction lives in s_r until the prolongation has
  // read it (one LDS array less: 5 blocks per CU instead of 4 at V(2,2) FP64)
  static_assert(EY * EX <= RY * RX, "coarse correction fits the right-hand-side array");
  S* const s_e = s_r;
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  const Level& L = I.lev[level];
  const Level& C = I.lev[level + 1];
  // the done flag (its address is in the tile) and the levels' scalars are
  // read together
  const int done = t.pcg->done;
  const int nx = L.nx, ny = L.ny;
  scalars_ready(done, nx, ny, C.nx, C.ny, L.ax.p, L.ay.p, L.z.p);
  if (done) return;
  const int i0 = t.i0, j0 = t.j0;
  const int Jb = ((j0 - H) >> 1) - 1, Ib = ((i0 - H) >> 1) - 1;
  // every global read of the thread is issued before the first LDS store.
  // Thread layout of the region loops: thread tid holds column cx of region
  // row cy (tid = cy RX + cx, cy < CR) and its element e is the cell (cy + e
  // CR, cx); the coarse-correction loops likewise over EX columns.  The
  // x-faces' last column (RX) is one more value per row, taken by threads
  // tid < RY.
  constexpr int CR = kNT / RX;
  constexpr int NP = (RY + CR - 1) / CR;            // region rows
  constexpr int NPY = (RY + 1 + CR - 1) / CR;       // y-face rows
  constexpr int CRE = kNT / EX;
  constexpr int NE = (EY + CRE - 1) / CRE;
  constexpr int NQ = FX * FY / kNT;
  static_assert(RY <= kNT, "one thread per row for the last x-face column");
  const int tid = threadIdx.x;
  const int cy = tid / RX, cx = tid - cy * RX;
  const bool tact = cy < CR;
  const int gi = wrap_any(i0 - H + cx, nx);          // grid column of the thread
  const int ey = tid / EX, ex = tid - ey * EX;
  const bool eact = ey < CRE;
  S axl[NP], ayl[NPY], el[NE], zl[NP], axe = S(0);
  double rl[NP], qt[NQ];
#pragma unroll
  for (int e = 0; e < NP; ++e) {
    const int rj = cy + e * CR, j = j0 - H + rj;
    axl[e] = (tact && rj < RY && j >= 0 && j < ny) ? ldS<S>(L.ax, (unsigned)(j * nx) + gi) : S(0);
  }
  if (tid < RY) {
    const int j = j0 - H + tid;
    if (j >= 0 && j < ny) axe = ldS<S>(L.ax, (unsigned)(j * nx) + wrap_any(i0 - H + RX, nx));
  }
#pragma unroll
  for (int e = 0; e < NPY; ++e) {
    const int rj = cy + e * CR, j = j0 - H + rj;
    ayl[e] = (tact && rj <= RY && j >= 0 && j <= ny) ? ldS<S>(L.ay, (unsigned)(j * nx) + gi) : S(0);
  }
  // the finished correction of the coarser level: zo where this kernel
  // produced it, z where the one-block coarse kernel did (level lg)
  const S* __restrict__ ec = (level + 1 < I.lg ? gas<const S>(C.zo) : gas<const S>(C.z));
  const int gei = wrap_any(Ib + ex, C.nx);
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int cj = ey + e * CRE, J = Jb + cj;
    el[e] = (eact && cj < EY && J >= 0 && J < C.ny) ? ec[(unsigned)(J * C.nx) + gei] : S(0);
  }
  const CDI_GLOBAL double* __restrict__ rin = rsel ? I.rr2 : I.rr;
#pragma unroll
  for (int e = 0; e < NP; ++e) {
    const int rj = cy + e * CR, j = j0 - H + rj;
    const bool in = tact && rj < RY && j >= 0 && j < ny;
    const unsigned o = in ? (unsigned)(j * nx) + gi : 0;
    if constexpr (L0) rl[e] = in ? rin[o] : 0.0;
    else rl[e] = in ? (double)ldS<S>(L.r, o) : 0.0;
    zl[e] = in ? ldS<S>(L.z, o) : S(0);
  }
#pragma unroll
  for (int e = 0; e < NQ; ++e) {   // level 0: q on the tile, for z.q
    const int k = tid + e * kNT;
    const int ty = k / FX, tx = k - ty * FX;
    const int j = j0 + ty, i = i0 + tx;
    qt[e] = (L0 && j < ny && i < nx) ? I.q[(unsigned)(j * nx) + i] : 0.0;
  }
#pragma unroll
  for (int e = 0; e < NP; ++e) {
    const int rj = cy + e * CR;
    if (tact && rj < RY) s_ax[rj * (RX + 1) + cx] = axl[e];
  }
  if (tid < RY) s_ax[tid * (RX + 1) + RX] = axe;
#pragma unroll
  for (int e = 0; e < NPY; ++e) {
    const int rj = cy + e * CR;
    if (tact && rj <= RY) s_ay[rj * RX + cx] = ayl[e];
  }
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int cj = ey + e * CRE;
    if (eact && cj < EY) s_e[cj * EX + ex] = el[e];
  }
  __syncthreads();
  // z += P e (bilinear prolongation from the staged coarse correction)
  const int iu = i0 - H + cx;                 // unwrapped grid column of the thread
  const int cI = (iu >> 1) - Ib, cI2 = cI + ((iu & 1) ? 1 : -1);   // staged coarse columns
#pragma unroll
  for (int e = 0; e < NP; ++e) {
    const int rj = cy + e * CR;
    if (!tact || rj >= RY) continue;
    const int j = j0 - H + rj;
    S z = 0;
    if (j >= 0 && j < ny) {
      const int J = j >> 1;
      int J2 = (j & 1) ? J + 1 : J - 1;
      if (J2 < 0 || J2 >= C.ny) J2 = J;
      const S a = s_e[(J - Jb) * EX + cI], b = s_e[(J - Jb) * EX + cI2];
      const S c = s_e[(J2 - Jb) * EX + cI], d = s_e[(J2 - Jb) * EX + cI2];
      z = zl[e] + (S(0.5625) * a + S(0.1875) * b + S(0.1875) * c + S(0.0625) * d);
    }
    zl[e] = z;
  }
  __syncthreads();   // every read of s_e (= s_r) is done
#pragma unroll
  for (int e = 0; e < NP; ++e) {
    const int rj = cy + e * CR;
    if (!tact || rj >= RY) continue;
    const int k = rj * RX + cx;
    s_r[k] = (S)rl[e];
    s_z[k] = zl[e];
  }
  __syncthreads();
  auto valid = [&](int rj) { const int j = j0 - H + rj; return j >= 0 && j < ny; };
  // half-sweeps black, red, ... (the reverse of the pre-smoothing), the
  // last one (red) on the tile itself; the colour of region cell (rj, ri) is
  // (rj + ri) & 1 (i0, j0, H even) and the sweeps visit only cells of their
  // colour (rows outside the grid hold 0 and keep it)
  static_assert(RX % 2 == 0, "colour-compact sweeps need an even region width");
#pragma unroll
  for (int sw = 0; sw < 2 * NU; ++sw) {
    lds_half_sweep<S, RY, RX>(s_z, s_r, s_ax, s_ay, sw + 1, (sw & 1) ? 0 : 1 /* black first */, valid);
    __syncthreads();
  }
  if constexpr (!L0) {
#pragma unroll
    for (int e = 0; e < NQ; ++e) {
      const int k = threadIdx.x + e * kNT;
      const int ty = k / FX, tx = k - ty * FX;
      const int j = j0 + ty, i = i0 + tx;
      if (j < ny && i < nx) (gas<S>(L.zo))[(unsigned)(j * nx) + i] = s_z[(ty + H) * RX + (tx + H)];
    }
    return;
  }
  // level 0: the FP64 preconditioned residual and its partial z.q
  double zq[1] = {0.0};
#pragma unroll
  for (int e = 0; e < NQ; ++e) {
    const int k = threadIdx.x + e * kNT;
    const int ty = k / FX, tx = k - ty * FX;
    const int j = j0 + ty, i = i0 + tx;
    if (j < ny && i < nx) {
      const S z = s_z[(ty + H) * RX + (tx + H)];
      I.zf[(unsigned)(j * nx) + i] = (double)z;
      zq[0] += (double)z * qt[e];
    }
  }
  block_sum<1>(zq, sh);
  if (threadIdx.x == 0) st_agent(&I.part[t.local], zq[0]);
  if (arrive_last(I.counters + 4 * kCounterStride, L.ntiles, t.local)) {
    const double s = sum_partials(I.part, L.ntiles, sh);
    if (threadIdx.x == 0) {
      PcgScalars* P = I.pcg;
      P->zq = s;
      // flexible CG: the new direction is K-orthogonalised against the last one
      P->beta = P->first ? 0.0 : (P->dq != 0.0 ? -s / P->dq : 0.0);
    }
  }
}

// ------------------------------------------------------------ V-cycle core
// One level as the cycle code sees it: coefficients, right-hand side,
// correction and a residual scratch of the level's size, each in global
// memory or in LDS.
template <typename S>
struct MgView {
  const S* ax;
  const S* ay;
  S* r;
  S* z;
  S* t;
  int nx, ny;
};

// V-cycle on levels lo..nl-1 of instance I by one block of kCoarseNT threads:
// pre-smoothing from zero (red z = r/D, black Gauss-Seidel), residual,
// restriction R = P^T/4 down to the coarsest level, its exact (mean-free)
// solve, then prolongation and post-smoothing (black, red) back up.  On
// return V(lo).z holds the correction; V(lo).r is not modified.  V(l)
// returns the view of level l (a functor, so that views into LDS keep their
// address space after inlining).
// Row part of the dense coarsest inverse a thread multiplies: entries
// (tid / 16, tid % 16 + 16 u), u < 4, loaded ahead of the cycle by the caller.
struct DensePart {
  double m[kDenseMax / 16];
};

// The reads are unconditional (index 0 of the instance's CG vector x stands in
// where there is no entry), so that no branch separates them from the other
// reads of the cycle's start and the block waits for one memory latency.
__device__ __forceinline__ void dense_part_load(const Inst& I, DensePart& dp) {
  const int n = I.lev[I.nlev - 1].nx * I.lev[I.nlev - 1].ny;
  const int row = threadIdx.x >> 4, part = threadIdx.x & 15;
  const CDI_GLOBAL double* src = I.cdense ? I.cinv : I.x;
#pragma unroll
  for (int u = 0; u < kDenseMax / 16; ++u) {
    const int k = part + 16 * u;
    const bool has = I.cdense && row < n && k < n;
    const double v = src[has ? row * n + k : 0];
    dp.m[u] = has ? v : 0.0;
  }
}

// One cell of a coarse level, owned by one thread for a whole pre- or
// post-smoothing: its coefficients, the reciprocal of its diagonal and its
// right-hand side are read from the level's arrays once and kept in
// registers, so a half-sweep reads only the four neighbouring corrections.
// The residual and operator are those of mg_cycle term for term; the
// Gauss-Seidel update multiplies by the reciprocal diagonal where the swept
// global levels divide (at most an ulp apart per update: the smoother stays
// a fixed linear map, which is all the flexible CG needs of it).
template <typename S>
struct OwnedCell {
  S aw, ae, as, an, iD, r;
  int c, w, e;
  bool own, hs, hn;
  int color;   // (i + j) & 1
};

template <typename S>
__device__ __forceinline__ OwnedCell<S> owned_cell(const MgView<S>& L, int c,
                                                   const double* rd = nullptr) {
  OwnedCell<S> o;
  const int nx = L.nx, ny = L.ny;
  o.own = c < nx * ny;
  const int j = o.own ? FastDiv(nx).div(c) : 0, i = c - j * nx;
  o.c = o.own ? c : 0;
  o.w = j * nx + wrap(i - 1, nx);
  o.e = j * nx + wrap(i + 1, nx);
  o.hs = j >= 1;
  o.hn = j + 1 < ny;
  o.color = (i + j) & 1;
  o.aw = o.own ? L.ax[o.c] : S(0);
  o.ae = o.own ? L.ax[o.e] : S(0);
  o.as = o.own ? L.ay[o.c] : S(0);
  o.an = o.own ? L.ay[o.c + nx] : S(0);
  o.iD = o.own ? S(1) / (o.aw + o.ae + o.as + o.an) : S(0);
  o.r = o.own ? (rd != nullptr ? (S)rd[o.c] : L.r[o.c]) : S(0);
  return o;
}

// A cell of the wide level read from global memory (level lg, right-hand
// side rd when given, else the level's r) with unconditional reads (a cell
// past the level reads cell 0), so that all of a thread's reads at the
// cycle's start are in flight together; owned_finish clears a cell past the
// level and forms the reciprocal diagonal once the reads have landed.
template <typename S>
__device__ __forceinline__ OwnedCell<S> wide_cell_load(const Level& L, int c, const double* rd) {
  OwnedCell<S> o;
  const int nx = L.nx, ny = L.ny;
  o.own = c < nx * ny;
  const int j = o.own ? FastDiv(nx).div(c) : 0, i = c - j * nx;
  o.c = o.own ? c : 0;
  o.w = j * nx + wrap(i - 1, nx);
  o.e = j * nx + wrap(i + 1, nx);
  o.hs = j >= 1;
  o.hn = j + 1 < ny;
  o.color = (i + j) & 1;
  const CDI_GLOBAL S* ax = gas<const S>(L.ax);
  const CDI_GLOBAL S* ay = gas<const S>(L.ay);
  const S aw = ax[o.c], ae = ax[o.e], as = ay[o.c], an = ay[o.c + nx];
  S rv;
  if constexpr (std::is_same<S, double>::value) {
    const double* rp = rd != nullptr ? rd : gas<const S>(L.r);
    rv = rp[o.c];
  } else {
    rv = rd != nullptr ? (S)rd[o.c] : gas<const S>(L.r)[o.c];
  }
  o.aw = aw;
  o.ae = ae;
  o.as = as;
  o.an = an;
  o.r = rv;
  return o;
}

template <typename S>
__device__ __forceinline__ void owned_finish(OwnedCell<S>& o) {
  o.aw = o.own ? o.aw : S(0);
  o.ae = o.own ? o.ae : S(0);
  o.as = o.own ? o.as : S(0);
  o.an = o.own ? o.an : S(0);
  o.r = o.own ? o.r : S(0);
  o.iD = o.own ? S(1) / (o.aw + o.ae + o.as + o.an) : S(0);
}

// Gauss-Seidel update of an owned cell (colour `color` only).
template <typename S>
__device__ __forceinline__ void owned_gs(const OwnedCell<S>& o, S* z, int nx, int color,
                                         bool from_zero) {
  if (!o.own || o.color != color) return;
  if (from_zero) { z[o.c] = o.r * o.iD; return; }
  S nb = o.aw * z[o.w] + o.ae * z[o.e];
  if (o.hs) nb += o.as * z[o.c - nx];
  if (o.hn) nb += o.an * z[o.c + nx];
  z[o.c] = (o.r + nb) * o.iD;
}

// Residual t = r - K z of an owned cell.
template <typename S>
__device__ __forceinline__ void owned_residual(const OwnedCell<S>& o, const S* z, S* t, int nx) {
  if (!o.own) return;
  const S zc = z[o.c];
  S kz = o.aw * (zc - z[o.w]) + o.ae * (zc - z[o.e]);
  if (o.hs) kz += o.as * (zc - z[o.c - nx]);
  if (o.hn) kz += o.an * (zc - z[o.c + nx]);
  t[o.c] = o.r - kz;
}

// Restriction R = P^T / 4 of a level's residual t (nx wide) to the right-hand
// side rc of the next coarser level, by one block of kCoarseNT threads.
template <typename S>
__device__ __forceinline__ void restrict_block(const S* t, int nx, S* rc, int cnx, int cny) {
  const FastDiv dc(cnx);
  for (int c = threadIdx.x; c < cnx * cny; c += kCoarseNT) {
    const int J = dc.div(c), Ic = c - J * cnx;
    S wy[4] = {S(0.25), S(0.75), S(0.75), S(0.25)};
    if (J == 0) { wy[0] = S(0); wy[1] = S(1); }
    if (J == cny - 1) { wy[3] = S(0); wy[2] = S(1); }
    const S wx[4] = {S(0.25), S(0.75), S(0.75), S(0.25)};
    S acc = 0;
    for (int dy = 0; dy < 4; ++dy) {
      if (wy[dy] == S(0)) continue;
      const int j = 2 * J - 1 + dy;
      S row = 0;
      for (int dx = 0; dx < 4; ++dx) row += wx[dx] * t[j * nx + wrap(2 * Ic - 1 + dx, nx)];
      acc += wy[dy] * row;
    }
    rc[c] = S(0.25) * acc;
  }
}

template <typename S, typename ViewF>
__device__ __forceinline__ void mg_cycle(const Inst& I, const ViewF& V, int lo, int nl, int nu,
                                         double* s_red, double* s_sc, double* s_vec,
                                         const DensePart* dp = nullptr) {
  const int tid = threadIdx.x;
  // cells of one colour only: h-th cell of colour `color` is row j = h / (nx/2),
  // column i = 2 (h mod nx/2) + ((j + color) & 1)  (swept levels have even nx)
  auto sweep = [&](int l, int color, bool from_zero) {
    const MgView<S> Lv = V(l);
    const int nx = Lv.nx, ny = Lv.ny, hx = nx >> 1;
    const FastDiv dh(hx);
    const S* ax = Lv.ax;
    const S* ay = Lv.ay;
    const S* r = Lv.r;
    S* z = Lv.z;
    for (int h = tid; h < hx * ny; h += kCoarseNT) {
      const int j = dh.div(h), i = 2 * (h - j * hx) + ((j + color) & 1);
      const int c = j * nx + i;
      const int ie = wrap(i + 1, nx), iw = wrap(i - 1, nx);
      const S aw = ax[c], ae = ax[j * nx + ie], as = ay[c], an = ay[c + nx];
      const S rD = mg_rcp(aw + ae + as + an);
      if (from_zero) { z[c] = r[c] * rD; continue; }
      S nb = aw * z[j * nx + iw] + ae * z[j * nx + ie];
      if (j >= 1) nb += as * z[c - nx];
      if (j + 1 < ny) nb += an * z[c + nx];
      z[c] = (r[c] + nb) * rD;
    }
  };
  // ---- down
  for (int l = lo; l < nl - 1; ++l) {
    const MgView<S> Lv = V(l), Cv = V(l + 1);
    const int nx = Lv.nx, ny = Lv.ny;
    if (nx * ny <= kCoarseNT) {   // one cell per thread: coefficients in registers
      const OwnedCell<S> oc = owned_cell<S>(Lv, tid);
      owned_gs<S>(oc, Lv.z, nx, 0, true);
      __syncthreads();
      owned_gs<S>(oc, Lv.z, nx, 1, false);
      __syncthreads();
      for (int k = 1; k < nu; ++k) {
        owned_gs<S>(oc, Lv.z, nx, 0, false);
        __syncthreads();
        owned_gs<S>(oc, Lv.z, nx, 1, false);
        __syncthreads();
      }
      owned_residual<S>(oc, Lv.z, Lv.t, nx);
    } else {
    sweep(l, 0, true);
    __syncthreads();
    sweep(l, 1, false);
    __syncthreads();
    for (int k = 1; k < nu; ++k) {
      sweep(l, 0, false);
      __syncthreads();
      sweep(l, 1, false);
      __syncthreads();
    }
    {
      const S* ax = Lv.ax;
      const S* ay = Lv.ay;
      const S* r = Lv.r;
      const S* z = Lv.z;
      S* t = Lv.t;
      const FastDiv dn(nx);
      for (int c = tid; c < nx * ny; c += kCoarseNT) {
        const int j = dn.div(c), i = c - j * nx;
        const int ie = wrap(i + 1, nx), iw = wrap(i - 1, nx);
        const S zc = z[c];
        S kz = ax[c] * (zc - z[j * nx + iw]) + ax[j * nx + ie] * (zc - z[j * nx + ie]);
        if (j >= 1) kz += ay[c] * (zc - z[c - nx]);
        if (j + 1 < ny) kz += ay[c + nx] * (zc - z[c + nx]);
        t[c] = r[c] - kz;
      }
    }
    }
    __syncthreads();
    restrict_block<S>(Lv.t, nx, Cv.r, Cv.nx, Cv.ny);
    __syncthreads();
  }
  // ---- coarsest level: exact solve (mean-free part)
  {
    const MgView<S> L = V(nl - 1);
    const int nx = L.nx, ny = L.ny, n = nx * ny;
    const S* r = L.r;
    S* z = L.z;
    if (I.cdense) {
      // z = M r with 16 lanes per row (n <= 64 rows x 16 = 1024 threads)
      const int row = tid >> 4, part = tid & 15;
      double acc = 0.0;
      if (row < n) {
        if (dp) {   // the row part was loaded ahead (same order of terms)
#pragma unroll
          for (int u = 0; u < kDenseMax / 16; ++u)
            if (part + 16 * u < n) acc += dp->m[u] * (double)r[part + 16 * u];
        } else {
          const double* M = I.cinv + (size_t)row * n;
          for (int k = part; k < n; k += 16) acc += M[k] * (double)r[k];
        }
      }
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
      if (row < n && part == 0) z[row] = (S)acc;
      __syncthreads();
    } else {
      // Coarsest grids beyond the dense inverse (dimensions that stop halving,
      // e.g. 30 x 15, or a density that varies): Jacobi-preconditioned CG in
      // FP64, in the single-reduction form of Chronopoulos and Gear (both
      // inner products of an iteration in one reduction: two barriers per
      // iteration), one cell per thread.  Only the waves that own cells work
      // (up to 256 cells one to four waves, then eight, then all sixteen):
      // the others neither repeat the scalar recurrence nor take issue slots
      // from the working waves on their SIMD; they pass the barriers and read
      // the stop flag that thread 0 publishes.  The preconditioned residual is
      // shared through an FP64 LDS vector, so the recurrence stays consistent
      // on the mixed path.  As the coarsest solve inside the preconditioner it
      // stops when the preconditioned residual norm (r, D^-1 r) has fallen by
      // kCoarseCgRtol^2; the flexible outer CG tolerates the inexact solve (and
      // the constant the Jacobi scaling adds to the correction, which K does
      // not see).
      double m[1] = {0.0};
      for (int c = tid; c < n; c += kCoarseNT) m[0] += (double)r[c];
      block_allsum<1, kCoarseNT>(m, s_red);
      const double mean = m[0] / n;
      constexpr int NW = kCoarseNT / 64;
      const int naw = n > 512 ? NW : n > 256 ? NW / 2 : (n + 63) >> 6;   // working waves
      const bool act = (tid >> 6) < naw;
      const int c = tid;
      const bool own = c < n;
      const int j = own ? c / nx : 0, i = own ? c - j * nx : 0;
      const int cw = j * nx + wrap(i - 1, nx), ce = j * nx + wrap(i + 1, nx);
      // wall neighbours stand in for themselves (their coefficient is 0)
      const int cs = (own && j >= 1) ? c - nx : c, cn = (own && j + 1 < ny) ? c + nx : c;
      const double aw = own ? (double)L.ax[c] : 0.0, ae = own ? (double)L.ax[ce] : 0.0;
      const double as = (own && j >= 1) ? (double)L.ay[c] : 0.0;
      const double an = (own && j + 1 < ny) ? (double)L.ay[c + nx] : 0.0;
      const double iD = own ? 1.0 / (aw + ae + as + an) : 0.0;
      double xr = 0.0, rr = own ? (double)r[c] - mean : 0.0, ur = rr * iD, pr = 0.0, sr = 0.0;
      double gam_old = 0.0, den_old = 0.0, gam0 = 0.0;
      const int lane = tid & 63;
      // partial sums a lane of a working wave reads: (r, D^-1 r) of wave
      // `lane` in the first row of 16 lanes, (K u, u) in the second
      const int pidx = lane < 16 ? lane : lane < 32 ? NW + lane - 16 : -1;
      const bool pread = pidx >= 0 && (lane & 15) < naw;
      if (tid == 0) s_sc[3] = 0.0;   // stop flag
      for (int it = 0;; ++it) {
        // u = D^-1 r to LDS; the previous iteration's reads of s_vec happened
        // before its second barrier, the flag was written after it
        if (own) s_vec[c] = ur;
        __syncthreads();
        // the neighbours are read with the flag (one LDS round trip)
        double uw = 0.0, ue = 0.0, us = 0.0, un = 0.0;
        if (own) {
          uw = s_vec[cw];
          ue = s_vec[ce];
          us = s_vec[cs];
          un = s_vec[cn];
        }
        if (s_sc[3] != 0.0) break;
        double wv = 0.0;
        if (act) {
          wv = aw * (ur - uw) + ae * (ur - ue) + as * (ur - us) + an * (ur - un);
          const double g0 = wave_sum(rr * ur), g1 = wave_sum(wv * ur);   // (r, D^-1 r), (K u, u)
          if (lane == 0) {
            s_red[tid >> 6] = g0;
            s_red[NW + (tid >> 6)] = g1;
          }
        }
        __syncthreads();
        if (act) {
          // the per-wave sums added in the same order in every lane
          const double t = row16_sum(pread ? s_red[pidx] : 0.0);
          const double gam = lane_value(t, 0), del = lane_value(t, 16);
          if (it == 0) gam0 = gam;
          bool stop = !(gam > kCoarseCgRtol * kCoarseCgRtol * gam0) || it >= 2 * n;
          // beta = gam / gam_old; with alpha_old = gam_old / den_old the
          // denominator del - beta gam / alpha_old is del - beta^2 den_old
          double beta = 0.0, den = del;
          if (!stop && it > 0) {
            beta = gam / gam_old;
            den = del - beta * beta * den_old;
          }
          stop = stop || !(den > 0.0);
          if (!stop) {
            const double alpha = gam / den;
            pr = ur + beta * pr;   // p = u + beta p
            sr = wv + beta * sr;   // s = K p
            xr += alpha * pr;
            rr -= alpha * sr;
            ur = rr * iD;
            gam_old = gam;
            den_old = den;
          }
          if (tid == 0 && stop) s_sc[3] = 1.0;
        }
      }
      if (own) z[c] = (S)xr;
      __syncthreads();
    }
  }
  // ---- up: prolong, post-smooth (black, red)
  for (int l = nl - 2; l >= lo; --l) {
    const MgView<S> Lv = V(l), Cv = V(l + 1);
    const int nx = Lv.nx, ny = Lv.ny;
    const int cnx = Cv.nx, cny = Cv.ny;
    S* z = Lv.z;
    const S* e = Cv.z;
    const FastDiv dn(nx);
    for (int c = tid; c < nx * ny; c += kCoarseNT) {
      const int j = dn.div(c), i = c - j * nx;
      z[c] += prolong<S>(e, cnx, cny, j, i);
    }
    __syncthreads();
    if (nx * ny <= kCoarseNT) {   // one cell per thread: coefficients in registers
      const OwnedCell<S> oc = owned_cell<S>(Lv, tid);
      for (int k = 0; k < nu; ++k) {
        owned_gs<S>(oc, z, nx, 1, false);
        __syncthreads();
        owned_gs<S>(oc, z, nx, 0, false);
        __syncthreads();
      }
    } else {
      for (int k = 0; k < nu; ++k) {
        sweep(l, 1, false);
        __syncthreads();
        sweep(l, 0, false);
        __syncthreads();
      }
    }
  }
}

// LDS of the single-block cycle over the coarse levels lc..nl-1.
template <typename S>
struct CoarseLds {
  S ax[kCLX], ay[kCLY], r[kCLX], z[kCLX], t[kCLX];
  double cg[kCoarseNT];   // shared FP64 vector of the coarsest CG
  double red[2 * kCoarseNT / 64];
  double sc[4];
};

// View of coarse level l (lc <= l < nl) inside the CoarseLds arrays; the
// levels are stored one after the other from lc.
template <typename S>
__device__ __forceinline__ MgView<S> coarse_view(const Inst& I, CoarseLds<S>& C, int l) {
  const int a = I.cpre_x[l - I.lc], b = I.cpre_y[l - I.lc];
  MgView<S> v;
  v.nx = I.lev[l].nx; v.ny = I.lev[l].ny;
  v.ax = C.ax + a; v.ay = C.ay + b;
  v.r = C.r + a; v.z = C.z + a; v.t = C.t;
  return v;
}

// Load the coefficients of levels lc..nl-1 into LDS, where they are stored
// level after level (the layout of coarse_view), and, with rdst, the rn
// values of a right-hand side (S values from rs, or FP64 from rd).  Every
// global read of a thread is issued before its first LDS store: the block
// waits for one memory latency instead of one per level and array.
template <typename S>
__device__ __forceinline__ void coarse_load_coef(const Inst& I, CoarseLds<S>& C,
                                                 S* rdst = nullptr, const S* rs = nullptr,
                                                 const double* rd = nullptr, int rn = 0) {
  constexpr int NX = (kCLX + kCoarseNT - 1) / kCoarseNT;
  constexpr int NY = (kCLY + kCoarseNT - 1) / kCoarseNT;
  // flat index f of the concatenated x (y) arrays -> level and offset, by
  // selects over the coarse levels' prefix sums (a fixed number of them, so
  // the scalar reads of every level's base address are issued together and
  // the vector reads that follow are unconditional: element 0 of level lc
  // stands in past the last level)
  auto locate = [&](int f, bool yf, const CDI_GLOBAL S*& src) {
    const Level& L0 = I.lev[I.lc];
    src = yf ? gas<const S>(L0.ay) : gas<const S>(L0.ax);
    bool found = false;
#pragma unroll
    for (int m = 0; m < kMaxCoarseLevels; ++m) {
      const int lo = yf ? I.cpre_y[m] : I.cpre_x[m];
      const int hi = yf ? I.cpre_y[m + 1] : I.cpre_x[m + 1];
      const Level& L = I.lev[min(I.lc + m, kMaxLevels - 1)];
      const CDI_GLOBAL S* base = yf ? gas<const S>(L.ay) : gas<const S>(L.ax);
      const bool here = f >= lo && f < hi;
      src = here ? base + (f - lo) : src;
      found = found || here;
    }
    return found;
  };
  S gx[NX], gy[NY];
  bool hx[NX], hy[NY];
#pragma unroll
  for (int e = 0; e < NX; ++e) {
    const CDI_GLOBAL S* src;
    hx[e] = locate(threadIdx.x + e * kCoarseNT, false, src);
    gx[e] = *src;
  }
#pragma unroll
  for (int e = 0; e < NY; ++e) {
    const CDI_GLOBAL S* src;
    hy[e] = locate(threadIdx.x + e * kCoarseNT, true, src);
    gy[e] = *src;
  }
  S gr = S(0);
  const bool hr = rdst != nullptr && (int)threadIdx.x < rn;
  if constexpr (std::is_same<S, double>::value) {
    const double* rp = rd != nullptr ? rd : rs;
    if (rdst != nullptr) gr = rp[hr ? threadIdx.x : 0];
  } else {
    if (hr) gr = rd != nullptr ? (S)rd[threadIdx.x] : rs[threadIdx.x];
  }
#pragma unroll
  for (int e = 0; e < NX; ++e)
    if (hx[e]) C.ax[threadIdx.x + e * kCoarseNT] = gx[e];
#pragma unroll
  for (int e = 0; e < NY; ++e)
    if (hy[e]) C.ay[threadIdx.x + e * kCoarseNT] = gy[e];
  if (hr) rdst[threadIdx.x] = gr;
}

// LDS of the wide level of the one-block cycle: level lc - 1 when the cycle
// starts there (more than kCoarseCells cells, at most kWideCells).
template <typename S>
struct WideLds {
  S z[kWideCells], t[kWideCells];
};

// Cell of colour `col` with colour-compact index h on an nx x ny level (nx
// even): row h / (nx/2), column 2 (h mod nx/2) + ((row + col) & 1); nx ny
// (no cell) past the last one.
__device__ __forceinline__ int wide_cell_index(int h, int col, int nx, int ny) {
  const int hx = nx >> 1;
  if (h >= hx * ny) return nx * ny;
  const int j = h / hx;
  return j * nx + 2 * (h - j * hx) + ((j + col) & 1);
}

// V-cycle from the wide level (level lc - 1, nx x ny): every thread owns up
// to kWideOwn of its cells, whose coefficients, reciprocal diagonal and
// right-hand side the caller has read into registers together with the
// other levels' coefficients: oc[2 m + col] is the cell of colour col with
// colour-compact index tid + m kCoarseNT, so a half-sweep runs the update
// only on cells of its colour, in every lane.  The level's correction and
// residual are in LDS, and the levels from lc run in mg_cycle.  The
// arithmetic is that of mg_cycle's owned cells; only the storage differs, so
// a barrier phase costs LDS latency instead of a pass over global memory.
template <typename S>
__device__ __forceinline__ void wide_cycle(const Inst& I, int nx, int ny,
                                           const OwnedCell<S> (&oc)[kWideOwn], WideLds<S>& W,
                                           CoarseLds<S>& C, const DensePart* dp) {
  const int tid = threadIdx.x;
  {
#pragma unroll
    for (int m = 0; m < kWideOwn / 2; ++m) owned_gs<S>(oc[2 * m + 0], W.z, nx, 0, true);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kWideOwn / 2; ++m) owned_gs<S>(oc[2 * m + 1], W.z, nx, 1, false);
    __syncthreads();
    for (int s = 1; s < I.nu_c; ++s) {
#pragma unroll
      for (int m = 0; m < kWideOwn / 2; ++m) owned_gs<S>(oc[2 * m + 0], W.z, nx, 0, false);
      __syncthreads();
#pragma unroll
      for (int m = 0; m < kWideOwn / 2; ++m) owned_gs<S>(oc[2 * m + 1], W.z, nx, 1, false);
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < kWideOwn; ++k) owned_residual<S>(oc[k], W.z, W.t, nx);
  }
  __syncthreads();
  const MgView<S> Cv = coarse_view<S>(I, C, I.lc);
  restrict_block<S>(W.t, nx, Cv.r, Cv.nx, Cv.ny);
  __syncthreads();
  mg_cycle<S>(I, [&](int l) { return coarse_view<S>(I, C, l); }, I.lc, I.nlev, I.nu_c, C.red, C.sc,
              C.cg, dp);
  // prolongation over all cells (the barrier below orders it before the
  // smoothing, whose cells are spread over the threads by colour)
  const FastDiv dn(nx);
  for (int c = tid; c < nx * ny; c += kCoarseNT) {
    const int j = dn.div(c), i = c - j * nx;
    W.z[c] += prolong<S>(Cv.z, Cv.nx, Cv.ny, j, i);
  }
  __syncthreads();
  {
    for (int s = 0; s < I.nu_c; ++s) {
#pragma unroll
      for (int m = 0; m < kWideOwn / 2; ++m) owned_gs<S>(oc[2 * m + 1], W.z, nx, 1, false);
      __syncthreads();
#pragma unroll
      for (int m = 0; m < kWideOwn / 2; ++m) owned_gs<S>(oc[2 * m + 0], W.z, nx, 0, false);
      __syncthreads();
    }
  }
}

// Level view of a one-block V-cycle: levels from lc in LDS, finer levels in
// global memory (level 0 reads `r0`, the others their own r; the residual
// scratch of the global levels is I.mg_t).
template <typename S>
__device__ __forceinline__ MgView<S> mixed_view(const Inst& I, CoarseLds<S>& C, S* r0, int l) {
  if (l >= I.lc) return coarse_view<S>(I, C, l);
  const Level& L = I.lev[l];
  MgView<S> v;
  v.nx = L.nx; v.ny = L.ny;
  v.ax = gas<const S>(L.ax); v.ay = gas<const S>(L.ay);
  v.r = l == 0 ? r0 : gas<S>(L.r);
  v.z = gas<S>(L.z);
  v.t = gas<S>(I.mg_t);
  return v;
}

// ------------------------------------------------ single-block coarse cycle
// Every level from lg down runs in one block: levels lg..lc-1 from global
// memory (L2-resident at these sizes), levels from lc in LDS (coefficients,
// right-hand side, correction, scratch); a start level lg = lc - 1 keeps its
// correction and residual in LDS too (wide_cycle).  lg trades launches of the tiled
// kernels against one CU's throughput and is chosen per context.  With
// lg == 0 the block holds the whole problem and also applies the CG update,
// the stopping test and beta.
template <typename S>
__global__ void __launch_bounds__(kCoarseNT) k_mg_coarse(const Inst* __restrict__ insts,
                                                          int update, int parity, int rsel) {
  __shared__ CoarseLds<S> C;
  __shared__ WideLds<S> W;
  const Inst& I = insts[blockIdx.x];
  const int lg = I.lg, lc = I.lc, nl = I.nlev;
  // the done flag and the start level's scalars are read together
  const int done = I.pcg->done;
  const Level& Lg = I.lev[lg];
  scalars_ready(done, lc, nl, Lg.nx, Lg.ny, Lg.ax.p, Lg.ay.p, Lg.r.p);
  if (done) return;
  const bool wide = lg + 1 == lc && I.lev[lg].nx * I.lev[lg].ny <= kWideCells &&
                    (I.lev[lg].nx & 1) == 0;
  const int tid = threadIdx.x;
  double* __restrict__ rcur = rsel ? I.rr2 : I.rr;   // level-0 residual the cycle reads
  // ---- CG update when the whole grid is handled here
  if (lg == 0 && update) {
    const Level& L0 = I.lev[0];
    const int n = L0.nx * L0.ny;
    const double alpha = I.pcg->alpha;
    const CDI_GLOBAL double* __restrict__ d = parity ? I.d1 : I.d0;
    const CDI_GLOBAL double* __restrict__ rin = rsel ? I.rr : I.rr2;
    double red[2] = {0.0, 0.0};
    for (int c = tid; c < n; c += kCoarseNT) {
      const double x = I.x[c] + alpha * d[c];
      const double r = rin[c] - alpha * I.q[c];
      I.x[c] = x;
      rcur[c] = r;
      red[0] += r * r;
      red[1] += x;
    }
    block_sum<2, kCoarseNT>(red, C.red);
    if (tid == 0) {
      pcg_stop_test(I.pcg, red[0], red[1], (double)n);
      C.sc[0] = I.pcg->done;
    }
    __syncthreads();
    if (C.sc[0] != 0.0) return;
  }
  // the dense coarsest inverse's row parts are loaded with the coefficients,
  // long before the cycle reaches the coarsest level
  static_assert(kDenseMax * 16 <= kCoarseNT, "16 threads per dense row");
  DensePart dp;
  dense_part_load(I, dp);
  S* r0 = I.mixed ? gas<S>(I.mg_r0) : (S*)(void*)rcur;
  auto view = [&](int l) { return mixed_view<S>(I, C, r0, l); };
  // the wide level's cells, read before the LDS levels' coefficients so
  // that the block waits for one memory latency; on level 0 the right-hand
  // side is the FP64 residual itself (its S copy r0 is written below)
  OwnedCell<S> woc[kWideOwn];
  if (wide) {
    const Level& L = I.lev[lg];
#pragma unroll
    for (int k = 0; k < kWideOwn; ++k)
      woc[k] = wide_cell_load<S>(L, wide_cell_index(tid + (k >> 1) * kCoarseNT, k & 1, L.nx, L.ny),
                                 lg == 0 ? rcur : nullptr);
  }
  {
    // right-hand side of level lg: into LDS with the coefficients when lg is
    // an LDS level (at most kCoarseCells = kCoarseNT cells), into the S copy
    // of the level-0 residual on the mixed path
    const Level& L = I.lev[lg];
    const int n = L.nx * L.ny;
    if (lg >= lc) {
      coarse_load_coef<S>(I, C, coarse_view<S>(I, C, lg).r, gas<const S>(L.r),
                          lg == 0 ? rcur : nullptr, n);
    } else {
      coarse_load_coef<S>(I, C);
      if (lg == 0 && I.mixed)
        for (int c = tid; c < n; c += kCoarseNT) r0[c] = (S)rcur[c];
    }
  }
  __syncthreads();
  if (wide) {
#pragma unroll
    for (int k = 0; k < kWideOwn; ++k) owned_finish<S>(woc[k]);
  }
  if (lg >= lc)   // LDS levels only: views the compiler knows to be LDS (ds_ instructions)
    mg_cycle<S>(I, [&](int l) { return coarse_view<S>(I, C, l); }, lg, nl, I.nu_c, C.red, C.sc, C.cg,
                &dp);
  else if (wide)
    wide_cycle<S>(I, I.lev[lg].nx, I.lev[lg].ny, woc, W, C, &dp);
  else
    mg_cycle<S>(I, view, lg, nl, I.nu_c, C.red, C.sc, C.cg, &dp);
  // ---- publish the level-lg correction (and beta when it is level 0)
  {
    const Level& L = I.lev[lg];
    const int n = L.nx * L.ny;
    const S* z = wide ? W.z : view(lg).z;
    if (lg > 0) {
      if (lg >= lc || wide)
        for (int c = tid; c < n; c += kCoarseNT) (gas<S>(L.z))[c] = z[c];
    } else {
      double zq[1] = {0.0};
      for (int c = tid; c < n; c += kCoarseNT) {
        const double zz = (double)z[c];
        I.zf[c] = zz;
        zq[0] += zz * I.q[c];
      }
      block_sum<1, kCoarseNT>(zq, C.red);
      if (tid == 0) {
        PcgScalars* P = I.pcg;
        P->zq = zq[0];
        P->beta = P->first ? 0.0 : (P->dq != 0.0 ? -zq[0] / P->dq : 0.0);
      }
    }
  }
}

// Coarse-level coefficients of level l from level l-1: a coarse face covers
// two fine faces; its coefficient is their mean times 1/4 (h doubles).
// Level by level this is the mean of the 2^l level-0 faces times 4^-l, with
// coalesced (stride-2) reads instead of stride-2^l ones.
template <typename S>
__device__ __forceinline__ void mg_coef_level(const Inst& I, int l, int start, int stride) {
  const Level& F = I.lev[l - 1];
  const Level& C = I.lev[l];
  const S* fax = gas<const S>(F.ax);
  const S* fay = gas<const S>(F.ay);
  const int n = C.nx * (C.ny + 1);
  for (int c = start; c < n; c += stride) {
    const int J = c / C.nx, Ic = c - J * C.nx;
    if (J < C.ny)
      (gas<S>(C.ax))[c] = (fax[(unsigned)((2 * J) * F.nx) + 2 * Ic] + fax[(unsigned)((2 * J + 1) * F.nx) + 2 * Ic]) *
                      S(0.125);
    S b = 0;
    if (J >= 1 && J < C.ny)
      b = (fay[(unsigned)((2 * J) * F.nx) + 2 * Ic] + fay[(unsigned)((2 * J) * F.nx) + 2 * Ic + 1]) * S(0.125);
    (gas<S>(C.ay))[c] = b;
  }
}

// Level l (below the instance's coarse start level lg) of every instance
// that has it (grid.y = instance).
template <typename S>
__global__ void __launch_bounds__(kNT) k_mg_coef(const Inst* __restrict__ insts, int l,
                                                 int only_variable) {
  const Inst& I = insts[blockIdx.y];
  if (l >= I.nlev || l >= I.lg || (only_variable && I.coef_const)) return;
  mg_coef_level<S>(I, l, blockIdx.x * kNT + threadIdx.x, gridDim.x * kNT);
}

// The levels from lg (at least 1) of every instance (grid = instances), one
// block each, level after level with a barrier between (the block's own
// global writes are visible to it after the barrier): the small levels in
// one launch instead of one launch per level.
template <typename S>
__global__ void __launch_bounds__(kCoarseNT) k_mg_coef_small(const Inst* __restrict__ insts,
                                                             int only_variable) {
  const Inst& I = insts[blockIdx.x];
  if (only_variable && I.coef_const) return;
  for (int l = I.lg > 1 ? I.lg : 1; l < I.nlev; ++l) {
    mg_coef_level<S>(I, l, threadIdx.x, kCoarseNT);
    __syncthreads();
  }
}

// Dense inverse of the coarsest operator K_c + s 11^T / n (s its mean
// diagonal): symmetric positive definite, inverted in LDS by Gauss-Jordan
// without pivoting.  For a mean-free right-hand side the product is the
// mean-free solution of K_c z = r.
template <typename S>
__device__ __forceinline__ void coarse_inverse(const Inst& I, double* B, double* s_red,
                                               double* s_shift_slot) {
  if (!I.cdense) return;
  const Level& L = I.lev[I.nlev - 1];
  const int nx = L.nx, ny = L.ny, n = nx * ny;
  const S* ax = gas<const S>(L.ax);
  const S* ay = gas<const S>(L.ay);
  const int tid = threadIdx.x;
  for (int k = tid; k < n * n; k += kCoarseNT) B[k] = 0.0;
  __syncthreads();
  double dsum[1] = {0.0};
  for (int c = tid; c < n; c += kCoarseNT) {   // one thread builds one row
    const int j = c / nx, i = c - j * nx;
    const int ie = wrap(i + 1, nx), iw = wrap(i - 1, nx);
    const double aw = (double)ax[c], ae = (double)ax[j * nx + ie];
    double d = 0.0;
    if (iw != i) { B[c * n + j * nx + iw] -= aw; d += aw; }
    if (ie != i) { B[c * n + j * nx + ie] -= ae; d += ae; }
    if (j >= 1) { const double a = (double)ay[c]; B[c * n + c - nx] -= a; d += a; }
    if (j + 1 < ny) { const double a = (double)ay[c + nx]; B[c * n + c + nx] -= a; d += a; }
    B[c * n + c] += d;
    dsum[0] += d;
  }
  block_sum<1, kCoarseNT>(dsum, s_red);
  if (tid == 0) *s_shift_slot = dsum[0] / n / n;
  __syncthreads();
  const double shift = *s_shift_slot;
  for (int k = tid; k < n * n; k += kCoarseNT) B[k] += shift;
  __syncthreads();
  constexpr int PER = (kDenseMax * kDenseMax + kCoarseNT - 1) / kCoarseNT;
  for (int k = 0; k < n; ++k) {
    const double ipiv = 1.0 / B[k * n + k];
    double nv[PER];
    int cnt = 0;
    for (int e = tid; e < n * n; e += kCoarseNT, ++cnt) {
      const int r = e / n, c = e - r * n;
      double v;
      if (r == k && c == k) v = ipiv;
      else if (r == k) v = B[k * n + c] * ipiv;
      else if (c == k) v = -B[r * n + k] * ipiv;
      else v = B[e] - B[r * n + k] * (B[k * n + c] * ipiv);
      nv[cnt] = v;
    }
    __syncthreads();
    cnt = 0;
    for (int e = tid; e < n * n; e += kCoarseNT, ++cnt) B[e] = nv[cnt];
    __syncthreads();
  }
  for (int k = tid; k < n * n; k += kCoarseNT) I.cinv[k] = B[k];
}

template <typename S>
__global__ void __launch_bounds__(kCoarseNT) k_coarse_inv(const Inst* __restrict__ insts) {
  __shared__ double B[kDenseMax * kDenseMax];
  __shared__ double s_red[kCoarseNT / 64 + 1];
  coarse_inverse<S>(insts[blockIdx.x], B, s_red, s_red + kCoarseNT / 64);
}

}  // namespace cdi
