// Persistent form of the time step: one workgroup of kCoarseNT threads
// advances one instance through whole RK4 steps -- phase preparation and the
// stage operator (the tiled kernels' tile bodies, four tiles at a time), the
// projection right-hand side, the flexible CG with its V-cycle and stopping
// test, and the projection -- separated by block barriers, with no host
// round trip and no inter-block synchronisation.  A batch is one launch with
// one workgroup per instance, so an ensemble of small grids keeps as many
// compute units busy as it has members and each member stops iterating on
// its own residual.  Per-cell arithmetic is the tiled path's (shared device
// functions); only the order of the CG reductions differs.
#pragma once
#include "diag_kernels.h"

namespace cdi {

constexpr int PNT = kCoarseNT;   // threads of a persistent workgroup
constexpr int PQ = PNT / kNT;    // tiles processed at once by the stage bodies

template <typename S>
struct PersistLds {
  union {
    PrepLds<S> prep[PQ];
    StageLds<S> stage[PQ];
    CoarseLds<S> coarse;
    double B[kDenseMax * kDenseMax];
  } u;
  double red[4 * PNT / 64];
  double sc[8];
};

// Block-wide sum of NV values, returned to every thread.
template <int NV>
__device__ __forceinline__ void pall_sum(double (&v)[NV], double* red, double* sc) {
  block_sum<NV, PNT>(v, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < NV; ++k) sc[k] = v[k];
  __syncthreads();
  for (int k = 0; k < NV; ++k) v[k] = sc[k];
  __syncthreads();
}

// One projection solve K x = -(b - mean b) by flexible CG with the V-cycle
// preconditioner, to relative residual rtol; guess as in k_pcg_init.  Leaves
// x in I.x and returns the iteration count.
template <typename S>
__device__ int persist_solve(const Inst& I, PersistLds<S>& L, int guess,
                             int stage, int hw, double bmean, double rtol, int maxit, bool& zero,
                             double& xmean, double& relres, bool& converged) {
  const int nx = I.nx, ny = I.ny, n = nx * ny;
  const int tid = threadIdx.x;
  const FastDiv dn(nx);
  double* x = I.x;
  double* r = I.rr;
  double* d = I.d0;
  double* q = I.q;
  const GuessSrc G = guess_src(I, stage, hw);
  double s2[2] = {0.0, 0.0};
  for (int c = tid; c < n; c += PNT) {
    const int j = dn.div(c), i = c - j * nx;
    double f, rv;
    pcg_init_cell(I, G, guess, j, i, bmean, f, rv);
    s2[0] += f * f;
    s2[1] += rv * rv;
  }
  pall_sum<2>(s2, L.red, L.sc);
  const double fnorm = sqrt(s2[0]);
  zero = s2[0] == 0.0;
  relres = zero ? 0.0 : sqrt(s2[1]) / fnorm;
  S* r0 = I.mixed ? gas<S>(I.mg_r0) : (S*)(void*)r;
  const bool lds0 = I.lc == 0;
  auto view = [&](int l) { return mixed_view<S>(I, L.u.coarse, r0, l); };
  int it = 0;
  double dq_old = 0.0;
  (void)ny;
  while (!zero && relres > rtol && it < maxit) {
    // z = M r
    if (lds0 || I.mixed) {
      S* rl = lds0 ? view(0).r : r0;
      for (int c = tid; c < n; c += PNT) rl[c] = (S)r[c];
      __syncthreads();
    }
    mg_cycle<S>(I, view, 0, I.nlev, I.nu, L.red, L.sc, L.u.coarse.cg);
    const S* z = view(0).z;
    // flexible CG: the new direction is K-orthogonalised against the last one
    double beta = 0.0;
    if (it > 0) {
      double zq[1] = {0.0};
      for (int c = tid; c < n; c += PNT) zq[0] += (double)z[c] * q[c];
      pall_sum<1>(zq, L.red, L.sc);
      beta = dq_old != 0.0 ? -zq[0] / dq_old : 0.0;
    }
    for (int c = tid; c < n; c += PNT) d[c] = it > 0 ? (double)z[c] + beta * d[c] : (double)z[c];
    __syncthreads();
    double dd[2] = {0.0, 0.0};
    for (int c = tid; c < n; c += PNT) {
      const int j = dn.div(c), i = c - j * nx;
      const double qv = apply_K(I, d, j, i);
      q[c] = qv;
      dd[0] += d[c] * r[c];
      dd[1] += d[c] * qv;
    }
    pall_sum<2>(dd, L.red, L.sc);
    const double alpha = dd[1] != 0.0 ? dd[0] / dd[1] : 0.0;
    double rr[1] = {0.0};
    for (int c = tid; c < n; c += PNT) {
      x[c] += alpha * d[c];
      const double rv = r[c] - alpha * q[c];
      r[c] = rv;
      rr[0] += rv * rv;
    }
    pall_sum<1>(rr, L.red, L.sc);
    relres = sqrt(rr[0]) / fnorm;
    dq_old = dd[1];
    ++it;
    if (alpha == 0.0) break;   // stagnation: no further progress possible
  }
  double sx[1] = {0.0};
  for (int c = tid; c < n; c += PNT) sx[0] += x[c];
  pall_sum<1>(sx, L.red, L.sc);
  xmean = sx[0] / n;
  converged = zero || relres <= rtol;
  return it;
}

// nsteps RK4 steps, one instance per workgroup, the first of them step
// number step0 (its pressure-history ring slot is step0 mod 4).  guess: 0
// zero, 1 previous pressure (the per-stage history once `hist` + steps done
// >= 1, its time extrapolation once >= 2).  accumulate: add this launch's count of
// unconverged solves and its largest iteration count to the ones recorded.
template <typename S>
__global__ void __launch_bounds__(PNT) k_step_persistent(const Tile* __restrict__ tiles,
                                                         const Inst* __restrict__ insts,
                                                         int nsteps, int step0, int hist, int guess,
                                                         int order,
                                                         double rtol, int maxit, int accumulate) {
  __shared__ PersistLds<S> L;
  const Inst& I = insts[blockIdx.x];
  PcgScalars* P = I.pcg;
  const int tid = threadIdx.x, q4 = tid / kNT, lt = tid - q4 * kNT;
  const int nx = I.nx, ny = I.ny, n = nx * ny;
  const FastDiv dn(nx);
  const bool variable_rho = I.rho1 != I.rho2;
  const double RKc[4] = {0.5, 0.5, 1.0, 1.0};
  const double RKb[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
  bool coef_done = false;
  int nfail = 0, max_it = 0;
  for (int s = 0; s < nsteps; ++s) {
    for (int k = 0; k < 4; ++k) {
      const int src = k == 0 ? 0 : (k == 2 ? 2 : 1);
      const int dst = (k == 0 || k == 2) ? 1 : 2;
      const CDI_GLOBAL double* phd = dst == 1 ? I.phi_a : I.phi_b;
      // phase preparation and stage operator, PQ tiles at a time
      for (int base = 0; base < I.ntiles; base += PQ) {
        const int ti = base + q4;
        const bool active = ti < I.ntiles;
        const Tile t = tiles[I.first_tile + (active ? ti : 0)];
        phase_prep_tile<S>(t, I, src, L.u.prep[q4], lt, active);
        __syncthreads();
      }
      for (int base = 0; base < I.ntiles; base += PQ) {
        const int ti = base + q4;
        const bool active = ti < I.ntiles;
        const Tile t = tiles[I.first_tile + (active ? ti : 0)];
        stage_tile<S>(t, I, k, src, dst, RKc[k], RKb[k], k == 3, L.u.stage[q4], lt, active);
        __syncthreads();
      }
      // projection right-hand side and operator coefficients
      const double tfac = RKc[k];
      double bs[1] = {0.0};
      for (int c = tid; c < n; c += PNT) {
        const int j = dn.div(c), i = c - j * nx;
        bs[0] += rhs_cell<S>(I, phd, j, i, tfac);
      }
      pall_sum<1>(bs, L.red, L.sc);
      const double bmean = bs[0] / n;
      if (variable_rho || !coef_done) {
        for (int l = 1; l < I.nlev; ++l) {
          mg_coef_level<S>(I, l, tid, PNT);
          __syncthreads();
        }
        coarse_inverse<S>(I, L.u.B, L.red, L.sc);
        __syncthreads();
        coef_done = true;
      }
      coarse_load_coef<S>(I, L.u.coarse);
      __syncthreads();
      int gm = guess;
      const int hs = hist + s;
      if (gm == 1 && hs >= 1) gm = history_mode(hs, order);
      bool zero, conv;
      double xmean, relres;
      const int hw = (step0 + s) & 3;   // history ring slot of this step
      const int it = persist_solve<S>(I, L, gm, k, hw, bmean, rtol, maxit, zero, xmean, relres, conv);
      if (!conv) ++nfail;
      max_it = it > max_it ? it : max_it;
      if (tid == 0) {
        P->bmean = bmean;
        P->iters = it;
        P->iters_total += it;
        P->relres = relres;
        P->nonfinite = isfinite(relres) ? 0 : 1;
        P->converged = conv ? 1 : 0;
        P->zero_rhs = zero ? 1 : 0;
        P->xmean = xmean;
        P->done = 1;
      }
      for (int c = tid; c < n; c += PNT) {
        const int j = dn.div(c), i = c - j * nx;
        project_cell(I, tfac, k == 3, phd, k, hw, zero, xmean, j, i);
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    P->nfail = (accumulate ? P->nfail : 0) + nfail;
    P->max_iters = accumulate && P->max_iters > max_it ? P->max_iters : max_it;
  }
  (void)ny;
}

}  // namespace cdi
