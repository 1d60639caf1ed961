// Diagnostics and operator-evaluation kernels: FP64 reductions of the state
// (mass, phase-field bounds, divergence, kinetic energy, finiteness) and the
// GNBC wall values of the current state (Sec. 5.1 metrics).
#pragma once
#include <climits>

#include "poisson_kernels.h"

namespace cdi {

constexpr int kMaxContacts = 2;   // phi = 1/2 wall crossings stored per wall

struct DiagOut {
  double mass, phi_min, phi_max, max_div, ke, nonfinite;
  double contact_x[2][kMaxContacts];   // [wall][first crossings in column order]
  double wetted_len[2], theta_est[2];
  int n_contact[2];
  double pad[3];
};

template <int NV, int NT = kNT>
__device__ __forceinline__ void block_max(double (&v)[NV], double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_max(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k * (NT / 64) + w] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = sh[k * (NT / 64)];
      for (int ww = 1; ww < NT / 64; ++ww) s = fmax(s, sh[k * (NT / 64) + ww]);
      v[k] = s;
    }
  }
  __syncthreads();
}

// Cell reductions of instance state: sum(phi), -min(phi), max(phi),
// max |div u|, kinetic energy, non-finite count.
__global__ void __launch_bounds__(kNT) k_diag(const Tile* __restrict__ tiles,
                                              const Inst* __restrict__ insts, DiagOut* out) {
  __shared__ double sh[3 * kNT / 64];
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  const int nx = I.nx, ny = I.ny;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int i = t.i0 + tx, j = t.j0 + ty;
  double s[3] = {0.0, 0.0, 0.0};      // sum phi, ke, nonfinite
  double m[3] = {-1e300, -1e300, 0.0}; // -min phi, max phi, max |div|
  if (i < nx && j < ny) {
    const size_t o = (size_t)j * nx + i;
    const double ph = I.phi[o];
    const double u = I.u[o], v = I.v[o];
    const double ue = I.u[(size_t)j * nx + wrap(i + 1, nx)], vn = I.v[o + nx];
    s[0] = ph;
    const double r1 = I.rho1, r2 = I.rho2;
    const double rc = (r1 - r2) * ph + r2;
    const double rw = (r1 - r2) * I.phi[(size_t)j * nx + wrap(i - 1, nx)] + r2;
    double ke = 0.5 * (rw + rc) * u * u;
    if (j >= 1) ke += 0.5 * ((r1 - r2) * I.phi[o - nx] + r2 + rc) * v * v;
    s[1] = 0.5 * ke * I.h * I.h;
    const double pr = I.p[o];
    s[2] = (isfinite(ph) && isfinite(u) && isfinite(v) && isfinite(pr)) ? 0.0 : 1.0;
    m[0] = -ph;
    m[1] = ph;
    m[2] = fabs(((ue - u) + (vn - v)) * I.inv_h);
  }
  block_sum<3>(s, sh);
  __syncthreads();
  if (threadIdx.x == 0) {
    st_agent(&I.part[t.local], s[0]);
    st_agent(&I.part[I.ntiles + t.local], s[1]);
    st_agent(&I.part[2 * I.ntiles + t.local], s[2]);
  }
  block_max<3>(m, sh);
  if (threadIdx.x == 0) {
    st_agent(&I.part[3 * I.ntiles + t.local], m[0]);
    st_agent(&I.part[4 * I.ntiles + t.local], m[1]);
    st_agent(&I.part[5 * I.ntiles + t.local], m[2]);
  }
  if (arrive_last(I.counters + 5 * kCounterStride, I.ntiles, t.local)) {
    const int n = I.ntiles;
    const double a = sum_partials(I.part, n, sh);
    const double b = sum_partials(I.part + n, n, sh);
    const double c = sum_partials(I.part + 2 * n, n, sh);
    double mm[3] = {-1e300, -1e300, 0.0};
    for (int k = threadIdx.x; k < n; k += kNT) {
      mm[0] = fmax(mm[0], ld_agent(&I.part[3 * n + k]));
      mm[1] = fmax(mm[1], ld_agent(&I.part[4 * n + k]));
      mm[2] = fmax(mm[2], ld_agent(&I.part[5 * n + k]));
    }
    block_max<3>(mm, sh);
    if (threadIdx.x == 0) {
      DiagOut& D = out[t.inst];
      D.mass = a * I.h * I.h;
      D.ke = b;
      D.nonfinite = c;
      D.phi_min = -mm[0];
      D.phi_max = mm[1];
      D.max_div = mm[2];
    }
  }
}

// GNBC wall values (u^Y, u_wall - U) of the current state at every wall
// corner; needs the wall arrays of k_phase_prep on the caller phase field.
__global__ void __launch_bounds__(kNT) k_wall(const Inst* __restrict__ insts) {
  const Inst& I = insts[blockIdx.x];
  const int nx = I.nx, ny = I.ny;
  for (int c = threadIdx.x; c < 2 * nx; c += kNT) {
    const int wall = c / nx, i = c - wall * nx;
    const double ur = I.u[(size_t)(wall == 0 ? 0 : ny - 1) * nx + i];
    double uY, usl;
    (void)gnbc_corner(I, wall, i, ur, uY, usl);
    I.uY[c] = uY;
    I.uslip[c] = usl;
  }
}

// Contact angle of a circular cap whose base chord is L and whose area is
// `area`: the root on (0, pi) of (L / (2 sin t))^2 (t - sin t cos t) = area
// (the cap of radius R = L / (2 sin t) has area R^2 (t - sin t cos t)),
// found by bisection.
__device__ inline double cap_angle(double L, double area) {
  auto f = [&](double t) {
    const double s = sin(t);
    const double r = L / (2.0 * s);
    return r * r * (t - s * cos(t)) - area;
  };
  double lo = 1e-6, hi = M_PI - 1e-6;
  double flo = f(lo);
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    const double fm = f(mid);
    if ((fm > 0.0) == (flo > 0.0)) {
      lo = mid;
      flo = fm;
    } else {
      hi = mid;
    }
  }
  return 0.5 * (lo + hi);
}

// Contact-line measures of Sec. 5.1 at each wall: the positions where the
// wall phase field (extrapolated per column from the first two cell rows,
// Sec. 4) crosses 1/2, by linear interpolation between column centres
// (x periodic, a column that holds exactly 1/2 counts as a crossing at its
// centre), numbered in column order; the wetted length |x1 - x0| of a wall
// with exactly two crossings; and the contact angle of the circular cap
// with that chord and the instance's phase-field area sum(phi) h^2.  One
// block per (instance, wall); needs k_phase_prep's wall arrays on the caller
// phase field and k_diag's mass.
__global__ void __launch_bounds__(kNT) k_contact(const Inst* __restrict__ insts,
                                                 DiagOut* __restrict__ out) {
  __shared__ int sh[kNT / 64];
  const int wall = blockIdx.y;
  const Inst& I = insts[blockIdx.x];
  const int nx = I.nx;
  const double* __restrict__ W = I.wall + (size_t)wall * 5 * nx;   // phi_w per column
  auto crosses = [&](int i) {
    const double a = W[i] - 0.5, b = W[wrap(i + 1, nx)] - 0.5;
    return a == 0.0 || a * b < 0.0;
  };
  auto block_int = [&](int v, bool is_min) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const int o = __shfl_xor(v, off, 64);
      v = is_min ? min(v, o) : v + o;
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    int r = sh[0];
    for (int w = 1; w < kNT / 64; ++w) r = is_min ? min(r, sh[w]) : r + sh[w];
    return r;
  };
  int cnt = 0;
  for (int i = threadIdx.x; i < nx; i += kNT) cnt += crosses(i) ? 1 : 0;
  const int total = block_int(cnt, false);
  int cols[kMaxContacts];
  int last = -1;
#pragma unroll
  for (int m = 0; m < kMaxContacts; ++m) {
    int best = INT_MAX;
    // this thread's columns ascend: its first crossing past `last` is its smallest
    for (int i = threadIdx.x; i < nx; i += kNT)
      if (i > last && crosses(i)) {
        best = i;
        break;
      }
    best = block_int(best, true);
    cols[m] = best;
    if (best != INT_MAX) last = best;
  }
  if (threadIdx.x == 0) {
    DiagOut& D = out[blockIdx.x];
    const double h = I.h;
    for (int m = 0; m < kMaxContacts; ++m) {
      double x = 0.0;
      if (cols[m] != INT_MAX) {
        const int i = cols[m];
        const double a = W[i] - 0.5, b = W[wrap(i + 1, nx)] - 0.5;
        x = (i + 0.5) * h;
        if (a != 0.0) x += h * a / (a - b);
      }
      D.contact_x[wall][m] = x;
    }
    D.n_contact[wall] = total;
    double L = 0.0, th = 0.0;
    if (total == 2) {
      L = fabs(D.contact_x[wall][1] - D.contact_x[wall][0]);
      th = cap_angle(L, D.mass);
    }
    D.wetted_len[wall] = L;
    D.theta_est[wall] = th;
  }
}

// Copy a user right-hand side into the solver and build the operator from
// the caller phase field (standalone pressure solve); also resets the CG.
template <typename S>
__global__ void __launch_bounds__(kNT) k_solve_setup(const Tile* __restrict__ tiles,
                                                     const Inst* __restrict__ insts,
                                                     const double* __restrict__ bin, double rtol,
                                                     int maxit) {
  __shared__ double sh[2 * kNT / 64];
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  const int nx = I.nx, ny = I.ny;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int i = t.i0 + tx, j = t.j0 + ty;
  double bs[2] = {0.0, 0.0};
  if (i < nx && j < ny) {
    const size_t o = (size_t)j * nx + i;
    const double r1 = I.rho1, r2 = I.rho2;
    const double rc = (r1 - r2) * I.phi[o] + r2;
    const double rw = (r1 - r2) * I.phi[(size_t)j * nx + wrap(i - 1, nx)] + r2;
    const double ih2 = I.inv_h * I.inv_h;
    const double ax = ih2 / (0.5 * (rw + rc));
    double ay = 0.0;
    if (j >= 1) ay = ih2 / (0.5 * ((r1 - r2) * I.phi[o - nx] + r2 + rc));
    I.ax0[o] = ax;
    I.ay0[o] = ay;
    if (I.mixed) {
      (gas<S>(I.lev[0].ax))[o] = (S)ax;
      (gas<S>(I.lev[0].ay))[o] = (S)ay;
    }
    const double b = bin ? bin[o] : I.b[o];
    I.b[o] = b;
    bs[0] = b;
    bs[1] = b * b;
  }
  block_sum<2>(bs, sh);
  if (threadIdx.x == 0) {
    st_agent(&I.part[t.local], bs[0]);
    st_agent(&I.part[I.ntiles + t.local], bs[1]);
  }
  if (arrive_last(I.counters + 0 * kCounterStride, I.ntiles, t.local)) {
    const double s = sum_partials(I.part, I.ntiles, sh);
    const double s2 = sum_partials(I.part + I.ntiles, I.ntiles, sh);
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

// Regularisation velocity of each instance's next step.  Fixed gamma:
// gamma itself (k_gamma_init, once).  gamma_factor > 0 (the paper's gamma =
// 2.5 |u|_max, Sec. 5): min(gamma, gamma_factor * max |u|, |v|) over the
// faces of the state the step starts from -- the largest value per cell tile,
// then over the tiles' partials by the last block (k_gamma_step, at the
// start of every step).
__global__ void k_gamma_init(const Inst* __restrict__ insts, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) insts[k].pcg->gamma_step = insts[k].gamma;
}

__global__ void __launch_bounds__(kNT) k_gamma_step(const Tile* __restrict__ tiles,
                                                    const Inst* __restrict__ insts) {
  __shared__ double sh[kNT / 64];
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (!(I.gamma_factor > 0.0)) return;   // the same for every block of the instance
  const int nx = I.nx, ny = I.ny;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int i = t.i0 + tx, j = t.j0 + ty;
  double m = 0.0;
  if (i < nx && j < ny) {   // v rows 0..ny-1; row ny is a wall and holds 0
    const size_t o = (size_t)j * nx + i;
    m = fmax(fabs(I.u[o]), fabs(I.v[o]));
  }
  m = block_max(m, sh);
  if (threadIdx.x == 0) st_agent(&I.part[t.local], m);
  if (arrive_last(I.counters + 0 * kCounterStride, I.ntiles, t.local)) {
    double mm = 0.0;
    for (int k = threadIdx.x; k < I.ntiles; k += kNT) mm = fmax(mm, ld_agent(&I.part[k]));
    mm = block_max(mm, sh);
    if (threadIdx.x == 0) I.pcg->gamma_step = fmin(I.gamma, I.gamma_factor * mm);
  }
}

// Every instance's CG scalars side by side (one thread per instance), so that
// the host reads a batch's scalars with one copy instead of one per instance.
__global__ void k_gather_pcg(const Inst* __restrict__ insts, int n, PcgScalars* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = *insts[k].pcg;
}

// Graph path bookkeeping, one thread per instance: clear the step's miss flag
// and iteration maximum (begin), or record whether the solve just enqueued
// converged within its fixed iteration budget (end).
__global__ void k_graph_mark(const Inst* __restrict__ insts, int n, int begin) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  PcgScalars* P = insts[k].pcg;
  if (begin) {
    P->miss = 0;
    P->step_iters = 0;
  } else {
    if (!P->done) P->miss = 1;
    if (P->iters > P->step_iters) P->step_iters = P->iters;
  }
}

// Step snapshot of instance blockIdx.y: the fields phi, u, p, the stage
// pressure history hp[d][stage] (d-major; n values each) and v (n + nx) stored
// one after another in I.snap (save), or copied back from it.  One launch
// instead of a copy per field.
__global__ void __launch_bounds__(kNT) k_snapshot(const Inst* __restrict__ insts, int save) {
  const Inst& I = insts[blockIdx.y];
  const size_t n = (size_t)I.nx * I.ny;
  constexpr size_t kF = 3 + 4 * kHistDepth;   // fields of n values before v
  const size_t total = (kF + 1) * n + I.nx;
  for (size_t e = (size_t)blockIdx.x * kNT + threadIdx.x; e < total; e += (size_t)gridDim.x * kNT) {
    const size_t f = e / n < kF ? e / n : kF;
    const size_t o = e - f * n;
    double* fld;
    switch (f) {
      case 0: fld = I.phi; break;
      case 1: fld = I.u; break;
      case 2: fld = I.p; break;
      default: fld = f < kF ? I.hp[(f - 3) / 4][(f - 3) % 4] : I.v; break;
    }
    if (save) I.snap[e] = fld[o];
    else fld[o] = I.snap[e];
  }
}

// Mean-free solution of a standalone solve into the caller's buffer.
__global__ void __launch_bounds__(kNT) k_solve_out(const Tile* __restrict__ tiles,
                                                   const Inst* __restrict__ insts, double* pout) {
  const Tile t = tiles[blockIdx.x];
  const Inst& I = insts[t.inst];
  const int nx = I.nx, ny = I.ny;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int i = t.i0 + tx, j = t.j0 + ty;
  if (i >= nx || j >= ny) return;
  const size_t o = (size_t)j * nx + i;
  const bool zero = I.pcg->zero_rhs != 0;
  pout[o] = zero ? 0.0 : I.x[o] - I.pcg->xmean;
}

// Learned-guess features of one instance's projection: phi, rho/rho_max and
// (b - mean b)/rms (0 where rms = 0), FP32 [3][ny][nx]; optionally the
// normalised target p / (rms rho_max h^2) from the pressure p (the right-hand
// sides of the projections vary on the grid scale, so h^2 sets the scale).
__global__ void __launch_bounds__(kNT) k_features(const Inst* __restrict__ insts, int idx,
                                                  const double* __restrict__ phi,
                                                  const double* __restrict__ p,
                                                  float* __restrict__ feat,
                                                  float* __restrict__ target) {
  const Inst& I = insts[idx];
  const size_t n = (size_t)I.nx * I.ny;
  const double rmax = fmax(I.rho1, I.rho2);
  const double mean = I.pcg->bmean, rms = I.pcg->brms;
  const double pscale = rms * rmax * I.h * I.h;
  for (size_t c = blockIdx.x * (size_t)kNT + threadIdx.x; c < n; c += (size_t)gridDim.x * kNT) {
    const double ph = phi[c];
    feat[c] = (float)ph;
    feat[n + c] = (float)(((I.rho1 - I.rho2) * ph + I.rho2) / rmax);
    // the right-hand side peaks at hundreds of its rms near the interface:
    // asinh keeps its sign and small values and compresses the peaks
    feat[2 * n + c] = rms > 0.0 ? (float)asinh((I.b[c] - mean) / rms) : 0.f;
    if (target) target[c] = pscale > 0.0 ? (float)(p[c] / pscale) : 0.f;
  }
}

// Training target scaled to unit rms (one block; FP64 sum of squares in a
// fixed order).  The guess enters the solve only through the energy-norm fit
// of k_guess_fit, which is invariant to its scale, so the network is trained
// on the shape of the pressure: snapshots whose pressure levels differ by
// orders of magnitude then weigh alike in the loss.
__global__ void __launch_bounds__(kNT) k_target_unit_rms(float* __restrict__ target, size_t n) {
  __shared__ double sh[kNT / 64];
  __shared__ double s_scale;
  double s[1] = {0.0};
  for (size_t c = threadIdx.x; c < n; c += kNT) s[0] += (double)target[c] * target[c];
  block_sum<1>(s, sh);
  if (threadIdx.x == 0) s_scale = s[0] > 0.0 ? 1.0 / sqrt(s[0] / (double)n) : 0.0;
  __syncthreads();
  const double f = s_scale;
  for (size_t c = threadIdx.x; c < n; c += kNT) target[c] = (float)(target[c] * f);
}

// Pressure guess from the network output: g = y rms rho_max h^2, held in zf
// until k_guess_fit combines it with the previous pressure.
__global__ void __launch_bounds__(kNT) k_guess_apply(const Inst* __restrict__ insts,
                                                     const float* __restrict__ y) {
  const Inst& I = insts[0];
  const size_t n = (size_t)I.nx * I.ny;
  const double pscale = I.pcg->brms * fmax(I.rho1, I.rho2) * I.h * I.h;
  for (size_t c = blockIdx.x * (size_t)kNT + threadIdx.x; c < n; c += (size_t)gridDim.x * kNT)
    I.zf[c] = (double)y[c] * pscale;
}

}  // namespace cdi
