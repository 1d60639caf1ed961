// Device-side data structures and helpers of the CDI + GNBC step (gfx950).
//
// Every kernel works on a list of tiles that may span several independent
// instances (the batched ensemble); a single problem is a batch of one.  Each
// instance carries its own grid, parameters, state pointers and multigrid
// hierarchy, all inside caller-owned device memory.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cdi {

constexpr int kMaxLevels = 14;
constexpr int kNT = 256;          // threads per block of every tiled kernel
constexpr double kDeltaN = 1e-12; // normal-vector regularisation: n = G/(|G| + dN)
constexpr double kDeltaPsi = 1e-12;

// One multigrid level of one instance.  Coefficients a = 1/(rho_f h_l^2) on
// x-faces (ny_l * nx_l, face i = west face of cell i) and y-faces
// ((ny_l+1) * nx_l, face j = south face of cell j; rows 0 and ny_l are walls
// and hold 0).  The storage type S is double (FP64 path) or float (mixed).
struct Level {
  int nx, ny;
  int first_tile, ntiles;   // tiles of this level in the level's tile list
  void* ax;                 // S[ny*nx]
  void* ay;                 // S[(ny+1)*nx]
  void* r;                  // S[ny*nx]  residual / right-hand side of the level
  void* z;                  // S[ny*nx]  correction of the level
};

// Per-instance scalars of the flexible CG, written by the last block of the
// reduction kernels (deterministic fixed-order sums).
struct PcgScalars {
  double alpha, beta;
  double dr, dq, zq;        // (d, r), (d, q), (z, q)
  double rr, fnorm, relres;
  double bmean, xmean;
  double rtol;
  int done;                 // 1 once converged (or maxit reached): kernels exit early
  int iters;
  int maxit;
  int first;                // 1 before the first direction is formed
  int converged;
  int pad;
  unsigned counter[8];      // arrival counters of the last-block reductions
};

struct Inst {
  // grid and physics (Sec. 2, Sec. 4)
  int nx, ny;
  int nlev, lc;             // multigrid levels; first level done by the coarse kernel
  int slip_model, mixed;
  int first_tile, ntiles;   // tiles of level 0 in the cell tile list
  double h, inv_h, eps, gamma, sigma, cos_eq;
  double rho1, rho2, mu1, mu2, beta1, beta2, uw_bot, uw_top, dt;
  // caller state (FP64)
  double* phi; double* u; double* v; double* p;
  // workspace: stage state and RK accumulators (FP64)
  double* phi_a; double* phi_b;        // ping-pong stage phase field
  double* us; double* vs;              // stage velocity after projection
  double* mx; double* my;              // (rho u)* before division
  double* ustar; double* vstar;        // u* before projection
  double* acc_phi; double* acc_mx; double* acc_my;
  // phase-field quantities (S)
  void* nhx; void* nhy; void* muc;
  double* wall;                        // [2 walls][5 q][nx]: phi_w, psi_w, dpsi_w, kappa_w, dphi_w
  double* uY; double* uslip;           // [2][nx] wall corner diagnostics
  // level-0 FP64 coefficients a = 1/(rho_f h^2) of the pressure operator
  double* ax0; double* ay0;
  // pressure (FP64 CG vectors)
  double* b; double* x; double* rr; double* d0; double* d1; double* q;
  double* zf;                          // FP64 copy of level-0 correction (mixed path)
  double* part;                        // reduction partials, [8][ntiles]
  PcgScalars* pcg;
  Level lev[kMaxLevels];
  double* coarse_ws;                   // coarse CG vectors
};

struct Tile {
  int inst;
  int i0, j0;
  int level;
  int local;                // index of this tile among the instance's tiles of the level
  int pad[3];
};

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) { T o = __shfl_xor(v, off, 64); v = o > v ? o : v; }
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) { T o = __shfl_xor(v, off, 64); v = o < v ? o : v; }
  return v;
}

// Fixed-order block sum of NV values per thread; result valid in thread 0.
// Every thread of the block must call it (it contains a barrier).
template <int NV, int NT = kNT>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh /* >= NV*NT/64 */) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k * (NT / 64) + w] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int ww = 0; ww < NT / 64; ++ww) s += sh[k * (NT / 64) + ww];
      v[k] = s;
    }
  }
}

// Coherent load of a value published by another block of the same launch.
__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Last-block-done: every block of an instance publishes its partial, then
// counts itself in; the last one to arrive sees all partials.
__device__ __forceinline__ bool arrive_last(unsigned* counter, int nblocks) {
  __shared__ int s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned prev = atomicAdd(counter, 1u);
    s_last = (prev == (unsigned)(nblocks - 1));
    if (s_last) {
      __threadfence();
      atomicExch(counter, 0u);
    }
  }
  __syncthreads();
  return s_last != 0;
}

}  // namespace cdi
