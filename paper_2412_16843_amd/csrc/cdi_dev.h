// Device-side data structures and helpers of the CDI + GNBC step (gfx950).
//
// Every kernel works on a list of tiles that may span several independent
// instances (the batched ensemble); a single problem is a batch of one.  Each
// instance carries its own grid, parameters, state pointers and multigrid
// hierarchy, all inside caller-owned device memory.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cdi_math.h"

namespace cdi {

constexpr int kMaxLevels = 14;
// levels held in the one-block coarse kernel's LDS (from a level of at most
// 1024 cells, halving while above 64: 1024, 256, 64)
constexpr int kMaxCoarseLevels = 4;
constexpr int kHistDepth = 4;    // steps of per-stage pressure kept for the initial guess
constexpr int kNT = 256;          // threads per block of every tiled kernel
constexpr double kDeltaN = 1e-12; // normal-vector regularisation: n = G/(|G| + dN)
constexpr double kDeltaPsi = 1e-12;

// Pointer to device global memory held in a descriptor struct.  The host
// stores and reads it as a plain pointer; device code reads it as a pointer
// into the global address space, so that every access through it is a
// global (not flat) memory instruction: a flat access also counts against the
// LDS wait counter, so an LDS wait of a kernel with flat loads in flight
// would wait for those loads too.  (The global-space pointer must leave the
// conversion function as such: converted back to a generic pointer inside
// the same function, the compiler folds the pair of casts away.)
#if defined(__HIP_DEVICE_COMPILE__)
#define CDI_GLOBAL __attribute__((address_space(1)))
#else
#define CDI_GLOBAL
#endif
template <typename T>
struct gptr {
  T* p;
  gptr() = default;
  __host__ __device__ constexpr gptr(T* q) : p(q) {}
  __host__ __device__ __forceinline__ operator CDI_GLOBAL T*() const { return (CDI_GLOBAL T*)p; }
  __host__ __device__ __forceinline__ CDI_GLOBAL T* operator->() const { return (CDI_GLOBAL T*)p; }
};
// Typed view of an untyped global pointer (arrays whose element type S is
// the instance's storage precision).
template <typename U>
__host__ __device__ __forceinline__ CDI_GLOBAL U* gas(gptr<void> g) { return (CDI_GLOBAL U*)g.p; }

// One multigrid level of one instance.  Coefficients a = 1/(rho_f h_l^2) on
// x-faces (ny_l * nx_l, face i = west face of cell i) and y-faces
// ((ny_l+1) * nx_l, face j = south face of cell j; rows 0 and ny_l are walls
// and hold 0).  The storage type S is double (FP64 path) or float (mixed).
struct Level {
  int nx, ny;
  int first_tile, ntiles;   // tiles of this level in the level's tile list
  gptr<void> ax;                 // S[ny*nx]
  gptr<void> ay;                 // S[(ny+1)*nx]
  gptr<void> r;                  // S[ny*nx]  residual / right-hand side of the level
  gptr<void> z;                  // S[ny*nx]  correction of the level (pre-smoothed on tiled levels)
  gptr<void> zo;                 // S[ny*nx]  post-smoothed correction written by the tiled up-sweep
                            //           (levels 1..lg-1; a launch never reads what it writes)
};

// Per-instance scalars of the flexible CG, written by the last block of the
// reduction kernels (deterministic fixed-order sums).
struct PcgScalars {
  double alpha, beta;
  double dr, dq, zq;        // (d, r), (d, q), (z, q)
  double rr, fnorm, relres;
  double bmean, xmean, brms;
  double gscale, gscale2;   // x0 = gscale p + gscale2 g for the learned guess g
  double gamma_step;        // regularisation velocity of the current step
  double rtol;
  int done;                 // 1 once converged (or maxit reached): kernels exit early
  int iters;
  int maxit;
  int first;                // 1 before the first direction is formed
  int converged;
  int zero_rhs;             // 1 when the right-hand side vanished (p = 0)
  int coef_ok;              // persistent path: coarse coefficients current
  int nfail;                // persistent path: solves that stopped at maxit
  int max_iters;            // persistent path: largest iteration count
  int miss;                 // graph path: a solve of the step ended unconverged
  int step_iters;           // graph path: largest iteration count of the step
  int nonfinite;            // 1 once a norm of the solve was NaN or Inf (the solve stops)
  int gbase;                // guess mode of the fitted base of the learned guess (1, 3..6)
  int pad;
  long long iters_total;    // CG iterations run since the context was set up (every launch
                            // form, tuning trials and redone graph steps included)
};

struct Inst {
  // grid and physics (Sec. 2, Sec. 4)
  int nx, ny;
  int nlev, lc;             // multigrid levels; first level held in the coarse kernel's LDS
  int lg;                   // first level done by the one-block coarse kernel (lg <= lc)
  // LDS offsets of the coarse levels lc + m (cells, y-faces): prefix sums,
  // the total repeated past the last level
  int cpre_x[kMaxCoarseLevels + 1], cpre_y[kMaxCoarseLevels + 1];
  int nu;                   // red-black sweep pairs before and after the coarse correction
  int nu_c;                 // sweep pairs on the levels of the one-block coarse cycle: nu + 1
                            // (its sweeps cost barrier latency, not bandwidth, and the extra
                            // pair saves outer CG iterations)
  int slip_model, mixed;
  int first_tile, ntiles;   // tiles of level 0 in the cell tile list
  int first_wide, nwide;    // tiles of level 0 in the wide tile list
  double h, inv_h, eps, inv_eps, gamma, sigma, cos_eq;
  double gamma_factor;      // > 0: gamma of a step = min(gamma, gamma_factor max|u|)
  double rho1, rho2, mu1, mu2, beta1, beta2, uw_bot, uw_top, dt;
  // caller state (FP64)
  gptr<double> phi; gptr<double> u; gptr<double> v; gptr<double> p;
  // workspace: stage state and RK accumulators (FP64)
  gptr<double> phi_a; gptr<double> phi_b;        // ping-pong stage phase field
  gptr<double> us; gptr<double> vs;              // stage velocity after projection
  gptr<double> mx; gptr<double> my;              // (rho u)* before division
  gptr<double> ustar; gptr<double> vstar;        // u* before projection
  gptr<double> acc_phi; gptr<double> acc_mx; gptr<double> acc_my;
  // phase-field quantities (S)
  gptr<void> nhx; gptr<void> nhy; gptr<void> muc;
  gptr<double> wall;                        // [2 walls][5 q][nx]: phi_w, psi_w, dpsi_w, kappa_w, dphi_w
  gptr<double> uY; gptr<double> uslip;           // [2][nx] wall corner diagnostics
  // level-0 FP64 coefficients a = 1/(rho_f h^2) of the pressure operator
  gptr<double> ax0; gptr<double> ay0;
  // pressure (FP64 CG vectors)
  gptr<double> b; gptr<double> x; gptr<double> rr; gptr<double> rr2; gptr<double> d0; gptr<double> d1; gptr<double> q;
  gptr<double> zf;                          // FP64 copy of level-0 correction (mixed path)
  gptr<double> hp[kHistDepth][4];           // pressure of each RK stage d + 1 steps back (d = 0: the last step)
  gptr<double> part;                        // reduction partials, [8][ntiles]
  gptr<PcgScalars> pcg;
  gptr<unsigned> counters;                  // [8 kinds][kCounterStride] arrival counters
  Level lev[kMaxLevels];
  gptr<double> snap;                        // graph path: state at the start of the step
  gptr<void> mg_t;                          // S [ny*nx] residual scratch of the one-block V-cycle
  gptr<void> mg_r0;                         // S [ny*nx] level-0 residual copy (mixed, one-block V-cycle)
  gptr<double> cinv;                        // dense inverse of the coarsest operator (n <= 64)
  int cdense;                          // 1 if cinv is used for the coarsest solve
  int coef_const;                      // 1: uniform density, operator coefficients constant
};

struct Tile {
  int inst;
  int i0, j0;
  int level;
  int local;                // index of this tile among the instance's tiles of the level
  int pad;
  gptr<PcgScalars> pcg;     // the instance's CG scalars (set on the multigrid and wide tiles):
                            // its done flag is read with the instance's descriptor, not after it
};
static_assert(sizeof(Tile) == 32, "tile descriptor layout");

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Quotient by a runtime divisor d >= 1 for any non-negative int n: a
// double-precision reciprocal estimate (off by at most one) corrected by one
// exact integer step (the GPU has no integer divide instruction; the generic
// sequence costs tens of operations).
// Initial-guess mode of a solve whose RK stage has hs >= 1 steps of pressure
// history: 3 + q, where q is the order of the polynomial extrapolation in
// time through the last q + 1 steps (0 the last step's pressure, 1 linear,
// 2 quadratic, 3 cubic), the highest that hs supports, at most max_order.
__host__ __device__ inline int history_mode(int hs, int max_order) {
  const int q = hs - 1 < max_order ? hs - 1 : max_order;
  return 3 + q;
}

struct FastDiv {
  int d;
  double inv;
  __device__ __forceinline__ explicit FastDiv(int d_) : d(d_), inv(1.0 / (double)d_) {}
  __device__ __forceinline__ int div(int n) const {
    int q = (int)((double)n * inv);
    const int r = n - q * d;
    q += (r >= d) - (r < 0);
    return q;
  }
};

// Scalar-memory values a block needs before its first vector read: one
// empty asm makes them all ready at this point, so that their loads and the
// done-flag load are in flight together (one latency) instead of being
// issued one after another behind the flag's branch.
template <typename A, typename B, typename C, typename D, typename E, typename F>
__device__ __forceinline__ void scalars_ready(const A& a, const B& b, const C& c, const D& d,
                                              const E& e, const F& f) {
  asm volatile("" : : "s"(a), "s"(b), "s"(c), "s"(d), "s"(e), "s"(f));
}
template <typename A, typename B, typename C, typename D, typename E, typename F, typename G>
__device__ __forceinline__ void scalars_ready(const A& a, const B& b, const C& c, const D& d,
                                              const E& e, const F& f, const G& g) {
  asm volatile("" : : "s"(a), "s"(b), "s"(c), "s"(d), "s"(e), "s"(f), "s"(g));
}
template <typename A, typename B, typename C, typename D, typename E, typename F, typename G,
          typename H>
__device__ __forceinline__ void scalars_ready(const A& a, const B& b, const C& c, const D& d,
                                              const E& e, const F& f, const G& g, const H& h) {
  asm volatile("" : : "s"(a), "s"(b), "s"(c), "s"(d), "s"(e), "s"(f), "s"(g), "s"(h));
}

// Periodic index for any offset: halo columns of a tile wider than the grid
// can lie more than one period away.
__device__ __forceinline__ int wrap_any(int i, int n) {
  while (i < 0) i += n;
  while (i >= n) i -= n;
  return i;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// A double moved between lanes by a DPP pattern (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double lane_value(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wave, the same bits in every lane.  Within each
// row of 16 lanes, DPP exchanges (ALU latency, no LDS round trip) with the
// partner lane: adjacent pairs, then pairs of pairs, then mirrored halves of
// 8, then mirrored halves of the row -- each lane adds the same two values as
// its partner (addition is commutative), so the row's lanes agree bit for
// bit; the four row sums are then added in a fixed order.
// Sum over each row of 16 lanes (the four DPP exchanges of wave_sum): every
// lane of a row holds its row's sum, the same bits in each.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);   // row_half_mirror
  v += dpp_move<0x140>(v);   // row_mirror
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
  v = row16_sum(v);
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
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
  __syncthreads();   // sh may be reused right after
}

// Fixed-order block sum of NV values per thread, result in every thread
// (each thread adds the per-wave sums in the same order).  One barrier; the
// caller places a barrier between the last read of `sh` and its next use.
// Maximum of v over the block, in every thread (max is exact in any order).
// sh holds >= NT / 64 doubles; every thread must call it.
template <int NT = kNT>
__device__ __forceinline__ double block_max(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = sh[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) m = fmax(m, sh[w]);
  __syncthreads();
  return m;
}

template <int NV, int NT = kNT>
__device__ __forceinline__ void block_allsum(double (&v)[NV], double* sh /* >= NV*NT/64 */) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k * (NT / 64) + w] = v[k];
  }
  __syncthreads();
  // lane ww < NW of every wave reads wave ww's sum; an xor butterfly over
  // those NW lanes leaves the same total in each of them (every pairwise
  // addition is commutative, so all lanes hold identical bits), and lane 0's
  // copy goes to the whole wave
  constexpr int NW = NT / 64;
  static_assert((NW & (NW - 1)) == 0, "a power-of-two number of waves");
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double t = lane < NW ? sh[k * NW + lane] : 0.0;
#pragma unroll
    for (int off = NW / 2; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    v[k] = __shfl(t, 0, 64);
  }
}

// Coherent load / store of a value exchanged between blocks of one launch.
// Both bypass the per-XCD L2 (device-coherent access), so publishing a
// partial needs no L2 write-back or invalidation (an agent-scope fence would
// flush and invalidate the whole L2 of the block's XCD).
__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Last-block-done: every block of an instance publishes its partial (thread 0,
// st_agent), then counts itself in once that store has completed; the last
// one to arrive reads all partials with ld_agent.  Arrivals are spread over
// g = ceil(sqrt(nblocks)) (at most kSubCounters) counters -- block `local`
// uses counter local % g -- whose last arrivals count into counter 0, so no
// single address takes more than ~2 sqrt(nblocks) serialised atomics.
constexpr int kSubCounters = 64;
constexpr int kCounterStride = kSubCounters + 1;   // counters per reduction kind

__device__ __forceinline__ int arrival_groups(int nblocks) {
  int g = 1;
  while (g * g < nblocks && g < kSubCounters) ++g;
  return g;
}

__device__ __forceinline__ bool arrive_last(unsigned* counters, int nblocks, int local) {
  __shared__ int s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_s_waitcnt(0);   // the partial store is complete (acknowledged)
    const int g = arrival_groups(nblocks);
    bool last;
    if (g == 1) {
      const unsigned prev = atomicAdd(&counters[0], 1u);
      last = prev == (unsigned)(nblocks - 1);
      if (last) atomicExch(&counters[0], 0u);
    } else {
      const int sub = local % g;
      const int members = (nblocks - sub + g - 1) / g;
      const unsigned prev = atomicAdd(&counters[1 + sub], 1u);
      last = false;
      if (prev == (unsigned)(members - 1)) {
        atomicExch(&counters[1 + sub], 0u);
        const unsigned top = atomicAdd(&counters[0], 1u);
        last = top == (unsigned)(g - 1);
        if (last) atomicExch(&counters[0], 0u);
      }
    }
    s_last = last;
  }
  __syncthreads();
  return s_last != 0;
}

// Sum of n per-block partials, read by every thread of the last block in a
// fixed thread/partial mapping and combined by a fixed-order tree: the result
// (valid in thread 0) does not depend on block completion order.  Each thread
// adds its partials k = tid, tid + NT, ... in that order; they are loaded 8 at
// a time, so a thread waits once per 8 partials instead of once per partial
// (4096 tiles of a 2048 x 1024 grid are 16 partials per thread).
template <int NT = kNT>
__device__ __forceinline__ double sum_partials(const double* src, int n, double* sh) {
  constexpr int U = 8;
  double v[1] = {0.0};
  int k = threadIdx.x;
  for (; k + (U - 1) * NT < n; k += U * NT) {
    double t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) t[u] = ld_agent(&src[k + u * NT]);
#pragma unroll
    for (int u = 0; u < U; ++u) v[0] += t[u];
  }
  for (; k < n; k += NT) v[0] += ld_agent(&src[k]);
  block_sum<1, NT>(v, sh);
  return v[0];
}

// NV sums at once: out[m] = sum of src[m * stride + k], k < n, each with the
// order and tree of sum_partials (the same bits), their loads in flight
// together.  sh holds >= NV * NT / 64 doubles.
template <int NV, int NT = kNT>
__device__ __forceinline__ void sum_partials_n(const double* src, int stride, int n,
                                               double (&out)[NV], double* sh) {
  constexpr int U = NV >= 4 ? 2 : 8 / NV;
#pragma unroll
  for (int m = 0; m < NV; ++m) out[m] = 0.0;
  int k = threadIdx.x;
  for (; k + (U - 1) * NT < n; k += U * NT) {
    double t[NV][U];
#pragma unroll
    for (int m = 0; m < NV; ++m)
#pragma unroll
      for (int u = 0; u < U; ++u) t[m][u] = ld_agent(&src[m * stride + k + u * NT]);
#pragma unroll
    for (int m = 0; m < NV; ++m)
#pragma unroll
      for (int u = 0; u < U; ++u) out[m] += t[m][u];
  }
  for (; k < n; k += NT) {
    double t[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m) t[m] = ld_agent(&src[m * stride + k]);
#pragma unroll
    for (int m = 0; m < NV; ++m) out[m] += t[m];
  }
  block_sum<NV, NT>(out, sh);
}

}  // namespace cdi
