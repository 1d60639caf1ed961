// Host side of the three-dimensional C ABI (include/cdi3.h): validation,
// workspace layout and the stream-ordered launch sequence of one RK4 step
// (4 stage evaluations, 4 variable-density projections by a CG with a
// geometric multigrid V-cycle preconditioner).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/cdi3.h"
#include "cdi3_kernels.h"
#include "host_util.h"

using namespace cdi3;
using cdi_host::fail;

struct cdi3_ctx {
  Ctx3 h;                    // host copy of the device descriptor
  Ctx3* d = nullptr;         // device copy (in the workspace)
  hipStream_t stream = nullptr;
  double gamma = 0.0, gamma_factor = 0.0, rtol = 1e-10;
  int maxit = 200, guess = CDI_GUESS_PREV;
  int nu = 1;                // red-black sweep pairs before and after the coarse correction
  double t = 0.0;
  int64_t step = 0;
  int hist = 0;              // completed steps in the pressure history (<= 4)
  int last_iters = 0;
  double last_relres = 0.0;
  double* pinned = nullptr;  // host-visible scalars
  hipEvent_t e0 = nullptr, e1 = nullptr;
};

namespace {

constexpr double RK_C3[4] = {0.0, 0.5, 0.5, 1.0};
constexpr double RK_B3[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
unsigned blocks(long n) { return (unsigned)((n + kNT3 - 1) / kNT3); }

struct Shape3 {
  int nx, ny, nz, nlev;
  int lnx[kMaxLev3], lny[kMaxLev3], lnz[kMaxLev3];
  double h, dt;
};

cdi_status resolve3(const cdi3_params* in, Shape3& S) {
  if (!in) return fail(CDI_ERR_ARG, "params is NULL");
  const cdi_params& p = in->base;
  if (p.abi_version != CDI_ABI_VERSION)
    return fail(CDI_ERR_ARG, "abi_version %d != %d", p.abi_version, CDI_ABI_VERSION);
  if (p.nx < 8 || p.ny < 8 || in->nz < 8 || (p.nx & 1) || (p.ny & 1) || (in->nz & 1))
    return fail(CDI_ERR_SHAPE, "nx=%d ny=%d nz=%d: all must be even and >= 8", p.nx, p.ny, in->nz);
  if ((long long)p.nx * (p.ny + 1) * in->nz >= (1LL << 31))
    return fail(CDI_ERR_SHAPE, "grid of %d x %d x %d: more than 2^31 - 1 faces", p.nx, p.ny, in->nz);
  if (!(p.lx > 0) || !(p.ly > 0) || !(in->lz > 0)) return fail(CDI_ERR_ARG, "lx, ly, lz must be > 0");
  const double h = p.lx / p.nx;
  if (std::fabs(p.ly / p.ny - h) > 1e-12 * h || std::fabs(in->lz / in->nz - h) > 1e-12 * h)
    return fail(CDI_ERR_SHAPE, "lx/nx, ly/ny and lz/nz must be equal");
  if (!(p.eps > 0) || !(p.gamma > 0) || !(p.sigma >= 0)) return fail(CDI_ERR_ARG, "eps, gamma > 0, sigma >= 0");
  if (!(p.theta_eq > 0 && p.theta_eq < M_PI)) return fail(CDI_ERR_ARG, "theta_eq must be in (0, pi)");
  if (!(p.rho1 > 0 && p.rho2 > 0) || !(p.mu1 >= 0 && p.mu2 >= 0) || !(p.beta1 > 0 && p.beta2 > 0))
    return fail(CDI_ERR_ARG, "densities and friction > 0, viscosities >= 0");
  if (!std::isfinite(p.u_wall_bot) || !std::isfinite(p.u_wall_top) ||
      !std::isfinite(in->w_wall_bot) || !std::isfinite(in->w_wall_top))
    return fail(CDI_ERR_ARG, "wall speeds must be finite");
  if (p.slip_model < CDI_SLIP_1A || p.slip_model > CDI_SLIP_4B) return fail(CDI_ERR_ARG, "bad slip_model");
  if (p.precision != CDI_FP64) return fail(CDI_ERR_ARG, "the 3-D path computes in FP64 only");
  if (p.guess != CDI_GUESS_ZERO && p.guess != CDI_GUESS_PREV) return fail(CDI_ERR_ARG, "guess: zero or prev");
  if (p.mg_smooth < 0 || p.mg_smooth > 2) return fail(CDI_ERR_ARG, "mg_smooth: 0, 1 or 2 in 3-D");
  if (p.poisson_rtol < 0 || p.poisson_maxit < 0 || p.gamma_factor < 0 || p.dt < 0 || p.cfl < 0)
    return fail(CDI_ERR_ARG, "bad solver limits or time step");
  S.nx = p.nx; S.ny = p.ny; S.nz = in->nz; S.h = h;
  int nx = S.nx, ny = S.ny, nz = S.nz, l = 0;
  S.lnx[0] = nx; S.lny[0] = ny; S.lnz[0] = nz;
  while ((long)nx * ny * nz > kCoarseMax3 && !(nx & 1) && !(ny & 1) && !(nz & 1)) {
    if (l + 1 >= kMaxLev3) return fail(CDI_ERR_SHAPE, "too many multigrid levels");
    nx /= 2; ny /= 2; nz /= 2; ++l;
    S.lnx[l] = nx; S.lny[l] = ny; S.lnz[l] = nz;
  }
  if ((long)nx * ny * nz > kCoarseMax3)
    return fail(CDI_ERR_SHAPE, "coarsest multigrid level %d x %d x %d has more than %d cells", nx, ny,
                nz, kCoarseMax3);
  S.nlev = l + 1;
  if (p.dt > 0) {
    S.dt = p.dt;
  } else {
    const double cfl = p.cfl > 0 ? p.cfl : 0.2;
    double m = INFINITY;
    const double uw = std::max({std::fabs(p.u_wall_bot), std::fabs(p.u_wall_top),
                                std::fabs(in->w_wall_bot), std::fabs(in->w_wall_top)});
    if (uw > 0) m = std::min(m, h / uw);
    const double nu = std::max(p.mu1 / p.rho1, p.mu2 / p.rho2);
    if (nu > 0) m = std::min(m, h * h / nu);
    if (p.sigma > 0) m = std::min(m, std::sqrt((p.rho1 + p.rho2) * h * h * h / (4.0 * M_PI * p.sigma)));
    m = std::min(m, h * h / (p.gamma * p.eps));
    S.dt = cfl * m;
  }
  return CDI_OK;
}

// Carve the workspace (base == nullptr: sizes only); returns the bytes used.
size_t carve3(const Shape3& S, char* base, Ctx3* C) {
  const long N = (long)S.nx * S.ny * S.nz, NV = (long)S.nx * (S.ny + 1) * S.nz;
  const long NW = 2L * S.nz * S.nx;
  size_t off = 0;
  auto take = [&](long n) {
    double* p = base ? (double*)(base + off) : nullptr;
    off = align256(off + sizeof(double) * (size_t)n);
    return p;
  };
  Ctx3 tmp{};
  Ctx3& c = C ? *C : tmp;
  c.phi_a = take(N); c.phi_b = take(N);
  c.us = take(N); c.vs = take(NV); c.ws = take(N);
  c.acc_phi = take(N); c.acc_mx = take(N); c.acc_my = take(NV); c.acc_mz = take(N);
  c.mx = take(N); c.my = take(NV); c.mz = take(N);
  c.psi = take(N); c.nxv = take(N); c.nyv = take(N); c.nzv = take(N); c.muc = take(N);
  c.kap_p = nullptr;
  c.wall = take(5 * NW);
  c.Fx = take(N); c.Fy = take(NV); c.Fz = take(N);
  c.fmx = take(N); c.fmy = take(NV); c.fmz = take(N);
  c.txy = take(NV); c.tyz = take(NV); c.txz = take(N);
  c.uYx = take(NW); c.uYz = take(NW); c.slx = take(NW); c.slz = take(NW);
  c.b = take(N); c.x = take(N); c.r = take(N); c.z = take(N); c.d = take(N); c.q = take(N);
  c.part = take(5L * blocks(NV) + 16);
  c.scal = take(S_NSCAL);
  for (int d = 0; d < 4; ++d)
    for (int st = 0; st < 4; ++st) c.hp[d][st] = take(N);
  c.nlev = S.nlev;
  for (int l = 0; l < S.nlev; ++l) {
    Lev3& L = c.lev[l];
    L.nx = S.lnx[l]; L.ny = S.lny[l]; L.nz = S.lnz[l];
    const long n = (long)L.nx * L.ny * L.nz, nv = (long)L.nx * (L.ny + 1) * L.nz;
    L.ax = take(n); L.ay = take(nv); L.az = take(n);
    if (l == 0) {
      L.r = c.r;
      L.x = c.z;
    } else {
      L.r = take(n);
      L.x = take(n);
    }
  }
  off = align256(off + sizeof(Ctx3));
  return off;
}

// One V(nu,nu) cycle: z = M r on level 0 (the CG residual and correction);
// nu red-black sweep pairs on the way down (the first red half-sweep from
// zero) and nu black-red pairs on the way up.
void vcycle(cdi3_ctx* c) {
  const Ctx3& H = c->h;
  const int nl = H.nlev;
  auto cells = [&](int l) { return (long)H.lev[l].nx * H.lev[l].ny * H.lev[l].nz; };
  for (int l = 0; l < nl - 1; ++l) {
    for (int s = 0; s < c->nu; ++s) {
      k3_mg_smooth<<<blocks(cells(l) / 2), kNT3, 0, c->stream>>>(c->d, l, 0, s == 0 ? 1 : 0);
      k3_mg_smooth<<<blocks(cells(l) / 2), kNT3, 0, c->stream>>>(c->d, l, 1, 0);
    }
    k3_mg_restrict<<<blocks(cells(l + 1)), kNT3, 0, c->stream>>>(c->d, l);
  }
  k3_mg_coarse<<<1, kCoarseMax3, 0, c->stream>>>(c->d, nl - 1);
  for (int l = nl - 2; l >= 0; --l) {
    k3_mg_prolong<<<blocks(cells(l)), kNT3, 0, c->stream>>>(c->d, l);
    for (int s = 0; s < c->nu; ++s) {
      k3_mg_smooth<<<blocks(cells(l) / 2), kNT3, 0, c->stream>>>(c->d, l, 1, 0);
      k3_mg_smooth<<<blocks(cells(l) / 2), kNT3, 0, c->stream>>>(c->d, l, 0, 0);
    }
  }
}

cdi_status read_relres(cdi3_ctx* c, double& relres) {
  HIPCHK(hipMemcpyAsync(c->pinned, c->h.scal + S_RELRES, sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  relres = c->pinned[0];
  return CDI_OK;
}

// Pressure solve of K x = -(b - mean b) into h.x for RK stage `stage`.  The
// initial guess (CDI_GUESS_PREV): the extrapolation in time of the stage's
// pressure through the last min(hist, 4) steps (order hist - 1, at most
// cubic), the state's pressure before the first step; CDI_GUESS_ZERO: 0.
cdi_status solve3(cdi3_ctx* c, int stage, int& iters, double& relres) {
  const Ctx3& H = c->h;
  const long N = (long)H.nx * H.ny * H.nz;
  const unsigned nb = blocks(N);
  for (int l = 0; l + 1 < H.nlev; ++l) {
    const Lev3& G = H.lev[l + 1];
    k3_mg_coef<<<blocks((long)G.nx * (G.ny + 1) * G.nz), kNT3, 0, c->stream>>>(c->d, l);
  }
  const bool prev = c->guess == CDI_GUESS_PREV;
  if (prev) {
    Guess3 g{};
    g.stage = stage;
    g.q = std::min(c->hist, 4) - 1;
    for (int d = 0; d <= g.q; ++d) g.slot[d] = (int)((c->step - 1 - d) & 3);
    k3_guess<<<nb, kNT3, 0, c->stream>>>(c->d, g);
  }
  k3_pcg_init<<<nb, kNT3, 0, c->stream>>>(c->d, prev ? 1 : 0);
  k3_finalize<<<1, 1024, 0, c->stream>>>(c->d, (int)nb, 1);
  iters = 0;
  cdi_status s = read_relres(c, relres);
  if (s != CDI_OK) return s;
  if (!std::isfinite(relres)) return fail(CDI_ERR_NONFINITE, "3-D pressure solve: non-finite residual");
  if (relres > c->rtol) {
    vcycle(c);
    k3_dot_rz<<<nb, kNT3, 0, c->stream>>>(c->d);
    k3_finalize<<<1, 1024, 0, c->stream>>>(c->d, (int)nb, 4);
    k3_dir<<<nb, kNT3, 0, c->stream>>>(c->d, 1);
    while (iters < c->maxit) {
      k3_spmv<<<nb, kNT3, 0, c->stream>>>(c->d);
      k3_finalize<<<1, 1024, 0, c->stream>>>(c->d, (int)nb, 2);
      k3_update<<<nb, kNT3, 0, c->stream>>>(c->d);
      k3_finalize<<<1, 1024, 0, c->stream>>>(c->d, (int)nb, 3);
      ++iters;
      s = read_relres(c, relres);
      if (s != CDI_OK) return s;
      if (!std::isfinite(relres)) return fail(CDI_ERR_NONFINITE, "3-D pressure solve: non-finite residual");
      if (relres <= c->rtol) break;
      vcycle(c);
      k3_dot_rz<<<nb, kNT3, 0, c->stream>>>(c->d);
      k3_finalize<<<1, 1024, 0, c->stream>>>(c->d, (int)nb, 4);
      k3_dir<<<nb, kNT3, 0, c->stream>>>(c->d, 0);
    }
  }
  k3_sum_x<<<nb, kNT3, 0, c->stream>>>(c->d);
  k3_finalize<<<1, 1024, 0, c->stream>>>(c->d, (int)nb, 5);
  HIPCHK(hipGetLastError());
  return CDI_OK;
}

void set_gamma(cdi3_ctx* c) {
  const long N = (long)c->h.nx * c->h.ny * c->h.nz;
  k3_absmax<<<blocks(N), kNT3, 0, c->stream>>>(c->d);
  k3_gamma<<<1, 1024, 0, c->stream>>>(c->d, (int)blocks(N), c->gamma, c->gamma_factor);
}

// The stage operator: phase preparation, wall quantities, fluxes, edge
// stresses and momentum / RK4 update (kst < 0: evaluation only).
void stage3(cdi3_ctx* c, int kst, int src, int dst, double c_next, double b_k, int write_wall) {
  const Ctx3& H = c->h;
  const long N = (long)H.nx * H.ny * H.nz, NV = (long)H.nx * (H.ny + 1) * H.nz;
  k3_psi<<<blocks(N), kNT3, 0, c->stream>>>(c->d, src);
  k3_prep<<<blocks(N), kNT3, 0, c->stream>>>(c->d, src);
  k3_wall<<<blocks(2L * H.nz * H.nx), kNT3, 0, c->stream>>>(c->d, src);
  k3_flux<<<blocks(N), kNT3, 0, c->stream>>>(c->d, src, kst);
  k3_edges<<<blocks(NV), kNT3, 0, c->stream>>>(c->d, src, kst, write_wall);
  k3_mom<<<blocks(N), kNT3, 0, c->stream>>>(c->d, kst, src, dst, c_next, b_k);
}

cdi_status step3(cdi3_ctx* c) {
  const Ctx3& H = c->h;
  const long N = (long)H.nx * H.ny * H.nz;
  if (c->gamma_factor > 0) set_gamma(c);
  for (int k = 0; k < 4; ++k) {
    const int src = k == 0 ? 0 : (k == 2 ? 2 : 1);
    const int dst = (k == 0 || k == 2) ? 1 : 2;
    const double tfac = k < 3 ? RK_C3[k + 1] : 1.0;
    stage3(c, k, src, dst, tfac, RK_B3[k], k == 3);
    k3_rhs<<<blocks(N), kNT3, 0, c->stream>>>(c->d, dst, tfac);
    k3_finalize<<<1, 1024, 0, c->stream>>>(c->d, (int)blocks(N), 0);
    int it = 0;
    double rel = 0.0;
    cdi_status s = solve3(c, k, it, rel);
    if (s != CDI_OK) return s;
    c->last_iters = it;
    c->last_relres = rel;
    k3_project<<<blocks(N), kNT3, 0, c->stream>>>(c->d, dst, tfac, k == 3, (int)(c->step & 3), k);
    HIPCHK(hipGetLastError());
    if (rel > c->rtol) return fail(CDI_ERR_NOCONV, "3-D pressure solve: relres %.3e after %d iterations", rel, it);
  }
  c->t += H.dt;
  c->step += 1;
  c->hist = std::min(c->hist + 1, 4);
  return CDI_OK;
}

}  // namespace

extern "C" {

cdi_status cdi3_workspace_bytes(const cdi3_params* params, size_t* bytes) {
  Shape3 S;
  cdi_status s = resolve3(params, S);
  if (s != CDI_OK) return s;
  if (!bytes) return fail(CDI_ERR_ARG, "bytes is NULL");
  *bytes = carve3(S, nullptr, nullptr);
  return CDI_OK;
}

cdi_status cdi3_init(const cdi3_params* params, const cdi3_fields* fields, void* workspace,
                     size_t workspace_bytes, void* hip_stream, cdi3_ctx** out) {
  if (!out) return fail(CDI_ERR_ARG, "out is NULL");
  *out = nullptr;
  Shape3 S;
  cdi_status s = resolve3(params, S);
  if (s != CDI_OK) return s;
  if (!fields || !fields->phi || !fields->u || !fields->v || !fields->w || !fields->p)
    return fail(CDI_ERR_ARG, "fields (phi, u, v, w, p) must be non-NULL");
  const size_t need = carve3(S, nullptr, nullptr);
  if (!workspace || workspace_bytes < need)
    return fail(CDI_ERR_ARG, "workspace of %zu bytes, %zu needed", workspace_bytes, need);
  if ((uintptr_t)workspace & 255) return fail(CDI_ERR_ARG, "workspace must be 256-byte aligned");
  cdi3_ctx* c = new cdi3_ctx();
  const cdi_params& p = params->base;
  Ctx3& H = c->h;
  carve3(S, (char*)workspace, &H);
  H.nx = S.nx; H.ny = S.ny; H.nz = S.nz; H.slip_model = p.slip_model;
  H.h = S.h; H.inv_h = 1.0 / S.h; H.eps = p.eps; H.inv_eps = 1.0 / p.eps; H.sigma = p.sigma;
  H.cos_eq = std::cos(p.theta_eq);
  H.rho1 = p.rho1; H.rho2 = p.rho2; H.mu1 = p.mu1; H.mu2 = p.mu2; H.beta1 = p.beta1; H.beta2 = p.beta2;
  H.uwb = p.u_wall_bot; H.uwt = p.u_wall_top; H.wwb = params->w_wall_bot; H.wwt = params->w_wall_top;
  H.dt = S.dt;
  H.phi = fields->phi; H.u = fields->u; H.v = fields->v; H.w = fields->w; H.p = fields->p;
  c->d = (Ctx3*)((char*)workspace + need - align256(sizeof(Ctx3)));
  c->stream = (hipStream_t)hip_stream;
  c->gamma = p.gamma;
  c->gamma_factor = p.gamma_factor;
  c->rtol = p.poisson_rtol > 0 ? p.poisson_rtol : 1e-10;
  c->maxit = p.poisson_maxit > 0 ? p.poisson_maxit : 200;
  c->nu = p.mg_smooth > 0 ? p.mg_smooth : 2;   // V(2,2) unless asked otherwise
  c->guess = p.guess;
  auto bail = [&](hipError_t e, const char* what) {
    if (c->pinned) (void)hipHostFree(c->pinned);
    delete c;
    return fail(CDI_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
  };
  hipError_t e = hipHostMalloc((void**)&c->pinned, 8 * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) return bail(e, "hipHostMalloc");
  // zero the workspace once (wall rows of the v-layout arrays stay 0)
  if ((e = hipMemsetAsync(workspace, 0, need, c->stream)) != hipSuccess) return bail(e, "clear workspace");
  if ((e = hipMemcpyAsync(c->d, &H, sizeof(Ctx3), hipMemcpyHostToDevice, c->stream)) != hipSuccess)
    return bail(e, "copy descriptor");
  std::vector<double> sc(S_NSCAL, 0.0);
  sc[S_GAMMA] = p.gamma;
  if ((e = hipMemcpyAsync(H.scal, sc.data(), sizeof(double) * S_NSCAL, hipMemcpyHostToDevice,
                          c->stream)) != hipSuccess)
    return bail(e, "copy scalars");
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return bail(e, "init sync");
  if ((e = hipEventCreate(&c->e0)) != hipSuccess) return bail(e, "event");
  if ((e = hipEventCreate(&c->e1)) != hipSuccess) return bail(e, "event");
  *out = c;
  return CDI_OK;
}

cdi_status cdi3_step(cdi3_ctx* c, int32_t nsteps) {
  if (!c) return fail(CDI_ERR_ARG, "ctx is NULL");
  if (nsteps < 0) return fail(CDI_ERR_ARG, "nsteps < 0");
  for (int s = 0; s < nsteps; ++s) {
    cdi_status st = step3(c);
    if (st != CDI_OK) return st;
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  return CDI_OK;
}

cdi_status cdi3_eval_rhs(cdi3_ctx* c, double* l_phi, double* l_mx, double* l_my, double* l_mz,
                         double* uY_x, double* uY_z) {
  if (!c) return fail(CDI_ERR_ARG, "ctx is NULL");
  if (!l_phi || !l_mx || !l_my || !l_mz) return fail(CDI_ERR_ARG, "output pointer is NULL");
  const Ctx3& H = c->h;
  const size_t N = (size_t)H.nx * H.ny * H.nz, NV = (size_t)H.nx * (H.ny + 1) * H.nz;
  const size_t NW = 2 * (size_t)H.nz * H.nx;
  set_gamma(c);
  stage3(c, -1, 0, 0, 0.0, 0.0, 1);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(l_phi, H.acc_phi, N * 8, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(l_mx, H.acc_mx, N * 8, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(l_my, H.acc_my, NV * 8, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(l_mz, H.acc_mz, N * 8, hipMemcpyDeviceToDevice, c->stream));
  if (uY_x) HIPCHK(hipMemcpyAsync(uY_x, H.uYx, NW * 8, hipMemcpyDeviceToDevice, c->stream));
  if (uY_z) HIPCHK(hipMemcpyAsync(uY_z, H.uYz, NW * 8, hipMemcpyDeviceToDevice, c->stream));
  return CDI_OK;
}

cdi_status cdi3_kappa_p(cdi3_ctx* c, double* kappa_p) {
  if (!c || !kappa_p) return fail(CDI_ERR_ARG, "NULL argument");
  const long N = (long)c->h.nx * c->h.ny * c->h.nz;
  k3_psi<<<blocks(N), kNT3, 0, c->stream>>>(c->d, 0);
  k3_kappa_p<<<blocks(N), kNT3, 0, c->stream>>>(c->d, 0, kappa_p);
  HIPCHK(hipGetLastError());
  return CDI_OK;
}

cdi_status cdi3_diagnostics(cdi3_ctx* c, cdi3_diag* out) {
  if (!c || !out) return fail(CDI_ERR_ARG, "NULL argument");
  const Ctx3& H = c->h;
  const long N = (long)H.nx * H.ny * H.nz;
  const size_t NW = 2 * (size_t)H.nz * H.nx;
  set_gamma(c);
  stage3(c, -1, 0, 0, 0.0, 0.0, 1);   // fills the slip arrays of the current state
  const unsigned nb = blocks(N);
  // partials after the stage's scratch: the diag kernel writes 5 x nb values
  double* dp = H.Fx;
  k3_diag<<<nb, kNT3, 0, c->stream>>>(c->d, dp);
  HIPCHK(hipGetLastError());
  std::vector<double> part(5 * (size_t)nb), w(4 * NW);
  HIPCHK(hipMemcpyAsync(part.data(), dp, part.size() * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(w.data(), H.slx, NW * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(w.data() + NW, H.slz, NW * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(w.data() + 2 * NW, H.uYx, NW * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(w.data() + 3 * NW, H.uYz, NW * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  double mass = 0, ke = 0, pmax = -INFINITY, pminn = -INFINITY, dmax = 0;
  for (unsigned b = 0; b < nb; ++b) {
    mass += part[b];
    ke += part[nb + b];
    pmax = std::max(pmax, part[2 * nb + b]);
    pminn = std::max(pminn, part[3 * nb + b]);
    dmax = std::max(dmax, part[4 * nb + b]);
  }
  const double h3 = H.h * H.h * H.h;
  *out = cdi3_diag{};
  out->t = c->t;
  out->step = c->step;
  out->mass = mass * h3;
  out->phi_min = -pminn;
  out->phi_max = pmax;
  out->max_div = dmax;
  out->ke = 0.5 * ke * h3;
  const size_t half = NW / 2;
  for (int wall = 0; wall < 2; ++wall) {
    double ms = 0, my = 0;
    for (size_t e = wall * half; e < (wall + 1) * half; ++e) {
      ms = std::max({ms, std::fabs(w[e]), std::fabs(w[NW + e])});
      my = std::max({my, std::fabs(w[2 * NW + e]), std::fabs(w[3 * NW + e])});
    }
    out->max_slip[wall] = ms;
    out->max_uY[wall] = my;
  }
  out->last_iters = c->last_iters;
  out->last_relres = c->last_relres;
  return CDI_OK;
}

cdi_status cdi3_time_stage(cdi3_ctx* c, int32_t reps, double* ms) {
  if (!c || !ms || reps < 1) return fail(CDI_ERR_ARG, "bad argument");
  set_gamma(c);
  stage3(c, -1, 0, 0, 0.0, 0.0, 0);   // warm
  HIPCHK(hipEventRecord(c->e0, c->stream));
  for (int r = 0; r < reps; ++r) stage3(c, -1, 0, 0, 0.0, 0.0, 0);
  HIPCHK(hipEventRecord(c->e1, c->stream));
  HIPCHK(hipEventSynchronize(c->e1));
  float t = 0.f;
  HIPCHK(hipEventElapsedTime(&t, c->e0, c->e1));
  *ms = (double)t / reps;
  return CDI_OK;
}

void cdi3_destroy(cdi3_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->e0) (void)hipEventDestroy(c->e0);
  if (c->e1) (void)hipEventDestroy(c->e1);
  if (c->pinned) (void)hipHostFree(c->pinned);
  delete c;
}

}  // extern "C"
