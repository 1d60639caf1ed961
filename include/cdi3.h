/* Three-dimensional CDI + GNBC time step on one MI355X (gfx950).
 *
 * The paper states its wall model for a general wall -- inward normal
 * n_wall, tangential direction tau_wall, and the interface curvature kappa_p
 * in the plane containing n_phi and n_wall in the curvature correction
 * 1 + kappa_p psi of Models 3A..4B (Sec. 2, slip BC; Sec. 3.1.2) -- and
 * computes in two dimensions (Sec. 4).  This entry set carries the same
 * discretisation to three: x and z periodic, walls at y = 0 and y = ly, the
 * Young slip a vector in the wall plane, and
 *     kappa_p = kappa + t_q . (grad grad psi) t_q,
 * t_q = n_phi x n_wall / |n_phi x n_wall| the direction along the contact
 * line, i.e. the energy-based curvature (eq. curvature) with the normal
 * curvature along the contact line removed; where psi has no tangential
 * gradient (no contact line) kappa_p = kappa.
 *
 * Layouts (device, FP64, x fastest; caller-owned):
 *   phi, p, u, w   nz * ny * nx       element (k, j, i) at (k ny + j) nx + i;
 *                                     u on the x-face i, w on the z-face k
 *   v              nz * (ny+1) * nx   element (k, j, i) at (k (ny+1) + j) nx + i,
 *                                     the y-face j; rows 0 and ny are walls (v = 0)
 * Wall arrays (slip outputs): 2 walls x nz x nx, wall 0 = y = 0, element
 * (wall, k, i) at (wall nz + k) nx + i; the x-slip lives on the xy-edge
 * (i h, wall, (k + 1/2) h), the z-slip on the yz-edge ((i + 1/2) h, wall, k h).
 *
 * Every call is asynchronous on the context's stream unless stated; errors
 * are reported as in cdi.h (cdi_last_error for the message).
 */
#ifndef CDI3_H
#define CDI3_H

#include "cdi.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Problem statement: `base` as in cdi.h (nx, ny, lx, ly, the physical
 * parameters, dt / cfl, slip_model, poisson_rtol / poisson_maxit, guess =
 * CDI_GUESS_ZERO or CDI_GUESS_PREV, gamma_factor), plus the z extent and the
 * z components of the wall speeds.  base.precision must be CDI_FP64 and
 * base.mg_smooth 1 (V(1,1)) or 2 (V(2,2); also 0).  nx, ny, nz even and
 * >= 8; lz / nz must equal the x and y spacing; nx (ny+1) nz < 2^31; the
 * multigrid hierarchy (halving all
 * three directions while all stay even and the level has more than 1024
 * cells) must end on at most 1024 cells (else CDI_ERR_SHAPE). */
typedef struct {
  cdi_params base;
  int32_t nz;
  int32_t pad;
  double lz;
  double w_wall_bot;   /* tangential +z speed of the wall y = 0  */
  double w_wall_top;   /* tangential +z speed of the wall y = ly */
} cdi3_params;

typedef struct {
  double* phi;
  double* u;
  double* v;
  double* w;
  double* p;
} cdi3_fields;

typedef struct cdi3_ctx cdi3_ctx;

typedef struct {
  double t;
  int64_t step;
  double mass;          /* sum(phi) h^3                                */
  double phi_min, phi_max;
  double max_div;       /* max |div u| over cells                      */
  double max_slip[2];   /* max |u_wall - U_wall| over both components, per wall */
  double max_uY[2];     /* max |u^Y| over both components, per wall    */
  double ke;            /* 1/2 sum rho_f |u|^2 h^3                      */
  int32_t last_iters;   /* CG iterations of the last pressure solve    */
  int32_t pad;
  double last_relres;
} cdi3_diag;

/* Device bytes of the workspace of one context (256-byte aligned). */
cdi_status cdi3_workspace_bytes(const cdi3_params* params, size_t* bytes);

/* Validate the parameters, lay out the workspace, and take the fields.
 * workspace: device memory of cdi3_workspace_bytes bytes, 256-byte aligned;
 * fields: device pointers (layouts above), the initial state; hip_stream: a
 * hipStream_t or NULL.  Returns CDI_ERR_ARG / CDI_ERR_SHAPE on invalid input
 * before any device work. */
cdi_status cdi3_init(const cdi3_params* params, const cdi3_fields* fields, void* workspace,
                     size_t workspace_bytes, void* hip_stream, cdi3_ctx** out);

/* Advance by nsteps RK4 steps (4 stage evaluations and 4 projections each;
 * Sec. 4).  Each pressure solve is a CG with a geometric multigrid V-cycle
 * preconditioner (base.mg_smooth red-black pairs each way), started
 * (CDI_GUESS_PREV) from the extrapolation in time of the same RK stage's
 * pressure through the last up to four steps (order up to cubic; the
 * state's pressure before the first step) or from zero (CDI_GUESS_ZERO);
 * CDI_ERR_NOCONV if a solve stops at poisson_maxit,
 * CDI_ERR_NONFINITE on a NaN / Inf residual.  Synchronises the stream (the
 * host reads each solve's residual). */
cdi_status cdi3_step(cdi3_ctx* ctx, int32_t nsteps);

/* The stage operator on the current state: L_phi, L_mx (nz ny nx), L_my
 * (nz (ny+1) nx, wall rows 0), L_mz (nz ny nx); uY_x, uY_z (wall arrays,
 * may be NULL): the Young slip.  All device pointers. */
cdi_status cdi3_eval_rhs(cdi3_ctx* ctx, double* l_phi, double* l_mx, double* l_my, double* l_mz,
                         double* uY_x, double* uY_z);

/* kappa_p at every cell of the current phase field (device, nz ny nx). */
cdi_status cdi3_kappa_p(cdi3_ctx* ctx, double* kappa_p);

/* Diagnostics of the current state (synchronises the stream). */
cdi_status cdi3_diagnostics(cdi3_ctx* ctx, cdi3_diag* out);

/* Device time (ms) of one stage-operator evaluation (the phase preparation,
 * wall quantities, fluxes, edge stresses and momentum kernels), averaged over
 * reps launches of each on the current state (synchronises). */
cdi_status cdi3_time_stage(cdi3_ctx* ctx, int32_t reps, double* ms);

void cdi3_destroy(cdi3_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif
