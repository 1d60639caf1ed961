/*
 * cdi.h -- C ABI of the MI355X (gfx950) CDI + GNBC time step.
 *
 * One time step of the conservative diffuse-interface two-phase flow solver
 * with the mass-conserving GNBC contact-line treatment of Brown, Mirjalili,
 * Khanwale & Mani (arXiv:2412.16843):
 *   - CDI phase-field equation with the regularisation (sharpening) flux
 *     R = gamma [eps grad(phi) - phi(1-phi) n]            (Sec. 2, eq. CDI)
 *   - no-flux phase-field walls and no-penetration walls   (Sec. 2, no-flux BC)
 *   - mixture momentum with the consistent mass flux rho u - S,
 *     S = (rho1 - rho2) R, variable viscosity               (Sec. 2, eq. NS_momentum)
 *   - energy-based surface tension F = mu_c grad(phi) with the psi-form
 *     chemical potential                                    (Sec. 2, eqs. EB surface
 *                                                            tension, chemical potential)
 *   - GNBC slip u_slip = (mu/beta) du/dn + u^Y, Model 4A u^Y (Sec. 2 eq. u_slip_Y,
 *                                                            Sec. 3.1.2 eq. Model 4A)
 *   - one-sided wall-normal stencils and linear extrapolation to the wall,
 *     no phase-field ghost values                           (Sec. 4)
 *   - RK4 with a variable-density pressure projection after every stage,
 *     pressure by multigrid-preconditioned flexible CG      (Sec. 4; the paper
 *                                                            defers the coupling
 *                                                            to its references)
 *
 * Grid: uniform staggered, nx x ny cells of size h = lx/nx = ly/ny, x periodic,
 * walls at y = 0 and y = ly.  All arrays are row-major with x fastest:
 *   phi, p : ny * nx      cell centres ((i+1/2)h, (j+1/2)h)
 *   u      : ny * nx      x-faces (i h, (j+1/2)h)
 *   v      : (ny+1) * nx  y-faces ((i+1/2)h, j h); rows 0 and ny are the walls
 *                         and must hold 0 (no penetration)
 * phi = 1 is fluid 1.  The pressure p is the solution of
 *   sum_faces (p_nb - p) / (rho_face h^2) = div(u*) / tau,  mean(p) = 0.
 *
 * Memory ownership: every device pointer (fields, workspace, RHS buffers) is
 * owned by the caller and only borrowed for the lifetime of the context; the
 * library allocates no device memory.  The context itself (host memory) is
 * created by cdi_init / cdi_init_batch and freed by cdi_destroy.  All work is
 * enqueued on the caller's HIP stream.
 *
 * Errors: every function returns a cdi_status (0 = success, < 0 = error) and
 * never aborts; cdi_last_error() returns a thread-local message describing
 * the last error.  Arguments are validated before any device work.
 */
#ifndef CDI_H
#define CDI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CDI_ABI_VERSION 3

typedef enum {
  CDI_OK = 0,
  CDI_ERR_ARG = -1,       /* invalid parameter value or null pointer            */
  CDI_ERR_SHAPE = -2,     /* grid not supported (see cdi_init)                  */
  CDI_ERR_DEVICE = -3,    /* a HIP runtime call failed                          */
  CDI_ERR_NOCONV = -4,    /* pressure solve hit poisson_maxit before poisson_rtol */
  CDI_ERR_NONFINITE = -5, /* a NaN / Inf appeared in the state                  */
  CDI_ERR_STATE = -6      /* call not valid in the context's current state      */
} cdi_status;

enum { CDI_SLIP_1A = 0, CDI_SLIP_1B, CDI_SLIP_2A, CDI_SLIP_2B,
       CDI_SLIP_3A, CDI_SLIP_3B, CDI_SLIP_4A, CDI_SLIP_4B };
enum { CDI_FP64 = 0, CDI_MIXED = 1 };
enum { CDI_GUESS_ZERO = 0, CDI_GUESS_PREV = 1, CDI_GUESS_LEARNED = 2 };
enum { CDI_LAUNCH_TILED = 0, CDI_LAUNCH_PERSISTENT = 1, CDI_LAUNCH_GRAPH = 2 };

/* Problem statement (Sec. 2 and Sec. 4 of the paper).  Any field left 0 where
 * a default is stated takes that default. */
typedef struct {
  int32_t abi_version;   /* must be CDI_ABI_VERSION                                  */
  int32_t nx, ny;        /* cells; nx >= 8, ny >= 8, both even, nx (ny+1) < 2^31   */
  double lx, ly;         /* domain; lx/nx must equal ly/ny (uniform h)                */
  double eps;            /* interface thickness eps > 0               (eq. CDI)       */
  double gamma;          /* regularisation velocity gamma > 0         (eq. CDI)       */
  double sigma;          /* surface tension sigma >= 0                (eq. chem. pot.)*/
  double theta_eq;       /* equilibrium contact angle in (0, pi), radians, measured
                            inside fluid 1                              (eq. u_slip_Y) */
  double rho1, rho2;     /* densities of fluid 1 (phi = 1) and fluid 2, > 0          */
  double mu1, mu2;       /* viscosities, >= 0                                         */
  double beta1, beta2;   /* wall friction, > 0; beta = (beta1-beta2) phi + beta2      */
  double u_wall_bot;     /* tangential (+x) speed of the wall y = 0                   */
  double u_wall_top;     /* tangential (+x) speed of the wall y = ly                  */
  double dt;             /* > 0: fixed step; 0: cfl * min(h/|U|, h^2/nu, capillary,
                            h^2/(gamma eps)) fixed at init                            */
  double cfl;            /* used when dt == 0; 0 -> 0.2                               */
  int32_t slip_model;    /* CDI_SLIP_4A (paper's choice); 1A..4B also accepted        */
  int32_t precision;     /* CDI_FP64 or CDI_MIXED (FP32 stencils and V-cycle, FP64
                            phase field, flux accumulation, CG vectors, residual)     */
  int32_t guess;         /* initial guess of each pressure solve                      */
  double poisson_rtol;   /* stop when ||f - K x||_2 <= rtol ||f||_2; 0 -> 1e-10       */
  int32_t poisson_maxit; /* 0 -> 200                                                  */
  int32_t mg_smooth;     /* red-black Gauss-Seidel sweep pairs before and after the
                            coarse correction on the tiled levels (the levels of the
                            one-block coarse cycle take one pair more; the persistent
                            launch takes mg_smooth on every level): 1 or 2; 0 -> 1;
                            larger values return CDI_ERR_ARG; equal across a batch   */
  double gamma_factor;   /* > 0: the regularisation velocity of each step is
                            min(gamma, gamma_factor * max |u|, |v| over the faces of
                            the state the step starts from), the paper's rule
                            gamma = 2.5 |u|_max (Sec. 5); gamma is then its upper
                            bound, the value the time step of dt == 0 is sized for.
                            0: gamma fixed.  < 0 returns CDI_ERR_ARG.  Not available
                            with the persistent launch (CDI_ERR_ARG there).          */
} cdi_params;

/* Device pointers of one instance's state, layouts as above (caller-owned,
 * FP64).  On cdi_init phi holds the initial phase field, u and v the initial
 * velocity (walls of v = 0), p the initial pressure guess (may be zero). */
typedef struct {
  double* phi;
  double* u;
  double* v;
  double* p;
} cdi_fields;

typedef struct cdi_ctx cdi_ctx;

typedef struct {
  int32_t iterations;  /* flexible-CG iterations of the solve                    */
  int32_t converged;   /* 1 if relres <= poisson_rtol                            */
  int32_t guess_used;  /* CDI_GUESS_* actually used                              */
  int32_t pad;
  double relres;       /* ||f - K x|| / ||f|| (recursive residual)               */
  double bnorm;        /* ||f||                                                  */
  double ms;           /* device time of the solve, milliseconds                 */
} cdi_solve_info;

typedef struct {
  double t;            /* simulated time                                         */
  int64_t step;        /* steps taken                                            */
  double mass;         /* sum(phi) h^2 (FP64)                                    */
  double mass0;        /* mass at init                                           */
  double phi_min, phi_max;
  double max_div;      /* max |div u| over cells                                 */
  double max_uslip[2]; /* max |u_wall - U_wall| per wall (0 bottom, 1 top)       */
  double max_uY[2];    /* max |u^Y| per wall                                     */
  double ke;           /* kinetic energy 1/2 sum rho_f |u|^2 h^2                 */
  int32_t last_iters;  /* iterations of the last pressure solve                  */
  int32_t nonfinite;   /* 1 if a NaN / Inf was found                             */
  double last_relres;
  /* Contact lines (Sec. 5.1 measures): where the wall phase field,
   * extrapolated per column from the first two cell rows (Sec. 4), crosses
   * 1/2, by linear interpolation between column centres (x periodic). */
  int32_t n_contact[2];  /* crossings per wall (0 bottom, 1 top)                 */
  double contact_x[4];   /* the first two crossings of each wall in column order:
                            bottom x0, x1, then top x0, x1; 0 where absent      */
  double wetted_len[2];  /* |x1 - x0| of a wall with exactly two crossings, else 0 */
  double theta_est[2];   /* contact angle (radians) of the circular cap with chord
                            wetted_len and area `mass` (root of
                            (L / (2 sin t))^2 (t - sin t cos t) = mass), meaningful
                            for a single drop on that wall; 0 when wetted_len is 0 */
} cdi_diag;

/* Bytes of caller-provided device workspace for `n` instances described by
 * params[0..n-1] (same layout as cdi_init_batch).  Returns 0 on invalid
 * parameters (cdi_last_error() tells why). */
size_t cdi_workspace_bytes(const cdi_params* params, int32_t n);

/* Time step that cdi_init would fix for these parameters (dt, or the CFL rule
 * when dt == 0).  Host-only; no device work.  Returns a negative value on
 * invalid parameters. */
double cdi_default_dt(const cdi_params* params);

/* Create a context for one instance.  `workspace` must point to at least
 * cdi_workspace_bytes(params, 1) bytes of device memory, 256-byte aligned.
 * `hip_stream` is a hipStream_t (NULL = default stream).  The initial state
 * in `fields` is read when cdi_step runs.  Supported grids: nx, ny even,
 * nx, ny >= 8, and the multigrid hierarchy (halving both directions while
 * both stay even and the level has more than 64 cells) must end on a grid of
 * at most 1024 cells. */
cdi_status cdi_init(const cdi_params* params, const cdi_fields* fields, void* workspace,
                    size_t workspace_bytes, void* hip_stream, cdi_ctx** out);

/* Same for an ensemble of n independent instances (uneven grids allowed);
 * every kernel of a step covers all instances in one launch, and each
 * instance's pressure solve stops on its own convergence test. */
cdi_status cdi_init_batch(const cdi_params* params, int32_t n, const cdi_fields* fields,
                          void* workspace, size_t workspace_bytes, void* hip_stream,
                          cdi_ctx** out);

/* Advance every instance by nsteps RK4 steps (4 stage evaluations and 4
 * projections each).  Returns CDI_ERR_NOCONV if a pressure solve did not reach
 * poisson_rtol within poisson_maxit (the fields then hold the best iterate);
 * CDI_ERR_NONFINITE if a non-finite value was detected: a solve whose
 * right-hand side or residual norm is NaN or Inf stops at once and the step
 * returns after that stage (the fields are then not a valid state). */
cdi_status cdi_step(cdi_ctx* ctx, int32_t nsteps);

/* Advance n distinct contexts by nsteps each at the same time: one host
 * thread per context runs its cdi_step.  Contexts created on different
 * streams overlap on the GPU, so one part of a batch fills the compute
 * units while another waits on its latency-bound phases (the one-block
 * coarse cycle, the host's convergence checks) -- an ensemble split into two
 * contexts runs faster than one context holding it all.  Returns CDI_OK, the
 * first hard error of any context (cdi_last_error gives its message), or
 * CDI_ERR_NOCONV if a context reported it.  Not safe to call on a context
 * that another thread uses at the same time. */
cdi_status cdi_step_concurrent(cdi_ctx* const* ctxs, int32_t n, int32_t nsteps);

/* Standalone pressure solve of instance 0 with the density of its current
 * phase field: sum_faces (p_nb - p)/(rho_f h^2) = b - mean(b).  b: device,
 * ny*nx (NULL = the right-hand side of the last projection); p: device,
 * ny*nx, in: initial guess when params.guess == CDI_GUESS_PREV, out: the
 * mean-free solution.  info may be NULL.  Returns CDI_ERR_NOCONV when
 * poisson_maxit iterations did not reach poisson_rtol (p holds the last
 * iterate, info the iterations and residual), CDI_ERR_NONFINITE when b (or
 * the residual) is not finite; a right-hand side whose mean-free part is
 * zero gives p = 0 without an iteration. */
cdi_status cdi_solve_pressure(cdi_ctx* ctx, const double* b, double* p, cdi_solve_info* info);

/* CG iterations each instance has run since the context was set up
 * (per_instance: host array of n_instances entries), every launch form,
 * autotuning trials and redone graph steps included: with the algorithmic
 * bytes of an iteration, the memory traffic of a run's pressure solves.
 * Synchronises the stream. */
cdi_status cdi_cg_iterations(cdi_ctx* ctx, int64_t* per_instance);

/* Diagnostics of instance `idx` for its current state, computed on the device
 * (FP64 reductions; contact-line positions, wetted length and cap angle of
 * Sec. 5.1): mass and phase-field bounds (Sec. 2, conservation and
 * boundedness), slip maxima (Sec. 2 slip BC), contact lines (Sec. 5.1).
 * Synchronises the stream.  Returns CDI_ERR_NONFINITE (after filling `out`)
 * when the state holds a NaN or Inf. */
cdi_status cdi_diagnostics(cdi_ctx* ctx, int32_t idx, cdi_diag* out);

/* Stage operator of instance 0 on its current fields (no time update, no
 * projection): writes L_phi (ny*nx), L_mx (ny*nx) and L_my ((ny+1)*nx, wall
 * rows 0) to the caller's device buffers, and the wall values per corner
 * (2*nx each, bottom then top) of u^Y and u_wall - U_wall when the optional
 * pointers are non-NULL.  The right-hand side of eq. CDI and of the momentum
 * equation without the pressure gradient. */
cdi_status cdi_eval_rhs(cdi_ctx* ctx, double* l_phi, double* l_mx, double* l_my,
                        double* u_y, double* u_slip);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the stage
 * operator of cdi_eval_rhs for one instance without a context or workspace.
 * params: the problem as for cdi_init (validated the same way; the solver
 * fields poisson_* and guess are ignored); fields: device pointers phi, u, v
 * (p is not read), layouts as above; outputs as for cdi_eval_rhs: L_phi and
 * L_mx (ny*nx), L_my ((ny+1)*nx, wall rows written as 0), and, when non-NULL,
 * u^Y and u_wall - U_wall per wall corner (2*nx each, bottom then top).  All
 * work is enqueued on hip_stream (NULL = default stream) and the call
 * returns without synchronising.
 * Its scratch (instance descriptor, tile list, CG scalars, reduction
 * partials and counters, wall values when u_y / u_slip are NULL; the
 * phase-field quantities n and mu_c are formed in the kernel's LDS) lives in
 * a file-scope device array of CDI_NOALLOC_SCRATCH_BYTES bytes that every
 * GPU the library runs on holds until the process ends; the call performs
 * no device or pinned-host allocation and no memset (a kernel clears the
 * counters).  A grid whose scratch does not fit (about 0.4 bytes per cell:
 * beyond ~170 M cells) returns CDI_ERR_SHAPE.  Every call on one GPU
 * shares that GPU's array and keeps the last call's contents: calls that
 * overlap on one GPU (different streams or host threads without ordering)
 * race. */
#define CDI_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
cdi_status cdi_eval_rhs_noalloc(const cdi_params* params, const cdi_fields* fields,
                                double* l_phi, double* l_mx, double* l_my, double* u_y,
                                double* u_slip, void* hip_stream);

/* Measurement hook.  While enabled, every launch of the named kernel family
 * ("phase_prep", "stage", "rhs", "pcg_init", "mg_down" (finest level, with the
 * fused CG update), "mg_down_other", "mg_coarse", "mg_up" (finest level),
 * "mg_up_other", "mg_coef", "pcg_spmv", "pcg_xmean", "project", "net",
 * "persistent") is bracketed
 * by HIP events on the context stream; NULL disables.  Resets the totals. */
cdi_status cdi_timing_enable(cdi_ctx* ctx, const char* kernel);

/* Summed device time (ms) and number of the measured launches since
 * cdi_timing_enable.  Synchronises the stream. */
cdi_status cdi_timing_read(cdi_ctx* ctx, double* total_ms, int64_t* launches);

/* ------------------------------------------------------------------------
 * Learned pressure guess.  A small encoder-decoder network (4 levels,
 * 32/64/128/256 channels, 3x3 convolutions, BF16 matrix cores with FP32
 * accumulation) maps the features (phi, rho/max(rho1,rho2), b_hat) of a
 * projection to a normalised pressure; its output is only the initial guess
 * of the flexible CG, which still iterates to poisson_rtol.
 *   b_hat = (b - mean b) / rms(b - mean b),
 *   g     = y * rms(b - mean b) * max(rho1, rho2) * h^2,
 * and the initial guess is x0 = a p_prev + c g with (a, c) the Galerkin fit
 * on span{p_prev, g} (p_prev the previous pressure) computed on the device,
 * so that x0 is never worse than p_prev or zero in the energy norm of the
 * operator.
 * Parameters are FP32 in a fixed order (per 3x3 layer e0, e1, e2, e3, d2,
 * d1, d0: weights [co][ci][3][3] then biases [co]; then the 1x1 output layer
 * weights [32] and bias [1]), owned by the caller. */
typedef struct cdi_net cdi_net;

/* Number of FP32 parameters. */
size_t cdi_net_param_count(void);

/* Device workspace bytes of a network for `batch` images of h x w cells
 * (h, w multiples of 8); train != 0 adds the gradient buffers. */
size_t cdi_net_workspace_bytes(int32_t batch, int32_t h, int32_t w, int32_t train);

/* Create a network over caller-owned params (and grads when train != 0),
 * workspace and stream.  Packs the BF16 weights. */
cdi_status cdi_net_init(const float* params, float* grads, int32_t batch, int32_t h, int32_t w,
                        int32_t train, void* workspace, size_t workspace_bytes, void* hip_stream,
                        cdi_net** out);

/* Re-pack the BF16 weights after the caller changed params. */
cdi_status cdi_net_repack(cdi_net* net);

/* x: FP32 [batch][3][h][w] features; y: FP32 [batch][h][w] output. */
cdi_status cdi_net_forward(cdi_net* net, const float* x, float* y);

/* Mean-squared-error gradients of the last forward pass against target
 * (FP32 [batch][h][w]) into grads; loss (device FP32 scalar) may be NULL. */
cdi_status cdi_net_backward(cdi_net* net, const float* target, float* loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; step counts from 1) on
 * params with caller-owned FP32 moments m, v (zero-initialised). */
cdi_status cdi_net_adam(cdi_net* net, float* m, float* v, int32_t step, double lr);

void cdi_net_destroy(cdi_net* net);
const char* cdi_net_last_error(void);

/* Use `net` (batch 1, h = ny, w = nx of instance 0, same stream) for the
 * initial guess of the pressure solves of a single-instance context while
 * its guess mode is CDI_GUESS_LEARNED; NULL detaches (the previous pressure
 * is then used).  The context borrows the network. */
cdi_status cdi_guess_attach(cdi_ctx* ctx, cdi_net* net);

/* How cdi_step enqueues the work of a step (same discretisation and solver
 * either way; results agree to the solver tolerance, not bitwise, because
 * the CG reductions are summed in a different order):
 *   CDI_LAUNCH_TILED (default): every phase of the step is a launch over
 *     tiles of every instance (many workgroups per instance); the host
 *     checks the CG stopping test every few iterations.
 *   CDI_LAUNCH_PERSISTENT: one launch per 32 steps with one workgroup of
 *     1024 threads per instance running whole steps, CG loop and stopping
 *     test included, with no host round trip (pays off for small grids and
 *     ensembles of them).
 *   CDI_LAUNCH_GRAPH: the tiled kernels of a whole step captured once in a
 *     HIP graph with a fixed CG iteration budget per solve (the largest
 *     recent count + 1; iterations after convergence return at once, so the
 *     results are bitwise those of CDI_LAUNCH_TILED) and replayed every step
 *     on a stream of the library's own, ordered after and before the
 *     caller's stream by events; one host synchronisation per step.  A step
 *     that needs more iterations than the budget is redone from a snapshot
 *     on the stream path and the budget grows.  The first steps of a run,
 *     until the pressure history of the extrapolated guess is complete
 *     (order + 1 steps, cdi_set_extrapolation), take the stream path.
 * PERSISTENT and GRAPH are not available with CDI_GUESS_LEARNED and an
 * attached network (cdi_step then returns CDI_ERR_STATE); PERSISTENT is not
 * available with gamma_factor > 0 (CDI_ERR_ARG). */
cdi_status cdi_set_launch(cdi_ctx* ctx, int32_t mode);
cdi_status cdi_get_launch(cdi_ctx* ctx, int32_t* mode);

/* Graph launch counters: steps replayed from the captured graph, steps
 * redone on the stream path after exceeding the budget, and the current
 * CG iteration budget per solve (0 = no graph captured). */
cdi_status cdi_graph_stats(cdi_ctx* ctx, int64_t* replays, int64_t* redone, int32_t* budget);

/* Rows per thread of the wide-tile CG kernels (right-hand side, CG start,
 * CG direction and operator product, projection): 1 (64 x 4 cell tiles,
 * more and shorter workgroups, suits small grids) or 4 (64 x 16 cell tiles,
 * fewer workgroups, shorter halos and fewer partial sums on large grids).
 * cdi_init picks 4 from 2^18 cells per batch on, else 1. */
cdi_status cdi_set_tile_rows(cdi_ctx* ctx, int32_t rows);
cdi_status cdi_get_tile_rows(cdi_ctx* ctx, int32_t* rows);

/* Rows of the strips of the FP64 stage kernel (59 columns each, advanced
 * four rows at a time): 16, 32 or 64.  Taller strips recompute fewer halo
 * rows; shorter ones give the GPU more workgroups.  cdi_init picks the
 * tallest that gives every compute unit several strips (about 2300 per
 * batch).  Results agree across strip heights to rounding.  Other values
 * return CDI_ERR_ARG. */
cdi_status cdi_set_strip_rows(cdi_ctx* ctx, int32_t rows);
cdi_status cdi_get_strip_rows(cdi_ctx* ctx, int32_t* rows);

/* Start of the one-block coarse kernel of the V-cycle: it runs every level
 * with at most `cells` cells (levels up to 1024 cells in its LDS; a start
 * level just above those, at most 4096 cells, with its correction and
 * residual in LDS and its cells in registers; larger ones from global
 * memory); the finer levels run as tiled kernels.  Larger
 * values mean fewer launches per CG iteration but more work on one compute
 * unit.  cells in [1024, 2^20]; cdi_init sets 4096. */
cdi_status cdi_set_coarse_cells(cdi_ctx* ctx, int32_t cells);
cdi_status cdi_get_coarse_cells(cdi_ctx* ctx, int32_t* cells);

/* Order of the time extrapolation that forms each solve's initial guess
 * (previous-pressure guess): the same RK stage's pressure of the last q + 1
 * steps, combined with the weights of the polynomial through them (q = 0:
 * the last step's pressure; 1: linear, 2 p1 - p2; 2: quadratic, 3 p1 - 3 p2
 * + p3; 3: cubic, 4 p1 - 6 p2 + 4 p3 - p4), lowered while fewer steps
 * exist.  order in [0, 3]; cdi_init sets 3.  The guess is an implementation
 * choice of the solver (the paper does not specify one): it changes the
 * iteration count, not the converged solution. */
cdi_status cdi_set_extrapolation(cdi_ctx* ctx, int32_t order);
cdi_status cdi_get_extrapolation(cdi_ctx* ctx, int32_t* order);

/* Red-black sweep pairs of the V-cycle's tiled levels (1 or 2; the value of
 * mg_smooth at init; the one-block coarse cycle takes one pair more).
 * Changes the iteration count, not the converged solution. */
cdi_status cdi_set_mg_smooth(cdi_ctx* ctx, int32_t nu);
cdi_status cdi_get_mg_smooth(cdi_ctx* ctx, int32_t* nu);

/* Autotuner: times `trial_steps` steps (after warm-up steps) of every launch
 * candidate -- tiled with 1 and 2 sweep pairs, 1 and 4 rows per thread, the
 * coarse kernel starting at 1024, 4096 and 16384 cells; persistent (with the
 * fastest tiled sweep count; skipped when an instance has more than 16384
 * cells, where one block per instance cannot compete, and with gamma_factor
 * > 0); graph (with the
 * fastest tiled shape) -- each
 * from the same saved state, restores that state (fields, pressure history,
 * time and step counters), and keeps the fastest candidate for later
 * cdi_step calls.  The pressure still meets poisson_rtol in every candidate.
 * `scratch` is caller-owned device memory of at least cdi_tune_bytes(ctx)
 * bytes for the saved state.  Synchronises the stream. */
typedef struct {
  int32_t launch;          /* chosen CDI_LAUNCH_*                                  */
  int32_t tile_rows;       /* chosen rows per thread (1 or 4)                      */
  int32_t coarse_cells;    /* chosen coarse-kernel threshold                       */
  int32_t mg_smooth;       /* chosen sweep pairs                                   */
  int32_t ncand;           /* candidates timed                                     */
  int32_t strip_rows;      /* stage-kernel strip height (cdi_tune_concurrent only,
                              else 0)                                              */
  double ms_per_step[14];  /* tiled [sweeps 1, 2] x [rows 1, 4] x [coarse 1024,
                              4096, 16384] (row-major), persistent, graph;
                              -1 = skipped                                         */
} cdi_tune_info;

size_t cdi_tune_bytes(const cdi_ctx* ctx);
cdi_status cdi_tune(cdi_ctx* ctx, int32_t trial_steps, void* scratch, size_t scratch_bytes,
                    cdi_tune_info* out);

/* Autotuner for contexts advanced together by cdi_step_concurrent: one tiled
 * shape (sweep pairs, rows per thread, coarse-kernel threshold; the 12 tiled
 * candidates of cdi_tune) for all n contexts, each candidate timed as the
 * host wall time of `trial_steps` concurrent steps (after one warm-up step)
 * between device synchronisations of every context's stream, and every
 * context restored to its saved state after each candidate, as cdi_tune
 * does.  The shape that is fastest alone is not the fastest when the
 * contexts share the GPU.  scratch[k]: device memory of at least
 * cdi_tune_bytes(ctxs[k]) bytes (scratch_bytes[k]); out (may be NULL) as
 * cdi_tune (ms_per_step slots 12 and 13 are -1).  With that shape it then
 * times the stage kernel's strip heights (16, 32, 64 rows) the same way and
 * keeps the fastest (out->strip_rows).  Sets the tiled launch on every
 * context.  Synchronises every stream. */
cdi_status cdi_tune_concurrent(cdi_ctx* const* ctxs, int32_t n, int32_t trial_steps,
                               void* const* scratch, const size_t* scratch_bytes,
                               cdi_tune_info* out);

/* Switch the initial-guess mode (CDI_GUESS_*) of later pressure solves. */
cdi_status cdi_set_guess(cdi_ctx* ctx, int32_t guess);

/* Features and normalised target of instance idx's last projection (after
 * cdi_step: the final-stage projection of the last step): features FP32
 * [3][ny][nx] = (phi, rho / max(rho1, rho2), asinh((b - mean b) / rms b)),
 * target FP32 [ny][nx] (may be NULL) = the pressure scaled to unit rms (the
 * learned guess enters the solve through a scale-invariant fit), both device
 * buffers. */
cdi_status cdi_guess_features(cdi_ctx* ctx, int32_t idx, float* features, float* target);

/* Release the context (host memory only; caller buffers are untouched). */
void cdi_destroy(cdi_ctx* ctx);

/* Message of the last error on this thread ("" if none). */
const char* cdi_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CDI_H */
