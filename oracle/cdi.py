"""FP64 CPU oracle of one CDI + GNBC time step (TEST INFRASTRUCTURE).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg use this
module.  It is written from the paper (arXiv:2412.16843) and shares no code
with the HIP path.

Grid (Sec. 4): uniform staggered grid, spacing h, x periodic, walls at y = 0
and y = Ly.  Arrays are row-major, x fastest:
  phi, p   (ny, nx)    cell centres ((i+1/2)h, (j+1/2)h)
  u        (ny, nx)    x-face i of row j, at (i h, (j+1/2) h)
  v        (ny+1, nx)  y-face j of column i, at ((i+1/2) h, j h); rows 0, ny
                       are the walls and hold v = 0 (no penetration, Sec. 2)
Corner (i, j) sits at (i h, j h); corner rows 0 and ny lie on the walls.

Readings of points the paper leaves open (each used identically by the GPU
path):
  * n = G / (|G| + DELTA_N), G the cell-centred gradient of phi;
  * psi = eps ln((clip(phi) + DELTA_PSI) / (1 - clip(phi) + DELTA_PSI));
  * face values are arithmetic means of the two adjacent cells, corner
    viscosity the mean of the four surrounding cells;
  * momentum advection uses the mass flux m = rho2 u + (rho1 - rho2) F, F the
    very face flux of the phi update (Sec. 2, S = (rho1 - rho2) R);
  * wall quantities of the slip models: per column linear extrapolation
    q_w = (3 q_0 - q_1) / 2 from the two cells nearest the wall (Sec. 4),
    averaged to the corner; the slip enters the momentum as a Robin wall
    velocity / wall shear stress;
  * RK4 with a projection after every stage and after the final combine
    (4 pressure solves per step), pressure absent from the right-hand side.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Tuple

import numpy as np

from . import poisson

DELTA_N = 1e-12      # normal-vector regularisation (1/length)
DELTA_PSI = 1e-12    # keeps psi finite at phi in {0, 1}

RK_C = (0.0, 0.5, 0.5, 1.0)
RK_B = (1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0)


# ---------------------------------------------------------------------------
# cell-centred difference operators (Sec. 4): second-order central in the
# interior, second-order one-sided in the wall-normal direction on the first
# and last cell rows.  No ghost value of phi is ever formed.
# ---------------------------------------------------------------------------

def ddx(q: np.ndarray, h: float) -> np.ndarray:
    return (np.roll(q, -1, axis=1) - np.roll(q, 1, axis=1)) / (2.0 * h)


def ddy(q: np.ndarray, h: float) -> np.ndarray:
    out = np.empty_like(q)
    out[1:-1] = (q[2:] - q[:-2]) / (2.0 * h)
    out[0] = (-3.0 * q[0] + 4.0 * q[1] - q[2]) / (2.0 * h)
    out[-1] = (3.0 * q[-1] - 4.0 * q[-2] + q[-3]) / (2.0 * h)
    return out


def d2dx2(q: np.ndarray, h: float) -> np.ndarray:
    return (np.roll(q, -1, axis=1) - 2.0 * q + np.roll(q, 1, axis=1)) / (h * h)


def d2dy2(q: np.ndarray, h: float) -> np.ndarray:
    out = np.empty_like(q)
    out[1:-1] = (q[2:] - 2.0 * q[1:-1] + q[:-2]) / (h * h)
    out[0] = (2.0 * q[0] - 5.0 * q[1] + 4.0 * q[2] - q[3]) / (h * h)
    out[-1] = (2.0 * q[-1] - 5.0 * q[-2] + 4.0 * q[-3] - q[-4]) / (h * h)
    return out


# ---------------------------------------------------------------------------
# phase-field quantities (Sec. 2)
# ---------------------------------------------------------------------------

def psi_of(phi: np.ndarray, eps: float) -> np.ndarray:
    """Approximate signed distance psi = eps ln(phi / (1 - phi)) (eq. psi)."""
    ph = np.clip(phi, 0.0, 1.0)
    return eps * np.log((ph + DELTA_PSI) / (1.0 - ph + DELTA_PSI))


def normal(phi: np.ndarray, h: float) -> Tuple[np.ndarray, np.ndarray]:
    """Interface normal n = grad(phi) / |grad(phi)| (Sec. 2, eq. CDI)."""
    gx = ddx(phi, h)
    gy = ddy(phi, h)
    mag = np.sqrt(gx * gx + gy * gy) + DELTA_N
    return gx / mag, gy / mag


def psi_derivatives(psi: np.ndarray, h: float):
    """(d psi/dx, d psi/dy, laplacian psi) with the wall-row one-sided stencils."""
    return ddx(psi, h), ddy(psi, h), d2dx2(psi, h) + d2dy2(psi, h)


def curvature(phi, psix, psiy, lap, eps):
    """Energy-based curvature kappa = (1 - 2 phi)(1 - |grad psi|^2)/eps - lap psi
    (eq. curvature)."""
    return (1.0 - 2.0 * phi) * (1.0 - psix * psix - psiy * psiy) / eps - lap


def chemical_potential(phi, psix, psiy, lap, eps, sigma):
    """psi-form chemical potential (eq. chemical potential):
    6 sigma [phi(1-phi)(1-2phi)(1-|grad psi|^2)/eps - phi(1-phi) lap psi]."""
    g = phi * (1.0 - phi)
    return 6.0 * sigma * (g * (1.0 - 2.0 * phi) * (1.0 - psix * psix - psiy * psiy) / eps
                          - g * lap)


def chemical_potential_gl(phi, eps, sigma, h):
    """Ginzburg-Landau form 6 sigma [phi(1-phi)(1-2phi)/eps - eps lap phi]
    (Sec. 2), analytically equal to the psi form; used only as a cross-check."""
    lap = d2dx2(phi, h) + d2dy2(phi, h)
    return 6.0 * sigma * (phi * (1.0 - phi) * (1.0 - 2.0 * phi) / eps - eps * lap)


# ---------------------------------------------------------------------------
# wall slip (Sec. 2 slip BC, Sec. 3 Models 1A..4B, Sec. 4 extrapolation)
# ---------------------------------------------------------------------------

def _extrap(q: np.ndarray, wall: str) -> np.ndarray:
    """Linear extrapolation of a cell field to the wall, per column."""
    if wall == "bot":
        return 0.5 * (3.0 * q[0] - q[1])
    return 0.5 * (3.0 * q[-1] - q[-2])


def _to_corner(qw: np.ndarray) -> np.ndarray:
    """Average a per-column wall value to the wall corners x = i h."""
    return 0.5 * (np.roll(qw, 1) + qw)


def slip_velocity_Y(phi: np.ndarray, p, wall: str, model: str | None = None,
                    fields: Dict[str, np.ndarray] | None = None) -> Dict[str, np.ndarray]:
    """Contact-line (Young's) slip u^Y at the corners of one wall.

    Every phase-field quantity is extrapolated from the first two cell rows to
    the wall (Sec. 4) and averaged to the corner; the wall-normal derivative is
    taken along the inward normal (bottom: +y, top: -y) and the tangential one
    along +x on both walls.  Returns the corner values used and u^Y.
    """
    model = model or p.slip_model
    h, eps = p.h, p.eps
    if fields is None:
        psi = psi_of(phi, eps)
        psix, psiy, lap = psi_derivatives(psi, h)
        kap = curvature(phi, psix, psiy, lap, eps)
        fields = dict(psi=psi, psiy=psiy, kappa=kap, phiy=ddy(phi, h))
    sgn = 1.0 if wall == "bot" else -1.0
    phw = _extrap(phi, wall)
    psw = _extrap(fields["psi"], wall)
    dpsw = _extrap(fields["psiy"], wall)
    kaw = _extrap(fields["kappa"], wall)
    dphw = _extrap(fields["phiy"], wall)

    phc = np.clip(_to_corner(phw), 0.0, 1.0)
    psc = _to_corner(psw)
    kac = _to_corner(kaw)
    dpsi_n = sgn * _to_corner(dpsw)
    dpsi_t = (psw - np.roll(psw, 1)) / h
    dphi_n = sgn * _to_corner(dphw)
    dphi_t = (phw - np.roll(phw, 1)) / h
    g = phc * (1.0 - phc)
    beta = p.beta2 + (p.beta1 - p.beta2) * phc
    ce = math.cos(p.theta_eq)
    corr = 1.0 + kac * psc          # curvature correction (Sec. 3.1.2)
    gradphi = np.sqrt(dphi_n ** 2 + dphi_t ** 2)
    gradpsi = np.sqrt(dpsi_n ** 2 + dpsi_t ** 2)
    pre = -6.0 * p.sigma / beta
    if model == "1A":
        uY = pre * (eps * dphi_n + g * ce) * dphi_t
    elif model == "1B":
        uY = pre * (eps * dphi_n + eps * gradphi * ce) * dphi_t
    elif model == "3A":
        uY = pre * (eps * dphi_n + g * corr * ce) * dphi_t
    elif model == "3B":
        uY = pre * (eps * dphi_n + eps * gradphi * corr * ce) * dphi_t
    elif model == "2A":
        uY = pre * (g * dpsi_n + g * ce) * g / eps * dpsi_t
    elif model == "2B":
        uY = pre * (g * dpsi_n + g * gradpsi * ce) * g / eps * dpsi_t
    elif model == "4A":
        uY = pre * (g * dpsi_n + g * corr * ce) * g / eps * dpsi_t
    elif model == "4B":
        uY = pre * (g * dpsi_n + g * gradpsi * corr * ce) * g / eps * dpsi_t
    else:
        raise ValueError(f"unknown slip model {model!r}")
    return dict(phi_c=phc, psi_c=psc, kappa_c=kac, dpsi_n=dpsi_n, dpsi_t=dpsi_t,
                beta=beta, uY=uY, phi_w=phw)


def wall_stress(phi, u, p, fields) -> Dict[str, Dict[str, np.ndarray]]:
    """GNBC wall velocity and shear stress at both walls.

    u_slip = u_wall - U_wall = (mu/beta) du_tau/dn + u^Y (Sec. 2, slip BC),
    with du_tau/dn = 2 (u_first_row - u_wall)/h along the inward normal, solved
    for u_wall; the wall shear stress is mu du/dy at the wall.
    """
    h = p.h
    out = {}
    for wall, urow, U in (("bot", u[0], p.u_wall_bot), ("top", u[-1], p.u_wall_top)):
        s = slip_velocity_Y(phi, p, wall, fields=fields)
        mu_w = p.mu2 + (p.mu1 - p.mu2) * s["phi_c"]
        lam = 2.0 * mu_w / (s["beta"] * h)
        uw = (U + s["uY"] + lam * urow) / (1.0 + lam)
        if wall == "bot":
            tau = 2.0 * mu_w * (urow - uw) / h
        else:
            tau = 2.0 * mu_w * (uw - urow) / h
        s.update(u_wall=uw, tau=tau, u_slip=uw - U)
        out[wall] = s
    return out


# ---------------------------------------------------------------------------
# stage operator
# ---------------------------------------------------------------------------

def rho_of(phi, p):
    return (p.rho1 - p.rho2) * phi + p.rho2


def mu_of(phi, p):
    return (p.mu1 - p.mu2) * phi + p.mu2


def face_rho(phi, p):
    """Face densities: x-faces (ny, nx), y-faces (ny+1, nx) with wall rows = nan."""
    rho = rho_of(phi, p)
    rfx = 0.5 * (np.roll(rho, 1, axis=1) + rho)
    ny, nx = phi.shape
    rfy = np.full((ny + 1, nx), np.nan)
    rfy[1:ny] = 0.5 * (rho[:-1] + rho[1:])
    return rfx, rfy


def phase_fields(phi: np.ndarray, p) -> Dict[str, np.ndarray]:
    h, eps = p.h, p.eps
    nxv, nyv = normal(phi, h)
    psi = psi_of(phi, eps)
    psix, psiy, lap = psi_derivatives(psi, h)
    kap = curvature(phi, psix, psiy, lap, eps)
    muc = chemical_potential(phi, psix, psiy, lap, eps, p.sigma)
    return dict(nx=nxv, ny=nyv, psi=psi, psix=psix, psiy=psiy, lap=lap, kappa=kap,
                muc=muc, phiy=ddy(phi, h))


def phi_fluxes(phi, u, v, f, p):
    """CDI face fluxes F = u phi_f - R_f (eq. CDI) with R = gamma[eps grad phi
    - phi(1-phi) n]; the wall y-faces carry F = 0 (no-flux + no-penetration)."""
    h, eps, gam = p.h, p.eps, p.gamma
    ny, nx = phi.shape
    phL = np.roll(phi, 1, axis=1)
    phf = 0.5 * (phL + phi)
    nxf = 0.5 * (np.roll(f["nx"], 1, axis=1) + f["nx"])
    Rx = gam * (eps * (phi - phL) / h - phf * (1.0 - phf) * nxf)
    Fx = u * phf - Rx
    Fy = np.zeros((ny + 1, nx))
    phb, pht = phi[:-1], phi[1:]
    phfy = 0.5 * (phb + pht)
    nyf = 0.5 * (f["ny"][:-1] + f["ny"][1:])
    Ry = gam * (eps * (pht - phb) / h - phfy * (1.0 - phfy) * nyf)
    Fy[1:ny] = v[1:ny] * phfy - Ry
    return Fx, Fy


def stage_rhs(phi, u, v, p):
    """L(phi, u, v) -> (L_phi, L_mx, L_my, wall dict): the semi-discrete
    right-hand sides of the CDI equation and of the mixture momentum
    (eq. NS_momentum without the pressure gradient)."""
    h = p.h
    ny, nx = phi.shape
    f = phase_fields(phi, p)
    Fx, Fy = phi_fluxes(phi, u, v, f, p)
    Lphi = -((np.roll(Fx, -1, axis=1) - Fx) + (Fy[1:] - Fy[:-1])) / h

    # mass fluxes rho u - S with S = (rho1 - rho2) R
    drho = p.rho1 - p.rho2
    mx = p.rho2 * u + drho * Fx
    my = p.rho2 * v + drho * Fy            # zero on both walls
    mu = mu_of(phi, p)
    muc = f["muc"]
    walls = wall_stress(phi, u, p, f)

    # ---- corner shear stress tau_xy at corners (i, j), j = 0..ny
    tauxy = np.zeros((ny + 1, nx))
    mu4 = 0.25 * (mu[:-1] + np.roll(mu[:-1], 1, axis=1) + mu[1:] + np.roll(mu[1:], 1, axis=1))
    dudy = (u[1:] - u[:-1]) / h
    dvdx = (v[1:ny] - np.roll(v[1:ny], 1, axis=1)) / h
    tauxy[1:ny] = mu4 * (dudy + dvdx)
    tauxy[0] = walls["bot"]["tau"]
    tauxy[ny] = walls["top"]["tau"]

    # ---- x-momentum at u[j, i]
    fc = 0.5 * (mx + np.roll(mx, -1, axis=1)) * 0.5 * (u + np.roll(u, -1, axis=1))  # cell i
    fcy = np.zeros((ny + 1, nx))                                                      # corner (i, j)
    fcy[1:ny] = (0.5 * (np.roll(my[1:ny], 1, axis=1) + my[1:ny])
                 * 0.5 * (u[:-1] + u[1:]))
    tauxx = 2.0 * mu * (np.roll(u, -1, axis=1) - u) / h                               # cell i
    stx = 0.5 * (np.roll(muc, 1, axis=1) + muc) * (phi - np.roll(phi, 1, axis=1)) / h
    Lmx = (-((fc - np.roll(fc, 1, axis=1)) + (fcy[1:] - fcy[:-1])) / h
           + (tauxx - np.roll(tauxx, 1, axis=1)) / h
           + (tauxy[1:] - tauxy[:-1]) / h
           + stx)

    # ---- y-momentum at interior v[j, i], j = 1..ny-1
    gc = 0.5 * (my[:-1] + my[1:]) * 0.5 * (v[:-1] + v[1:])                           # cell row c
    fcx = 0.5 * (mx[:-1] + mx[1:]) * 0.5 * (np.roll(v[1:ny], 1, axis=1) + v[1:ny])   # corner (i, j)
    tauyy = 2.0 * mu * (v[1:] - v[:-1]) / h                                            # cell
    sty = 0.5 * (muc[:-1] + muc[1:]) * (phi[1:] - phi[:-1]) / h
    Lmy = np.zeros((ny + 1, nx))
    Lmy[1:ny] = (-((np.roll(fcx, -1, axis=1) - fcx) + (gc[1:] - gc[:-1])) / h
                 + (tauyy[1:] - tauyy[:-1]) / h
                 + (np.roll(tauxy[1:ny], -1, axis=1) - tauxy[1:ny]) / h
                 + sty)
    return Lphi, Lmx, Lmy, walls


# ---------------------------------------------------------------------------
# projection and time step
# ---------------------------------------------------------------------------

def divergence(u, v, h):
    return ((np.roll(u, -1, axis=1) - u) + (v[1:] - v[:-1])) / h


def project(us, vs, phi, tau, p, solver=None):
    """Make (us, vs) discretely divergence-free with the variable-density
    pressure of A p = div(u*) / tau; returns (u, v, p)."""
    h = p.h
    rfx, rfy = face_rho(phi, p)
    b = divergence(us, vs, h) / tau
    b = b - b.mean()
    if solver is None:
        pr = poisson.solve(b, rho_of(phi, p), rfx, rfy, h)
    else:
        pr = solver(b, phi)
    u = us - tau * (pr - np.roll(pr, 1, axis=1)) / (h * rfx)
    v = vs.copy()
    v[1:-1] = vs[1:-1] - tau * (pr[1:] - pr[:-1]) / (h * rfy[1:-1])
    v[0] = 0.0
    v[-1] = 0.0
    return u, v, pr


@dataclasses.dataclass
class State:
    phi: np.ndarray
    u: np.ndarray
    v: np.ndarray
    p: np.ndarray
    t: float = 0.0
    step: int = 0

    def copy(self) -> "State":
        return State(self.phi.copy(), self.u.copy(), self.v.copy(), self.p.copy(),
                     self.t, self.step)


def initial_state(phi0: np.ndarray) -> State:
    ny, nx = phi0.shape
    return State(phi0.astype(np.float64).copy(), np.zeros((ny, nx)), np.zeros((ny + 1, nx)),
                 np.zeros((ny, nx)))


def step_gamma(u: np.ndarray, v: np.ndarray, p) -> float:
    """Regularisation velocity of a step that starts from velocities (u, v).
    The paper sets gamma = 2.5 |u|_max (Sec. 5, drop and Couette cases); with
    gamma_factor > 0 it is read here as gamma_factor times the largest face
    velocity magnitude |u| or |v| of the starting state, bounded above by the
    fixed gamma (the value the time step is sized for).  gamma_factor = 0
    keeps gamma fixed."""
    f = getattr(p, "gamma_factor", 0.0)
    if f <= 0.0:
        return p.gamma
    return min(p.gamma, f * max(float(np.abs(u).max()), float(np.abs(v).max())))


def step(s: State, p, solver=None) -> State:
    """One RK4 step (Sec. 4) of the coupled CDI / momentum system with a
    projection after every stage and after the final combination; gamma is
    held for the whole step (step_gamma)."""
    if getattr(p, "gamma_factor", 0.0) > 0.0:
        p = p.replace(gamma=step_gamma(s.u, s.v, p), gamma_factor=0.0)
    dt = p.dt
    phi0, u0, v0 = s.phi, s.u, s.v
    rfx0, rfy0 = face_rho(phi0, p)
    mx0 = rfx0 * u0
    my0 = np.zeros_like(v0)
    my0[1:-1] = rfy0[1:-1] * v0[1:-1]
    acc_phi = acc_mx = acc_my = None
    ph, uu, vv = phi0, u0, v0
    pr = s.p
    for k in range(4):
        Lphi, Lmx, Lmy, _ = stage_rhs(ph, uu, vv, p)
        if k == 0:
            acc_phi, acc_mx, acc_my = RK_B[0] * Lphi, RK_B[0] * Lmx, RK_B[0] * Lmy
        else:
            acc_phi = acc_phi + RK_B[k] * Lphi
            acc_mx = acc_mx + RK_B[k] * Lmx
            acc_my = acc_my + RK_B[k] * Lmy
        if k < 3:
            c = RK_C[k + 1] * dt
            ph = phi0 + c * Lphi
            uu, vv = _momentum_to_velocity(mx0 + c * Lmx, my0 + c * Lmy, ph, p)
            uu, vv, pr = project(uu, vv, ph, c, p, solver)
    ph = phi0 + dt * acc_phi
    uu, vv = _momentum_to_velocity(mx0 + dt * acc_mx, my0 + dt * acc_my, ph, p)
    uu, vv, pr = project(uu, vv, ph, dt, p, solver)
    return State(ph, uu, vv, pr, s.t + dt, s.step + 1)


def _momentum_to_velocity(mx, my, phi, p):
    rfx, rfy = face_rho(phi, p)
    u = mx / rfx
    v = np.zeros_like(my)
    v[1:-1] = my[1:-1] / rfy[1:-1]
    return u, v


def run(phi0: np.ndarray, p, steps: int, solver=None) -> State:
    s = initial_state(phi0)
    for _ in range(steps):
        s = step(s, p, solver)
    return s


# ---------------------------------------------------------------------------
# diagnostics (Sec. 5.1)
# ---------------------------------------------------------------------------

def contact_points(phi_w: np.ndarray, h: float):
    """x positions where the extrapolated wall phase field crosses 1/2, by
    linear interpolation between column centres (periodic)."""
    n = phi_w.size
    xs = (np.arange(n) + 0.5) * h
    out = []
    for i in range(n):
        a, b = phi_w[i] - 0.5, phi_w[(i + 1) % n] - 0.5
        if a == 0.0:
            out.append(xs[i])
        elif a * b < 0.0:
            out.append(xs[i] + h * a / (a - b))
    return out


def cap_angle(L: float, area: float) -> float:
    """Contact angle of a circular cap with wetted length L and area `area`:
    root of area = (L / (2 sin t))^2 (t - sin t cos t) on (0, pi)."""
    f = lambda t: (L / (2.0 * math.sin(t))) ** 2 * (t - math.sin(t) * math.cos(t)) - area
    lo, hi = 1e-6, math.pi - 1e-6
    flo = f(lo)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        fm = f(mid)
        if (fm > 0) == (flo > 0):
            lo, flo = mid, fm
        else:
            hi = mid
    return 0.5 * (lo + hi)


def diagnostics(s: State, p) -> Dict[str, float]:
    h = p.h
    f = phase_fields(s.phi, p)
    walls = wall_stress(s.phi, s.u, p, f)
    rfx, rfy = face_rho(s.phi, p)
    ke = 0.5 * h * h * (np.sum(rfx * s.u ** 2) + np.sum(rfy[1:-1] * s.v[1:-1] ** 2))
    out = dict(mass=float(np.sum(s.phi) * h * h), phi_min=float(s.phi.min()),
               phi_max=float(s.phi.max()),
               max_div=float(np.max(np.abs(divergence(s.u, s.v, h)))),
               max_uslip_bot=float(np.max(np.abs(walls["bot"]["u_slip"]))),
               max_uslip_top=float(np.max(np.abs(walls["top"]["u_slip"]))),
               max_uY_bot=float(np.max(np.abs(walls["bot"]["uY"]))),
               max_uY_top=float(np.max(np.abs(walls["top"]["uY"]))),
               ke=float(ke))
    for wall in ("bot", "top"):
        cps = contact_points(walls[wall]["phi_w"], h)
        out[f"n_contact_{wall}"] = len(cps)
        out[f"contact_x_{wall}"] = cps[:2]
        if len(cps) == 2:
            L = abs(cps[1] - cps[0])
            out[f"wetted_len_{wall}"] = L
            out[f"theta_est_{wall}"] = cap_angle(L, out["mass"])
    return out
