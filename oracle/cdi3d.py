"""FP64 CPU oracle of the three-dimensional CDI + GNBC time step (TEST
INFRASTRUCTURE).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg use this
module.  It shares no code with the HIP path.  The paper states its model for
a general wall (inward normal n_wall, tangential direction tau_wall, the
curvature kappa_p of the interface in the plane containing n_phi and n_wall;
Sec. 2, slip BC, and Sec. 3.1.2) and computes in two dimensions only
(Sec. 4); this module is the same discretisation carried to three.

Grid: uniform staggered grid of spacing h, x and z periodic, walls at y = 0
and y = Ly.  Arrays have shape (nz, ny, nx), x fastest:
  phi, p   (nz, ny, nx)     cell centres
  u        (nz, ny, nx)     x-face i (x = i h)
  v        (nz, ny+1, nx)   y-face j (y = j h); rows 0 and ny lie on the walls
                            and hold v = 0 (no penetration, Sec. 2)
  w        (nz, ny, nx)     z-face k (z = k h)
Edges (where shear stresses and cross advection fluxes live):
  xy-edge (k, j, i) at (i h, j h, (k+1/2) h), rows j = 0..ny (0, ny on walls)
  yz-edge (k, j, i) at ((i+1/2) h, j h, k h), rows j = 0..ny (0, ny on walls)
  xz-edge (k, j, i) at (i h, (j+1/2) h, k h)

Readings beyond those of the two-dimensional oracle (oracle.cdi):
  * the Young slip is a vector in the wall plane: the bracket of each model
    times the tangential derivative along x (at the xy-edges, where u lives)
    and along z (at the yz-edges, where w lives), each from the two wall
    columns beside the edge;
  * |grad phi| and |grad psi| of the B models include the other tangential
    component (its central difference averaged over the same two columns);
  * kappa_p = kappa + t_q . (grad grad psi) t_q, t_q = n_phi x n_wall / |.|
    the direction along the contact line: the energy-based curvature with
    the out-of-plane normal curvature removed, i.e. the two-dimensional
    curvature of the paper's eq. curvature taken in the plane of n_phi and
    n_wall.  With n_wall = y, t_q = (-psi_z, 0, psi_x)/|.|; the denominator
    carries DELTA_T^2 so that a column with no tangential gradient (no
    contact line) takes kappa_p = kappa.  A z-invariant field gives
    kappa_p = kappa exactly, the paper's two-dimensional value;
  * viscous stress mu (grad u + grad u^T) with edge viscosities the mean of
    the four cells around the edge; advection of the mass flux m by face and
    edge means, as in two dimensions.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .cdi import DELTA_N, RK_B, RK_C, psi_of

DELTA_T = 1e-12    # regularises |t_q| where the tangential gradient of psi vanishes


def _rx(q, s):
    return np.roll(q, s, axis=-1)


def _rz(q, s):
    return np.roll(q, s, axis=0)


# ---------------------------------------------------------------------------
# cell-centred differences: central in x and z (periodic), central in y in
# the interior and second-order one-sided on the first and last cell rows.
# ---------------------------------------------------------------------------

def ddx(q, h):
    return (_rx(q, -1) - _rx(q, 1)) / (2.0 * h)


def ddz(q, h):
    return (_rz(q, -1) - _rz(q, 1)) / (2.0 * h)


def ddy(q, h):
    out = np.empty_like(q)
    out[:, 1:-1] = (q[:, 2:] - q[:, :-2]) / (2.0 * h)
    out[:, 0] = (-3.0 * q[:, 0] + 4.0 * q[:, 1] - q[:, 2]) / (2.0 * h)
    out[:, -1] = (3.0 * q[:, -1] - 4.0 * q[:, -2] + q[:, -3]) / (2.0 * h)
    return out


def d2dx2(q, h):
    return (_rx(q, -1) - 2.0 * q + _rx(q, 1)) / (h * h)


def d2dz2(q, h):
    return (_rz(q, -1) - 2.0 * q + _rz(q, 1)) / (h * h)


def d2dy2(q, h):
    out = np.empty_like(q)
    out[:, 1:-1] = (q[:, 2:] - 2.0 * q[:, 1:-1] + q[:, :-2]) / (h * h)
    out[:, 0] = (2.0 * q[:, 0] - 5.0 * q[:, 1] + 4.0 * q[:, 2] - q[:, 3]) / (h * h)
    out[:, -1] = (2.0 * q[:, -1] - 5.0 * q[:, -2] + 4.0 * q[:, -3] - q[:, -4]) / (h * h)
    return out


def d2dxdz(q, h):
    return (_rz(_rx(q, -1), -1) - _rz(_rx(q, 1), -1) - _rz(_rx(q, -1), 1)
            + _rz(_rx(q, 1), 1)) / (4.0 * h * h)


# ---------------------------------------------------------------------------
# phase-field quantities (Sec. 2)
# ---------------------------------------------------------------------------

def normal(phi, h):
    """n = grad(phi) / (|grad(phi)| + DELTA_N), three components."""
    gx, gy, gz = ddx(phi, h), ddy(phi, h), ddz(phi, h)
    mag = np.sqrt(gx * gx + gy * gy + gz * gz) + DELTA_N
    return gx / mag, gy / mag, gz / mag


def psi_derivatives(psi, h):
    """(psi_x, psi_y, psi_z, laplacian psi) with the wall-row stencils."""
    return ddx(psi, h), ddy(psi, h), ddz(psi, h), d2dx2(psi, h) + d2dy2(psi, h) + d2dz2(psi, h)


def curvature(phi, px, py, pz, lap, eps):
    """Energy-based curvature (eq. curvature) in three dimensions: the sum of
    the principal curvatures, (1 - 2 phi)(1 - |grad psi|^2)/eps - lap psi."""
    return (1.0 - 2.0 * phi) * (1.0 - px * px - py * py - pz * pz) / eps - lap


def chemical_potential(phi, px, py, pz, lap, eps, sigma):
    g = phi * (1.0 - phi)
    return 6.0 * sigma * (g * (1.0 - 2.0 * phi) * (1.0 - px * px - py * py - pz * pz) / eps
                          - g * lap)


def contact_line_curvature(psi, px, pz, h):
    """t_q . (grad grad psi) t_q with t_q = (-psi_z, 0, psi_x)/|.|, the normal
    curvature term of psi along the contact-line direction (walls normal to
    y): (psi_z^2 psi_xx - 2 psi_x psi_z psi_xz + psi_x^2 psi_zz)/(psi_x^2 +
    psi_z^2 + DELTA_T^2)."""
    pxx, pzz, pxz = d2dx2(psi, h), d2dz2(psi, h), d2dxdz(psi, h)
    return ((pz * pz * pxx - 2.0 * px * pz * pxz + px * px * pzz)
            / (px * px + pz * pz + DELTA_T * DELTA_T))


def inplane_curvature(phi, psi, h, eps):
    """kappa_p: the energy-based curvature in the plane containing n_phi and
    n_wall (Sec. 2; Sec. 3.1.2 curvature correction)."""
    px, py, pz, lap = psi_derivatives(psi, h)
    return curvature(phi, px, py, pz, lap, eps) + contact_line_curvature(psi, px, pz, h)


def phase_fields(phi, p) -> Dict[str, np.ndarray]:
    h, eps = p.h, p.eps
    nxv, nyv, nzv = normal(phi, h)
    psi = psi_of(phi, eps)
    px, py, pz, lap = psi_derivatives(psi, h)
    kap = curvature(phi, px, py, pz, lap, eps)
    kp = kap + contact_line_curvature(psi, px, pz, h)
    muc = chemical_potential(phi, px, py, pz, lap, eps, p.sigma)
    return dict(nx=nxv, ny=nyv, nz=nzv, psi=psi, psix=px, psiy=py, psiz=pz, lap=lap,
                kappa=kap, kappa_p=kp, muc=muc, phiy=ddy(phi, h))


# ---------------------------------------------------------------------------
# wall slip (Sec. 2 slip BC, Sec. 3 Models 1A..4B, Sec. 4 extrapolation)
# ---------------------------------------------------------------------------

def _extrap(q, wall):
    """Linear extrapolation of a cell field to the wall, per (k, i) column."""
    if wall == "bot":
        return 0.5 * (3.0 * q[:, 0] - q[:, 1])
    return 0.5 * (3.0 * q[:, -1] - q[:, -2])


def _model_uY(model, p, phc, psc, kac, dpsi_n, dpsi_t, dpsi_o, dphi_n, dphi_t, dphi_o):
    eps = p.eps
    g = phc * (1.0 - phc)
    beta = p.beta2 + (p.beta1 - p.beta2) * phc
    ce = math.cos(p.theta_eq)
    corr = 1.0 + kac * psc
    gradphi = np.sqrt(dphi_n ** 2 + dphi_t ** 2 + dphi_o ** 2)
    gradpsi = np.sqrt(dpsi_n ** 2 + dpsi_t ** 2 + dpsi_o ** 2)
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
    return uY, beta


def slip_velocity_Y(phi, p, wall, model=None, fields=None) -> Dict[str, np.ndarray]:
    """Young slip at one wall: uYx at the wall's xy-edges (k, i) and uYz at its
    yz-edges (k, i), both (nz, nx).  Wall quantities (phi, psi, d psi/dy,
    kappa_p, d phi/dy) are extrapolated per column from the first two cell
    rows (Sec. 4) and averaged to each edge from the two columns beside it;
    the normal derivative is along the inward normal, the tangential ones
    along +x and +z."""
    model = model or p.slip_model
    h = p.h
    if fields is None:
        fields = phase_fields(phi, p)
    sgn = 1.0 if wall == "bot" else -1.0
    phw = _extrap(phi, wall)
    psw = _extrap(fields["psi"], wall)
    dpsw = _extrap(fields["psiy"], wall)
    kpw = _extrap(fields["kappa_p"], wall)
    dphw = _extrap(fields["phiy"], wall)

    def avx(q):   # to the xy-edge between columns i-1 and i
        return 0.5 * (np.roll(q, 1, axis=1) + q)

    def avz(q):   # to the yz-edge between columns k-1 and k
        return 0.5 * (np.roll(q, 1, axis=0) + q)

    def cx(q):
        return (np.roll(q, -1, axis=1) - np.roll(q, 1, axis=1)) / (2.0 * h)

    def cz(q):
        return (np.roll(q, -1, axis=0) - np.roll(q, 1, axis=0)) / (2.0 * h)

    out = {"phi_w": phw}
    for comp, av, dt, other in (("x", avx, lambda q: (q - np.roll(q, 1, axis=1)) / h, cz),
                                ("z", avz, lambda q: (q - np.roll(q, 1, axis=0)) / h, cx)):
        phc = np.clip(av(phw), 0.0, 1.0)
        uY, beta = _model_uY(model, p, phc, av(psw), av(kpw), sgn * av(dpsw), dt(psw),
                             av(other(psw)), sgn * av(dphw), dt(phw), av(other(phw)))
        out[f"phi_{comp}"] = phc
        out[f"beta_{comp}"] = beta
        out[f"uY{comp}"] = uY
    return out


def wall_stress(phi, u, w, p, fields) -> Dict[str, Dict[str, np.ndarray]]:
    """GNBC wall velocity and shear stress of both tangential components at
    both walls: u_slip = (mu/beta) du_tau/dn + u^Y with du_tau/dn = 2 (first
    row - wall value)/h, solved for the wall value (as in two dimensions)."""
    h = p.h
    out = {}
    for wall, r, Ux, Uz in (("bot", 0, p.u_wall_bot, p.w_wall_bot),
                            ("top", -1, p.u_wall_top, p.w_wall_top)):
        s = slip_velocity_Y(phi, p, wall, fields=fields)
        for comp, row, U in (("x", u[:, r], Ux), ("z", w[:, r], Uz)):
            mu_w = p.mu2 + (p.mu1 - p.mu2) * s[f"phi_{comp}"]
            lam = 2.0 * mu_w / (s[f"beta_{comp}"] * h)
            uw = (U + s[f"uY{comp}"] + lam * row) / (1.0 + lam)
            tau = 2.0 * mu_w * (row - uw) / h if wall == "bot" else 2.0 * mu_w * (uw - row) / h
            s[f"wall_{comp}"] = uw
            s[f"tau_{comp}"] = tau
            s[f"slip_{comp}"] = uw - U
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
    """Face densities: x-faces, y-faces (wall rows nan), z-faces."""
    rho = rho_of(phi, p)
    nz, ny, nx = phi.shape
    rfy = np.full((nz, ny + 1, nx), np.nan)
    rfy[:, 1:ny] = 0.5 * (rho[:, :-1] + rho[:, 1:])
    return 0.5 * (_rx(rho, 1) + rho), rfy, 0.5 * (_rz(rho, 1) + rho)


def phi_fluxes(phi, u, v, w, f, p):
    """CDI face fluxes F = u phi_f - gamma[eps dphi/dn_f - phi_f(1 - phi_f) n_f]
    on x-, y- and z-faces (eq. CDI); the wall y-faces carry F = 0."""
    h, eps, gam = p.h, p.eps, p.gamma
    nz, ny, nx = phi.shape
    phL = _rx(phi, 1)
    phf = 0.5 * (phL + phi)
    nf = 0.5 * (_rx(f["nx"], 1) + f["nx"])
    Fx = u * phf - gam * (eps * (phi - phL) / h - phf * (1.0 - phf) * nf)
    Fy = np.zeros((nz, ny + 1, nx))
    phb, pht = phi[:, :-1], phi[:, 1:]
    phfy = 0.5 * (phb + pht)
    nfy = 0.5 * (f["ny"][:, :-1] + f["ny"][:, 1:])
    Fy[:, 1:ny] = v[:, 1:ny] * phfy - gam * (eps * (pht - phb) / h - phfy * (1.0 - phfy) * nfy)
    phB = _rz(phi, 1)
    phfz = 0.5 * (phB + phi)
    nfz = 0.5 * (_rz(f["nz"], 1) + f["nz"])
    Fz = w * phfz - gam * (eps * (phi - phB) / h - phfz * (1.0 - phfz) * nfz)
    return Fx, Fy, Fz


def stage_rhs(phi, u, v, w, p):
    """L(phi, u, v, w) -> (L_phi, L_mx, L_my, L_mz, wall dict): right-hand sides
    of the CDI equation and of the three momentum components (eq.
    NS_momentum without the pressure gradient)."""
    h = p.h
    nz, ny, nx = phi.shape
    f = phase_fields(phi, p)
    Fx, Fy, Fz = phi_fluxes(phi, u, v, w, f, p)
    Lphi = -((_rx(Fx, -1) - Fx) + (Fy[:, 1:] - Fy[:, :-1]) + (_rz(Fz, -1) - Fz)) / h

    drho = p.rho1 - p.rho2
    mx = p.rho2 * u + drho * Fx
    my = p.rho2 * v + drho * Fy            # zero on both walls
    mz = p.rho2 * w + drho * Fz
    mu = mu_of(phi, p)
    muc = f["muc"]
    walls = wall_stress(phi, u, w, p, f)

    # ---- shear stresses on the edges
    tauxy = np.zeros((nz, ny + 1, nx))
    mu4 = 0.25 * (mu[:, :-1] + _rx(mu[:, :-1], 1) + mu[:, 1:] + _rx(mu[:, 1:], 1))
    tauxy[:, 1:ny] = mu4 * ((u[:, 1:] - u[:, :-1]) / h + (v[:, 1:ny] - _rx(v[:, 1:ny], 1)) / h)
    tauxy[:, 0] = walls["bot"]["tau_x"]
    tauxy[:, ny] = walls["top"]["tau_x"]
    tauyz = np.zeros((nz, ny + 1, nx))
    mu4 = 0.25 * (mu[:, :-1] + _rz(mu[:, :-1], 1) + mu[:, 1:] + _rz(mu[:, 1:], 1))
    tauyz[:, 1:ny] = mu4 * ((w[:, 1:] - w[:, :-1]) / h + (v[:, 1:ny] - _rz(v[:, 1:ny], 1)) / h)
    tauyz[:, 0] = walls["bot"]["tau_z"]
    tauyz[:, ny] = walls["top"]["tau_z"]
    mu4 = 0.25 * (mu + _rx(mu, 1) + _rz(mu, 1) + _rz(_rx(mu, 1), 1))
    tauxz = mu4 * ((u - _rz(u, 1)) / h + (w - _rx(w, 1)) / h)

    # ---- x-momentum at u (k, j, i)
    fc = 0.5 * (mx + _rx(mx, -1)) * 0.5 * (u + _rx(u, -1))                   # cell
    fcy = np.zeros((nz, ny + 1, nx))                                          # xy-edge
    fcy[:, 1:ny] = 0.5 * (_rx(my[:, 1:ny], 1) + my[:, 1:ny]) * 0.5 * (u[:, :-1] + u[:, 1:])
    fcz = 0.5 * (_rx(mz, 1) + mz) * 0.5 * (_rz(u, 1) + u)                     # xz-edge
    tauxx = 2.0 * mu * (_rx(u, -1) - u) / h
    stx = 0.5 * (_rx(muc, 1) + muc) * (phi - _rx(phi, 1)) / h
    Lmx = (-((fc - _rx(fc, 1)) + (fcy[:, 1:] - fcy[:, :-1]) + (_rz(fcz, -1) - fcz)) / h
           + (tauxx - _rx(tauxx, 1)) / h
           + (tauxy[:, 1:] - tauxy[:, :-1]) / h
           + (_rz(tauxz, -1) - tauxz) / h
           + stx)

    # ---- y-momentum at interior v (k, j, i), j = 1..ny-1
    gc = 0.5 * (my[:, :-1] + my[:, 1:]) * 0.5 * (v[:, :-1] + v[:, 1:])       # cell
    fcx = 0.5 * (mx[:, :-1] + mx[:, 1:]) * 0.5 * (_rx(v[:, 1:ny], 1) + v[:, 1:ny])   # xy-edge
    fcz2 = 0.5 * (mz[:, :-1] + mz[:, 1:]) * 0.5 * (_rz(v[:, 1:ny], 1) + v[:, 1:ny])  # yz-edge
    tauyy = 2.0 * mu * (v[:, 1:] - v[:, :-1]) / h
    sty = 0.5 * (muc[:, :-1] + muc[:, 1:]) * (phi[:, 1:] - phi[:, :-1]) / h
    Lmy = np.zeros((nz, ny + 1, nx))
    Lmy[:, 1:ny] = (-((_rx(fcx, -1) - fcx) + (gc[:, 1:] - gc[:, :-1]) + (_rz(fcz2, -1) - fcz2)) / h
                    + (tauyy[:, 1:] - tauyy[:, :-1]) / h
                    + (_rx(tauxy[:, 1:ny], -1) - tauxy[:, 1:ny]) / h
                    + (_rz(tauyz[:, 1:ny], -1) - tauyz[:, 1:ny]) / h
                    + sty)

    # ---- z-momentum at w (k, j, i)
    gz = 0.5 * (mz + _rz(mz, -1)) * 0.5 * (w + _rz(w, -1))                   # cell
    fxz = 0.5 * (_rz(mx, 1) + mx) * 0.5 * (_rx(w, 1) + w)                     # xz-edge
    fyz = np.zeros((nz, ny + 1, nx))                                          # yz-edge
    fyz[:, 1:ny] = 0.5 * (_rz(my[:, 1:ny], 1) + my[:, 1:ny]) * 0.5 * (w[:, :-1] + w[:, 1:])
    tauzz = 2.0 * mu * (_rz(w, -1) - w) / h
    stz = 0.5 * (_rz(muc, 1) + muc) * (phi - _rz(phi, 1)) / h
    Lmz = (-((_rx(fxz, -1) - fxz) + (fyz[:, 1:] - fyz[:, :-1]) + (gz - _rz(gz, 1))) / h
           + (tauzz - _rz(tauzz, 1)) / h
           + (_rx(tauxz, -1) - tauxz) / h
           + (tauyz[:, 1:] - tauyz[:, :-1]) / h
           + stz)
    return Lphi, Lmx, Lmy, Lmz, walls


# ---------------------------------------------------------------------------
# projection (the two-dimensional operator of oracle.poisson with z faces)
# ---------------------------------------------------------------------------

def divergence(u, v, w, h):
    return ((_rx(u, -1) - u) + (v[:, 1:] - v[:, :-1]) + (_rz(w, -1) - w)) / h


def assemble_A(rfx, rfy, rfz, h) -> sp.csr_matrix:
    """A p = sum over a cell's non-wall faces of (p_nb - p)/(rho_f h^2), cell
    index (k ny + j) nx + i; x and z periodic, wall faces omitted."""
    nz, ny, nx = rfx.shape
    cell = np.arange(nx * ny * nz).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []

    def couple(a, b, c):
        a, b, c = a.reshape(-1), b.reshape(-1), c.reshape(-1)
        rows.extend([a, b, a, b])
        cols.extend([b, a, a, b])
        vals.extend([c, c, -c, -c])

    couple(cell, _rx(cell, 1), 1.0 / rfx)
    couple(cell[:, 1:], cell[:, :-1], 1.0 / rfy[:, 1:ny])
    couple(cell, _rz(cell, 1), 1.0 / rfz)
    n = nx * ny * nz
    return sp.coo_matrix((np.concatenate(vals) / (h * h),
                          (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsr()


def apply_A(pr, rfx, rfy, rfz, h):
    nz, ny, nx = pr.shape
    fx = (pr - _rx(pr, 1)) / rfx
    fy = np.zeros((nz, ny + 1, nx))
    fy[:, 1:ny] = (pr[:, 1:] - pr[:, :-1]) / rfy[:, 1:ny]
    fz = (pr - _rz(pr, 1)) / rfz
    return ((_rx(fx, -1) - fx) + (fy[:, 1:] - fy[:, :-1]) + (_rz(fz, -1) - fz)) / (h * h)


def solve_pressure(b, rfx, rfy, rfz, h):
    """Exact solve of A p = b (b mean-free) by sparse LU with one cell pinned,
    then the mean removed."""
    A = assemble_A(rfx, rfy, rfz, h).tolil()
    A[0, :] = 0.0
    A[0, 0] = 1.0
    rhs = b.reshape(-1).copy()
    rhs[0] = 0.0
    pr = spla.splu(A.tocsc()).solve(rhs).reshape(b.shape)
    return pr - pr.mean()


def project(us, vs, ws, phi, tau, p):
    h = p.h
    rfx, rfy, rfz = face_rho(phi, p)
    b = divergence(us, vs, ws, h) / tau
    b = b - b.mean()
    pr = solve_pressure(b, rfx, rfy, rfz, h)
    u = us - tau * (pr - _rx(pr, 1)) / (h * rfx)
    v = vs.copy()
    v[:, 1:-1] = vs[:, 1:-1] - tau * (pr[:, 1:] - pr[:, :-1]) / (h * rfy[:, 1:-1])
    v[:, 0] = 0.0
    v[:, -1] = 0.0
    w = ws - tau * (pr - _rz(pr, 1)) / (h * rfz)
    return u, v, w, pr


# ---------------------------------------------------------------------------
# time step (RK4 with a projection after every stage and the final combine)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class State3:
    phi: np.ndarray
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    p: np.ndarray
    t: float = 0.0
    step: int = 0


def initial_state(phi0) -> State3:
    nz, ny, nx = phi0.shape
    z = np.zeros((nz, ny, nx))
    return State3(phi0.astype(np.float64).copy(), z.copy(), np.zeros((nz, ny + 1, nx)), z.copy(),
                  z.copy())


def step_gamma(u, v, w, p) -> float:
    f = getattr(p, "gamma_factor", 0.0)
    if f <= 0.0:
        return p.gamma
    return min(p.gamma, f * max(float(np.abs(u).max()), float(np.abs(v).max()),
                                float(np.abs(w).max())))


def _momentum_to_velocity(mx, my, mz, phi, p):
    rfx, rfy, rfz = face_rho(phi, p)
    v = np.zeros_like(my)
    v[:, 1:-1] = my[:, 1:-1] / rfy[:, 1:-1]
    return mx / rfx, v, mz / rfz


def step(s: State3, p) -> State3:
    if getattr(p, "gamma_factor", 0.0) > 0.0:
        p = p.replace(gamma=step_gamma(s.u, s.v, s.w, p), gamma_factor=0.0)
    dt = p.dt
    phi0 = s.phi
    rfx0, rfy0, rfz0 = face_rho(phi0, p)
    mx0 = rfx0 * s.u
    my0 = np.zeros_like(s.v)
    my0[:, 1:-1] = rfy0[:, 1:-1] * s.v[:, 1:-1]
    mz0 = rfz0 * s.w
    ph, uu, vv, ww, pr = phi0, s.u, s.v, s.w, s.p
    acc = None
    for k in range(4):
        L = stage_rhs(ph, uu, vv, ww, p)[:4]
        acc = [RK_B[0] * q for q in L] if k == 0 else [a + RK_B[k] * q for a, q in zip(acc, L)]
        if k < 3:
            c = RK_C[k + 1] * dt
            ph = phi0 + c * L[0]
            uu, vv, ww = _momentum_to_velocity(mx0 + c * L[1], my0 + c * L[2], mz0 + c * L[3], ph, p)
            uu, vv, ww, pr = project(uu, vv, ww, ph, c, p)
    ph = phi0 + dt * acc[0]
    uu, vv, ww = _momentum_to_velocity(mx0 + dt * acc[1], my0 + dt * acc[2], mz0 + dt * acc[3], ph, p)
    uu, vv, ww, pr = project(uu, vv, ww, ph, dt, p)
    return State3(ph, uu, vv, ww, pr, s.t + dt, s.step + 1)


def run(phi0, p, steps: int) -> State3:
    s = initial_state(phi0)
    for _ in range(steps):
        s = step(s, p)
    return s


def diagnostics(s: State3, p) -> Dict[str, float]:
    h = p.h
    f = phase_fields(s.phi, p)
    walls = wall_stress(s.phi, s.u, s.w, p, f)
    rfx, rfy, rfz = face_rho(s.phi, p)
    ke = 0.5 * h ** 3 * (np.sum(rfx * s.u ** 2) + np.sum(rfy[:, 1:-1] * s.v[:, 1:-1] ** 2)
                         + np.sum(rfz * s.w ** 2))
    return dict(mass=float(np.sum(s.phi) * h ** 3), phi_min=float(s.phi.min()),
                phi_max=float(s.phi.max()),
                max_div=float(np.max(np.abs(divergence(s.u, s.v, s.w, h)))),
                max_slip_bot=float(max(np.abs(walls["bot"]["slip_x"]).max(),
                                       np.abs(walls["bot"]["slip_z"]).max())),
                max_uY_bot=float(max(np.abs(walls["bot"]["uYx"]).max(),
                                     np.abs(walls["bot"]["uYz"]).max())),
                ke=float(ke))
