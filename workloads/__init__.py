"""Seeded synthetic workloads of the CDI + GNBC time step.

This module holds the problem set-up only: physical parameters, the time-step
rule, the paper's prescribed initial phase fields and the seeded ensemble draw.
It contains none of the method's arithmetic (no stencil, no flux, no slip
model, no pressure solve), so that both the CPU oracle and the HIP product
path can take their inputs from here without sharing any code of the method.

Initial fields:
  * equilibrium drop on the bottom wall -- the prescribed equilibrium phase
    field of Sec. 3.1 (eq. "prescribed phase field"), with the equal-area
    radius read as R = sqrt(A0 / (theta - sin(theta) cos(theta))) (the printed
    formula is garbled; this reading keeps the drop area that the text
    requires for every theta);
  * two-phase Couette slab -- the initial phase field of Sec. 5.2
    (eq. "couette flow initial phi"), fluid 1 in [Lx/4, 3Lx/4].
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

# slip-model identifiers (Sec. 3, eqs. Model 1A ... Model 4B)
SLIP_MODELS = ("1A", "1B", "2A", "2B", "3A", "3B", "4A", "4B")


@dataclasses.dataclass
class Params:
    """Physical and numerical parameters of one CDI + GNBC problem.

    Names follow the paper: phi = 1 is fluid 1 (Sec. 2), eps the interface
    thickness, gamma the regularisation velocity scale, sigma the surface
    tension, theta_eq the equilibrium contact angle measured inside fluid 1
    (radians), beta1/beta2 the wall friction of each fluid (Sec. 2, slip BC),
    u_wall_bot/u_wall_top the tangential wall speeds (+x).  gamma_factor > 0
    selects the paper's velocity-dependent regularisation (Sec. 5: gamma =
    2.5 |u|_max): each step takes min(gamma, gamma_factor * max |u|, |v|).
    """
    nx: int
    ny: int
    lx: float
    ly: float
    eps: float
    gamma: float
    sigma: float
    theta_eq: float
    rho1: float
    rho2: float
    mu1: float
    mu2: float
    beta1: float
    beta2: float
    u_wall_bot: float = 0.0
    u_wall_top: float = 0.0
    dt: float = 0.0
    slip_model: str = "4A"
    gamma_factor: float = 0.0   # > 0: gamma of a step = min(gamma, factor * max|u|)

    @property
    def h(self) -> float:
        return self.lx / self.nx

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)


def dt_from_cfl(p: Params, cfl: float = 0.2) -> float:
    """Fixed time step: cfl * min(advective, viscous, capillary, CDI-diffusive).

    advective  h / max|U_wall|          (skipped when both walls are at rest)
    viscous    h^2 / max(mu1/rho1, mu2/rho2)
    capillary  sqrt((rho1 + rho2) h^3 / (4 pi sigma))  (skipped when sigma = 0)
    diffusive  h^2 / (gamma eps)
    """
    h = p.h
    lim = []
    uw = max(abs(p.u_wall_bot), abs(p.u_wall_top))
    if uw > 0:
        lim.append(h / uw)
    nu = max(p.mu1 / p.rho1, p.mu2 / p.rho2)
    if nu > 0:
        lim.append(h * h / nu)
    if p.sigma > 0:
        lim.append(math.sqrt((p.rho1 + p.rho2) * h ** 3 / (4.0 * math.pi * p.sigma)))
    if p.gamma * p.eps > 0:
        lim.append(h * h / (p.gamma * p.eps))
    return cfl * min(lim)


def cell_centres(nx: int, ny: int, h: float) -> Tuple[np.ndarray, np.ndarray]:
    """(X, Y) of cell centres, arrays of shape (ny, nx), x fastest."""
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    return np.meshgrid(x, y)


def equal_area_radius(r0: float, theta: float) -> float:
    """Radius of a circular cap with contact angle theta and the area of a
    half disc of radius r0 (Sec. 3.1, equal-area reading)."""
    a0 = 0.5 * math.pi * r0 * r0
    return math.sqrt(a0 / (theta - math.sin(theta) * math.cos(theta)))


def drop_phi(nx: int, ny: int, lx: float, ly: float, r0: float, theta: float,
             eps: float, xc: float | None = None) -> np.ndarray:
    """Prescribed equilibrium drop (Sec. 3.1): tanh profile of a circle of
    radius R centred at (xc, -R cos(theta)), sampled at cell centres."""
    h = lx / nx
    X, Y = cell_centres(nx, ny, h)
    R = equal_area_radius(r0, theta)
    if xc is None:
        xc = lx / 2.0
    yc = -R * math.cos(theta)
    r = np.sqrt((X - xc) ** 2 + (Y - yc) ** 2)
    return 0.5 * (1.0 + np.tanh((R - r) / (2.0 * eps)))


def couette_phi(nx: int, ny: int, lx: float, ly: float, eps: float) -> np.ndarray:
    """Two-phase Couette slab (Sec. 5.2): fluid 1 between Lx/4 and 3Lx/4."""
    h = lx / nx
    X, _ = cell_centres(nx, ny, h)
    return (0.5 * (1.0 + np.tanh((X - lx / 4.0) / (2.0 * eps)))
            + 0.5 * (1.0 + np.tanh((3.0 * lx / 4.0 - X) / (2.0 * eps))) - 1.0)


@dataclasses.dataclass
class Case:
    name: str
    params: Params
    phi0: np.ndarray
    steps: int
    kind: str  # "drop" | "couette"
    r0: float = 0.0


def _finish(name, p, phi0, steps, kind, r0=0.0, dt=None) -> Case:
    p = p.replace(dt=dt if dt is not None else dt_from_cfl(p))
    return Case(name, p, np.ascontiguousarray(phi0, dtype=np.float64), steps, kind, r0)


def drop_case(nx: int, ny: int, theta_eq_deg: float = 60.0, ratio: float = 1.0,
              lx: float = 2.0, ly: float = 1.0, r0: float = 0.3, steps: int = 500,
              name: str | None = None) -> Case:
    """Equilibrium drop: semicircle (90 deg) relaxing to theta_eq.

    ratio = 1: rho = mu = 0.01 (Sec. 5.1 constants); ratio r: fluid 1 (the
    drop) has rho1 = mu1 = 0.01 r, fluid 2 keeps 0.01.  sigma = 1, beta = 10,
    eps = h, gamma = 1.
    """
    h = lx / nx
    p = Params(nx=nx, ny=ny, lx=lx, ly=ly, eps=h, gamma=1.0, sigma=1.0,
               theta_eq=math.radians(theta_eq_deg), rho1=0.01 * ratio, rho2=0.01,
               mu1=0.01 * ratio, mu2=0.01, beta1=10.0, beta2=10.0)
    phi0 = drop_phi(nx, ny, lx, ly, r0, math.pi / 2, p.eps)
    return _finish(name or f"drop{nx}x{ny}", p, phi0, steps, "drop", r0)


def couette_case(nx: int, ny: int, lx: float = 4.0, ly: float = 1.0, ratio: float = 1.0,
                 ca: float = 0.1, slip_length: float = 0.02, theta_eq_deg: float = 90.0,
                 u_wall: float = 1.0, steps: int = 4000, name: str | None = None) -> Case:
    """Two-phase Couette flow: walls at -U (bottom) and +U (top).

    rho2 = mu2 = 1, fluid 1 scaled by `ratio`; sigma = mu2 U / Ca;
    beta = mu2 / slip_length (both fluids); eps = h; gamma = 2.5 U.
    """
    h = lx / nx
    mu2 = 1.0
    p = Params(nx=nx, ny=ny, lx=lx, ly=ly, eps=h, gamma=2.5 * abs(u_wall),
               sigma=mu2 * abs(u_wall) / ca, theta_eq=math.radians(theta_eq_deg),
               rho1=1.0 * ratio, rho2=1.0, mu1=mu2 * ratio, mu2=mu2,
               beta1=mu2 / slip_length, beta2=mu2 / slip_length,
               u_wall_bot=-u_wall, u_wall_top=u_wall)
    phi0 = couette_phi(nx, ny, lx, ly, p.eps)
    return _finish(name or f"couette{nx}x{ny}", p, phi0, steps, "couette")


def paper_couette_case(variant: str = "asymmetric", nx: int = 512, steps: int = 2000,
                       name: str | None = None) -> Case:
    """The two-phase Couette flow of Sec. 5.2 in the molecular-dynamics units
    it is stated in: domain 108.8 x 13.6 (Ny = Nx / 8), rho = 0.81, mu = 1.95
    for both fluids, sigma = 5.5, eps = 0.33 sqrt(2)/2, gamma = 2.5 U, top wall
    at +U and bottom wall at -U, the slab of fluid 1 in [Lx/4, 3Lx/4].

    symmetric: theta_eq = 90 deg, beta1 = beta2 = 1.2, U = 0.25;
    asymmetric: theta_eq = acos(0.38), beta1 = 1.2, beta2 = 0.591, U = 0.20.
    """
    if nx % 8:
        raise ValueError("Nx must be a multiple of 8 (Lx / Ly = 8)")
    if variant == "symmetric":
        theta, b1, b2, U = math.pi / 2, 1.2, 1.2, 0.25
    elif variant == "asymmetric":
        theta, b1, b2, U = math.acos(0.38), 1.2, 0.591, 0.20
    else:
        raise ValueError(variant)
    lx, ly = 108.8, 13.6
    eps = 0.33 * math.sqrt(2.0) / 2.0
    p = Params(nx=nx, ny=nx // 8, lx=lx, ly=ly, eps=eps, gamma=2.5 * U, sigma=5.5,
               theta_eq=theta, rho1=0.81, rho2=0.81, mu1=1.95, mu2=1.95, beta1=b1, beta2=b2,
               u_wall_bot=-U, u_wall_top=U)
    phi0 = couette_phi(nx, nx // 8, lx, ly, eps)
    return _finish(name or f"couette_{variant}{nx}x{nx // 8}", p, phi0, steps, "couette")


def config1() -> Case:
    """2D equilibrium drop, 64x32 on 2x1, theta 90 -> 60 deg, 500 steps (FP64)."""
    return drop_case(64, 32, 60.0, 1.0, steps=500, name="drop64x32")


def config2() -> Case:
    """2D two-phase Couette, 256x64 on 4x1, U = +-1, Ca = 0.1, l_s = 0.02, 4000 steps (FP64)."""
    return couette_case(256, 64, steps=4000, name="couette256x64")


def config3(theta_eq_deg: float = 60.0, nx: int = 1024, steps: int = 20000) -> Case:
    """2D equilibrium drop, 1024x512, density/viscosity ratio 10 (mixed precision)."""
    return drop_case(nx, nx // 2, theta_eq_deg, 10.0, steps=steps,
                     name=f"drop{nx}x{nx // 2}_r10_th{int(theta_eq_deg)}")


CONFIG3_THETAS = (30.0, 60.0, 120.0, 150.0)


def config4(seed: int = 20241216, n: int = 64, steps: int = 1000) -> List[Case]:
    """Seeded ensemble of uneven drop / Couette instances (2x1 domains).

    Nx uniform in {128, 160, ..., 512}, Ny = Nx/2; theta_eq ~ U[30, 150] deg;
    Ca ~ logU[0.01, 0.2]; density (= viscosity) ratio in {1, 10} on fluid 1.
    Drops: rho2 = mu2 = 0.01, sigma = mu2 / Ca, beta = 10, gamma = 1.
    Couette: slab [0.5, 1.5], U = +-1, rho2 = mu2 = 1, sigma = mu2 U / Ca,
    beta = mu2 / 0.02, gamma = 2.5.
    """
    rng = np.random.default_rng(seed)
    cases = []
    sizes = np.arange(128, 513, 32)
    for k in range(n):
        kind = "drop" if rng.random() < 0.5 else "couette"
        nx = int(rng.choice(sizes))
        ny = nx // 2
        th = float(rng.uniform(30.0, 150.0))
        ca = float(math.exp(rng.uniform(math.log(0.01), math.log(0.2))))
        ratio = float(rng.choice([1.0, 10.0]))
        if kind == "drop":
            c = drop_case(nx, ny, th, ratio, steps=steps, name=f"ens{k:02d}_drop{nx}")
            p = c.params.replace(sigma=c.params.mu2 / ca)
            cases.append(_finish(c.name, p, c.phi0, steps, "drop", c.r0))
        else:
            c = couette_case(nx, ny, lx=2.0, ly=1.0, ratio=ratio, ca=ca, theta_eq_deg=th,
                             steps=steps, name=f"ens{k:02d}_couette{nx}")
            cases.append(c)
    return cases


def config5(kind: str = "drop", nx: int = 2048) -> Case:
    """Learned-guess evaluation grid: 2048x1024 on 2x1, ratio 10."""
    if kind == "drop":
        return drop_case(nx, nx // 2, 60.0, 10.0, steps=200, name=f"drop{nx}x{nx // 2}_r10")
    return couette_case(nx, nx // 2, lx=2.0, ly=1.0, ratio=10.0, steps=200,
                        name=f"couette{nx}x{nx // 2}_r10")


def random_fields(nx: int, ny: int, seed: int, amp: float = 0.1):
    """Seeded smooth-ish random velocity fields (u: (ny, nx), v: (ny+1, nx),
    v = 0 on both walls) used to exercise every stencil in parity tests."""
    rng = np.random.default_rng(seed)
    u = amp * rng.standard_normal((ny, nx))
    v = amp * rng.standard_normal((ny + 1, nx))
    v[0] = 0.0
    v[-1] = 0.0
    return u, v


# ---------------------------------------------------------------------------
# three-dimensional set-up (x and z periodic, walls at y = 0 and y = Ly)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Params3(Params):
    """Parameters of a 3-D problem: those of Params plus the z extent (nz
    cells over lz, the same spacing h as x and y) and the z components of
    the tangential wall speeds."""
    nz: int = 8
    lz: float = 1.0
    w_wall_bot: float = 0.0
    w_wall_top: float = 0.0


def cell_centres3(nx: int, ny: int, nz: int, h: float):
    """(X, Y, Z) of cell centres, arrays of shape (nz, ny, nx), x fastest."""
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    z = (np.arange(nz) + 0.5) * h
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def equal_volume_radius(r0: float, theta: float) -> float:
    """Radius of a spherical cap with contact angle theta and the volume of a
    half ball of radius r0 (the 3-D analogue of the equal-area reading)."""
    c = math.cos(theta)
    return r0 * (2.0 / (2.0 - 3.0 * c + c ** 3)) ** (1.0 / 3.0)


def cap_phi3(nx: int, ny: int, nz: int, h: float, r0: float, theta: float, eps: float,
             xc: float, zc: float) -> np.ndarray:
    """Spherical-cap drop on the bottom wall: tanh profile of a sphere of
    radius R centred at (xc, -R cos(theta), zc), sampled at cell centres."""
    X, Y, Z = cell_centres3(nx, ny, nz, h)
    R = equal_volume_radius(r0, theta)
    r = np.sqrt((X - xc) ** 2 + (Y + R * math.cos(theta)) ** 2 + (Z - zc) ** 2)
    return 0.5 * (1.0 + np.tanh((R - r) / (2.0 * eps)))


def drop3_case(nx: int, ny: int, nz: int, theta_eq_deg: float = 60.0, ratio: float = 1.0,
               r0: float = 0.3, steps: int = 100, h: float | None = None,
               name: str | None = None) -> "Case":
    """Spherical-cap drop relaxing on the bottom wall of a periodic box
    (the 3-D counterpart of drop_case)."""
    h = h if h is not None else 2.0 / nx
    lx, ly, lz = nx * h, ny * h, nz * h
    eps = 0.75 * h
    p = Params3(nx=nx, ny=ny, lx=lx, ly=ly, eps=eps, gamma=1.0, sigma=1.0,
                theta_eq=math.radians(theta_eq_deg), rho1=ratio, rho2=1.0, mu1=0.1, mu2=0.1,
                beta1=10.0, beta2=10.0, nz=nz, lz=lz)
    p = p.replace(dt=dt_from_cfl(p))
    phi0 = cap_phi3(nx, ny, nz, h, r0, math.radians(90.0), eps, lx / 2.0, lz / 2.0)
    return Case(name or f"drop3d{nx}x{ny}x{nz}", p, phi0, steps, "drop3", r0)


def random_fields3(nx: int, ny: int, nz: int, seed: int, amp: float = 0.1):
    """Seeded random velocity fields of a 3-D grid (u, w: (nz, ny, nx); v:
    (nz, ny+1, nx) with v = 0 on both walls) for parity tests."""
    rng = np.random.default_rng(seed)
    u = amp * rng.standard_normal((nz, ny, nx))
    v = amp * rng.standard_normal((nz, ny + 1, nx))
    w = amp * rng.standard_normal((nz, ny, nx))
    v[:, 0] = 0.0
    v[:, -1] = 0.0
    return u, v, w
