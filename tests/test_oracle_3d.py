"""Pins of the three-dimensional oracle (oracle/cdi3d.py).

The 3-D oracle is pinned to things other than itself:
  * a z-invariant field is the paper's two-dimensional setting, so every
    3-D quantity must equal the (already pinned) two-dimensional oracle's on
    each z-slice, with w and L_mz zero and kappa_p = kappa (Sec. 2);
  * swapping x and z (a reflection the continuous problem is invariant
    under) must swap u and w, L_mx and L_mz, the x- and z-slip;
  * closed forms of the in-plane curvature kappa_p (the curvature of the
    interface in the plane containing n_phi and n_wall, Sec. 2 and Sec.
    3.1.2) on exact distance profiles: a sphere (kappa = 2/r, kappa_p = 1/r),
    a cylinder lying along the diagonal of the wall plane (kappa_p = kappa =
    1/r) and a cylinder standing on the wall (kappa = 1/r, kappa_p = 0),
    converging at second order;
  * the projection leaves a discretely divergence-free field; the sparse
    operator equals its matrix-free form; mass is conserved by a step.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import cdi, cdi3d


def _p2(nx=32, ny=16, model="4A", **kw):
    base = dict(nx=nx, ny=ny, lx=2.0, ly=1.0, eps=1.5 * 2.0 / nx, gamma=1.0, sigma=1.0,
                theta_eq=math.radians(60), rho1=10.0, rho2=1.0, mu1=0.2, mu2=0.05,
                beta1=10.0, beta2=5.0, u_wall_bot=0.1, u_wall_top=-0.2, slip_model=model)
    base.update(kw)
    p = W.Params(**base)
    return p.replace(dt=W.dt_from_cfl(p))


def _p3(p2, nz, **kw):
    d = {f: getattr(p2, f) for f in p2.__dataclass_fields__}
    d.update(nz=nz, lz=nz * p2.h)
    d.update(kw)
    return W.Params3(**d)


def _drop2(nx=32, ny=16, theta=75.0, xc=None):
    return W.drop_phi(nx, ny, 2.0, 1.0, 0.35, math.radians(theta), 1.5 * 2.0 / nx, xc=xc)


def _tile(a, nz):
    return np.repeat(a[None], nz, axis=0)


# ------------------------------------------------------------ 2-D reduction
@pytest.mark.parametrize("model", W.SLIP_MODELS)
def test_z_invariant_stage_equals_two_dimensional_oracle(model):
    """With phi, u, v independent of z and w = 0 the 3-D stage operator is the
    2-D one on every slice: L_phi, L_mx, L_my and both walls' x-slip equal,
    L_mz = 0, the z-slip 0 and kappa_p = kappa exactly."""
    p2 = _p2(model=model)
    nz = 3
    p3 = _p3(p2, nz)
    phi = _drop2(xc=0.83)
    u, v = W.random_fields(32, 16, seed=5)
    L2 = cdi.stage_rhs(phi, u, v, p2)
    L3 = cdi3d.stage_rhs(_tile(phi, nz), _tile(u, nz), _tile(v, nz), np.zeros((nz, 16, 32)), p3)
    for a, b in ((L2[0], L3[0]), (L2[1], L3[1]), (L2[2], L3[2])):
        scale = np.abs(a).max()
        assert np.abs(b - a[None]).max() <= 1e-13 * scale
    assert np.abs(L3[3]).max() <= 1e-14 * np.abs(L2[1]).max()
    for wall in ("bot", "top"):
        assert np.allclose(L3[4][wall]["uYx"], L2[3][wall]["uY"][None], rtol=0,
                           atol=1e-14 * max(np.abs(L2[3][wall]["uY"]).max(), 1e-30))
        assert np.all(L3[4][wall]["uYz"] == 0.0)
        assert np.all(L3[4][wall]["slip_z"] == 0.0)
    f3 = cdi3d.phase_fields(_tile(phi, nz), p3)
    assert np.array_equal(f3["kappa_p"], f3["kappa"])
    f2 = cdi.phase_fields(phi, p2)
    assert np.allclose(f3["kappa"], f2["kappa"][None], rtol=1e-13, atol=1e-10)


def test_z_invariant_steps_equal_two_dimensional_steps():
    """Two full RK4 steps (projections included) of a z-invariant drop with
    density ratio 10 agree with the 2-D oracle slice by slice."""
    p2 = _p2(nx=24, ny=12)
    nz = 2
    p3 = _p3(p2, nz)
    phi = _drop2(nx=24, ny=12, xc=0.9)
    s2 = cdi.initial_state(phi)
    s3 = cdi3d.initial_state(_tile(phi, nz))
    for _ in range(2):
        s2 = cdi.step(s2, p2)
        s3 = cdi3d.step(s3, p3)
    for a, b in ((s2.phi, s3.phi), (s2.u, s3.u), (s2.v, s3.v)):
        assert np.abs(b - a[None]).max() <= 1e-12 * max(np.abs(a).max(), 1e-30)
    assert np.abs(s3.w).max() <= 1e-14
    assert np.allclose(s3.p - s3.p.mean(), (s2.p - s2.p.mean())[None], atol=1e-10)


# ---------------------------------------------------------- x <-> z symmetry
@pytest.mark.parametrize("model", ["1B", "3B", "4A", "4B"])
def test_swapping_x_and_z_swaps_the_momentum_components(model):
    """The reflection (x, y, z) -> (z, y, x) maps u <-> w; the operator must
    commute with it: L_mx <-> L_mz, L_phi and L_my transposed, x-slip <->
    z-slip.  A dropped, misplaced or wrongly signed z term fails this."""
    n, ny = 12, 8
    h = 1.0 / n
    p2 = _p2(nx=n, ny=ny, lx=1.0, ly=ny * h, eps=1.5 * h, model=model)
    p3 = _p3(p2, n, u_wall_bot=0.1, w_wall_bot=-0.05, u_wall_top=0.0, w_wall_top=0.0)
    p3t = p3.replace(u_wall_bot=-0.05, w_wall_bot=0.1)
    phi = W.cap_phi3(n, ny, n, h, 0.3, math.radians(70), 1.5 * h, 0.43, 0.61)
    u, v, w = W.random_fields3(n, ny, n, seed=11)
    T = lambda a: np.ascontiguousarray(np.swapaxes(a, 0, 2))
    A = cdi3d.stage_rhs(phi, u, v, w, p3)
    B = cdi3d.stage_rhs(T(phi), T(w), T(v), T(u), p3t)
    for a, b in ((A[0], B[0]), (A[2], B[2]), (A[1], B[3]), (A[3], B[1])):
        assert np.abs(T(a) - b).max() <= 1e-12 * np.abs(a).max()
    for wall in ("bot", "top"):
        for ca, cb in (("uYx", "uYz"), ("uYz", "uYx"), ("tau_x", "tau_z")):
            a, b = A[4][wall][ca], B[4][wall][cb]
            assert np.abs(a.T - b).max() <= 1e-12 * max(np.abs(a).max(), 1e-30)


# -------------------------------------------------- kappa_p closed forms
def _distance_profile(n, dist, eps):
    """phi of an exact distance function psi = dist (positive inside)."""
    return 1.0 / (1.0 + np.exp(-dist / eps))


def _curvature_errors(shape_fn, n, which):
    h = 1.0 / n
    eps = 0.05
    X, Y, Z = W.cell_centres3(n, n, n, h)
    dist, r = shape_fn(X, Y, Z)
    phi = _distance_profile(n, dist, eps)
    psi = cdi.psi_of(phi, eps)
    f = cdi3d.phase_fields(phi, W.Params3(nx=n, ny=n, lx=1.0, ly=1.0, eps=eps, gamma=1, sigma=1,
                                          theta_eq=1.0, rho1=1, rho2=1, mu1=1, mu2=1, beta1=1,
                                          beta2=1, nz=n, lz=1.0))
    tang = np.sqrt(f["psix"] ** 2 + f["psiz"] ** 2)
    # cells near the interface, away from the walls' one-sided rows, with a
    # clear contact-line direction
    sel = (np.abs(dist) < eps) & (tang > 0.3)
    sel[:, :3] = False
    sel[:, -3:] = False
    # away from the periodic seams (a profile need not be periodic)
    sel[:3] = False
    sel[-3:] = False
    sel[:, :, :3] = False
    sel[:, :, -3:] = False
    assert sel.sum() > 20
    out = {}
    for key, exact in which.items():
        out[key] = np.abs(f[key][sel] - exact(r[sel])).max()
    return out


@pytest.mark.parametrize("shape", ["sphere", "diagonal_cylinder", "standing_cylinder"])
def test_inplane_curvature_closed_forms(shape):
    """kappa_p on exact distance profiles: the sphere's in-plane section is a
    great circle (kappa_p = 1/r, kappa = 2/r); a cylinder lying along the
    wall diagonal is straight along the contact line (kappa_p = kappa =
    1/r); a cylinder standing on the wall has straight in-plane sections
    (kappa_p = 0, kappa = 1/r).  Errors fall at second order."""
    R = 0.3
    c = np.array([0.47, 0.52, 0.55])
    if shape == "sphere":
        def fn(X, Y, Z):
            r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
            return R - r, r
        which = {"kappa_p": lambda r: 1.0 / r, "kappa": lambda r: 2.0 / r}
    elif shape == "diagonal_cylinder":
        a = np.array([1.0, 0.0, 1.0]) / math.sqrt(2.0)

        def fn(X, Y, Z):
            d = np.stack([X - c[0], Y - c[1], Z - c[2]])
            along = a[0] * d[0] + a[2] * d[2]
            r = np.sqrt(np.maximum((d ** 2).sum(0) - along ** 2, 0.0))
            return R - r, r
        which = {"kappa_p": lambda r: 1.0 / r, "kappa": lambda r: 1.0 / r}
    else:
        def fn(X, Y, Z):
            r = np.sqrt((X - c[0]) ** 2 + (Z - c[2]) ** 2)
            return R - r, r
        which = {"kappa_p": lambda r: 0.0 * r, "kappa": lambda r: 1.0 / r}
    e1 = _curvature_errors(fn, 32, which)
    e2 = _curvature_errors(fn, 64, which)
    for key in which:
        assert e2[key] < 0.05 * (2.0 / R), (key, e1[key], e2[key])
        assert e1[key] / e2[key] > 3.0, (key, e1[key], e2[key])


def test_kappa_p_with_no_tangential_gradient_is_kappa():
    """A flat film parallel to the wall has no contact-line direction: the
    regularised t_q gives kappa_p = kappa (here 0 up to the profile's
    discretisation)."""
    n = 16
    h = 1.0 / n
    X, Y, Z = W.cell_centres3(n, n, n, h)
    phi = 1.0 / (1.0 + np.exp(-(0.4 - Y) / 0.05))
    p3 = W.Params3(nx=n, ny=n, lx=1.0, ly=1.0, eps=0.05, gamma=1, sigma=1, theta_eq=1.0,
                   rho1=1, rho2=1, mu1=1, mu2=1, beta1=1, beta2=1, nz=n, lz=1.0)
    f = cdi3d.phase_fields(phi, p3)
    assert np.array_equal(f["kappa_p"], f["kappa"])


# ------------------------------------------------------------ projection
def test_projection_is_divergence_free_and_operator_consistent():
    n, ny = 8, 6
    h = 1.0 / n
    p2 = _p2(nx=n, ny=ny, lx=1.0, ly=ny * h, eps=1.5 * h)
    p3 = _p3(p2, 4)
    rng = np.random.default_rng(3)
    phi = rng.uniform(0.0, 1.0, (4, ny, n))
    u, v, w = W.random_fields3(n, ny, 4, seed=9)
    rfx, rfy, rfz = cdi3d.face_rho(phi, p3)
    x = rng.standard_normal((4, ny, n))
    A = cdi3d.assemble_A(rfx, rfy, rfz, h)
    assert np.allclose(A @ x.reshape(-1), cdi3d.apply_A(x, rfx, rfy, rfz, h).reshape(-1),
                       rtol=1e-13, atol=1e-9)
    # symmetric, rows sum to zero (constants are the null space)
    assert abs(A - A.T).max() < 1e-9
    assert np.abs(A @ np.ones(A.shape[0])).max() < 1e-9
    uu, vv, ww, pr = cdi3d.project(u, v, w, phi, 0.01, p3)
    div = cdi3d.divergence(uu, vv, ww, h)
    assert np.abs(div).max() <= 1e-9 * np.abs(cdi3d.divergence(u, v, w, h)).max()
    assert np.all(vv[:, 0] == 0.0) and np.all(vv[:, -1] == 0.0)


def test_step_conserves_mass_and_keeps_no_penetration():
    case = W.drop3_case(16, 8, 8, theta_eq_deg=50.0, ratio=5.0, r0=0.35)
    p = case.params.replace(w_wall_top=0.05)
    s = cdi3d.initial_state(case.phi0)
    m0 = cdi3d.diagnostics(s, p)["mass"]
    for _ in range(2):
        s = cdi3d.step(s, p)
    d = cdi3d.diagnostics(s, p)
    assert abs(d["mass"] - m0) <= 1e-13 * m0
    assert d["max_div"] <= 1e-8
    assert np.all(s.v[:, 0] == 0.0) and np.all(s.v[:, -1] == 0.0)
    assert d["max_uY_bot"] > 0.0


@pytest.mark.parametrize("model", ["1A", "1B"])
def test_slip_vector_converges_to_the_continuum_formula(model):
    """On phi = 1/2 + 0.2 sin(2 pi x) cos(2 pi z)(1 + y) (linear in y, so the
    wall extrapolation is exact) both slip components converge at second
    order to the model formula evaluated with the exact wall values:
    u^Y_tau = -(6 sigma/beta)[eps dphi/dn + B cos(theta_eq)] dphi/dtau, with
    B = phi(1 - phi) (1A) or eps |grad phi| including the other tangential
    component (1B), at the x-edges for tau = x and the z-edges for tau = z."""
    errs = []
    for n in (16, 32, 64):
        h = 1.0 / n
        ny = n // 2
        p = W.Params3(nx=n, ny=ny, lx=1.0, ly=ny * h, eps=0.05, gamma=1.0, sigma=1.3,
                      theta_eq=math.radians(55), rho1=1, rho2=1, mu1=1, mu2=1, beta1=7.0,
                      beta2=7.0, slip_model=model, nz=n, lz=1.0)
        X, Y, Z = W.cell_centres3(n, ny, n, h)
        phi = 0.5 + 0.2 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Z) * (1.0 + Y)
        s = cdi3d.slip_velocity_Y(phi, p, "bot")
        err = 0.0
        for comp, xs, zs in (("x", 0.0, 0.5), ("z", 0.5, 0.0)):
            x = (np.arange(n) + xs) * h
            z = (np.arange(n) + zs) * h
            Zg, Xg = np.meshgrid(z, x, indexing="ij")
            sx, cx = np.sin(2 * np.pi * Xg), np.cos(2 * np.pi * Xg)
            sz, cz = np.sin(2 * np.pi * Zg), np.cos(2 * np.pi * Zg)
            ph = 0.5 + 0.2 * sx * cz
            dn = 0.2 * sx * cz
            dx = 0.2 * 2 * np.pi * cx * cz
            dz = -0.2 * 2 * np.pi * sx * sz
            B = ph * (1 - ph) if model == "1A" else p.eps * np.sqrt(dn ** 2 + dx ** 2 + dz ** 2)
            dt = dx if comp == "x" else dz
            exact = -6.0 * p.sigma / p.beta1 * (p.eps * dn + B * math.cos(p.theta_eq)) * dt
            err = max(err, np.abs(s[f"uY{comp}"] - exact).max() / np.abs(exact).max())
        errs.append(err)
    assert errs[-1] < 2e-3, errs
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


def _prescribed_cap(n, theta_deg=60.0, R=0.5):
    """The paper's prescribed equilibrium field (Sec. 3.1) in three
    dimensions: the tanh profile of a sphere of radius R whose cap meets the
    bottom wall at theta_eq (eps = h)."""
    h = 2.0 / n
    nx, ny, nz = n, n // 2, n
    th = math.radians(theta_deg)
    p = W.Params3(nx=nx, ny=ny, lx=nx * h, ly=ny * h, eps=h, gamma=1, sigma=1, theta_eq=th,
                  rho1=1, rho2=1, mu1=0.1, mu2=0.1, beta1=10, beta2=10, nz=nz, lz=nz * h)
    X, Y, Z = W.cell_centres3(nx, ny, nz, h)
    r = np.sqrt((X - nx * h / 2) ** 2 + (Y + R * math.cos(th)) ** 2 + (Z - nz * h / 2) ** 2)
    return p, 0.5 * (1.0 + np.tanh((R - r) / (2.0 * h)))


def _max_slip(phi, p, model, fields):
    s = cdi3d.slip_velocity_Y(phi, p.replace(slip_model=model), "bot", fields=fields)
    return max(np.abs(s["uYx"]).max(), np.abs(s["uYz"]).max())


def test_curvature_correction_needs_the_inplane_curvature():
    """Sec. 3.1.2 derives the correction 1 + kappa_p psi from the in-plane
    section of the contact line.  On the prescribed 3-D cap at theta_eq the
    spurious slip of Model 4A must therefore fall under refinement with
    kappa_p, but not with the full (two principal curvatures) kappa in its
    place, nor for Model 2A without the correction."""
    res = {}
    for n in (24, 48):
        p, phi = _prescribed_cap(n)
        f = cdi3d.phase_fields(phi, p)
        full = dict(f)
        full["kappa_p"] = f["kappa"]
        res[n] = (_max_slip(phi, p, "4A", f), _max_slip(phi, p, "4A", full),
                  _max_slip(phi, p, "2A", f))
    (a1, b1, c1), (a2, b2, c2) = res[24], res[48]
    assert a1 / a2 > 1.6, res            # converges with kappa_p
    assert b1 / b2 < 1.25 and c1 / c2 < 1.4, res   # does not with kappa or without the correction
    assert a2 < 0.3 * b2 and a2 < 0.3 * c2, res
