"""Parity of the three-dimensional HIP path (include/cdi3.h) with the 3-D
oracle (oracle/cdi3d.py), element by element on seeded inputs: the stage
operator for all eight slip models (the slip vector with the in-plane
curvature kappa_p), kappa_p itself, full RK4 steps with their projections,
and the reduction of a z-invariant problem to the two-dimensional library
path.  Grids span several blocks with ragged tails and a two-to-four-level
multigrid hierarchy."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import cdi3d

pytestmark = pytest.mark.gpu


def _solver(p, phi, u=None, v=None, w=None, rtol=1e-12, guess="prev"):
    from paper_2412_16843_amd.solver3 import CDISolver3
    return CDISolver3(p, phi, u, v, w, rtol=rtol, guess=guess)


def _case(nx, ny, nz, model="4A", ratio=5.0, seed=3):
    h = 1.0 / nx * 2.0
    p = W.Params3(nx=nx, ny=ny, lx=nx * h, ly=ny * h, eps=1.3 * h, gamma=1.0, sigma=1.0,
                  theta_eq=math.radians(65), rho1=ratio, rho2=1.0, mu1=0.3, mu2=0.1,
                  beta1=8.0, beta2=4.0, u_wall_bot=0.05, u_wall_top=-0.1, slip_model=model,
                  nz=nz, lz=nz * h, w_wall_bot=0.02, w_wall_top=0.04)
    p = p.replace(dt=W.dt_from_cfl(p))
    phi = W.cap_phi3(nx, ny, nz, h, 0.35 * min(nx, nz) * h / 2, math.radians(70), p.eps,
                     0.47 * nx * h, 0.53 * nz * h)
    u, v, w = W.random_fields3(nx, ny, nz, seed=seed, amp=0.05)
    return p, phi, u, v, w


def _close(a, b, rel):
    scale = max(np.abs(b).max(), 1e-300)
    return np.abs(a - b).max() <= rel * scale, np.abs(a - b).max() / scale


@pytest.mark.parametrize("model", W.SLIP_MODELS)
def test_stage_operator_matches_oracle(model):
    p, phi, u, v, w = _case(20, 10, 12, model=model)
    s = _solver(p, phi, u, v, w)
    g = s.eval_rhs()
    s.close()
    Lphi, Lmx, Lmy, Lmz, walls = cdi3d.stage_rhs(phi, u, v, w, p)
    for name, a, b in (("Lphi", g["Lphi"], Lphi), ("Lmx", g["Lmx"], Lmx), ("Lmy", g["Lmy"], Lmy),
                       ("Lmz", g["Lmz"], Lmz)):
        ok, err = _close(a, b, 1e-12)
        assert ok, (model, name, err)
    for wi, wall in enumerate(("bot", "top")):
        for comp in ("x", "z"):
            ok, err = _close(g[f"uY{comp}"][wi], walls[wall][f"uY{comp}"], 1e-11)
            assert ok, (model, wall, comp, err)


def test_stage_operator_larger_grid_ragged_blocks():
    """Several hundred blocks, grid sizes not multiples of the block."""
    p, phi, u, v, w = _case(52, 20, 36, model="4B", ratio=10.0, seed=8)
    s = _solver(p, phi, u, v, w)
    g = s.eval_rhs()
    s.close()
    L = cdi3d.stage_rhs(phi, u, v, w, p)
    for a, b in ((g["Lphi"], L[0]), (g["Lmx"], L[1]), (g["Lmy"], L[2]), (g["Lmz"], L[3])):
        ok, err = _close(a, b, 1e-12)
        assert ok, err


def test_kappa_p_matches_oracle():
    p, phi, u, v, w = _case(24, 12, 16)
    s = _solver(p, phi)
    kp = s.kappa_p()
    s.close()
    ref = cdi3d.phase_fields(phi, p)["kappa_p"]
    ok, err = _close(kp, ref, 1e-12)
    assert ok, err


def test_one_step_matches_oracle():
    p, phi, u, v, w = _case(20, 10, 12, ratio=5.0)
    # a divergence-free start: project the random field with the oracle
    u, v, w, _ = cdi3d.project(u, v, w, phi, p.dt, p)
    s = _solver(p, phi, u, v, w, rtol=1e-13)
    s.step(1)
    g = s.state()
    d = s.diagnostics()
    s.close()
    st = cdi3d.step(cdi3d.State3(phi, u, v, w, np.zeros_like(phi)), p)
    for name in ("phi", "u", "v", "w"):
        ok, err = _close(g[name], getattr(st, name), 1e-9)
        assert ok, (name, err)
    assert d["max_div"] < 1e-8 * max(1.0, np.abs(u).max() / p.h)


def test_five_steps_match_oracle_and_conserve_mass():
    case = W.drop3_case(16, 8, 12, theta_eq_deg=55.0, ratio=3.0, r0=0.4)
    p = case.params.replace(u_wall_top=0.05, w_wall_bot=-0.03)
    s = _solver(p, case.phi0, rtol=1e-13)
    m0 = s.diagnostics()["mass"]
    s.step(5)
    g = s.state()
    d = s.diagnostics()
    s.close()
    st = cdi3d.run(case.phi0, p, 5)
    for name in ("phi", "u", "v", "w"):
        ok, err = _close(g[name], getattr(st, name), 1e-9)
        assert ok, (name, err)
    assert abs(d["mass"] - m0) <= 1e-12 * m0
    ref = cdi3d.diagnostics(st, p)
    assert abs(d["max_uY_bot"] - ref["max_uY_bot"]) <= 1e-8 * max(ref["max_uY_bot"], 1e-30)


def test_z_invariant_step_equals_two_dimensional_library_step():
    """A z-invariant 3-D problem stepped by the 3-D kernels equals the 2-D
    library's step on every slice (two independent kernel sets)."""
    from paper_2412_16843_amd.solver import CDISolver
    c2 = W.drop_case(32, 16, 60.0, 5.0, name="drop32x16")
    p2 = c2.params.replace(u_wall_bot=0.1)
    nz = 8
    d = {f: getattr(p2, f) for f in p2.__dataclass_fields__}
    d.update(nz=nz, lz=nz * p2.h)
    p3 = W.Params3(**d)
    s2 = CDISolver(p2, c2.phi0, rtol=1e-13)
    s2.step(2)
    a = s2.state(0)
    s2.close()
    s3 = _solver(p3, np.repeat(c2.phi0[None], nz, axis=0), rtol=1e-13)
    s3.step(2)
    b = s3.state()
    s3.close()
    for name in ("phi", "u", "v"):
        ok, err = _close(b[name], np.repeat(a[name][None], nz, axis=0), 1e-9)
        assert ok, (name, err)
    assert np.abs(b["w"]).max() <= 1e-12


def test_velocity_dependent_gamma_and_zero_guess_match_oracle():
    """gamma = min(gamma, 2.5 max |u|) per step (the paper's rule, Sec. 5)
    and solves started from zero instead of the previous pressure."""
    p, phi, u, v, w = _case(20, 10, 12, model="3A", ratio=4.0, seed=21)
    p = p.replace(gamma_factor=2.5)
    u, v, w, _ = cdi3d.project(u, v, w, phi, p.dt, p)
    s = _solver(p, phi, u, v, w, rtol=1e-13, guess="zero")
    s.step(2)
    g = s.state()
    s.close()
    st = cdi3d.State3(phi, u, v, w, np.zeros_like(phi))
    for _ in range(2):
        st = cdi3d.step(st, p)
    for name in ("phi", "u", "v", "w"):
        ok, err = _close(g[name], getattr(st, name), 1e-9)
        assert ok, (name, err)


def test_history_guess_and_smoothing_change_only_the_iteration_count():
    """Solves started from the cubic extrapolation of each RK stage's pressure
    history (CDI_GUESS_PREV, four steps deep after the fourth step) and from
    zero, with V(1,1) and V(2,2) smoothing, reach the same state; the history
    start needs fewer iterations once the history is full."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_16843_amd.solver3 import CDISolver3
    case = W.drop3_case(32, 16, 16, theta_eq_deg=70.0, ratio=4.0, r0=0.35)
    runs = {}
    for guess, nu in (("prev", 2), ("zero", 2), ("prev", 1)):
        s = CDISolver3(case.params, case.phi0, rtol=1e-13, guess=guess, mg_smooth=nu)
        its = []
        for _ in range(7):
            s.step(1)
            its.append(s.diagnostics()["last_iters"])
        runs[(guess, nu)] = (s.state(), its)
        s.close()
    ref = runs[("zero", 2)][0]
    for key in (("prev", 2), ("prev", 1)):
        for name in ("phi", "u", "v", "w", "p"):
            ok, err = _close(runs[key][0][name], ref[name], 1e-9)
            assert ok, (key, name, err)
    assert runs[("prev", 2)][1][-1] < runs[("zero", 2)][1][-1], runs
    assert runs[("prev", 2)][1][-1] <= runs[("prev", 1)][1][-1], runs


def test_nonfinite_state_is_reported():
    """A NaN in the phase field makes the step return CDI_ERR_NONFINITE (the
    pressure solve sees a non-finite residual) instead of running on."""
    from paper_2412_16843_amd import _lib as L
    p, phi, u, v, w = _case(20, 10, 12)
    phi = phi.copy()
    phi[3, 4, 5] = np.nan
    s = _solver(p, phi)
    with pytest.raises(L.CDIError) as e:
        s.step(1)
    s.close()
    assert "NONFINITE" in str(e.value)
