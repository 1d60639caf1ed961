"""Error behaviour of the HIP path through the C ABI (statuses of
include/cdi.h): a solve that cannot reach its tolerance, right-hand sides
that vanish, and non-finite input.  Every case ends with ordinary kernel
exits: the solves stop on their own flags (maxit, a zero or non-finite norm),
never on a fault.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

NOCONV, NONFINITE = -4, -5


def _solver(*a, **k):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_16843_amd.solver import CDISolver
    return CDISolver(*a, **k)


def test_unreachable_tolerance_reports_noconv_and_keeps_the_context_usable():
    from paper_2412_16843_amd._lib import CDIError
    import torch
    case = W.drop_case(64, 32, 60.0, 10.0)
    s = _solver(case.params, case.phi0, rtol=1e-14, maxit=2, guess="zero")
    with pytest.raises(CDIError) as e:
        s.step(1)
    assert e.value.status == NOCONV
    d = s.diagnostics()
    assert d["last_iters"] == 2 and d["nonfinite"] == 0
    g = s.state()
    assert all(np.isfinite(g[k]).all() for k in g)
    # a standalone solve reports the same status and returns its last iterate
    b = np.random.default_rng(0).standard_normal((32, 64))
    pg, info = s.solve_pressure(torch.as_tensor(b))
    assert info["status"] == NOCONV and info["converged"] == 0 and info["iterations"] == 2
    assert info["relres"] > 1e-14 and np.isfinite(pg.cpu().numpy()).all()
    s.close()


@pytest.mark.parametrize("value", [0.0, 3.25])
def test_vanishing_right_hand_side_gives_zero_pressure(value):
    """b = 0, or a constant (whose mean-free part is 0): p = 0 exactly, no
    CG iteration."""
    import torch
    case = W.drop_case(64, 32, 60.0, 10.0)
    s = _solver(case.params, case.phi0, rtol=1e-12, guess="zero")
    pg, info = s.solve_pressure(torch.full((32, 64), value, dtype=torch.float64))
    s.close()
    assert info["status"] == 0 and info["converged"] == 1 and info["iterations"] == 0
    assert np.array_equal(pg.cpu().numpy(), np.zeros((32, 64)))


def test_single_fluid_at_rest_stays_exactly_at_rest():
    """phi = 1 everywhere (one fluid), u = 0, walls at rest: no CDI flux, no
    surface tension and no Young stress, so every stage's right-hand side is
    exactly zero; the solves take the zero-right-hand-side exit and nothing
    moves, bit for bit."""
    case = W.drop_case(64, 32, 60.0, 10.0)
    phi = np.ones_like(case.phi0)
    s = _solver(case.params, phi, rtol=1e-12)
    s.step(3)
    g = s.state()
    d = s.diagnostics()
    s.close()
    assert d["last_iters"] == 0
    for k in ("u", "v", "p"):
        assert np.array_equal(g[k], np.zeros_like(g[k])), k
    assert np.array_equal(g["phi"], phi)


def test_non_finite_right_hand_side_stops_the_solve():
    from paper_2412_16843_amd._lib import CDIError
    import torch
    case = W.drop_case(64, 32, 60.0, 10.0)
    s = _solver(case.params, case.phi0, rtol=1e-12, maxit=200, guess="zero")
    b = np.random.default_rng(1).standard_normal((32, 64))
    b[7, 11] = np.nan
    with pytest.raises(CDIError) as e:
        s.solve_pressure(torch.as_tensor(b))
    assert e.value.status == NONFINITE
    # the context still solves a finite right-hand side afterwards
    b[7, 11] = 0.0
    pg, info = s.solve_pressure(torch.as_tensor(b))
    assert info["status"] == 0 and info["converged"] == 1
    s.close()


def test_non_finite_phase_field_is_refused_at_init():
    from paper_2412_16843_amd._lib import CDIError
    case = W.drop_case(64, 32, 60.0, 10.0)
    phi = case.phi0.copy()
    phi[3, 5] = np.inf
    with pytest.raises(CDIError) as e:
        _solver(case.params, phi)
    assert e.value.status == NONFINITE


def test_non_finite_state_is_reported_by_the_next_step():
    from paper_2412_16843_amd._lib import CDIError
    case = W.drop_case(64, 32, 60.0, 10.0)
    s = _solver(case.params, case.phi0, rtol=1e-12, maxit=200)
    s.step(2)
    g = s.state()
    u = g["u"].copy()
    u[10, 20] = np.nan
    s.set_state(0, u=u)
    with pytest.raises(CDIError) as e:
        s.step(1)
    assert e.value.status == NONFINITE
    s.close()
