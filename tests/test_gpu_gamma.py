"""The velocity-dependent regularisation of Sec. 5 (gamma = 2.5 |u|_max,
cdi_params.gamma_factor > 0) on the HIP path against the oracle.

Each step takes gamma = min(gamma, gamma_factor * max |u|, |v|) over the
faces of the state it starts from (a max-reduction kernel at the start of
the step, also inside the captured graph); the persistent launch keeps gamma
fixed and refuses the mode.
"""
import numpy as np
import pytest

import workloads as W
from oracle import cdi

pytestmark = pytest.mark.gpu

FIELDS = ("phi", "u", "v", "p")


def _solver(*a, **k):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_16843_amd.solver import CDISolver
    return CDISolver(*a, **k)


def relerr(a, b):
    scale = np.abs(b).max()
    return float(np.abs(a - b).max() / (scale if scale > 0 else 1.0))


def test_stage_operator_with_the_state_velocity_gamma():
    case = W.drop_case(96, 48, 120.0, 10.0)
    p = case.params.replace(gamma=5.0, gamma_factor=2.5)
    rng = np.random.default_rng(7)
    phi = np.clip(case.phi0 + 0.05 * rng.standard_normal(case.phi0.shape)
                  * case.phi0 * (1 - case.phi0), 0.0, 1.0)
    u, v = W.random_fields(p.nx, p.ny, 8, amp=0.2)
    s = _solver(p, phi, u0=u, v0=v)
    lphi, lmx, lmy, _, _ = [t.cpu().numpy() for t in s.eval_rhs()]
    s.close()
    g = cdi.step_gamma(u, v, p)
    assert 0.0 < g < p.gamma
    Lphi, Lmx, Lmy, _ = cdi.stage_rhs(phi, u, v, p.replace(gamma=g, gamma_factor=0.0))
    errs = dict(phi=relerr(lphi, Lphi), mx=relerr(lmx, Lmx), my=relerr(lmy, Lmy))
    assert max(errs.values()) < 1e-12, errs


@pytest.mark.parametrize("make,steps", [
    (lambda: W.drop_case(64, 32, 60.0, 10.0), 20),
    (lambda: W.couette_case(128, 32, lx=4.0, ly=1.0, ratio=3.0), 20),
])
def test_time_steps_with_the_velocity_gamma_match_oracle(make, steps):
    case = make()
    p = case.params.replace(gamma_factor=2.5)
    s = _solver(p, case.phi0, rtol=1e-13, maxit=400)
    s.step(steps)
    g = s.state()
    s.close()
    o = cdi.run(case.phi0, p, steps)
    errs = {k: relerr(g[k], getattr(o, k)) for k in FIELDS}
    print(case.name, errs)
    assert max(errs.values()) < 1e-10, errs
    # the velocity gamma differs from the fixed one: the runs differ
    o_fixed = cdi.run(case.phi0, case.params, steps)
    assert relerr(o.phi, o_fixed.phi) > 1e-8


def test_graph_launch_with_the_velocity_gamma_is_bitwise_the_stream_launch():
    case = W.drop_case(64, 32, 60.0, 10.0)
    p = case.params.replace(gamma_factor=2.5)
    a = _solver(p, case.phi0, rtol=1e-12, maxit=400, launch="tiled")
    b = _solver(p, case.phi0, rtol=1e-12, maxit=400, launch="graph")
    b.set_tile_rows(a.get_tile_rows())
    for _ in range(4):
        a.step(3)
        b.step(3)
        ga, gb = a.state(), b.state()
        for f in FIELDS:
            assert np.array_equal(ga[f], gb[f]), f
    assert b.graph_stats()["replays"] >= 1
    a.close()
    b.close()


def test_persistent_launch_refuses_the_velocity_gamma():
    from paper_2412_16843_amd._lib import CDIError
    case = W.drop_case(64, 32, 60.0, 10.0)
    s = _solver(case.params.replace(gamma_factor=2.5), case.phi0)
    with pytest.raises(CDIError) as e:
        s.set_launch("persistent")
    assert e.value.status == -1
    info = s.tune(trial_steps=2)
    assert info["launch"] != "persistent"
    assert info["ms_per_step"]["persistent"] < 0   # not timed
    s.close()
