"""Graph launch of the tiled path: one RK4 step captured in a HIP graph with
a fixed CG iteration budget per solve and replayed every step.

Iterations past convergence return at once, so the graph's results must be
bitwise those of the stream (tiled) launch -- including across a budget
miss, where the step is redone from its snapshot on the stream path -- and
match the FP64 oracle to 1e-10 like every other form.  Each test replays the
graph several times with host synchronisation and eager work in between.
The first steps, which build the pressure history the captured guess needs
(as many as the time-extrapolation order plus one), run on the stream path.
"""
import numpy as np
import pytest

import workloads as W
from oracle import cdi

pytestmark = pytest.mark.gpu


def _solver(*a, **k):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_16843_amd.solver import CDISolver
    return CDISolver(*a, **k)


def relerr(a, b):
    scale = np.abs(b).max()
    return float(np.abs(a - b).max() / (scale if scale > 0 else 1.0))


FIELDS = ("phi", "u", "v", "p")


@pytest.mark.parametrize("make", [
    lambda: W.drop_case(64, 32, 60.0, 10.0),           # variable density: coefficients in the graph
    lambda: W.couette_case(256, 64, lx=4.0, ly=1.0),   # uniform density, two global MG levels
])
def test_graph_bitwise_equals_stream_launch(make):
    case = make()
    steps = 12
    a = _solver(case.params, case.phi0, rtol=1e-12, maxit=400, launch="tiled")
    b = _solver(case.params, case.phi0, rtol=1e-12, maxit=400, launch="graph")
    b.set_tile_rows(a.get_tile_rows())
    for _ in range(steps // 3):          # host syncs and eager reads between replays
        a.step(3)
        b.step(3)
        ga, gb = a.state(), b.state()
        for f in FIELDS:
            assert np.array_equal(ga[f], gb[f]), f
    st = b.graph_stats()
    order = b.get_extrapolation()
    da, db = a.diagnostics(), b.diagnostics()
    a.close()
    b.close()
    print(case.name, st, "iters", da["last_iters"], db["last_iters"])
    # the first order + 1 steps build the pressure history on the stream path
    assert st["replays"] == steps - (order + 1)
    assert st["budget"] >= 1
    assert da["last_iters"] == db["last_iters"]
    assert da["step"] == db["step"] and da["t"] == db["t"]


@pytest.mark.parametrize("cells", [1024, 4096])
def test_graph_budget_miss_redoes_the_step_bitwise(cells):
    """Switching to the zero initial guess makes the solves need more
    iterations than the captured budget: the step is redone from its
    snapshot and the trajectory stays bitwise that of the stream launch.
    At 4096 cells the one-block coarse kernel owns every level of the 64x32
    grid and uses the scratch array next to the snapshot (a snapshot that
    overran its area was caught here)."""
    case = W.drop_case(64, 32, 60.0, 10.0)
    a = _solver(case.params, case.phi0, rtol=1e-12, maxit=400, launch="tiled")
    b = _solver(case.params, case.phi0, rtol=1e-12, maxit=400, launch="graph")
    b.set_tile_rows(a.get_tile_rows())
    for s in (a, b):
        s.set_coarse_cells(cells)
    for s in (a, b):
        s.step(6)
        s.set_guess("zero")
        s.step(4)
        s.set_guess("prev")
        s.step(4)
    st = b.graph_stats()
    ga, gb = a.state(), b.state()
    a.close()
    b.close()
    print("graph stats after the guess switch:", st)
    assert st["redone"] >= 1
    for f in FIELDS:
        assert np.array_equal(ga[f], gb[f]), f


def test_graph_batched_ensemble_matches_oracle():
    cases = [W.drop_case(64, 32, 60.0, 10.0, name="a"),
             W.couette_case(96, 48, lx=2.0, ly=1.0, ratio=1.0, theta_eq_deg=70.0, name="b"),
             W.couette_case(160, 80, lx=2.0, ly=1.0, ratio=10.0, ca=0.05, name="d")]
    steps = 6
    s = _solver([c.params for c in cases], [c.phi0 for c in cases], rtol=1e-13, maxit=400,
                launch="graph")
    s.step(steps)
    out = [s.state(k) for k in range(len(cases))]
    st = s.graph_stats()
    order = s.get_extrapolation()
    s.close()
    assert st["replays"] == steps - (order + 1)
    for k, c in enumerate(cases):
        o = cdi.run(c.phi0, c.params, steps)
        for f, ref in (("phi", o.phi), ("u", o.u), ("v", o.v), ("p", o.p)):
            assert relerr(out[k][f], ref) < 1e-10, (c.name, f, relerr(out[k][f], ref))


def test_graph_mixed_precision_matches_stream_bitwise():
    case = W.drop_case(128, 64, 60.0, 10.0)
    a = _solver(case.params, case.phi0, precision="mixed", rtol=1e-10, launch="tiled")
    b = _solver(case.params, case.phi0, precision="mixed", rtol=1e-10, launch="graph")
    b.set_tile_rows(a.get_tile_rows())
    a.step(8)
    b.step(8)
    ga, gb = a.state(), b.state()
    a.close()
    b.close()
    for f in FIELDS:
        assert np.array_equal(ga[f], gb[f]), f
