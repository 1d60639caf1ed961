"""Mixed-precision and batched-ensemble forms of the HIP path.

Mixed precision: FP32 stencils and V-cycle, FP64 phase field, phi-flux
differences, CG vectors, residual and reductions.  Its bar: every pressure
solve reaches the FP64 relative residual 1e-10, the mass drift stays at
FP64 round-off (<= 1e-12 relative), and the per-field error against the FP64
oracle is reported (bounded here by FP32 round-off amplified over the run).

Batched ensemble: uneven instances in one set of launches; each instance must
be bitwise identical to the same instance run alone (no cross-talk) and match
the oracle like the single-instance FP64 path.
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


@pytest.mark.parametrize("make,steps", [
    (lambda: W.drop_case(128, 64, 60.0, 10.0), 20),
    (lambda: W.couette_case(128, 32, lx=4.0, ly=1.0), 20),
])
def test_mixed_precision_against_fp64_oracle(make, steps):
    case = make()
    s = _solver(case.params, case.phi0, precision="mixed", rtol=1e-10)
    iters = []
    for _ in range(steps):
        s.step(1)
        d = s.diagnostics()
        iters.append(d["last_iters"])
        assert d["last_relres"] <= 1e-10
    g = s.state()
    s.close()
    o = cdi.run(case.phi0, case.params, steps)
    errs = {k: relerr(g[k], ref) for k, ref in (("phi", o.phi), ("u", o.u), ("v", o.v),
                                                  ("p", o.p))}
    print(f"{case.name} mixed vs FP64 oracle after {steps} steps:", errs, "iters", iters[-1])
    drift = abs(d["mass"] - d["mass0"]) / d["mass0"]
    assert drift <= 1e-12, drift
    assert errs["phi"] < 1e-5, errs
    assert max(errs.values()) < 1e-3, errs


@pytest.mark.parametrize("coarse_cells", [1024, 4096])
def test_batched_ensemble_matches_solo_and_oracle(coarse_cells):
    """Four instances of different sizes in one context: bitwise the solo
    runs, and the oracle to 1e-10.  With coarse_cells 4096 the one-block
    coarse kernel of each instance starts at its wide level (64x32 level 0,
    48x24, 64x32 and 80x40 level 1), each block deciding for itself."""
    cases = [W.drop_case(64, 32, 60.0, 10.0, name="a"),
             W.couette_case(96, 48, lx=2.0, ly=1.0, ratio=1.0, theta_eq_deg=70.0, name="b"),
             W.drop_case(128, 64, 120.0, 1.0, name="c"),
             W.couette_case(160, 80, lx=2.0, ly=1.0, ratio=10.0, ca=0.05, name="d")]
    steps = 4
    s = _solver([c.params for c in cases], [c.phi0 for c in cases], rtol=1e-13, maxit=400)
    s.set_coarse_cells(coarse_cells)
    s.step(steps)
    batched = [s.state(k) for k in range(len(cases))]
    s.close()
    for k, c in enumerate(cases):
        solo = _solver(c.params, c.phi0, rtol=1e-13, maxit=400)
        solo.set_coarse_cells(coarse_cells)
        solo.step(steps)
        g = solo.state()
        solo.close()
        for f in ("phi", "u", "v", "p"):
            assert np.array_equal(batched[k][f], g[f]), (c.name, f)
        o = cdi.run(c.phi0, c.params, steps)
        for f, ref in (("phi", o.phi), ("u", o.u), ("v", o.v), ("p", o.p)):
            assert relerr(g[f], ref) < 1e-10, (c.name, f, relerr(g[f], ref))


def test_config4_ensemble_runs_and_conserves_mass():
    """The seeded 64-instance ensemble (128x64 .. 512x256, drops and Couette,
    theta_eq in [30, 150] deg, Ca log-uniform, density ratio 1 or 10) in one
    batched context, mixed precision: every instance stays finite, bounded
    and mass-conserving."""
    cases = W.config4(steps=3)
    s = _solver([c.params for c in cases], [c.phi0 for c in cases], precision="mixed")
    s.step(3)
    for k in range(len(cases)):
        d = s.diagnostics(k)
        assert d["nonfinite"] == 0
        assert abs(d["mass"] - d["mass0"]) <= 1e-12 * d["mass0"]
        assert -1e-6 < d["phi_min"] and d["phi_max"] < 1 + 1e-6
        assert d["last_relres"] <= 1e-10
    s.close()
