"""Initial guess of the pressure solves by time extrapolation of each RK
stage's pressure over the last q + 1 steps (q = 0..3).

The guess is an implementation choice of the solver: every order must give
the oracle's fields to the parity bar (1e-10 relative per field; the GPU
solves to 1e-13 here), and higher orders must not need more CG iterations
once the history is full.  On the two-phase Couette the pressure changes
smoothly in time, so the guess error falls by about two orders of magnitude
per extrapolation order (2.6e-5, 2.4e-7, 3e-9 relative for linear,
quadratic, cubic after 160 steps, measured with the oracle).
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


def test_every_extrapolation_order_matches_oracle_and_saves_iterations():
    case = W.config2()
    warm, steps = 20, 20
    o = cdi.run(case.phi0, case.params, warm + steps)
    iters = {}
    for order in (0, 1, 2, 3):
        s = _solver(case.params, case.phi0, rtol=1e-13, maxit=400)
        s.set_extrapolation(order)
        assert s.get_extrapolation() == order
        s.step(warm)
        s.timing_enable("pcg_spmv")
        s.step(steps)
        _, n = s.timing_read()
        s.timing_enable(None)
        g = s.state()
        s.close()
        iters[order] = n
        errs = {k: relerr(g[k], ref) for k, ref in (("phi", o.phi), ("u", o.u), ("v", o.v),
                                                      ("p", o.p))}
        assert max(errs.values()) < 1e-10, (order, errs)
    print("CG iterations over 20 steps by extrapolation order:", iters)
    assert iters[1] <= iters[0] and iters[2] <= iters[1] and iters[3] <= iters[2], iters
    assert iters[3] < iters[1], iters


def test_extrapolation_order_is_validated():
    from paper_2412_16843_amd._lib import CDIError
    case = W.config1()
    s = _solver(case.params, case.phi0)
    assert s.get_extrapolation() == 3
    for bad in (-1, 4):
        with pytest.raises(CDIError):
            s.set_extrapolation(bad)
    assert s.get_extrapolation() == 3
    s.close()
