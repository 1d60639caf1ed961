"""The mixed-precision equilibrium-drop workload at full size: 1024 x 512 on
2 x 1, density and viscosity ratio 10, theta_eq in {30, 60, 120, 150} deg
(Sec. 5.1 drop, the angles of the paper's contact-angle range).

* One FP64 step of each angle against the FP64 oracle (exact sparse-LU
  projections) at 1e-10 relative per field, the GPU solves at 1e-13.
* One mixed step of each angle (FP32 stencils and V-cycle; FP64 phase field,
  phi-flux differences, CG vectors, residual, reductions) against the same
  oracle step: the solve reaches 1e-10, mass drifts by at most 1e-12, and the
  per-field error stays at FP32 round-off level (bounds in MIXED_BOUND).
* 200 steps of all four angles in one batched context, mixed against FP64
  on the GPU (the FP64 path being pinned to the oracle above).

The oracle steps (about 40 s each on one core) run in four child processes
that write their fields to a temporary folder.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FIELDS = ("phi", "u", "v", "p")
# error of the mixed path, a few times above what was measured on the MI355X:
# one step against the FP64 oracle (measured at most 8.6e-11, 2.4e-7, 8.2e-7
# and 2.1e-7 for phi, u, v, p over the four angles) ...
MIXED_BOUND = {"phi": 5e-10, "u": 2e-6, "v": 5e-6, "p": 2e-6}
# ... and after 200 steps against the FP64 GPU path (measured at most 1.3e-8,
# 5.7e-8, 2.5e-7, 3.0e-7)
MIXED_200_BOUND = {"phi": 1e-7, "u": 5e-7, "v": 2e-6, "p": 2e-6}


def _solver(*a, **k):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_16843_amd.solver import CDISolver
    return CDISolver(*a, **k)


def relerr(a, b):
    scale = np.abs(b).max()
    return float(np.abs(a - b).max() / (scale if scale > 0 else 1.0))


_CHILD = """
import sys, numpy as np
import workloads as W
from oracle import cdi
th, out = float(sys.argv[1]), sys.argv[2]
c = W.config3(th)
o = cdi.run(c.phi0, c.params, 1)
np.savez(out, phi=o.phi, u=o.u, v=o.v, p=o.p)
"""


@pytest.fixture(scope="module")
def oracle_steps(tmp_path_factory):
    pytest.importorskip("torch")
    d = tmp_path_factory.mktemp("config3_oracle")
    env = dict(os.environ, PYTHONPATH=ROOT, OMP_NUM_THREADS="1")
    procs = {}
    for th in W.CONFIG3_THETAS:
        out = str(d / f"th{int(th)}.npz")
        procs[th] = (subprocess.Popen([sys.executable, "-c", _CHILD, str(th), out], env=env,
                                      cwd=ROOT), out)
    refs = {}
    for th, (pr, out) in procs.items():
        assert pr.wait(timeout=600) == 0, th
        with np.load(out) as z:
            refs[th] = {k: z[k].copy() for k in FIELDS}
    return refs


@pytest.mark.parametrize("theta", W.CONFIG3_THETAS)
def test_config3_fp64_step_matches_oracle(theta, oracle_steps):
    case = W.config3(theta)
    s = _solver(case.params, case.phi0, rtol=1e-13, maxit=400)
    s.step(1)
    g = s.state()
    s.close()
    errs = {k: relerr(g[k], oracle_steps[theta][k]) for k in FIELDS}
    print(f"config3 theta {theta:.0f} one FP64 step vs oracle:", errs)
    assert max(errs.values()) < 1e-10, errs


@pytest.mark.parametrize("theta", W.CONFIG3_THETAS)
def test_config3_mixed_step_against_oracle(theta, oracle_steps):
    case = W.config3(theta)
    m = _solver(case.params, case.phi0, precision="mixed", rtol=1e-10)
    m.step(1)
    d = m.diagnostics()
    gm = m.state()
    m.close()
    errs = {k: relerr(gm[k], oracle_steps[theta][k]) for k in FIELDS}
    print(f"config3 theta {theta:.0f} one mixed step vs FP64 oracle:", errs,
          "relres", d["last_relres"], "mass drift", abs(d["mass"] - d["mass0"]) / d["mass0"])
    assert d["last_relres"] <= 1e-10
    assert abs(d["mass"] - d["mass0"]) <= 1e-12 * d["mass0"]
    for k in FIELDS:
        assert errs[k] < MIXED_BOUND[k], (k, errs)


def test_config3_mixed_against_fp64_over_200_steps():
    cases = [W.config3(th) for th in W.CONFIG3_THETAS]
    ps, phis = [c.params for c in cases], [c.phi0 for c in cases]
    f = _solver(ps, phis, rtol=1e-10)
    m = _solver(ps, phis, precision="mixed", rtol=1e-10)
    f.step(200)
    m.step(200)
    for k, c in enumerate(cases):
        gf, gm = f.state(k), m.state(k)
        dm = m.diagnostics(k)
        errs = {q: relerr(gm[q], gf[q]) for q in FIELDS}
        print(f"config3 theta {c.params.theta_eq * 180 / np.pi:.0f} mixed vs FP64, 200 steps:",
              errs, "mass drift", abs(dm["mass"] - dm["mass0"]) / dm["mass0"])
        assert dm["last_relres"] <= 1e-10
        assert abs(dm["mass"] - dm["mass0"]) <= 1e-12 * dm["mass0"]
        for q in FIELDS:
            assert errs[q] < MIXED_200_BOUND[q], (c.name, q, errs)
    f.close()
    m.close()
