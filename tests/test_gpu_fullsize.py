"""Parity at the workloads' full sizes, in the launch configuration the bench
times (tiled launch, the wide-tile shape chosen for the grid size).

* Stage operator (phase prep, CDI flux, GNBC walls, momentum, surface
  tension) on the 1024x512 and 2048x1024 density-ratio-10 grids, element by
  element against the oracle: 1e-12 relative, as on the small grids.
* Pressure solves on the same grids: the returned pressure satisfies the
  oracle's own discrete operator to the requested 1e-10 relative residual
  (a property that holds at any size; an exact solve at 2 M unknowns would
  take minutes on the CPU), and is mean-free.
* One full RK4 step of the 1024x512 ratio-10 drop (4 variable-density
  projections): FP64 GPU vs oracle 1e-10 per field; the mixed-precision path
  against the same oracle step with its error reported.
* The full 64-instance seeded ensemble (128x64 .. 512x256) in one batched
  FP64 context for two steps, sampled instances (smallest, largest, a drop
  and a Couette at each density ratio) against the oracle at 1e-10.
"""
import numpy as np
import pytest

import workloads as W
from oracle import cdi, poisson

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


def _perturbed(case, seed, amp=0.05):
    rng = np.random.default_rng(seed)
    phi = case.phi0 + amp * rng.standard_normal(case.phi0.shape) * case.phi0 * (1 - case.phi0)
    u, v = W.random_fields(case.params.nx, case.params.ny, seed + 1, amp=0.2)
    return np.clip(phi, 0.0, 1.0), u, v


FULL = [
    ("config3_drop1024x512_r10", lambda: W.config3(60.0)),
    ("config5_drop2048x1024_r10", lambda: W.config5("drop", 2048)),
    ("config5_couette2048x1024_r10", lambda: W.config5("couette", 2048)),
]


@pytest.mark.parametrize("name,make", FULL)
def test_stage_operator_at_full_size(name, make):
    case = make()
    p = case.params
    phi, u, v = _perturbed(case, 21)
    s = _solver(p, phi, u0=u, v0=v)
    lphi, lmx, lmy, uy, us = [t.cpu().numpy() for t in s.eval_rhs()]
    s.close()
    Lphi, Lmx, Lmy, walls = cdi.stage_rhs(phi, u, v, p)
    uy_ref = np.stack([walls["bot"]["uY"], walls["top"]["uY"]])
    errs = dict(phi=relerr(lphi, Lphi), mx=relerr(lmx, Lmx), my=relerr(lmy, Lmy),
                uY=float(np.abs(uy - uy_ref).max() / max(np.abs(uy_ref).max(), 1e-300)))
    print(name, "stage operator vs oracle:", errs)
    assert max(errs.values()) < 1e-12, errs


@pytest.mark.parametrize("name,make", FULL[:2])
def test_pressure_solve_at_full_size_meets_residual(name, make):
    case = make()
    p = case.params
    rng = np.random.default_rng(5)
    # a right-hand side with both smooth and grid-scale content
    y, x = np.mgrid[0:p.ny, 0:p.nx]
    b = (np.sin(2 * np.pi * x / p.nx) * np.cos(np.pi * (y + 0.5) / p.ny)
         + 0.1 * rng.standard_normal((p.ny, p.nx)))
    s = _solver(p, case.phi0, rtol=1e-10, guess="zero")
    import torch
    pg, info = s.solve_pressure(torch.as_tensor(b))
    pg = pg.cpu().numpy()
    s.close()
    rfx, rfy = cdi.face_rho(case.phi0, p)
    bm = b - b.mean()
    res = poisson.apply_A(pg, rfx, rfy, p.h) - bm
    rel = np.linalg.norm(res) / np.linalg.norm(bm)
    print(name, "iterations", info["iterations"], "relres (GPU)", info["relres"],
          "true relres (oracle operator)", rel)
    assert info["converged"] == 1
    assert rel <= 2e-10, rel
    assert abs(pg.mean()) <= 1e-12 * np.abs(pg).max()


def test_config3_one_step_fp64_and_mixed_against_oracle():
    case = W.config3(60.0)
    o = cdi.run(case.phi0, case.params, 1)
    ref = {"phi": o.phi, "u": o.u, "v": o.v, "p": o.p}
    s = _solver(case.params, case.phi0, rtol=1e-13, maxit=400)
    s.step(1)
    g = s.state()
    s.close()
    errs = {k: relerr(g[k], ref[k]) for k in FIELDS}
    print("config3 one step FP64 vs oracle:", errs)
    assert max(errs.values()) < 1e-10, errs
    m = _solver(case.params, case.phi0, precision="mixed", rtol=1e-10)
    m.step(1)
    d = m.diagnostics()
    gm = m.state()
    m.close()
    errs = {k: relerr(gm[k], ref[k]) for k in FIELDS}
    print("config3 one step mixed vs FP64 oracle:", errs)
    assert d["last_relres"] <= 1e-10
    assert abs(d["mass"] - d["mass0"]) <= 1e-12 * d["mass0"]
    assert errs["phi"] < 1e-6 and max(errs.values()) < 1e-3, errs


def test_config4_full_ensemble_sampled_against_oracle():
    cases = W.config4()
    steps = 2
    s = _solver([c.params for c in cases], [c.phi0 for c in cases], rtol=1e-13, maxit=400)
    s.step(steps)
    size = [c.params.nx * c.params.ny for c in cases]
    pick = {int(np.argmin(size)), int(np.argmax(size))}
    for kind in ("drop", "couette"):
        for ratio in (1.0, 10.0):
            for k, c in enumerate(cases):
                if kind in c.name and abs(c.params.rho1 / c.params.rho2 - ratio) < 1e-9:
                    pick.add(k)
                    break
    for k in sorted(pick):
        c = cases[k]
        g = s.state(k)
        o = cdi.run(c.phi0, c.params, steps)
        errs = {f: relerr(g[f], ref) for f, ref in (("phi", o.phi), ("u", o.u), ("v", o.v),
                                                     ("p", o.p))}
        print(c.name, c.params.nx, "x", c.params.ny, "vs oracle:", errs)
        assert max(errs.values()) < 1e-10, (c.name, errs)
    s.close()
