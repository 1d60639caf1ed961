"""Persistent launch of the HIP path (one workgroup per instance runs whole
steps, CG loop and stopping test included).

Same discretisation and solver as the tiled launch, only the summation order
of the CG reductions differs, so its bar is the tiled path's: relative error
<= 1e-10 against the FP64 oracle per field with the pressure solved to 1e-13,
mass conserved to round-off; mixed precision within the tiled mixed path's
bounds; batched instances matching their solo runs to the solver tolerance.
Cases span single-level-in-LDS grids (<= 1024 cells), grids with global
levels, uneven batches and runs longer than one launch (32 steps).
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


def _oracle(case, steps):
    o = cdi.run(case.phi0, case.params, steps)
    return {"phi": o.phi, "u": o.u, "v": o.v, "p": o.p}, o


@pytest.mark.parametrize("make,steps", [
    (lambda: W.drop_case(32, 16, 60.0, lx=2.0, ly=1.0), 6),          # whole grid in LDS
    (lambda: W.drop_case(64, 32, 60.0), 5),
    (lambda: W.drop_case(64, 32, 60.0, 10.0), 5),
    (lambda: W.couette_case(128, 32, lx=4.0, ly=1.0), 5),
    (lambda: W.couette_case(96, 48, lx=2.0, ly=1.0, ratio=10.0, theta_eq_deg=70.0), 5),
])
def test_persistent_step_parity_short(make, steps):
    case = make()
    s = _solver(case.params, case.phi0, rtol=1e-13, maxit=400, launch="persistent")
    assert s.get_launch() == "persistent"
    s.step(steps)
    g = s.state()
    d = s.diagnostics()
    s.close()
    ref, _ = _oracle(case, steps)
    errs = {k: relerr(g[k], ref[k]) for k in FIELDS}
    print(case.name, "persistent vs oracle:", errs, "last iters", d["last_iters"])
    assert max(errs.values()) < 1e-10, errs
    assert abs(d["mass"] - d["mass0"]) <= 1e-13 * d["mass0"]
    assert d["last_relres"] <= 1e-13


def test_persistent_config1_full_run_parity():
    """Equilibrium drop 64x32, theta 90 -> 60 deg, 500 steps in one call
    (16 launches of at most 32 steps)."""
    case = W.config1()
    s = _solver(case.params, case.phi0, rtol=1e-13, maxit=400, launch="persistent")
    s.step(case.steps)
    g = s.state()
    d = s.diagnostics()
    s.close()
    ref, o = _oracle(case, case.steps)
    errs = {k: relerr(g[k], ref[k]) for k in FIELDS}
    print("config1 persistent per-field relative error:", errs)
    assert max(errs.values()) < 1e-10, errs
    od = cdi.diagnostics(o, case.params)
    assert abs(d["mass"] - od["mass"]) < 1e-12 * od["mass"]
    assert abs(d["max_uslip_bot"] - od["max_uslip_bot"]) < 1e-9 * od["max_uslip_bot"]


def test_persistent_couette256x64_matches_oracle_and_tiled():
    """Two-phase Couette 256x64 (two global levels below the LDS levels):
    40 steps, persistent vs oracle and vs the tiled launch at the default
    tolerance 1e-10."""
    case = W.config2()
    steps = 40
    s = _solver(case.params, case.phi0, rtol=1e-13, maxit=400, launch="persistent")
    s.step(steps)
    g = s.state()
    s.close()
    ref, _ = _oracle(case, steps)
    errs = {k: relerr(g[k], ref[k]) for k in FIELDS}
    print("couette256x64 persistent vs oracle:", errs)
    assert max(errs.values()) < 1e-10, errs
    # default tolerance: both launches agree to what the solver guarantees
    a = _solver(case.params, case.phi0, launch="persistent")
    b = _solver(case.params, case.phi0, launch="tiled")
    a.step(steps)
    b.step(steps)
    ga, gb = a.state(), b.state()
    ia, ib = a.diagnostics()["last_iters"], b.diagnostics()["last_iters"]
    a.close()
    b.close()
    errs = {k: relerr(ga[k], gb[k]) for k in FIELDS}
    print("persistent vs tiled at rtol 1e-10:", errs, "iters", ia, ib)
    assert max(errs.values()) < 1e-8, errs
    assert abs(ia - ib) <= 2


def test_persistent_batched_uneven_ensemble():
    """Four uneven instances in one persistent launch: each matches the oracle
    (1e-10) and its own solo tiled run."""
    cases = [W.drop_case(64, 32, 60.0, 10.0, name="a"),
             W.couette_case(96, 48, lx=2.0, ly=1.0, ratio=1.0, theta_eq_deg=70.0, name="b"),
             W.drop_case(32, 16, 120.0, 1.0, name="c"),
             W.couette_case(160, 80, lx=2.0, ly=1.0, ratio=10.0, ca=0.05, name="d")]
    steps = 4
    s = _solver([c.params for c in cases], [c.phi0 for c in cases], rtol=1e-13, maxit=400,
                launch="persistent")
    s.step(steps)
    batched = [s.state(k) for k in range(len(cases))]
    s.close()
    for k, c in enumerate(cases):
        solo = _solver(c.params, c.phi0, rtol=1e-13, maxit=400)
        solo.step(steps)
        g = solo.state()
        solo.close()
        ref, _ = _oracle(c, steps)
        for f in FIELDS:
            assert relerr(batched[k][f], g[f]) < 1e-11, (c.name, f)
            assert relerr(batched[k][f], ref[f]) < 1e-10, (c.name, f)


def test_persistent_mixed_precision_against_fp64_oracle():
    case = W.drop_case(128, 64, 60.0, 10.0)
    steps = 20
    s = _solver(case.params, case.phi0, precision="mixed", rtol=1e-10, launch="persistent")
    s.step(steps)
    d = s.diagnostics()
    g = s.state()
    s.close()
    assert d["last_relres"] <= 1e-10
    ref, _ = _oracle(case, steps)
    errs = {k: relerr(g[k], ref[k]) for k in FIELDS}
    print("mixed persistent vs FP64 oracle:", errs)
    assert abs(d["mass"] - d["mass0"]) <= 1e-12 * d["mass0"]
    assert errs["phi"] < 1e-5, errs
    assert max(errs.values()) < 1e-3, errs


def test_switching_launch_mid_run_keeps_the_trajectory():
    """3 tiled steps, 3 persistent, 3 tiled: the pressure history and state
    carry across launch forms."""
    case = W.drop_case(64, 32, 60.0, 10.0)
    s = _solver(case.params, case.phi0, rtol=1e-13, maxit=400)
    for mode in ("tiled", "persistent", "tiled"):
        s.set_launch(mode)
        s.step(3)
    g = s.state()
    s.close()
    ref, _ = _oracle(case, 9)
    errs = {k: relerr(g[k], ref[k]) for k in FIELDS}
    assert max(errs.values()) < 1e-10, errs


@pytest.mark.parametrize("rows", [1, 4])
def test_wide_tile_rows_match_oracle(rows):
    """Both wide-tile shapes of the CG kernels (1 and 4 rows per thread)."""
    case = W.drop_case(128, 64, 60.0, 10.0)
    s = _solver(case.params, case.phi0, rtol=1e-13, maxit=400)
    s.set_tile_rows(rows)
    assert s.get_tile_rows() == rows
    s.step(4)
    g = s.state()
    s.close()
    ref, _ = _oracle(case, 4)
    errs = {k: relerr(g[k], ref[k]) for k in FIELDS}
    assert max(errs.values()) < 1e-10, errs


def test_autotune_restores_state_and_keeps_the_trajectory():
    """cdi_tune times every candidate from a saved state and restores it:
    the run continues as if the tuner had not run."""
    case = W.drop_case(64, 32, 60.0, 10.0)
    s = _solver(case.params, case.phi0, rtol=1e-13, maxit=400)
    s.step(3)
    d0 = s.diagnostics()
    info = s.tune(trial_steps=3)
    print("tune:", info)
    assert info["launch"] in ("tiled", "persistent")
    assert all(v > 0 for v in info["ms_per_step"].values())
    d1 = s.diagnostics()
    assert d1["step"] == d0["step"] and d1["t"] == d0["t"]
    assert d1["mass"] == d0["mass"]
    s.step(3)
    g = s.state()
    s.close()
    ref, _ = _oracle(case, 6)
    errs = {k: relerr(g[k], ref[k]) for k in FIELDS}
    assert max(errs.values()) < 1e-10, errs


@pytest.mark.parametrize("cells", [1024, 4096, 16384])
@pytest.mark.parametrize("make,precision", [
    (lambda: W.couette_case(256, 64, lx=4.0, ly=1.0), "fp64"),   # levels 16384 / 4096 / 1024
    (lambda: W.drop_case(128, 64, 60.0, 10.0), "fp64"),          # 8192 / 2048 / 512
    (lambda: W.drop_case(128, 64, 60.0, 10.0), "mixed"),
    (lambda: W.couette_case(96, 48, lx=2.0, ly=1.0, ratio=10.0), "fp64"),  # 4608 / 1152 / 288
])
def test_coarse_kernel_start_level_matches_oracle(cells, make, precision):
    """The one-block coarse kernel taking over the levels with at most
    `cells` cells (global memory above 1024 cells, the whole grid at 16384
    for 256x64): same solution as the oracle.  At 4096 it starts at the
    wide level just above the LDS levels (4096, 2048 and 1152 cells: two,
    one and a partial set of cells of each colour per thread)."""
    case = make()
    rtol = 1e-13 if precision == "fp64" else 1e-10
    s = _solver(case.params, case.phi0, rtol=rtol, maxit=400, precision=precision)
    s.set_coarse_cells(cells)
    assert s.get_coarse_cells() == cells
    s.step(5)
    d = s.diagnostics()
    g = s.state()
    s.close()
    ref, _ = _oracle(case, 5)
    errs = {k: relerr(g[k], ref[k]) for k in FIELDS}
    print(case.name, precision, cells, errs, "iters", d["last_iters"])
    assert d["last_relres"] <= rtol
    if precision == "fp64":
        assert max(errs.values()) < 1e-10, errs
    else:
        assert errs["phi"] < 1e-5 and max(errs.values()) < 1e-3, errs


def test_autotune_stays_inside_its_scratch():
    """The tuner's saved state fills exactly cdi_tune_bytes: guard bytes
    right after the scratch are untouched (regression: a state copy once
    overran it by one field)."""
    torch = pytest.importorskip("torch")
    import ctypes as C
    from paper_2412_16843_amd import _lib as L
    case = W.drop_case(64, 32, 60.0, 10.0)
    s = _solver(case.params, case.phi0, rtol=1e-12)
    s.step(2)
    nb = s.lib.cdi_tune_bytes(s.ctx)
    guard = 1 << 16
    buf = torch.full((nb + guard + 256,), 0x5A, dtype=torch.uint8, device="cuda")
    off = (-buf.data_ptr()) % 256
    info = L.cdi_tune_info()
    L.check(s.lib.cdi_tune(s.ctx, 2, buf.data_ptr() + off, nb, C.byref(info)))
    torch.cuda.synchronize()
    tail = buf[off + nb:off + nb + guard].cpu().numpy()
    s.close()
    assert (tail == 0x5A).all()


@pytest.mark.parametrize("launch", ["tiled", "persistent"])
@pytest.mark.parametrize("make", [
    lambda: W.couette_case(256, 64, lx=4.0, ly=1.0),
    lambda: W.drop_case(128, 64, 60.0, 10.0),
])
def test_two_sweep_pairs_match_oracle_in_fewer_iterations(launch, make):
    """V(2,2) smoothing (mg_smooth = 2): same solution as the oracle, and
    fewer CG iterations per solve than V(1,1)."""
    case = make()
    its = {}
    for nu in (1, 2):
        s = _solver(case.params, case.phi0, rtol=1e-13, maxit=400, launch=launch, mg_smooth=nu)
        s.step(4)
        its[nu] = s.diagnostics()["last_iters"]
        g = s.state()
        s.close()
        if nu == 2:
            ref, _ = _oracle(case, 4)
            errs = {k: relerr(g[k], ref[k]) for k in FIELDS}
            assert max(errs.values()) < 1e-10, errs
    print(case.name, launch, "iterations V(1,1) / V(2,2):", its)
    assert its[2] < its[1]


@pytest.mark.parametrize("launch", ["tiled", "persistent"])
def test_coarsest_cg_grid_matches_oracle(launch):
    """240 x 120 halves to a 30 x 15 coarsest grid (450 cells, beyond the
    dense inverse): the V-cycle ends in the single-reduction CG of the coarse
    kernel.  FP64 against the oracle at 1e-10 (CG to 1e-13); the mixed path
    reaches the residual with the mass conserved."""
    case = W.drop_case(240, 120, 60.0, 10.0)
    steps = 3
    ref, _ = _oracle(case, steps)
    s = _solver(case.params, case.phi0, rtol=1e-13, maxit=400, launch=launch)
    s.step(steps)
    d = s.diagnostics()
    g = s.state()
    s.close()
    errs = {k: relerr(g[k], ref[k]) for k in FIELDS}
    print(launch, "240x120 FP64 vs oracle:", errs, "iterations", d["last_iters"])
    assert max(errs.values()) < 1e-10, errs
    assert d["last_iters"] <= 40
    m = _solver(case.params, case.phi0, precision="mixed", rtol=1e-10, launch=launch)
    m.step(steps)
    dm = m.diagnostics()
    m.close()
    assert dm["last_relres"] <= 1e-10
    assert abs(dm["mass"] - dm["mass0"]) <= 1e-12 * dm["mass0"]
