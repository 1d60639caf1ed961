"""The allocation-free stage operator (cdi_eval_rhs_noalloc) against the
context entry point cdi_eval_rhs through the C ABI: the same kernels on the
same fields, so the outputs must agree bit for bit.  Two calls in a row on
one GPU share the scratch array; the second, on a smaller grid, must not see
anything of the first.  The operator itself is also checked against the
oracle (1e-12 relative, as the stage-operator parity tests)."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from oracle import cdi

pytestmark = pytest.mark.gpu


def _torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _perturbed(case, seed):
    rng = np.random.default_rng(seed)
    phi = case.phi0 + 0.05 * rng.standard_normal(case.phi0.shape) * case.phi0 * (1 - case.phi0)
    u, v = W.random_fields(case.params.nx, case.params.ny, seed + 1, amp=0.2)
    return np.clip(phi, 0.0, 1.0), u, v


def _noalloc(p, phi, u, v, precision="fp64"):
    torch = _torch()
    from paper_2412_16843_amd import _lib as L
    lib = L.lib()
    dev = torch.device("cuda:0")
    t = {k: torch.as_tensor(np.ascontiguousarray(a), device=dev).clone()
         for k, a in (("phi", phi), ("u", u), ("v", v))}
    cp = L.make_params(p, precision)
    cf = L.cdi_fields(t["phi"].data_ptr(), t["u"].data_ptr(), t["v"].data_ptr(), None)
    ny, nx = p.ny, p.nx
    # outputs filled with garbage: every element must be written by the call
    out = dict(lphi=torch.full((ny, nx), np.nan, dtype=torch.float64, device=dev),
               lmx=torch.full((ny, nx), np.nan, dtype=torch.float64, device=dev),
               lmy=torch.full((ny + 1, nx), np.nan, dtype=torch.float64, device=dev),
               uy=torch.full((2, nx), np.nan, dtype=torch.float64, device=dev),
               us=torch.full((2, nx), np.nan, dtype=torch.float64, device=dev))
    stream = torch.cuda.current_stream(dev)
    st = lib.cdi_eval_rhs_noalloc(C.byref(cp), C.byref(cf), out["lphi"].data_ptr(),
                                  out["lmx"].data_ptr(), out["lmy"].data_ptr(),
                                  out["uy"].data_ptr(), out["us"].data_ptr(), stream.cuda_stream)
    L.check(st)
    torch.cuda.synchronize(dev)
    return {k: v.cpu().numpy() for k, v in out.items()}


def _ctx(p, phi, u, v, precision="fp64"):
    _torch()
    from paper_2412_16843_amd.solver import CDISolver
    s = CDISolver(p, phi, u0=u, v0=v, precision=precision)
    lphi, lmx, lmy, uy, us = [x.cpu().numpy() for x in s.eval_rhs()]
    s.close()
    return dict(lphi=lphi, lmx=lmx, lmy=lmy, uy=uy, us=us)


CASES = [
    # (name, case, precision, gamma_factor): the second of each pair is smaller
    ("drop1024x512_r10", lambda: W.drop_case(1024, 512, 60.0, 10.0), "fp64", 0.0),
    ("couette256x64", lambda: W.config2(), "fp64", 0.0),
    ("drop512x256_mixed", lambda: W.drop_case(512, 256, 120.0, 10.0), "mixed", 0.0),
    ("drop96x48_dyn_gamma", lambda: W.drop_case(96, 48, 30.0, 10.0), "fp64", 2.5),
]


def test_noalloc_matches_context_entry_point_on_two_calls_in_a_row():
    results = []
    for name, make, prec, gf in CASES:
        case = make()
        p = case.params.replace(gamma_factor=gf)
        phi, u, v = _perturbed(case, 31)
        print("case", name, p.nx, "x", p.ny, prec, "gamma_factor", gf, flush=True)
        a = _noalloc(p, phi, u, v, prec)
        b = _ctx(p, phi, u, v, prec)
        for k in a:
            assert np.isfinite(a[k]).all(), (name, k)
            assert np.array_equal(a[k], b[k]), (name, k, np.abs(a[k] - b[k]).max())
        if prec == "fp64":
            Lphi, Lmx, Lmy, walls = cdi.stage_rhs(phi, u, v, p)
            for k, ref in (("lphi", Lphi), ("lmx", Lmx), ("lmy", Lmy)):
                err = np.abs(a[k] - ref).max() / np.abs(ref).max()
                assert err < 1e-12, (name, k, err)
            uy_ref = np.stack([walls["bot"]["uY"], walls["top"]["uY"]])
            assert np.abs(a["uy"] - uy_ref).max() <= 1e-12 * max(np.abs(uy_ref).max(), 1e-300)
        results.append(name)
    assert len(results) == len(CASES)
