"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and validates parameters on the host before any device work
(error codes of include/cdi.h)."""
import ctypes as C
import math
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cdi.h")
HEADER3 = os.path.join(ROOT, "include", "cdi3.h")


def _lib():
    from paper_2412_16843_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libcdi.so not built")
    return L


def test_header_declarations_are_exported():
    L = _lib()
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    decl = set(re.findall(r"\b(cdi_[a-z_]+)\s*\(", text))
    assert {"cdi_init", "cdi_step", "cdi_solve_pressure", "cdi_diagnostics"} <= decl
    lib = L.lib()
    for name in sorted(decl):
        assert hasattr(lib, name), name
    assert set(L.EXPORTS) == decl
    text3 = re.sub(r"/\*.*?\*/", "", open(HEADER3).read(), flags=re.S)
    decl3 = set(re.findall(r"\b(cdi3_[a-z_]+)\s*\(", text3))
    assert {"cdi3_init", "cdi3_step", "cdi3_eval_rhs", "cdi3_kappa_p"} <= decl3
    for name in sorted(decl3):
        assert hasattr(lib, name), name
    assert set(L.EXPORTS3) == decl3


def test_struct_layouts_match_header():
    """The ctypes mirrors list the header's struct members in order."""
    L = _lib()
    text = open(HEADER).read()
    structs = {m.group(2): m.group(1)
               for m in re.finditer(r"typedef struct \{([^}]*)\}\s*(\w+);", text)}
    for cname, py in (("cdi_params", L.cdi_params), ("cdi_fields", L.cdi_fields),
                      ("cdi_solve_info", L.cdi_solve_info), ("cdi_diag", L.cdi_diag),
                      ("cdi_tune_info", L.cdi_tune_info)):
        body = structs[cname]
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        names = []
        for stmt in body.split(";"):
            stmt = stmt.strip()
            if not stmt:
                continue
            parts = stmt.replace("*", " ").split()
            for tok in " ".join(parts[1:]).split(","):
                names.append(re.sub(r"\[.*\]", "", tok).strip())
        assert names == [f[0] for f in py._fields_], (cname, names)


def test_3d_struct_layouts_match_header():
    L = _lib()
    text = open(HEADER3).read()
    structs = {m.group(2): m.group(1)
               for m in re.finditer(r"typedef struct \{([^}]*)\}\s*(\w+);", text)}
    for cname, py in (("cdi3_params", L.cdi3_params), ("cdi3_fields", L.cdi3_fields),
                      ("cdi3_diag", L.cdi3_diag)):
        body = re.sub(r"/\*.*?\*/", "", structs[cname], flags=re.S)
        names = []
        for stmt in body.split(";"):
            stmt = stmt.strip()
            if stmt:
                parts = stmt.replace("*", " ").split()
                names += [re.sub(r"\[.*\]", "", t).strip() for t in " ".join(parts[1:]).split(",")]
        assert names == [f[0] for f in py._fields_], (cname, names)


@pytest.mark.parametrize("kw,status", [(dict(nz=7), -2), (dict(nz=6), -2), (dict(lz=0.9), -2),
                                       (dict(precision="mixed"), -1), (dict(slip_model="5Z"), -1)])
def test_3d_invalid_parameters_rejected_on_the_host(kw, status):
    L = _lib()
    case = W.drop3_case(16, 8, 8)
    p = case.params
    prec = kw.pop("precision", "fp64")
    if "slip_model" in kw:
        cp = L.make_params3(p)
        cp.base.slip_model = 17
    else:
        p = p.replace(**kw)
        cp = L.make_params3(p)
        cp.base.precision = L.CDI_MIXED if prec == "mixed" else L.CDI_FP64
    n = C.c_size_t(0)
    assert L.lib().cdi3_workspace_bytes(C.byref(cp), C.byref(n)) == status
    ok = L.make_params3(case.params)
    assert L.lib().cdi3_workspace_bytes(C.byref(ok), C.byref(n)) == 0 and n.value > 0


def _params(**kw):
    c = W.config1()
    p = c.params.replace(**kw) if kw else c.params
    return p


def test_workspace_and_default_dt_host_only():
    L = _lib()
    lib = L.lib()
    p = _params(dt=0.0)
    cp = L.make_params(p)
    assert lib.cdi_workspace_bytes(C.byref(cp), 1) > 64 * 32 * 8 * 20
    # the library's CFL rule equals the set-up rule of the workloads
    assert math.isclose(lib.cdi_default_dt(C.byref(cp)), W.dt_from_cfl(p), rel_tol=1e-14)
    c2 = W.config2()
    cp2 = L.make_params(c2.params.replace(dt=0.0))
    assert math.isclose(lib.cdi_default_dt(C.byref(cp2)), W.dt_from_cfl(c2.params), rel_tol=1e-14)
    two = (L.cdi_params * 2)(cp, cp2)
    assert lib.cdi_workspace_bytes(two, 2) > lib.cdi_workspace_bytes(C.byref(cp), 1)


@pytest.mark.parametrize("kw,status", [
    (dict(nx=63), -2), (dict(ny=6), -2), (dict(eps=0.0), -1), (dict(theta_eq=0.0), -1),
    (dict(theta_eq=math.pi), -1), (dict(beta1=0.0), -1), (dict(gamma=-1.0), -1),
    (dict(rho2=0.0), -1), (dict(lx=3.0), -2), (dict(dt=-1.0), -1),
    # empty, negative and below-minimum grids
    (dict(nx=0), -2), (dict(ny=0), -2), (dict(nx=-8), -2), (dict(nx=2, ny=2), -2),
    (dict(gamma_factor=-1.0), -1), (dict(gamma_factor=float("nan")), -1)])
def test_invalid_parameters_rejected_before_device_work(kw, status):
    L = _lib()
    lib = L.lib()
    cp = L.make_params(_params(**kw))
    ctx = C.c_void_p()
    f = L.cdi_fields(1, 1, 1, 1)   # never dereferenced: validation comes first
    st = lib.cdi_init(C.byref(cp), C.byref(f), 256, 1 << 30, None, C.byref(ctx))
    assert st == status, (st, lib.cdi_last_error())
    assert ctx.value is None
    assert len(lib.cdi_last_error()) > 0


def test_null_and_small_workspace_rejected():
    L = _lib()
    lib = L.lib()
    cp = L.make_params(_params())
    f = L.cdi_fields(1, 1, 1, 1)
    ctx = C.c_void_p()
    assert lib.cdi_init(C.byref(cp), C.byref(f), None, 1 << 30, None, C.byref(ctx)) == -1
    assert lib.cdi_init(C.byref(cp), C.byref(f), 256, 16, None, C.byref(ctx)) == -1
    assert lib.cdi_init(C.byref(cp), C.byref(f), 257, 1 << 30, None, C.byref(ctx)) == -1
    nf = L.cdi_fields(None, 1, 1, 1)
    assert lib.cdi_init(C.byref(cp), C.byref(nf), 256, 1 << 30, None, C.byref(ctx)) == -1
    assert lib.cdi_step(None, 1) == -1


def test_smoothing_sweeps_validated_on_host():
    """mg_smooth: 0 -> 1, 1 and 2 accepted, larger rejected before device work."""
    L = _lib()
    lib = L.lib()
    f = L.cdi_fields(1, 1, 1, 1)
    ctx = C.c_void_p()
    for nu in (0, 1, 2):
        cp = L.make_params(_params(), mg_smooth=nu)
        assert lib.cdi_workspace_bytes(C.byref(cp), 1) > 0, nu
    cp = L.make_params(_params(), mg_smooth=3)
    assert lib.cdi_workspace_bytes(C.byref(cp), 1) == 0
    assert lib.cdi_init(C.byref(cp), C.byref(f), 256, 1 << 30, None, C.byref(ctx)) == -1
    assert b"mg_smooth" in lib.cdi_last_error()


def test_noalloc_entry_point_rejects_a_grid_beyond_its_scratch():
    """cdi_eval_rhs_noalloc checks the scratch its grid needs against the
    fixed array before any device work: a 32768 x 16384 grid (537 M cells,
    2.1 M tiles) does not fit the 64 MiB and returns CDI_ERR_SHAPE with a
    message."""
    L = _lib()
    lib = L.lib()
    big = W.config1().params.replace(nx=32768, ny=16384, eps=2.0 / 32768)
    cp = L.make_params(big)
    dummy = 256   # never dereferenced: the size check comes first
    cf = L.cdi_fields(dummy, dummy, dummy, None)
    st = lib.cdi_eval_rhs_noalloc(C.byref(cp), C.byref(cf), dummy, dummy, dummy, None, None,
                                  None)
    assert st == -2
    assert b"scratch" in lib.cdi_last_error()
    # a null field pointer is an argument error, also before any device work
    cf0 = L.cdi_fields(None, dummy, dummy, None)
    small = L.make_params(W.config1().params)
    assert lib.cdi_eval_rhs_noalloc(C.byref(small), C.byref(cf0), dummy, dummy, dummy, None,
                                    None, None) == -1


def test_ensemble_split_by_size_covers_and_balances():
    """The groups of a concurrently stepped ensemble: every instance in exactly
    one group, and the seeded 64-instance ensemble split into two halves of
    nearly equal cell count."""
    from paper_2412_16843_amd.solver import split_by_size
    cells = [64 * 32, 96 * 48, 128 * 64, 160 * 80, 96 * 48, 512 * 256, 256 * 128]
    for g in (1, 2, 3):
        parts = split_by_size(cells, g)
        assert sorted(k for p in parts for k in p) == list(range(len(cells)))
        assert len(parts) == g
    assert split_by_size([5, 7], 4) == [[1], [0]]
    ens = [c.params.nx * c.params.ny for c in W.config4(steps=1)]
    halves = [sum(ens[k] for k in p) for p in split_by_size(ens, 2)]
    assert abs(halves[0] - halves[1]) <= 0.02 * sum(halves), halves


def test_3d_mg_smooth_validated_on_the_host():
    """3-D multigrid smoothing: 0 (the default V(2,2)), 1 and 2 accepted, 3
    rejected before any device work."""
    L = _lib()
    p = W.drop3_case(16, 8, 8).params
    n = C.c_size_t(0)
    for nu in (0, 1, 2):
        cp = L.make_params3(p, mg_smooth=nu)
        assert L.lib().cdi3_workspace_bytes(C.byref(cp), C.byref(n)) == 0
    cp = L.make_params3(p, mg_smooth=3)
    assert L.lib().cdi3_workspace_bytes(C.byref(cp), C.byref(n)) == -1
    assert b"mg_smooth" in L.lib().cdi_last_error()
