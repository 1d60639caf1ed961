"""Device diagnostics through the C ABI (cdi_diagnostics) against the oracle's
diagnostics of the same state: mass, bounds, slip maxima and the contact-line
measures of Sec. 5.1 (phi = 1/2 wall crossings, wetted length, cap angle),
on a spreading drop (two crossings on the bottom wall, none on the top) and
a two-phase Couette flow (two crossings on each wall)."""
import math

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


CASES = [
    ("drop96x48_r10", lambda: W.drop_case(96, 48, 60.0, 10.0), 20),
    ("drop64x32_theta150", lambda: W.drop_case(64, 32, 150.0), 30),
    ("couette128x32", lambda: W.couette_case(128, 32, lx=4.0, ly=1.0, theta_eq_deg=70.0), 20),
]


@pytest.mark.parametrize("name,make,steps", CASES)
def test_device_diagnostics_match_oracle(name, make, steps):
    case = make()
    s = _solver(case.params, case.phi0, rtol=1e-13, maxit=400)
    s.step(steps)
    d = s.diagnostics()
    g = s.state()
    s.close()
    st = cdi.initial_state(g["phi"])
    st.u, st.v, st.p = g["u"], g["v"], g["p"]
    o = cdi.diagnostics(st, case.params)
    print(name, {k: d[k] for k in ("n_contact_bot", "n_contact_top", "contact_x_bot",
                                   "contact_x_top", "wetted_len_bot", "theta_est_bot")})
    assert abs(d["mass"] - o["mass"]) <= 1e-13 * o["mass"]
    assert d["phi_min"] == o["phi_min"] and d["phi_max"] == o["phi_max"]
    assert abs(d["ke"] - o["ke"]) <= 1e-12 * o["ke"]
    # wall maxima against the larger wall's scale (far from a contact line the
    # slip is a product of phi(1 - phi) factors near round-off)
    for q in ("max_uslip", "max_uY"):
        scale = max(o[q + "_bot"], o[q + "_top"])
        for wall in ("bot", "top"):
            k = f"{q}_{wall}"
            assert abs(d[k] - o[k]) <= 1e-11 * scale, (k, d[k], o[k])
    # |div u| after the projection is a difference of O(|u|/h) face terms
    uscale = (np.abs(g["u"]).max() + np.abs(g["v"]).max()) / case.params.h
    assert abs(d["max_div"] - o["max_div"]) <= 1e-13 * uscale
    for wall in ("bot", "top"):
        assert d[f"n_contact_{wall}"] == o[f"n_contact_{wall}"], wall
        xs, xo = d[f"contact_x_{wall}"], o[f"contact_x_{wall}"]
        assert len(xs) == len(xo)
        for a, b in zip(xs, xo):
            assert abs(a - b) <= 1e-12 * case.params.lx, (wall, xs, xo)
        if o[f"n_contact_{wall}"] == 2:
            assert abs(d[f"wetted_len_{wall}"] - o[f"wetted_len_{wall}"]) <= 1e-12
            assert abs(d[f"theta_est_{wall}"] - o[f"theta_est_{wall}"]) <= 1e-10
        else:
            assert d[f"wetted_len_{wall}"] == 0.0 and d[f"theta_est_{wall}"] == 0.0
    if "drop" in name:
        assert d["n_contact_bot"] == 2 and d["n_contact_top"] == 0
        # the drop is still spreading (90 deg -> 60) or receding (-> 150)
        assert 0.0 < d["theta_est_bot"] < math.pi
    else:
        assert d["n_contact_bot"] == 2 and d["n_contact_top"] == 2
