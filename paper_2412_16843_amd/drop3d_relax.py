"""Three-dimensional drop relaxation on a wall (GPU).

A half ball of fluid 1 (density ratio 10) sits on the bottom wall of a
periodic box and relaxes toward the spherical cap of the same volume that
meets the wall at theta_eq, driven by the GNBC slip with the in-plane
curvature kappa_p (Model 4A by default).  Printed at each output time: the
contact radius a (from the wetted area of the wall phase field, a =
sqrt(A/pi), A = h^2 sum phi_w), the cap angle implied by a and the drop
volume, the equal-volume equilibrium radius a_eq, the largest slip and the
mass drift.

    python -m paper_2412_16843_amd.drop3d_relax --n 64 --t-end 8 --outputs 16
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import workloads as W  # noqa: E402


def cap_volume(a: float, theta: float) -> float:
    """Volume of a spherical cap with contact radius a and contact angle theta."""
    c, s = math.cos(theta), math.sin(theta)
    return math.pi * a ** 3 * (2.0 - 3.0 * c + c ** 3) / (3.0 * s ** 3)


def cap_angle(a: float, volume: float) -> float:
    """Contact angle of the cap with contact radius a and the given volume
    (bisection on (0, pi); the volume grows with the angle)."""
    lo, hi = 1e-6, math.pi - 1e-6
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if cap_volume(a, mid) < volume:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def contact_radius(phi: np.ndarray, h: float) -> float:
    phw = np.clip(0.5 * (3.0 * phi[:, 0] - phi[:, 1]), 0.0, 1.0)
    return math.sqrt(h * h * phw.sum() / math.pi)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--theta", type=float, default=60.0)
    ap.add_argument("--model", default="4A")
    ap.add_argument("--t-end", type=float, default=8.0)
    ap.add_argument("--outputs", type=int, default=16)
    ap.add_argument("--max-seconds", type=float, default=600.0)
    a = ap.parse_args(argv)
    from paper_2412_16843_amd.solver3 import CDISolver3
    n = a.n
    case = W.drop3_case(n, n // 2, n, theta_eq_deg=a.theta, ratio=10.0, r0=0.35)
    p = case.params.replace(slip_model=a.model)
    h = p.h
    vol = float(case.phi0.sum()) * h ** 3
    theta = math.radians(a.theta)
    a_eq = (3.0 * vol / (math.pi * (2.0 - 3.0 * math.cos(theta) + math.cos(theta) ** 3))) ** (1 / 3) \
        * math.sin(theta)
    s = CDISolver3(p, case.phi0, rtol=1e-10)
    steps_total = int(round(a.t_end / p.dt))
    per = max(1, steps_total // a.outputs)
    t0 = time.time()
    print(json.dumps({"n": n, "dt": p.dt, "steps": steps_total, "volume": vol, "a_eq": a_eq,
                      "theta_eq_deg": a.theta, "model": a.model}), flush=True)
    done = 0
    while done < steps_total and time.time() - t0 < a.max_seconds:
        k = min(per, steps_total - done)
        s.step(k)
        done += k
        d = s.diagnostics()
        st = s.state()
        rc = contact_radius(st["phi"], h)
        print(json.dumps({"t": round(d["t"], 4), "a": rc, "a_over_a_eq": rc / a_eq,
                          "theta_deg": math.degrees(cap_angle(rc, d["mass"])),
                          "max_slip": max(d["max_slip_bot"], d["max_slip_top"]),
                          "mass_drift": abs(d["mass"] - vol) / vol, "cg_iters": d["last_iters"],
                          "wall_s": round(time.time() - t0, 1)}), flush=True)
    s.close()


if __name__ == "__main__":
    main()
