"""The two-phase Couette flow of Sec. 5.2 run to steady state on the GPU.

The slab of fluid 1 between Lx/4 and 3Lx/4 is sheared by walls moving at +U
(top) and -U (bottom); its four contact lines move until the slip of the
generalized Navier boundary condition balances the wall motion.  At steady
state each contact line is at rest, so the wall velocity there vanishes:
u_wall = U_wall + u_slip = 0, i.e. the slip at the contact line equals
-U_wall.  The run reports the four contact-line positions (phi = 1/2
crossings of the wall value extrapolated from the first two rows, from the
library's device diagnostics), their drift over the last output interval and
the wall velocity at each of them.  On each wall the slab of fluid 1 gives
two crossings; in column order the first is where phi rises through 1/2
(the slab's left edge) and the second where it falls.

    python -m paper_2412_16843_amd.couette_steady --variant asymmetric --t-end 600
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

import workloads as W


def sample(x: float, f: np.ndarray, h: float) -> float:
    """Linear interpolation at position x of a periodic array whose entry i
    sits at x = i h (the wall corners)."""
    n = f.size
    s = x / h
    i = int(np.floor(s)) % n
    t = s - np.floor(s)
    return float((1 - t) * f[i] + t * f[(i + 1) % n])


def run(variant: str, nx: int, t_end: float, outputs: int, gamma_factor: float) -> dict:
    from paper_2412_16843_amd.solver import CDISolver
    case = W.paper_couette_case(variant, nx)
    p = case.params
    if gamma_factor > 0:   # the paper's gamma = 2.5 |u|_max, bounded by 2.5 x 2 U
        p = p.replace(gamma=2.0 * p.gamma, gamma_factor=gamma_factor, dt=0.0)
        p = p.replace(dt=W.dt_from_cfl(p))
    h = p.h
    s = CDISolver(p, case.phi0, rtol=1e-10)
    s.tune()
    per = max(1, int(round(t_end / outputs / p.dt)))
    t0 = time.perf_counter()
    prev = None
    for k in range(outputs):
        s.step(per)
        d = s.diagnostics()
        pos = np.array(d["contact_x_bot"] + d["contact_x_top"])
        drift = float(np.abs(pos - prev).max()) if prev is not None and pos.shape == prev.shape else None
        prev = pos
        print(f"{variant} t {(k + 1) * per * p.dt:8.2f} contact lines {np.round(pos, 3).tolist()} "
              f"drift {drift} {time.perf_counter() - t0:.0f} s", flush=True)
    # wall velocity u_wall = U + u_slip at each contact line (u_slip from the
    # solver's wall values; the GNBC wall velocity of a corner is U + u_slip)
    slip = s.eval_rhs()[4].cpu().numpy()        # [2][nx]: bottom, top corner slip
    d = s.diagnostics()
    s.close()
    res = {"variant": variant, "nx": nx, "ny": nx // 8, "t": outputs * per * p.dt,
           "steps": outputs * per, "gamma_factor": gamma_factor,
           "contact_lines": {}, "last_drift": drift,
           "mass_drift": abs(d["mass"] - d["mass0"]) / d["mass0"],
           "phi_min": d["phi_min"], "phi_max": d["phi_max"]}
    for wall, U, row in (("bot", p.u_wall_bot, 0), ("top", p.u_wall_top, 1)):
        xs = d[f"contact_x_{wall}"]
        for name, x in zip(("rising", "falling"), xs):
            # the slip array is indexed by wall corner, corner i at x = i h
            us = sample(x, slip[row], h)
            res["contact_lines"][f"{wall}_{name}_{x:.3f}"] = {
                "x": x, "u_slip": us, "u_wall": U + us}
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--variant", default="asymmetric", choices=["symmetric", "asymmetric"])
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--t-end", type=float, default=600.0)
    ap.add_argument("--outputs", type=int, default=12)
    ap.add_argument("--gamma-factor", type=float, default=2.5)
    a = ap.parse_args(argv)
    print(json.dumps(run(a.variant, a.nx, a.t_end, a.outputs, a.gamma_factor)), flush=True)


if __name__ == "__main__":
    main()
