"""Spurious slip of the eight slip models on the prescribed equilibrium
field, under mesh refinement (Sec. 3.1).

The prescribed drop of Sec. 3.1 (radius 0.15 half disc on the bottom wall of
a 1 x 0.5 channel, tanh profile of a circular cap at theta = theta_eq) is an
exact equilibrium of the sharp-interface problem, so any u^Y the discrete
wall routine returns on it is spurious.  The interface thickness follows
eps = C h^(2/3) with C = 0.175, i.e. eps / h from 0.7 at Nx = 64 to 1.4 at
Nx = 512 (the paper's range): eps -> 0 while the interface is resolved by
more cells.  For each resolution and model the study evaluates u^Y with the
library's stage operator (cdi_eval_rhs, the GPU kernels) and reports
max |u^Y| and its convergence rate between resolutions (the GPU values are
compared with the oracle at every resolution of the study in
tests/test_gpu_parity.py).  Models 3A/3B/4A/4B carry the
curvature correction and vanish in the continuum limit; Models 1A/1B/2A/2B
keep a model error (Sec. 3.1).

    python -m paper_2412_16843_amd.slip_mesh_study --nx 64 128 256 512

prints one line per resolution and a JSON line at the end.
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np

import workloads as W

EPS_COEF = 0.175
R0, LX, LY = 0.15, 1.0, 0.5


def prescribed(nx: int, theta_deg: float, model: str):
    """Parameters and phase field of the prescribed equilibrium drop at Nx."""
    h = LX / nx
    eps = EPS_COEF * h ** (2.0 / 3.0)
    c = W.drop_case(nx, nx // 2, theta_deg, 1.0, lx=LX, ly=LY, r0=R0)
    p = c.params.replace(eps=eps, slip_model=model)
    phi = W.drop_phi(nx, nx // 2, LX, LY, R0, math.radians(theta_deg), eps)
    return p, phi


def run(nxs=(64, 128, 256, 512), theta_deg: float = 60.0, verbose: bool = True) -> dict:
    from paper_2412_16843_amd.solver import CDISolver
    out = {"theta_deg": theta_deg, "eps_coef": EPS_COEF, "nx": list(nxs), "models": {}}
    for model in W.SLIP_MODELS:
        rows = []
        for nx in nxs:
            p, phi = prescribed(nx, theta_deg, model)
            s = CDISolver(p, phi)
            uy = s.eval_rhs()[3].cpu().numpy()[0]     # bottom wall corners
            s.close()
            row = {"nx": nx, "eps_over_h": round(p.eps / p.h, 4),
                   "max_uY": float(np.abs(uy).max())}
            rows.append(row)
        for a, b in zip(rows, rows[1:]):
            b["rate"] = math.log2(a["max_uY"] / b["max_uY"]) if b["max_uY"] > 0 else None
        out["models"][model] = rows
        if verbose:
            print(model, " ".join(f"Nx {r['nx']}: {r['max_uY']:.3e}"
                                  + (f" (rate {r['rate']:.2f})" if r.get("rate") else "")
                                  for r in rows), flush=True)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--nx", type=int, nargs="+", default=[64, 128, 256, 512])
    ap.add_argument("--theta", type=float, default=60.0)
    a = ap.parse_args(argv)
    print(json.dumps(run(a.nx, a.theta)), flush=True)


if __name__ == "__main__":
    main()
