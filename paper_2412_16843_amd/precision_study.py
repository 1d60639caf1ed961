"""Mixed precision against FP64 on the equilibrium-drop workload.

The drop of Sec. 5.1 on a 1024 x 512 grid over 2 x 1, density and viscosity
ratio 10 (fluid 1, the drop, heavier), theta_eq in {30, 60, 120, 150} deg,
20000 steps.  The FP64 form and the mixed form (FP32 stencils and V-cycle;
FP64 phase field, phi-flux differences, CG vectors, residual and reductions)
each run the four angles in one batched context.  The FP64 GPU path is the
reference: it matches the FP64 oracle to 1e-10 per field after one step
(tests/test_gpu_config3.py), and an oracle run of 20000 steps at this size is
beyond the CPU (about 40 s per step).  At each checkpoint the study reports,
per angle and field, max |mixed - fp64| / max |fp64|, the mass drift of each
form, the relative residual of each form's last solve, and the wetted length
and cap angle of both forms (device diagnostics).

    python -m paper_2412_16843_amd.precision_study --steps 20000 --every 1000

prints one progress line per checkpoint and a JSON line at the end.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

import workloads as W

FIELDS = ("phi", "u", "v", "p")


def relerr(a: np.ndarray, b: np.ndarray) -> float:
    scale = float(np.abs(b).max())
    return float(np.abs(a - b).max() / (scale if scale > 0 else 1.0))


def run(steps: int = 20000, every: int = 1000, nx: int = 1024, thetas=W.CONFIG3_THETAS,
        verbose: bool = True) -> dict:
    from paper_2412_16843_amd.solver import CDISolver
    cases = [W.config3(th, nx=nx, steps=steps) for th in thetas]
    ps, phis = [c.params for c in cases], [c.phi0 for c in cases]
    f = CDISolver(ps, phis, rtol=1e-10)
    m = CDISolver(ps, phis, precision="mixed", rtol=1e-10)
    out = {"grid": f"{nx}x{nx // 2}", "ratio": 10, "thetas_deg": list(thetas), "steps": steps,
           "dt": ps[0].dt, "checkpoints": []}
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(every, steps - done)
        f.step(n)
        m.step(n)
        done += n
        rec = {"step": done, "t": done * ps[0].dt, "angles": {}}
        for k, th in enumerate(thetas):
            gf, gm = f.state(k), m.state(k)
            df, dm = f.diagnostics(k), m.diagnostics(k)
            rec["angles"][f"{th:.0f}"] = {
                "err": {q: relerr(gm[q], gf[q]) for q in FIELDS},
                "mass_drift_fp64": abs(df["mass"] - df["mass0"]) / df["mass0"],
                "mass_drift_mixed": abs(dm["mass"] - dm["mass0"]) / dm["mass0"],
                "relres_fp64": df["last_relres"], "relres_mixed": dm["last_relres"],
                "iters_fp64": df["last_iters"], "iters_mixed": dm["last_iters"],
                "wetted_len_fp64": df["wetted_len_bot"], "wetted_len_mixed": dm["wetted_len_bot"],
                "theta_est_fp64_deg": math.degrees(df["theta_est_bot"]),
                "theta_est_mixed_deg": math.degrees(dm["theta_est_bot"]),
                "phi_min_mixed": dm["phi_min"], "phi_max_mixed": dm["phi_max"]}
        out["checkpoints"].append(rec)
        if verbose:
            worst = {q: max(a["err"][q] for a in rec["angles"].values()) for q in FIELDS}
            drift = max(a["mass_drift_mixed"] for a in rec["angles"].values())
            print(f"step {done} worst mixed-vs-FP64 error {worst} mixed mass drift {drift:.2e} "
                  f"{time.perf_counter() - t0:.0f} s", flush=True)
    f.close()
    m.close()
    out["seconds"] = round(time.perf_counter() - t0, 1)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--out", default=None, help="also write the JSON result to this file")
    a = ap.parse_args(argv)
    r = run(a.steps, a.every, a.nx)
    s = json.dumps(r)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(s + "\n")
    print(s, flush=True)


if __name__ == "__main__":
    main()
