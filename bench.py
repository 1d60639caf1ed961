#!/usr/bin/env python3
"""Throughput of the CDI + GNBC time step on one MI355X.

One "step" is one full RK4 time step of every instance of the workload: 4
stage evaluations (fused phase-field preparation, CDI-flux / momentum / GNBC
stage kernel, projection right-hand side) and 4 variable-density pressure
projections by multigrid-preconditioned flexible CG to a relative residual of
1e-10.  The default workload is the seeded 64-instance ensemble of uneven
drop and Couette grids (128x64 .. 512x256, 3.9 M cells), FP64, over its
1000-step run: the largest single-GPU configuration of the benchmark set.
The instances are split into four batched contexts of nearly equal size, one
stream each, advanced together (cdi_step_concurrent) with one tiled shape
tuned under concurrency (cdi_tune_concurrent): one context's kernels fill the
GPU while another waits on its latency-bound phases.  The same
instances in one context are timed beside it (single_context).

Prints one JSON line:
  metric/value/unit       Mcell-steps/s = sum over instances of nx * ny *
                          steps / wall time / 1e6, inputs resident in HBM,
                          timed between two device synchronisations with no
                          per-kernel instrumentation
  step_roofline           the whole step's algorithmic bytes (stages,
                          projections and every CG iteration each instance
                          ran in the timed steps, cdi_cg_iterations) over
                          the timed wall time, against 8 TB/s
  roofline                the bandwidth-bound kernel family with the most
                          device time: its algorithmic bytes per launch over
                          its average launch time (start / end timestamps of
                          its own launches, taken in a separate pass on the
                          library stream), against the 8 TB/s HBM peak
  dominant_kernel         the family with the most device time overall and its
                          share (the one-block coarse cycle, when it leads,
                          is bound by barrier latency, not bandwidth)
  kernel_time_ms_per_step device time per step of every kernel family
  poisson_learned_vs_plain  pressure time to solution at 1e-10 on the
                          2048x1024 ratio-10 grid: zero guess, previous
                          pressure and the learned guess
  cpu_baseline            the FP64 CPU oracle on a bounded sample of the same
                          workload on this host (all cores, and one thread)
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per cell and launch of each kernel family (FP64
# path): every array element the kernel must read or write, counted once.
ALGO_BYTES_PER_CELL = {
    # the stage kernel with the phase preparation fused in: stage phi, u, v;
    # base phi, u, v; RK accumulators read+write (stages 1-2), next phi and
    # (rho u)* written: mean over the 4 stages (n, mu_c and the wall values
    # are formed in LDS)
    "stage": (72 + 120 + 120 + 96) / 4,
    # (rho u)*, next phi read; u*, v*, b, a_x, a_y written
    "rhs": 3 * 8 + 5 * 8,
    # CG step fused in (x, d, r, q read; x, r written), then r, a_x, a_y read,
    # z written, coarse r written (1/4 cell); counted for level 0
    "mg_down": 4 * 8 + 2 * 8 + 2 * 8 + 8 + 2,
    # r, a_x, a_y, z, q read, coarse z (1/4); z written
    "mg_up": 5 * 8 + 2 + 8,
    # z, d_old, a_x, a_y, r read; d, q written
    "pcg_spmv": 5 * 8 + 2 * 8,
    # u*, v*, x, a_x, a_y read; u, v, p written; the stage's slot of the
    # pressure-history ring written; final stage only: next phi copied (1/4)
    "project": 5 * 8 + 3 * 8 + 8 + 16 / 4,
    # b, guess (four history fields: cubic extrapolation), a_x, a_y read; x,
    # r written
    "pcg_init": 7 * 8 + 2 * 8,
}

# every family the library can time (cdi_timing_enable)
FAMILIES = ("stage", "rhs", "pcg_init", "pcg_spmv", "mg_down", "mg_down_other",
            "mg_coarse", "mg_up", "mg_up_other", "mg_coef", "pcg_xmean", "project")


def mg_levels(nx: int, ny: int, coarse_cells: int = 1024):
    """Multigrid hierarchy of the library: halve while both sizes are even and
    the level has more than 64 cells; levels at or below `coarse_cells` cells
    run in the single-block coarse kernel."""
    levels = [(nx, ny)]
    while nx % 2 == 0 and ny % 2 == 0 and nx * ny > 64:
        nx //= 2
        ny //= 2
        levels.append((nx, ny))
    lc = next(k for k, (a, b) in enumerate(levels) if a * b <= coarse_cells)
    return levels, lc


def _coarse_bytes(p, coarse_cells: int) -> float:
    """Right-hand side of the first level the coarse kernel runs read and its
    correction written, the x- and y-face coefficients of every level from
    there read, and the dense inverse of the coarsest grid (up to 64 cells,
    uniform density only: with a variable density the coarsest grid is
    solved by CG in LDS)."""
    levels, lg = mg_levels(p.nx, p.ny, coarse_cells)
    coef = sum(a * b + a * (b + 1) for a, b in levels[lg:])
    n0 = levels[lg][0] * levels[lg][1]
    nc = levels[-1][0] * levels[-1][1]
    dense = nc * nc if (nc <= 64 and p.rho1 == p.rho2) else 0
    return 8.0 * (2 * n0 + coef + dense)


def algo_bytes_per_launch(fam: str, params, coarse_cells: int = 1024) -> float:
    """Algorithmic bytes of one launch of kernel family `fam` over every
    instance in `params` (one launch covers all instances of a batch)."""
    if not isinstance(params, (list, tuple)):
        params = [params]
    if fam in ALGO_BYTES_PER_CELL:
        return ALGO_BYTES_PER_CELL[fam] * sum(p.nx * p.ny for p in params)
    if fam == "mg_coarse":
        return sum(_coarse_bytes(p, coarse_cells) for p in params)
    raise KeyError(fam)


def traffic_record(fam: str, workload_name: str):
    """HBM bytes per launch of kernel family `fam` from the committed
    rocprofv3 --pmc summary, if it was taken on the current sources."""
    from paper_2412_16843_amd import rocprof_summary as R
    path = os.path.join(ROOT, "profiles", f"k_{fam}_{workload_name}_traffic.md")
    rec = R.read_record(path)
    if not rec or rec.get("src_sha256") != R.source_hash() or rec.get("kernel") != f"k_{fam}":
        return None
    return rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]


# algorithmic bytes per fine cell of the multigrid levels below the finest,
# per CG iteration (each level moves r, a_x, a_y in, z out and the coarse r on
# the way down, r, a_x, a_y, z in and z out on the way up: ~74 B per level
# cell, a quarter of the cells per level)
MG_COARSE_BYTES_PER_FINE_CELL = 74.0 / 3.0


def step_bytes_per_cell(iters_per_step: float) -> float:
    """Algorithmic bytes per cell of one RK4 step with `iters_per_step` CG
    iterations summed over its 4 solves."""
    b = ALGO_BYTES_PER_CELL
    per_stage = b["stage"] + b["rhs"] + b["pcg_init"] + b["project"]
    per_iter = b["pcg_spmv"] + b["mg_down"] + b["mg_up"] + MG_COARSE_BYTES_PER_FINE_CELL
    return 4 * per_stage + iters_per_step * per_iter


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def family_times(s, steps: int, families=FAMILIES):
    """Device time (ms) and launch count of every kernel family over `steps`
    steps each, one family timed at a time."""
    out = {}
    for k in families:
        s.timing_enable(k)
        s.step(steps)
        ms, n = s.timing_read()
        out[k] = (ms, n)
    s.timing_enable(None)
    return out


def hbm_case(CDISolver, nx: int = 2048, steps: int = 10):
    """Per-kernel algorithmic bandwidth on an nx x nx/2 density-ratio-10 drop
    (FP64), where the stencil and multigrid kernels are bandwidth bound, and
    the whole step's algorithmic bytes over its time."""
    import torch
    case = W.drop_case(nx, nx // 2, 60.0, 10.0, name=f"drop{nx}x{nx // 2}_r10")
    s = CDISolver(case.params, case.phi0, guess="prev", rtol=1e-10)
    s.step(3)
    out = {"workload": case.name, "peak": HBM_PEAK_GBS, "unit": "GB/s", "kernels": {}}
    probe = 2
    iters_per_step = None
    for fam in ("stage", "rhs", "pcg_init", "mg_down", "mg_up", "pcg_spmv", "project"):
        s.timing_enable(fam)
        s.step(probe)
        ms, n = s.timing_read()
        avg = ms / max(n, 1) * 1e-3
        gbs = algo_bytes_per_launch(fam, case.params) / avg / 1e9 if avg > 0 else 0.0
        out["kernels"][fam] = {"achieved": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                               "avg_launch_us": round(avg * 1e6, 2)}
        if fam == "pcg_spmv":
            iters_per_step = n / probe
    s.timing_enable(None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    cells = case.params.nx * case.params.ny
    out["mcell_steps_per_s"] = round(cells * steps / dt / 1e6, 2)
    out["steps"] = steps
    bpc = step_bytes_per_cell(iters_per_step)
    out["step"] = {"cg_iters_per_step": iters_per_step, "algo_bytes_per_cell": round(bpc, 1),
                   "achieved": round(bpc * cells * steps / dt / 1e9, 1),
                   "frac": round(bpc * cells * steps / dt / 1e9 / HBM_PEAK_GBS, 4)}
    s.close()
    return out


ENSEMBLE = "ensemble64"


def workload(name: str):
    """List of cases of a named workload (one entry for a single grid)."""
    if name in (ENSEMBLE, "config4"):
        return W.config4()
    if name in ("couette256x64", "config2"):
        return [W.config2()]
    if name in ("drop64x32", "config1"):
        return [W.config1()]
    if name.startswith("drop") and "x" in name:
        nx = int(name[4:].split("x")[0])
        return [W.drop_case(nx, nx // 2, 60.0, 10.0, steps=200, name=f"drop{nx}x{nx // 2}_r10")]
    raise SystemExit(f"unknown workload {name}")


def _cells(cases) -> int:
    return sum(c.params.nx * c.params.ny for c in cases)


def timed_rate(s, cases, steps: int):
    """Mcell-steps/s of `steps` steps, between two device synchronisations,
    with no instrumentation enabled."""
    import torch
    s.timing_enable(None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return _cells(cases) * steps / dt / 1e6, dt


def secondary_rate(CDISolver, name: str, precision: str, steps: int, warmup: int = 10,
                   tune: bool = True):
    """Throughput of another workload / precision (reported beside the headline)."""
    cases = workload(name)
    s = CDISolver([c.params for c in cases], [c.phi0 for c in cases], precision=precision,
                  guess="prev", rtol=1e-10)
    s.step(warmup)
    tuned = s.tune(trial_steps=5) if tune else None
    rate, dt = timed_rate(s, cases, steps)
    d = s.diagnostics()
    out = {"workload": name, "precision": precision, "value": round(rate, 3),
           "unit": "Mcell-steps/s", "steps": steps, "ms_per_step": round(dt / steps * 1e3, 4),
           "launch": s.get_launch(), "last_pcg_iters": d["last_iters"]}
    if tuned:
        out["tile_rows"], out["coarse_cells"] = tuned["tile_rows"], tuned["coarse_cells"]
        out["mg_smooth"] = tuned["mg_smooth"]
    s.close()
    return out


# ------------------------------------------------------- three dimensions
# Algorithmic bytes per cell of one 3-D stage-operator evaluation in its
# unfused kernel sequence (FP64): psi (phi in, psi out), phase preparation
# (phi, psi in; n, mu_c out), fluxes (phi, n, u, v, w in; three face fluxes
# and three mass fluxes out), edge stresses (phi, u, v, w in; three edge
# stresses out), momentum and RK4 (fluxes, mass fluxes, u, v, w, phi, mu_c,
# edge stresses, four accumulators, base phi, u, v, w in; four
# accumulators, next phi and three momenta out).  The per-column wall
# quantities are O(nx nz) and left out.
ALGO_BYTES_3D_STAGE = 8 * ((1 + 1) + (2 + 4) + (5 + 6) + (4 + 3) + (20 + 8))


def three_d_case(CDISolver3, nx: int = 256, steps: int = 20, warmup: int = 20):
    """3-D spherical-cap drop relaxing on the bottom wall of an nx x nx/2 x
    nx/2 periodic box (FP64, Model 4A with the in-plane curvature kappa_p,
    V(2,2) multigrid, extrapolated pressure guess): whole-step throughput
    over `steps` steps after `warmup`, CG iterations, and the stage
    operator's algorithmic bandwidth."""
    import torch
    case = W.drop3_case(nx, nx // 2, nx // 2, theta_eq_deg=60.0, ratio=10.0, r0=0.3)
    s = CDISolver3(case.params, case.phi0, rtol=1e-10)
    s.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    d = s.diagnostics()
    ms = s.time_stage(10)
    cells = nx * (nx // 2) * (nx // 2)
    gbs = ALGO_BYTES_3D_STAGE * cells / (ms * 1e-3) / 1e9
    s.close()
    return {"workload": f"drop3d{nx}x{nx // 2}x{nx // 2}_r10", "cells": cells,
            "value": round(cells * steps / dt / 1e6, 3), "unit": "Mcell-steps/s",
            "steps": steps, "warmup": warmup, "ms_per_step": round(dt / steps * 1e3, 3),
            "last_pcg_iters": d["last_iters"], "mass_drift": abs(d["mass"] - case.phi0.sum() * case.params.h ** 3),
            "stage": {"ms": round(ms, 4), "algo_bytes_per_cell": ALGO_BYTES_3D_STAGE,
                      "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(gbs / HBM_PEAK_GBS, 4)}}


# ----------------------------------------------------------- CPU baseline
def _oracle_instance_step(args):
    """One oracle step of ensemble instance k from its initial state (CPU
    child process, one thread).  Returns (cells, seconds)."""
    k, name = args
    from oracle import cdi
    c = workload(name)[k]
    s = cdi.initial_state(c.phi0)
    t0 = time.perf_counter()
    cdi.step(s, c.params)
    return c.params.nx * c.params.ny, time.perf_counter() - t0


def _cpu_leg(name: str, workers: int, budget_s: float):
    """Child-process body of the CPU baseline: the oracle's first step of the
    workload's instances, over `workers` processes of one thread each (all
    instances), or in one thread in order until `budget_s` seconds."""
    t0 = time.perf_counter()
    n_inst = len(workload(name))
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            res = pool.map(_oracle_instance_step, [(k, name) for k in range(n_inst)],
                           chunksize=1)
        wall = time.perf_counter() - t0
        cells = sum(r[0] for r in res)
        done = n_inst
    else:
        cells, done = 0, 0
        for k in range(n_inst):
            c, _ = _oracle_instance_step((k, name))
            cells += c
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
        wall = time.perf_counter() - t0
    print(json.dumps({"cells": cells, "instances": done, "wall_s": wall}), flush=True)


def cpu_baseline(name: str, budget_s: float = 15.0):
    """The oracle as it stands (NumPy/SciPy FP64, never tuned for this),
    timed in child processes that never touch the GPU: once with one process
    per core over all of the workload's instances, once in a single thread
    on the first instances within `budget_s`.  Each instance takes one step
    from its initial state."""
    cores = min(os.cpu_count() or 1, 16)
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    legs = {}
    for workers in (cores, 1):
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-leg", name,
                            "--cpu-workers", str(workers), "--cpu-budget", str(budget_s)],
                           env=env, capture_output=True, text=True, timeout=600)
        if r.returncode != 0:
            raise RuntimeError("CPU baseline leg failed:\n" + r.stderr[-2000:])
        legs[workers] = json.loads(r.stdout.strip().splitlines()[-1])
    multi, single = legs[cores], legs[1]
    n_inst = len(workload(name))
    return dict(
        value=multi["cells"] / multi["wall_s"] / 1e6, unit="Mcell-steps/s", cores=cores,
        kind="oracle",
        sample=(f"first step of each of the {multi['instances']} instances of {name} from its "
                f"initial state, {cores} single-threaded processes ({multi['wall_s']:.1f} s wall, "
                f"NumPy/SciPy FP64)"),
        single_thread=dict(
            value=single["cells"] / single["wall_s"] / 1e6, unit="Mcell-steps/s", cores=1,
            sample=(f"first step of the first {single['instances']} of {n_inst} instances of "
                    f"{name} from their initial state, one thread ({single['wall_s']:.1f} s)")))


# ------------------------------------------------- learned vs plain Poisson
def poisson_learned_vs_plain(nx: int = 2048, train_seconds: float = 60.0, verbose: bool = False):
    """Pressure time-to-solution at relative residual 1e-10 on the 2048x1024
    density-ratio-10 grid (drop and Couette): zero guess, previous-step
    pressure and the learned guess (network inference, Galerkin fit on
    span{previous pressure, network output}, flexible CG), all on the GPU.
    The network is trained first, on the GPU, on ~10^4 snapshots the solver
    generates on the first three workloads (every step of the 64x32 drop,
    every 4th of the 256x64 Couette, one 256x256 crop of every step of the
    four 1024x512 ratio-10 drops over 2000 steps), for `train_seconds`."""
    import torch
    from paper_2412_16843_amd import learned, train_guess
    from paper_2412_16843_amd.solver import CDISolver
    ny = nx // 2
    t0 = time.perf_counter()
    data = train_guess.collect_configs(verbose=verbose)
    t_collect = time.perf_counter() - t0
    counts = {k: int(v[0].shape[0]) for k, v in data.items()}
    log(f"collected {sum(counts.values())} snapshots in {t_collect:.0f} s: {counts}")
    params, losses, iters = train_guess.train_multi(data, seconds=train_seconds, verbose=verbose)
    t_train = time.perf_counter() - t0 - t_collect
    log(f"trained {iters} iterations in {t_train:.0f} s")
    del data
    torch.cuda.empty_cache()
    rows = []
    for case in (W.config5("drop", nx), W.config5("couette", nx)):
        s = CDISolver(case.params, case.phi0, guess="prev", rtol=1e-10)
        inf = learned.GuessNet(1, ny, nx, params=params, train=False, stream=s.stream)
        s.attach_guess(inf)
        s.step(10)
        for _ in range(3):
            p_prev = s.fields[0]["p"].clone()
            s.step(1)
            rec = {}
            for mode in ("zero", "prev", "learned"):
                s.set_guess(mode)
                _, info = s.solve_last_rhs(p0=p_prev if mode != "zero" else None)
                rec[mode] = (info["iterations"], info["ms"])
            s.set_guess("prev")
            rows.append(rec)
        s.timing_enable("net")
        s.set_guess("learned")
        s.solve_last_rhs()
        net_ms, net_n = s.timing_read()
        s.timing_enable(None)
        inf.close()
        s.close()
    mean = lambda m, k: sum(r[m][k] for r in rows) / len(rows)
    first, last = train_guess.loss_summary(losses)
    return {
        "grid": f"{nx}x{ny}", "rtol": 1e-10, "solves": len(rows),
        "iters_zero": mean("zero", 0), "iters_prev": mean("prev", 0),
        "iters_learned": mean("learned", 0),
        "ms_zero": round(mean("zero", 1), 3), "ms_prev": round(mean("prev", 1), 3),
        "ms_learned": round(mean("learned", 1), 3),
        "ms_inference": round(net_ms / max(net_n, 1), 3),
        "train": {"snapshots": counts, "snapshots_total": sum(counts.values()),
                  "iters": iters, "batch": 8, "seconds": round(t_train, 1),
                  "loss_first10pct": round(first, 4), "loss_last10pct": round(last, 4),
                  "collect_s": round(t_collect, 1)},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default=ENSEMBLE)
    ap.add_argument("--groups", type=int, default=4,
                    help="contexts the headline batch is split into, stepped concurrently")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--kernel", default="auto",
                    help="kernel family for the roofline entry (auto: largest device time)")
    ap.add_argument("--launch", default="auto", choices=["auto", "tiled", "persistent"],
                    help="auto: the library's autotuner picks the launch form and tile shape")
    ap.add_argument("--tile-rows", type=int, default=0,
                    help="with --launch tiled: rows per thread of the wide-tile kernels (1 or 4)")
    ap.add_argument("--coarse-cells", type=int, default=0,
                    help="with --launch tiled: level size from which one block runs the V-cycle")
    ap.add_argument("--mg-smooth", type=int, default=0,
                    help="with --launch tiled: red-black sweep pairs per smoothing (1 or 2)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-hbm-case", action="store_true",
                    help="skip the per-kernel HBM fractions on the 2048x1024 and 8192x4096 grids")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the mixed-precision ensemble and the Couette 256x64 lines")
    ap.add_argument("--no-3d", action="store_true",
                    help="skip the 3-D drop (in-plane curvature) throughput record")
    ap.add_argument("--no-poisson", action="store_true",
                    help="skip the learned-vs-plain pressure time-to-solution at 2048x1024")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with a 256 MiB device copy (calibrates rocprofv3 --pmc byte counters)")
    ap.add_argument("--cpu-leg", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-workers", type=int, default=1, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_leg:
        _cpu_leg(args.cpu_leg, args.cpu_workers, args.cpu_budget)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library "
              "advances its instances on a single GPU and has no multi-GPU decomposition.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2412_16843_amd.solver import CDISolver, EnsembleSolver

    cases = workload(args.workload)
    params = [c.params for c in cases]
    log(f"workload {args.workload}: {len(cases)} instance(s), {_cells(cases)} cells")

    def configure(solver):
        if args.launch != "auto":
            # a fixed launch form and shape, e.g. the autotuner's pick, for
            # profiler runs (which would otherwise tune under the profiler)
            solver.set_launch(args.launch)
            if args.tile_rows:
                solver.set_tile_rows(args.tile_rows)
            if args.coarse_cells:
                solver.set_coarse_cells(args.coarse_cells)
            if args.mg_smooth:
                solver.set_mg_smooth(args.mg_smooth)

    # the headline: the batch in `groups` concurrent contexts, K steps with
    # no instrumentation
    groups = max(1, min(args.groups, len(cases)))
    head = EnsembleSolver(params, [c.phi0 for c in cases], groups=groups,
                          precision=args.precision, guess="prev", rtol=1e-10)
    for g in head.solvers:
        configure(g)
    head.step(args.warmup)
    torch.cuda.synchronize()
    head_tuned = head.tune(trial_steps=10) if args.launch == "auto" else None
    it0 = head.cg_iterations()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    head.step(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = _cells(cases) * args.steps / elapsed / 1e6
    # whole-step algorithmic bytes of the timed steps: every instance's
    # stages, projections and the CG iterations it actually ran
    it1 = head.cg_iterations()
    cells_k = [p.nx * p.ny for p in params]
    b = ALGO_BYTES_PER_CELL
    per_stage = b["stage"] + b["rhs"] + b["pcg_init"] + b["project"]
    per_iter = b["pcg_spmv"] + b["mg_down"] + b["mg_up"] + MG_COARSE_BYTES_PER_FINE_CELL
    cell_iters = sum(c * (e1 - e0) for c, e0, e1 in zip(cells_k, it0, it1))
    step_bytes = 4 * per_stage * _cells(cases) * args.steps + per_iter * cell_iters
    step_gbs = step_bytes / elapsed / 1e9
    step_roofline = {"cg_iters_per_step": round(cell_iters / (_cells(cases) * args.steps), 3),
                     "algo_bytes_per_cell_step": round(step_bytes / (_cells(cases) * args.steps), 1),
                     "achieved": round(step_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(step_gbs / HBM_PEAK_GBS, 4)}
    head_cfg = [{"instances": len(ix), "cells": sum(params[k].nx * params[k].ny for k in ix),
                 "launch": g.get_launch(), "tile_rows": g.get_tile_rows(),
                 "coarse_cells": g.get_coarse_cells(), "mg_smooth": g.get_mg_smooth(),
                 "strip_rows": g.get_strip_rows()}
                for ix, g in zip(head.groups, head.solvers)]
    head.close()
    del head
    torch.cuda.empty_cache()
    log(f"timed {args.steps} steps in {groups} concurrent context(s): "
        f"{elapsed * 1e3 / args.steps:.3f} ms/step, {value:.2f} Mcell-steps/s")

    # the same batch in one context: its rate over the same steps, then the
    # per-family device times (the roofline entry) in a separate pass
    s = CDISolver(params, [c.phi0 for c in cases], precision=args.precision, guess="prev",
                  rtol=1e-10)
    configure(s)
    s.step(args.warmup)
    torch.cuda.synchronize()
    tuned = None
    if args.launch == "auto":   # the tuner times candidates from the warmed-up state
        tuned = s.tune(trial_steps=10)
        log(f"tuned: {tuned['launch']} rows {tuned['tile_rows']} coarse {tuned['coarse_cells']} "
            f"nu {tuned['mg_smooth']}")
    single_value, single_elapsed = timed_rate(s, cases, args.steps)
    log(f"one context, {args.steps} steps: {single_elapsed * 1e3 / args.steps:.3f} ms/step, "
        f"{single_value:.2f} Mcell-steps/s")

    # separate pass: device time of every kernel family (its own launches'
    # start / end timestamps), the dominant one is the roofline entry
    probe = 5
    fam_t = family_times(s, probe)
    kernel_ms = {k: round(ms / probe, 4) for k, (ms, n) in fam_t.items() if n}
    total_dev_ms = sum(ms for ms, _ in fam_t.values())
    dominant = max(fam_t, key=lambda k: fam_t[k][0])
    fam = args.kernel
    if fam == "auto":
        # the roofline entry is the bandwidth-bound family with the most
        # device time; the one-block-per-instance coarse cycle is bound by
        # barrier latency on one CU per instance and is reported beside it
        fam = max((k for k in fam_t if k in ALGO_BYTES_PER_CELL), key=lambda k: fam_t[k][0])
    k_ms, k_n = fam_t[fam] if fam in fam_t else (0.0, 0)
    coarse_cells = s.get_coarse_cells()
    try:
        per_launch_bytes = algo_bytes_per_launch(fam, params, coarse_cells)
    except KeyError:
        per_launch_bytes = None
    avg_s = (k_ms / max(k_n, 1)) * 1e-3
    achieved = per_launch_bytes / avg_s / 1e9 if (avg_s > 0 and per_launch_bytes) else 0.0
    name = args.workload if len(cases) > 1 else cases[0].name
    iters_per_step = fam_t["pcg_spmv"][1] / probe if fam_t.get("pcg_spmv") else None
    out = {
        "metric": "Mcell-steps/s per CDI-GNBC step",
        "value": round(value, 4),
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": name, "instances": len(cases), "cells": _cells(cases),
                   "grids": (f"{min(p.nx for p in params)}x{min(p.ny for p in params)} .. "
                             f"{max(p.nx for p in params)}x{max(p.ny for p in params)}"),
                   "precision": args.precision, "poisson_rtol": 1e-10,
                   "cg_iters_per_step": iters_per_step,
                   "steps_of_run": args.warmup + args.steps,
                   "concurrent_contexts": head_cfg, "autotune": head_tuned,
                   "parallelism": "single-gpu"},
        "single_context": {"value": round(single_value, 4), "unit": "Mcell-steps/s",
                           "steps": args.steps,
                           "ms_per_step": round(single_elapsed / args.steps * 1e3, 5),
                           "launch": s.get_launch(), "tile_rows": s.get_tile_rows(),
                           "coarse_cells": coarse_cells, "mg_smooth": s.get_mg_smooth(),
                           "autotune": tuned},
        "step_roofline": step_roofline,
        "roofline": {"bound": "hbm", "kernel": fam, "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": traffic_record(fam, name),
                     "launches": k_n, "avg_launch_us": round(avg_s * 1e6, 3),
                     "algo_bytes_per_launch": per_launch_bytes,
                     "share_of_device_time": round(k_ms / max(1e-9, total_dev_ms), 4)},
        "dominant_kernel": {"kernel": dominant,
                            "bound": "latency" if dominant not in ALGO_BYTES_PER_CELL else "hbm",
                            "share_of_device_time": round(fam_t[dominant][0] / max(1e-9, total_dev_ms), 4),
                            "avg_launch_us": round(fam_t[dominant][0] / max(1, fam_t[dominant][1]) * 1e3, 3)},
        "kernel_time_ms_per_step": kernel_ms,
    }
    s.close()
    del s
    torch.cuda.empty_cache()
    if args.copy_calibration:
        n = 256 * 2**20 // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if not args.no_secondary:
        out["secondary"] = []
        if args.workload == ENSEMBLE:
            log("secondary: mixed-precision ensemble")
            out["secondary"].append(secondary_rate(CDISolver, ENSEMBLE, "mixed", 100))
        log("secondary: Couette 256x64")
        out["secondary"].append(secondary_rate(CDISolver, "couette256x64", "fp64", 400,
                                               warmup=20))
    if not args.no_hbm_case:
        # 2048x1024: ~0.5 GB of state, mostly served by the 256 MB MALL;
        # 8192x4096: ~8 GB, DRAM bound
        log("HBM cases: 2048x1024 and 8192x4096 drops")
        out["roofline_hbm_case"] = [hbm_case(CDISolver, 2048), hbm_case(CDISolver, 8192, steps=5)]
        torch.cuda.empty_cache()
    if not args.no_3d:
        from paper_2412_16843_amd.solver3 import CDISolver3
        log("3-D drop 256x128x128")
        out["three_d"] = three_d_case(CDISolver3)
        torch.cuda.empty_cache()
    if not args.no_poisson:
        log("learned vs plain pressure guess at 2048x1024")
        out["poisson_learned_vs_plain"] = poisson_learned_vs_plain()
        torch.cuda.empty_cache()
    if not args.no_cpu:
        log("CPU baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
