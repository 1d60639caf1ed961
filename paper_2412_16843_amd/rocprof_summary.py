"""Summaries of rocprofv3 output for the profiles/ folder.

Two uses:

  kernel statistics (``--kernel-trace --stats`` run), per kernel and per
  (kernel, grid size):
      python -m paper_2412_16843_amd.rocprof_summary stats <run>_kernel_stats.csv
      python -m paper_2412_16843_amd.rocprof_summary grid <run>_kernel_trace.csv

  instruction counters per launch of the kernels whose name contains a
  string (any number of ``--pmc`` runs of the same command):
      python -m paper_2412_16843_amd.rocprof_summary counters --kernel k_stage \\
          <pass1>_counter_collection.csv <pass2>_counter_collection.csv ...

  HBM traffic per launch (two ``--pmc`` runs of the same command, one with
  FETCH_SIZE, one with WRITE_SIZE; each must also run a plain device copy of
  known size, which bench.py does with ``--copy-calibration``):
      python -m paper_2412_16843_amd.rocprof_summary traffic \\
          <fetch>_counter_collection.csv <write>_counter_collection.csv \\
          --kernel k_mg_coarse --copy-bytes 268435456 --workload couette256x64

The traffic record ends with one JSON line (``traffic-record: {...}``) that
bench.py reads back to fill ``roofline.traffic`` as long as the kernels are
unchanged (sha256 over the device-code headers, stored in the record).
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def source_hash() -> str:
    """sha256 over the two-dimensional solver's device code: its kernels live
    in the csrc/*.h headers (the .hip files hold host code only); the
    network's (net_*.h) and the three-dimensional path's (cdi3_*.h) headers
    are left out, their kernels are not in these records."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith(".h") and not name.startswith(("net_", "cdi3_")) and name != "host_util.h":
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode())
                h.update(f.read())
    return h.hexdigest()


def _short(name: str) -> str:
    base = name.split("(")[0]
    return base.replace("void ", "").replace("cdi::", "")


def stats(path: str, top: int = 20) -> str:
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | total (ms) | average (us) | min (us) | max (us) | share (%) |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        out.append("| `{}` | {} | {:.2f} | {:.2f} | {:.2f} | {:.2f} | {:.2f} |".format(
            _short(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e6,
            float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
            float(r["Percentage"])))
    return "\n".join(out)


def by_grid(trace_csv: str, top: int = 24) -> str:
    """Per (kernel, grid size) launch durations from a --kernel-trace CSV: the
    multigrid kernels run once per level, so the level-0 launches (largest
    grid) are the ones a kernel family of bench.py times."""
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(trace_csv)):
        grid = r.get("Grid_Size") or r.get("Grid_Size_X")
        agg[(_short(r["Kernel_Name"]), int(grid))].append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out = ["| kernel | grid | calls | total (ms) | average (us) | min (us) | max (us) |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for (name, grid), d in sorted(agg.items(), key=lambda kv: -sum(kv[1]))[:top]:
        out.append("| `{}` | {} | {} | {:.2f} | {:.2f} | {:.2f} | {:.2f} |".format(
            name, grid, len(d), sum(d) / 1e3, sum(d) / len(d), min(d), max(d)))
    return "\n".join(out)


def _per_kernel(path: str):
    """(kernel short name, grid size) -> list of counter values (KiB)."""
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        agg[(_short(r["Kernel_Name"]), int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    return agg


def _copy_value(agg, copy_bytes: int):
    """Counter value (KiB) of the largest plain copy in the run."""
    best = None
    for (name, grid), vals in agg.items():
        if "copyBuffer" in name or "copy" in name.lower():
            v = max(vals)
            if best is None or v > best:
                best = v
    if best is None:
        raise SystemExit("no copy kernel found in the counter run")
    return best


def traffic(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: int, workload: str):
    fa, wa = _per_kernel(fetch_csv), _per_kernel(write_csv)
    kib = copy_bytes / 1024.0
    f_scale = kib / _copy_value(fa, copy_bytes)
    w_scale = kib / _copy_value(wa, copy_bytes)
    lines = [f"Calibration: a device copy of {copy_bytes} bytes reads FETCH_SIZE x {f_scale:.3f} "
             f"and WRITE_SIZE x {w_scale:.3f} of its true bytes (both counters in KiB).", "",
             "| kernel | grid | launches | read (KiB/launch, scaled) | write (KiB/launch, scaled) |",
             "|---|---:|---:|---:|---:|"]
    rec = None
    for key in sorted(fa, key=lambda k: -sum(fa[k])):
        name, grid = key
        if "cdi" not in key[0] and not name.startswith("k_"):
            continue
        fv = sum(fa[key]) / len(fa[key]) * f_scale
        wv = (sum(wa[key]) / len(wa[key]) * w_scale) if key in wa else float("nan")
        lines.append(f"| `{name}` | {grid} | {len(fa[key])} | {fv:.1f} | {wv:.1f} |")
        if kernel in name and (rec is None or grid > rec["grid"]):
            rec = dict(grid=grid, read=fv * 1024.0, write=wv * 1024.0)
    if rec is None:
        raise SystemExit(f"kernel {kernel} not found")
    record = {"workload": workload, "kernel": kernel, "grid": rec["grid"],
              "read_bytes_per_launch": round(rec["read"]), "write_bytes_per_launch": round(rec["write"]),
              "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
              "src_sha256": source_hash()}
    lines += ["", "traffic-record: " + json.dumps(record)]
    return "\n".join(lines)


def counters(paths, kernel: str) -> str:
    """Mean of every counter per launch of each kernel matching `kernel`, and
    the issue shares they imply.  SQ_WAVE_CYCLES, SQ_ACTIVE_INST_* and
    SQ_WAIT_* count quad-cycles (4 clocks) summed over waves; GRBM_GUI_ACTIVE
    counts clocks summed over the 8 XCDs; the MI355X has 1024 SIMDs."""
    tot = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(lambda: collections.defaultdict(set))
    for path in paths:
        for r in csv.DictReader(open(path)):
            name = _short(r["Kernel_Name"])
            if kernel not in name:
                continue
            c = r["Counter_Name"]
            tot[name][c] += float(r["Counter_Value"])
            disp[name][c].add((path, r["Dispatch_Id"]))
    lines = []
    for name in sorted(tot):
        per = {c: v / max(len(disp[name][c]), 1) for c, v in tot[name].items()}
        n = max(len(d) for d in disp[name].values())
        lines += [f"### `{name}` ({n} launches per pass)", "", "| counter | per launch |", "|---|---:|"]
        lines += [f"| {c} | {v:.4g} |" for c, v in sorted(per.items())]
        if "GRBM_GUI_ACTIVE" in per:
            clocks = per["GRBM_GUI_ACTIVE"] / 8.0
            lines += ["", f"- kernel clocks (GRBM_GUI_ACTIVE / 8 XCDs): {clocks:.4g}"]
            simd = clocks * 1024
            for c, what in (("SQ_ACTIVE_INST_VALU", "VALU busy"),
                            ("SQ_ACTIVE_INST_ANY", "instruction issue (all types, summed over waves)"),
                            ("SQ_WAIT_ANY", "waves waiting (summed over waves)")):
                if c in per:
                    lines.append(f"- {what}: {4 * per[c] / simd:.3f} of SIMD clocks")
            if "SQ_WAVE_CYCLES" in per:
                lines.append(f"- resident waves per SIMD: {4 * per['SQ_WAVE_CYCLES'] / simd:.2f}")
        lines.append("")
    if not lines:
        raise SystemExit(f"kernel {kernel} not found")
    return "\n".join(lines)


def read_record(path: str):
    """The traffic record of a summary file, or None."""
    try:
        for line in open(path):
            if line.startswith("traffic-record: "):
                return json.loads(line[len("traffic-record: "):])
    except OSError:
        return None
    return None


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=20)
    gsub = sub.add_parser("grid")
    gsub.add_argument("trace_csv")
    gsub.add_argument("--top", type=int, default=24)
    cs = sub.add_parser("counters")
    cs.add_argument("csv", nargs="+")
    cs.add_argument("--kernel", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--workload", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats(a.csv, a.top))
    elif a.cmd == "grid":
        print(by_grid(a.trace_csv, a.top))
    elif a.cmd == "counters":
        print(counters(a.csv, a.kernel))
    else:
        print(traffic(a.fetch_csv, a.write_csv, a.kernel, a.copy_bytes, a.workload))


if __name__ == "__main__":
    sys.exit(main())
