"""Text summaries of rocprofv3 output, as committed under profiles/.

    python -m paper_1805_10164_amd.profiling stats KERNEL_STATS_CSV --command CMD
        per-kernel calls, total / average / min / max duration and share of GPU time.

    python -m paper_1805_10164_amd.profiling valu COUNTERS_CSV --command CMD [--work K=UNITS]
        per-kernel averages of the SQ / GRBM counters of one --pmc run, with the VALU issue
        fraction SQ_ACTIVE_INST_VALU * 4 / (SIMDs * GRBM_GUI_ACTIVE per XCD) and, for kernels
        given a work count, VALU lane-instructions per unit of work.

    python -m paper_1805_10164_amd.profiling traffic --fetch COUNTERS_CSV --write COUNTERS_CSV
        --calib-mib M --kernel NAME --source FILE [--command-fetch CMD --command-write CMD]
        [--grid-size ITEMS] [--match SHORT_NAME_PREFIX]
        HBM bytes per launch of kernel NAME from a FETCH_SIZE run and a WRITE_SIZE run (KiB per
        dispatch).  Each counter is scaled by what it reads for the plain copy dispatch of the
        same run (a negation that reads and writes M MiB, see bench.py --calib-copy-mb), so the
        result is in bytes actually moved.  The JSON records the source file's SHA-256; bench.py
        uses the figure only while the source is unchanged.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CALIB_KERNEL = "neg_kernel"


def short_name(name: str) -> str:
    n = name.split("(")[0].replace("mcnegf::", "").replace("void ", "")
    return n[:44]


def stats(path: str, command: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = [f"# command: {command}", f"# source: {os.path.basename(path)}",
           f"{'kernel':44s} {'calls':>5s} {'total_ms':>9s} {'avg_us':>10s} {'min_us':>10s} "
           f"{'max_us':>10s} {'pct':>6s}"]
    for r in rows:
        out.append(f"{short_name(r['Name']):44s} {int(r['Calls']):5d} "
                   f"{int(r['TotalDurationNs']) / 1e6:9.3f} {float(r['AverageNs']) / 1e3:10.1f} "
                   f"{int(r['MinNs']) / 1e3:10.1f} {int(r['MaxNs']) / 1e3:10.1f} "
                   f"{float(r['Percentage']):6.2f}")
    return "\n".join(out) + "\n"


SIMDS = 256 * 4  # compute units x SIMDs per CU
XCDS = 8


def valu(path: str, command: str, work=None) -> str:
    """Per-kernel averages of every counter in a --pmc CSV plus the VALU issue fraction.
    GRBM_GUI_ACTIVE is summed over the XCDs, so one XCD's busy cycles are its 1/XCDS."""
    per = {}
    for r in csv.DictReader(open(path)):
        k = short_name(r["Kernel_Name"])
        d = per.setdefault(k, {})
        d.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    out = [f"# command: {command}", f"# source: {os.path.basename(path)}",
           "# valu_issue = SQ_ACTIVE_INST_VALU * 4 / (1024 SIMDs * GRBM_GUI_ACTIVE / 8 XCDs)"]
    names = sorted({c for d in per.values() for c in d})
    out.append(f"{'kernel':44s} " + " ".join(f"{c:>20s}" for c in names) + f" {'valu_issue':>10s}")
    for k, d in per.items():
        avg = {c: sum(v) / len(v) for c, v in d.items()}
        line = f"{k:44s} " + " ".join(f"{avg.get(c, float('nan')):20.4g}" for c in names)
        g = avg.get("GRBM_GUI_ACTIVE", 0.0)
        a = avg.get("SQ_ACTIVE_INST_VALU")
        line += f" {a * 4 / (SIMDS * g / XCDS):10.3f}" if g and a is not None else f" {'-':>10s}"
        out.append(line)
    for k, units in (work or {}).items():
        d = per.get(k)
        if d and "SQ_INSTS_VALU" in d:
            v = sum(d["SQ_INSTS_VALU"]) / len(d["SQ_INSTS_VALU"])
            out.append(f"# {k}: {v * 64 / units:.1f} VALU lane-instructions per unit "
                       f"({units:.4g} units per launch)")
    return "\n".join(out) + "\n"


def _counter(path: str, counter: str, grid_size=None):
    """(values of kernel dispatches by short name, calibration value) for one counter; with
    grid_size, only dispatches of that many work-items (one workload of a multi-workload run)."""
    per, calib = {}, None
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        v = float(r["Counter_Value"])
        if CALIB_KERNEL in r["Kernel_Name"]:
            calib = v
            continue
        if grid_size is not None and int(r["Grid_Size"]) != int(grid_size):
            continue
        per.setdefault(short_name(r["Kernel_Name"]), []).append(v)
    return per, calib


def traffic(fetch_csv, write_csv, calib_mib, kernel, source, cmd_fetch="", cmd_write="",
            grid_size=None, match=None):
    fetch, cf = _counter(fetch_csv, "FETCH_SIZE", grid_size)
    write, cw = _counter(write_csv, "WRITE_SIZE", grid_size)
    if cf is None or cw is None:
        raise SystemExit("calibration dispatch not found in the counter files")
    if match:  # a short-name prefix that picks one template instance
        key = next((k for k in fetch if k.startswith(match)), None)
    else:
        key = next((k for k in fetch if k.split("<")[0] == kernel), None)
    if key is None or key not in write:
        raise SystemExit(f"kernel {kernel} not found in the counter files")
    known_kib = calib_mib * 1024.0
    fs, ws = known_kib / cf, known_kib / cw
    f, w = fetch[key], write[key]
    per_launch = [1024.0 * (a * fs + b * ws) for a, b in zip(f, w)]
    src = os.path.join(ROOT, source)
    return {
        "kernel": kernel,
        "source": source,
        "source_sha256": hashlib.sha256(open(src, "rb").read()).hexdigest(),
        "fetch_kib_per_dispatch": f,
        "write_kib_per_dispatch": w,
        "calibration": {"copy_mib_read_and_written": calib_mib, "fetch_kib_read": cf,
                        "write_kib_read": cw, "fetch_scale": fs, "write_scale": ws},
        "hbm_bytes_per_dispatch": per_launch,
        "hbm_bytes_per_launch": sum(per_launch) / len(per_launch),
        "dispatch": {"short_name": key, "grid_size": grid_size},
        "commands": {"fetch": cmd_fetch, "write": cmd_write},
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--command", default="")
    v = sub.add_parser("valu")
    v.add_argument("csv")
    v.add_argument("--command", default="")
    v.add_argument("--work", action="append", default=[],
                   help="SHORT_NAME=UNITS_PER_LAUNCH (e.g. walk steps of one launch)")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--calib-mib", type=float, required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--source", required=True)
    t.add_argument("--command-fetch", default="")
    t.add_argument("--command-write", default="")
    t.add_argument("--grid-size", type=int, default=None,
                   help="only dispatches of this many work-items")
    t.add_argument("--match", default=None, help="short-name prefix of the dispatches")
    a = ap.parse_args(argv)
    if a.what == "stats":
        sys.stdout.write(stats(a.csv, a.command))
    elif a.what == "valu":
        work = {w.split("=")[0]: float(w.split("=")[1]) for w in a.work}
        sys.stdout.write(valu(a.csv, a.command, work))
    else:
        rec = traffic(a.fetch, a.write, a.calib_mib, a.kernel, a.source, a.command_fetch,
                      a.command_write, a.grid_size, a.match)
        json.dump(rec, sys.stdout, indent=1)
        sys.stdout.write("\n")


if __name__ == "__main__":
    main()
