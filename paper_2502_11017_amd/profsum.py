"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2502_11017_amd.profsum stats   STATS_CSV [--top N] [--match TEXT]
    python -m paper_2502_11017_amd.profsum traffic FETCH_CSV WRITE_CSV --kernel NAME
           --copy-bytes N --source FILE [--workload TEXT] [--command TEXT ...]
           [--last N] [--bench-line FILE]

``stats`` prints the kernel table of a ``--kernel-trace --stats`` run
(calls, total and average duration per kernel).

``traffic`` turns two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs into
HBM bytes per launch of one kernel and prints them as JSON.  Both counters
are reported in KiB per dispatch; each is scaled by what it reads for the
largest device copy in the same run (a plain copy of ``--copy-bytes`` read
and written), so the figures are in bytes actually moved.  With ``--last``
only the final N dispatches count (the timed step of a bench run), and
``--bench-line`` adds that run's algorithmic bytes per launch of the same
launches for the ratio.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def kernel_stats(path, top=25, match=None):
    """Kernel table; with ``match`` only kernels whose name contains it, the
    others folded into one line."""
    rows = _rows(path)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    rest = []
    if match:
        rest = [r for r in rows if match not in r["Name"]]
        rows = [r for r in rows if match in r["Name"]]
    out = [f"{'kernel':<70} {'calls':>7} {'total ms':>10} {'avg us':>10} {'share':>7}"]
    for r in rows[:top]:
        name = r["Name"]
        name = name if len(name) <= 70 else name[:67] + "..."
        out.append(f"{name:<70} {int(r['Calls']):>7} {float(r['TotalDurationNs']) / 1e6:>10.3f} "
                   f"{float(r['AverageNs']) / 1e3:>10.2f} {float(r['TotalDurationNs']) / total:>7.1%}")
    if rest:
        rt = sum(float(r["TotalDurationNs"]) for r in rest)
        out.append(f"{'other kernels (not matching ' + repr(match) + ')':<70} "
                   f"{sum(int(r['Calls']) for r in rest):>7} {rt / 1e6:>10.3f} {'':>10} {rt / total:>7.1%}")
    out.append(f"{'all kernels':<70} {sum(int(r['Calls']) for r in rows + rest):>7} {total / 1e6:>10.3f}")
    return "\n".join(out)


def _per_dispatch(path):
    """{dispatch id: (kernel name, counter sum)}; a counter is summed over its
    instances (one row per XCD or channel)."""
    d = {}
    for r in _rows(path):
        k = int(r["Dispatch_Id"])
        name, v = d.get(k, (r["Kernel_Name"], 0.0))
        d[k] = (name, v + float(r["Counter_Value"]))
    return d


def _copy_scale(d, copy_bytes, what):
    copies = [v for name, v in d.values() if "copyBuffer" in name or "copy_kernel" in name.lower()]
    if not copies:
        raise SystemExit(f"no device copy kernel in the {what} run")
    kib = max(copies)
    return copy_bytes / (kib * 1024.0), kib


def pass_traffic(fetch_csv, write_csv, kernel, copy_bytes, last=0):
    f = _per_dispatch(fetch_csv)
    w = _per_dispatch(write_csv)
    fs, fkib = _copy_scale(f, copy_bytes, "FETCH_SIZE")
    ws, wkib = _copy_scale(w, copy_bytes, "WRITE_SIZE")
    fk = [v for _, (name, v) in sorted(f.items()) if kernel in name]
    wk = [v for _, (name, v) in sorted(w.items()) if kernel in name]
    if not fk or len(fk) != len(wk):
        raise SystemExit(f"{kernel}: {len(fk)} FETCH and {len(wk)} WRITE dispatches")
    if last > 0:  # only the final `last` dispatches (the timed step of the run)
        fk, wk = fk[-last:], wk[-last:]
    n = len(fk)
    fb = sum(fk) * 1024.0 * fs / n
    wb = sum(wk) * 1024.0 * ws / n
    return {"kernel": kernel, "launches": n,
            "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
            "bytes_per_launch": fb + wb,
            "calibration": {"copy_bytes": copy_bytes, "fetch_kib_for_copy": fkib, "write_kib_for_copy": wkib,
                            "fetch_scale": fs, "write_scale": ws}}


def main(argv=None):
    ap = argparse.ArgumentParser(prog="profsum")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=25)
    s.add_argument("--match", default=None)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--source", required=True)
    t.add_argument("--workload", default="")
    t.add_argument("--command", action="append", default=[])
    t.add_argument("--last", type=int, default=0, help="average over the final N dispatches only")
    t.add_argument("--bench-line", default=None,
                   help="file holding the bench JSON line of the same run (its algorithmic bytes per launch)")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(kernel_stats(a.csv, a.top, a.match))
        return 0
    rec = pass_traffic(a.fetch_csv, a.write_csv, a.kernel, a.copy_bytes, a.last)
    if a.bench_line:
        with open(a.bench_line) as f:
            line = [ln for ln in f if ln.startswith("{")][-1]
        roof = json.loads(line)["roofline"]
        rec["algorithmic_bytes_per_launch_same_launches"] = roof["algorithmic_bytes_per_launch"]
        rec["traffic_over_algorithmic"] = rec["bytes_per_launch"] / roof["algorithmic_bytes_per_launch"]
    with open(a.source, "rb") as f:
        rec["source"] = os.path.relpath(a.source)
        rec["source_sha256_16"] = hashlib.sha256(f.read()).hexdigest()[:16]
    rec["workload"] = a.workload
    rec["commands"] = a.command
    json.dump(rec, sys.stdout, indent=1)
    print()
    return 0


if __name__ == "__main__":
    sys.exit(main())
