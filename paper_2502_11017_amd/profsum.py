"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2502_11017_amd.profsum stats   STATS_CSV [--top N] [--match TEXT]
    python -m paper_2502_11017_amd.profsum levels  TRACE_CSV [--skip N]
    python -m paper_2502_11017_amd.profsum durations TRACE_CSV
    python -m paper_2502_11017_amd.profsum mfma    COUNTER_CSV [--match TEXT] [--simds N] [--ghz F]
    python -m paper_2502_11017_amd.profsum lds     COUNTER_CSV [--match TEXT] [--cus N] [--ghz F]
    python -m paper_2502_11017_amd.profsum waits   COUNTER_CSV [--match TEXT]
    python -m paper_2502_11017_amd.profsum traffic FETCH_CSV WRITE_CSV --kernel NAME
           --copy-bytes N --source FILE [--workload TEXT] [--command TEXT ...]
           [--last N] [--bench-line FILE]

``stats`` prints the kernel table of a ``--kernel-trace --stats`` run
(calls, total and average duration per kernel).

``levels`` splits a single-stream ``--kernel-trace`` timeline of selections
into tree levels (a selection starts at its input scan ``k_amax``, a level at
``k_panel_from_A`` or ``k_merge_init``) and prints, per level and averaged
over the selections after ``--skip``, the wall time, the kernel time of the
streaming pass, the fresh-B kernel and the controller, and the gaps between
kernels (launch and host latency: wall minus kernel time).

``mfma`` reads one ``--pmc`` run of the MFMA counters
(SQ_INSTS_VALU_MFMA_MOPS_F64/_BF16/_F8, SQ_VALU_MFMA_BUSY_CYCLES,
GRBM_GUI_ACTIVE) and prints per kernel the counted MFMA flops per dispatch
(MOPS x 512), the rate over each dispatch's own duration, and the MFMA busy
share: busy cycles summed over the SIMDs divided by (duration x clock x
SIMDs), with the 2.4 GHz peak engine clock unless --ghz says otherwise.

``lds`` reads one ``--pmc`` run of SQ_INSTS_LDS_LOAD_BANDWIDTH,
SQ_LDS_IDX_ACTIVE and SQ_LDS_BANK_CONFLICT and prints per kernel the bytes
read from LDS per dispatch (64-byte units x 64), their rate over the
dispatch's duration and its share of the LDS peak (128 bytes per clock per
compute unit), and the bank-conflict share of the cycles the LDS was busy
with indexed accesses.

``waits`` reads one ``--pmc`` run of SQ_WAVE_CYCLES with SQ_WAIT_ANY,
SQ_WAIT_INST_ANY and SQ_ACTIVE_INST_* counters and prints each as a share of
the wave cycles: waiting on a wait count (memory, LDS), waiting for an
instruction to issue (dependencies, a busy matrix pipe), and issuing.

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


_CLASSES = (("k_pass", "pass"), ("k_fresh", "fresh"), ("k_ctl", "ctl"))


def _kclass(name):
    for key, cls in _CLASSES:
        if key + "<" in name or key + "(" in name:
            return cls
    return "other"


def level_table(path, skip=0):
    """Per-level averages over the selections of a single-stream trace."""
    rows = sorted(_rows(path), key=lambda r: int(r["Start_Timestamp"]))
    sels, cur_sel = [], None
    for r in rows:
        name = r["Kernel_Name"]
        if "k_amax" in name:
            cur_sel = []
            sels.append(cur_sel)
        if cur_sel is None:
            continue
        # a level starts at the leaves' panel copy or at a merge set-up (a
        # polish level's panel copy follows its merge set-up: same level)
        if ("k_panel_from_A" in name and not cur_sel) or "k_merge_init" in name:
            cur_sel.append([])
        if cur_sel:
            cur_sel[-1].append((name, int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    sels = [s for s in sels[skip:] if s]
    if not sels:
        raise SystemExit("no selection in the trace")
    nlev = min(len(s) for s in sels)
    out = [f"{len(sels)} selection(s), {nlev} levels; times in ms per selection (average)",
           f"{'level':>5} {'wall':>8} {'pass':>8} {'fresh':>8} {'ctl':>8} {'other':>8} {'gaps':>8} "
           f"{'launches':>9} {'ctl avg us':>11}"]
    tot = dict(wall=0.0, pass_=0.0, fresh=0.0, ctl=0.0, other=0.0, n=0.0, nctl=0.0)
    for lv in range(nlev):
        acc = dict(wall=0.0, pass_=0.0, fresh=0.0, ctl=0.0, other=0.0, n=0.0, nctl=0.0)
        for s in sels:
            ks = s[lv]
            # the level ends where the next one starts (the last level: its last kernel before assembly)
            acc["wall"] += (max(e for _, _, e in ks) - ks[0][1]) / 1e6
            for name, b, e in ks:
                c = _kclass(name)
                acc["pass_" if c == "pass" else c] += (e - b) / 1e6
                acc["nctl"] += c == "ctl"
            acc["n"] += len(ks)
        k = len(sels)
        a = {key: v / k for key, v in acc.items()}
        busy = a["pass_"] + a["fresh"] + a["ctl"] + a["other"]
        for key in tot:
            tot[key] += a[key]
        out.append(f"{lv:>5} {a['wall']:>8.3f} {a['pass_']:>8.3f} {a['fresh']:>8.3f} {a['ctl']:>8.3f} "
                   f"{a['other']:>8.3f} {a['wall'] - busy:>8.3f} {a['n']:>9.0f} "
                   f"{1e3 * a['ctl'] / max(1.0, a['nctl']):>11.1f}")
    busy = tot["pass_"] + tot["fresh"] + tot["ctl"] + tot["other"]
    out.append(f"{'all':>5} {tot['wall']:>8.3f} {tot['pass_']:>8.3f} {tot['fresh']:>8.3f} {tot['ctl']:>8.3f} "
               f"{tot['other']:>8.3f} {tot['wall'] - busy:>8.3f} {tot['n']:>9.0f} "
               f"{1e3 * tot['ctl'] / max(1.0, tot['nctl']):>11.1f}")
    return "\n".join(out)


def duration_table(path, names=("k_pass", "k_fresh", "k_ctl")):
    """Percentiles (p10, p50, p90, max; us) of the per-launch durations of
    the named kernels in a --kernel-trace CSV."""
    d = {k: [] for k in names}
    for r in _rows(path):
        for k in names:
            if k + "<" in r["Kernel_Name"] or k + "(" in r["Kernel_Name"]:
                d[k].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out = []
    for k in names:
        v = sorted(d[k])
        if not v:
            continue
        pct = lambda q: v[min(len(v) - 1, int(round(q * (len(v) - 1))))]  # noqa: E731
        out.append(f"  {k:8s} {len(v):5d} launches: p10 {pct(0.1):6.1f}  p50 {pct(0.5):6.1f}  p90 {pct(0.9):6.1f}"
                   f"  max {v[-1]:6.1f}")
    return "\n".join(out)


def mfma_table(path, match=None, simds=1024, ghz=2.4):
    """Per kernel: dispatches, average duration, MFMA flops per dispatch by
    type, the rate they give over the dispatch's own duration, and the MFMA
    busy share: busy cycles summed over the SIMDs / (duration x clock x SIMDs).
    (GRBM_GUI_ACTIVE is kept in the table but not used for the share: under
    counter collection it spans the collection window, not the kernel.)"""
    per = {}  # dispatch -> (name, duration ns, {counter: [values]})
    for r in _rows(path):
        if match and match not in r["Kernel_Name"]:
            continue
        d = int(r["Dispatch_Id"])
        name, dur, cnt = per.setdefault(d, (r["Kernel_Name"], int(r["End_Timestamp"]) - int(r["Start_Timestamp"]), {}))
        cnt.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    agg = {}
    for name, dur, cnt in per.values():
        a = agg.setdefault(name, dict(n=0, dur=0.0, f64=0.0, bf16=0.0, f8=0.0, busy=0.0))
        a["n"] += 1
        a["dur"] += dur
        for key, ctr in (("f64", "SQ_INSTS_VALU_MFMA_MOPS_F64"), ("bf16", "SQ_INSTS_VALU_MFMA_MOPS_BF16"),
                         ("f8", "SQ_INSTS_VALU_MFMA_MOPS_F8")):
            a[key] += 512.0 * sum(cnt.get(ctr, [0.0]))
        a["busy"] += sum(cnt.get("SQ_VALU_MFMA_BUSY_CYCLES", [0.0]))
    out = [f"{'kernel':<52} {'disp':>4} {'avg us':>9} {'F64 GFLOP':>10} {'BF16 GFLOP':>11} {'F8 GFLOP':>9} "
           f"{'TFLOP/s':>8} {'MFMA busy':>10}"]
    for name, a in sorted(agg.items(), key=lambda kv: -kv[1]["busy"]):
        n = a["n"]
        short = name if len(name) <= 52 else name[:49] + "..."
        flops = a["f64"] + a["bf16"] + a["f8"]
        rate = flops / a["dur"] / 1e3 if a["dur"] > 0 else float("nan")
        util = a["busy"] / (a["dur"] * ghz * simds) if a["dur"] > 0 else float("nan")
        out.append(f"{short:<52} {n:>4} {a['dur'] / n / 1e3:>9.1f} {a['f64'] / n / 1e9:>10.3f} "
                   f"{a['bf16'] / n / 1e9:>11.3f} {a['f8'] / n / 1e9:>9.3f} {rate:>8.1f} {util:>10.3f}")
    return "\n".join(out)


def lds_table(path, match=None, cus=256, ghz=2.4):
    """Per kernel: dispatches, average duration, bytes loaded from LDS per
    dispatch, their rate and share of the LDS peak (128 B per clock per CU),
    and bank-conflict cycles / indexed-access cycles."""
    per = {}
    for r in _rows(path):
        if match and match not in r["Kernel_Name"]:
            continue
        d = int(r["Dispatch_Id"])
        name, dur, cnt = per.setdefault(d, (r["Kernel_Name"], int(r["End_Timestamp"]) - int(r["Start_Timestamp"]), {}))
        cnt[r["Counter_Name"]] = cnt.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    agg = {}
    for name, dur, cnt in per.values():
        a = agg.setdefault(name, dict(n=0, dur=0.0, ld=0.0, act=0.0, conf=0.0))
        a["n"] += 1
        a["dur"] += dur
        a["ld"] += 64.0 * cnt.get("SQ_INSTS_LDS_LOAD_BANDWIDTH", 0.0)
        a["act"] += cnt.get("SQ_LDS_IDX_ACTIVE", 0.0)
        a["conf"] += cnt.get("SQ_LDS_BANK_CONFLICT", 0.0)
    peak = 128.0 * cus * ghz  # bytes per ns
    out = [f"{'kernel':<52} {'disp':>4} {'avg us':>9} {'LDS GB':>8} {'TB/s':>6} {'of peak':>8} {'conflict':>9}"]
    for name, a in sorted(agg.items(), key=lambda kv: -kv[1]["ld"]):
        n = a["n"]
        short = name if len(name) <= 52 else name[:49] + "..."
        rate = a["ld"] / a["dur"] if a["dur"] > 0 else float("nan")  # bytes per ns = GB/s
        conf = a["conf"] / a["act"] if a["act"] > 0 else float("nan")
        out.append(f"{short:<52} {n:>4} {a['dur'] / n / 1e3:>9.1f} {a['ld'] / n / 1e9:>8.2f} {rate / 1e3:>6.1f} "
                   f"{rate / peak:>8.3f} {conf:>9.3f}")
    return "\n".join(out)


def waits_table(path, match=None):
    """Per kernel: each SQ_WAIT_* / SQ_ACTIVE_INST_* counter of the run as a
    share of SQ_WAVE_CYCLES (both in quad-cycles, summed over dispatches)."""
    agg = {}
    for r in _rows(path):
        if match and match not in r["Kernel_Name"]:
            continue
        a = agg.setdefault(r["Kernel_Name"], {})
        a[r["Counter_Name"]] = a.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    cols = ["SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS",
            "SQ_ACTIVE_INST_VMEM", "SQ_ACTIVE_INST_MISC"]
    names = ["wait", "wait issue", "active", "VALU", "LDS", "VMEM", "misc"]
    out = [f"{'kernel':<52} " + " ".join(f"{n:>10}" for n in names)]
    for name, a in sorted(agg.items()):
        wc = a.get("SQ_WAVE_CYCLES", 0.0)
        short = name if len(name) <= 52 else name[:49] + "..."
        vals = [a.get(c, float("nan")) / wc if wc > 0 else float("nan") for c in cols]
        out.append(f"{short:<52} " + " ".join(f"{v:>10.3f}" for v in vals))
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
    lv = sub.add_parser("levels")
    lv.add_argument("csv")
    lv.add_argument("--skip", type=int, default=0, help="selections to leave out at the start (warm-up)")
    du = sub.add_parser("durations")
    du.add_argument("csv")
    mf = sub.add_parser("mfma")
    mf.add_argument("csv")
    mf.add_argument("--match", default=None)
    mf.add_argument("--simds", type=int, default=1024, help="SIMDs of the GPU (4 per compute unit)")
    mf.add_argument("--ghz", type=float, default=2.4, help="engine clock for the busy share")
    ld = sub.add_parser("lds")
    ld.add_argument("csv")
    ld.add_argument("--match", default=None)
    ld.add_argument("--cus", type=int, default=256, help="compute units of the GPU")
    ld.add_argument("--ghz", type=float, default=2.4, help="engine clock for the LDS peak")
    wt = sub.add_parser("waits")
    wt.add_argument("csv")
    wt.add_argument("--match", default=None)
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
    t.add_argument("--roof-key", default="roofline",
                   help="the bench line's roofline record of this kernel (roofline: k_pass, roofline_fresh: k_fresh)")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(kernel_stats(a.csv, a.top, a.match))
        return 0
    if a.cmd == "levels":
        print(level_table(a.csv, a.skip))
        return 0
    if a.cmd == "durations":
        print(duration_table(a.csv))
        return 0
    if a.cmd == "waits":
        print(waits_table(a.csv, a.match))
        return 0
    if a.cmd == "lds":
        print(lds_table(a.csv, a.match, a.cus, a.ghz))
        return 0
    if a.cmd == "mfma":
        print(mfma_table(a.csv, a.match, a.simds, a.ghz))
        return 0
    rec = pass_traffic(a.fetch_csv, a.write_csv, a.kernel, a.copy_bytes, a.last)
    if a.bench_line:
        with open(a.bench_line) as f:
            line = [ln for ln in f if ln.startswith("{")][-1]
        roof = json.loads(line)[a.roof_key]
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
