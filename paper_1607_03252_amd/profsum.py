"""Summaries of rocprofv3 output for the profiles kept with the sources.

  trace: per (kernel, launch grid) call counts and durations from a
         ``--kernel-trace`` CSV (``*_kernel_trace.csv``);
  pmc:   HBM bytes per dispatch of one kernel from two ``--pmc`` runs
         (FETCH_SIZE and WRITE_SIZE, KiB per dispatch), each scaled by what
         the same counter reads for a plain device copy of known size run in
         the same process (``bench.py --calib-copy``), written as JSON together
         with the hash of the kernel source it was taken on.

  python -m paper_1607_03252_amd.profsum trace CSV OUT --title T --command C
  python -m paper_1607_03252_amd.profsum pmc FETCH_CSV WRITE_CSV OUT --match K@GRID ...
         --command C [--copy-bytes B] [--tiles TJ:TK:CH,TJ:TK:CH]
"""
import argparse
import collections
import csv
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "mg_kernels.hip")


JSON_MARK = "-- summary (json) --"


def read_summary(path):
    """The JSON block of a summary written by ``pmc``."""
    txt = open(path).read()
    return json.loads(txt.split(JSON_MARK, 1)[1])


SWEEP_END = b"// ---- point kernels"


def source_hash(path=KERNEL_SOURCE):
    """SHA-256 of the device code the fused sweep is built from: the kernel
    source up to the end of the sweep kernel (its helpers and the kernel),
    with comments and blank space removed, so that an edit of the comments
    alone does not invalidate counters taken on the same code."""
    with open(path, "rb") as f:
        src = f.read().split(SWEEP_END, 1)[0].decode()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = " ".join(src.split())
    return hashlib.sha256(src.encode()).hexdigest()


def short_name(s):
    m = re.search(r"(k_[A-Za-z0-9_]+(?:<[^>]*>)?)", s)
    if m:
        return m.group(1)
    if "copyBuffer" in s:
        return "copyBuffer"
    if "elementwise" in s:
        return "torch_elementwise"
    return s.split("(")[0][:40]


def trace_table(path, top=30):
    rows = list(csv.DictReader(open(path)))
    d = collections.defaultdict(list)
    for r in rows:
        key = (short_name(r["Kernel_Name"]), int(r["Grid_Size_X"]))
        d[key].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    tot = sum(sum(v) for v in d.values())
    out = ["%-36s %10s %6s %11s %10s %6s" % ("kernel", "grid", "calls", "avg_us", "total_ms", "pct")]
    for (nm, g), v in sorted(d.items(), key=lambda kv: -sum(kv[1]))[:top]:
        out.append("%-36s %10d %6d %11.1f %10.3f %6.1f" % (nm[:36], g, len(v), sum(v) / len(v) / 1e3,
                                                          sum(v) / 1e6, 100.0 * sum(v) / tot))
    return "\n".join(out)


def stats_table(path, top=16):
    rows = list(csv.DictReader(open(path)))
    out = ["%-36s %7s %14s %12s %7s" % ("kernel", "calls", "total_ns", "avg_ns", "pct")]
    for r in rows[:top]:
        out.append("%-36s %7s %14s %12.1f %7.2f" % (short_name(r["Name"])[:36], r["Calls"],
                                                   r["TotalDurationNs"], float(r["AverageNs"]),
                                                   float(r["Percentage"])))
    return "\n".join(out)


def counter_values(path, counter):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        d[(short_name(r["Kernel_Name"]), int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    return d


def pmc_summary(fetch_csv, write_csv, matches, copy_bytes):
    f = counter_values(fetch_csv, "FETCH_SIZE")
    w = counter_values(write_csv, "WRITE_SIZE")

    def copy_kib(d):
        # the largest copy-like dispatch is the calibration copy
        best = 0.0
        for (nm, _), v in d.items():
            if nm in ("copyBuffer", "torch_elementwise") or "copy" in nm:
                best = max(best, max(v))
        return best

    cf, cw = copy_kib(f), copy_kib(w)
    fs = (copy_bytes / 1024.0) / cf if cf else None
    ws = (copy_bytes / 1024.0) / cw if cw else None
    def sel(d):
        return [v for (nm, g), v in d.items() if any(nm == k and g == gr for k, gr in matches)]
    fk, wk = sel(f), sel(w)
    fv = [x for v in fk for x in v]
    wv = [x for v in wk for x in v]
    res = {"kernels": ["%s @ grid %d" % m for m in matches], "dispatches_fetch": len(fv),
           "dispatches_write": len(wv),
           "fetch_kib": sum(fv) / len(fv) if fv else None,
           "write_kib": sum(wv) / len(wv) if wv else None,
           "copy_bytes": copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
           "fetch_scale": fs, "write_scale": ws}
    if fv and wv and fs and ws:
        res["hbm_bytes_per_launch"] = 1024.0 * (res["fetch_kib"] * fs + res["write_kib"] * ws)
    table = ["%-6s %-36s %10s %6s %14s" % ("ctr", "kernel", "grid", "n", "avg_KiB")]
    for lab, d in (("FETCH", f), ("WRITE", w)):
        for (nm, g), v in sorted(d.items(), key=lambda kv: -sum(kv[1]))[:14]:
            table.append("%-6s %-36s %10d %6d %14.0f" % (lab, nm[:36], g, len(v), sum(v) / len(v)))
    return res, "\n".join(table)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("out")
    t.add_argument("--title", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--stats", default="", help="the run's *_kernel_stats.csv")
    p = sub.add_parser("pmc")
    p.add_argument("fetch_csv")
    p.add_argument("write_csv")
    p.add_argument("out")
    p.add_argument("--match", action="append", required=True,
                   help="KERNEL@GRID (repeatable): the dispatches averaged over")
    p.add_argument("--command", required=True)
    p.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    p.add_argument("--tiles", default="",
                   help="TJ:TK:CHUNKS,TJ:TK:CHUNKS of the plain and the fused-correction sweep")
    a = ap.parse_args()
    if a.cmd == "trace":
        txt = "%s\ncommand: %s\n\nper kernel and launch grid:\n%s\n" % (a.title, a.command,
                                                                  trace_table(a.csv))
        if a.stats:
            txt += "\nrocprofv3 --stats (per kernel name):\n" + stats_table(a.stats) + "\n"
        open(a.out, "w").write(txt)
        print(txt)
    else:
        matches = [(m.rsplit("@", 1)[0], int(m.rsplit("@", 1)[1])) for m in a.match]
        res, table = pmc_summary(a.fetch_csv, a.write_csv, matches, a.copy_bytes)
        res["command"] = a.command
        res["tiles"] = ([[int(x) for x in t.split(":")] for t in a.tiles.split(",")]
                        if a.tiles else None)
        res["kernel_source_sha256"] = source_hash()
        with open(a.out, "w") as f:
            f.write("HBM traffic counters, per dispatch\ncommand: %s\n\n%s\n\n%s\n%s\n" % (
                a.command, table, JSON_MARK, json.dumps(res, indent=1)))
        print(open(a.out).read())


if __name__ == "__main__":
    main()
