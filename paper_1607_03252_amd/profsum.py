"""Summaries of rocprofv3 output for the profiles kept with the sources.

  trace: per (kernel, launch grid) call counts and durations from a
         ``--kernel-trace`` CSV (``*_kernel_trace.csv``);
  pmc:   HBM bytes per dispatch of one kernel from two ``--pmc`` runs
         (FETCH_SIZE and WRITE_SIZE, KiB per dispatch), each scaled by what
         the same counter reads for a plain device copy of known size run in
         the same process (``bench.py --calib-copy``), written as JSON together
         with the hash of the kernel source it was taken on.

  sweeps: the finest-grid smoothing launches of the last K batches of a run,
         restricted to the V-cycles in which every solve still cycles (the
         selection bench.py's roofline uses): durations from a kernel trace,
         and HBM bytes from the two counter runs when given.

  python -m paper_1607_03252_amd.profsum trace CSV OUT --title T --command C
  python -m paper_1607_03252_amd.profsum pmc FETCH_CSV WRITE_CSV OUT --match K@GRID ...
         --command C [--copy-bytes B] [--tiles TJ:TK:CH,TJ:TK:CH]
  python -m paper_1607_03252_amd.profsum sweeps TRACE_CSV OUT --batches K --cycles-upto M
         --bytes-per-kind B0,B1,B2,B3 --title T --command C
         [--fetch FETCH_CSV --write WRITE_CSV --pmc-command C2 --tiles ...]
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


KIND_NAMES = ["plain", "coarse_correction", "output_residual", "input_residual"]


def sweep_kind(name):
    """0 plain, 1 with the coarse-grid correction, 2 output residual norm,
    3 input residual norm (the kinds of mg_profile_records)."""
    if "res_out" in name:
        return 2
    if "res_in" in name:
        return 3
    m = re.match(r"k_sweep<[^,]+,\s*\d+,\s*\d+,\s*(true|false)", name)
    return 1 if m and m.group(1) == "true" else 0


def _order_key(r):
    for k in ("Dispatch_Id", "Correlation_Id"):
        if r.get(k) not in (None, ""):
            return int(r[k])
    return int(r["Start_Timestamp"])


def finest_sweeps(rows, batches, cycles_upto, nu1=2, nu2=2):
    """Rows (one per dispatch) of the finest-grid sweeps in cycles 1..cycles_upto
    of the last `batches` batches.  A batch starts at k_init_state.  Each
    V-cycle has one bottom (k_vsmall or k_coarsest dispatches, consecutive
    ones taken together), which splits the batch's sweep dispatches into
    segments: S_0 before the first bottom is cycle 1's pre-smoothing, K levels
    of nu1 sweeps from the finest grid down; S_c between bottoms c and c + 1
    is cycle c's post-smoothing (K levels of nu2 sweeps, the finest grid's
    last) followed by cycle c + 1's pre-smoothing.  So cycle c's finest
    sweeps are the first nu1 of its pre-smoothing and the last nu2 of its
    post-smoothing.  (Every cycle of a batch, also one on the lists of its
    last solves, visits the same K levels.)  Returns [(kind, cycle, row)]."""
    rows = sorted(rows, key=_order_key)
    names = [short_name(r["Kernel_Name"]) for r in rows]
    starts = [i for i, nm in enumerate(names) if nm == "k_init_state"]
    if len(starts) < batches:
        raise ValueError("the run has %d batches, fewer than %d" % (len(starts), batches))
    out = []
    for b in range(len(starts) - batches, len(starts)):
        lo = starts[b]
        hi = starts[b + 1] if b + 1 < len(starts) else len(rows)
        segs, cur, at_bottom = [], [], False
        for i in range(lo, hi):
            nm = names[i]
            if nm.startswith("k_vsmall") or nm.startswith("k_coarsest"):
                if not at_bottom:
                    segs.append(cur)
                    cur = []
                at_bottom = True
            elif nm.startswith("k_sweep"):
                cur.append(i)
                at_bottom = False
        segs.append(cur)
        if len(segs) < 2 or len(segs[0]) % nu1:
            continue
        K = len(segs[0]) // nu1
        for c in range(1, len(segs)):
            if c > cycles_upto:
                break
            pre = (segs[0] if c == 1 else segs[c - 1][K * nu2:])[:nu1]
            post = segs[c][:K * nu2][-nu2:]
            for i in pre + post:
                out.append((sweep_kind(names[i]), c, rows[i]))
    return out


def sweeps_summary(trace_csv, batches, cycles_upto, bytes_per_kind, fetch_csv=None,
                   write_csv=None, copy_bytes=float(1 << 30)):
    rows = list(csv.DictReader(open(trace_csv)))
    sel = finest_sweeps(rows, batches, cycles_upto)
    per = collections.defaultdict(list)
    names = {}
    for kind, cyc, r in sel:
        per[kind].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        names[kind] = short_name(r["Kernel_Name"])
    res = {"launches": len(sel), "batches": batches, "cycles_upto": cycles_upto, "per_kind": {}}
    tot_ns, tot_b = 0, 0.0
    for k in sorted(per):
        v = per[k]
        b = bytes_per_kind[k]
        res["per_kind"][KIND_NAMES[k]] = {"kernel": names[k], "launches": len(v),
                                          "avg_us": sum(v) / len(v) / 1e3, "bytes": b,
                                          "GBps": b * len(v) / (sum(v) * 1e-9) / 1e9}
        tot_ns += sum(v)
        tot_b += b * len(v)
    res["avg_launch_us"] = tot_ns / max(1, len(sel)) / 1e3
    res["bytes_per_launch"] = tot_b / max(1, len(sel))
    res["achieved_GBps"] = tot_b / (tot_ns * 1e-9) / 1e9 if tot_ns else None
    if fetch_csv and write_csv:
        fsel = _counter_sel(fetch_csv, "FETCH_SIZE", batches, cycles_upto)
        wsel = _counter_sel(write_csv, "WRITE_SIZE", batches, cycles_upto)
        cf = _copy_kib(fetch_csv, "FETCH_SIZE")
        cw = _copy_kib(write_csv, "WRITE_SIZE")
        fs = (copy_bytes / 1024.0) / cf if cf else None
        ws = (copy_bytes / 1024.0) / cw if cw else None
        tr = {}
        for k in sorted(set(fsel) | set(wsel)):
            fk, wk = fsel.get(k, []), wsel.get(k, [])
            if fk and wk and fs and ws:
                hbm = 1024.0 * (sum(fk) / len(fk) * fs + sum(wk) / len(wk) * ws)
                tr[KIND_NAMES[k]] = {"dispatches": [len(fk), len(wk)], "fetch_kib": sum(fk) / len(fk),
                                     "write_kib": sum(wk) / len(wk), "hbm_bytes": hbm,
                                     "over_algorithmic": hbm / bytes_per_kind[k]}
        res["traffic_per_kind"] = tr
        res["fetch_scale"], res["write_scale"] = fs, ws
        res["copy_fetch_kib"], res["copy_write_kib"] = cf, cw
        if tr:
            # weighted like the durations: by the launches of each kind
            w = {KIND_NAMES[k]: len(per[k]) for k in per}
            tot = sum(w[nm] for nm in tr)
            res["hbm_bytes_per_launch"] = sum(tr[nm]["hbm_bytes"] * w[nm] for nm in tr) / tot
    return res


def _counter_sel(path, counter, batches, cycles_upto):
    rows = [r for r in csv.DictReader(open(path)) if r.get("Counter_Name") == counter]
    sel = finest_sweeps(rows, batches, cycles_upto)
    d = collections.defaultdict(list)
    for kind, _, r in sel:
        d[kind].append(float(r["Counter_Value"]))
    return d


def _copy_kib(path, counter):
    best = 0.0
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        nm = short_name(r["Kernel_Name"])
        if nm in ("copyBuffer", "torch_elementwise") or "copy" in nm:
            best = max(best, float(r["Counter_Value"]))
    return best


def kernel_overlap(rows):
    """Concurrency of the kernels of a trace (rows with Start_Timestamp and
    End_Timestamp, ns): busy time (the union of their intervals), summed
    kernel time, the mean number running while any runs (their ratio), and
    the share of busy time in which two or more run at once.  Kernels that
    end and start at the same instant do not overlap."""
    ev = []
    for r in rows:
        a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        if b > a:
            ev += [(a, 1), (b, -1)]
    ev.sort(key=lambda e: (e[0], e[1]))  # ends before starts at the same time
    busy = over = total = 0
    cur, last = 0, None
    for t, d in ev:
        if last is not None and cur > 0:
            busy += t - last
            total += cur * (t - last)
            if cur > 1:
                over += t - last
        cur += d
        last = t
    return {"kernels": len(ev) // 2, "busy_ns": busy, "kernel_ns": total,
            "span_ns": (ev[-1][0] - ev[0][0]) if ev else 0,
            "mean_concurrency": total / busy if busy else 0.0,
            "overlap_share": over / busy if busy else 0.0}


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("out")
    t.add_argument("--title", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--stats", default="", help="the run's *_kernel_stats.csv")
    t.add_argument("--overlap", action="store_true",
                   help="also the kernels' concurrency (several queues at once)")
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
    w = sub.add_parser("sweeps")
    w.add_argument("csv")
    w.add_argument("out")
    w.add_argument("--batches", type=int, required=True)
    w.add_argument("--cycles-upto", type=int, required=True)
    w.add_argument("--bytes-per-kind", required=True,
                   help="algorithmic bytes per launch of kinds 0,1,2,3")
    w.add_argument("--title", required=True)
    w.add_argument("--command", required=True)
    w.add_argument("--stats", default="")
    w.add_argument("--fetch", default="")
    w.add_argument("--write", default="")
    w.add_argument("--pmc-command", default="")
    w.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    w.add_argument("--tiles", default="")
    a = ap.parse_args()
    if a.cmd == "sweeps":
        bpk = [float(x) for x in a.bytes_per_kind.split(",")]
        res = sweeps_summary(a.csv, a.batches, a.cycles_upto, bpk, a.fetch or None,
                             a.write or None, a.copy_bytes)
        res["command"] = a.command
        if a.pmc_command:
            res["pmc_command"] = a.pmc_command
        res["tiles"] = ([[int(x) for x in t.split(":")] for t in a.tiles.split(",")]
                        if a.tiles else None)
        res["kernel_source_sha256"] = source_hash()
        lines = ["%s" % a.title, "command: %s" % a.command]
        if a.pmc_command:
            lines.append("counters: %s" % a.pmc_command)
        lines += ["", "finest-grid sweeps, cycles 1..%d of the last %d batches (every solve active):"
                  % (a.cycles_upto, a.batches),
                  "%-18s %-40s %6s %10s %12s %9s" % ("kind", "kernel", "calls", "avg_us", "bytes", "GB/s")]
        for nm, v in res["per_kind"].items():
            lines.append("%-18s %-40s %6d %10.1f %12.4g %9.1f" % (nm, v["kernel"][:40], v["launches"],
                                                                 v["avg_us"], v["bytes"], v["GBps"]))
        lines.append("all kinds: %d launches, mean %.1f us, %.4g B algorithmic per launch, %.1f GB/s"
                     % (res["launches"], res["avg_launch_us"], res["bytes_per_launch"],
                        res["achieved_GBps"] or 0.0))
        for nm, v in res.get("traffic_per_kind", {}).items():
            lines.append("traffic %-18s %10.4g B per launch (%.3f x algorithmic)"
                         % (nm, v["hbm_bytes"], v["over_algorithmic"]))
        if a.stats:
            lines += ["", "rocprofv3 --stats (every launch of the run, per kernel name):",
                      stats_table(a.stats)]
        lines += ["", "per kernel and launch grid (every launch of the run):", trace_table(a.csv)]
        txt = "\n".join(lines) + "\n\n" + JSON_MARK + "\n" + json.dumps(res, indent=1) + "\n"
        open(a.out, "w").write(txt)
        print(txt)
        return
    if a.cmd == "trace":
        txt = "%s\ncommand: %s\n\nper kernel and launch grid:\n%s\n" % (a.title, a.command,
                                                                  trace_table(a.csv))
        if a.stats:
            txt += "\nrocprofv3 --stats (per kernel name):\n" + stats_table(a.stats) + "\n"
        if a.overlap:
            with open(a.csv) as f:
                o = kernel_overlap(list(csv.DictReader(f)))
            txt += ("\nconcurrency: %d kernels over %.3f ms busy (%.3f ms span); summed kernel "
                    "time %.3f ms = %.2f kernels running on average while any runs; two or more "
                    "at once during %.1f%% of the busy time\n"
                    % (o["kernels"], o["busy_ns"] / 1e6, o["span_ns"] / 1e6, o["kernel_ns"] / 1e6,
                       o["mean_concurrency"], 100.0 * o["overlap_share"]))
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
