"""Benchmark of the MLMC multigrid hot path on one MI355X.

Default workload (one step): one batch of 16 MLMC samples of one 257^3 solve
each (level 0 of n0 = 257), seeds 16*s .. 16*s+15 for step s, lognormal
coefficient with sigma^2 = 2, lambda = 0.05 (4x4x4 separable KL), f = 1,
FP64 V(2,2) red-black Gauss-Seidel to relative residual 1e-8, QoI = integral
of u.  Inputs are generated on the device from seeds; everything stays
resident in HBM (only the 16 seeds cross PCIe per step).

Prints one JSON line (the byte model is in the repository's design notes):
  value        = samples per second over the timed steps;
  roofline     = the fused red-black sweeps on the 257^3 grids: algorithmic
                 bytes of the launches of the cycles in which every solve
                 still cycles, over their summed duration (HIP events on the
                 plan's stream, eager profiled steps after the timed region),
                 against the 8 TB/s HBM peak; traffic from the committed
                 counter summary when it was taken on the same sweep source
                 and tile shapes;
  cpu_baseline = the FP64 CPU oracle on the same workload: every host thread
                 generates one sample's field and runs one V-cycle (with its
                 residual), scaled by the GPU run's mean cycle count to
                 samples per second; plus the single-thread latency;
  extra        = the 64-pair level-1 batch (65^3 + 33^3), the mixed-precision
                 form on the same 257^3 inputs (one and two FP32 V-cycles per
                 FP64 defect-correction step), and a device copy's rate.
"""
import argparse
import concurrent.futures as cf
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# algorithmic bytes per interior node of one fused red-black sweep with a
# constant right-hand side: wh (8) + u read (8) + u written (8); with the KL
# coefficient evaluated in the sweep (plan option kl = 1) wh is not read: 16;
# the sweep with the coarse-grid correction also reads the coarse iterate once
SWEEP_BYTES_PER_NODE = 24.0
SWEEP_KL_BYTES_PER_NODE = 16.0
COARSE_BYTES_PER_NODE = 8.0


def kl_inline(args):
    """Whether the plan options turn the in-kernel KL coefficient on."""
    for spec in args.opt:
        name, value = spec.split("=")
        if name == "kl":
            return int(value) != 0
    return False
# byte model of one FP64 V(2,2) cycle per finest-grid node (whole hierarchy)
VCYCLE_BYTES_PER_NODE = 195.0
# the same with the KL coefficient formed in the finest grid's four sweeps and
# its residual-restriction (8 bytes per node each not read)
VCYCLE_KL_BYTES_PER_NODE = VCYCLE_BYTES_PER_NODE - 5 * 8.0
# mixed precision: an FP32 V(2,2) cycle (~98) per cycle, plus the FP64 defect
# and update (48) once per outer step of inner_cycles cycles
MIXED_FP32_CYCLE_BYTES = 98.0
MIXED_FP64_STEP_BYTES = 48.0


def mixed_bytes_per_node(inner_cycles=1):
    """Byte model of one V-cycle of mixed precision per finest-grid node."""
    return MIXED_FP32_CYCLE_BYTES + MIXED_FP64_STEP_BYTES / inner_cycles


KIND_NAMES = {0: "plain", 1: "coarse_correction", 2: "output_residual", 3: "input_residual"}

CFG4 = dict(n=257, samples=16, sigma2=2.0, corr_len=0.05, tol=1e-8)


def host_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline_config4(threads, cycles_mean):
    """The oracle on the default workload's inputs.  Each of `threads` host
    threads takes one sample (seeds 10^6..): the coefficient field, then one
    V(2,2) cycle with its residual norm (the oracle's solve with one fixed
    cycle); per-sample time = field + cycles_mean x cycle.  Also one sample's
    field and cycle on a single thread (latency)."""
    import oracle as O
    n, s2, lam = CFG4["n"], CFG4["sigma2"], CFG4["corr_len"]

    def one(seed):
        t0 = time.perf_counter()
        k = O.field(n, s2, lam, O.gaussians(seed, 0))
        t1 = time.perf_counter()
        O.solve(k, O.rhs(n), fixed_cycles=1)
        return t1 - t0, time.perf_counter() - t1

    tf1, tc1 = one(10**6)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(one, range(10**6 + 1, 10**6 + 1 + threads)))
    wall = time.perf_counter() - t0
    tf = sum(r[0] for r in res) / len(res)
    tc = sum(r[1] for r in res) / len(res)
    per_sample = tf + cycles_mean * tc
    return {"value": threads / per_sample, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": "%d samples of the 257^3 workload (seeds 1e6+1..), one per thread: field "
                      "(%.2f s) + one V(2,2) cycle with residual (%.2f s) each, scaled to %.2f "
                      "cycles per sample; %.1f s wall" % (threads, tf, tc, cycles_mean, wall),
            "single_thread_latency_s": tf1 + cycles_mean * tc1,
            "single_thread_field_s": tf1, "single_thread_cycle_s": tc1, **host_info()}


def cpu_baseline_pairs(n0, level, threads, min_seconds, max_samples=4096):
    """The oracle on `threads` host threads, one level-pair sample per thread,
    in rounds of `threads` samples until min_seconds have passed."""
    import oracle as O
    done, seed = 0, 10**6
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        while True:
            seeds = list(range(seed, seed + threads))
            list(ex.map(lambda s: O.mlmc_sample(n0, level, s), seeds))
            seed += threads
            done += threads
            dt = time.perf_counter() - t0
            if dt >= min_seconds or done >= max_samples:
                break
    return done / dt, dt, done


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--samples", type=int, default=64, help="level-pair batch size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="headline only (no level-pair, mixed-precision or copy figures)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="host threads of the oracle baseline (default min(16, nproc))")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="minimum wall time of the level-pair oracle baseline")
    ap.add_argument("--workload", default="config4",
                    choices=["config4", "levelpair", "single", "mixed", "fp32mix", "serve",
                             "adaptive", "fmg", "fe", "spde"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="precision of the default workload")
    ap.add_argument("--inner-cycles", type=int, default=1,
                    help="mixed precision: FP32 V-cycles per FP64 defect-correction step")
    ap.add_argument("--eps", type=float, default=5e-6,
                    help="adaptive workload: the MLMC tolerance (absolute, on Q)")
    ap.add_argument("--serve-requests", type=int, default=2048)
    ap.add_argument("--serve-slots", default="128,64,16,4",
                    help="slots per lane of each level, or 'auto' (an eighth of the budget)")
    ap.add_argument("--serve-budget-gib", type=float, default=8.0,
                    help="HBM budget the server's lanes share (GiB)")
    ap.add_argument("--serve-loads", default="0.5,0.8,0.95")
    ap.add_argument("--no-fifo", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the smoother's tile shapes first (default: the library's shapes)")
    ap.add_argument("--profile-steps", type=int, default=2)
    ap.add_argument("--tile", action="append", default=[],
                    help="n:tj:tk:chunks, pins a smoother tile shape (skips the autotuner)")
    ap.add_argument("--tile-pro", action="append", default=[],
                    help="n:tj:tk:chunks, the shape of the sweep with the fused coarse correction")
    ap.add_argument("--opt", action="append", default=[],
                    help="name=value, a plan option (mg_plan_set_option), e.g. norm=0")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (counter calibration)")
    return ap.parse_args()


def main():
    args = parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(samples shard across GPUs by seed range; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1607_03252_amd as M
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(3)
    if not os.path.exists(M.LIB_PATH):
        raise SystemExit("libmlmcmg.so is not built: run `python -m paper_1607_03252_amd.build`")
    threads = args.cpu_threads or min(16, os.cpu_count() or 1)
    if args.workload != "config4":
        fn = {"levelpair": bench_levelpair, "single": bench_single, "mixed": bench_mixed,
              "fp32mix": bench_fp32mix, "serve": bench_serve,
              "adaptive": bench_adaptive, "fmg": bench_option, "fe": bench_option,
              "spde": bench_option}[args.workload]
        out = fn(args, M, torch, np)
        if args.workload == "levelpair" and not args.no_cpu_baseline:
            v, cdt, done = cpu_baseline_pairs(33, 1, threads, args.cpu_seconds)
            out["cpu_baseline"] = {"value": v, "unit": "samples/s", "cores": threads,
                                   "kind": "oracle",
                                   "sample": "%d samples of the same level pair (seeds 1e6..), "
                                             "one sample per thread, %.1f s wall" % (done, cdt),
                                   **host_info()}
        print(json.dumps(out), flush=True)
        return

    out = bench_config4(args, M, torch, np, M.MG_FP64 if args.precision == "fp64" else M.MG_MIXED,
                        inner=args.inner_cycles)
    if not args.no_extra:
        extra = {}
        lp = bench_levelpair(args, M, torch, np, steps=min(args.steps, 10), profile=False)
        extra["levelpair_65_33_x64"] = {k: lp[k] for k in ("value", "unit", "ms_per_step")}
        extra["levelpair_65_33_x64"]["fine_cycles_mean"] = lp["per_level"]["1"]["fine_cycles_mean"]
        if args.precision == "fp64":
            for inner in (1, 2):
                mx = bench_config4(args, M, torch, np, M.MG_MIXED, steps=min(args.steps, 5),
                                   warmup=1, profile=False, inner=inner)
                key = "mixed_precision_257_x16" + ("" if inner == 1 else "_inner%d" % inner)
                extra[key] = {
                    "value": mx["value"], "unit": "samples/s", "ms_per_step": mx["ms_per_step"],
                    "inner_cycles": inner,
                    "fine_cycles_mean": mx["per_level"]["0"]["fine_cycles_mean"],
                    "speedup_vs_fp64": mx["value"] / out["value"],
                    "max_rel_dQ_vs_fp64": float(np.max(np.abs(mx["_Q"] - out["_Q"])
                                                       / np.abs(out["_Q"])))}
        cp = device_copy(torch)
        cp["sweep_fraction_of_copy"] = out["roofline"]["achieved"] / cp["GBps"]
        extra["device_copy"] = cp
        out["extra"] = extra
    out.pop("_Q", None)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_config4(threads, out["per_level"]["0"]["fine_cycles_mean"])
    print(json.dumps(out), flush=True)


def device_copy(torch, nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of nbytes (the streaming rate any kernel
    of this path can hope for on this GPU), timed with events."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbps = 2.0 * nbytes / (ms * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return {"bytes": nbytes, "GBps": gbps, "frac_of_peak": gbps / HBM_PEAK_GBPS}


def sweep_roofline(M, P, n, samples, cycles_min, kl=True):
    """Algorithmic bytes over duration of the timed sweep launches on the n^3
    grids in cycles 1..cycles_min of each profiled batch (every solve still
    cycles there, so every launch moves every grid); kl: the sweeps form the
    coefficient themselves (16 instead of 24 bytes per node)."""
    cyc, kind, gn, ms = M.mg_profile_records(P)
    nodes = samples * float(n - 2) ** 3
    nc = (n - 1) // 2 + 1
    coarse = samples * float(nc - 2) ** 3
    sel = (cyc <= cycles_min) & (gn == n) & (kind <= 3)
    per_kind = {}
    tot_b, tot_ms = 0.0, 0.0
    for k in sorted(set(kind[sel].tolist())):
        m = sel & (kind == k)
        per = SWEEP_KL_BYTES_PER_NODE if kl else SWEEP_BYTES_PER_NODE
        b = per * nodes + (COARSE_BYTES_PER_NODE * coarse if k == 1 else 0.0)
        avg = float(ms[m].mean())
        per_kind[KIND_NAMES[k]] = {"launches": int(m.sum()), "avg_us": 1e3 * avg,
                                   "bytes_per_launch": b, "GBps": b / (avg * 1e-3) / 1e9}
        tot_b += b * int(m.sum())
        tot_ms += float(ms[m].sum())
    achieved = tot_b / (tot_ms * 1e-3) / 1e9 if tot_ms else 0.0
    return {"achieved": achieved, "launches": int(sel.sum()),
            "avg_launch_us": 1e3 * tot_ms / max(1, int(sel.sum())),
            "bytes_per_launch": tot_b / max(1, int(sel.sum())), "per_kind": per_kind,
            "launches_excluded": int((~sel).sum())}


def read_traffic(name, tiles):
    """HBM bytes per launch from a committed counter summary, if it was taken
    on the current sweep source and the same tile shapes."""
    summ = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(summ):
        return None, None, None
    from paper_1607_03252_amd import profsum
    rec = profsum.read_summary(summ)
    if rec.get("kernel_source_sha256") == profsum.source_hash() and rec.get("tiles") == tiles:
        return rec.get("hbm_bytes_per_launch"), os.path.relpath(summ, ROOT), rec
    return None, None, None


def bench_config4(args, M, torch, np, precision, steps=None, warmup=None, profile=True, inner=1):
    n, S = CFG4["n"], CFG4["samples"]
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    P = M.mg_plan_create(n0=n, max_level=0, sigma2=CFG4["sigma2"], corr_len=CFG4["corr_len"],
                         tol=CFG4["tol"], nu1=2, nu2=2, max_cycles=50, precision=precision)
    for spec in args.opt:
        name, value = spec.split("=")
        M.mg_plan_set_option(P, name, int(value))
    if precision == M.MG_MIXED:
        M.mg_plan_set_option(P, "inner_cycles", inner)
    for spec in args.tile:
        nn, tj, tk, ch = (int(x) for x in spec.split(":"))
        M.mg_set_tile(P, nn, tj, tk, ch)
    for spec in args.tile_pro:
        nn, tj, tk, ch = (int(x) for x in spec.split(":"))
        M.mg_set_tile_for(P, nn, 1, tj, tk, ch)
    Y = torch.zeros(S, dtype=torch.float64, device="cuda")
    Qf, Qc = torch.zeros_like(Y), torch.zeros_like(Y)

    def step(s, cyc_out):
        seeds = np.arange(s * S, (s + 1) * S, dtype=np.uint64)
        st = M.mlmc_sample_batch(P, 0, seeds, S, Y, Qf, Qc, cyc_out)
        assert st == M.MG_OK, st

    if args.autotune and not args.tile:
        M.mg_autotune(P, 0, S, 3)
    tiles = [list(M.mg_get_tile(P, n)), list(M.mg_get_tile_for(P, n, 1))]
    cyc_w = torch.zeros(2 * S, dtype=torch.int32, device="cuda")
    for s in range(warmup):
        step(10**5 + s, cyc_w)
    cyc_all = torch.zeros(max(1, steps), 2 * S, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_step = []
    for s in range(steps):
        # (a batch call returns once its solves have finished: the time
        # between returns is that batch's solve latency)
        step(s, cyc_all[s])
        t_step.append(time.perf_counter())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lat_ms = 1e3 * np.diff(np.asarray([t0] + t_step))
    cyc_np = cyc_all.cpu().numpy().reshape(max(1, steps), S, 2)[:, :, 0]
    cyc_mean = float(cyc_np.mean())
    value = S * steps / dt
    ms_step = 1e3 * dt / steps
    vc = VCYCLE_KL_BYTES_PER_NODE if kl_inline(args) else VCYCLE_BYTES_PER_NODE
    per_node = vc if precision == M.MG_FP64 else mixed_bytes_per_node(inner)
    eff = per_node * n**3 * float(cyc_np.sum()) / dt / 1e9
    out = {
        "metric": "MLMC samples/sec per level + V-cycle HBM GB/s; p50/p99 solve latency",
        "value": value, "unit": "samples/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if precision == M.MG_FP64 else "f64+f32",
        "data": "synthetic (Philox-seeded 64-term KL lognormal fields)",
        "config": {"workload": "mlmc_level0_n257_x16_sigma2_2_lambda_0.05"
                               + ("" if precision == M.MG_FP64 else "_mixed_precision"
                                  + ("" if inner == 1 else "_inner%d" % inner)),
                   "n": n, "samples_per_step": S, "sigma2": CFG4["sigma2"],
                   "corr_len": CFG4["corr_len"], "tol": CFG4["tol"],
                   "cycle": "V(2,2) red-black GS, 8 levels", "parallelism": "single GPU",
                   "tiles": {str(n): tiles[0]}, "tiles_pro": {str(n): tiles[1]},
                   "options": dict(o.split("=") for o in args.opt)},
        "per_level": {"0": {"samples_per_s": value, "fine_cycles_mean": cyc_mean,
                            "effective_vcycle_GBps": eff, "batch_latency_ms": ms_step,
                            "batch_latency_p50_ms": _pct(lat_ms, 50),
                            "batch_latency_p99_ms": _pct(lat_ms, 99)}},
    }
    # the QoI of step 0's seeds (an untimed step), for the mixed vs FP64 comparison
    step(0, cyc_w)
    out["_Q"] = Qf.cpu().numpy().copy()
    if profile and precision == M.MG_FP64:
        # eager steps with every sweep launch on the 257^3 grids timed by HIP
        # events; only the cycles in which every solve still cycles count
        M.mg_profile_enable(P, True)
        cyc_p = torch.zeros(max(1, args.profile_steps), 2 * S, dtype=torch.int32, device="cuda")
        for s in range(args.profile_steps):
            step(s, cyc_p[s])
        torch.cuda.synchronize()
        cmin = int(cyc_p.cpu().numpy().reshape(-1, S, 2)[:, :, 0].min())
        rf = sweep_roofline(M, P, n, S, cmin, kl_inline(args))
        M.mg_profile_enable(P, False)
        traffic, src, rec = read_traffic("k_sweep_config4_257x16.txt", tiles)
        out["roofline"] = {"bound": "hbm", "achieved": rf["achieved"], "peak": HBM_PEAK_GBPS,
                           "unit": "GB/s", "frac": rf["achieved"] / HBM_PEAK_GBPS,
                           "traffic": traffic, "traffic_source": src,
                           "kernel": "k_sweep family (fused red-black sweeps, 257^3 grids)",
                           "bytes_per_node": (SWEEP_KL_BYTES_PER_NODE if kl_inline(args)
                                              else SWEEP_BYTES_PER_NODE),
                           "coefficient": "evaluated in the sweep (KL)" if kl_inline(args)
                                          else "read from memory",
                           "launches": rf["launches"], "avg_launch_us": rf["avg_launch_us"],
                           "bytes_per_launch": rf["bytes_per_launch"],
                           "profile_steps": args.profile_steps,
                           "all_active_cycles": cmin,
                           "launches_excluded": rf["launches_excluded"],
                           "per_kind": rf["per_kind"], "tiles": tiles}
        if rec:
            out["roofline"]["traffic_over_algorithmic"] = traffic / rf["bytes_per_launch"]
    if args.calib_copy:
        calib_copy(torch)
    P.destroy()
    torch.cuda.empty_cache()
    return out


def calib_copy(torch):
    """A plain 1 GiB device-to-device copy (three times): the counter runs
    scale FETCH_SIZE and WRITE_SIZE by what they read for it."""
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def bench_levelpair(args, M, torch, np, steps=None, profile=True):
    """64 coupled samples of fine 65^3 and coarse 33^3 per step (level 1 of
    n0 = 33, sigma^2 = 1, lambda = 0.1), seeds 64*s .. 64*s+63 for step s."""
    n0, level, S = 33, 1, args.samples
    steps = args.steps if steps is None else steps
    P = M.mg_plan_create(n0=n0, max_level=level, sigma2=1.0, corr_len=0.1, tol=1e-8,
                         nu1=2, nu2=2, max_cycles=50)
    for spec in args.opt:
        name, value = spec.split("=")
        M.mg_plan_set_option(P, name, int(value))
    Y = torch.zeros(S, dtype=torch.float64, device="cuda")
    Qf, Qc = torch.zeros_like(Y), torch.zeros_like(Y)
    cyc = torch.zeros(2 * S, dtype=torch.int32, device="cuda")

    def step(s, cyc_out=None):
        seeds = np.arange(s * S, (s + 1) * S, dtype=np.uint64)
        st = M.mlmc_sample_batch(P, level, seeds, S, Y, Qf, Qc, cyc if cyc_out is None else cyc_out)
        assert st == M.MG_OK, st

    for spec in args.tile:
        nn, tj, tk, ch = (int(x) for x in spec.split(":"))
        if nn in (65, 33):
            M.mg_set_tile(P, nn, tj, tk, ch)
    for spec in args.tile_pro:
        nn, tj, tk, ch = (int(x) for x in spec.split(":"))
        if nn in (65, 33):
            M.mg_set_tile_for(P, nn, 1, tj, tk, ch)
    if args.autotune and not args.tile:
        M.mg_autotune(P, level, S, 3)
    tiles = {n: M.mg_get_tile(P, n) for n in (65, 33)}
    tiles_pro = {n: M.mg_get_tile_for(P, n, 1) for n in (65, 33)}
    for s in range(args.warmup):
        step(10**5 + s)
    torch.cuda.synchronize()
    cyc_all = torch.zeros(max(1, steps), 2 * S, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_step = []
    for s in range(steps):
        step(s, cyc_all[s])  # (returns once the batch has finished)
        t_step.append(time.perf_counter())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lat_ms = 1e3 * np.diff(np.asarray([t0] + t_step))
    cyc_np = cyc_all.cpu().numpy().reshape(max(1, steps), S, 2)
    cyc_mean = float(cyc_np[:, :, 0].mean())
    value = S * steps / dt
    ms_step = 1e3 * dt / steps
    nf, nc = (n0 - 1) * 2**level + 1, (n0 - 1) * 2**(level - 1) + 1
    nodes = (nf**3 * cyc_np[:, :, 0].sum() + nc**3 * cyc_np[:, :, 1].sum())
    eff = (VCYCLE_KL_BYTES_PER_NODE if kl_inline(args) else VCYCLE_BYTES_PER_NODE) * float(nodes) / dt / 1e9
    out = _line("MLMC samples/sec per level + V-cycle HBM GB/s; p50/p99 solve latency", value,
                "samples/s", steps, args.warmup, ms_step,
                {"workload": "mlmc_level_pair_fine65_coarse33_x64", "n0": n0, "level": level,
                 "samples_per_step": S, "sigma2": 1.0, "corr_len": 0.1, "tol": 1e-8,
                 "cycle": "V(2,2) red-black GS", "parallelism": "single GPU",
                 "tiles": {str(k): list(v) for k, v in tiles.items()},
                 "tiles_pro": {str(k): list(v) for k, v in tiles_pro.items()},
                 "options": dict(o.split("=") for o in args.opt)})
    out["per_level"] = {str(level): {"samples_per_s": value, "fine_cycles_mean": cyc_mean,
                                     "effective_vcycle_GBps": eff, "batch_latency_ms": ms_step,
                                     "batch_latency_p50_ms": _pct(lat_ms, 50),
                                     "batch_latency_p99_ms": _pct(lat_ms, 99)}}
    if profile:
        M.mg_profile_enable(P, True)
        cyc_p = torch.zeros(max(1, args.profile_steps), 2 * S, dtype=torch.int32, device="cuda")
        for s in range(args.profile_steps):
            step(s, cyc_p[s])
        torch.cuda.synchronize()
        cmin = int(cyc_p.cpu().numpy().reshape(-1, S, 2)[:, :, 0].min())
        rf = sweep_roofline(M, P, nf, S, cmin, kl_inline(args))
        M.mg_profile_enable(P, False)
        tl = [list(tiles[65]), list(tiles_pro[65])]
        traffic, src, rec = read_traffic("k_sweep_levelpair65_33x64.txt", tl)
        out["roofline"] = {"bound": "hbm", "achieved": rf["achieved"], "peak": HBM_PEAK_GBPS,
                           "unit": "GB/s", "frac": rf["achieved"] / HBM_PEAK_GBPS,
                           "traffic": traffic, "traffic_source": src,
                           "kernel": "k_sweep family (fused red-black sweeps, 65^3 grids)",
                           "launches": rf["launches"], "avg_launch_us": rf["avg_launch_us"],
                           "bytes_per_launch": rf["bytes_per_launch"],
                           "all_active_cycles": cmin, "per_kind": rf["per_kind"], "tiles": tl}
        if rec:
            out["roofline"]["traffic_over_algorithmic"] = traffic / rf["bytes_per_launch"]
    if args.calib_copy:
        calib_copy(torch)
    P.destroy()
    return out


# ---- the paper's own choices as plan options (one JSON line each) ---------------------

# algorithmic bytes per node of one sweep of each option's dominant kernel:
# the finite-element colour passes read u and the three coupling arrays and
# write u (40); the SPDE box colour passes read z and b and write z (24)
FE_SWEEP_BYTES_PER_NODE = 40.0
SPDE_SWEEP_BYTES_PER_NODE = 24.0

OPTION_FORMS = {
    # workload: (plan options, nu1, nu2, oracle call, description)
    "fmg": ({"solver": 1, "qoi": 1}, 4, 4,
            "FMG-2V(4,4) with the point QoI u(1/4,1/4,1/4) (Section 7.1)"),
    "fe": ({"operator": 1}, 2, 2,
           "P1 finite elements on Kuhn tetrahedra, V(2,2) to 1e-8 (Section 3.1)"),
    "spde": ({"field": 1}, 2, 2,
             "SPDE (Whittle-Matern) field sampler on the box (-1,2)^3, V(2,2) to 1e-8 "
             "(Section 3.2)"),
}


def cpu_baseline_option(form, n0, level, threads, min_seconds, max_samples=256):
    """The oracle's step-by-step version of the same option on `threads` host
    threads, one level-pair sample per thread, in rounds until min_seconds.
    The oracle's SPDE sample at n0 = 33 takes minutes on one thread, so that
    form is timed on the same pipeline at n0 = 17 (a level pair with 1/8 of
    the nodes, box and sample grids alike) and its per-sample time scaled by
    the node ratio, 8."""
    import oracle as O
    scale, n0o = (8.0, (n0 - 1) // 2 + 1) if form == "spde" else (1.0, n0)
    call = {"fmg": lambda s: O.mlmc_sample_ex(n0o, level, s, solver="fmg", qoi="point", nu1=4,
                                              nu2=4, fmg_cycles=2),
            "fe": lambda s: O.mlmc_sample_fe(n0o, level, s),
            "spde": lambda s: O.mlmc_sample_spde(n0o, level, s)}[form]
    t1 = time.perf_counter()
    call(10**6)
    single = time.perf_counter() - t1
    print("oracle %s: one sample on one thread %.2f s" % (form, single), file=sys.stderr, flush=True)
    done, seed = 0, 10**6 + 1
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        while True:
            list(ex.map(call, range(seed, seed + threads)))
            seed += threads
            done += threads
            dt = time.perf_counter() - t0
            print("oracle %s: %d samples, %.1f s" % (form, done, dt), file=sys.stderr, flush=True)
            if dt >= min_seconds or done >= max_samples:
                break
    what = ("%d samples of the same level pair and option (seeds 1e6+1..), one per thread, "
            "%.1f s wall" % (done, dt))
    if scale != 1.0:
        what = ("%d SPDE level-pair samples of n0 = %d (box 97^3 + 49^3, grids 33^3 + 17^3; "
                "seeds 1e6+1..), one per thread, %.1f s wall; rate divided by %g, the node "
                "ratio to the n0 = 33 workload" % (done, n0o, dt, scale))
    return {"value": done / dt / scale, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": what, "single_thread_latency_s": single * scale, **host_info()}


def bench_option(args, M, torch, np):
    """One of the paper's own choices (plan options) on the level-pair shape:
    64 coupled samples of fine 65^3 and coarse 33^3 per step (level 1 of
    n0 = 33, sigma^2 = 1, lambda = 0.1), seeds 64*s .. 64*s+63 for step s;
    samples/s, the roofline of the option's dominant sweep on the 65^3 grids
    (HIP events around every such sweep in profiled eager steps), the FD
    V(2,2) level pair in the same process, and the oracle beside it."""
    form = args.workload
    opts, nu1, nu2, desc = OPTION_FORMS[form]
    n0, level, S = 33, 1, args.samples
    nf, nc = (n0 - 1) * 2**level + 1, (n0 - 1) * 2**(level - 1) + 1
    P = M.mg_plan_create(n0=n0, max_level=level, sigma2=1.0, corr_len=0.1, tol=1e-8,
                         nu1=nu1, nu2=nu2, max_cycles=50)
    for name, value in opts.items():
        M.mg_plan_set_option(P, name, value)
    Y = torch.zeros(S, dtype=torch.float64, device="cuda")
    Qf, Qc = torch.zeros_like(Y), torch.zeros_like(Y)

    def step(s, cyc_out):
        seeds = np.arange(s * S, (s + 1) * S, dtype=np.uint64)
        st = M.mlmc_sample_batch(P, level, seeds, S, Y, Qf, Qc, cyc_out)
        assert st == M.MG_OK, st

    cyc_w = torch.zeros(2 * S, dtype=torch.int32, device="cuda")
    for s in range(args.warmup):
        step(10**5 + s, cyc_w)
    steps = args.steps
    cyc_all = torch.zeros(max(1, steps), 2 * S, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        step(s, cyc_all[s])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    cyc_np = cyc_all.cpu().numpy().reshape(max(1, steps), S, 2)
    value = S * steps / dt
    out = _line("MLMC samples/sec per level + V-cycle HBM GB/s; p50/p99 solve latency", value,
                "samples/s", steps, args.warmup, 1e3 * dt / steps,
                {"workload": "mlmc_level_pair_fine65_coarse33_x64_" + form, "n0": n0,
                 "level": level, "samples_per_step": S, "sigma2": 1.0, "corr_len": 0.1,
                 "form": desc, "options": opts, "cycle": "V(%d,%d)" % (nu1, nu2),
                 "parallelism": "single GPU"})
    out["per_level"] = {str(level): {"samples_per_s": value,
                                     "fine_cycles_mean": float(cyc_np[:, :, 0].mean()),
                                     "coarse_cycles_mean": float(cyc_np[:, :, 1].mean()),
                                     "batch_latency_ms": 1e3 * dt / steps}}
    # the dominant sweep: HIP events around every sweep on the 65^3 grids (the
    # 193^3 box grids for the SPDE sampler) of profiled eager steps, counted
    # in the cycles in which every solve still cycles
    M.mg_profile_enable(P, True)
    cyc_p = torch.zeros(max(1, args.profile_steps), 2 * S, dtype=torch.int32, device="cuda")
    for s in range(args.profile_steps):
        step(s, cyc_p[s])
    torch.cuda.synchronize()
    cyc_r, kind, gn, ms = M.mg_profile_records(P)
    M.mg_profile_enable(P, False)
    if form == "spde":
        nt = 3 * (nf - 1) + 1
        sel = (kind == 5) & (gn == nt)
        # the cycles before each box solve's last one (in the last, solves
        # that converged earlier may have stopped; cycle numbers restart with
        # every box solve)
        idx = np.flatnonzero(sel)
        runs = np.split(idx, np.flatnonzero(np.diff(cyc_r[idx]) < 0) + 1) if idx.size else []
        for r in runs:
            last = cyc_r[r].max()
            sel[r[cyc_r[r] == last]] = False
        per_launch = SPDE_SWEEP_BYTES_PER_NODE * S * float(nt) ** 3
        kname = "k_spde_colour (two colour passes, %d^3 box grids)" % nt
        bpn = SPDE_SWEEP_BYTES_PER_NODE
    elif form == "fe":
        cmin = int(cyc_p.cpu().numpy().reshape(-1, S, 2)[:, :, 0].min())
        sel = (kind == 4) & (gn == nf) & (cyc_r <= cmin)
        per_launch = FE_SWEEP_BYTES_PER_NODE * S * float(nf - 2) ** 3
        kname = "k_fe_colour (two colour passes, %d^3 grids)" % nf
        bpn = FE_SWEEP_BYTES_PER_NODE
    else:
        # the fixed FMG schedule on its last stage: every solve takes every
        # one of the stage's cycles
        sel = (kind <= 3) & (gn == nf) & (cyc_r <= 2)
        per_launch = SWEEP_BYTES_PER_NODE * S * float(nf - 2) ** 3
        kname = "k_sweep family (fused red-black sweeps, %d^3 grids, last FMG stage)" % nf
        bpn = SWEEP_BYTES_PER_NODE
    n_sel = int(sel.sum())
    avg_ms = float(ms[sel].mean()) if n_sel else float("nan")
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if n_sel else 0.0
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBPS, "traffic": None, "kernel": kname,
                       "bytes_per_node": bpn, "launches": n_sel, "avg_launch_us": 1e3 * avg_ms,
                       "bytes_per_launch": per_launch, "profile_steps": args.profile_steps}
    P.destroy()
    torch.cuda.empty_cache()
    if not args.no_extra:
        fd = bench_levelpair(args, M, torch, np, steps=max(3, steps // 2), profile=False)
        out["extra"] = {"fd_vcycle_level_pair_samples_per_s": fd["value"],
                        "speed_vs_fd_vcycle": value / fd["value"]}
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline_option(form, n0, level, threads, args.cpu_seconds)
    return out


# ---- the other execution forms (one JSON line each, --workload ...) ----------------

def _line(metric, value, unit, steps, warmup, ms_step, config, higher=True, dtype="f64"):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": ms_step, "higher_is_better": higher,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic (Philox-seeded 64-term KL lognormal fields)", "config": config}


def _apply_opts(M, P, args):
    """The --opt name=value plan options."""
    for spec in args.opt:
        name, value = spec.split("=")
        M.mg_plan_set_option(P, name, int(value))


def _pct(x, q):
    import numpy as np
    return float(np.percentile(np.asarray(x), q)) if len(x) else None


def _samples(M, torch, P, level, seeds):
    n = len(seeds)
    Y = torch.zeros(n, dtype=torch.float64, device="cuda")
    Qf, Qc = torch.zeros_like(Y), torch.zeros_like(Y)
    cyc = torch.zeros(2 * n, dtype=torch.int32, device="cuda")
    return Y, Qf, Qc, cyc


def bench_single(args, M, torch, np):
    """One sample of level 0 on 33^3 (31^3 unknowns, five multigrid levels):
    latency per sample, HIP graphs vs eager launches, and of mg_solve alone."""
    n0, reps = 33, max(200, args.steps)
    P = M.mg_plan_create(n0=n0, max_level=0)
    _apply_opts(M, P, args)
    for spec in args.tile:
        nn, tj, tk, ch = (int(x) for x in spec.split(":"))
        M.mg_set_tile(P, nn, tj, tk, ch)
    for spec in args.tile_pro:
        nn, tj, tk, ch = (int(x) for x in spec.split(":"))
        M.mg_set_tile_for(P, nn, 1, tj, tk, ch)
    Y, Qf, Qc, cyc = _samples(M, torch, P, 0, [0])
    seeds = np.zeros(1, dtype=np.uint64)
    res = {}
    for mode in (1, 0):
        M.mg_plan_set_option(P, "graph", mode)
        for _ in range(max(10, args.warmup)):
            M.mlmc_sample_batch(P, 0, seeds, 1, Y, Qf, Qc, cyc)
        lat = []
        for _ in range(reps):
            t0 = time.perf_counter()
            M.mlmc_sample_batch(P, 0, seeds, 1, Y, Qf, Qc, cyc)
            lat.append(1e6 * (time.perf_counter() - t0))
        res["graph" if mode else "eager"] = {"p50_us": _pct(lat, 50), "p99_us": _pct(lat, 99)}
    cycles = int(cyc[0].item())
    # the solve alone on the same coefficient (mg_solve: caller's k, f, u)
    k = torch.empty(n0**3, dtype=torch.float64, device="cuda")
    M.mlmc_field(P, n0, 0, 0, k)
    f = torch.ones_like(k)
    u = torch.zeros_like(k)
    lat = []
    for r in range(reps + 10):
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M.mg_solve(P, n0, k, f, u)
        if r >= 10:
            lat.append(1e6 * (time.perf_counter() - t0))
    res["mg_solve"] = {"p50_us": _pct(lat, 50), "p99_us": _pct(lat, 99)}
    out = _line("single-sample latency (p50, HIP graphs)", res["graph"]["p50_us"], "us", reps,
                args.warmup, res["graph"]["p50_us"] / 1e3,
                {"workload": "single_sample_level0_n33", "n": n0, "seed": 0, "sigma2": 1.0,
                 "corr_len": 0.1, "tol": 1e-8, "cycle": "V(2,2) red-black GS, 5 levels"},
                higher=False)
    out["latency"] = res
    out["cycles"] = cycles
    return out


def bench_mixed(args, M, torch, np):
    """Batched uneven form: levels 0..3 of n0 = 17 (17^3 .. 129^3 fine grids)
    with 128/64/48/16 samples in one batch (384 solves), against the same
    samples as per-level batches and one at a time."""
    counts = {0: 128, 1: 64, 2: 48, 3: 16}
    levels, seeds = [], []
    s = 0
    for l, c in counts.items():
        levels += [l] * c
        seeds += list(range(s, s + c))
        s += c
    n = len(levels)
    P = M.mg_plan_create(n0=17, max_level=3)
    _apply_opts(M, P, args)
    Y, Qf, Qc, cyc = _samples(M, torch, P, 0, seeds)
    sd = np.asarray(seeds, dtype=np.uint64)
    for _ in range(max(1, args.warmup)):
        M.mlmc_sample_mixed(P, levels, sd, n, Y, Qf, Qc, cyc)
    steps = max(1, min(args.steps, 10))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        M.mlmc_sample_mixed(P, levels, sd, n, Y, Qf, Qc, cyc)
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t0) / steps
    cy = cyc.cpu().numpy().reshape(n, 2)
    nodes = 0.0
    for i, l in enumerate(levels):
        nf = 16 * 2**l + 1
        nodes += nf**3 * cy[i, 0] + ((nf - 1) // 2 + 1)**3 * cy[i, 1] * (l > 0)
    # the same samples level by level, and one sample at a time
    per_level, t_levels, t_plain = {}, 0.0, 0.0
    for l, c in counts.items():
        Pl = M.mg_plan_create(n0=17, max_level=3)
        idx = [i for i in range(n) if levels[i] == l]
        s_l = sd[idx]
        Yl, Qfl, Qcl, cl = _samples(M, torch, Pl, l, idx)
        M.mlmc_sample_batch(Pl, l, s_l, len(idx), Yl, Qfl, Qcl, cl)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            M.mlmc_sample_batch(Pl, l, s_l, len(idx), Yl, Qfl, Qcl, cl)
        torch.cuda.synchronize()
        tl = (time.perf_counter() - t0) / steps
        t_levels += tl
        same = bool(torch.equal(Yl, Y[idx]))
        P1 = M.mg_plan_create(n0=17, max_level=3)
        Y1, Qf1, Qc1, c1 = _samples(M, torch, P1, l, [0])
        M.mlmc_sample_batch(P1, l, s_l[:1], 1, Y1, Qf1, Qc1, c1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(len(idx)):
            M.mlmc_sample_batch(P1, l, s_l[i:i + 1], 1, Y1, Qf1, Qc1, c1)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        t_plain += tp
        per_level[str(l)] = {"samples": c, "fine_n": 16 * 2**l + 1,
                             "level_batch_samples_per_s": c / tl,
                             "one_at_a_time_samples_per_s": c / tp,
                             "mixed_equals_level_batch": same}
    value = n / t_mixed
    out = _line("MLMC samples/s, levels 0..3 in one batch", value, "samples/s", steps,
                args.warmup, 1e3 * t_mixed,
                {"workload": "mixed_levels_n0_17_counts_128_64_48_16", "n0": 17,
                 "levels": "0..3", "counts": [128, 64, 48, 16], "solves": 384, "sigma2": 1.0,
                 "corr_len": 0.1, "tol": 1e-8})
    out["per_level"] = per_level
    out["speedup_vs_level_batches"] = t_levels / t_mixed
    out["speedup_vs_one_at_a_time"] = t_plain / t_mixed
    out["effective_vcycle_GBps"] = ((VCYCLE_KL_BYTES_PER_NODE if kl_inline(args)
                                     else VCYCLE_BYTES_PER_NODE) * nodes / t_mixed / 1e9)
    return out


def bench_fp32mix(args, M, torch, np):
    """Mixed precision: 16 samples on 257^3 (sigma^2 = 2, lambda = 0.05),
    FP32 inner V-cycles in FP64 defect correction against plain FP64."""
    S, n = 16, 257
    seeds = np.arange(S, dtype=np.uint64)
    res = {}
    Q = {}
    for name, prec, inner in (("fp64", M.MG_FP64, 1), ("mixed", M.MG_MIXED, 1),
                              ("mixed_inner2", M.MG_MIXED, 2)):
        P = M.mg_plan_create(n0=n, max_level=0, sigma2=2.0, corr_len=0.05, precision=prec)
        if prec == M.MG_MIXED:
            M.mg_plan_set_option(P, "inner_cycles", inner)
        Y, Qf, Qc, cyc = _samples(M, torch, P, 0, seeds)
        M.mlmc_sample_batch(P, 0, seeds, S, Y, Qf, Qc, cyc)
        steps = max(1, min(args.steps, 3))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            M.mlmc_sample_batch(P, 0, seeds, S, Y, Qf, Qc, cyc)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        c = cyc.cpu().numpy().reshape(S, 2)[:, 0]
        per_node = VCYCLE_KL_BYTES_PER_NODE if prec == M.MG_FP64 else mixed_bytes_per_node(inner)
        res[name] = {"batch_s": dt, "samples_per_s": S / dt, "cycles_mean": float(c.mean()),
                     "effective_GBps": per_node * n**3 * float(c.sum()) / dt / 1e9}
        Q[name] = Qf.cpu().numpy()
        del P
        torch.cuda.empty_cache()
    dq = float(np.max(np.abs(Q["mixed"] - Q["fp64"]) / np.abs(Q["fp64"])))
    out = _line("MLMC samples/s, mixed precision 257^3", res["mixed"]["samples_per_s"],
                "samples/s", 3, 1, 1e3 * res["mixed"]["batch_s"],
                {"workload": "mixed_precision_n257_x16", "n": n, "samples": S, "sigma2": 2.0,
                 "corr_len": 0.05, "tol": 1e-8}, dtype="f64+f32")
    out["forms"] = res
    out["speedup_mixed_vs_fp64"] = res["fp64"]["batch_s"] / res["mixed"]["batch_s"]
    out["max_rel_dQ_mixed_vs_fp64"] = dq
    out["speedup_mixed_inner2_vs_fp64"] = res["fp64"]["batch_s"] / res["mixed_inner2"]["batch_s"]
    out["max_rel_dQ_mixed_inner2_vs_fp64"] = float(
        np.max(np.abs(Q["mixed_inner2"] - Q["fp64"]) / np.abs(Q["fp64"])))
    return out


def bench_adaptive(args, M, torch, np):
    """The whole estimator: Algorithm 2 (adaptive MLMC) to tolerance eps on
    levels 0..4 of n0 = 17 (17^3 .. 257^3 fine grids), sigma^2 = 1,
    lambda = 0.1, theta = 1/2, alpha = 2/3, N_Init = 32; wall time from eps to
    the estimate, with the number of samples and V-cycles it took."""
    P = M.mg_plan_create(n0=17, max_level=4, sigma2=1.0, corr_len=0.1)
    _apply_opts(M, P, args)
    M.mlmc_adaptive(P, eps=4 * args.eps, n_init=8, seed0=10**6)  # warm-up: workspaces, graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = M.mlmc_adaptive(P, eps=args.eps, n_init=32, seed0=0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    total = int(sum(r["N"]))
    out = _line("MLMC estimate to tolerance (Algorithm 2): wall time", dt, "s", 1, 1, 1e3 * dt,
                {"workload": "adaptive_mlmc_n0_17_levels_0_4", "n0": 17, "max_level": 4,
                 "eps": args.eps, "theta": 0.5, "alpha": 2.0 / 3.0, "n_init": 32,
                 "sigma2": 1.0, "corr_len": 0.1, "tol": 1e-8}, higher=False)
    out["estimate"] = {"Q": r["Q"], "L": r["L"], "N": r["N"], "mean": r["mean"], "var": r["var"],
                       "sampling_rms": r["sampling_rms"], "bias_estimate": r["bias_estimate"],
                       "bias_ok": r["bias_ok"], "iterations": r["iterations"]}
    out["samples"] = total
    out["samples_per_s"] = total / dt
    P.destroy()
    return out


def bench_serve(args, M, torch, np):
    """Serving: requests for samples of levels 0..3 of n0 = 33 (33^3 .. 257^3
    fine grids), level l with probability proportional to 4^-l, through the
    continuous-batching server; saturation throughput, then Poisson arrivals
    at fractions of it (p50/p99 latency), and the same traces through a plain
    first-in-first-out path that solves one sample at a time."""
    L, N = 3, args.serve_requests
    slots = None if args.serve_slots == "auto" else [int(x) for x in args.serve_slots.split(",")]
    budget = int(args.serve_budget_gib * (1 << 30))
    loads = [float(x) for x in args.serve_loads.split(",")]
    p = np.array([4.0 ** -l for l in range(L + 1)])
    lv = np.random.Generator(np.random.PCG64(0)).choice(L + 1, size=N, p=p / p.sum())
    gaps = np.random.Generator(np.random.PCG64(1)).exponential(1.0, size=N)
    P = M.mg_plan_create(n0=33, max_level=L, hbm_budget=budget)
    S = M.Server(P, slots, queue_capacity=N + 1)
    slots = [S.slots(l) for l in range(L + 1)]

    def run_server(arrivals):
        # arrivals: server-clock times (None: all at once)
        res = []
        base = S.now()
        i = 0
        while len(res) < N:
            now = S.now() - base
            while i < N and (arrivals is None or arrivals[i] <= now):
                S.submit(int(lv[i]), i, i, base + (0.0 if arrivals is None else arrivals[i]))
                i += 1
            q, r, _ = S.counts()
            if q == 0 and r == 0 and i < N:
                while S.now() - base < arrivals[i]:
                    pass
                continue
            res += S.step(1)
        lat = [x["t_done"] - x["t_arrival"] for x in res]
        span = max(x["t_done"] for x in res) - base
        return res, lat, span

    # warm: the lanes a burst opens and their graphs
    for i in range(N):
        S.submit(int(lv[i]), 10**6 + i, -1)
    while S.counts()[1] or S.counts()[0]:
        S.step(1)

    def lane_changes(m0, m1):
        return {"opened": m1["opened"] - m0["opened"], "evicted": m1["evicted"] - m0["evicted"],
                "seconds": m1["lane_seconds"] - m0["lane_seconds"]}

    mem0 = S.memory()
    res, lat, span = run_server(None)
    mem_sat = S.memory()
    sat = N / span
    acc = {l: M.mlmc_acc_init() for l in range(L + 1)}
    for x in res:
        M.mlmc_acc_add(acc[x["level"]], [x["Y"]])
    est, var_sum = 0.0, 0.0
    for l in range(L + 1):
        m, v = M.mlmc_acc_result(acc[l])
        est += m
        var_sum += v / max(1, acc[l].n)
    out = _line("served MLMC samples/s at saturation (levels 0..3 of n0=33)", sat, "samples/s",
                N, N, 1e3 * span / N,
                {"workload": "serve_n0_33_levels_0_3_p_4^-l", "n0": 33, "levels": "0..3",
                 "requests": N, "lane_slots": slots, "hbm_budget_bytes": budget,
                 "cycles_per_step": 1, "sigma2": 1.0, "corr_len": 0.1, "tol": 1e-8})
    out["saturation"] = {"samples_per_s": sat, "p50_ms": 1e3 * _pct(lat, 50),
                         "p99_ms": 1e3 * _pct(lat, 99),
                         "mlmc_estimate": est, "sampling_rms": var_sum ** 0.5,
                         "memory": mem_sat, "lane_changes": lane_changes(mem0, mem_sat),
                         "requests_per_level": [int((lv == l).sum()) for l in range(L + 1)]}
    # the plain path: one plan per level, one sample per call, in arrival order
    fifo_plans = {}
    if not args.no_fifo:
        for l in range(L + 1):
            Pl = M.mg_plan_create(n0=33, max_level=L)
            bufs = _samples(M, torch, Pl, l, [0])
            M.mlmc_sample_batch(Pl, l, np.zeros(1, dtype=np.uint64), 1, *bufs)
            fifo_plans[l] = (Pl, bufs)
    out["loads"] = {}
    for rho in loads:
        lam = rho * sat
        arr = np.cumsum(gaps) / lam
        mem0 = S.memory()
        res, lat, span = run_server(arr)
        rec = {"offered_per_s": lam, "served_per_s": N / span, "p50_ms": 1e3 * _pct(lat, 50),
               "p99_ms": 1e3 * _pct(lat, 99), "memory": S.memory(),
               "lane_changes": lane_changes(mem0, S.memory()),
               "per_level_p50_p99_ms": {
                   str(l): [1e3 * _pct([x["t_done"] - x["t_arrival"] for x in res if x["level"] == l], q)
                            for q in (50, 99)] for l in range(L + 1)}}
        if fifo_plans:
            lat_f = []
            t0 = time.perf_counter()
            for i in range(N):
                while time.perf_counter() - t0 < arr[i]:
                    pass
                Pl, bufs = fifo_plans[int(lv[i])]
                M.mlmc_sample_batch(Pl, int(lv[i]), np.array([i], dtype=np.uint64), 1, *bufs)
                lat_f.append(time.perf_counter() - t0 - arr[i])
            span_f = time.perf_counter() - t0
            rec["fifo"] = {"served_per_s": N / span_f, "p50_ms": 1e3 * _pct(lat_f, 50),
                           "p99_ms": 1e3 * _pct(lat_f, 99)}
        out["loads"][str(rho)] = rec
        print("load %.2f: %s" % (rho, json.dumps(rec)), file=sys.stderr, flush=True)
    return out


if __name__ == "__main__":
    main()
