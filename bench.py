"""Benchmark of the MLMC multigrid hot path on one MI355X.

Workload (one step): one MLMC level-pair batch of 64 coupled samples, fine
65^3 and coarse 33^3 grids on one omega each (n0 = 33, level 1), seeds
64*s .. 64*s+63 for step s, sigma^2 = 1, lambda = 0.1, f = 1, V(2,2)
red-black Gauss-Seidel to relative residual 1e-8, QoI = integral of u,
Y_1 = Q_1 - Q_0 per sample.  Inputs are generated on the device from seeds;
everything stays resident in HBM.

Prints one JSON line (see the repository's design notes for the byte model):
  value      = samples (Y_1 values) per second over the timed steps;
  roofline   = the finest-grid smoothing kernel's algorithmic bytes per
               launch / its mean launch time (HIP events on the plan's stream)
               against the 8 TB/s HBM peak;
  cpu_baseline = the FP64 CPU oracle on a bounded sample of the same
               workload, one sample per thread.
"""
import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# algorithmic bytes per interior node of one fused red-black sweep with a
# constant right-hand side: wh (8) + u read (8) + u written (8)
SWEEP_BYTES_PER_NODE = 24.0
# byte model of one FP64 V(2,2) cycle per finest-grid node (whole hierarchy)
VCYCLE_BYTES_PER_NODE = 195.0


def cpu_baseline(n0, level, samples, threads):
    import oracle as O
    seeds = list(range(10**6, 10**6 + samples))
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(lambda s: O.mlmc_sample(n0, level, s), seeds))
    dt = time.perf_counter() - t0
    return samples / dt, dt, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--samples", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=16)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=3)
    ap.add_argument("--tile", action="append", default=[],
                    help="n:tj:tk:chunks, pins a smoother tile shape (skips the autotuner)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
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
        from paper_1607_03252_amd import build
        build.build()

    n0, level, S = 33, 1, args.samples
    P = M.mg_plan_create(n0=n0, max_level=level, sigma2=1.0, corr_len=0.1, tol=1e-8,
                         nu1=2, nu2=2, max_cycles=50)
    Y = torch.zeros(S, dtype=torch.float64, device="cuda")
    Qf, Qc = torch.zeros_like(Y), torch.zeros_like(Y)
    cyc = torch.zeros(2 * S, dtype=torch.int32, device="cuda")

    def step(s):
        seeds = np.arange(s * S, (s + 1) * S, dtype=np.uint64)
        st = M.mlmc_sample_batch(P, level, seeds, S, Y, Qf, Qc, cyc)
        assert st == M.MG_OK, st

    for spec in args.tile:
        nn, tj, tk, ch = (int(x) for x in spec.split(":"))
        M.mg_set_tile(P, nn, tj, tk, ch)
    if not args.no_autotune and not args.tile:
        M.mg_autotune(P, level, S, 3)
    tiles = {n: M.mg_get_tile(P, n) for n in (65, 33, 17, 9, 5)}
    for s in range(args.warmup):
        step(10**5 + s)
    torch.cuda.synchronize()
    cycles_f = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(s)
        cycles_f.append(cyc.view(S, 2)[:, 0].float().mean())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    cyc_mean = float(torch.stack(cycles_f).mean().item())
    # per-kernel timing of the finest-grid smoother: HIP events on the plan's
    # stream around each launch (eager launches, same kernels and inputs)
    M.mg_profile_enable(P, True)
    for s in range(args.profile_steps):
        step(s)
    launches, ms, nodes = M.mg_profile_read(P)
    M.mg_profile_enable(P, False)

    if args.calib_copy:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    value = S * args.steps / dt
    ms_step = 1e3 * dt / args.steps
    avg_ms = ms / max(launches, 1)
    bytes_launch = SWEEP_BYTES_PER_NODE * nodes
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9 if launches else 0.0
    nf, nc = (n0 - 1) * 2**level + 1, (n0 - 1) * 2**(level - 1) + 1
    eff = VCYCLE_BYTES_PER_NODE * (nf**3 + nc**3) * S * cyc_mean * args.steps / dt / 1e9

    out = {
        "metric": "MLMC samples/sec per level + V-cycle HBM GB/s; p50/p99 solve latency",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (Philox-seeded 64-term KL lognormal fields)",
        "config": {"workload": "mlmc_level_pair_fine65_coarse33_x64", "n0": n0, "level": level,
                   "samples_per_step": S, "sigma2": 1.0, "corr_len": 0.1, "tol": 1e-8,
                   "cycle": "V(2,2) red-black GS", "parallelism": "single GPU",
                   "tiles": {str(k): list(v) for k, v in tiles.items()}},
        "per_level": {str(level): {"samples_per_s": value, "fine_cycles_mean": cyc_mean,
                                   "effective_vcycle_GBps": eff,
                                   "batch_latency_ms": ms_step}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": None,
                     "kernel": "k_sweep (fused red-black sweep, 65^3 grids)", "launches": launches,
                     "tile": list(tiles[65]),
                     "avg_launch_us": avg_ms * 1e3, "bytes_per_launch": bytes_launch},
    }
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        v, cdt, _ = cpu_baseline(n0, level, args.cpu_samples, threads)
        out["cpu_baseline"] = {"value": v, "unit": "samples/s", "cores": threads, "kind": "oracle",
                               "sample": "%d samples of the same level pair (seeds 1e6..), one "
                                         "sample per thread, %.1f s wall" % (args.cpu_samples, cdt)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
