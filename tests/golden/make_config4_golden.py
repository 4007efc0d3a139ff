"""Write tests/golden/config4_fp64_257.json: the FP64 CPU oracle's results on
the mixed-precision workload's inputs (16 samples of one 257^3 solve each,
seeds 0..15, MLMC level 0 of n0 = 257, sigma^2 = 2, lambda = 0.05, f = 1,
zero initial guess, V(2,2) red-black Gauss-Seidel to relative residual 1e-8).

Calls only the oracle (oracle/); nothing here comes from the HIP library.
For every seed: Q = integral of u, the cycle count and the relative residual
history, and Q_next, the integral of the iterate after one more V(2,2) cycle
(the result of a solver that stops one cycle later, e.g. at an even count).  For seeds 0 and 1 also ||u||_2 over the interior, u on the
sub-lattice of every 16th vertex per axis, and the projections <u, w_q> on
16 Rademacher vectors w_q (entries +-1 over the interior vertices, drawn
from numpy's PCG64 with seed 1000 + q, 0 -> -1 and 1 -> +1), from which a
test estimates the relative L2 difference of another solution without the
full field.

Usage: python tests/golden/make_config4_golden.py [THREADS]
(about 2.5 minutes of one core per seed).
"""
import concurrent.futures as cf
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402

N, SIGMA2, LAM, TOL = 257, 2.0, 0.05, 1e-8
SEEDS = list(range(16))
DETAIL = (0, 1)
STRIDE = 16
NPROJ = 16


def rademacher(q, m):
    return np.random.Generator(np.random.PCG64(1000 + q)).integers(0, 2, size=m).astype(np.float64) * 2.0 - 1.0


def one(seed):
    xi = O.gaussians(seed, 0)
    k = O.field(N, SIGMA2, LAM, xi)
    u, cyc, rel, hist = O.solve(k, O.rhs(N), tol=TOL, max_cycles=50)
    rec = {"seed": seed, "Q": O.qoi(u), "cycles": cyc, "relres": rel, "history": hist.tolist(),
           "Q_next": O.qoi(O.vcycle(k, O.rhs(N), u))}
    if seed in DETAIL:
        ui = u[1:-1, 1:-1, 1:-1].ravel()
        rec["norm2"] = O.norm2(u)
        rec["sub"] = u[::STRIDE, ::STRIDE, ::STRIDE].ravel().tolist()
        rec["proj"] = [float(np.dot(rademacher(q, ui.size), ui)) for q in range(NPROJ)]
    print("seed %d: Q %.17g cycles %d" % (seed, rec["Q"], cyc), flush=True)
    return rec


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    with cf.ThreadPoolExecutor(threads) as ex:
        recs = list(ex.map(one, SEEDS))
    out = {"workload": "16 x 257^3, level 0 of n0 = 257, sigma2 2, lambda 0.05, f = 1, "
                       "V(2,2) red-black GS to relres 1e-8, FP64 CPU oracle",
           "n": N, "sigma2": SIGMA2, "lambda": LAM, "tol": TOL, "stride": STRIDE,
           "nproj": NPROJ, "samples": recs}
    with open(os.path.join(HERE, "config4_fp64_257.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
