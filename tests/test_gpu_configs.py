"""GPU parity at the sizes of the benchmark workloads, through the C ABI.

  * mixed-precision workload's inputs (16 samples of 257^3, sigma^2 = 2,
    lambda = 0.05): the FP64 path and the mixed-precision path against the
    FP64 oracle's results stored in tests/golden/config4_fp64_257.json
    (written by tests/golden/make_config4_golden.py, which calls only the
    oracle); the mixed solution's FP64 residual computed by the oracle's own
    operator;
  * the coefficient field at 129^3 and 257^3 against the oracle's;
  * the batched uneven workload's counts (levels 0..3 of n0 = 17, 128/64/48/16
    samples in one batch) against the oracle on a few samples per level;
  * serving at n0 = 33 (levels 0..2: 33^3 .. 129^3 fine grids): served results
    equal the same samples computed alone, bit for bit, and the oracle;
  * the MLMC level accumulator (Section 2.3: mean and s^2 with divisor N)
    fed a batch's device Y, against the oracle's accumulator;
  * the largest grids (513^3, 1025^3) with k = 1 against the closed form of
    the discrete QoI.

Bars: Q within 1e-9 |Q| and equal cycle counts (the oracle's stopping rule;
mixed precision with two FP32 cycles per step: the count rounded up to an even
one, and Q against the oracle's iterate after that many cycles),
u within relative L2 1e-10 (estimated from 16 Rademacher projections of the
interior values, each of which has expectation of square ||du||^2), and the
sub-lattice values within 1e-10 of max |u|.  Set MLMC_MEASURE_OUT to a file
name to append the measured differences (one JSON line per check).
"""
import concurrent.futures as cf
import json
import os

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN4 = os.path.join(HERE, "golden", "config4_fp64_257.json")
THREADS = min(16, os.cpu_count() or 4)


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch


@pytest.fixture(scope="module")
def M(torch):
    import paper_1607_03252_amd as M
    if not os.path.exists(M.LIB_PATH):
        raise RuntimeError("libmlmcmg.so is not built")
    M.lib()
    return M


@pytest.fixture(scope="module")
def golden4():
    with open(GOLDEN4) as f:
        return json.load(f)


def measure(**kw):
    path = os.environ.get("MLMC_MEASURE_OUT")
    print(json.dumps(kw), flush=True)
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(kw) + "\n")


def rademacher(q, m):
    # the weights of tests/golden/make_config4_golden.py
    return np.random.Generator(np.random.PCG64(1000 + q)).integers(0, 2, size=m).astype(np.float64) * 2.0 - 1.0


def compare_u(rec, u, nproj, stride):
    """(relative L2 estimate from projections, sub-lattice max error / max |u|)."""
    ui = u[1:-1, 1:-1, 1:-1].ravel()
    dp = np.array([np.dot(rademacher(q, ui.size), ui) - rec["proj"][q] for q in range(nproj)])
    rel_l2 = float(np.sqrt(np.mean(dp * dp)) / rec["norm2"])
    sub = np.asarray(rec["sub"])
    dsub = float(np.max(np.abs(u[::stride, ::stride, ::stride].ravel() - sub)) / np.max(np.abs(sub)))
    return rel_l2, dsub


def batch(M, torch, P, level, seeds):
    n = len(seeds)
    Y = torch.zeros(n, dtype=torch.float64, device="cuda")
    Qf, Qc = torch.zeros_like(Y), torch.zeros_like(Y)
    cyc = torch.zeros(2 * n, dtype=torch.int32, device="cuda")
    st = M.mlmc_sample_batch(P, level, np.asarray(seeds, dtype=np.uint64), n, Y, Qf, Qc, cyc)
    return (st, Y.cpu().numpy(), Qf.cpu().numpy(), Qc.cpu().numpy(),
            cyc.cpu().numpy().reshape(n, 2))


def solve_field(M, torch, P, n, seed):
    """mg_solve with f = 1 on the device field of (seed, level 0)."""
    k = torch.empty(n**3, dtype=torch.float64, device="cuda")
    M.mlmc_field(P, n, seed, 0, k)
    f = torch.ones_like(k)
    u = torch.zeros_like(k)
    st, cyc, rel = M.mg_solve(P, n, k, f, u)
    return st, cyc, rel, u.cpu().numpy().reshape(n, n, n)


def qoi(u):
    n = u.shape[0]
    h = 1.0 / (n - 1)
    return h**3 * float(np.sum(u[1:-1, 1:-1, 1:-1]))


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed2"])
def test_config4_batch_against_oracle(M, torch, golden4, precision):
    g = golden4
    print("config4 batch: 16 x 257^3, precision %s" % precision, flush=True)
    P = M.mg_plan_create(n0=g["n"], max_level=0, sigma2=g["sigma2"], corr_len=g["lambda"],
                         tol=g["tol"], precision=M.MG_FP64 if precision == "fp64" else M.MG_MIXED)
    if precision == "mixed2":  # two FP32 V-cycles per FP64 defect-correction step
        M.mg_plan_set_option(P, "inner_cycles", 2)
    seeds = [r["seed"] for r in g["samples"]]
    st, Y, Qf, Qc, cyc = batch(M, torch, P, 0, seeds)
    assert st == M.MG_OK
    # the oracle's Q after the GPU's cycle count: its converged iterate, or
    # (two inner cycles per step stop at an even count) one cycle later
    ref = [r["Q"] if int(cyc[i, 0]) == r["cycles"] else
           r["Q_next"] if int(cyc[i, 0]) == r["cycles"] + 1 else float("nan")
           for i, r in enumerate(g["samples"])]
    dq = [abs(Qf[i] - q) / abs(q) for i, q in enumerate(ref)]
    measure(check="config4_batch_Q", precision=precision, max_rel_dQ=max(dq),
            cycles=cyc[:, 0].tolist(), oracle_cycles=[r["cycles"] for r in g["samples"]])
    assert np.array_equal(Y, Qf) and np.all(Qc == 0.0) and np.all(cyc[:, 1] == 0)
    oc = [r["cycles"] for r in g["samples"]]
    if precision == "fp64":
        assert cyc[:, 0].tolist() == oc
    else:
        # outer steps judged by the FP64 residual: the FP64 count rounded up
        # to a multiple of the cycles per step
        per = 2 if precision == "mixed2" else 1
        assert all(int(c) == -(-o // per) * per for c, o in zip(cyc[:, 0], oc))
    assert max(dq) <= 1e-9
    P.destroy()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_config4_solution_against_oracle(M, torch, golden4, precision):
    g = golden4
    n = g["n"]
    P = M.mg_plan_create(n0=n, max_level=0, sigma2=g["sigma2"], corr_len=g["lambda"],
                         tol=g["tol"], precision=M.MG_FP64 if precision == "fp64" else M.MG_MIXED)
    for rec in [r for r in g["samples"] if "proj" in r]:
        print("config4 solve: 257^3 seed %d precision %s" % (rec["seed"], precision), flush=True)
        st, cyc, rel, u = solve_field(M, torch, P, n, rec["seed"])
        assert st == M.MG_OK
        rel_l2, dsub = compare_u(rec, u, g["nproj"], g["stride"])
        dq = abs(qoi(u) - rec["Q"]) / abs(rec["Q"])
        measure(check="config4_solution", precision=precision, seed=rec["seed"], cycles=cyc,
                oracle_cycles=rec["cycles"], relres=rel, rel_l2_est=rel_l2, sub_max_rel=dsub,
                rel_dQ=dq)
        assert cyc == rec["cycles"] if precision == "fp64" else abs(cyc - rec["cycles"]) <= 1
        assert rel <= g["tol"]
        assert rel_l2 <= 1e-10 and dsub <= 1e-10 and dq <= 1e-9
        if precision == "mixed" and rec["seed"] == 0:
            # the mixed solution's FP64 residual by the oracle's own operator
            k = O.field(n, g["sigma2"], g["lambda"], O.gaussians(rec["seed"], 0))
            b = O.rhs(n)
            rho = O.norm2(O.residual(k, b, u)) / O.norm2(b)
            measure(check="config4_mixed_oracle_residual", seed=rec["seed"], rho=rho, relres=rel)
            assert rho <= g["tol"]
            assert abs(rho - rel) <= 1e-3 * rho
    P.destroy()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n,sigma2,lam,seed,level", [(129, 1.0, 0.1, 5, 2), (257, 2.0, 0.05, 3, 0)])
def test_field_large_grids(M, torch, n, sigma2, lam, seed, level):
    P = M.mg_plan_create(n0=n, max_level=0, sigma2=sigma2, corr_len=lam)
    k = torch.empty(n**3, dtype=torch.float64, device="cuda")
    M.mlmc_field(P, n, seed, level, k)
    kg = k.cpu().numpy().reshape(n, n, n)
    ko = O.field(n, sigma2, lam, O.gaussians(seed, level))
    err = float(np.max(np.abs(kg - ko) / ko))
    measure(check="field", n=n, max_rel=err)
    assert err <= 1e-13
    P.destroy()


def test_batched_uneven_counts_against_oracle(M, torch):
    """Levels 0..3 of n0 = 17 with 128/64/48/16 samples in one batch (seeds in
    level order); three samples per level against the oracle."""
    counts = [128, 64, 48, 16]
    levels, seeds = [], []
    for l, c in enumerate(counts):
        levels += [l] * c
        seeds += list(range(len(seeds), len(seeds) + c))
    n = len(levels)
    P = M.mg_plan_create(n0=17, max_level=3)
    Y = torch.zeros(n, dtype=torch.float64, device="cuda")
    Qf, Qc = torch.zeros_like(Y), torch.zeros_like(Y)
    cyc = torch.zeros(2 * n, dtype=torch.int32, device="cuda")
    st = M.mlmc_sample_mixed(P, levels, np.asarray(seeds, dtype=np.uint64), n, Y, Qf, Qc, cyc)
    assert st == M.MG_OK
    Y, Qf, Qc = Y.cpu().numpy(), Qf.cpu().numpy(), Qc.cpu().numpy()
    cyc = cyc.cpu().numpy().reshape(n, 2)
    pick = []
    start = 0
    for l, c in enumerate(counts):
        pick += [start, start + c // 2, start + c - 1]
        start += c
    with cf.ThreadPoolExecutor(THREADS) as ex:
        refs = list(ex.map(lambda i: O.mlmc_sample(17, levels[i], seeds[i]), pick))
    worst = 0.0
    for i, r in zip(pick, refs):
        worst = max(worst, abs(Qf[i] - r["Qf"]) / abs(r["Qf"]))
        assert abs(Qf[i] - r["Qf"]) <= 1e-9 * abs(r["Qf"])
        assert abs(Y[i] - r["Y"]) <= 1e-9 * (abs(r["Qf"]) + abs(r["Qc"]))
        assert tuple(cyc[i]) == tuple(r["cycles"])
    measure(check="config3_counts", max_rel_dQ=worst)


def test_serving_n0_33_equals_alone_and_oracle(M, torch):
    """Requests of levels 0..2 of n0 = 33 (33^3, 65^3 + 33^3, 129^3 + 65^3)
    through resident slots of a server, admitted while others are mid-solve;
    again under an HBM budget that holds the level-2 lane beside a level-0
    lane but not beside a level-1 lane, so lanes are evicted and reopened."""
    reqs = [(l, 500 + 7 * i) for i, l in enumerate([0, 1, 2, 0, 0, 1, 2, 0, 1, 0, 2, 0])]

    def serve(S, reqs):
        for tag, (lv, sd) in enumerate(reqs):
            assert S.submit(lv, sd, tag) == M.MG_OK
        res = {}
        for _ in range(100000):
            for r in S.step(1):
                res[r["tag"]] = r
            if len(res) == len(reqs):
                break
        assert len(res) == len(reqs)
        return res

    def lane_bytes(level):
        # the bytes a server counts for one lane of `level`
        Sx = M.Server(M.mg_plan_create(n0=33, max_level=2), [4, 2, 2])
        serve(Sx, [(level, 1)])
        return Sx.memory()["used"]

    lb = [lane_bytes(l) for l in range(3)]
    S = M.Server(M.mg_plan_create(n0=33, max_level=2), [4, 2, 2])
    res = serve(S, reqs)
    budget = lb[2] + lb[0] + lb[0] // 2
    assert budget < lb[2] + lb[1]
    St = M.Server(M.mg_plan_create(n0=33, max_level=2, hbm_budget=budget), [4, 2, 2])
    res_t = serve(St, reqs)
    mem = St.memory()
    assert mem["peak"] <= budget and mem["evicted"] > 0
    for tag in res:
        a, b = res[tag], res_t[tag]
        assert (a["Y"], a["Qf"], a["Qc"], a["cycles"]) == (b["Y"], b["Qf"], b["Qc"], b["cycles"])
    Pr = M.mg_plan_create(n0=33, max_level=2)
    for tag, (lv, sd) in enumerate(reqs):
        st, Y, Qf, Qc, cyc = batch(M, torch, Pr, lv, [sd])
        r = res[tag]
        assert r["status"] == M.MG_OK
        assert (r["Y"], r["Qf"], r["Qc"]) == (Y[0], Qf[0], Qc[0])
        assert r["cycles"] == tuple(int(c) for c in cyc[0])
    with cf.ThreadPoolExecutor(THREADS) as ex:
        refs = list(ex.map(lambda q: O.mlmc_sample(33, q[0], q[1]), reqs))
    for tag, o in enumerate(refs):
        r = res[tag]
        assert abs(r["Qf"] - o["Qf"]) <= 1e-9 * abs(o["Qf"])
        assert abs(r["Y"] - o["Y"]) <= 1e-9 * (abs(o["Qf"]) + abs(o["Qc"]))
        assert r["cycles"] == tuple(o["cycles"])
    S.destroy()
    St.destroy()


def test_serving_config5_levels_0_to_3_under_a_tight_budget(M, torch):
    """Config 5's level range (n0 = 33: 33^3 up to 257^3 + 129^3) through a
    server whose HBM budget holds the level-3 lane beside one level-0 lane
    and nothing else, with a mix of levels in the 4^-l proportions: lanes are
    evicted and reopened, and every served sample equals the same sample
    computed alone, bit for bit (Y, Q_f, Q_c and both cycle counts)."""
    slots = [8, 4, 2, 1]

    def serve(S, reqs):
        for tag, (lv, sd) in enumerate(reqs):
            assert S.submit(lv, sd, tag) == M.MG_OK
        res = {}
        for _ in range(100000):
            for r in S.step(1):
                res[r["tag"]] = r
            if len(res) == len(reqs):
                break
        assert len(res) == len(reqs)
        return res

    def lane_bytes(level):
        Sx = M.Server(M.mg_plan_create(n0=33, max_level=3), slots)
        serve(Sx, [(level, 1)])
        b = Sx.memory()["used"]
        Sx.destroy()
        return b

    lb = [lane_bytes(l) for l in range(4)]
    budget = lb[3] + lb[0] + lb[0] // 2
    assert budget < lb[3] + lb[1]
    rng = np.random.default_rng(55)
    p = np.array([4.0 ** -l for l in range(4)])
    lv = list(rng.choice(4, size=22, p=p / p.sum()))
    lv[5], lv[14] = 3, 3  # two level-3 requests among the small ones
    reqs = [(int(l), 900 + 11 * i) for i, l in enumerate(lv)]
    S = M.Server(M.mg_plan_create(n0=33, max_level=3, hbm_budget=budget), slots)
    res = serve(S, reqs)
    mem = S.memory()
    assert mem["peak"] <= budget and mem["evicted"] > 0
    Pr = M.mg_plan_create(n0=33, max_level=3)
    for tag, (l, sd) in enumerate(reqs):
        st, Y, Qf, Qc, cyc = batch(M, torch, Pr, l, [sd])
        r = res[tag]
        assert r["status"] == M.MG_OK
        assert (r["Y"], r["Qf"], r["Qc"]) == (Y[0], Qf[0], Qc[0]), (tag, l)
        assert r["cycles"] == tuple(int(c) for c in cyc[0])
    S.destroy()


def test_level_accumulator_fed_device_y(M, torch):
    """Section 2.3: the level mean and s^2 (divisor N) from a batch's device Y
    (mlmc_acc_add reading device memory) against the oracle's accumulator
    fed the oracle's own Y of the same seeds, and bit for bit against the
    oracle's accumulator fed the GPU's Y."""
    P = M.mg_plan_create(n0=9, max_level=2)
    seeds = list(range(300, 364))
    n = len(seeds)
    Y = torch.zeros(n, dtype=torch.float64, device="cuda")
    Qf, Qc = torch.zeros_like(Y), torch.zeros_like(Y)
    assert M.mlmc_sample_batch(P, 2, np.asarray(seeds, dtype=np.uint64), n, Y, Qf, Qc) == M.MG_OK
    acc = M.mlmc_acc_init()
    M.mlmc_acc_add(acc, Y[:40])   # two calls: the accumulator carries its shift
    M.mlmc_acc_add(acc, Y[40:])
    mean, var = M.mlmc_acc_result(acc)
    assert acc.n == n
    yg = Y.cpu().numpy()
    same = O.LevelAcc()
    for y in yg:
        same.add(float(y))
    assert (mean, var) == same.result()
    refs = [O.mlmc_sample(9, 2, s) for s in seeds]
    ref = O.LevelAcc()
    for r in refs:
        ref.add(r["Y"])
    m_o, v_o = ref.result()
    scale = max(abs(r["Qf"]) + abs(r["Qc"]) for r in refs)
    assert abs(mean - m_o) <= 1e-9 * scale
    # s^2 of values that agree to 1e-9 * scale agrees to about 2 * 1e-9 * scale * |Y|
    assert abs(var - v_o) <= 4e-9 * scale * float(np.max(np.abs(yg))) + 1e-300
    assert var > 0.0


@pytest.mark.parametrize("n", [513, 1025])
def test_largest_grids_constant_coefficient_closed_form(M, torch, n):
    """The largest grids: 513^3 (the largest on which the fused kernels'
    32-bit whole-grid offsets fit) and 1025^3 (the largest a plan takes; its
    finest level runs the colour sweeps and the separate residual kernels).
    With sigma^2 = 0 (k = 1) the QoI of the discrete problem has the mode-sum
    closed form of tests/closed_forms.py; 16 fixed V(2,2) cycles leave an
    algebraic error far below the bar (the FP64 residual floor at 1025^3,
    about 4e-11 relative, is above the usual tolerance's reach)."""
    from closed_forms import q_const_modes
    print("largest grids: one sample of %d^3, sigma^2 = 0, 16 cycles" % n, flush=True)
    P = M.mg_plan_create(n0=n, max_level=0, sigma2=0.0)
    Y = torch.zeros(1, dtype=torch.float64, device="cuda")
    Qf, Qc = torch.zeros_like(Y), torch.zeros_like(Y)
    cyc = torch.zeros(2, dtype=torch.int32, device="cuda")
    st = M.mlmc_sample_batch(P, 0, np.array([3], dtype=np.uint64), 1, Y, Qf, Qc, cyc,
                             fixed_cycles=16)
    assert st == M.MG_OK
    q = q_const_modes(n)
    got = float(Qf.item())
    measure(check="largest_grid_closed_form", n=n, cycles=int(cyc[0].item()), Q=got,
            closed_form=q, rel_dQ=abs(got - q) / q)
    assert int(cyc[0].item()) == 16
    assert abs(got - q) <= 1e-9 * q
    P.destroy()
    torch.cuda.empty_cache()
