"""GPU tests of mixed precision with several FP32 inner cycles per FP64
defect-correction step (plan option "inner_cycles").

A step computes the FP64 defect r = b' - A'u, runs c FP32 V(2,2) cycles on
A'e = r from e = 0 and adds e to u in FP64.  The V-cycle is linear in the
error, so in exact arithmetic the step equals c FP64 V-cycles; the FP32 error
of e is removed by the next step's FP64 defect.  Convergence is judged by the
FP64 residual after every step, so the reported cycle count is a multiple of c:
the first multiple of c at which the residual meets tol, i.e. the FP64
oracle's count rounded up to a multiple of c (within one step of c cycles
either way where the FP32 rounding of a step moves a residual across tol).

Bars: Q within 1e-9 |Q| of the FP64 oracle run for the same number of cycles
(the bar of the one-inner-cycle mixed path: the FP32 rounding of a step's
correction is removed by the next step's FP64 defect, and that of the last
step is below 1e-7 of a correction that is itself at the tolerance level);
the served results equal the same samples computed alone, bit for bit.
"""
import os

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


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


def _plan(M, c, **kw):
    P = M.mg_plan_create(precision=M.MG_MIXED, **kw)
    assert M.mg_plan_set_option(P, "inner_cycles", c) == M.MG_OK
    return P


def _batch(M, torch, P, level, seeds, fixed=0):
    n = len(seeds)
    Y = torch.zeros(n, dtype=torch.float64, device="cuda")
    Qf, Qc = torch.zeros_like(Y), torch.zeros_like(Y)
    cyc = torch.zeros(2 * n, dtype=torch.int32, device="cuda")
    st = M.mlmc_sample_batch(P, level, np.asarray(seeds, dtype=np.uint64), n, Y, Qf, Qc, cyc,
                             fixed_cycles=fixed)
    return (st, Y.cpu().numpy(), Qf.cpu().numpy(), Qc.cpu().numpy(),
            cyc.cpu().numpy().reshape(n, 2))


def test_inner_cycles_option_checks(M, torch):
    P = M.mg_plan_create(precision=M.MG_MIXED)
    for bad in (0, 9, -1):
        with pytest.raises(M.MGError):
            M.mg_plan_set_option(P, "inner_cycles", bad)
    for ok in (1, 2, 8):
        assert M.mg_plan_set_option(P, "inner_cycles", ok) == M.MG_OK


@pytest.mark.parametrize("c", [2, 3])
@pytest.mark.parametrize("n0,level", [(17, 1), (17, 2)])
def test_inner_cycles_against_oracle(M, torch, c, n0, level):
    seeds = list(range(300, 312))
    print("inner_cycles %d: n0 %d level %d, %d samples" % (c, n0, level, len(seeds)), flush=True)
    P = _plan(M, c, n0=n0, max_level=level, sigma2=1.0, corr_len=0.1)
    st, Y, Qf, Qc, cyc = _batch(M, torch, P, level, seeds)
    assert st == M.MG_OK
    worst, shifted = 0.0, 0
    for i, s in enumerate(seeds):
        o = O.mlmc_sample(n0, level, s, sigma2=1.0, lam=0.1)
        for k in range(2):
            up = -(-o["cycles"][k] // c) * c  # the oracle's count rounded up to a multiple of c
            assert cyc[i, k] % c == 0 and abs(int(cyc[i, k]) - up) <= c, (s, cyc[i], o["cycles"])
            shifted += int(cyc[i, k]) != up
        # the oracle with the GPU's cycle counts (fine and coarse solve)
        of = O.mlmc_sample(n0, level, s, sigma2=1.0, lam=0.1, fixed_cycles=int(cyc[i, 0]))
        oc = O.mlmc_sample(n0, level, s, sigma2=1.0, lam=0.1, fixed_cycles=int(cyc[i, 1]))
        for got, ref in ((Qf[i], of["Qf"]), (Qc[i], oc["Qc"])):
            worst = max(worst, abs(got - ref) / abs(ref))
            assert abs(got - ref) <= 1e-9 * abs(ref), (s, got, ref)
        assert Y[i] == Qf[i] - Qc[i]
    print("max rel dQ at equal cycle counts %.3e; counts off the rounded-up oracle count: %d"
          % (worst, shifted), flush=True)
    P.destroy()


def test_inner_cycles_fixed_count_rounds_up(M, torch):
    # fixed_cycles = 5 with two inner cycles per step: three steps, six cycles
    seeds = [11, 12, 13]
    P = _plan(M, 2, n0=17, max_level=1)
    st, Y, Qf, Qc, cyc = _batch(M, torch, P, 1, seeds, fixed=5)
    assert st == M.MG_OK and np.all(cyc == 6)
    worst = 0.0
    for i, s in enumerate(seeds):
        o = O.mlmc_sample(17, 1, s, fixed_cycles=6)
        for got, ref in ((Qf[i], o["Qf"]), (Qc[i], o["Qc"])):
            worst = max(worst, abs(got - ref) / abs(ref))
            assert abs(got - ref) <= 1e-9 * abs(ref), (s, got, ref)
    print("max rel dQ after six cycles %.3e" % worst, flush=True)
    P.destroy()


def test_inner_cycles_noconv_reported(M, torch):
    P = _plan(M, 2, n0=17, max_level=0, max_cycles=2)
    st, Y, Qf, Qc, cyc = _batch(M, torch, P, 0, [1, 2])
    assert st == M.MG_ENOCONV and np.all(cyc[:, 0] == -1)
    P.destroy()


def _serve_all(S, reqs):
    for tag, (lv, sd) in enumerate(reqs):
        assert S.submit(lv, sd, tag) == 0
    res = {}
    for _ in range(10000):
        for r in S.step(1, 4096):
            res[r["tag"]] = r
        if len(res) == len(reqs):
            break
    return res


def test_inner_cycles_server_equals_alone(M, torch):
    rng = np.random.default_rng(5)
    reqs = [(int(l), 9100 + 7 * i) for i, l in enumerate(rng.choice(3, size=12, p=[0.6, 0.3, 0.1]))]
    P = _plan(M, 2, n0=9, max_level=2)
    S = M.Server(P, [2, 2, 1])
    res = _serve_all(S, reqs)
    assert len(res) == len(reqs)
    P_ref = _plan(M, 2, n0=9, max_level=2)
    for lv in range(3):
        tags = [t for t, (l, _) in enumerate(reqs) if l == lv]
        if not tags:
            continue
        st, Y, Qf, Qc, cyc = _batch(M, torch, P_ref, lv, [reqs[t][1] for t in tags])
        assert st == M.MG_OK
        for i, t in enumerate(tags):
            r = res[t]
            assert r["status"] == M.MG_OK
            assert r["Y"] == Y[i] and r["Qf"] == Qf[i] and r["Qc"] == Qc[i], (lv, t)
            assert r["cycles"] == tuple(int(x) for x in cyc[i])
