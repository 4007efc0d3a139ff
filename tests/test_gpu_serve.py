"""GPU tests of the serving form (mg_serve_*).

Requests of mixed levels pass through resident slots that are reused while
other samples are mid-solve.  Each served sample must equal the same (level,
seed) computed alone by mlmc_sample_batch, bit for bit (Y, Q_f, Q_c and both
cycle counts), and, for one sample per level, the CPU oracle.
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
        from paper_1607_03252_amd import build
        build.build()
    M.lib()
    return M


def _alone(M, torch, P, level, seeds):
    n = len(seeds)
    Y = torch.zeros(n, dtype=torch.float64, device="cuda")
    Qf, Qc = torch.zeros_like(Y), torch.zeros_like(Y)
    cyc = torch.zeros(2 * n, dtype=torch.int32, device="cuda")
    st = M.mlmc_sample_batch(P, level, np.asarray(seeds, dtype=np.uint64), n, Y, Qf, Qc, cyc)
    assert st == M.MG_OK
    return Y.cpu().numpy(), Qf.cpu().numpy(), Qc.cpu().numpy(), cyc.cpu().numpy().reshape(n, 2)


def _serve_all(S, reqs, max_out=4096, cycles=1):
    for tag, (lv, sd) in enumerate(reqs):
        assert S.submit(lv, sd, tag) == 0
    res = {}
    for _ in range(10000):
        for r in S.step(cycles, max_out):
            assert r["tag"] not in res
            res[r["tag"]] = r
        if len(res) == len(reqs):
            break
    return res


def _check_equal_alone(M, torch, P_ref, reqs, res):
    by_level = {}
    for tag, (lv, sd) in enumerate(reqs):
        by_level.setdefault(lv, []).append(tag)
    for lv, tags in by_level.items():
        Y, Qf, Qc, cyc = _alone(M, torch, P_ref, lv, [reqs[t][1] for t in tags])
        for i, t in enumerate(tags):
            r = res[t]
            assert r["status"] == M.MG_OK and r["level"] == lv and r["seed"] == reqs[t][1]
            assert r["Y"] == Y[i] and r["Qf"] == Qf[i] and r["Qc"] == Qc[i], (lv, t)
            assert r["cycles"] == tuple(int(c) for c in cyc[i])


def _requests(seed, n, levels=4):
    rng = np.random.default_rng(seed)
    p = np.array([4.0 ** -l for l in range(levels)])
    lv = rng.choice(levels, size=n, p=p / p.sum())
    return [(int(l), 7000 + 13 * i) for i, l in enumerate(lv)]


def test_served_samples_equal_alone_and_oracle(M, torch):
    P = M.mg_plan_create(n0=9, max_level=3)
    S = M.Server(P, [4, 3, 2, 1])
    assert [S.slots(l) for l in range(4)] == [4, 3, 2, 1]
    reqs = _requests(1, 30)
    res = _serve_all(S, reqs)
    assert len(res) == len(reqs)
    assert S.counts() == (0, 0, len(reqs))
    for r in res.values():
        assert 0.0 <= r["t_arrival"] <= r["t_admit"] <= r["t_done"]
    P_ref = M.mg_plan_create(n0=9, max_level=3)
    _check_equal_alone(M, torch, P_ref, reqs, res)
    for lv in range(4):
        t = next((t for t, (l, _) in enumerate(reqs) if l == lv), None)
        if t is None:
            continue
        o = O.mlmc_sample(9, lv, reqs[t][1])
        r = res[t]
        assert abs(r["Qf"] - o["Qf"]) <= 1e-9 * abs(o["Qf"])
        assert abs(r["Y"] - o["Y"]) <= 1e-9 * (abs(o["Qf"]) + abs(o["Qc"]))
        assert r["cycles"] == tuple(o["cycles"])


def test_small_max_out_eager_and_plan_reuse(M, torch):
    # results held back by max_out come with later calls; eager launches give
    # the same results; the plan also runs batches between server steps
    P = M.mg_plan_create(n0=9, max_level=2)
    M.mg_plan_set_option(P, "graph", 0)
    S = M.Server(P, [3, 2, 1])
    reqs = _requests(2, 14, levels=3)
    for tag, (lv, sd) in enumerate(reqs):
        S.submit(lv, sd, tag)
    res = {}
    for it in range(10000):
        for r in S.step(2, 2):
            res[r["tag"]] = r
        if it == 3:
            _alone(M, torch, P, 1, [1, 2, 3])
        if len(res) == len(reqs):
            break
    assert len(res) == len(reqs)
    _check_equal_alone(M, torch, M.mg_plan_create(n0=9, max_level=2), reqs, res)


def test_mixed_precision_server(M, torch):
    P = M.mg_plan_create(n0=9, max_level=2, precision=M.MG_MIXED)
    S = M.Server(P, [2, 2, 1])
    reqs = _requests(3, 10, levels=3)
    res = _serve_all(S, reqs)
    _check_equal_alone(M, torch, M.mg_plan_create(n0=9, max_level=2, precision=M.MG_MIXED),
                       reqs, res)


def test_budget_sizing_and_queue_limit(M, torch):
    budget = 64 << 20
    P = M.mg_plan_create(n0=9, max_level=3, hbm_budget=budget)
    S = M.Server(P, None, queue_capacity=3)
    for l in range(4):
        f = M.mg_sample_footprint(P, l)
        k = S.slots(l)
        assert f > 0 and 1 <= k <= 256
        assert k == 1 or (k - 1) * f <= budget // 8
    assert S.memory()["lanes"] == 0 and S.memory()["used"] == 0  # nothing until requests come
    assert all(S.submit(0, i, i) == M.MG_OK for i in range(3))
    assert S.submit(0, 9, 9) == M.MG_EBUSY
    with pytest.raises(M.MGError):
        S.submit(4, 0, 0)
    while S.counts()[2] < 3:
        S.step()
    mem = S.memory()
    assert mem["lanes"] == 1 and 0 < mem["used"] <= budget and mem["budget"] == budget
    # one lane of a level larger than the budget: refused at creation
    with pytest.raises(M.MGError):
        M.Server(M.mg_plan_create(n0=9, max_level=1, hbm_budget=1 << 20), [64, 64])
    # a level with no slots is not served
    S0 = M.Server(M.mg_plan_create(n0=9, max_level=1), [2, 0])
    with pytest.raises(M.MGError):
        S0.submit(1, 0, 0)


def _lane_bytes(M, n0, L, slots, level):
    """Bytes the server counts for one lane of `level` (a server that opens
    only that lane)."""
    S = M.Server(M.mg_plan_create(n0=n0, max_level=L), slots)
    S.submit(level, 1, 0)
    while S.counts()[2] < 1:
        S.step()
    return S.memory()["used"]


def test_footprint_admission_under_a_tight_budget(M, torch):
    # the budget holds the level-3 lane and the level-0 lane but not one more
    # lane beside them: requests of mixed levels force lanes to be evicted and
    # larger requests to reserve memory; every sample still equals its value
    # computed alone, and the counted bytes never pass the budget
    slots = [4, 2, 2, 1]
    lb = [_lane_bytes(M, 9, 3, slots, l) for l in range(4)]
    assert lb[0] < lb[1] < lb[2] < lb[3]
    budget = lb[3] + lb[0] + lb[0] // 2
    assert budget < lb[3] + lb[1] and budget >= lb[2] + lb[1] + lb[0]
    P = M.mg_plan_create(n0=9, max_level=3, hbm_budget=budget)
    S = M.Server(P, slots)
    reqs = _requests(5, 40)
    res = _serve_all(S, reqs)
    assert len(res) == len(reqs)
    mem = S.memory()
    assert mem["peak"] <= budget and mem["used"] <= budget
    assert mem["evicted"] > 0 and mem["opened"] > 4
    _check_equal_alone(M, torch, M.mg_plan_create(n0=9, max_level=3), reqs, res)
    # a level-3 request behind many small ones, on a fresh server: the
    # level-0 lanes hold too much for its lane, so it reserves memory, they
    # drain and are evicted, and it is served
    S2 = M.Server(M.mg_plan_create(n0=9, max_level=3, hbm_budget=budget), slots)
    small = [(0, 9000 + i) for i in range(24)] + [(3, 9100)] + [(0, 9200 + i) for i in range(8)]
    assert 6 * lb[0] + lb[3] > budget
    res2 = _serve_all(S2, small)
    assert len(res2) == len(small)
    mem = S2.memory()
    assert mem["peak"] <= budget and mem["evicted"] > 0
    _check_equal_alone(M, torch, M.mg_plan_create(n0=9, max_level=3), small, res2)
