"""GPU tests of the paper's solver schedule and QoIs through the C ABI.

  * plan option "solver" = 1: full multigrid (nested iteration, Section 7.1's
    FMG-2V(4,4) with nu1 = nu2 = 4, two cycles per grid) on MLMC samples,
    against the oracle's FMG (or_fmg) on the same omega;
  * plan option "qoi" = 1 / 2: the point value u(1/4,1/4,1/4) and the flux
    of -k grad u across x_2 = 1/4 (Section 3), with FMG and with V-cycles to
    tol, against the oracle's QoIs of the same solves.
Bars as for the integral QoI: |dQ| <= 1e-9 |Q| (flux and point values are
O(1e-2) and bounded away from zero for these fields), |dY| <= 1e-9
(|Q_f| + |Q_c|), cycle counts equal.
"""
import concurrent.futures as cf
import os

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 4)
KIND = {"integral": 0, "point": 1, "flux": 2}


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


def run(M, torch, P, levels, seeds, mixed=False):
    n = len(seeds)
    Y = torch.zeros(n, dtype=torch.float64, device="cuda")
    Qf, Qc = torch.zeros_like(Y), torch.zeros_like(Y)
    cyc = torch.zeros(2 * n, dtype=torch.int32, device="cuda")
    sd = np.asarray(seeds, dtype=np.uint64)
    if mixed:
        st = M.mlmc_sample_mixed(P, levels, sd, n, Y, Qf, Qc, cyc)
    else:
        st = M.mlmc_sample_batch(P, levels, sd, n, Y, Qf, Qc, cyc)
    assert st == M.MG_OK
    return Y.cpu().numpy(), Qf.cpu().numpy(), Qc.cpu().numpy(), cyc.cpu().numpy().reshape(n, 2)


def check(refs, Y, Qf, Qc, cyc):
    for i, r in enumerate(refs):
        assert abs(Qf[i] - r["Qf"]) <= 1e-9 * abs(r["Qf"]), (i, Qf[i], r["Qf"])
        assert abs(Qc[i] - r["Qc"]) <= 1e-9 * abs(r["Qc"]), (i, Qc[i], r["Qc"])
        assert abs(Y[i] - r["Y"]) <= 1e-9 * (abs(r["Qf"]) + abs(r["Qc"]))
        assert tuple(int(c) for c in cyc[i]) == tuple(r["cycles"])


@pytest.mark.parametrize("qoi", ["integral", "point", "flux"])
@pytest.mark.parametrize("n0,level", [(5, 0), (5, 1), (9, 2), (17, 2)])
def test_fmg_samples_against_oracle(M, torch, qoi, n0, level):
    print("fmg: n0 %d level %d qoi %s" % (n0, level, qoi), flush=True)
    P = M.mg_plan_create(n0=n0, max_level=level, nu1=4, nu2=4)
    M.mg_plan_set_option(P, "solver", 1)
    M.mg_plan_set_option(P, "qoi", KIND[qoi])
    seeds = [11, 12, 13, 14, 15]
    Y, Qf, Qc, cyc = run(M, torch, P, level, seeds)
    with cf.ThreadPoolExecutor(THREADS) as ex:
        refs = list(ex.map(lambda s: O.mlmc_sample_ex(n0, level, s, solver="fmg", qoi=qoi, nu1=4,
                                                      nu2=4, fmg_cycles=2), seeds))
    check(refs, Y, Qf, Qc, cyc)
    # batch independence: one sample alone gives the same bits
    Y1, Qf1, Qc1, _ = run(M, torch, P, level, seeds[2:3])
    assert (Y1[0], Qf1[0], Qc1[0]) == (Y[2], Qf[2], Qc[2])
    P.destroy()


def test_fmg_mixed_levels_and_129(M, torch):
    # FMG-2V(4,4) on levels 0..2 of n0 = 33 (33^3, 65^3 + 33^3, 129^3 + 65^3)
    # in one mixed-level call, point QoI, and a one-cycle schedule
    P = M.mg_plan_create(n0=33, max_level=2, nu1=4, nu2=4)
    M.mg_plan_set_option(P, "solver", 1)
    M.mg_plan_set_option(P, "qoi", 1)
    levels = [2, 0, 1, 2, 0, 1]
    seeds = [3, 4, 5, 6, 7, 8]
    Y, Qf, Qc, cyc = run(M, torch, P, levels, seeds, mixed=True)
    with cf.ThreadPoolExecutor(THREADS) as ex:
        refs = list(ex.map(lambda a: O.mlmc_sample_ex(33, a[0], a[1], solver="fmg", qoi="point",
                                                      nu1=4, nu2=4), zip(levels, seeds)))
    check(refs, Y, Qf, Qc, cyc)
    M.mg_plan_set_option(P, "fmg_cycles", 1)
    Y, Qf, Qc, cyc = run(M, torch, P, 1, [9, 10])
    refs = [O.mlmc_sample_ex(33, 1, s, solver="fmg", qoi="point", nu1=4, nu2=4, fmg_cycles=1)
            for s in (9, 10)]
    check(refs, Y, Qf, Qc, cyc)
    P.destroy()


@pytest.mark.parametrize("qoi", ["point", "flux"])
def test_vcycle_samples_with_point_and_flux_qoi(M, torch, qoi):
    P = M.mg_plan_create(n0=17, max_level=2)
    M.mg_plan_set_option(P, "qoi", KIND[qoi])
    seeds = list(range(40, 52))
    Y, Qf, Qc, cyc = run(M, torch, P, 2, seeds)
    with cf.ThreadPoolExecutor(THREADS) as ex:
        refs = list(ex.map(lambda s: O.mlmc_sample_ex(17, 2, s, qoi=qoi), seeds))
    check(refs, Y, Qf, Qc, cyc)
    P.destroy()


def test_option_checks(M, torch):
    P = M.mg_plan_create(n0=3, max_level=1)
    with pytest.raises(M.MGError):
        M.mg_plan_set_option(P, "qoi", 1)  # x* is not a vertex of the 3^3 grid
    Pm = M.mg_plan_create(n0=9, max_level=1, precision=M.MG_MIXED)
    with pytest.raises(M.MGError):
        M.mg_plan_set_option(Pm, "solver", 1)
    Ps = M.mg_plan_create(n0=9, max_level=1)
    M.mg_plan_set_option(Ps, "solver", 1)
    with pytest.raises(M.MGError):
        M.Server(Ps, [2, 2])
