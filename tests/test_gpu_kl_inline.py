"""GPU tests of the smoother and transfer that evaluate the KL coefficient
themselves (plan option "kl"): the samples are identical, bit for bit (Y,
Q_f, Q_c and both cycle counts), to those of the kernels that read the
stored coefficient, on the level-pair, the 257^3, the mixed-level and the
full-multigrid forms, with graphs and eagerly.  (Their agreement with the
oracle follows: the parity tests run with kl = 0, the default.)"""
import os

import numpy as np
import pytest

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


def _batch(M, torch, P, level, seeds):
    n = len(seeds)
    Y = torch.zeros(n, dtype=torch.float64, device="cuda")
    Qf, Qc = torch.zeros_like(Y), torch.zeros_like(Y)
    cyc = torch.zeros(2 * n, dtype=torch.int32, device="cuda")
    st = M.mlmc_sample_batch(P, level, np.asarray(seeds, dtype=np.uint64), n, Y, Qf, Qc, cyc)
    assert st == M.MG_OK
    return [a.cpu().numpy() for a in (Y, Qf, Qc, cyc)]


def _mixed(M, torch, P, levels, seeds):
    n = len(seeds)
    Y = torch.zeros(n, dtype=torch.float64, device="cuda")
    Qf, Qc = torch.zeros_like(Y), torch.zeros_like(Y)
    cyc = torch.zeros(2 * n, dtype=torch.int32, device="cuda")
    st = M.mlmc_sample_mixed(P, np.asarray(levels, dtype=np.int32),
                             np.asarray(seeds, dtype=np.uint64), n, Y, Qf, Qc, cyc)
    assert st == M.MG_OK
    return [a.cpu().numpy() for a in (Y, Qf, Qc, cyc)]


def _same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("graph", [1, 0])
def test_level_pairs_identical(M, torch, graph):
    print("kl inline: 32 level-1 pairs 65^3 + 33^3, graph %d" % graph, flush=True)
    P = M.mg_plan_create(n0=33, max_level=1)
    M.mg_plan_set_option(P, "graph", graph)
    seeds = list(range(500, 532))
    M.mg_plan_set_option(P, "kl", 1)
    on = _batch(M, torch, P, 1, seeds)
    M.mg_plan_set_option(P, "kl", 0)
    off = _batch(M, torch, P, 1, seeds)
    _same(on, off)
    P.destroy()


def test_257_batch_identical(M, torch):
    print("kl inline: 16 x 257^3, sigma^2 2, lambda 0.05", flush=True)
    P = M.mg_plan_create(n0=257, max_level=0, sigma2=2.0, corr_len=0.05)
    seeds = list(range(16))
    M.mg_plan_set_option(P, "kl", 1)
    on = _batch(M, torch, P, 0, seeds)
    M.mg_plan_set_option(P, "kl", 0)
    off = _batch(M, torch, P, 0, seeds)
    _same(on, off)
    P.destroy()
    torch.cuda.empty_cache()


def test_mixed_levels_identical(M, torch):
    print("kl inline: levels 0..3 of n0 17 in one batch", flush=True)
    P = M.mg_plan_create(n0=17, max_level=3)
    levels = [0] * 12 + [1] * 6 + [2] * 3 + [3] * 2
    seeds = list(range(900, 900 + len(levels)))
    M.mg_plan_set_option(P, "kl", 1)
    on = _mixed(M, torch, P, levels, seeds)
    M.mg_plan_set_option(P, "kl", 0)
    off = _mixed(M, torch, P, levels, seeds)
    _same(on, off)
    P.destroy()


def test_fmg_identical(M, torch):
    print("kl inline: FMG-2V(4,4), level 2 of n0 17", flush=True)
    P = M.mg_plan_create(n0=17, max_level=2, nu1=4, nu2=4)
    M.mg_plan_set_option(P, "solver", 1)
    seeds = list(range(40, 48))
    M.mg_plan_set_option(P, "kl", 1)
    on = _batch(M, torch, P, 2, seeds)
    M.mg_plan_set_option(P, "kl", 0)
    off = _batch(M, torch, P, 2, seeds)
    _same(on, off)
    P.destroy()


def test_option_checks(M, torch):
    P = M.mg_plan_create(n0=9, max_level=0)
    with pytest.raises(M.MGError):
        M.mg_plan_set_option(P, "kl", 2)
    M.mg_plan_set_option(P, "kl", 0)
    M.mg_plan_set_option(P, "kl", 1)
    P.destroy()
