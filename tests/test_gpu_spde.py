"""GPU tests of the SPDE field sampler (plan option "field" = 1, Section 3.2,
eq. spde) through the C ABI, against the oracle's sampler (or_spde_*,
or_mlmc_sample_spde): the same white noise, box operator, V-cycles and
stopping rule (relative residual 1e-10 over every box vertex).

Bars: the field k within relative 1e-10 (the two box solves stop at the same
cycle; their iterates then agree to rounding); samples: Q within 1e-9 |Q|,
Y within 1e-9 (|Q_f| + |Q_c|), equal cycle counts of the PDE solves."""
import concurrent.futures as cf
import os

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu
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


def oracle_fields(n_f, sigma2, lam, seed, level, coarse):
    nt = O.box_n(n_f)
    xi = O.white_noise(seed, level, nt**3)
    b = O.spde_rhs(n_f, xi)
    kappa = 1.0 / lam
    if not coarse:
        z, _, _ = O.spde_solve(b, 1.0 / (n_f - 1), kappa, tol=1e-10)
        return O.spde_to_k(n_f, sigma2, lam, z)
    n_c = (n_f - 1) // 2 + 1
    z, _, _ = O.spde_solve(O.spde_restrict(b), 1.0 / (n_c - 1), kappa, tol=1e-10)
    return O.spde_to_k(n_c, sigma2, lam, z)


@pytest.mark.parametrize("n0,level,lam,coarse", [(9, 0, 0.25, False), (9, 1, 0.1, False),
                                                 (9, 1, 0.1, True), (17, 1, 0.25, True)])
def test_spde_field_against_oracle(M, torch, n0, level, lam, coarse):
    sigma2, seed = 1.0, 77
    print("spde field n0 %d level %d coarse %s" % (n0, level, coarse), flush=True)
    P = M.mg_plan_create(n0=n0, max_level=level, sigma2=sigma2, corr_len=lam)
    M.mg_plan_set_option(P, "field", 1)
    n_f = O.grid_n(n0, level)
    n = (n_f - 1) // 2 + 1 if coarse else n_f
    k = torch.empty(n**3, dtype=torch.float64, device="cuda")
    M.mlmc_field(P, n, seed, level, k)
    kg = k.cpu().numpy().reshape(n, n, n)
    ko = oracle_fields(n_f, sigma2, lam, seed, level, coarse)
    err = float(np.max(np.abs(kg - ko) / ko))
    print("max rel field error %.3e" % err, flush=True)
    assert err <= 1e-10
    P.destroy()


@pytest.mark.parametrize("n0,level", [(5, 0), (5, 1), (9, 2)])
def test_spde_samples_against_oracle(M, torch, n0, level):
    sigma2, lam = 1.0, 0.2
    P = M.mg_plan_create(n0=n0, max_level=level, sigma2=sigma2, corr_len=lam)
    M.mg_plan_set_option(P, "field", 1)
    seeds = [5, 6, 7, 8]
    n = len(seeds)
    Y = torch.zeros(n, dtype=torch.float64, device="cuda")
    Qf, Qc = torch.zeros_like(Y), torch.zeros_like(Y)
    cyc = torch.zeros(2 * n, dtype=torch.int32, device="cuda")
    assert M.mlmc_sample_batch(P, level, np.asarray(seeds, dtype=np.uint64), n, Y, Qf, Qc, cyc) == M.MG_OK
    Y, Qf, Qc = Y.cpu().numpy(), Qf.cpu().numpy(), Qc.cpu().numpy()
    cyc = cyc.cpu().numpy().reshape(n, 2)
    with cf.ThreadPoolExecutor(THREADS) as ex:
        refs = list(ex.map(lambda s: O.mlmc_sample_spde(n0, level, s, sigma2=sigma2, lam=lam), seeds))
    for i, r in enumerate(refs):
        assert abs(Qf[i] - r["Qf"]) <= 1e-9 * abs(r["Qf"])
        assert abs(Qc[i] - r["Qc"]) <= 1e-9 * abs(r["Qc"])
        assert abs(Y[i] - r["Y"]) <= 1e-9 * (abs(r["Qf"]) + abs(r["Qc"]))
        assert tuple(int(c) for c in cyc[i]) == tuple(r["cycles"])
    P.destroy()


def test_spde_option_checks(M, torch):
    P = M.mg_plan_create(n0=9, max_level=1)
    M.mg_plan_set_option(P, "field", 1)
    with pytest.raises(M.MGError):
        M.mg_plan_set_option(P, "solver", 1)
    with pytest.raises(M.MGError):
        M.Server(P, [2, 2])
    k = torch.empty(33**3, dtype=torch.float64, device="cuda")
    with pytest.raises(M.MGError):
        M.mlmc_field(P, 33, 1, 1, k)  # neither n_1 = 17 nor n_0 = 9
