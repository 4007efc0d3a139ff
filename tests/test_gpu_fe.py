"""GPU tests of the P1 finite-element operator (plan option "operator" = 1,
Section 3.1 on the Kuhn tetrahedra of the vertex grid) through the C ABI,
against the oracle's element-by-element assembly (or_fe_*).

Bars as for the FD operator: solution after the oracle's cycle count within
relative L2 1e-10, equal cycle counts to tol, Q within 1e-9 |Q| and Y within
1e-9 (|Q_f| + |Q_c|); a sample alone equals the same sample in a batch bit
for bit."""
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


@pytest.mark.parametrize("n,sigma2,lam,seed", [(17, 1.0, 0.1, 2), (33, 2.0, 0.05, 3), (65, 1.0, 0.1, 4)])
def test_fe_solve_against_oracle(M, torch, n, sigma2, lam, seed):
    print("fe solve n %d" % n, flush=True)
    k = O.field(n, sigma2, lam, O.gaussians(seed, 0))
    b = O.rhs(n)
    uo, co, ro = O.fe_solve(k, b, tol=1e-8)
    P = M.mg_plan_create(n0=n, max_level=0)
    M.mg_plan_set_option(P, "operator", 1)
    dk = torch.from_numpy(k.ravel().copy()).cuda()
    df = torch.ones_like(dk)
    du = torch.zeros_like(dk)
    st, cyc, rel = M.mg_solve(P, n, dk, df, du)
    assert st == M.MG_OK and cyc == co
    assert abs(rel - ro) <= 1e-6 * ro
    ug = du.cpu().numpy().reshape(n, n, n)
    err = np.linalg.norm((ug - uo).ravel()) / np.linalg.norm(uo.ravel())
    assert err <= 1e-10, err
    # fixed-cycle parity (two cycles: far from converged, every rounding shows)
    uo2, _, _ = O.fe_solve(k, b, fixed_cycles=2)
    du.zero_()
    M.mg_solve(P, n, dk, df, du, 0.0, 2)
    ug2 = du.cpu().numpy().reshape(n, n, n)
    assert np.linalg.norm((ug2 - uo2).ravel()) / np.linalg.norm(uo2.ravel()) <= 1e-10
    # the FE solution differs from the FD one on a random field
    P2 = M.mg_plan_create(n0=n, max_level=0)
    du.zero_()
    M.mg_solve(P2, n, dk, df, du)
    assert np.linalg.norm((du.cpu().numpy().reshape(n, n, n) - ug).ravel()) > 1e-4 * np.linalg.norm(ug)


@pytest.mark.parametrize("qoi", ["integral", "point"])
@pytest.mark.parametrize("n0,level", [(9, 0), (9, 2), (17, 2)])
def test_fe_samples_against_oracle(M, torch, qoi, n0, level):
    print("fe samples n0 %d level %d %s" % (n0, level, qoi), flush=True)
    P = M.mg_plan_create(n0=n0, max_level=level)
    M.mg_plan_set_option(P, "operator", 1)
    M.mg_plan_set_option(P, "qoi", 0 if qoi == "integral" else 1)
    seeds = [21, 22, 23, 24, 25, 26]
    n = len(seeds)
    Y = torch.zeros(n, dtype=torch.float64, device="cuda")
    Qf, Qc = torch.zeros_like(Y), torch.zeros_like(Y)
    cyc = torch.zeros(2 * n, dtype=torch.int32, device="cuda")
    assert M.mlmc_sample_batch(P, level, np.asarray(seeds, dtype=np.uint64), n, Y, Qf, Qc, cyc) == M.MG_OK
    Y, Qf, Qc = Y.cpu().numpy(), Qf.cpu().numpy(), Qc.cpu().numpy()
    cyc = cyc.cpu().numpy().reshape(n, 2)
    with cf.ThreadPoolExecutor(THREADS) as ex:
        refs = list(ex.map(lambda s: O.mlmc_sample_fe(n0, level, s, qoi=qoi), seeds))
    for i, r in enumerate(refs):
        assert abs(Qf[i] - r["Qf"]) <= 1e-9 * abs(r["Qf"])
        assert abs(Qc[i] - r["Qc"]) <= 1e-9 * abs(r["Qc"])
        assert abs(Y[i] - r["Y"]) <= 1e-9 * (abs(r["Qf"]) + abs(r["Qc"]))
        assert tuple(int(c) for c in cyc[i]) == tuple(r["cycles"])
    Y1 = torch.zeros(1, dtype=torch.float64, device="cuda")
    M.mlmc_sample_batch(P, level, np.asarray(seeds[3:4], dtype=np.uint64), 1, Y1)
    assert Y1.item() == Y[3]
    P.destroy()


def test_fe_option_checks(M, torch):
    P = M.mg_plan_create(n0=9, max_level=1)
    M.mg_plan_set_option(P, "operator", 1)
    for name, value in (("solver", 1), ("qoi", 2)):
        with pytest.raises(M.MGError):
            M.mg_plan_set_option(P, name, value)
    with pytest.raises(M.MGError):
        M.Server(P, [2, 2])
    Pm = M.mg_plan_create(n0=9, max_level=1, precision=M.MG_MIXED)
    with pytest.raises(M.MGError):
        M.mg_plan_set_option(Pm, "operator", 1)
    # back to FD: the plan's samples equal a fresh FD plan's
    M.mg_plan_set_option(P, "operator", 0)
    Y = torch.zeros(2, dtype=torch.float64, device="cuda")
    Y2 = torch.zeros_like(Y)
    M.mlmc_sample_batch(P, 1, np.array([1, 2], dtype=np.uint64), 2, Y)
    M.mlmc_sample_batch(M.mg_plan_create(n0=9, max_level=1), 1, np.array([1, 2], dtype=np.uint64), 2, Y2)
    assert torch.equal(Y, Y2)
