"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Bars (arXiv 1607.03252 gives no precision; these are the stated tolerances):
  * Philox words: bit-exact (integer work);
  * normals: within 1e-14 max(1, |xi|) (log/sin/cos differ by ulps between libm
    and the device math library);
  * coefficient k: relative 1e-13;
  * solution u after the same cycle count: relative L2 <= 1e-10;
  * QoI Q and Y: |dQ| <= 1e-9 |Q|, |dY| <= 1e-9 (|Qf| + |Qc|);
  * cycle counts equal (tol-driven runs).
Batched and single-sample results must agree bit for bit (the per-sample
reductions use a fixed tree that does not depend on the batch).
"""
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
        from paper_1607_03252_amd import build
        build.build()
    M.lib()
    return M


def plan(M, **kw):
    return M.mg_plan_create(**kw)


def oracle_samples(n0, level, seeds, **kw):
    with cf.ThreadPoolExecutor(THREADS) as ex:
        return list(ex.map(lambda s: O.mlmc_sample(n0, level, int(s), **kw), seeds))


def rel_l2(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


@pytest.mark.parametrize("level", [0, 1, 3, 2**31 - 1])
def test_philox_words_bitexact(M, torch, level):
    P = plan(M)
    seeds = np.array([0, 1, 2, 63, 2**32 + 9, 2**64 - 1], dtype=np.uint64)
    w = torch.zeros(128 * seeds.size, dtype=torch.int32, device="cuda")
    nrm = torch.zeros(64 * seeds.size, dtype=torch.float64, device="cuda")
    M.mlmc_philox(P, seeds, seeds.size, level, w, nrm)
    got = w.cpu().numpy().view(np.uint32).reshape(seeds.size, 128)
    xi = nrm.cpu().numpy().reshape(seeds.size, 64)
    for i, s in enumerate(seeds):
        assert np.array_equal(got[i], O.philox_words(int(s), level))
        ref = O.gaussians(int(s), level)
        assert np.all(np.abs(xi[i] - ref) <= 1e-14 * np.maximum(1.0, np.abs(ref)))


@pytest.mark.parametrize("n,sigma2,lam", [(3, 1.0, 0.1), (17, 1.0, 0.1), (33, 2.0, 0.05),
                                          (65, 1.0, 0.1)])
def test_field_matches_oracle(M, torch, n, sigma2, lam):
    P = plan(M, sigma2=sigma2, corr_len=lam)
    for seed, level in [(0, 0), (7, 1), (123, 2)]:
        k = torch.zeros(n**3, dtype=torch.float64, device="cuda")
        M.mlmc_field(P, n, seed, level, k)
        ref = O.field(n, sigma2, lam, O.gaussians(seed, level))
        got = k.cpu().numpy().reshape(n, n, n)
        assert np.max(np.abs(got - ref) / ref) <= 1e-13


def _solve_gpu(M, torch, P, k, f, u0, tol=1e-8, fixed=0):
    n = k.shape[0]
    dk = torch.from_numpy(k.ravel().copy()).cuda()
    df = torch.from_numpy(f.ravel().copy()).cuda()
    du = torch.from_numpy(u0.ravel().copy()).cuda()
    st, cyc, rel = M.mg_solve(P, n, dk, df, du, tol, fixed)
    return st, cyc, rel, du.cpu().numpy().reshape(n, n, n)


@pytest.mark.parametrize("n,sigma2,lam,seed", [(9, 1.0, 0.1, 0), (17, 1.0, 0.1, 1),
                                               (33, 1.0, 0.1, 0), (65, 2.0, 0.05, 3)])
def test_mg_solve_matches_oracle(M, torch, n, sigma2, lam, seed):
    k = O.field(n, sigma2, lam, O.gaussians(seed, 0))
    f = np.ones((n, n, n))
    h = 1.0 / (n - 1)
    uo, co, ro, _ = O.solve(k, h * h * f, tol=1e-8, max_cycles=50)
    P = plan(M)
    st, cyc, rel, u = _solve_gpu(M, torch, P, k, f, np.zeros_like(k), tol=1e-8)
    assert st == M.MG_OK and cyc == co
    assert rel <= 1e-8 and abs(rel - ro) <= 1e-6 * ro
    assert rel_l2(u, uo) <= 1e-10
    # fixed-cycle (parity) mode gives the same iterate
    st, cyc2, _, u2 = _solve_gpu(M, torch, P, k, f, np.zeros_like(k), tol=-1, fixed=co)
    assert cyc2 == co and np.array_equal(u2, u)


def test_mg_solve_general_rhs_and_initial_guess(M, torch):
    n = 33
    rng = np.random.default_rng(5)
    k = O.field(n, 1.0, 0.1, O.gaussians(11, 0))
    f = rng.uniform(-1.0, 2.0, (n, n, n))
    u0 = rng.standard_normal((n, n, n))  # boundary values must be replaced by 0
    h = 1.0 / (n - 1)
    bo = h * h * f
    bo[0, :, :] = bo[-1] = 0.0
    uo, co, ro, _ = O.solve(k, bo, u0=u0, fixed_cycles=3, max_cycles=3)
    P = plan(M)
    st, cyc, rel, u = _solve_gpu(M, torch, P, k, f, u0, tol=-1, fixed=3)
    assert cyc == 3
    assert rel_l2(u, uo) <= 1e-10
    assert np.all(u[0] == 0) and np.all(u[:, :, -1] == 0)


def test_mg_solve_nonconvergence_reported(M, torch):
    n = 17
    k = O.field(n, 1.0, 0.1, O.gaussians(0, 0))
    P = plan(M, max_cycles=2)
    st, cyc, rel, _ = _solve_gpu(M, torch, P, k, np.ones_like(k), np.zeros_like(k), tol=1e-12)
    assert st == M.MG_ENOCONV and rel > 1e-12


def _batch(M, torch, P, level, seeds, fixed=0):
    n = len(seeds)
    Y = torch.zeros(n, dtype=torch.float64, device="cuda")
    Qf = torch.zeros_like(Y)
    Qc = torch.zeros_like(Y)
    cyc = torch.zeros(2 * n, dtype=torch.int32, device="cuda")
    st = M.mlmc_sample_batch(P, level, np.asarray(seeds, dtype=np.uint64), n, Y, Qf, Qc, cyc,
                             fixed)
    return st, Y.cpu().numpy(), Qf.cpu().numpy(), Qc.cpu().numpy(), cyc.cpu().numpy().reshape(n, 2)


def _check_samples(got, ref):
    st, Y, Qf, Qc, cyc = got
    for i, r in enumerate(ref):
        assert abs(Qf[i] - r["Qf"]) <= 1e-9 * abs(r["Qf"])
        assert abs(Qc[i] - r["Qc"]) <= 1e-9 * max(abs(r["Qc"]), 1e-300)
        assert abs(Y[i] - r["Y"]) <= 1e-9 * (abs(r["Qf"]) + abs(r["Qc"]))
        assert tuple(cyc[i]) == tuple(r["cycles"])


def test_single_sample_33(M, torch):
    # 33^3 grid, sigma^2 = 1, lambda = 0.1, seed 0, level 0, V(2,2) to 1e-8
    P = plan(M, n0=33, max_level=0)
    got = _batch(M, torch, P, 0, [0])
    assert got[0] == M.MG_OK
    _check_samples(got, oracle_samples(33, 0, [0]))
    assert got[4][0, 1] == 0 and got[3][0] == 0.0


def test_level_pair_65_33_64_samples(M, torch):
    # 64 coupled samples, fine 65^3 and coarse 33^3 on one omega, seeds 0..63
    P = plan(M, n0=33, max_level=1)
    seeds = list(range(64))
    got = _batch(M, torch, P, 1, seeds)
    assert got[0] == M.MG_OK
    _check_samples(got, oracle_samples(33, 1, seeds))


def test_sample_alone_equals_sample_in_batch(M, torch):
    P = plan(M, n0=33, max_level=1)
    seeds = list(range(100, 164))
    full = _batch(M, torch, P, 1, seeds)
    for i in (0, 17, 63):
        alone = _batch(M, torch, P, 1, [seeds[i]])
        for a, b in zip(alone[1:], full[1:]):
            assert np.array_equal(a[0], b[i])


def test_repeated_batch_on_one_plan_is_identical(M, torch):
    # a reused workspace must not leak the previous solution into the next
    # batch's initial guess
    P = plan(M, n0=17, max_level=1)
    a = _batch(M, torch, P, 1, [21, 22, 23])
    _batch(M, torch, P, 1, [40, 41, 42])
    b = _batch(M, torch, P, 1, [21, 22, 23])
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("n0,level,count", [(3, 0, 1), (3, 1, 2), (5, 2, 3), (9, 1, 5),
                                            (17, 0, 7)])
def test_small_and_ragged_batches(M, torch, n0, level, count):
    P = plan(M, n0=n0, max_level=level)
    seeds = [1000 + 13 * i for i in range(count)]
    got = _batch(M, torch, P, level, seeds)
    assert got[0] == M.MG_OK
    _check_samples(got, oracle_samples(n0, level, seeds))


def test_fixed_cycle_mode_and_noconv(M, torch):
    P = plan(M, n0=17, max_level=1)
    seeds = [3, 4, 5]
    got = _batch(M, torch, P, 1, seeds, fixed=4)
    assert got[0] == M.MG_OK and np.all(got[4] == 4)
    ref = oracle_samples(17, 1, seeds, fixed_cycles=4)
    _check_samples(got, ref)
    P2 = plan(M, n0=17, max_level=1, max_cycles=2)
    got = _batch(M, torch, P2, 1, seeds)
    assert got[0] == M.MG_ENOCONV and np.all(got[4] == -1)


def test_constant_coefficient_closed_form(M, torch):
    P = plan(M, n0=33, max_level=1, sigma2=0.0, tol=1e-12)
    st, Y, Qf, Qc, cyc = _batch(M, torch, P, 1, [1, 2])
    assert st == M.MG_OK
    assert abs(Y[0] - 8.7966342e-5) < 1e-12 and Y[0] == Y[1]


def test_empty_and_invalid_inputs_are_rejected(M, torch):
    """Empty batches, levels outside the plan, grid sizes that are not
    2^m + 1 (or beyond 1025) and negative cycle counts are refused with
    MG_EINVAL before any device work; a valid call on the same plan then
    still gives the results of a fresh plan."""
    import ctypes as C
    P = M.mg_plan_create(n0=9, max_level=2)
    L = M.lib()
    Y = torch.zeros(4, dtype=torch.float64, device="cuda")
    seeds = np.arange(4, dtype=np.uint64)
    sp = seeds.ctypes.data_as(C.POINTER(C.c_uint64))
    yp = C.c_void_p(Y.data_ptr())
    assert L.mlmc_sample_batch(P.handle, 0, sp, 0, yp, None, None, None, 0) == M.MG_EINVAL
    assert L.mlmc_sample_batch(P.handle, 3, sp, 4, yp, None, None, None, 0) == M.MG_EINVAL
    assert L.mlmc_sample_batch(P.handle, -1, sp, 4, yp, None, None, None, 0) == M.MG_EINVAL
    assert L.mlmc_sample_batch(P.handle, 1, None, 4, yp, None, None, None, 0) == M.MG_EINVAL
    assert L.mlmc_sample_batch(P.handle, 1, sp, 4, None, None, None, None, 0) == M.MG_EINVAL
    assert L.mlmc_sample_batch(P.handle, 1, sp, 4, yp, None, None, None, -1) == M.MG_EINVAL
    lv = np.array([0, 1, 3, 2], dtype=np.int32)
    lp = lv.ctypes.data_as(C.POINTER(C.c_int))
    assert L.mlmc_sample_mixed(P.handle, lp, sp, 4, yp, None, None, None, 0) == M.MG_EINVAL
    assert L.mlmc_sample_mixed(P.handle, lp, sp, 0, yp, None, None, None, 0) == M.MG_EINVAL
    assert P.error()  # the reason is recorded
    for n in (2, 8, 10, 2049):
        k = torch.ones(max(1, n) ** 3 if n < 100 else 8, dtype=torch.float64, device="cuda")
        assert L.mg_solve(P.handle, n, C.c_void_p(k.data_ptr()), C.c_void_p(k.data_ptr()),
                          C.c_void_p(k.data_ptr()), 0.0, 0, None, None) == M.MG_EINVAL
    k = torch.ones(9 ** 3, dtype=torch.float64, device="cuda")
    assert L.mg_solve(P.handle, 9, None, C.c_void_p(k.data_ptr()), C.c_void_p(k.data_ptr()),
                      0.0, 0, None, None) == M.MG_EINVAL
    # the plan still works and gives the results of a fresh plan
    Qf = torch.zeros_like(Y)
    assert M.mlmc_sample_batch(P, 2, seeds, 4, Y, Qf) == M.MG_OK
    Y2, Qf2 = torch.zeros_like(Y), torch.zeros_like(Y)
    assert M.mlmc_sample_batch(M.mg_plan_create(n0=9, max_level=2), 2, seeds, 4, Y2, Qf2) == M.MG_OK
    assert torch.equal(Y, Y2) and torch.equal(Qf, Qf2)
