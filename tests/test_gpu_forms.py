"""GPU tests of the execution forms against each other and the oracle.

  * the fused single-pass smoother and the two-pass colour smoother compute
    the same red-black Gauss-Seidel iterates (same arithmetic in the same
    order): results agree bit for bit;
  * every compiled tile shape and plane chunking of the fused smoother gives
    bit-identical results;
  * HIP-graph-captured cycles give the same results as eager launches;
  * mixed precision (FP32 inner V-cycles inside FP64 defect correction)
    reaches the FP64 relative residual 1e-8, checked with the oracle's own
    residual; its solution and QoI errors against the FP64 oracle are bounded
    by what that residual allows (stated in the test);
  * batches mixing grid sizes of several levels (nested cycles) equal
    per-level batches bit for bit.
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


def _batch(M, torch, P, level, seeds, fixed=0):
    n = len(seeds)
    Y = torch.zeros(n, dtype=torch.float64, device="cuda")
    Qf, Qc = torch.zeros_like(Y), torch.zeros_like(Y)
    cyc = torch.zeros(2 * n, dtype=torch.int32, device="cuda")
    st = M.mlmc_sample_batch(P, level, np.asarray(seeds, dtype=np.uint64), n, Y, Qf, Qc, cyc, fixed)
    return st, Y.cpu().numpy(), Qf.cpu().numpy(), Qc.cpu().numpy(), cyc.cpu().numpy()


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def test_fused_and_colour_smoothers_agree(M, torch):
    P = M.mg_plan_create(n0=17, max_level=2)
    seeds = [5, 6, 7, 8]
    M.mg_plan_set_option(P, "graph", 0)
    fused = _batch(M, torch, P, 2, seeds)
    M.mg_plan_set_option(P, "smoother", 1)
    colour = _batch(M, torch, P, 2, seeds)
    assert fused[0] == colour[0] == M.MG_OK
    assert _same(fused, colour)


@pytest.mark.parametrize("n0,level,prec", [(17, 2, 0), (9, 1, 0), (17, 1, 1)])
def test_small_vcycle_matches_per_level_launches(M, torch, n0, level, prec):
    # the LDS V-cycle on grids <= 17 (one launch) against one launch per level
    # and step: the same updates in the same arithmetic, bit for bit
    seeds = [21, 22, 23, 24, 25]
    out = {}
    for ns in (17, 9, 5, 0):
        P = M.mg_plan_create(n0=n0, max_level=level, precision=prec)
        M.mg_plan_set_option(P, "small_vcycle", ns)
        out[ns] = _batch(M, torch, P, level, seeds)
        assert out[ns][0] == M.MG_OK
    for ns in (17, 9, 5):
        assert _same(out[ns], out[0]), ns


@pytest.mark.parametrize("n0,level,prec,nseeds", [(33, 1, 0, 3), (33, 2, 0, 3), (33, 1, 1, 3),
                                                  (33, 0, 0, 1), (17, 3, 0, 1)])
def test_fused_transfer_matches_separate_kernels(M, torch, n0, level, prec, nseeds):
    # residual + full weighting in one pass (r never stored) against the
    # residual kernel followed by the restriction kernel: bit for bit (few
    # grids per launch: the fused transfer splits its plane marches)
    seeds = [31, 32, 33][:nseeds]
    out = {}
    for tr in (0, 1):
        P = M.mg_plan_create(n0=n0, max_level=level, precision=prec)
        M.mg_plan_set_option(P, "transfer", tr)
        out[tr] = _batch(M, torch, P, level, seeds)
        assert out[tr][0] == M.MG_OK
    assert _same(out[0], out[1])


@pytest.mark.parametrize("n0,level,fixed", [(33, 1, 0), (17, 2, 0), (33, 0, 0), (33, 1, 3)])
def test_norm_in_sweeps_matches_separate_reduction(M, torch, n0, level, fixed):
    # the convergence norm summed inside the sweeps (black points in a cycle's
    # last sweep, red points in the next cycle's first, judged one cycle late)
    # against the residual reduction after each cycle: the same per-point
    # residuals, so the same stopping cycle and bit-identical results
    seeds = [41, 42, 43, 44]
    out = {}
    for nm in (0, 1):
        P = M.mg_plan_create(n0=n0, max_level=level)
        M.mg_plan_set_option(P, "norm", nm)
        out[nm] = _batch(M, torch, P, level, seeds, fixed=fixed)
        assert out[nm][0] == M.MG_OK
    assert _same(out[0], out[1])


def test_norm_in_sweeps_single_solve_relres(M, torch):
    # mg_solve: same cycles and iterate; the relative residual differs only by
    # the summation order of the squared residuals
    n = 65
    k = O.field(n, 2.0, 0.05, O.gaussians(12, 0))
    f = np.ones_like(k)
    res = {}
    for nm in (0, 1):
        P = M.mg_plan_create()
        M.mg_plan_set_option(P, "norm", nm)
        res[nm] = _solve(M, torch, P, k, f)
        assert res[nm][0] == M.MG_OK
    assert res[0][1] == res[1][1]
    assert np.array_equal(res[0][3], res[1][3])
    assert abs(res[0][2] - res[1][2]) <= 1e-12 * res[0][2]
    # against the oracle's residual of the same iterate: near tol the residual
    # is a difference of terms ~||b||, each point's rounding ~1e-16 ||b||, so
    # its relative accuracy is ~1e-16 / rho ~ 1e-8 for rho ~ 1e-8
    h = 1.0 / (n - 1)
    b = h * h * f
    ro = O.norm2(O.residual(k, b, res[1][3])) / O.norm2(b)
    assert abs(res[1][2] - ro) <= 1e-6 * ro


def test_small_vcycle_single_solve(M, torch):
    # a whole 17^3 solve in the LDS kernel (mg_solve), against per-level launches
    n = 17
    k = O.field(n, 1.0, 0.1, O.gaussians(9, 0))
    f = np.ones_like(k)
    res = {}
    for ns in (17, 0):
        P = M.mg_plan_create()
        M.mg_plan_set_option(P, "small_vcycle", ns)
        res[ns] = _solve(M, torch, P, k, f)
    assert res[17][:2] == res[0][:2]
    assert np.array_equal(res[17][3], res[0][3])


@pytest.mark.parametrize("n0,level", [(33, 1), (65, 1)])
def test_tile_shapes_and_chunks_bit_identical(M, torch, n0, level):
    P = M.mg_plan_create(n0=n0, max_level=level)
    seeds = [11, 12, 13]
    ref = _batch(M, torch, P, level, seeds, fixed=3)
    nf = (n0 - 1) * 2**level + 1
    shapes = [(16, 64), (8, 64), (4, 64), (16, 32), (8, 32), (4, 32), (16, 16), (8, 16), (4, 16),
              (8, 8)]
    for n in (nf, (nf - 1) // 2 + 1):
        for tj, tk in shapes:
            if (n - 1) % tj or (n - 1) % tk or tk > n - 1:
                continue
            for chunks in (1, 3):
                M.mg_set_tile(P, n, tj, tk, chunks)
                got = _batch(M, torch, P, level, seeds, fixed=3)
                assert _same(got, ref), (n, tj, tk, chunks)


def test_graph_and_eager_bit_identical(M, torch):
    P = M.mg_plan_create(n0=33, max_level=1)
    seeds = list(range(300, 316))
    M.mg_plan_set_option(P, "graph", 1)
    g1 = _batch(M, torch, P, 1, seeds)
    g2 = _batch(M, torch, P, 1, seeds)  # replay of the cached graphs
    M.mg_plan_set_option(P, "graph", 0)
    e = _batch(M, torch, P, 1, seeds)
    assert g1[0] == M.MG_OK
    assert _same(g1, e) and _same(g2, e)


def test_autotune_keeps_results(M, torch):
    P = M.mg_plan_create(n0=33, max_level=1)
    seeds = [1, 2, 3]
    before = _batch(M, torch, P, 1, seeds)
    M.mg_autotune(P, 1, 8, 2)
    tj, tk, ch = M.mg_get_tile(P, 65)
    assert 64 % tj == 0 and 64 % tk == 0 and ch >= 0  # 0: automatic chunking
    after = _batch(M, torch, P, 1, seeds)
    assert _same(before, after)


def _solve(M, torch, P, k, f, tol=1e-8, fixed=0):
    n = k.shape[0]
    dk = torch.from_numpy(k.ravel().copy()).cuda()
    df = torch.from_numpy(f.ravel().copy()).cuda()
    du = torch.zeros(n**3, dtype=torch.float64, device="cuda")
    st, cyc, rel = M.mg_solve(P, n, dk, df, du, tol, fixed)
    return st, cyc, rel, du.cpu().numpy().reshape(n, n, n)


@pytest.mark.parametrize("n,sigma2,lam", [(33, 1.0, 0.1), (65, 2.0, 0.05), (129, 2.0, 0.05)])
def test_mixed_precision_reaches_fp64_residual(M, torch, n, sigma2, lam):
    k = O.field(n, sigma2, lam, O.gaussians(4, 0))
    f = np.ones_like(k)
    h = 1.0 / (n - 1)
    b = h * h * f
    Pm = M.mg_plan_create(precision=M.MG_MIXED)
    st, cyc, rel, u = _solve(M, torch, Pm, k, f)
    assert st == M.MG_OK
    # the oracle's own FP64 residual of the mixed-precision solution
    rho = O.norm2(O.residual(k, b, u)) / O.norm2(b)
    assert rho <= 1e-8, rho
    assert abs(rho - rel) <= 1e-3 * rho
    uo, co, _, _ = O.solve(k, b, tol=1e-8)
    du = np.linalg.norm((u - uo).ravel()) / np.linalg.norm(uo.ravel())
    dq = abs(O.qoi(u) - O.qoi(uo)) / abs(O.qoi(uo))
    # the FP32 inner cycles' rounding is contracted by the later outer steps:
    # the mixed solution agrees with the FP64 oracle's at the same stopping
    # cycle to the FP64 parity bars (measured: about 1e-14 in u and Q)
    assert abs(cyc - co) <= 1
    assert du <= 1e-10 and dq <= 1e-9, (du, dq)
    print("mixed n=%d cycles=%d (fp64 %d) rel=%.2e du=%.2e dq=%.2e" % (n, cyc, co, rel, du, dq))


def test_mixed_precision_batch(M, torch):
    P = M.mg_plan_create(n0=33, max_level=1, precision=M.MG_MIXED)
    seeds = list(range(20))
    st, Y, Qf, Qc, cyc = _batch(M, torch, P, 1, seeds)
    assert st == M.MG_OK and np.all(cyc > 0)
    for i in (0, 7, 19):
        r = O.mlmc_sample(33, 1, seeds[i])
        assert abs(Qf[i] - r["Qf"]) <= 1e-9 * abs(r["Qf"])
        assert abs(Qc[i] - r["Qc"]) <= 1e-9 * abs(r["Qc"])


def test_mixed_level_batch_equals_per_level_batches(M, torch):
    # four levels of n0 = 17 (17^3, 33^3, 65^3, 129^3 finest grids) in one batch
    P = M.mg_plan_create(n0=17, max_level=3)
    counts = {0: 6, 1: 4, 2: 3, 3: 2}
    levels, seeds = [], []
    for l, c in counts.items():
        levels += [l] * c
        seeds += [1000 * l + i for i in range(c)]
    order = np.random.default_rng(0).permutation(len(levels))  # interleave the levels
    levels = [levels[i] for i in order]
    seeds = [seeds[i] for i in order]
    n = len(levels)
    Y = torch.zeros(n, dtype=torch.float64, device="cuda")
    Qf, Qc = torch.zeros_like(Y), torch.zeros_like(Y)
    cyc = torch.zeros(2 * n, dtype=torch.int32, device="cuda")
    assert M.mlmc_sample_mixed(P, levels, np.asarray(seeds, dtype=np.uint64), n, Y, Qf, Qc, cyc) == M.MG_OK
    Y, Qf, Qc, cyc = Y.cpu().numpy(), Qf.cpu().numpy(), Qc.cpu().numpy(), cyc.cpu().numpy().reshape(n, 2)
    P2 = M.mg_plan_create(n0=17, max_level=3)
    for l in counts:
        idx = [i for i in range(n) if levels[i] == l]
        st, y, qf, qc, cy = _batch(M, torch, P2, l, [seeds[i] for i in idx])
        assert st == M.MG_OK
        assert np.array_equal(Y[idx], y) and np.array_equal(Qf[idx], qf) and np.array_equal(Qc[idx], qc)
        assert np.array_equal(cyc[idx].ravel(), cy)
    # and against the oracle for one sample of each level
    for l in counts:
        i = [k for k in range(n) if levels[k] == l][0]
        r = O.mlmc_sample(17, l, seeds[i])
        assert abs(Qf[i] - r["Qf"]) <= 1e-9 * abs(r["Qf"])
        assert abs(Y[i] - r["Y"]) <= 1e-9 * (abs(r["Qf"]) + abs(r["Qc"]))
        assert tuple(cyc[i]) == tuple(r["cycles"])
