"""GPU test of the allocation-free solve (mg_solve_noalloc, for callers that
cannot allocate device memory) against mg_solve, through the C ABI.

Both entry points run the same kernels in the same order, so the bar is
bit-for-bit equality of u, the cycle count and the relative residual.  Two
calls in a row on one plan, the second on a smaller grid (the static
workspace keeps the first call's contents), in FP64 and in mixed precision;
sizes above the workspace's limit are rejected."""
import ctypes as C
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


def _problem(M, torch, P, n, seed):
    k = torch.empty(n**3, dtype=torch.float64, device="cuda")
    M.mlmc_field(P, n, seed, 0, k)
    h = 1.0 / (n - 1)
    x = torch.arange(n, dtype=torch.float64, device="cuda") * h
    # a non-constant right-hand side, so the workspace's b array is exercised
    f = (1.0 + x[:, None, None] * x[None, :, None] - 0.5 * x[None, None, :]).expand(n, n, n)
    return k, f.contiguous().view(-1)


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_solve_equals_mg_solve(M, torch, precision):
    P = M.mg_plan_create(n0=33, max_level=0, precision=precision)
    for n, seed in ((129, 3), (33, 4)):
        print("noalloc: precision %d n %d seed %d" % (precision, n, seed), flush=True)
        k, f = _problem(M, torch, P, n, seed)
        u_ref = torch.zeros(n**3, dtype=torch.float64, device="cuda")
        u_na = torch.full((n**3,), 7.0, dtype=torch.float64, device="cuda")
        u_na.view(n, n, n)[1:-1, 1:-1, 1:-1] = 0.0  # boundary entries are set to 0 by the call
        st0, c0, r0 = M.mg_solve(P, n, k, f, u_ref)
        st1, c1, r1 = M.mg_solve_noalloc(P, n, k, f, u_na)
        torch.cuda.synchronize()
        assert st0 == st1 == M.MG_OK
        assert c0 == c1 and c0 > 0
        assert r0 == r1 and r0 <= 1e-8
        assert torch.equal(u_ref, u_na)
        # a fixed cycle count (parity mode) also agrees
        u_ref.zero_()
        u_na.zero_()
        M.mg_solve(P, n, k, f, u_ref, 0.0, 3)
        M.mg_solve_noalloc(P, n, k, f, u_na, 0.0, 3)
        assert torch.equal(u_ref, u_na)
    P.destroy()


def test_noalloc_rejects_sizes_beyond_the_workspace(M, torch):
    P = M.mg_plan_create(n0=33, max_level=0)
    n = 257
    k = torch.ones(n**3, dtype=torch.float64, device="cuda")
    f = torch.ones_like(k)
    u = torch.zeros_like(k)
    cyc, rel = C.c_int(0), C.c_double(0.0)
    st = M.lib().mg_solve_noalloc(P.handle, n, C.c_void_p(k.data_ptr()), C.c_void_p(f.data_ptr()),
                                  C.c_void_p(u.data_ptr()), 0.0, 0, C.byref(cyc), C.byref(rel))
    assert st == M.MG_EINVAL
    assert "static workspace" in P.error()
    assert torch.count_nonzero(u).item() == 0  # nothing was launched
    P.destroy()
