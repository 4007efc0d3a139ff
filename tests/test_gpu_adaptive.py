"""GPU test of the adaptive MLMC driver (mlmc_adaptive, Section 2.3,
Algorithm 2) against the oracle's driver of the same algorithm.

Both take the same seeds (sample i of every level: seed0 + i), so the
samples agree to the parity bars (Q within 1e-9); the driver's decisions
(L and every N_l after each round) must then be the same, and the level
means, s^2 and the estimate agree within the bars the samples carry."""
import os

import pytest

import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_1607_03252_amd as M
    if not os.path.exists(M.LIB_PATH):
        raise RuntimeError("libmlmcmg.so is not built")
    M.lib()
    return M


@pytest.mark.parametrize("n0,max_level,eps,n_init,seed0,sigma2", [
    (5, 3, 4e-4, 8, 100, 1.0),
    (9, 2, 2e-4, 16, 7, 1.0),
    (5, 3, 2.5e-5, 4, 0, 0.0),
])
def test_adaptive_matches_oracle_driver(M, n0, max_level, eps, n_init, seed0, sigma2):
    theta, alpha = 0.5, 2.0 / 3.0
    print("adaptive: n0 %d L<=%d eps %g" % (n0, max_level, eps), flush=True)
    ref = O.adaptive_mlmc(n0, max_level, eps, theta, alpha, n_init, seed0=seed0, sigma2=sigma2,
                          lam=0.1)
    P = M.mg_plan_create(n0=n0, max_level=max_level, sigma2=sigma2, corr_len=0.1)
    got = M.mlmc_adaptive(P, eps, theta, alpha, n_init=n_init, seed0=seed0, max_batch=64)
    assert got["trace"] == [(L, list(N)) for L, N in ref["trace"]]
    assert got["L"] == ref["L"] and got["N"] == ref["N"] and got["bias_ok"] == ref["bias_ok"]
    assert got["iterations"] == ref["iterations"]
    scale = abs(ref["mean"][0])
    for l in range(ref["L"] + 1):
        assert abs(got["mean"][l] - ref["mean"][l]) <= 1e-9 * scale
        assert abs(got["var"][l] - ref["var"][l]) <= 1e-8 * scale * scale
        assert got["cost"][l] == ref["cost"][l]  # cycle counts equal: same node-cycles
    assert abs(got["Q"] - ref["Q"]) <= 1e-9 * scale
    assert got["sampling_rms"] ** 2 <= theta * eps * eps * (1.0 + 1e-9)
    P.destroy()
