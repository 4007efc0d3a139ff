"""Pins of the oracle's MLMC sample and statistics (Section 2.2, eq. MLMC_defn,
Algorithm 1; the estimator s_l^2 with divisor N of Section 2.3)."""
import math
import statistics

import numpy as np
import pytest

import oracle as O
from test_oracle_operator_mg import dst_solve


def test_compensated_sum_matches_fsum():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.standard_normal(10000) * 1e8, rng.standard_normal(10000),
                        [1e16, 1.0, -1e16]])
    rng.shuffle(x)
    assert O.csum(x) == math.fsum(x)
    u = np.zeros((9, 9, 9))
    u[1:-1, 1:-1, 1:-1] = rng.standard_normal((7, 7, 7))
    assert O.qoi(u) == pytest.approx(math.fsum(u.ravel()) / 8**3, rel=1e-15)


def test_level_accumulator_matches_fsum_statistics():
    rng = np.random.default_rng(4)
    y = 1e-3 + 1e-7 * rng.standard_normal(5000)  # small spread on a large offset
    acc = O.LevelAcc()
    for v in y:
        acc.add(float(v))
    mean, var = acc.result()
    m_ref = math.fsum(y) / len(y)
    v_ref = math.fsum((yy - m_ref) ** 2 for yy in y) / len(y)
    assert abs(mean - m_ref) <= 1e-15 * abs(m_ref)
    assert abs(var - v_ref) <= 1e-9 * v_ref
    assert var == pytest.approx(statistics.pvariance(y), rel=1e-9)


def test_constant_coefficient_sample_is_closed_form():
    # sigma^2 = 0 gives k = 1 for every omega: Y_1 = Q_h(65) - Q_h(33) exactly
    s = O.mlmc_sample(33, 1, 7, sigma2=0.0, tol=1e-12)
    q = []
    for n in (65, 33):
        ex = dst_solve(O.rhs(n)[1:-1, 1:-1, 1:-1])
        q.append((1.0 / (n - 1)) ** 3 * math.fsum(ex.ravel()))
    assert s["Qf"] == pytest.approx(q[0], rel=1e-10)
    assert s["Qc"] == pytest.approx(q[1], rel=1e-10)
    assert s["Y"] == pytest.approx(q[0] - q[1], rel=1e-6, abs=1e-15)
    assert abs(s["Y"] - 8.7966342e-5) < 1e-12


def test_sample_couples_fine_and_coarse_on_one_omega():
    n0, level, seed = 9, 1, 12
    s = O.mlmc_sample(n0, level, seed, sigma2=1.0, lam=0.1, tol=1e-10)
    kf, kc = O.sample_fields(n0, level, seed, 1.0, 0.1)
    assert np.array_equal(kc, kf[::2, ::2, ::2])
    uf, cf, _, _ = O.solve(kf, O.rhs(17), tol=1e-10)
    uc, cc, _, _ = O.solve(kc, O.rhs(9), tol=1e-10)
    assert s["Qf"] == O.qoi(uf) and s["Qc"] == O.qoi(uc)
    assert s["Y"] == O.qoi(uf) - O.qoi(uc)
    assert s["cycles"] == (cf, cc)
    s0 = O.mlmc_sample(n0, 0, seed, tol=1e-10)
    assert s0["Qc"] == 0.0 and s0["Y"] == s0["Qf"] and s0["cycles"][1] == 0


@pytest.mark.slow
def test_level_differences_decay():
    # V[Y_l] -> 0 as the grids refine (Section 2.2): with the smooth truncated
    # field and an O(h^2) scheme the level variances fall by about 16 per level
    n0, S = 5, 40
    var, mean = [], []
    for level in (1, 2, 3):
        acc = O.LevelAcc()
        for seed in range(S):
            acc.add(O.mlmc_sample(n0, level, 1000 * level + seed, tol=1e-10)["Y"])
        m, v = acc.result()
        mean.append(abs(m))
        var.append(v)
    assert var[0] > 4 * var[1] > 16 * var[2]
    assert mean[0] > 2 * mean[1] > 4 * mean[2]
