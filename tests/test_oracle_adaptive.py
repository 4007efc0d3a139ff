"""Pins of the oracle's adaptive MLMC driver (Section 2.3, Algorithm 2).

  * eq. (quasioptimal_Nl) against numbers worked out by hand;
  * sigma^2 = 0: every Y_l is deterministic (s_l^2 = 0), so N_l stays N_Init
    and the level choice follows from the bias test alone, which the k = 1
    closed form of the discrete QoI (type-I discrete sine transform, scipy)
    fixes; the estimate telescopes to Q_h(n_L);
  * a random-coefficient run: the sampling error after the last round is
    below eps_s^2 = theta eps^2 (eq. def:eps), which eq. (quasioptimal_Nl)
    guarantees by construction, the level means are the plain sample means
    of independent oracle samples, and the (L, N) trace never decreases.
"""
import math

import numpy as np
import pytest
import scipy.fft

import oracle as O


def test_quasioptimal_n_hand_values():
    # eps_s^2 = 1e-6, s^2 = (4e-4, 1e-5, 2.5e-7), C = (1, 8, 64):
    # sum sqrt(s^2 C) = 0.02 + sqrt(8e-5) + 0.004 = 0.032944271909999...
    # N_0 = 0.0329443 * 0.02 / 1e-6 = 658.885 -> 659
    # N_1 = 0.0329443 * sqrt(1.25e-6) / 1e-6 = 36.833 -> 37
    # N_2 = 0.0329443 * 6.25e-5 / 1e-6 = 2.059 -> 3
    assert O.quasioptimal_n(1e-6, [4e-4, 1e-5, 2.5e-7], [1.0, 8.0, 64.0]) == [659, 37, 3]
    # a level without variance needs no samples beyond those it has:
    # N_0 = 0.02 * 0.02 / 1.1e-6 = 363.64 -> 364
    assert O.quasioptimal_n(1.1e-6, [4e-4, 0.0], [1.0, 8.0]) == [364, 0]


def _q_const(n):
    """Discrete QoI h^3 sum u of the k = 1, f = 1 problem (DST-I closed form)."""
    m = n - 2
    h = 1.0 / (n - 1)
    p = np.arange(1, m + 1)
    lam = 2.0 - 2.0 * np.cos(np.pi * p / (m + 1))
    L = lam[:, None, None] + lam[None, :, None] + lam[None, None, :]
    b = np.full((m, m, m), h * h)
    u = scipy.fft.idstn(scipy.fft.dstn(b, type=1) / L, type=1)
    return h**3 * float(u.sum())


def test_zero_variance_levels_follow_the_bias_test():
    n0, alpha, theta = 5, 2.0 / 3.0, 0.5
    q = [_q_const(O.grid_n(n0, l)) for l in range(4)]
    y = [q[0]] + [q[l] - q[l - 1] for l in range(1, 4)]
    # choose eps so that the bias test fails at L = 1, 2 and passes at L = 3
    thr = [abs(y[l]) / (8.0**alpha - 1.0) for l in range(4)]
    eps_b = math.sqrt(thr[2] * thr[3])            # between the level-2 and level-3 estimates
    eps = eps_b / math.sqrt(1.0 - theta)
    r = O.adaptive_mlmc(n0, 3, eps, theta, alpha, n_init=4, sigma2=0.0, tol=1e-12)
    assert r["L"] == 3 and r["bias_ok"]
    assert r["N"] == [4, 4, 4, 4]
    assert r["var"] == [0.0, 0.0, 0.0, 0.0]
    assert [t[0] for t in r["trace"]] == [2, 3, 3]
    for l in range(4):
        assert r["mean"][l] == pytest.approx(y[l], rel=1e-9, abs=1e-14)
    assert r["Q"] == pytest.approx(q[3], rel=1e-10)
    assert r["bias_estimate"] == pytest.approx(thr[3], rel=1e-8)
    # a looser eps stops one level earlier
    r2 = O.adaptive_mlmc(n0, 3, math.sqrt(thr[1] * thr[2]) / math.sqrt(1.0 - theta), theta, alpha,
                         n_init=4, sigma2=0.0, tol=1e-12)
    assert r2["L"] == 2 and r2["Q"] == pytest.approx(q[2], rel=1e-10)


def test_random_field_run_meets_sampling_tolerance():
    n0, theta, alpha, eps = 5, 0.5, 2.0 / 3.0, 4e-4
    r = O.adaptive_mlmc(n0, 3, eps, theta, alpha, n_init=8, seed0=100, sigma2=1.0, lam=0.1)
    L = r["L"]
    assert 1 <= L <= 3
    assert r["sampling_rms"] ** 2 <= theta * eps * eps * (1.0 + 1e-12)
    assert r["Q"] == pytest.approx(math.fsum(r["mean"]), rel=1e-15)
    assert max(r["N"]) > 8  # the variances asked for more samples than N_Init
    prev_L, prev_N = 1, [8, 8]
    for Lt, Nt in r["trace"]:
        assert Lt >= prev_L and all(a >= b for a, b in zip(Nt, prev_N))
        prev_L, prev_N = Lt, Nt
    # level means and s^2 (divisor N) are those of independent samples
    for l in range(L + 1):
        ys = [O.mlmc_sample(n0, l, 100 + i)["Y"] for i in range(r["N"][l])]
        m = math.fsum(ys) / len(ys)
        v = math.fsum((y - m) ** 2 for y in ys) / len(ys)
        assert r["mean"][l] == pytest.approx(m, rel=1e-12, abs=1e-18)
        assert r["var"][l] == pytest.approx(v, rel=1e-9, abs=1e-24)


@pytest.mark.parametrize("n", [5, 9, 17, 33])
def test_mode_sum_closed_form_matches_dst_solution(n):
    """The mode-sum closed form of the k = 1 QoI (used at 1025^3 on the GPU,
    where a transform of the whole grid is out of reach) against the DST-I
    solution of the same discrete problem."""
    from closed_forms import q_const_modes
    assert q_const_modes(n) == pytest.approx(_q_const(n), rel=1e-13)
