"""Pins of the oracle's SPDE field sampler (Section 3.2, eq. spde):
(kappa^2 - Laplace) Z = W on the box (-1,2)^3 with natural Neumann boundary
conditions, lumped-mass P1 elements on the Kuhn tetrahedra of the box grid.

  * the assembled stiffness is symmetric with zero row sums (constants lie in
    the Neumann kernel of -Laplace), the lumped masses add up to the box
    volume and equal one cell volume at interior vertices;
  * restriction and prolongation on box grids are adjoint,
    <R b, v_c> = (1/2) <b, P v_c> (R = P^T / 2 is the scaled load transfer);
  * Whittle: the discrete solution's covariance E[Z_x Z_y] =
    sum_p G_xp G_yp f_p^2 (G the inverse of the scaled operator, from two
    deterministic solves; f_p the sampler's load per unit normal, from its
    load function on unit normals) approaches the exponential covariance
    exp(-kappa r) / (8 pi kappa) at the centre of D as h decreases;
  * the white noise is standard normal in Box-Muller pairs;
  * the field on D is exp(sigma sqrt(8 pi kappa) Z) at D's vertices (the
    middle third of the box grid).
"""
import math

import numpy as np
import pytest
import scipy.stats

import oracle as O


def test_box_operator_structure():
    nt = 7
    S, m = O.spde_operator(nt)
    assert np.all(np.abs(S.sum(axis=(3, 4, 5))) <= 1e-14)
    assert m.sum() == pytest.approx((nt - 1) ** 3, rel=1e-14)
    assert np.allclose(m[1:-1, 1:-1, 1:-1], 1.0, rtol=1e-14, atol=0)
    # symmetric: the coupling of p to p + d equals that of p + d to p
    for p in [(0, 0, 0), (3, 2, 6), (6, 6, 6), (1, 5, 0)]:
        for t in np.ndindex(3, 3, 3):
            q = tuple(a + b - 1 for a, b in zip(p, t))
            if all(0 <= x < nt for x in q):
                assert S[p][t] == pytest.approx(S[q][tuple(2 - x for x in t)], rel=1e-14, abs=1e-15)
    assert np.all(S[..., 1, 1, 1] > 0)


def test_restriction_is_half_the_transposed_prolongation():
    rng = np.random.Generator(np.random.PCG64(4))
    nt = 13
    b = rng.normal(size=(nt, nt, nt))
    vc = rng.normal(size=((nt - 1) // 2 + 1,) * 3)
    lhs = float(np.sum(O.spde_restrict(b) * vc))
    rhs = 0.5 * float(np.sum(b * O.spde_prolong_add(vc, np.zeros_like(b))))
    assert lhs == pytest.approx(rhs, rel=1e-13)


def _whittle(n, kappa, d_units):
    nt = O.box_n(n)
    h = 1.0 / (n - 1)
    # the sampler's load is b_p = f_p xi_p; f from unit normals: E[b b^T] = diag(f^2)
    f2 = O.spde_rhs(n, np.ones(nt**3)) ** 2
    c = (nt - 1) // 2
    e = np.zeros((nt, nt, nt))
    e[c, c, c] = 1.0
    g, _, _ = O.spde_solve(e, h, kappa, tol=1e-12)
    d = int(round(d_units / h))
    e2 = np.zeros((nt, nt, nt))
    e2[c + d, c, c] = 1.0
    g2, _, _ = O.spde_solve(e2, h, kappa, tol=1e-12)
    var = float(np.sum(g * g * f2)) * 8 * math.pi * kappa
    cov = float(np.sum(g * g2 * f2)) * 8 * math.pi * kappa / math.exp(-kappa * d_units)
    return var, cov


def test_whittle_covariance_is_approached():
    kappa = 4.0
    v9, c9 = _whittle(9, kappa, 0.25)
    v17, c17 = _whittle(17, kappa, 0.25)
    # ratios to the exponential covariance: variance within 6 %, covariance at
    # r = 1/4 within 2 % at h = 1/16, both closer than at h = 1/8
    assert abs(v17 - 1.0) < 0.06 and abs(v17 - 1.0) < abs(v9 - 1.0)
    assert abs(c17 - 1.0) < 0.02 and abs(c17 - 1.0) < abs(c9 - 1.0)


def test_white_noise_normals():
    xi = O.white_noise(7, 2, 200001)
    assert abs(xi.mean()) < 5 / math.sqrt(xi.size)
    assert abs(xi.var() - 1.0) < 5 * math.sqrt(2.0 / xi.size)
    assert scipy.stats.kstest(xi, "norm").pvalue > 1e-4
    # a stream of its own: not the KL normals of the same (seed, level)
    assert not np.allclose(xi[:64], O.gaussians(7, 2))
    # the first pair from the Philox block with counter (0, level, 1, 0)
    w = O.philox4x32_10([0, 2, 1, 0], [7, 0])
    U = [((int(w[0]) >> 5) * 2**26 + (int(w[1]) >> 6) + 1) * 2.0**-53,
         ((int(w[2]) >> 5) * 2**26 + (int(w[3]) >> 6) + 1) * 2.0**-53]
    R = math.sqrt(-2.0 * math.log(U[0]))
    assert xi[0] ** 2 + xi[1] ** 2 == pytest.approx(R * R, rel=1e-13)
    assert math.atan2(xi[1], xi[0]) % (2 * math.pi) == pytest.approx((2 * math.pi * U[1]) % (2 * math.pi), abs=1e-12)


def test_field_scaling_and_sample():
    n = 5
    nt = O.box_n(n)
    z = np.random.Generator(np.random.PCG64(2)).normal(size=(nt, nt, nt))
    k = O.spde_to_k(n, 2.0, 0.1, z)
    kappa = 10.0
    s = math.sqrt(2.0) * math.sqrt(8 * math.pi * kappa)
    assert np.allclose(np.log(k), s * z[n - 1:2 * n - 1, n - 1:2 * n - 1, n - 1:2 * n - 1], rtol=1e-13)
    r = O.mlmc_sample_spde(5, 1, 3, sigma2=1.0, lam=0.25)
    assert r["spde_cycles"][0] > 0 and r["spde_cycles"][1] > 0
    assert abs(r["Y"]) < 0.2 * abs(r["Qf"])
