"""Pins of the oracle's full multigrid and the paper's two other QoIs.

QoIs of Section 3: the point value u(x*) at x* = (1/4, 1/4, 1/4) (the point
of Section 7.1) and the flux of -k grad u across the plane x_2 = 1/4 (the
plane of Section 7.2; reading: the +x_2 direction, |Gamma| = 1).
  * k = 1, f = 1: the discrete solution in closed form (type-I discrete sine
    transform, scipy) fixes both discrete QoIs;
  * the manufactured solution u* = sin(pi x) sin(pi y) sin(pi z) with
    k = exp(x + 2y - z)/2: both QoIs converge at O(h^2) to their exact
    values, u*(x*) = (sqrt(2)/2)^3 and the flux
    -(pi cos(pi/4)/2) e^(1/2) I(1) I(-1), I(a) = pi (1 + e^a) / (a^2 + pi^2).
Full multigrid (nested iteration, Section 7.1's FMG-2V(4,4)): one pass
reaches the discretisation error (the textbook property of FMG): its error
against u* is that of the fully converged discrete solution up to a few
per cent, and its distance to that solution is a small fraction of it.
"""
import math

import numpy as np
import pytest
import scipy.fft

import oracle as O


def dst_solution(n):
    m = n - 2
    h = 1.0 / (n - 1)
    p = np.arange(1, m + 1)
    lam = 2.0 - 2.0 * np.cos(np.pi * p / (m + 1))
    L = lam[:, None, None] + lam[None, :, None] + lam[None, None, :]
    u = np.zeros((n, n, n))
    u[1:-1, 1:-1, 1:-1] = scipy.fft.idstn(scipy.fft.dstn(np.full((m, m, m), h * h), type=1) / L,
                                          type=1)
    return u


def manufactured(n):
    x = np.arange(n) / (n - 1)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    pi = math.pi
    k = np.exp(X + 2 * Y - Z) / 2.0
    us = np.sin(pi * X) * np.sin(pi * Y) * np.sin(pi * Z)
    gk_gu = k * pi * (np.cos(pi * X) * np.sin(pi * Y) * np.sin(pi * Z)
                      + 2 * np.sin(pi * X) * np.cos(pi * Y) * np.sin(pi * Z)
                      - np.sin(pi * X) * np.sin(pi * Y) * np.cos(pi * Z))
    return k, -gk_gu + 3 * pi**2 * k * us, us


def exact_flux():
    pi = math.pi
    I = lambda a: pi * (1.0 + math.exp(a)) / (a * a + pi * pi)
    return -(pi * math.cos(pi / 4) / 2.0) * math.exp(0.5) * I(1.0) * I(-1.0)


@pytest.mark.parametrize("n", [5, 9, 17, 33])
def test_point_and_flux_of_constant_k_closed_form(n):
    ud = dst_solution(n)
    c = (n - 1) // 4
    k = np.ones((n, n, n))
    u, _, _, _ = O.solve(k, O.rhs(n), tol=1e-13, max_cycles=60)
    assert O.point_qoi(u) == pytest.approx(ud[c, c, c], rel=1e-11)
    # flux of -grad u in +x_2: mean of the face planes on either side of j = c,
    # each h * sum over (i, k) of (u(j) - u(j+1)) with unit face coefficients
    h = 1.0 / (n - 1)
    Fm = h * np.sum(ud[1:-1, c - 1, 1:-1] - ud[1:-1, c, 1:-1])
    Fp = h * np.sum(ud[1:-1, c, 1:-1] - ud[1:-1, c + 1, 1:-1])
    assert O.flux_qoi(k, u) == pytest.approx(0.5 * (Fm + Fp), rel=1e-10)
    # u > 0 grows away from x_2 = 0, so the flux of -grad u in +x_2 is negative
    assert O.flux_qoi(k, u) < 0.0


def test_qois_converge_to_manufactured_values():
    pe, fe = (math.sqrt(2.0) / 2.0) ** 3, exact_flux()
    ep, ef = [], []
    for n in (17, 33, 65):
        k, f, us = manufactured(n)
        h = 1.0 / (n - 1)
        u, _, _, _ = O.solve(k, h * h * f, tol=1e-12, max_cycles=60)
        ep.append(abs(O.point_qoi(u) - pe))
        ef.append(abs(O.flux_qoi(k, u) - fe))
    for e in (ep, ef):
        r = [e[i] / e[i + 1] for i in range(2)]
        assert all(3.5 < x < 4.5 for x in r), (e, r)
    assert ef[-1] < 1e-3 * abs(fe)


@pytest.mark.parametrize("n", [17, 33, 65])
def test_fmg_reaches_discretisation_accuracy(n):
    k, f, us = manufactured(n)
    h = 1.0 / (n - 1)
    uh, _, _, _ = O.solve(k, h * h * f, tol=1e-13, max_cycles=60)
    uf = O.fmg(k, f, nu1=4, nu2=4, ncycles=2)
    e_h = np.max(np.abs(uh - us))
    e_fmg = np.max(np.abs(uf - us))
    d = np.max(np.abs(uf - uh))
    assert e_fmg <= 1.05 * e_h and d <= 0.05 * e_h, (e_h, e_fmg, d)
    # the boundary stays at the Dirichlet value
    assert np.all(uf[0] == 0.0) and np.all(uf[:, :, -1] == 0.0)


def test_fmg_one_cycle_per_grid_is_coarser_but_converges():
    # FMG-1V(1,1) on k = 1: each stage's error is bounded by a fixed factor of
    # the discretisation error, smaller with more cycles per stage
    n = 33
    k = np.ones((n, n, n))
    ud = dst_solution(n)
    f = np.ones((n, n, n))
    e1 = np.max(np.abs(O.fmg(k, f, 1, 1, 1) - ud))
    e2 = np.max(np.abs(O.fmg(k, f, 4, 4, 2) - ud))
    assert e2 < 0.1 * e1 and e1 < 0.1 * np.max(np.abs(ud))


def test_sample_ex_matches_the_plain_sample():
    # solver 'vcycle' with the integral QoI is the plain sample
    a = O.mlmc_sample(9, 1, 5)
    b = O.mlmc_sample_ex(9, 1, 5)
    assert (a["Y"], a["Qf"], a["Qc"], a["cycles"]) == (b["Y"], b["Qf"], b["Qc"], b["cycles"])
    r = O.mlmc_sample_ex(9, 1, 5, solver="fmg", qoi="point", nu1=4, nu2=4)
    assert r["cycles"] == (2, 2)
    assert abs(r["Y"]) < 0.1 * abs(r["Qf"])
