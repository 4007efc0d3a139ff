"""Pins of the oracle's P1 finite-element operator (Section 3.1: element-wise
assembly with the tetrahedron's coefficient the mean of its four vertex
values; Kuhn tetrahedra of the vertex grid, scaled by 1/h).

The oracle assembles every tetrahedron's element matrix from barycentric
gradients (inverse edge matrix), with no knowledge of the resulting pattern.
Pinned against what follows from the mathematics:
  * each Kuhn tetrahedron's gradients are orthogonal across its diagonal
    edges, so the operator couples axis neighbours only: the 20 other
    couplings of the 27-point row are exactly zero (red-black Gauss-Seidel
    is then an exact colouring), and the matrix is symmetric;
  * element matrices have zero row sums, so every assembled interior row
    sums to zero;
  * an axis edge lies in six Kuhn tetrahedra, and its coupling is minus one
    sixth of the sum of their four-vertex means, i.e.
    [6(k_p + k_q) + 2(k of the six off-axis vertices of those tetrahedra)]/24,
    checked for all three axes on a random coefficient;
  * k = 1 gives the 7-point Laplacian, so the solution is the DST-I closed form;
  * the manufactured solution converges at O(h^2) at the vertices.
"""
import math

import numpy as np
import pytest
import scipy.fft

import oracle as O


def random_k(n, seed=3):
    return np.exp(np.random.Generator(np.random.PCG64(seed)).normal(0.0, 1.0, size=(n, n, n)))


def test_pattern_symmetry_and_row_sums():
    n = 6  # odd interior extent on purpose: any n works for the assembly
    k = random_k(n)
    S = O.fe_stencil(k)
    axis = {(0, 1, 1), (2, 1, 1), (1, 0, 1), (1, 2, 1), (1, 1, 0), (1, 1, 2), (1, 1, 1)}
    for i in range(1, n - 1):
        for j in range(1, n - 1):
            for kk in range(1, n - 1):
                row = S[i, j, kk]
                for t in np.ndindex(3, 3, 3):
                    if t not in axis:
                        assert row[t] == 0.0
                assert abs(row.sum()) <= 1e-13 * row[1, 1, 1]
                assert row[1, 1, 1] > 0.0
                # symmetry: coupling p -> p + d equals p + d -> p
                for (a, b, c) in axis - {(1, 1, 1)}:
                    q = (i + a - 1, j + b - 1, kk + c - 1)
                    if all(1 <= x <= n - 2 for x in q):
                        assert row[a, b, c] == pytest.approx(S[q][2 - a, 2 - b, 2 - c], rel=1e-14)


def face_formula(k, p, d):
    """Minus the coupling of p and p + e_d from the six Kuhn tetrahedra of that edge."""
    e = [np.eye(3, dtype=int)[x] for x in range(3)]
    a, b = [x for x in range(3) if x != d]
    P = np.array(p)
    v = lambda off: k[tuple(P + off)]
    ed, ea, eb = e[d], e[a], e[b]
    s6 = v(0 * ed) + v(ed)
    s2 = v(ed + ea) + v(ed + eb) + v(ed + ea + eb) + v(-ea) + v(-eb) + v(-ea - eb)
    return (6.0 * s6 + 2.0 * s2) / 24.0


def test_axis_coupling_closed_form():
    n = 7
    k = random_k(n, seed=11)
    S = O.fe_stencil(k)
    for p in [(2, 3, 4), (1, 1, 1), (5, 2, 3), (3, 5, 1)]:
        for d in range(3):
            t = [1, 1, 1]
            t[d] = 2
            assert -S[p][tuple(t)] == pytest.approx(face_formula(k, p, d), rel=1e-14)


def test_constant_k_is_the_seven_point_laplacian():
    n = 9
    S = O.fe_stencil(np.ones((n, n, n)))
    row = S[4, 4, 4]
    assert row[1, 1, 1] == pytest.approx(6.0, rel=1e-14)
    for t in [(0, 1, 1), (2, 1, 1), (1, 0, 1), (1, 2, 1), (1, 1, 0), (1, 1, 2)]:
        assert row[t] == pytest.approx(-1.0, rel=1e-14)
    # the solution of A'u = h^2 equals the DST-I closed form of the FD Laplacian
    m = n - 2
    h = 1.0 / (n - 1)
    pp = np.arange(1, m + 1)
    lam = 2.0 - 2.0 * np.cos(np.pi * pp / (m + 1))
    L = lam[:, None, None] + lam[None, :, None] + lam[None, None, :]
    ud = scipy.fft.idstn(scipy.fft.dstn(np.full((m, m, m), h * h), type=1) / L, type=1)
    u, cyc, rel = O.fe_solve(np.ones((n, n, n)), O.rhs(n), tol=1e-13, max_cycles=60)
    assert np.max(np.abs(u[1:-1, 1:-1, 1:-1] - ud)) <= 1e-12 * np.max(ud)


def test_manufactured_solution_second_order():
    pi = math.pi
    errs = []
    for n in (9, 17, 33):
        x = np.arange(n) / (n - 1)
        X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
        k = np.exp(X + 2 * Y - Z) / 2.0
        us = np.sin(pi * X) * np.sin(pi * Y) * np.sin(pi * Z)
        gk_gu = k * pi * (np.cos(pi * X) * np.sin(pi * Y) * np.sin(pi * Z)
                          + 2 * np.sin(pi * X) * np.cos(pi * Y) * np.sin(pi * Z)
                          - np.sin(pi * X) * np.sin(pi * Y) * np.cos(pi * Z))
        f = -gk_gu + 3 * pi**2 * k * us
        h = 1.0 / (n - 1)
        u, _, _ = O.fe_solve(k, h * h * f, tol=1e-12, max_cycles=60)
        errs.append(np.max(np.abs(u - us)))
    r = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.5 < x < 4.5 for x in r), (errs, r)


def test_fe_operator_differs_from_fd_for_variable_k():
    # the two discretisations agree for constant k and differ otherwise
    n = 9
    k = random_k(n, seed=5)
    u = np.zeros((n, n, n))
    u[1:-1, 1:-1, 1:-1] = np.random.Generator(np.random.PCG64(1)).normal(size=(n - 2,) * 3)
    a, b = O.fe_apply(k, u), O.apply(k, u)
    assert np.max(np.abs(a - b)) > 1e-3 * np.max(np.abs(b))
    assert np.allclose(O.fe_apply(np.ones_like(k), u), O.apply(np.ones_like(k), u), rtol=1e-13,
                       atol=1e-13)


def test_fe_sample_contracts_and_couples_levels():
    r = O.mlmc_sample_fe(9, 1, 3)
    assert 0 < r["cycles"][0] <= 20 and 0 < r["cycles"][1] <= 20
    assert abs(r["Y"]) < 0.1 * abs(r["Qf"])
