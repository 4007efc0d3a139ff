"""Pins of the oracle's discretisation and multigrid solver.

Model problem (Section 3, eq. modweak): -div(k grad u) = f on (0,1)^3, u = 0 on
the boundary.  The oracle uses 7-point finite differences with harmonic-mean
face coefficients, scaled by h^2, and V(2,2) red-black Gauss-Seidel cycles
(the paper's solver is a multigrid with pre- and post-smoothing, Section 7.1).

Pins that do not reuse the oracle's own formulas:
  * k = 1: the scaled 7-point Laplacian is diagonalised by the type-I discrete
    sine transform (scipy), giving the discrete solution in closed form;
  * a manufactured smooth solution with a variable k converges at O(h^2);
  * the operator assembled column by column is symmetric positive definite;
  * a dense solve (numpy) of that matrix equals the multigrid solution;
  * one red-black sweep equals block Gauss-Seidel on the dense matrix split
    into its red and black blocks;
  * restriction and prolongation are adjoint (P = 8 R^T) and reproduce
    constants / hat functions;
  * constant-k V(2,2) contraction stays below 0.15.
"""
import math

import numpy as np
import pytest
import scipy.fft

import oracle as O


def dst_solve(b_int):
    """Solve the h^2-scaled 7-point Laplacian (k = 1) on interior values."""
    m = b_int.shape[0]
    p = np.arange(1, m + 1)
    lam1 = 2.0 - 2.0 * np.cos(np.pi * p / (m + 1))
    L = lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]
    bh = scipy.fft.dstn(b_int, type=1)
    return scipy.fft.idstn(bh / L, type=1)


def dense_matrix(k):
    """Columns of A' from the oracle's operator applied to unit vectors."""
    n = k.shape[0]
    m = n - 2
    idx = [(i, j, kk) for i in range(1, n - 1) for j in range(1, n - 1) for kk in range(1, n - 1)]
    A = np.zeros((m**3, m**3))
    for c, (i, j, kk) in enumerate(idx):
        e = np.zeros((n, n, n))
        e[i, j, kk] = 1.0
        A[:, c] = O.apply(k, e)[1:-1, 1:-1, 1:-1].ravel()
    return A, idx


def random_k(n, seed=0, sigma2=1.0, lam=0.1):
    return O.field(n, sigma2, lam, O.gaussians(seed, 0))


@pytest.mark.parametrize("n", [9, 17, 33])
def test_constant_k_matches_dst_closed_form(n):
    k = np.ones((n, n, n))
    b = O.rhs(n)
    u, cyc, rel, _ = O.solve(k, b, tol=1e-13, max_cycles=60)
    exact = dst_solve(b[1:-1, 1:-1, 1:-1])
    err = np.linalg.norm(u[1:-1, 1:-1, 1:-1] - exact) / np.linalg.norm(exact)
    assert err < 1e-11
    h = 1.0 / (n - 1)
    q_exact = h**3 * math.fsum(exact.ravel())
    assert abs(O.qoi(u) - q_exact) < 1e-12 * q_exact


def test_constant_k_qoi_converges_to_continuum():
    # int_D u for -Lap u = 1: (512/pi^8) sum over odd i,j,k of 1/((ijk)^2 (i^2+j^2+k^2))
    o = np.arange(1, 400, 2, dtype=np.float64)
    I, J, K = np.meshgrid(o, o, o, indexing="ij")
    q_cont = 512.0 / math.pi**8 * np.sum(1.0 / ((I * J * K) ** 2 * (I**2 + J**2 + K**2)))
    errs = []
    for n in (9, 17, 33):
        exact = dst_solve(O.rhs(n)[1:-1, 1:-1, 1:-1])
        errs.append(abs((1.0 / (n - 1)) ** 3 * exact.sum() - q_cont))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.5 < r < 4.5 for r in ratios), ratios


def _manufactured(n):
    x = np.arange(n) / (n - 1)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    pi = math.pi
    k = np.exp(X + 2 * Y - Z) / 2.0
    us = np.sin(pi * X) * np.sin(pi * Y) * np.sin(pi * Z)
    # f = -div(k grad u*) = -(grad k . grad u*) + 3 pi^2 k u*, grad k = k (1, 2, -1)
    gk_gu = k * pi * (np.cos(pi * X) * np.sin(pi * Y) * np.sin(pi * Z)
                      + 2 * np.sin(pi * X) * np.cos(pi * Y) * np.sin(pi * Z)
                      - np.sin(pi * X) * np.sin(pi * Y) * np.cos(pi * Z))
    f = -gk_gu + 3 * pi**2 * k * us
    return k, f, us


def test_manufactured_solution_second_order():
    errs = []
    for n in (9, 17, 33, 65):
        k, f, us = _manufactured(n)
        h = 1.0 / (n - 1)
        u, _, _, _ = O.solve(k, h * h * f, tol=1e-12, max_cycles=60)
        errs.append(np.max(np.abs(u - us)))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(3.6 < r < 4.4 for r in ratios), (errs, ratios)


def test_operator_symmetric_positive_definite():
    k = random_k(7, seed=4, sigma2=2.0, lam=0.05)
    A, _ = dense_matrix(k)
    assert np.max(np.abs(A - A.T)) < 1e-14 * np.max(np.abs(A))
    assert np.linalg.eigvalsh(A).min() > 0.0
    # k = 1: diagonal 6, off-diagonals -1 (h^2-scaled 7-point Laplacian)
    A1, _ = dense_matrix(np.ones((5, 5, 5)))
    assert np.allclose(np.diag(A1), 6.0) and set(np.unique(A1)) <= {-1.0, 0.0, 6.0}


def test_multigrid_equals_dense_solve():
    n = 9
    k = random_k(n, seed=9, sigma2=1.0, lam=0.1)
    b = O.rhs(n) * (1.0 + np.arange(n**3).reshape(n, n, n) % 5)  # non-constant rhs
    A, idx = dense_matrix(k)
    ud = np.linalg.solve(A, b[1:-1, 1:-1, 1:-1].ravel())
    u, cyc, rel, _ = O.solve(k, b, tol=1e-14, max_cycles=80)
    assert rel <= 1e-14
    assert np.linalg.norm(u[1:-1, 1:-1, 1:-1].ravel() - ud) / np.linalg.norm(ud) < 1e-12


def test_rbgs_sweep_equals_block_gauss_seidel():
    n = 7
    k = random_k(n, seed=2)
    rng = np.random.default_rng(0)
    b = rng.standard_normal((n, n, n))
    u0 = np.zeros((n, n, n))
    u0[1:-1, 1:-1, 1:-1] = rng.standard_normal((n - 2,) * 3)
    A, idx = dense_matrix(k)
    red = np.array([(i + j + kk) % 2 == 0 for (i, j, kk) in idx])
    blk = ~red
    bi = b[1:-1, 1:-1, 1:-1].ravel()
    v = u0[1:-1, 1:-1, 1:-1].ravel().copy()
    # red block is diagonal: red points couple only to black points
    assert np.count_nonzero(A[np.ix_(red, red)] - np.diag(np.diag(A[np.ix_(red, red)]))) == 0
    v[red] = (bi[red] - A[np.ix_(red, blk)] @ v[blk]) / np.diag(A)[red]
    v[blk] = (bi[blk] - A[np.ix_(blk, red)] @ v[red]) / np.diag(A)[blk]
    u1 = O.rbgs_sweep(k, b, u0)
    assert np.max(np.abs(u1[1:-1, 1:-1, 1:-1].ravel() - v)) < 1e-13 * np.max(np.abs(v))
    # boundary untouched
    assert np.array_equal(u1[0], u0[0])


def test_restriction_prolongation_adjoint():
    rng = np.random.default_rng(1)
    n, nc = 17, 9
    r = np.zeros((n, n, n))
    r[1:-1, 1:-1, 1:-1] = rng.standard_normal((n - 2,) * 3)
    e = np.zeros((nc, nc, nc))
    e[1:-1, 1:-1, 1:-1] = rng.standard_normal((nc - 2,) * 3)
    bc = O.restrict(r)  # = 4 R r (h^2 scaling)
    Pe = O.prolong_add(e, np.zeros((n, n, n)))
    lhs = math.fsum((r * Pe).ravel())
    rhs = 8.0 * math.fsum((bc / 4.0 * e).ravel())
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


def test_restriction_of_constant_and_prolongation_of_hat():
    n, nc = 17, 9
    r = np.zeros((n, n, n))
    r[1:-1, 1:-1, 1:-1] = 1.0
    bc = O.restrict(r)
    # full weighting preserves constants; the h^2 scaling multiplies by 4
    assert np.allclose(bc[1:-1, 1:-1, 1:-1], 4.0, rtol=0, atol=1e-15)
    e = np.zeros((nc, nc, nc))
    e[3, 4, 5] = 1.0
    Pe = O.prolong_add(e, np.zeros((n, n, n)))
    x = np.arange(n) / 2.0  # fine index in coarse units
    hat = lambda c: np.maximum(0.0, 1.0 - np.abs(x - c))
    expect = np.einsum("i,j,k->ijk", hat(3), hat(4), hat(5))
    assert np.array_equal(Pe, expect)


@pytest.mark.parametrize("n", [33, 65])
def test_constant_k_contraction_below_0p15(n):
    k = np.ones((n, n, n))
    _, cyc, _, hist = O.solve(k, O.rhs(n), fixed_cycles=6, max_cycles=6)
    rates = hist[1:] / hist[:-1]
    assert rates.max() < 0.15, rates


def test_random_k_contraction_and_fixed_cycles():
    n = 33
    k = random_k(n, seed=0)
    b = O.rhs(n)
    u, cyc, rel, hist = O.solve(k, b, tol=1e-8, max_cycles=50)
    assert rel <= 1e-8 and (cyc == 1 or hist[-2] > 1e-8)
    assert np.all(hist[1:] / hist[:-1] < 0.2)
    # fixed-cycle mode runs exactly that many cycles and reproduces the tol run
    u2, cyc2, rel2, _ = O.solve(k, b, tol=-1.0, fixed_cycles=cyc)
    assert cyc2 == cyc and np.array_equal(u, u2) and rel2 == rel


def test_nonconvergence_reported():
    n = 17
    k = random_k(n, seed=0)
    u, cyc, rel, _ = O.solve(k, O.rhs(n), tol=1e-30, max_cycles=3, allow_noconv=True)
    assert cyc == 3 and rel > 1e-30
    with pytest.raises(RuntimeError):
        O.solve(k, O.rhs(n), tol=1e-30, max_cycles=3)


def test_smallest_grids_exact():
    # n = 3: one unknown, one cycle solves it exactly
    k = random_k(3, seed=1)
    b = O.rhs(3)
    u, cyc, rel, _ = O.solve(k, b, tol=1e-15, max_cycles=2)
    A, _ = dense_matrix(k)
    assert cyc == 1 and abs(u[1, 1, 1] - b[1, 1, 1] / A[0, 0]) < 1e-18
    # n = 5: two-level cycle converges to the dense solution
    k = random_k(5, seed=1)
    b = O.rhs(5)
    A, _ = dense_matrix(k)
    ud = np.linalg.solve(A, b[1:-1, 1:-1, 1:-1].ravel())
    u, _, _, _ = O.solve(k, b, tol=1e-15, max_cycles=60)
    assert np.allclose(u[1:-1, 1:-1, 1:-1].ravel(), ud, rtol=1e-13, atol=0)


def test_initial_guess_boundary_is_forced_to_zero():
    n = 9
    k = random_k(n)
    b = O.rhs(n)
    u0 = np.full((n, n, n), 3.0)
    u, _, _, _ = O.solve(k, b, u0=u0, tol=1e-12, max_cycles=60)
    ref, _, _, _ = O.solve(k, b, tol=1e-12, max_cycles=60)
    assert np.all(u[0] == 0)
    # both iterates solve the same system to 1e-12: they agree far below the QoI scale
    assert np.max(np.abs(u - ref)) < 1e-9 * np.max(np.abs(ref))



def _series_conductivity(k_of_x, a, b):
    """Effective conductivity of the segment [a, b] of a 1D medium k(x): the
    steady flux per unit gradient, (b - a) / int_a^b dx / k(x), with the
    integral taken by adaptive quadrature (layers in series)."""
    import scipy.integrate
    mid = 0.5 * (a + b)
    inv, _ = scipy.integrate.quad(lambda x: 1.0 / k_of_x(x), a, b, points=[mid],
                                  epsabs=0.0, epsrel=1e-13)
    return (b - a) / inv


def test_face_coefficient_is_series_conductance_of_two_half_edges():
    """Section 3, eq. (modweak): the flux k grad u across the face between two
    vertices.  With k_p on the half-edge at p and k_q on the half-edge at q,
    the exact flux of the 1D two-layer problem fixes the face coefficient;
    the h^2-scaled operator's off-diagonal entry is minus that effective
    conductivity and its diagonal the sum over the six faces.  High-contrast
    vertex values (1e-2 .. 1e2) make any other mean (arithmetic, geometric)
    fail."""
    n = 5
    h = 1.0 / (n - 1)
    rng = np.random.Generator(np.random.PCG64(7))
    k = np.exp(rng.uniform(np.log(1e-2), np.log(1e2), size=(n, n, n)))
    steps = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]

    def ceff(p, q):
        kp, kq = k[p], k[q]
        return _series_conductivity(lambda x: kp if x < 0.5 * h else kq, 0.0, h)

    for p in [(2, 2, 2), (1, 2, 3)]:
        diag = 0.0
        for d in steps:
            q = tuple(a + b for a, b in zip(p, d))
            c = ceff(p, q)
            diag += c
            if min(q) >= 1 and max(q) <= n - 2:
                e = np.zeros((n, n, n))
                e[q] = 1.0
                assert O.apply(k, e)[p] == pytest.approx(-c, rel=1e-12, abs=0.0)
        # faces toward the boundary enter the diagonal with the boundary vertex's k
        e = np.zeros((n, n, n))
        e[p] = 1.0
        assert O.apply(k, e)[p] == pytest.approx(diag, rel=1e-12, abs=0.0)


def test_layered_high_contrast_exact_flux_solution():
    """A medium layered in x: k = 1e-3 up to x = 1/2 + h/2 (the vertex at 1/2
    and the half-edge beyond it), k = 1 beyond.  The exact solution of
    -(k u')' = 0 with constant flux F has u(x_{i+1}) - u(x_i) = F int dx/k over
    the edge (quadrature).  Sampled at the vertices and constant in y, z, it
    must satisfy the h^2-scaled equations exactly in every row whose y, z
    neighbours are interior and whose x neighbours carry the exact values,
    including the two rows at the interface; an arithmetic face mean gives a
    residual of the order of the flux there."""
    n = 9
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    xi_if = 0.5 + 0.5 * h

    def kx(s):
        return 1e-3 if s < xi_if else 1.0

    F = 1.0
    u = np.zeros(n)
    for i in range(n - 1):
        u[i + 1] = u[i] + F * h / _series_conductivity(kx, x[i], x[i + 1])
    k = np.broadcast_to(np.array([kx(s) for s in x])[:, None, None], (n, n, n)).copy()
    U = np.broadcast_to(u[:, None, None], (n, n, n)).copy()
    Au = O.apply(k, U)
    # rows i = 1..n-3 (i = n-2 has the boundary vertex, where u is forced to 0,
    # as a neighbour), j and k away from the y and z boundaries
    rows = Au[1:n - 2, 2:n - 2, 2:n - 2]
    assert np.max(np.abs(rows)) <= 1e-12 * F * h
    # the interface rows are really exercised: their two x fluxes are non-zero
    assert abs(u[5] - u[4]) > 100 * abs(u[6] - u[5])
