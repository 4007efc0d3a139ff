"""Pins of the oracle's random-number and random-field steps.

Random numbers: each sample omega is a fixed stream of Philox4x32-10 words
keyed by (seed, level) (Algorithm 1 needs one omega shared by the fine and
coarse solve of a sample, Section 2.2).  The generator is pinned bit for bit
against rocRAND's independent philox4x32_10 engine (host build), and the
derived normals against their distribution.

Field: log k is the 4x4x4 separable Karhunen-Loeve expansion of the
exponential covariance of Section 3.2 (eq. def:expcov) with the 1D kernel
exp(-|s-t|/lambda).  The 1D eigenpairs are pinned against a Nystrom
discretisation of the integral operator (numpy eigh), which shares nothing
with the oracle's root finding, and the field against a numpy evaluation from
those Nystrom eigenfunctions.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.integrate
import scipy.stats

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("rr") / "philox_rr")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", "-o", exe,
                           os.path.join(HERE, "helpers", "philox_rocrand.cpp")])

    def run(seed, level):
        out = subprocess.check_output([exe, str(seed), str(level)], text=True)
        return np.array([int(x) for x in out.split()], dtype=np.uint32)
    return run


@pytest.mark.parametrize("seed,level", [(0, 0), (1, 0), (63, 1), (2**32 + 7, 2),
                                        (0xFFFFFFFFFFFFFFFF, 3), (123456789, 0xFFFFFFFF)])
def test_philox_words_match_rocrand(rocrand_philox, seed, level):
    assert np.array_equal(O.philox_words(seed, level), rocrand_philox(seed, level))


def test_uniform_ints_range_and_uniformity():
    M = np.concatenate([O.uniform_ints(s, 1) for s in range(2000)])
    assert M.max() < 2**53
    U = (M.astype(np.float64) + 1.0) * 2.0**-53
    assert U.min() > 0.0 and U.max() <= 1.0
    # Kolmogorov-Smirnov against U(0,1) on 128000 draws
    assert scipy.stats.kstest(U, "uniform").pvalue > 1e-4


def test_gaussians_are_standard_normal():
    xi = np.concatenate([O.gaussians(s, 0) for s in range(4000)])
    assert abs(xi.mean()) < 5 / math.sqrt(xi.size)
    assert abs(xi.var() - 1.0) < 5 * math.sqrt(2.0 / xi.size)
    assert scipy.stats.kstest(xi, "norm").pvalue > 1e-4
    # different levels of one seed are different streams (independent levels)
    assert not np.array_equal(O.gaussians(5, 0), O.gaussians(5, 1))
    # deterministic
    assert np.array_equal(O.gaussians(5, 2), O.gaussians(5, 2))


def _nystrom(lam, nq=1600, nmodes=4):
    """Eigenpairs of exp(-|s-t|/lam) on [0,1] by composite Gauss-Legendre Nystrom."""
    panels = 200
    g, w = np.polynomial.legendre.leggauss(nq // panels)
    edges = np.linspace(0.0, 1.0, panels + 1)
    s = np.concatenate([(a + b) / 2 + (b - a) / 2 * g for a, b in zip(edges[:-1], edges[1:])])
    ws = np.concatenate([(b - a) / 2 * w for a, b in zip(edges[:-1], edges[1:])])
    K = np.exp(-np.abs(s[:, None] - s[None, :]) / lam)
    sq = np.sqrt(ws)
    ev, V = np.linalg.eigh(sq[:, None] * K * sq[None, :])
    order = np.argsort(ev)[::-1][:nmodes]
    theta = ev[order]
    phi_nodes = V[:, order] / sq[:, None]
    # Nystrom interpolation phi(x) = (1/theta) int K(x,t) phi(t) dt, with the
    # sign fixed so that phi(0) > 0 (the convention of sin(ws) + lam w cos(ws))
    signs = []
    for m in range(nmodes):
        Kx = np.exp(-np.abs(0.0 - s) / lam)
        v0 = Kx @ (ws * phi_nodes[:, m]) / theta[m]
        signs.append(1.0 if v0 > 0 else -1.0)
    signs = np.array(signs)

    def phi_fixed(m, x):
        x = np.atleast_1d(np.asarray(x, dtype=np.float64))
        Kx = np.exp(-np.abs(x[:, None] - s[None, :]) / lam)
        return signs[m] * (Kx @ (ws * phi_nodes[:, m])) / theta[m]
    return theta, phi_fixed


@pytest.mark.parametrize("lam", [0.1, 0.05, 0.3])
def test_kl_eigenpairs_match_nystrom(lam):
    om, th, nm = O.kl_1d(lam, 4)
    # one root per interval (m pi, (m+1) pi), increasing
    for m in range(4):
        assert m * math.pi < om[m] < (m + 1) * math.pi
    # the kernel's kink makes the Nystrom error O(1/nq^2): Richardson-extrapolate
    t1, _ = _nystrom(lam, nq=800)
    t2, phi_ny = _nystrom(lam, nq=1600)
    theta_ny = t2 + (t2 - t1) / 3.0
    assert np.allclose(th, theta_ny, rtol=1e-5, atol=0)
    x = np.linspace(0, 1, 41)
    for m in range(4):
        ph = np.array([O.kl_phi(lam, om[m], nm[m], xx) for xx in x])
        assert np.max(np.abs(ph - phi_ny(m, x))) < 1e-4


@pytest.mark.parametrize("lam", [0.1, 0.05])
def test_kl_orthonormal_and_eigen_equation(lam):
    om, th, nm = O.kl_1d(lam, 4)
    f = [lambda s, m=m: O.kl_phi(lam, om[m], nm[m], s) for m in range(4)]
    for a in range(4):
        for b in range(a, 4):
            v, _ = scipy.integrate.quad(lambda s: f[a](s) * f[b](s), 0, 1, limit=200)
            assert abs(v - (1.0 if a == b else 0.0)) < 1e-10
    # int_0^1 exp(-|s-t|/lam) phi(t) dt = theta phi(s), integrand split at the kink
    for m in range(4):
        for s in (0.0, 0.3, 0.77, 1.0):
            g = lambda t: math.exp(-abs(s - t) / lam) * f[m](t)
            v = 0.0
            if s > 0:
                v += scipy.integrate.quad(g, 0, s, limit=200, epsabs=1e-14)[0]
            if s < 1:
                v += scipy.integrate.quad(g, s, 1, limit=200, epsabs=1e-14)[0]
            assert abs(v - th[m] * f[m](s)) < 1e-10


def test_kl_trace():
    # trace of the 1D kernel is int_0^1 C(s,s) ds = 1; the tail after M modes
    # is about 2/(lam pi^2 M)
    lam = 0.1
    M = 3000
    om, th, nm = O.kl_1d(lam, M)
    tail = 2.0 / (lam * math.pi**2 * M)
    assert abs(th.sum() - (1.0 - tail)) < 0.2 * tail


@pytest.mark.parametrize("n", [5, 9, 17])
def test_field_matches_independent_evaluation(n):
    lam, sigma2 = 0.1, 1.0
    xi = O.gaussians(3, 1)
    k = O.field(n, sigma2, lam, xi)
    theta, phi = _nystrom(lam)
    x = np.arange(n) / (n - 1)
    P = np.stack([phi(m, x) for m in range(4)])  # [mode, vertex]
    c = (np.sqrt(sigma2) * np.sqrt(theta[:, None, None] * theta[None, :, None] * theta[None, None, :])
         * xi.reshape(4, 4, 4))
    Z = np.einsum("abc,ai,bj,ck->ijk", c, P, P, P)
    assert np.max(np.abs(np.log(k) - Z)) < 1e-3


def test_field_special_cases():
    xi = O.gaussians(11, 2)
    assert np.array_equal(O.field(9, 0.0, 0.1, xi), np.ones((9, 9, 9)))
    kf = O.field(33, 2.0, 0.05, xi)
    kc = O.field(17, 2.0, 0.05, xi)
    # coarse vertices are fine vertices at even indices: same value bit for bit
    assert np.array_equal(kc, kf[::2, ::2, ::2])
    assert np.array_equal(O.inject(kf), kc)
    assert (kf > 0).all()


def test_field_pointwise_variance():
    # Var Z(x) = sigma^2 sum_abc theta_a theta_b theta_c phi_a(x)^2 phi_b(y)^2 phi_c(z)^2
    lam, sigma2, n = 0.1, 1.0, 5
    theta, phi = _nystrom(lam)
    x = np.arange(n) / (n - 1)
    P2 = np.stack([phi(m, x) ** 2 for m in range(4)])
    v1 = theta @ P2  # per-axis variance factor
    var_expected = sigma2 * np.einsum("i,j,k->ijk", v1, v1, v1)
    S = 3000
    Z = np.stack([np.log(O.field(n, sigma2, lam, O.gaussians(s, 0))) for s in range(S)])
    var = Z.var(axis=0)
    # sample variance of a Gaussian: sd = var * sqrt(2/S)
    assert np.all(np.abs(var - var_expected) < 5 * var_expected * math.sqrt(2.0 / S))
    assert np.all(np.abs(Z.mean(axis=0)) < 5 * np.sqrt(var_expected / S))


def test_box_muller_pairs_radius_and_angle():
    """The normals come in Box-Muller pairs built from two uniforms of the same
    sample: (xi_2p, xi_2p+1) = R (cos a, sin a) with R^2 = -2 ln U_2p and
    a = 2 pi U_2p+1.  The uniforms come from the oracle's 53-bit integers,
    U = (M + 1) 2^-53, so both identities pin the pairing (which uniform is the
    radius, which the angle, cos on the even and sin on the odd index) beyond
    what the marginal moments can see."""
    for seed, level in [(0, 0), (1, 3), (2**40 + 5, 1), (0xFFFFFFFFFFFFFFFF, 7)]:
        M = O.uniform_ints(seed, level)
        U = (M.astype(np.float64) + 1.0) * 2.0**-53
        xi = O.gaussians(seed, level)
        x, y = xi[0::2], xi[1::2]
        r2 = -2.0 * np.log(U[0::2])
        assert np.allclose(x * x + y * y, r2, rtol=1e-13, atol=1e-300)
        a = np.mod(np.arctan2(y, x), 2.0 * np.pi)
        want = np.mod(2.0 * np.pi * U[1::2], 2.0 * np.pi)
        d = np.abs(a - want)
        d = np.minimum(d, 2.0 * np.pi - d)
        assert np.all(d <= 1e-12 * np.maximum(1.0, 1.0 / np.sqrt(r2)))


def test_box_muller_pair_members_uncorrelated():
    """Members of a pair are independent N(0,1): their correlation over 10^5
    pairs is zero within sampling error, and the angle is uniform (a repeated
    angle, xi_2p+1 = R cos a, would give correlation 1)."""
    xi = np.concatenate([O.gaussians(s, 2) for s in range(3200)])
    x, y = xi[0::2], xi[1::2]
    r = np.corrcoef(x, y)[0, 1]
    assert abs(r) < 5.0 / math.sqrt(x.size)
    a = np.mod(np.arctan2(y, x), 2.0 * np.pi) / (2.0 * np.pi)
    assert scipy.stats.kstest(a, "uniform").pvalue > 1e-4
