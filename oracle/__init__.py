"""ctypes/numpy view of the plain FP64 CPU oracle (``mlmc_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the product path
in ``paper_1607_03252_amd`` never does, and the two share no code.

Every array is an ``n x n x n`` float64 numpy array indexed ``[i, j, k]`` for
the vertex ``(i h, j h, k h)`` with ``h = 1/(n-1)`` (k, the z index, fastest).
Section and equation references are to arXiv 1607.03252.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mlmc_oracle.c")
_LIB = os.path.join(_HERE, "libmlmc_oracle.so")

OR_OK, OR_EINVAL, OR_ENOCONV = 0, -1, -3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
             "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp, ip, u32p, u64p = (C.POINTER(C.c_double), C.POINTER(C.c_int),
                              C.POINTER(C.c_uint32), C.POINTER(C.c_uint64))
        L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.or_philox_words.argtypes = [C.c_uint64, C.c_uint32, u32p]
        L.or_uniform_ints.argtypes = [C.c_uint64, C.c_uint32, u64p]
        L.or_gaussians.argtypes = [C.c_uint64, C.c_uint32, dp]
        L.or_kl_1d.argtypes = [C.c_double, C.c_int, dp, dp, dp]
        L.or_kl_phi.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double]
        L.or_kl_phi.restype = C.c_double
        L.or_field.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp]
        L.or_apply.argtypes = [C.c_int, dp, dp, dp]
        L.or_residual.argtypes = [C.c_int, dp, dp, dp, dp]
        L.or_rbgs_sweep.argtypes = [C.c_int, dp, dp, dp]
        L.or_restrict.argtypes = [C.c_int, dp, dp]
        L.or_prolong_add.argtypes = [C.c_int, dp, dp]
        L.or_inject.argtypes = [C.c_int, dp, dp]
        L.or_vcycle.argtypes = [C.c_int, dp, dp, dp, C.c_int, C.c_int]
        L.or_norm2.argtypes = [C.c_int, dp]
        L.or_norm2.restype = C.c_double
        L.or_solve.argtypes = [C.c_int, dp, dp, dp, C.c_int, C.c_int, C.c_double, C.c_int,
                               C.c_int, ip, dp, dp]
        L.or_qoi.argtypes = [C.c_int, dp]
        L.or_qoi.restype = C.c_double
        L.or_mlmc_sample.argtypes = [C.c_int, C.c_int, C.c_uint64, C.c_double, C.c_double,
                                     C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                     dp, dp, dp, ip]
        L.or_point_qoi.argtypes = [C.c_int, dp]
        L.or_point_qoi.restype = C.c_double
        L.or_flux_qoi.argtypes = [C.c_int, dp, dp]
        L.or_flux_qoi.restype = C.c_double
        L.or_fmg.argtypes = [C.c_int, dp, dp, dp, C.c_int, C.c_int, C.c_int]
        L.or_mlmc_sample_ex.argtypes = [C.c_int, C.c_int, C.c_uint64, C.c_double, C.c_double,
                                        C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                        C.c_int, C.c_int, dp, dp, dp, ip]
        L.or_fe_stencil.argtypes = [C.c_int, dp, dp]
        L.or_fe_apply.argtypes = [C.c_int, dp, dp, dp]
        L.or_fe_solve.argtypes = [C.c_int, dp, dp, dp, C.c_int, C.c_int, C.c_double, C.c_int,
                                  C.c_int, ip, dp]
        L.or_mlmc_sample_fe.argtypes = [C.c_int, C.c_int, C.c_uint64, C.c_double, C.c_double,
                                        C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                        dp, dp, dp, ip]
        L.or_white_noise.argtypes = [C.c_uint64, C.c_uint32, C.c_long, dp]
        L.or_white_noise.restype = None
        L.or_spde_operator.argtypes = [C.c_int, dp, dp]
        L.or_spde_restrict.argtypes = [C.c_int, dp, dp]
        L.or_spde_prolong_add.argtypes = [C.c_int, dp, dp]
        L.or_spde_solve.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp, C.c_int, C.c_int,
                                    C.c_double, C.c_int, ip, dp]
        L.or_spde_rhs.argtypes = [C.c_int, dp, dp]
        L.or_spde_to_k.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp]
        L.or_mlmc_sample_spde.argtypes = [C.c_int, C.c_int, C.c_uint64, C.c_double, C.c_double,
                                          C.c_int, C.c_int, C.c_double, C.c_int, C.c_double,
                                          dp, dp, dp, ip, ip]
        L.or_sum.argtypes = [dp, C.c_long]
        L.or_sum.restype = C.c_double
        _lib = L
    return _lib


def _d(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(st, what):
    if st != OR_OK:
        raise RuntimeError("oracle %s failed with status %d" % (what, st))


# ---- counter-based RNG (Philox4x32-10, SC'11 definition) -------------------
def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def philox_words(seed: int, level: int) -> np.ndarray:
    o = np.zeros(128, dtype=np.uint32)
    lib().or_philox_words(seed, level, o.ctypes.data_as(C.POINTER(C.c_uint32)))
    return o


def uniform_ints(seed: int, level: int) -> np.ndarray:
    o = np.zeros(64, dtype=np.uint64)
    lib().or_uniform_ints(seed, level, o.ctypes.data_as(C.POINTER(C.c_uint64)))
    return o


def gaussians(seed: int, level: int) -> np.ndarray:
    o = np.zeros(64)
    lib().or_gaussians(seed, level, _d(o))
    return o


# ---- KL expansion and field (Section 3.2, eq. def:expcov) -----------------
def kl_1d(lam: float, nterms: int = 4):
    om, th, nm = np.zeros(nterms), np.zeros(nterms), np.zeros(nterms)
    _check(lib().or_kl_1d(lam, nterms, _d(om), _d(th), _d(nm)), "kl_1d")
    return om, th, nm


def kl_phi(lam, omega, norm, s):
    return lib().or_kl_phi(lam, omega, norm, s)


def field(n: int, sigma2: float, lam: float, xi: np.ndarray) -> np.ndarray:
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    k = np.zeros((n, n, n))
    _check(lib().or_field(n, sigma2, lam, _d(xi), _d(k)), "field")
    return k


# ---- operator and multigrid pieces (Section 3, eq. modweak) ----------------
def apply(k, u):
    n = k.shape[0]
    out = np.zeros_like(k)
    _check(lib().or_apply(n, _d(k), _d(np.ascontiguousarray(u)), _d(out)), "apply")
    return out


def residual(k, b, u):
    n = k.shape[0]
    r = np.zeros_like(k)
    _check(lib().or_residual(n, _d(k), _d(b), _d(np.ascontiguousarray(u)), _d(r)), "residual")
    return r


def rbgs_sweep(k, b, u):
    """One red-then-black sweep; returns a new array."""
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    _check(lib().or_rbgs_sweep(k.shape[0], _d(k), _d(b), _d(u)), "rbgs")
    return u


def restrict(r):
    n = r.shape[0]
    nc = (n - 1) // 2 + 1
    bc = np.zeros((nc, nc, nc))
    _check(lib().or_restrict(n, _d(np.ascontiguousarray(r)), _d(bc)), "restrict")
    return bc


def prolong_add(ec, uf):
    uf = np.array(uf, dtype=np.float64, copy=True, order="C")
    _check(lib().or_prolong_add(ec.shape[0], _d(np.ascontiguousarray(ec)), _d(uf)), "prolong")
    return uf


def inject(kf):
    n = kf.shape[0]
    nc = (n - 1) // 2 + 1
    kc = np.zeros((nc, nc, nc))
    _check(lib().or_inject(n, _d(kf), _d(kc)), "inject")
    return kc


def vcycle(k, b, u, nu1=2, nu2=2):
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    _check(lib().or_vcycle(k.shape[0], _d(k), _d(b), _d(u), nu1, nu2), "vcycle")
    return u


def norm2(v):
    return lib().or_norm2(v.shape[0], _d(np.ascontiguousarray(v)))


def solve(k, b, u0=None, tol=1e-8, max_cycles=50, fixed_cycles=0, nu1=2, nu2=2,
          allow_noconv=False):
    """Returns (u, cycles, relres, history)."""
    n = k.shape[0]
    u = np.zeros_like(k) if u0 is None else np.array(u0, dtype=np.float64, copy=True, order="C")
    cyc = C.c_int(0)
    rel = C.c_double(0.0)
    hist = np.zeros(max(max_cycles, fixed_cycles, 1))
    st = lib().or_solve(n, _d(k), _d(b), _d(u), nu1, nu2, tol, max_cycles, fixed_cycles,
                        C.byref(cyc), C.byref(rel), _d(hist))
    if not (st == OR_OK or (allow_noconv and st == OR_ENOCONV)):
        _check(st, "solve")
    return u, cyc.value, rel.value, hist[:cyc.value].copy()


def qoi(u):
    return lib().or_qoi(u.shape[0], _d(np.ascontiguousarray(u)))


def mlmc_sample(n0, level, seed, sigma2=1.0, lam=0.1, tol=1e-8, max_cycles=50,
                fixed_cycles=0, nu1=2, nu2=2):
    """Returns dict(Y, Qf, Qc, cycles=(fine, coarse))."""
    Y, Qf, Qc = C.c_double(), C.c_double(), C.c_double()
    cyc = (C.c_int * 2)()
    st = lib().or_mlmc_sample(n0, level, seed, sigma2, lam, nu1, nu2, tol, max_cycles,
                              fixed_cycles, C.byref(Y), C.byref(Qf), C.byref(Qc), cyc)
    _check(st, "mlmc_sample")
    return dict(Y=Y.value, Qf=Qf.value, Qc=Qc.value, cycles=(cyc[0], cyc[1]))


def point_qoi(u):
    """u(1/4, 1/4, 1/4) (Section 3's point QoI; n = 4m + 1)."""
    return lib().or_point_qoi(u.shape[0], _d(np.ascontiguousarray(u)))


def flux_qoi(k, u):
    """Flux of -k grad u in +x_2 across x_2 = 1/4 (Section 3's flux QoI)."""
    return lib().or_flux_qoi(k.shape[0], _d(k), _d(np.ascontiguousarray(u)))


def fmg(k, f, nu1=4, nu2=4, ncycles=2):
    """Full multigrid (Section 7.1's FMG-ncycles V(nu1,nu2)); f: vertex values."""
    n = k.shape[0]
    u = np.zeros_like(k)
    _check(lib().or_fmg(n, _d(k), _d(np.ascontiguousarray(f, dtype=np.float64)), _d(u), nu1, nu2,
                        ncycles), "fmg")
    return u


QOI_KINDS = {"integral": 0, "point": 1, "flux": 2}


def mlmc_sample_ex(n0, level, seed, sigma2=1.0, lam=0.1, solver="vcycle", qoi="integral",
                   nu1=2, nu2=2, fmg_cycles=2, tol=1e-8, max_cycles=50, fixed_cycles=0):
    """One sample with solver 'vcycle' (to tol) or 'fmg' and a QoI kind."""
    Y, Qf, Qc = C.c_double(), C.c_double(), C.c_double()
    cyc = (C.c_int * 2)()
    st = lib().or_mlmc_sample_ex(n0, level, seed, sigma2, lam, nu1, nu2,
                                 1 if solver == "fmg" else 0, fmg_cycles, QOI_KINDS[qoi], tol,
                                 max_cycles, fixed_cycles, C.byref(Y), C.byref(Qf), C.byref(Qc), cyc)
    _check(st, "mlmc_sample_ex")
    return dict(Y=Y.value, Qf=Qf.value, Qc=Qc.value, cycles=(cyc[0], cyc[1]))


# ---- P1 finite elements on Kuhn tetrahedra (Section 3.1) ---------------------
def fe_stencil(k):
    """27 couplings per vertex of the 1/h-scaled P1 operator: array (n,n,n,3,3,3)."""
    n = k.shape[0]
    S = np.zeros((n, n, n, 3, 3, 3))
    _check(lib().or_fe_stencil(n, _d(k), _d(S)), "fe_stencil")
    return S


def fe_apply(k, u):
    out = np.zeros_like(k)
    _check(lib().or_fe_apply(k.shape[0], _d(k), _d(np.ascontiguousarray(u)), _d(out)), "fe_apply")
    return out


def fe_solve(k, b, tol=1e-8, max_cycles=50, fixed_cycles=0, nu1=2, nu2=2):
    """Returns (u, cycles, relres)."""
    n = k.shape[0]
    u = np.zeros_like(k)
    cyc, rel = C.c_int(0), C.c_double(0.0)
    _check(lib().or_fe_solve(n, _d(k), _d(b), _d(u), nu1, nu2, tol, max_cycles, fixed_cycles,
                             C.byref(cyc), C.byref(rel)), "fe_solve")
    return u, cyc.value, rel.value


def mlmc_sample_fe(n0, level, seed, sigma2=1.0, lam=0.1, qoi="integral", tol=1e-8,
                   max_cycles=50, fixed_cycles=0, nu1=2, nu2=2):
    Y, Qf, Qc = C.c_double(), C.c_double(), C.c_double()
    cyc = (C.c_int * 2)()
    st = lib().or_mlmc_sample_fe(n0, level, seed, sigma2, lam, nu1, nu2, QOI_KINDS[qoi], tol,
                                 max_cycles, fixed_cycles, C.byref(Y), C.byref(Qf), C.byref(Qc),
                                 cyc)
    _check(st, "mlmc_sample_fe")
    return dict(Y=Y.value, Qf=Qf.value, Qc=Qc.value, cycles=(cyc[0], cyc[1]))


# ---- SPDE sampler (Section 3.2, eq. spde) -----------------------------------
def box_n(n: int) -> int:
    """Vertices per axis of the box (-1,2)^3 at the spacing of an n grid on D."""
    return 3 * (n - 1) + 1


def white_noise(seed: int, level: int, count: int) -> np.ndarray:
    o = np.zeros(count)
    lib().or_white_noise(seed, level, count, _d(o))
    return o


def spde_operator(nt: int):
    """(stiffness couplings (nt,nt,nt,3,3,3), lumped mass m (nt,nt,nt)) of the box grid."""
    S = np.zeros((nt, nt, nt, 3, 3, 3))
    m = np.zeros((nt, nt, nt))
    _check(lib().or_spde_operator(nt, _d(S), _d(m)), "spde_operator")
    return S, m


def spde_restrict(r):
    nt = r.shape[0]
    ntc = (nt - 1) // 2 + 1
    bc = np.zeros((ntc, ntc, ntc))
    _check(lib().or_spde_restrict(nt, _d(np.ascontiguousarray(r)), _d(bc)), "spde_restrict")
    return bc


def spde_prolong_add(zc, zf):
    zf = np.array(zf, dtype=np.float64, copy=True, order="C")
    _check(lib().or_spde_prolong_add(zc.shape[0], _d(np.ascontiguousarray(zc)), _d(zf)), "spde_prolong")
    return zf


def spde_solve(b, h, kappa, tol=1e-10, max_cycles=50, nu1=2, nu2=2):
    """Returns (z, cycles, relres) of the scaled box system."""
    nt = b.shape[0]
    z = np.zeros_like(b)
    cyc, rel = C.c_int(0), C.c_double(0.0)
    st = lib().or_spde_solve(nt, h, kappa, _d(np.ascontiguousarray(b)), _d(z), nu1, nu2, tol,
                             max_cycles, C.byref(cyc), C.byref(rel))
    _check(st, "spde_solve")
    return z, cyc.value, rel.value


def spde_rhs(n: int, xi):
    nt = box_n(n)
    b = np.zeros((nt, nt, nt))
    _check(lib().or_spde_rhs(n, _d(np.ascontiguousarray(xi, dtype=np.float64)), _d(b)), "spde_rhs")
    return b


def spde_to_k(n, sigma2, lam, z):
    k = np.zeros((n, n, n))
    _check(lib().or_spde_to_k(n, sigma2, lam, _d(np.ascontiguousarray(z)), _d(k)), "spde_to_k")
    return k


def mlmc_sample_spde(n0, level, seed, sigma2=1.0, lam=0.1, tol=1e-8, max_cycles=50,
                     spde_tol=1e-10, nu1=2, nu2=2):
    Y, Qf, Qc = C.c_double(), C.c_double(), C.c_double()
    cyc, sc = (C.c_int * 2)(), (C.c_int * 2)()
    st = lib().or_mlmc_sample_spde(n0, level, seed, sigma2, lam, nu1, nu2, tol, max_cycles,
                                   spde_tol, C.byref(Y), C.byref(Qf), C.byref(Qc), cyc, sc)
    _check(st, "mlmc_sample_spde")
    return dict(Y=Y.value, Qf=Qf.value, Qc=Qc.value, cycles=(cyc[0], cyc[1]),
                spde_cycles=(sc[0], sc[1]))


def grid_n(n0: int, level: int) -> int:
    """Vertices per axis of MLMC level `level` (h_l = 2^-l h_0, Section 2.3)."""
    return (n0 - 1) * (1 << level) + 1


def sample_fields(n0, level, seed, sigma2, lam):
    """(k_fine, k_coarse or None) for one MLMC sample, from xi(seed, level)."""
    xi = gaussians(seed, level)
    kf = field(grid_n(n0, level), sigma2, lam, xi)
    kc = field(grid_n(n0, level - 1), sigma2, lam, xi) if level > 0 else None
    return kf, kc


def rhs(n: int, f: float = 1.0) -> np.ndarray:
    """b' = h^2 f on every vertex (boundary entries are ignored)."""
    h = 1.0 / (n - 1)
    return np.full((n, n, n), h * h * f)


def csum(x) -> float:
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
    return lib().or_sum(_d(x), x.size)


class LevelAcc(C.Structure):
    """Shifted compensated accumulator for one MLMC level (Section 2.3)."""
    _fields_ = [("n", C.c_long), ("shift", C.c_double), ("s1", C.c_double),
                ("c1", C.c_double), ("s2", C.c_double), ("c2", C.c_double)]

    def __init__(self):
        super().__init__()
        lib().or_acc_init(C.byref(self))

    def add(self, y: float):
        lib().or_acc_add(C.byref(self), C.c_double(y))

    def result(self):
        m, v = C.c_double(), C.c_double()
        lib().or_acc_result(C.byref(self), C.byref(m), C.byref(v))
        return m.value, v.value


# ---- adaptive MLMC (Section 2.3, Algorithm 2) -------------------------------
def quasioptimal_n(eps_s2, var, cost):
    """Eq. (quasioptimal_Nl): N_l ~ eps_s^-2 (sum_k sqrt(s_k^2 C_k)) sqrt(s_l^2 / C_l),
    rounded up; 0 for a level with s_l^2 = 0."""
    import math
    tot = sum(math.sqrt(v * c) for v, c in zip(var, cost))
    return [int(math.ceil(tot * math.sqrt(v / c) / eps_s2)) if v > 0.0 else 0
            for v, c in zip(var, cost)]


def adaptive_mlmc(n0, max_level, eps, theta, alpha, n_init, seed0=0, sigma2=1.0, lam=0.1,
                  tol=1e-8, max_iter=64):
    """Algorithm 2 step by step on the oracle's samples.

    Step 1: L = 1, N_0 = N_1 = N_Init.  Step 2: for every level, new samples
    (sample i of level l has seed seed0 + i) until there are N_l; the level's
    mean and s_l^2 (divisor N) and its cost C_l.  Step 3: N_l from eq.
    (quasioptimal_Nl) with eps_s^2 = theta eps^2 (eq. def:eps), never below
    the samples already taken; if |Yhat_L| > (8^alpha - 1) eps_b with
    eps_b^2 = (1 - theta) eps^2 (the bias estimate, eq. bias_estimate) and
    L < max_level, L -> L + 1 with N_L = N_Init.  Step 4: stop when no N_l
    and not L changed.  Step 5: Q = sum of the level means.

    Readings: C_l is the mean work of a sample of Y_l in node-cycles (fine
    grid vertices x its cycles, plus the coarse grid's), which only enters
    through ratios; the bias test takes the absolute value of Yhat_L.
    Returns a dict with the final L, N, means, variances, costs, Q, the
    sampling RMS sqrt(sum s_l^2 / N_l), the bias estimate, and `trace`: the
    (L, N) after every step 3."""
    import math
    eps_s2 = theta * eps * eps
    eps_b = math.sqrt((1.0 - theta) * eps * eps)
    L = 1
    N = [n_init, n_init]
    accs, work, done = [], [], []
    trace = []
    it = 0
    while True:
        it += 1
        while len(accs) < L + 1:
            accs.append(LevelAcc())
            work.append(0.0)
            done.append(0)
        for l in range(L + 1):
            while done[l] < N[l]:
                r = mlmc_sample(n0, l, seed0 + done[l], sigma2, lam, tol)
                accs[l].add(r["Y"])
                nf = grid_n(n0, l)
                w = float(nf) ** 3 * r["cycles"][0]
                if l > 0:
                    w += float(grid_n(n0, l - 1)) ** 3 * r["cycles"][1]
                work[l] += w
                done[l] += 1
        means = [a.result()[0] for a in accs[:L + 1]]
        var = [a.result()[1] for a in accs[:L + 1]]
        cost = [work[l] / done[l] for l in range(L + 1)]
        newN = [max(N[l], q) for l, q in enumerate(quasioptimal_n(eps_s2, var, cost))]
        changed = newN != N
        N = newN
        if abs(means[L]) > (8.0 ** alpha - 1.0) * eps_b and L < max_level:
            L += 1
            N.append(n_init)
            changed = True
        trace.append((L, list(N)))
        if not changed or it >= max_iter:
            break
    means = [a.result()[0] for a in accs[:L + 1]]
    var = [a.result()[1] for a in accs[:L + 1]]
    cost = [work[l] / done[l] for l in range(L + 1)]
    bias = abs(means[L]) / (8.0 ** alpha - 1.0)
    return {"L": L, "N": N, "mean": means, "var": var, "cost": cost,
            "Q": math.fsum(means),
            "sampling_rms": math.sqrt(sum(v / n for v, n in zip(var, N))),
            "bias_estimate": bias, "bias_ok": bias <= eps_b, "iterations": it,
            "trace": trace}
