"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/mlmcmg.h declares, rejects bad plan descriptions
before touching the device, and its host-side level accumulator (mean and
s^2 with divisor N, Section 2.3) matches correctly rounded sums."""
import ctypes as C
import math
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mlmcmg.h")


@pytest.fixture(scope="module")
def M():
    import paper_1607_03252_amd as M
    if not os.path.exists(M.LIB_PATH):
        from paper_1607_03252_amd import build
        build.build()
    M.lib()
    return M


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for must in ("mg_plan_create", "mg_plan_destroy", "mg_solve", "mlmc_sample_batch",
                 "mlmc_philox", "mlmc_field", "mg_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(M):
    out = subprocess.check_output(["nm", "-D", "--defined-only", M.LIB_PATH], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    assert sorted(M.exported_symbols()) == declared_functions()
    for n in declared_functions():
        getattr(M.lib(), n)


def test_plan_desc_defaults(M):
    d = M.mg_plan_desc_default()
    assert (d.n0, d.max_level, d.nu1, d.nu2, d.max_cycles) == (33, 0, 2, 2, 50)
    assert d.tol == 1e-8 and d.sigma2 == 1.0 and d.corr_len == 0.1 and d.kl_per_axis == 4
    assert C.sizeof(M.mg_plan_desc) == 80


@pytest.mark.parametrize("field,value", [("n0", 32), ("n0", 2), ("max_level", -1), ("nu1", -1),
                                         ("max_cycles", 0), ("tol", 0.0), ("sigma2", -1.0),
                                         ("corr_len", 0.0), ("precision", 7)])
def test_bad_plan_descriptions_rejected_on_host(M, field, value):
    d = M.mg_plan_desc_default()
    setattr(d, field, value)
    h = C.c_void_p()
    assert M.lib().mg_plan_create(C.byref(d), C.byref(h)) == M.MG_EINVAL
    assert not h.value


def test_unsupported_kl_modes(M):
    d = M.mg_plan_desc_default()
    d.kl_per_axis = 5
    h = C.c_void_p()
    assert M.lib().mg_plan_create(C.byref(d), C.byref(h)) == M.MG_ENOTIMPL


def test_null_plan_calls_fail_cleanly(M):
    L = M.lib()
    assert L.mg_solve(None, 9, None, None, None, 0.0, 0, None, None) == M.MG_EINVAL
    assert L.mlmc_sample_batch(None, 0, None, 1, None, None, None, None, 0) == M.MG_EINVAL
    assert L.mg_plan_destroy(None) == M.MG_EINVAL


def test_level_accumulator_host(M):
    rng = np.random.default_rng(7)
    y = 0.02 + 1e-6 * rng.standard_normal(20000)
    acc = M.mlmc_acc_init()
    M.mlmc_acc_add(acc, y[:7])
    M.mlmc_acc_add(acc, y[7:])
    mean, var = M.mlmc_acc_result(acc)
    m_ref = math.fsum(y) / y.size
    v_ref = math.fsum((v - m_ref) ** 2 for v in y) / y.size
    assert abs(mean - m_ref) <= 2e-16 * abs(m_ref)
    assert abs(var - v_ref) <= 1e-10 * v_ref
    empty = M.mlmc_acc_init()
    assert M.mlmc_acc_result(empty) == (0.0, 0.0)


@pytest.mark.parametrize("seed,level", [(0, 0), (1, 0), (63, 1), (2**32 + 7, 2),
                                        (0xFFFFFFFFFFFFFFFF, 3), (123456789, 2**31 - 1)])
def test_host_philox_words_match_oracle(M, seed, level):
    """mlmc_philox_words (host, no device work) gives the oracle's words of
    sample (seed, level) bit for bit; the oracle's generator is itself pinned
    against rocRAND's philox4x32_10 engine."""
    import oracle as O
    assert np.array_equal(M.mlmc_philox_words(seed, level), O.philox_words(seed, level))


def test_host_philox_words_rejects_bad_arguments(M):
    out = (C.c_uint32 * 128)()
    assert M.lib().mlmc_philox_words(0, -1, out) == M.MG_EINVAL
    assert M.lib().mlmc_philox_words(0, 0, None) == M.MG_EINVAL


def _exact_exp(x):
    from decimal import Decimal, getcontext
    getcontext().prec = 40
    return Decimal(x).exp()


def test_kl_exp_within_two_ulp_of_exact(M):
    """The exponential the kernels form k = exp(Z) and wh = exp(-Z)/2 with
    (Tang's table-driven method, evaluated on the host by the same code and
    table) against the exactly rounded value: within 2 units in the last
    place on random arguments that reach every table entry and both signs,
    on the multiples of ln2/32 (the table's nodes) and near 0, and exact
    at x = 0."""
    from decimal import Decimal
    rng = np.random.default_rng(7)
    xs = np.concatenate([rng.uniform(-40.0, 40.0, 4000), rng.uniform(-0.05, 0.05, 1000),
                         np.arange(-64, 65) * (math.log(2.0) / 32.0)])
    worst = 0.0
    for x in xs:
        got = M.mlmc_exp(float(x))
        ref = _exact_exp(float(x))
        ulp = math.ulp(float(ref))
        err = abs(Decimal(got) - ref) / Decimal(ulp)
        worst = max(worst, float(err))
    assert worst <= 2.0, worst
    assert M.mlmc_exp(0.0) == 1.0
    # arguments beyond +-700 are clamped
    assert M.mlmc_exp(800.0) == M.mlmc_exp(700.0)
    assert M.mlmc_exp(-800.0) == M.mlmc_exp(-700.0)
