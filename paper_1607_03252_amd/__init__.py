"""Python binding of libmlmcmg (include/mlmcmg.h): argument marshalling only.

Every step of the hot path runs in the HIP library; PyTorch supplies device
memory (CUDA tensors on ROCm) and the stream.  There is no CPU fallback: if
the library is missing or no GPU is present, calls raise.

Functions carry the C names: ``mg_plan_create``, ``mg_solve``,
``mlmc_sample_batch``, ``mlmc_sample_mixed``, ``mlmc_philox``, ``mlmc_field``,
``mlmc_acc_*``, ``mg_profile_*``, ``mg_sample_footprint``; the scheduler and
the server are the classes ``Sched`` (mg_sched_*) and ``Server``
(mg_serve_*).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlmcmg.so")

MG_OK, MG_EINVAL, MG_ENOMEM, MG_ENOCONV, MG_EHIP, MG_EBUSY, MG_ENOTIMPL = 0, -1, -2, -3, -4, -5, -6
MG_FP64, MG_MIXED = 0, 1
_NAMES = {0: "MG_OK", -1: "MG_EINVAL", -2: "MG_ENOMEM", -3: "MG_ENOCONV", -4: "MG_EHIP",
          -5: "MG_EBUSY", -6: "MG_ENOTIMPL"}


class MGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (_NAMES.get(status, "?"), status, msg))
        self.status = status


class mg_plan_desc(C.Structure):
    _fields_ = [("n0", C.c_int), ("max_level", C.c_int), ("nu1", C.c_int), ("nu2", C.c_int),
                ("max_cycles", C.c_int), ("tol", C.c_double), ("precision", C.c_int),
                ("sigma2", C.c_double), ("corr_len", C.c_double), ("kl_per_axis", C.c_int),
                ("hbm_budget", C.c_size_t), ("stream", C.c_void_p)]


class mg_ticket(C.Structure):
    _fields_ = [("tag", C.c_longlong), ("seed", C.c_uint64), ("level", C.c_int), ("slot", C.c_int),
                ("lane", C.c_int), ("t_arrival", C.c_double)]


MG_LANE_OPEN, MG_LANE_CLOSE = 1, 2


class mg_lane_event(C.Structure):
    _fields_ = [("kind", C.c_int), ("lane", C.c_int), ("level", C.c_int), ("first", C.c_int),
                ("nslots", C.c_int), ("bytes", C.c_size_t)]


class mg_result(C.Structure):
    _fields_ = [("tag", C.c_longlong), ("seed", C.c_uint64), ("level", C.c_int),
                ("status", C.c_int), ("Y", C.c_double), ("Qf", C.c_double), ("Qc", C.c_double),
                ("cycles_fine", C.c_int), ("cycles_coarse", C.c_int), ("t_arrival", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double)]


MLMC_MAX_LEVELS, MLMC_MAX_TRACE = 11, 64


class mlmc_adaptive_desc(C.Structure):
    _fields_ = [("eps", C.c_double), ("theta", C.c_double), ("alpha", C.c_double),
                ("n_init", C.c_int), ("max_iter", C.c_int), ("max_batch", C.c_int),
                ("seed0", C.c_uint64)]


class mlmc_adaptive_result(C.Structure):
    _fields_ = [("status", C.c_int), ("L", C.c_int), ("iterations", C.c_int), ("bias_ok", C.c_int),
                ("N", C.c_longlong * MLMC_MAX_LEVELS), ("mean", C.c_double * MLMC_MAX_LEVELS),
                ("var", C.c_double * MLMC_MAX_LEVELS), ("cost", C.c_double * MLMC_MAX_LEVELS),
                ("Q", C.c_double), ("sampling_rms", C.c_double), ("bias_estimate", C.c_double),
                ("trace_len", C.c_int), ("trace_L", C.c_int * MLMC_MAX_TRACE),
                ("trace_N", (C.c_longlong * MLMC_MAX_LEVELS) * MLMC_MAX_TRACE)]


class mlmc_level_acc(C.Structure):
    _fields_ = [("n", C.c_longlong), ("shift", C.c_double), ("s1", C.c_double),
                ("c1", C.c_double), ("s2", C.c_double), ("c2", C.c_double)]


_lib = None


def lib():
    """Load libmlmcmg.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmlmcmg.so is not built: run `python -m paper_1607_03252_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, ip, dp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double)
        L.mg_plan_desc_default.argtypes = [C.POINTER(mg_plan_desc)]
        L.mg_plan_desc_default.restype = None
        L.mg_plan_create.argtypes = [C.POINTER(mg_plan_desc), C.POINTER(vp)]
        L.mg_plan_destroy.argtypes = [vp]
        L.mg_plan_set_stream.argtypes = [vp, vp]
        L.mg_plan_get_desc.argtypes = [vp, C.POINTER(mg_plan_desc)]
        L.mlmc_adaptive_desc_default.argtypes = [C.POINTER(mlmc_adaptive_desc)]
        L.mlmc_adaptive_desc_default.restype = None
        L.mlmc_adaptive.argtypes = [vp, C.POINTER(mlmc_adaptive_desc), C.POINTER(mlmc_adaptive_result)]
        L.mg_solve.argtypes = [vp, C.c_int, vp, vp, vp, C.c_double, C.c_int, ip, dp]
        L.mg_solve_noalloc.argtypes = [vp, C.c_int, vp, vp, vp, C.c_double, C.c_int, ip, dp]
        L.mlmc_sample_batch.argtypes = [vp, C.c_int, C.POINTER(C.c_uint64), C.c_int, vp, vp, vp,
                                        vp, C.c_int]
        L.mlmc_sample_mixed.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_uint64), C.c_int,
                                        vp, vp, vp, vp, C.c_int]
        L.mlmc_philox.argtypes = [vp, C.POINTER(C.c_uint64), C.c_int, C.c_int, vp, vp]
        L.mlmc_field.argtypes = [vp, C.c_int, C.c_uint64, C.c_int, vp]
        L.mlmc_philox_words.argtypes = [C.c_uint64, C.c_int, C.POINTER(C.c_uint32)]
        L.mlmc_exp.argtypes = [C.c_double]
        L.mlmc_exp.restype = C.c_double
        L.mlmc_acc_init.argtypes = [C.POINTER(mlmc_level_acc)]
        L.mlmc_acc_init.restype = None
        L.mlmc_acc_add.argtypes = [C.POINTER(mlmc_level_acc), vp, C.c_int, C.c_int]
        L.mlmc_acc_result.argtypes = [C.POINTER(mlmc_level_acc), dp, dp]
        L.mlmc_acc_result.restype = None
        L.mg_profile_enable.argtypes = [vp, C.c_int]
        L.mg_profile_read.argtypes = [vp, C.POINTER(C.c_longlong), dp, dp]
        L.mg_profile_records.argtypes = [vp, C.c_int, ip, ip, ip, dp, ip]
        L.mg_plan_set_option.argtypes = [vp, C.c_char_p, C.c_longlong]
        L.mg_set_tile.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int]
        L.mg_get_tile.argtypes = [vp, C.c_int, ip, ip, ip]
        L.mg_set_tile_for.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
        L.mg_get_tile_for.argtypes = [vp, C.c_int, C.c_int, ip, ip, ip]
        L.mg_autotune.argtypes = [vp, C.c_int, C.c_int, C.c_int]
        L.mg_sample_footprint.argtypes = [vp, C.c_int, C.POINTER(C.c_size_t)]
        L.mg_sched_create.argtypes = [C.c_int, ip, C.POINTER(C.c_size_t), C.c_size_t, C.c_int,
                                      C.POINTER(vp)]
        L.mg_sched_destroy.argtypes = [vp]
        L.mg_sched_submit.argtypes = [vp, C.c_int, C.c_uint64, C.c_longlong, C.c_double]
        L.mg_sched_admit.argtypes = [vp, C.POINTER(mg_ticket), C.c_int, ip]
        L.mg_sched_release.argtypes = [vp, C.c_int]
        L.mg_sched_counts.argtypes = [vp, ip, ip]
        L.mg_sched_events.argtypes = [vp, C.POINTER(mg_lane_event), C.c_int, ip]
        L.mg_sched_set_inflight.argtypes = [vp, C.c_int, C.c_int]
        L.mg_sched_memory.argtypes = [vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t), ip]
        L.mg_serve_create.argtypes = [vp, ip, C.c_int, C.POINTER(vp)]
        L.mg_serve_destroy.argtypes = [vp]
        L.mg_serve_submit.argtypes = [vp, C.c_int, C.c_uint64, C.c_longlong, C.c_double]
        L.mg_serve_step.argtypes = [vp, C.c_int, C.POINTER(mg_result), C.c_int, ip]
        L.mg_serve_now.argtypes = [vp]
        L.mg_serve_now.restype = C.c_double
        L.mg_serve_counts.argtypes = [vp, ip, ip, C.POINTER(C.c_longlong)]
        L.mg_serve_slots.argtypes = [vp, C.c_int]
        L.mg_serve_memory.argtypes = [vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t),
                                      C.POINTER(C.c_size_t), ip, C.POINTER(C.c_longlong),
                                      C.POINTER(C.c_longlong), dp]
        L.mg_last_error.argtypes = [vp]
        L.mg_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def exported_symbols():
    """Names the public header declares (for the ABI check)."""
    return ["mg_plan_desc_default", "mg_plan_create", "mg_plan_destroy", "mg_plan_set_stream",
            "mg_solve", "mlmc_sample_batch", "mlmc_philox", "mlmc_field", "mlmc_acc_init",
            "mlmc_acc_add", "mlmc_acc_result", "mg_profile_enable", "mg_profile_read",
            "mg_last_error", "mg_plan_set_option", "mg_set_tile", "mg_get_tile", "mg_autotune",
            "mlmc_sample_mixed", "mg_sample_footprint", "mg_sched_create", "mg_sched_destroy",
            "mg_sched_submit", "mg_sched_admit", "mg_sched_release", "mg_sched_counts",
            "mg_serve_create", "mg_serve_destroy", "mg_serve_submit", "mg_serve_step",
            "mg_serve_now", "mg_serve_counts", "mg_serve_slots", "mg_set_tile_for",
            "mg_get_tile_for", "mlmc_philox_words", "mg_solve_noalloc",
            "mg_profile_records", "mg_plan_get_desc", "mlmc_adaptive_desc_default",
            "mlmc_adaptive", "mlmc_exp", "mg_sched_events", "mg_sched_set_inflight",
            "mg_sched_memory", "mg_serve_memory"]


def _torch():
    import torch
    return torch


def _current_stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype_name, numel=None, what="tensor"):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA (HIP) tensor" % what)
    if str(t.dtype) != "torch." + dtype_name:
        raise ValueError("%s must be %s, got %s" % (what, dtype_name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if numel is not None and t.numel() < numel:
        raise ValueError("%s needs at least %d elements, has %d" % (what, numel, t.numel()))
    return C.c_void_p(t.data_ptr())


class Plan:
    """Owning handle of an mg_plan."""

    def __init__(self, handle, desc):
        self.handle = handle
        self.desc = desc

    def error(self):
        return lib().mg_last_error(self.handle).decode()

    def check(self, st, allow=(MG_OK,)):
        if st not in allow:
            raise MGError(st, self.error())
        return st

    def destroy(self):
        if self.handle:
            lib().mg_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def mg_plan_desc_default() -> mg_plan_desc:
    d = mg_plan_desc()
    lib().mg_plan_desc_default(C.byref(d))
    return d


def mg_plan_create(desc: mg_plan_desc | None = None, **fields) -> Plan:
    d = desc if desc is not None else mg_plan_desc_default()
    for k, v in fields.items():
        setattr(d, k, v)
    h = C.c_void_p()
    st = lib().mg_plan_create(C.byref(d), C.byref(h))
    if st != MG_OK:
        raise MGError(st, "mg_plan_create rejected the description")
    return Plan(h, d)


def mg_plan_destroy(plan: Plan):
    plan.destroy()


def mg_plan_set_stream(plan: Plan, stream=None):
    s = _current_stream() if stream is None else C.c_void_p(stream)
    return plan.check(lib().mg_plan_set_stream(plan.handle, s))


def mg_plan_set_option(plan: Plan, name: str, value: int):
    return plan.check(lib().mg_plan_set_option(plan.handle, name.encode(), int(value)))


def mg_set_tile(plan: Plan, n: int, tj: int, tk: int, chunks: int = 1):
    return plan.check(lib().mg_set_tile(plan.handle, n, tj, tk, chunks))


def mg_get_tile(plan: Plan, n: int):
    a, b, c = C.c_int(), C.c_int(), C.c_int()
    plan.check(lib().mg_get_tile(plan.handle, n, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def mg_set_tile_for(plan: Plan, n: int, fused_correction: int, tj: int, tk: int, chunks: int = 1):
    return plan.check(lib().mg_set_tile_for(plan.handle, n, int(fused_correction), tj, tk, chunks))


def mg_get_tile_for(plan: Plan, n: int, fused_correction: int):
    a, b, c = C.c_int(), C.c_int(), C.c_int()
    plan.check(lib().mg_get_tile_for(plan.handle, n, int(fused_correction), C.byref(a), C.byref(b),
                                     C.byref(c)))
    return a.value, b.value, c.value


def mg_autotune(plan: Plan, level: int, n_samples: int, reps: int = 5):
    mg_plan_set_stream(plan)
    return plan.check(lib().mg_autotune(plan.handle, level, n_samples, reps))


def mg_solve(plan: Plan, n: int, k, f, u, tol: float = 0.0, fixed_cycles: int = 0):
    """Returns (status, cycles, relres); status MG_OK or MG_ENOCONV, else raises."""
    N = n * n * n
    pk, pf, pu = _ptr(k, "float64", N, "k"), _ptr(f, "float64", N, "f"), _ptr(u, "float64", N, "u")
    mg_plan_set_stream(plan)
    cyc, rel = C.c_int(0), C.c_double(0.0)
    st = lib().mg_solve(plan.handle, n, pk, pf, pu, tol, fixed_cycles, C.byref(cyc), C.byref(rel))
    plan.check(st, (MG_OK, MG_ENOCONV))
    return st, cyc.value, rel.value


def mg_solve_noalloc(plan: Plan, n: int, k, f, u, tol: float = 0.0, fixed_cycles: int = 0):
    """mg_solve on the library's static device workspace (n <= 129); returns
    (status, cycles, relres) like mg_solve."""
    N = n * n * n
    pk, pf, pu = _ptr(k, "float64", N, "k"), _ptr(f, "float64", N, "f"), _ptr(u, "float64", N, "u")
    mg_plan_set_stream(plan)
    cyc, rel = C.c_int(0), C.c_double(0.0)
    st = lib().mg_solve_noalloc(plan.handle, n, pk, pf, pu, tol, fixed_cycles, C.byref(cyc),
                                C.byref(rel))
    plan.check(st, (MG_OK, MG_ENOCONV))
    return st, cyc.value, rel.value


def _seeds(seeds):
    a = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    return a, a.ctypes.data_as(C.POINTER(C.c_uint64))


def mlmc_sample_batch(plan: Plan, level: int, seeds, n: int, Y_out, Qf_out=None, Qc_out=None,
                      cycles_out=None, fixed_cycles: int = 0):
    """n samples of Y_level; returns MG_OK or MG_ENOCONV, raises otherwise."""
    arr, sp = _seeds(seeds)
    if arr.size < n:
        raise ValueError("need %d seeds" % n)
    py = _ptr(Y_out, "float64", n, "Y_out")
    pqf = _ptr(Qf_out, "float64", n, "Qf_out")
    pqc = _ptr(Qc_out, "float64", n, "Qc_out")
    pc = _ptr(cycles_out, "int32", 2 * n, "cycles_out")
    mg_plan_set_stream(plan)
    st = lib().mlmc_sample_batch(plan.handle, level, sp, n, py, pqf, pqc, pc, fixed_cycles)
    return plan.check(st, (MG_OK, MG_ENOCONV))


def mlmc_sample_mixed(plan: Plan, levels, seeds, n: int, Y_out, Qf_out=None, Qc_out=None,
                      cycles_out=None, fixed_cycles: int = 0):
    """n samples, sample i of level levels[i]; returns MG_OK or MG_ENOCONV."""
    lv = np.ascontiguousarray(np.asarray(levels, dtype=np.int32))
    arr, sp = _seeds(seeds)
    if arr.size < n or lv.size < n:
        raise ValueError("need %d seeds and levels" % n)
    py = _ptr(Y_out, "float64", n, "Y_out")
    pqf = _ptr(Qf_out, "float64", n, "Qf_out")
    pqc = _ptr(Qc_out, "float64", n, "Qc_out")
    pc = _ptr(cycles_out, "int32", 2 * n, "cycles_out")
    mg_plan_set_stream(plan)
    st = lib().mlmc_sample_mixed(plan.handle, lv.ctypes.data_as(C.POINTER(C.c_int)), sp, n, py,
                                 pqf, pqc, pc, fixed_cycles)
    return plan.check(st, (MG_OK, MG_ENOCONV))


def mlmc_philox(plan: Plan, seeds, n: int, level: int, words_out=None, normals_out=None):
    arr, sp = _seeds(seeds)
    pw = _ptr(words_out, "int32", 128 * n, "words_out") if words_out is not None and \
        str(words_out.dtype) == "torch.int32" else _ptr(words_out, "uint32", 128 * n, "words_out")
    pn = _ptr(normals_out, "float64", 64 * n, "normals_out")
    mg_plan_set_stream(plan)
    return plan.check(lib().mlmc_philox(plan.handle, sp, n, level, pw, pn))


def mlmc_philox_words(seed: int, level: int) -> np.ndarray:
    """The 128 Philox words of sample (seed, level), computed on the host."""
    out = np.zeros(128, dtype=np.uint32)
    st = lib().mlmc_philox_words(int(seed), int(level), out.ctypes.data_as(C.POINTER(C.c_uint32)))
    if st != MG_OK:
        raise MGError(st, "mlmc_philox_words rejected its arguments")
    return out


def mlmc_exp(x: float) -> float:
    """The exponential the kernels form the KL coefficient with (host evaluation)."""
    return lib().mlmc_exp(float(x))


def mlmc_field(plan: Plan, n: int, seed: int, level: int, k_out):
    pk = _ptr(k_out, "float64", n * n * n, "k_out")
    mg_plan_set_stream(plan)
    return plan.check(lib().mlmc_field(plan.handle, n, seed, level, pk))


def mlmc_adaptive(plan: Plan, eps: float, theta: float = 0.5, alpha: float = 2.0 / 3.0,
                  n_init: int = 32, max_iter: int = 64, max_batch: int = 256, seed0: int = 0):
    """Algorithm 2 on the plan's samples; returns a dict like the C result."""
    d = mlmc_adaptive_desc()
    lib().mlmc_adaptive_desc_default(C.byref(d))
    d.eps, d.theta, d.alpha = eps, theta, alpha
    d.n_init, d.max_iter, d.max_batch, d.seed0 = n_init, max_iter, max_batch, seed0
    r = mlmc_adaptive_result()
    mg_plan_set_stream(plan)
    plan.check(lib().mlmc_adaptive(plan.handle, C.byref(d), C.byref(r)))
    L = r.L
    return {"L": L, "N": [r.N[l] for l in range(L + 1)], "mean": [r.mean[l] for l in range(L + 1)],
            "var": [r.var[l] for l in range(L + 1)], "cost": [r.cost[l] for l in range(L + 1)],
            "Q": r.Q, "sampling_rms": r.sampling_rms, "bias_estimate": r.bias_estimate,
            "bias_ok": bool(r.bias_ok), "iterations": r.iterations,
            "trace": [(r.trace_L[t], [r.trace_N[t][l] for l in range(r.trace_L[t] + 1)])
                      for t in range(r.trace_len)]}


def mlmc_acc_init() -> mlmc_level_acc:
    a = mlmc_level_acc()
    lib().mlmc_acc_init(C.byref(a))
    return a


def mlmc_acc_add(acc: mlmc_level_acc, y):
    """y: CUDA float64 tensor or host array-like."""
    torch = None
    try:
        import torch as _t
        torch = _t
    except ImportError:
        pass
    if torch is not None and isinstance(y, torch.Tensor) and y.is_cuda:
        p = _ptr(y.contiguous(), "float64", None, "y")
        st = lib().mlmc_acc_add(C.byref(acc), p, y.numel(), 1)
    else:
        a = np.ascontiguousarray(np.asarray(y, dtype=np.float64).ravel())
        st = lib().mlmc_acc_add(C.byref(acc), C.c_void_p(a.ctypes.data), a.size, 0)
    if st != MG_OK:
        raise MGError(st, "mlmc_acc_add failed")


def mlmc_acc_result(acc: mlmc_level_acc):
    m, v = C.c_double(), C.c_double()
    lib().mlmc_acc_result(C.byref(acc), C.byref(m), C.byref(v))
    return m.value, v.value


def mg_profile_enable(plan: Plan, on: bool = True):
    return plan.check(lib().mg_profile_enable(plan.handle, 1 if on else 0))


def mg_profile_read(plan: Plan):
    """(launches, total_ms, nodes_per_launch) of the finest-grid smoothing launches."""
    n, ms, nodes = C.c_longlong(), C.c_double(), C.c_double()
    plan.check(lib().mg_profile_read(plan.handle, C.byref(n), C.byref(ms), C.byref(nodes)))
    return n.value, ms.value, nodes.value


def mg_profile_records(plan: Plan):
    """Per timed sweep: (cycle, kind, grid_n, ms) arrays (see mg_profile_records)."""
    n = C.c_int()
    plan.check(lib().mg_profile_records(plan.handle, 0, None, None, None, None, C.byref(n)))
    m = n.value
    cyc, kind = np.zeros(m, dtype=np.int32), np.zeros(m, dtype=np.int32)
    gn, ms = np.zeros(m, dtype=np.int32), np.zeros(m)
    plan.check(lib().mg_profile_records(plan.handle, m, cyc.ctypes.data_as(C.POINTER(C.c_int)),
                                        kind.ctypes.data_as(C.POINTER(C.c_int)),
                                        gn.ctypes.data_as(C.POINTER(C.c_int)),
                                        ms.ctypes.data_as(C.POINTER(C.c_double)), C.byref(n)))
    return cyc, kind, gn, ms


# ---- serving -------------------------------------------------------------------

def mg_sample_footprint(plan: Plan, level: int) -> int:
    b = C.c_size_t()
    plan.check(lib().mg_sample_footprint(plan.handle, level, C.byref(b)))
    return b.value


class Sched:
    """Admission scheduler (host only): mg_sched_* on one handle.  Level l is
    served in lanes of lane_slots[l] slots costing lane_bytes[l] bytes; the
    open lanes share `budget` bytes."""

    def __init__(self, lane_slots, lane_bytes, budget, queue_capacity=1 << 16):
        a = np.ascontiguousarray(np.asarray(lane_slots, dtype=np.int32))
        b = np.ascontiguousarray(np.asarray(lane_bytes, dtype=np.uint64))
        if a.size != b.size:
            raise ValueError("lane_slots and lane_bytes need one entry per level")
        h = C.c_void_p()
        st = lib().mg_sched_create(int(a.size), a.ctypes.data_as(C.POINTER(C.c_int)),
                                   b.ctypes.data_as(C.POINTER(C.c_size_t)), int(budget),
                                   int(queue_capacity), C.byref(h))
        if st != MG_OK:
            raise MGError(st, "mg_sched_create rejected its arguments")
        self.handle = h

    def submit(self, level, seed, tag, t_arrival=0.0):
        """Returns the status (MG_OK, MG_EBUSY, MG_ENOMEM or MG_EINVAL)."""
        return lib().mg_sched_submit(self.handle, int(level), int(seed), int(tag), float(t_arrival))

    def admit(self, max_out=1024):
        """Tickets (tag, seed, level, slot, lane, t_arrival) of one pass."""
        buf = (mg_ticket * max(1, max_out))()
        n = C.c_int()
        st = lib().mg_sched_admit(self.handle, buf, max_out, C.byref(n))
        if st != MG_OK:
            raise MGError(st, "mg_sched_admit")
        return [(buf[i].tag, buf[i].seed, buf[i].level, buf[i].slot, buf[i].lane, buf[i].t_arrival)
                for i in range(n.value)]

    def events(self, max_out=1024):
        """Pending lane events (kind, lane, level, first, nslots, bytes)."""
        buf = (mg_lane_event * max_out)()
        n = C.c_int()
        st = lib().mg_sched_events(self.handle, buf, max_out, C.byref(n))
        if st != MG_OK:
            raise MGError(st, "mg_sched_events")
        return [(buf[i].kind, buf[i].lane, buf[i].level, buf[i].first, buf[i].nslots, buf[i].bytes)
                for i in range(n.value)]

    def set_inflight(self, lane, inflight):
        return lib().mg_sched_set_inflight(self.handle, int(lane), int(bool(inflight)))

    def release(self, slot):
        return lib().mg_sched_release(self.handle, int(slot))

    def counts(self):
        q, b = C.c_int(), C.c_int()
        lib().mg_sched_counts(self.handle, C.byref(q), C.byref(b))
        return q.value, b.value

    def memory(self):
        """(bytes of the open lanes, their maximum so far, open lanes)."""
        u, p, n = C.c_size_t(), C.c_size_t(), C.c_int()
        lib().mg_sched_memory(self.handle, C.byref(u), C.byref(p), C.byref(n))
        return u.value, p.value, n.value

    def __del__(self):
        try:
            if self.handle:
                lib().mg_sched_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


class Server:
    """Serving handle (mg_serve_*): continuous batching on one plan."""

    def __init__(self, plan: Plan, lane_slots=None, queue_capacity=1 << 16):
        self.plan = plan
        h = C.c_void_p()
        if lane_slots is None:
            p = None
        else:
            self._slots = np.ascontiguousarray(np.asarray(lane_slots, dtype=np.int32))
            if self._slots.size != plan.desc.max_level + 1:
                raise ValueError("lane_slots needs max_level + 1 entries")
            p = self._slots.ctypes.data_as(C.POINTER(C.c_int))
        plan.check(lib().mg_serve_create(plan.handle, p, int(queue_capacity), C.byref(h)))
        self.handle = h

    def submit(self, level, seed, tag, t_arrival=-1.0):
        """Returns MG_OK or MG_EBUSY (queue full); raises on bad arguments and
        on a level that is not served."""
        st = lib().mg_serve_submit(self.handle, int(level), int(seed), int(tag), float(t_arrival))
        return self.plan.check(st, (MG_OK, MG_EBUSY))

    def step(self, cycles=1, max_out=4096):
        """One scheduling step; returns the finished samples as dicts."""
        buf = (mg_result * max_out)()
        n = C.c_int()
        self.plan.check(lib().mg_serve_step(self.handle, int(cycles), buf, max_out, C.byref(n)))
        out = []
        for i in range(n.value):
            r = buf[i]
            out.append({"tag": r.tag, "seed": r.seed, "level": r.level, "status": r.status,
                        "Y": r.Y, "Qf": r.Qf, "Qc": r.Qc, "cycles": (r.cycles_fine, r.cycles_coarse),
                        "t_arrival": r.t_arrival, "t_admit": r.t_admit, "t_done": r.t_done})
        return out

    def now(self):
        return lib().mg_serve_now(self.handle)

    def counts(self):
        q, r, c = C.c_int(), C.c_int(), C.c_longlong()
        lib().mg_serve_counts(self.handle, C.byref(q), C.byref(r), C.byref(c))
        return q.value, r.value, c.value

    def slots(self, level):
        """Slots per lane of a level."""
        return lib().mg_serve_slots(self.handle, int(level))

    def memory(self):
        """Dict: used, peak and budget bytes, open lanes, lanes opened and
        evicted, host seconds spent opening and evicting lanes."""
        u, p, b = C.c_size_t(), C.c_size_t(), C.c_size_t()
        n, o, e, t = C.c_int(), C.c_longlong(), C.c_longlong(), C.c_double()
        lib().mg_serve_memory(self.handle, C.byref(u), C.byref(p), C.byref(b), C.byref(n),
                              C.byref(o), C.byref(e), C.byref(t))
        return {"used": u.value, "peak": p.value, "budget": b.value, "lanes": n.value,
                "opened": o.value, "evicted": e.value, "lane_seconds": t.value}

    def destroy(self):
        if getattr(self, "handle", None):
            lib().mg_serve_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def mg_serve_create(plan: Plan, lane_slots=None, queue_capacity=1 << 16) -> Server:
    return Server(plan, lane_slots, queue_capacity)
