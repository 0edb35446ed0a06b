"""ctypes binding of the C ABI in include/pdcs.h (argument marshalling only).

Every compute step runs inside libpdcs.so.  Importing this module loads the
library and fails loudly when it has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdcs.so")

PDCS_OK = 0
ERRORS = {-1: "invalid argument", -2: "unsupported", -3: "out of memory", -4: "HIP error",
          -5: "size", -6: "state"}
EXIT_OPTIMAL, EXIT_MAX_ITER, EXIT_TIME_LIMIT, EXIT_CONTINUE, EXIT_NUMERICAL_ERROR = 0, 1, 6, 7, 8
EXIT_PRIMAL_INFEASIBLE_LOW_ACC, EXIT_PRIMAL_INFEASIBLE_HIGH_ACC = 2, 3
EXIT_DUAL_INFEASIBLE_LOW_ACC, EXIT_DUAL_INFEASIBLE_HIGH_ACC = 4, 5
METHOD = {"auto": 0, "average": 1, "halpern": 2}
PRECISION = {"fp64": 0, "mixed": 1}


class PdcsError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({detail})")
        self.code = code


class pdcs_options(C.Structure):
    _fields_ = [("rel_tol", C.c_double), ("abs_tol", C.c_double), ("time_limit", C.c_double),
                ("max_iter", C.c_int64), ("use_preconditioner", C.c_int64), ("ruiz_iters", C.c_int64),
                ("l2_pass", C.c_int64), ("method", C.c_int64), ("check_every", C.c_int64),
                ("precision", C.c_int64), ("stall_checks", C.c_int64),
                ("polish_switch_tol", C.c_double), ("bisect_rel_eps", C.c_double),
                ("use_graph", C.c_int64), ("verbose", C.c_int64), ("keep_state", C.c_int64),
                ("time_kernels", C.c_int64), ("probe_passes", C.c_int64),
                ("trace_trials", C.c_int64), ("compact", C.c_int64), ("use_kkt_restart", C.c_int64),
                ("use_duality_gap_restart", C.c_int64), ("kkt_restart_freq", C.c_int64),
                ("duality_gap_restart_freq", C.c_int64), ("print_freq", C.c_int64),
                ("eps_primal_infeasible_low_acc", C.c_double), ("eps_dual_infeasible_low_acc", C.c_double),
                ("eps_primal_infeasible_high_acc", C.c_double), ("eps_dual_infeasible_high_acc", C.c_double),
                ("reserved", C.c_int64 * 4)]


class pdcs_info(C.Structure):
    _fields_ = [("exit_code", C.c_int64), ("iters", C.c_int64), ("accepted_iters", C.c_int64),
                ("restarts", C.c_int64), ("checks", C.c_int64), ("fp64_iters", C.c_int64),
                ("pobj", C.c_double), ("dobj", C.c_double), ("abs_p", C.c_double),
                ("abs_d", C.c_double), ("abs_gap", C.c_double), ("rel_p", C.c_double),
                ("rel_d", C.c_double), ("rel_gap", C.c_double), ("time_sec", C.c_double),
                ("omega", C.c_double), ("eta_hat", C.c_double), ("spmv_avg_ms", C.c_double),
                ("spmv_launches", C.c_int64), ("reserved", C.c_double * 4)]


class pdcs_state_scalars(C.Structure):
    _fields_ = [("omega", C.c_double), ("omega0", C.c_double), ("eta_hat", C.c_double),
                ("eta", C.c_double), ("beta", C.c_double), ("sum_eta", C.c_double),
                ("kbar", C.c_int64), ("k", C.c_int64), ("t", C.c_int64), ("accepted", C.c_int64),
                ("precision", C.c_int64), ("rho_cur", C.c_double), ("rho_avg", C.c_double),
                ("r_cur", C.c_double), ("r_avg", C.c_double), ("chosen", C.c_int64),
                ("ratio_p", C.c_double), ("ratio_d", C.c_double), ("trend_p", C.c_int64),
                ("trend_d", C.c_int64)]


_P = C.c_void_p
_DP = C.POINTER(C.c_double)
_I64 = C.c_int64

# name -> (restype, argtypes)
PROTOTYPES = {
    "pdcs_options_default": (None, [C.POINTER(pdcs_options)]),
    "pdcs_status_string": (C.c_char_p, [C.c_int]),
    "pdcs_last_error": (C.c_char_p, []),
    "pdcs_device_count": (C.c_int, []),
    "pdcs_problem_create": (C.c_int, [_I64, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, C.POINTER(_P)]),
    "pdcs_problem_create_conic": (C.c_int, [_I64, _I64, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P, C.POINTER(_P)]),
    "pdcs_problem_create_cones": (C.c_int, [_I64, _I64, _I64, _I64, _P, _I64, _I64, _P, _P, _P, _P, _P, _P, _P,
                                            C.POINTER(_P)]),
    "pdcs_project_cone": (C.c_int, [_I64, _I64, _I64, _P, _P, _P, _P]),
    "pdcs_problem_destroy": (None, [_P]),
    "pdcs_problem_dims": (C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64)]),
    "pdcs_problem_spmv": (C.c_int, [_P, _I64, _I64, _P, _P, _P]),
    "pdcs_problem_spmv_noalloc": (C.c_int, [_P, _I64, _I64, _P, _P, _P]),
    "pdcs_problem_set_layout": (C.c_int, [_P, _I64]),
    "pdcs_problem_set_band_schedule": (C.c_int, [_P, _I64, _I64, _I64]),
    "pdcs_problem_band_schedule": (C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64),
                                             C.POINTER(_I64), C.POINTER(_I64)]),
    "pdcs_batch_set_band_schedule": (C.c_int, [_P, _I64, _I64, _I64]),
    "pdcs_batch_band_schedule": (C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64),
                                           C.POINTER(_I64), C.POINTER(_I64)]),
    "pdcs_solve": (C.c_int, [_P, C.POINTER(pdcs_options), _P, _P, _P, C.POINTER(_P)]),
    "pdcs_solve_device": (C.c_int, [_P, C.POINTER(pdcs_options), _P, _P, _I64, _P, C.POINTER(_P)]),
    "pdcs_result_info": (C.c_int, [_P, C.POINTER(pdcs_info)]),
    "pdcs_result_primal": (C.c_int, [_P, _P, _I64]),
    "pdcs_result_dual": (C.c_int, [_P, _P, _I64]),
    "pdcs_result_slack": (C.c_int, [_P, _P, _I64]),
    "pdcs_result_primal_device": (C.c_int, [_P, _P, _I64, _P]),
    "pdcs_result_dual_device": (C.c_int, [_P, _P, _I64, _P]),
    "pdcs_result_slack_device": (C.c_int, [_P, _P, _I64, _P]),
    "pdcs_result_scaling": (C.c_int, [_P, _P, _I64, _P, _I64]),
    "pdcs_result_state": (C.c_int, [_P, C.POINTER(pdcs_state_scalars), _P, _P, _P, _P, _P, _P]),
    "pdcs_result_products": (C.c_int, [_P, _P, _P]),
    "pdcs_result_trace": (C.c_int, [_P, _P, _I64, C.POINTER(_I64)]),
    "pdcs_result_destroy": (None, [_P]),
    "pdcs_batch_create": (C.c_int, [_I64, _P, C.POINTER(_P)]),
    "pdcs_batch_solve": (C.c_int, [_P, C.POINTER(pdcs_options), _P, _P, _P, _P]),
    "pdcs_batch_solve_device": (C.c_int, [_P, C.POINTER(pdcs_options), _P, _P, _I64, _P, _P]),
    "pdcs_batch_autotune": (C.c_int, [_P, C.c_double]),
    "pdcs_batch_schedule": (C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64)]),
    "pdcs_batch_set_schedule": (C.c_int, [_P, _I64, _I64, _I64]),
    "pdcs_batch_set_layout": (C.c_int, [_P, _I64]),
    "pdcs_batch_destroy": (None, [_P]),
    "pdcs_mlp_create": (C.c_int, [_I64, _I64, _I64, C.c_uint64, C.POINTER(_P)]),
    "pdcs_mlp_forward": (C.c_int, [_P, _P, _P, _I64, _P]),
    "pdcs_mlp_train_step": (C.c_int, [_P, _P, _P, _I64, C.c_float, C.POINTER(C.c_float), _P]),
    "pdcs_mlp_gradients": (C.c_int, [_P, _P, _P, _I64, _P, C.POINTER(C.c_float), _P]),
    "pdcs_mlp_activation": (C.c_int, [_P, _I64, _P, _I64]),
    "pdcs_mlp_set_normalization": (C.c_int, [_P, _P, _P, _P, _P]),
    "pdcs_mlp_num_params": (C.c_int, [_P, C.POINTER(_I64)]),
    "pdcs_mlp_get_params": (C.c_int, [_P, _P]),
    "pdcs_mlp_set_params": (C.c_int, [_P, _P]),
    "pdcs_mlp_destroy": (None, [_P]),
}


def _bind_hip_runtime_of_torch():
    """torch ships its own libamdhip64.so.7 (same soname as /opt/rocm's).  Two
    HIP runtimes cannot share a process, so when torch is importable it is
    loaded first and libpdcs.so binds to the runtime torch already holds."""
    try:
        import torch  # noqa: F401
    except Exception:
        pass


def load_library(path: str = LIB_PATH) -> C.CDLL:
    _bind_hip_runtime_of_torch()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python paper_2603_15504_amd/build.py` "
                          "(there is no CPU fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        try:
            fn = getattr(lib, name)
        except AttributeError:
            MISSING.append(name)
            continue
        fn.restype = res
        fn.argtypes = args
    return lib


MISSING: list[str] = []


lib = load_library()


def _check(code: int, where: str):
    if code != PDCS_OK:
        raise PdcsError(code, where, lib.pdcs_last_error().decode(errors="replace"))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a, n=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} entries, got {a.size}")
    return a


# ---------------------------------------------------------------------------
# Same-name wrappers (marshalling only)
# ---------------------------------------------------------------------------
def pdcs_options_default(**overrides) -> pdcs_options:
    o = pdcs_options()
    lib.pdcs_options_default(C.byref(o))
    for k, v in overrides.items():
        if k == "method" and isinstance(v, str):
            v = METHOD[v]
        if k == "precision" and isinstance(v, str):
            v = PRECISION[v]
        if not hasattr(o, k):
            raise KeyError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def pdcs_status_string(code: int) -> str:
    return lib.pdcs_status_string(int(code)).decode()


def pdcs_device_count() -> int:
    return int(lib.pdcs_device_count())


def pdcs_problem_create(m, n, m_zero, row_ptr, col_idx, val, h, c, l=None, u=None) -> C.c_void_p:
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    val = _f64(val)
    h = _f64(h, m) if m > 0 else np.zeros(1)
    c = _f64(c, n)
    l = _f64(l, n)
    u = _f64(u, n)
    out = C.c_void_p()
    _check(lib.pdcs_problem_create(int(m), int(n), int(m_zero), _ptr(row_ptr), _ptr(col_idx), _ptr(val),
                                   _ptr(h), _ptr(c), _ptr(l), _ptr(u), C.byref(out)),
           "pdcs_problem_create")
    return out


def pdcs_problem_create_conic(m, n, m_zero, soc_dims, row_ptr, col_idx, val, h, c, l=None, u=None) -> C.c_void_p:
    soc = np.ascontiguousarray(np.asarray(soc_dims, dtype=np.int64).reshape(-1))
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    val = _f64(val)
    h = _f64(h, m) if m > 0 else np.zeros(1)
    c = _f64(c, n)
    l = _f64(l, n)
    u = _f64(u, n)
    out = C.c_void_p()
    _check(lib.pdcs_problem_create_conic(int(m), int(n), int(m_zero), int(soc.size), _ptr(soc) if soc.size else None,
                                         _ptr(row_ptr), _ptr(col_idx), _ptr(val), _ptr(h), _ptr(c), _ptr(l),
                                         _ptr(u), C.byref(out)),
           "pdcs_problem_create_conic")
    return out


def pdcs_problem_create_cones(m, n, m_zero, soc_dims, n_exp, n_dexp, row_ptr, col_idx, val, h, c, l=None,
                              u=None) -> C.c_void_p:
    soc = np.ascontiguousarray(np.asarray(soc_dims, dtype=np.int64).reshape(-1))
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    val = _f64(val)
    h = _f64(h, m) if m > 0 else np.zeros(1)
    c = _f64(c, n)
    l = _f64(l, n)
    u = _f64(u, n)
    out = C.c_void_p()
    _check(lib.pdcs_problem_create_cones(int(m), int(n), int(m_zero), int(soc.size), _ptr(soc) if soc.size else None,
                                         int(n_exp), int(n_dexp), _ptr(row_ptr), _ptr(col_idx), _ptr(val), _ptr(h),
                                         _ptr(c), _ptr(l), _ptr(u), C.byref(out)),
           "pdcs_problem_create_cones")
    return out


CONES = {"soc": 0, "exp": 1, "exp_dual": 2}


def pdcs_project_cone(cone, v, f, timed=False):
    """Projections of the rows of v (count x dim) onto diag(f_q) K, K named by
    cone ("soc", "exp" or "exp_dual"; dim 3 for the exponential cones), on the
    current GPU; with timed, also the kernel's duration in ms."""
    v = np.asarray(v, dtype=np.float64)
    v = np.ascontiguousarray(v.reshape(-1, v.shape[-1] if v.ndim > 1 else v.size))
    f = np.ascontiguousarray(np.broadcast_to(np.asarray(f, dtype=np.float64), v.shape))
    out = np.empty_like(v)
    ms = C.c_double(0.0)
    _check(lib.pdcs_project_cone(CONES[cone], int(v.shape[1]), int(v.shape[0]), _ptr(v), _ptr(f), _ptr(out),
                                 C.byref(ms) if timed else None), "pdcs_project_cone")
    return (out, ms.value) if timed else out


def pdcs_problem_destroy(p):
    lib.pdcs_problem_destroy(p)


def pdcs_problem_dims(p):
    m, n, z = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib.pdcs_problem_dims(p, C.byref(m), C.byref(n), C.byref(z)), "pdcs_problem_dims")
    return m.value, n.value, z.value


def pdcs_problem_spmv(p, transpose: int, precision: int, in_dev: int, out_dev: int, stream: int = 0):
    _check(lib.pdcs_problem_spmv(p, int(transpose), int(precision), C.c_void_p(in_dev),
                                 C.c_void_p(out_dev), C.c_void_p(stream) if stream else None),
           "pdcs_problem_spmv")


def pdcs_problem_spmv_noalloc(p, transpose: int, precision: int, in_dev: int, out_dev: int, stream: int = 0):
    _check(lib.pdcs_problem_spmv_noalloc(p, int(transpose), int(precision), C.c_void_p(in_dev),
                                         C.c_void_p(out_dev), C.c_void_p(stream) if stream else None),
           "pdcs_problem_spmv_noalloc")


LAYOUTS = {"auto": 0, "rows": 1, "bands": 2, "workgroup": 3}


def pdcs_problem_set_layout(p, layout: int):
    _check(lib.pdcs_problem_set_layout(p, int(layout)), "pdcs_problem_set_layout")


def pdcs_problem_set_band_schedule(p, rows: int, min_tiles: int, entry_cap: int):
    _check(lib.pdcs_problem_set_band_schedule(p, int(rows), int(min_tiles), int(entry_cap)),
           "pdcs_problem_set_band_schedule")


def _band_schedule(fn, h, name):
    v = [C.c_int64() for _ in range(5)]
    _check(fn(h, *[C.byref(x) for x in v]), name)
    return dict(rows=v[0].value, min_tiles=v[1].value, entry_cap=v[2].value, built_rows=v[3].value,
                windows=v[4].value)


def pdcs_problem_band_schedule(p) -> dict:
    return _band_schedule(lib.pdcs_problem_band_schedule, p, "pdcs_problem_band_schedule")


def pdcs_batch_set_band_schedule(b, rows: int, min_tiles: int, entry_cap: int):
    _check(lib.pdcs_batch_set_band_schedule(b, int(rows), int(min_tiles), int(entry_cap)),
           "pdcs_batch_set_band_schedule")


def pdcs_batch_band_schedule(b) -> dict:
    return _band_schedule(lib.pdcs_batch_band_schedule, b, "pdcs_batch_band_schedule")


def pdcs_solve(p, opts: pdcs_options | None = None, x0=None, y0=None, stream: int = 0) -> C.c_void_p:
    m, n, _ = pdcs_problem_dims(p)
    x0 = _f64(x0, n)
    y0 = _f64(y0, m)
    out = C.c_void_p()
    _check(lib.pdcs_solve(p, C.byref(opts) if opts is not None else None, _ptr(x0), _ptr(y0),
                          C.c_void_p(stream) if stream else None, C.byref(out)), "pdcs_solve")
    return out


def pdcs_solve_device(p, opts: pdcs_options | None, x0_dev: int, y0_dev: int, warm_dtype: int,
                      stream: int = 0) -> C.c_void_p:
    """Warm start from device pointers (0 = none); warm_dtype 0 = FP64, 1 = FP32."""
    out = C.c_void_p()
    _check(lib.pdcs_solve_device(p, C.byref(opts) if opts is not None else None,
                                 C.c_void_p(x0_dev) if x0_dev else None, C.c_void_p(y0_dev) if y0_dev else None,
                                 int(warm_dtype), C.c_void_p(stream) if stream else None, C.byref(out)),
           "pdcs_solve_device")
    return out


def pdcs_result_info(r) -> pdcs_info:
    info = pdcs_info()
    _check(lib.pdcs_result_info(r, C.byref(info)), "pdcs_result_info")
    return info


def _get_vec(fn, r, length, name):
    out = np.empty(length, dtype=np.float64)
    _check(fn(r, _ptr(out), int(length)), name)
    return out


def pdcs_result_primal(r, n):
    return _get_vec(lib.pdcs_result_primal, r, n, "pdcs_result_primal")


def pdcs_result_dual(r, m):
    return _get_vec(lib.pdcs_result_dual, r, m, "pdcs_result_dual")


def pdcs_result_slack(r, n):
    return _get_vec(lib.pdcs_result_slack, r, n, "pdcs_result_slack")


def pdcs_result_primal_device(r, x_dev: int, n: int, stream: int = 0):
    _check(lib.pdcs_result_primal_device(r, C.c_void_p(x_dev), int(n), C.c_void_p(stream) if stream else None),
           "pdcs_result_primal_device")


def pdcs_result_dual_device(r, y_dev: int, m: int, stream: int = 0):
    _check(lib.pdcs_result_dual_device(r, C.c_void_p(y_dev) if y_dev else None, int(m),
                                       C.c_void_p(stream) if stream else None), "pdcs_result_dual_device")


def pdcs_result_slack_device(r, lam_dev: int, n: int, stream: int = 0):
    _check(lib.pdcs_result_slack_device(r, C.c_void_p(lam_dev), int(n), C.c_void_p(stream) if stream else None),
           "pdcs_result_slack_device")


def pdcs_result_scaling(r, m, n):
    D1 = np.empty(m, dtype=np.float64)
    D2 = np.empty(n, dtype=np.float64)
    _check(lib.pdcs_result_scaling(r, _ptr(D1), m, _ptr(D2), n), "pdcs_result_scaling")
    return D1, D2


def pdcs_result_state(r, m, n, vectors: bool = True):
    s = pdcs_state_scalars()
    if not vectors:
        _check(lib.pdcs_result_state(r, C.byref(s), None, None, None, None, None, None), "pdcs_result_state")
        return s, None
    vec = {k: np.empty(n if k.startswith("x") else m) for k in ("x", "y", "x_hat", "y_hat", "x_a", "y_a")}
    _check(lib.pdcs_result_state(r, C.byref(s), _ptr(vec["x"]), _ptr(vec["y"]), _ptr(vec["x_hat"]),
                                 _ptr(vec["y_hat"]), _ptr(vec["x_a"]), _ptr(vec["y_a"])),
           "pdcs_result_state")
    return s, vec


TRACE_FIELDS = ("kbar", "eta", "eta_bar", "dx2", "dy2", "dydgdx", "accepted", "eta_next", "beta", "k",
                "pobj", "hy", "l_lam_plus", "u_lam_minus", "errp2", "errd2")


def pdcs_result_trace(r, max_trials: int) -> np.ndarray:
    out = np.empty((max(int(max_trials), 1), len(TRACE_FIELDS)), dtype=np.float64)
    cnt = C.c_int64()
    _check(lib.pdcs_result_trace(r, _ptr(out), int(max_trials), C.byref(cnt)), "pdcs_result_trace")
    return out[:cnt.value]


def pdcs_result_destroy(r):
    lib.pdcs_result_destroy(r)


def pdcs_batch_create(problems) -> C.c_void_p:
    arr = (C.c_void_p * len(problems))(*[p.value if isinstance(p, C.c_void_p) else p for p in problems])
    out = C.c_void_p()
    _check(lib.pdcs_batch_create(len(problems), C.cast(arr, C.c_void_p), C.byref(out)), "pdcs_batch_create")
    return out


def pdcs_batch_solve(b, count, opts=None, x0s=None, y0s=None, stream: int = 0, dims=None):
    """dims: the (m, n) of every instance; each warm-start entry must have n (x)
    or m (y) values, since the library reads exactly that many."""
    keep = []
    if dims is None:
        raise ValueError("pdcs_batch_solve needs the (m, n) of every instance")
    if len(dims) != count:
        raise ValueError(f"expected {count} instance sizes, got {len(dims)}")

    def ptr_array(vs, side):
        if vs is None:
            return None
        if len(vs) != count:
            raise ValueError(f"expected {count} warm-start entries, got {len(vs)}")
        arr = (C.c_void_p * count)()
        for i, v in enumerate(vs):
            if v is not None:
                a = _f64(v, dims[i][side])
                keep.append(a)
                arr[i] = a.ctypes.data
        keep.append(arr)
        return C.cast(arr, C.c_void_p)

    res = (C.c_void_p * count)()
    _check(lib.pdcs_batch_solve(b, C.byref(opts) if opts is not None else None, ptr_array(x0s, 1),
                                ptr_array(y0s, 0), C.c_void_p(stream) if stream else None,
                                C.cast(res, C.c_void_p)), "pdcs_batch_solve")
    return [C.c_void_p(res[i]) for i in range(count)]


def pdcs_batch_solve_device(b, count, opts, x0s_dev, y0s_dev, warm_dtype: int, stream: int = 0):
    """x0s_dev / y0s_dev: None or `count` device addresses (0 = no warm start for that instance)."""
    def ptr_array(vs):
        if vs is None:
            return None
        if len(vs) != count:
            raise ValueError(f"expected {count} warm-start pointers, got {len(vs)}")
        return (C.c_void_p * count)(*[int(v) if v else None for v in vs])

    xa, ya = ptr_array(x0s_dev), ptr_array(y0s_dev)
    res = (C.c_void_p * count)()
    _check(lib.pdcs_batch_solve_device(b, C.byref(opts) if opts is not None else None,
                                       C.cast(xa, C.c_void_p) if xa is not None else None,
                                       C.cast(ya, C.c_void_p) if ya is not None else None, int(warm_dtype),
                                       C.c_void_p(stream) if stream else None, C.cast(res, C.c_void_p)),
           "pdcs_batch_solve_device")
    return [C.c_void_p(res[i]) for i in range(count)]


def pdcs_batch_set_layout(b, layout: int):
    _check(lib.pdcs_batch_set_layout(b, int(layout)), "pdcs_batch_set_layout")


def pdcs_batch_autotune(b, time_budget_ms: float = 0.0):
    _check(lib.pdcs_batch_autotune(b, float(time_budget_ms)), "pdcs_batch_autotune")


def pdcs_batch_schedule(b):
    a, bb, c = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib.pdcs_batch_schedule(b, C.byref(a), C.byref(bb), C.byref(c)), "pdcs_batch_schedule")
    return a.value, bb.value, c.value


def pdcs_batch_set_schedule(b, iter_max, block_nnz, vec_per_block):
    _check(lib.pdcs_batch_set_schedule(b, int(iter_max), int(block_nnz), int(vec_per_block)),
           "pdcs_batch_set_schedule")


def pdcs_batch_destroy(b):
    lib.pdcs_batch_destroy(b)


# ---------------------------------------------------------------------------
# Convenience layer (still marshalling only)
# ---------------------------------------------------------------------------
@dataclass
class Solution:
    x: np.ndarray
    y: np.ndarray
    lam: np.ndarray
    info: dict
    D1: np.ndarray | None = None
    D2: np.ndarray | None = None
    state: dict | None = None
    trace: np.ndarray | None = None


def _info_dict(info: pdcs_info) -> dict:
    d = {name: getattr(info, name) for name, _ in pdcs_info._fields_ if name != "reserved"}
    d["status"] = pdcs_status_string(d["exit_code"])
    return d


class Problem:
    """An LP uploaded to the GPU (pdcs_problem)."""

    def __init__(self, m, n, m_zero, row_ptr, col_idx, val, h, c, l=None, u=None, soc=(), n_exp=0, n_dexp=0):
        """soc: dimensions of second-order-cone row blocks, then n_exp exponential
        and n_dexp dual-exponential blocks of 3 rows (the last rows)."""
        self.m, self.n = int(m), int(n)
        if n_exp or n_dexp:
            self.handle = pdcs_problem_create_cones(m, n, m_zero, soc, n_exp, n_dexp, row_ptr, col_idx, val, h, c,
                                                    l, u)
        elif len(soc):
            self.handle = pdcs_problem_create_conic(m, n, m_zero, soc, row_ptr, col_idx, val, h, c, l, u)
        else:
            self.handle = pdcs_problem_create(m, n, m_zero, row_ptr, col_idx, val, h, c, l, u)

    @classmethod
    def from_instance(cls, inst):
        return cls(inst.m, inst.n, inst.m_zero, inst.row_ptr, inst.col_idx, inst.val, inst.h, inst.c,
                   inst.l, inst.u, getattr(inst, "soc", ()), getattr(inst, "n_exp", 0), getattr(inst, "n_dexp", 0))

    def solve(self, x0=None, y0=None, with_scaling=False, device_out=False, **opts) -> Solution:
        """Host warm start (arrays) or, for torch tensors on the GPU, the device
        warm-start call (float64 or float32, read on torch's current stream).
        device_out=True returns x, y, lam as float64 torch tensors filled by the
        device-pointer result calls."""
        o = pdcs_options_default(**opts)
        dev = _is_device_tensor(x0) or _is_device_tensor(y0)
        if dev:
            dtype = _warm_dtype(x0, y0, {"x0": (x0, self.n), "y0": (y0, self.m)})
            r = pdcs_solve_device(self.handle, o, _dev_ptr(x0), _dev_ptr(y0), dtype, _torch_stream())
        else:
            r = pdcs_solve(self.handle, o, x0, y0)
        try:
            return _collect(r, self.m, self.n, with_scaling, bool(o.keep_state), int(o.trace_trials),
                            device_out=device_out)
        finally:
            pdcs_result_destroy(r)

    def set_layout(self, layout="auto"):
        """Matrix storage for the trial SpMVs: "auto", "rows", "bands" or "workgroup"."""
        pdcs_problem_set_layout(self.handle, LAYOUTS[layout] if isinstance(layout, str) else layout)

    def set_band_schedule(self, rows=8192, min_tiles=384, entry_cap=32768):
        pdcs_problem_set_band_schedule(self.handle, rows, min_tiles, entry_cap)

    def band_schedule(self) -> dict:
        return pdcs_problem_band_schedule(self.handle)

    def spmv(self, x_dev, out_dev, transpose=False, precision="fp64", stream=0):
        pdcs_problem_spmv(self.handle, 1 if transpose else 0, PRECISION[precision], x_dev, out_dev, stream)

    def close(self):
        if getattr(self, "handle", None):
            pdcs_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _is_device_tensor(a) -> bool:
    return a is not None and hasattr(a, "is_cuda") and bool(a.is_cuda)


def _dev_ptr(a) -> int:
    return 0 if a is None else int(a.data_ptr())


def _torch_stream() -> int:
    import torch

    return int(torch.cuda.current_stream().cuda_stream)


def _warm_dtype(x0, y0, want) -> int:
    """Check the device warm-start tensors (contiguous, one dtype, right length)
    and return the dtype code of the C ABI (0: float64, 1: float32)."""
    import torch

    codes = set()
    for name, (t, length) in want.items():
        if t is None:
            continue
        if not _is_device_tensor(t) or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous GPU tensor when the other one is")
        if t.numel() != length:
            raise ValueError(f"{name}: expected {length} entries, got {t.numel()}")
        if t.dtype == torch.float64:
            codes.add(0)
        elif t.dtype == torch.float32:
            codes.add(1)
        else:
            raise ValueError(f"{name} must be float64 or float32, got {t.dtype}")
    if len(codes) != 1:
        raise ValueError("x0 and y0 must share one dtype")
    return codes.pop()


def _device_vectors(r, m, n):
    import torch

    x = torch.empty(n, dtype=torch.float64, device="cuda")
    y = torch.empty(m, dtype=torch.float64, device="cuda")
    lam = torch.empty(n, dtype=torch.float64, device="cuda")
    st = _torch_stream()
    pdcs_result_primal_device(r, x.data_ptr(), n, st)
    pdcs_result_dual_device(r, y.data_ptr() if m > 0 else 0, m, st)
    pdcs_result_slack_device(r, lam.data_ptr(), n, st)
    # the copies are enqueued on torch's stream; the result handle is destroyed
    # right after, so wait for them here
    torch.cuda.current_stream().synchronize()
    return x, y, lam


def _collect(r, m, n, with_scaling, with_state, trace=0, device_out=False) -> Solution:
    info = _info_dict(pdcs_result_info(r))
    if device_out:
        sol = Solution(*_device_vectors(r, m, n), info)
    else:
        sol = Solution(pdcs_result_primal(r, n), pdcs_result_dual(r, m) if m > 0 else np.zeros(0),
                       pdcs_result_slack(r, n), info)
    if with_scaling:
        sol.D1, sol.D2 = pdcs_result_scaling(r, m, n)
    if with_state:
        s, vec = pdcs_result_state(r, m, n, True)
        st = {name: getattr(s, name) for name, _ in pdcs_state_scalars._fields_ if name != "reserved"}
        st.update(vec)
        gty = np.empty(n)
        gx = np.empty(m)
        _check(lib.pdcs_result_products(r, _ptr(gty), _ptr(gx)), "pdcs_result_products")
        st["gty_hat"] = gty
        st["gx_hat"] = gx
        sol.state = st
    if trace > 0:
        sol.trace = pdcs_result_trace(r, trace)
    return sol


class Batch:
    """Block-diagonal batch of LPs solved together (pdcs_batch)."""

    def __init__(self, problems):
        self.problems = list(problems)
        self.handle = pdcs_batch_create([p.handle for p in self.problems])

    def solve(self, x0s=None, y0s=None, with_scaling=False, device_out=False, **opts):
        """x0s / y0s: None or one entry per instance (None, a host array, or a
        GPU tensor; GPU tensors select the device warm-start call, one dtype for
        all of them)."""
        o = pdcs_options_default(**opts)
        count = len(self.problems)
        entries = [v for vs in (x0s, y0s) if vs is not None for v in vs if v is not None]
        if any(_is_device_tensor(v) for v in entries):
            for vs in (x0s, y0s):
                if vs is not None and len(vs) != count:
                    raise ValueError(f"expected {count} warm-start entries, got {len(vs)}")
            dtypes = set()
            for i, p in enumerate(self.problems):
                xi = x0s[i] if x0s is not None else None
                yi = y0s[i] if y0s is not None else None
                if xi is not None or yi is not None:
                    dtypes.add(_warm_dtype(xi, yi, {f"x0s[{i}]": (xi, p.n), f"y0s[{i}]": (yi, p.m)}))
            if len(dtypes) != 1:
                raise ValueError("device warm starts must share one dtype")
            rs = pdcs_batch_solve_device(self.handle, count, o,
                                         None if x0s is None else [_dev_ptr(v) for v in x0s],
                                         None if y0s is None else [_dev_ptr(v) for v in y0s],
                                         dtypes.pop(), _torch_stream())
        else:
            rs = pdcs_batch_solve(self.handle, count, o, x0s, y0s, dims=[(p.m, p.n) for p in self.problems])
        out = []
        try:
            for i, (r, p) in enumerate(zip(rs, self.problems)):
                out.append(_collect(r, p.m, p.n, with_scaling, bool(o.keep_state),
                                    int(o.trace_trials) if i == 0 else 0, device_out=device_out))
        finally:
            for r in rs:
                pdcs_result_destroy(r)
        return out

    def autotune(self, budget_ms=0.0):
        pdcs_batch_autotune(self.handle, budget_ms)
        return pdcs_batch_schedule(self.handle)

    def schedule(self):
        return pdcs_batch_schedule(self.handle)

    def set_schedule(self, iter_max, block_nnz, vec_per_block):
        pdcs_batch_set_schedule(self.handle, iter_max, block_nnz, vec_per_block)

    def set_layout(self, layout="auto"):
        """Matrix storage for the trial SpMVs of every instance: "auto", "rows", "bands" or "workgroup"."""
        pdcs_batch_set_layout(self.handle, LAYOUTS[layout] if isinstance(layout, str) else layout)

    def set_band_schedule(self, rows=8192, min_tiles=384, entry_cap=32768):
        pdcs_batch_set_band_schedule(self.handle, rows, min_tiles, entry_cap)

    def band_schedule(self) -> dict:
        return pdcs_batch_band_schedule(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            pdcs_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Warm-start MLP (pdcs_mlp_*)
# ---------------------------------------------------------------------------
def pdcs_mlp_create(d_in, width, d_out, seed=0):
    out = C.c_void_p()
    _check(lib.pdcs_mlp_create(int(d_in), int(width), int(d_out), int(seed), C.byref(out)), "pdcs_mlp_create")
    return out


def pdcs_mlp_forward(net, in_dev: int, out_dev: int, batch: int, stream: int = 0):
    _check(lib.pdcs_mlp_forward(net, C.c_void_p(in_dev), C.c_void_p(out_dev), int(batch),
                                C.c_void_p(stream) if stream else None), "pdcs_mlp_forward")


def pdcs_mlp_train_step(net, in_dev: int, target_dev: int, batch: int, lr: float, stream: int = 0,
                        wait: bool = True):
    """One Adam step; returns the loss before the step, or None (and does not
    wait for the step) when wait is False."""
    loss = C.c_float()
    _check(lib.pdcs_mlp_train_step(net, C.c_void_p(in_dev), C.c_void_p(target_dev), int(batch), float(lr),
                                   C.byref(loss) if wait else None, C.c_void_p(stream) if stream else None),
           "pdcs_mlp_train_step")
    return loss.value if wait else None


def pdcs_mlp_activation(net, which: int, batch: int, features: int) -> np.ndarray:
    out = np.empty((int(batch), int(features)), dtype=np.float32)
    _check(lib.pdcs_mlp_activation(net, int(which), _ptr(out), out.size), "pdcs_mlp_activation")
    return out


def pdcs_mlp_gradients(net, in_dev: int, target_dev: int, batch: int, grad_dev: int, stream: int = 0) -> float:
    loss = C.c_float()
    _check(lib.pdcs_mlp_gradients(net, C.c_void_p(in_dev), C.c_void_p(target_dev), int(batch),
                                  C.c_void_p(grad_dev) if grad_dev else None, C.byref(loss),
                                  C.c_void_p(stream) if stream else None), "pdcs_mlp_gradients")
    return loss.value


def pdcs_mlp_set_normalization(net, in_mean=None, in_scale=None, out_mean=None, out_scale=None):
    arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float32)
            for a in (in_mean, in_scale, out_mean, out_scale)]
    _check(lib.pdcs_mlp_set_normalization(net, *[_ptr(a) for a in arrs]), "pdcs_mlp_set_normalization")


def pdcs_mlp_num_params(net) -> int:
    n = C.c_int64()
    _check(lib.pdcs_mlp_num_params(net, C.byref(n)), "pdcs_mlp_num_params")
    return n.value


def pdcs_mlp_get_params(net) -> np.ndarray:
    out = np.empty(pdcs_mlp_num_params(net), dtype=np.float32)
    _check(lib.pdcs_mlp_get_params(net, _ptr(out)), "pdcs_mlp_get_params")
    return out


def pdcs_mlp_set_params(net, params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    if p.size != pdcs_mlp_num_params(net):
        raise ValueError("parameter count mismatch")
    _check(lib.pdcs_mlp_set_params(net, _ptr(p)), "pdcs_mlp_set_params")


def pdcs_mlp_destroy(net):
    lib.pdcs_mlp_destroy(net)


class MLP:
    """3-layer perceptron with BF16 MFMA kernels (pdcs_mlp).  Device tensors are
    torch tensors (float32, contiguous, row-major [batch x features])."""

    def __init__(self, d_in, width, d_out, seed=0):
        self.d_in, self.width, self.d_out = int(d_in), int(width), int(d_out)
        self.handle = pdcs_mlp_create(d_in, width, d_out, seed)

    def forward(self, u):
        import torch

        assert u.dtype == torch.float32 and u.is_contiguous() and u.shape[1] == self.d_in
        out = torch.empty((u.shape[0], self.d_out), dtype=torch.float32, device=u.device)
        pdcs_mlp_forward(self.handle, u.data_ptr(), out.data_ptr(), u.shape[0],
                         torch.cuda.current_stream().cuda_stream)
        return out

    def train_step(self, u, t, lr, wait=True):
        import torch

        return pdcs_mlp_train_step(self.handle, u.data_ptr(), t.data_ptr(), u.shape[0], lr,
                                   torch.cuda.current_stream().cuda_stream, wait)

    ACTIVATIONS = ("input", "h1", "h2", "dv", "dz2", "dz1")

    def activation(self, name, batch):
        """BF16 activation `name` (ACTIVATIONS) of the last call, widened to float32."""
        which = self.ACTIVATIONS.index(name)
        feats = (self.d_in, self.width, self.width, self.d_out, self.width, self.width)[which]
        return pdcs_mlp_activation(self.handle, which, batch, feats)

    def gradients(self, u, t):
        import torch

        g = torch.empty(pdcs_mlp_num_params(self.handle), dtype=torch.float32, device=u.device)
        loss = pdcs_mlp_gradients(self.handle, u.data_ptr(), t.data_ptr(), u.shape[0], g.data_ptr(),
                                  torch.cuda.current_stream().cuda_stream)
        return loss, g

    def set_normalization(self, in_mean=None, in_scale=None, out_mean=None, out_scale=None):
        """Per-feature standardization of inputs and outputs (host arrays)."""
        pdcs_mlp_set_normalization(self.handle, in_mean, in_scale, out_mean, out_scale)

    @property
    def params(self):
        return pdcs_mlp_get_params(self.handle)

    @params.setter
    def params(self, p):
        pdcs_mlp_set_params(self.handle, p)

    def close(self):
        if getattr(self, "handle", None):
            pdcs_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
