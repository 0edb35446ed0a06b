"""The C-ABI library loads and exports every symbol include/pdcs.h declares;
host-side argument validation (runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "pdcs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pdcs_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_2603_15504_amd as P

    lib = ctypes.CDLL(P.LIB_PATH)
    names = _declared_functions()
    assert len(names) >= 30
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert P.MISSING == []


def test_options_defaults_follow_the_paper():
    import paper_2603_15504_amd as P

    o = P.pdcs_options_default()
    assert o.rel_tol == 1e-6 and o.abs_tol == 1e-6 and o.time_limit == 1000.0
    assert o.use_preconditioner == 1 and o.method == 0
    assert P.pdcs_status_string(0) == "optimal" and P.pdcs_status_string(8) == "numerical_error"
    assert P.pdcs_status_string(6) == "time_limit"
    # engineering defaults of the added options
    assert o.check_every == 64 and o.stall_checks == 512 and o.probe_passes == 7
    assert o.use_graph == 1 and o.compact == 1 and o.precision == 0


def test_options_struct_matches_header():
    # the ctypes mirror has the C struct's size: every field is 8 bytes wide
    import ctypes
    import re

    import paper_2603_15504_amd as P

    hdr = open(__file__.replace("tests/test_abi.py", "include/pdcs.h")).read()
    body = hdr[hdr.index("typedef struct {", hdr.index("pdcs_options")):]
    body = body[: body.index("} pdcs_options;")]
    n = 0
    for decl in re.findall(r"^\s*(?:int64_t|double)\s+([^;]+);", body, re.M):
        for name in decl.split(","):
            m = re.search(r"\[(\d+)\]", name)
            n += int(m.group(1)) if m else 1
    assert ctypes.sizeof(P.pdcs_options) == 8 * n


def _tiny():
    row_ptr = np.array([0, 2, 3], dtype=np.int64)
    col = np.array([0, 1, 1], dtype=np.int32)
    val = np.array([1.0, 2.0, -1.0])
    return 2, 2, row_ptr, col, val, np.array([1.0, 0.5]), np.array([1.0, 1.0])


@pytest.mark.parametrize("case", ["bad_rowptr", "col_range", "unsorted", "nan_val", "nan_h", "l_gt_u",
                                  "mzero", "inf_c", "lower_plus_inf"])
def test_problem_validation_errors(case):
    import paper_2603_15504_amd as P

    m, n, rp, col, val, h, c = _tiny()
    l = np.zeros(n)
    u = np.ones(n)
    mz = 2
    if case == "bad_rowptr":
        rp = np.array([0, 3, 2], dtype=np.int64)
    elif case == "col_range":
        col = np.array([0, 2, 1], dtype=np.int32)
    elif case == "unsorted":
        col = np.array([1, 0, 1], dtype=np.int32)
    elif case == "nan_val":
        val = np.array([1.0, np.nan, 1.0])
    elif case == "nan_h":
        h = np.array([np.nan, 0.0])
    elif case == "l_gt_u":
        l = np.array([2.0, 0.0])
    elif case == "mzero":
        mz = 3
    elif case == "inf_c":
        c = np.array([np.inf, 0.0])
    elif case == "lower_plus_inf":
        l = np.array([np.inf, 0.0])
        u = np.array([np.inf, 1.0])
    with pytest.raises(P.PdcsError) as e:
        P.pdcs_problem_create(m, n, mz, rp, col, val, h, c, l, u)
    assert e.value.code == -1


def test_null_handles_are_rejected():
    import paper_2603_15504_amd as P

    assert P.lib.pdcs_result_info(None, None) == -1
    assert P.lib.pdcs_problem_dims(None, None, None, None) == -1
    assert P.lib.pdcs_batch_create(0, None, None) == -1
    assert P.lib.pdcs_mlp_create(0, 1, 1, 0, None) == -1


def test_new_option_defaults_follow_the_paper():
    # option list of Section 3: infeasibility tolerances, the duality-gap
    # restart switch and the print frequency
    import paper_2603_15504_amd as P

    o = P.pdcs_options_default()
    assert o.eps_primal_infeasible_low_acc == 1e-12 and o.eps_dual_infeasible_low_acc == 1e-12
    assert o.eps_primal_infeasible_high_acc == 1e-16 and o.eps_dual_infeasible_high_acc == 1e-16
    assert o.use_duality_gap_restart == 1 and o.use_kkt_restart == 0
    assert o.print_freq == 2000
    # 0: the check period falls back to check_every
    assert o.kkt_restart_freq == 0 and o.duality_gap_restart_freq == 0
    assert P.pdcs_status_string(2) == "primal_infeasible_low_acc"
    assert P.pdcs_status_string(5) == "dual_infeasible_high_acc"


def test_state_struct_matches_header():
    import paper_2603_15504_amd as P

    hdr = open(os.path.join(ROOT, "include", "pdcs.h")).read()
    end = hdr.index("} pdcs_state_scalars;")
    body = hdr[hdr.rindex("typedef struct {", 0, end):end]
    n = 0
    for decl in re.findall(r"^\s*(?:int64_t|double)\s+([^;]+);", body, re.M):
        n += len(decl.split(","))
    assert ctypes.sizeof(P.pdcs_state_scalars) == 8 * n


def test_batch_warm_start_lengths_checked_before_the_call():
    # the library reads exactly n_b / m_b values per instance, so the binding
    # refuses other lengths (and a wrong entry count) before calling it
    import paper_2603_15504_amd as P

    dims = [(3, 5), (2, 4)]
    with pytest.raises(ValueError):
        P.pdcs_batch_solve(None, 2, None, x0s=[np.zeros(4), None], dims=dims)
    with pytest.raises(ValueError):
        P.pdcs_batch_solve(None, 2, None, y0s=[np.zeros(3), np.zeros(3)], dims=dims)
    with pytest.raises(ValueError):
        P.pdcs_batch_solve(None, 2, None, x0s=[np.zeros(5)], dims=dims)
    with pytest.raises(ValueError):
        P.pdcs_batch_solve(None, 2, None, dims=dims[:1])
