"""GPU parity of the infeasibility tests (option list of Section 3, exit codes
2-5) against the FP64 oracle, through the C ABI.

Up to the first restart check an FP64 solve follows the oracle trial by trial,
so the ratios of that check are compared as numbers (1e-9 relative, or both
+inf).  Later exits are compared by exit code: the exact-certificate cases
(boxed rows, positive unbounded columns) exit at the first check on both
sides; the low-accuracy cases need the trend of three checks.
"""
import math

import numpy as np
import pytest

import lpgen
from oracle import pdcs_oracle as O

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_15504_amd")


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if P.pdcs_device_count() < 1:
        pytest.skip("no GPU visible")


CASES = {
    "sum_row": (lpgen.infeasible_sum_row, {}, {O.EXIT_PRIMAL_INFEASIBLE_HIGH_ACC}),
    "geq_pair": (lpgen.infeasible_geq_pair, {}, {O.EXIT_PRIMAL_INFEASIBLE_HIGH_ACC, O.EXIT_PRIMAL_INFEASIBLE_LOW_ACC}),
    "free_columns": (lpgen.infeasible_free_columns, {}, {O.EXIT_PRIMAL_INFEASIBLE_LOW_ACC}),
    "positive_columns": (lpgen.unbounded_positive_columns, {}, {O.EXIT_DUAL_INFEASIBLE_HIGH_ACC}),
    "free_pair": (lpgen.unbounded_free_pair, {"eps_dual_infeasible_low_acc": 1e-4},
                  {O.EXIT_DUAL_INFEASIBLE_LOW_ACC}),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("layout", ["rows", "bands", "workgroup"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_exit_codes_match_oracle(name, layout, precision):
    gen, kw, allowed = CASES[name]
    inst = gen(0)
    ref = O.solve(O.lpdata_from_instance(inst), O.Options(max_iter=20000, **kw))
    assert ref.exit_code in allowed
    prob = P.Problem.from_instance(inst)
    prob.set_layout(layout)
    sol = prob.solve(precision=precision, max_iter=20000, time_limit=60.0, **kw)
    print(f"{name} {layout} {precision}: gpu exit {sol.info['exit_code']} after {sol.info['iters']} trials, "
          f"oracle exit {ref.exit_code} after {ref.iters}", flush=True)
    assert sol.info["exit_code"] in allowed
    if ref.exit_code in (O.EXIT_PRIMAL_INFEASIBLE_HIGH_ACC, O.EXIT_DUAL_INFEASIBLE_HIGH_ACC) and ref.iters == 64:
        assert sol.info["iters"] == 64 and sol.info["exit_code"] == ref.exit_code


@pytest.mark.parametrize("name", ["free_columns", "free_pair", "sum_row"])
@pytest.mark.parametrize("layout", ["rows", "bands", "workgroup"])
def test_first_check_ratios_match_oracle(name, layout):
    gen, kw, _ = CASES[name]
    inst = gen(1)
    ref = O.solve(O.lpdata_from_instance(inst), O.Options(max_iter=64, check_every=64, **kw))
    c = ref.checks_log[0]
    prob = P.Problem.from_instance(inst)
    prob.set_layout(layout)
    sol = prob.solve(precision="fp64", max_iter=64, check_every=64, keep_state=True, **kw)
    st = sol.state
    assert sol.info["exit_code"] == ref.exit_code
    for key in ("ratio_p", "ratio_d"):
        want, got = c[key], st[key]
        if math.isinf(want):
            assert math.isinf(got), (key, got)
        else:
            assert got == pytest.approx(want, rel=1e-9, abs=1e-300), key


@pytest.mark.parametrize("layout", ["rows", "bands", "workgroup"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_feasible_lps_with_unbounded_columns_stay_optimal(layout, precision):
    # the tests are on by default: feasible LPs with free, one-sided and boxed
    # columns and >= rows must still end optimal.  The objective is compared
    # with HiGHS's optimum.  A relative KKT error of eps bounds |pobj - dobj|
    # by eps (1 + max(|pobj|, |dobj|)), but the primal residual is relative to
    # max(|h|, |Gx|), and with free columns |Gx| can be large: a 1e-7 answer
    # has been seen 2e-6 (relative) from the optimum.  The objective is compared
    # after a 1e-8 solve, where even 100 times that amplification stays within 1e-6.
    from scipy.optimize import linprog

    inst = lpgen.planted_lp(lpgen.rng_for(91, 1), 200, 500, per_col=5, m_zero=100)
    inst.l[:40] = -np.inf
    inst.u[:40] = np.inf
    inst.u[40:80] = np.inf
    lp = O.lpdata_from_instance(inst)
    G = lp.G.toarray()
    bounds = [(None if not np.isfinite(a) else a, None if not np.isfinite(b) else b) for a, b in zip(lp.l, lp.u)]
    hi = linprog(lp.c, A_eq=G[:100], b_eq=lp.h[:100], A_ub=-G[100:], b_ub=-lp.h[100:], bounds=bounds,
                 method="highs")
    assert hi.status == 0
    prob = P.Problem.from_instance(inst)
    prob.set_layout(layout)
    for tol in (1e-6, 1e-7, 1e-8):
        sol = prob.solve(precision=precision, time_limit=60.0, rel_tol=tol, abs_tol=tol)
        assert sol.info["exit_code"] == 0, (tol, sol.info)
        err = O.termination_errors(lp, sol.x, sol.y)
        assert max(err["rel_p"], err["rel_d"], err["rel_gap"]) <= tol * 1.0001
    assert abs(err["pobj"] - hi.fun) / (1 + abs(hi.fun)) <= 1e-6


def test_tests_off_runs_to_max_iter():
    inst = lpgen.infeasible_sum_row(2)
    off = dict(eps_primal_infeasible_low_acc=0.0, eps_dual_infeasible_low_acc=0.0,
               eps_primal_infeasible_high_acc=0.0, eps_dual_infeasible_high_acc=0.0)
    sol = P.Problem.from_instance(inst).solve(precision="fp64", max_iter=640, **off)
    assert sol.info["exit_code"] == O.EXIT_MAX_ITER and sol.info["iters"] == 640
