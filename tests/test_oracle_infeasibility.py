"""Pins of the oracle's infeasibility tests (option list of Section 3, exit codes
2-5 of the exit-code table) and of the restart-metric options.

The pins come from outside the oracle: hand-evaluated rays (tests/golden),
HiGHS's status for the generated infeasible and unbounded LPs, certificates
checked against the definition of infeasibility (a dual ray that makes every
box point violate the weighted constraints; a primal ray that stays feasible
and lowers the cost), and feasible LPs on which no test may fire.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import yaml
from scipy.optimize import linprog

import lpgen
from oracle import pdcs_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_lps.yaml")


def _f(v):
    return float(v)  # yaml leaves "inf" and "-inf" as strings; float() reads them


def _lp(d):
    G = sp.csr_matrix(np.array(d["G"], dtype=np.float64))
    vec = lambda v: np.array([_f(s) for s in v], dtype=np.float64)
    return O.LPData(G, vec(d["h"]), vec(d["c"]), vec(d["l"]), vec(d["u"]), int(d["m_zero"]))


def _highs_status(lp: O.LPData) -> int:
    mz = lp.m_zero
    G = lp.G.toarray()
    kw = {}
    if mz > 0:
        kw["A_eq"], kw["b_eq"] = G[:mz], lp.h[:mz]
    if lp.m > mz:
        kw["A_ub"], kw["b_ub"] = -G[mz:], -lp.h[mz:]
    bounds = [(None if not np.isfinite(a) else a, None if not np.isfinite(b) else b) for a, b in zip(lp.l, lp.u)]
    return int(linprog(lp.c, bounds=bounds, method="highs", **kw).status)


@pytest.mark.parametrize("idx", range(6))
def test_ratios_hand_values(idx):
    ex = yaml.safe_load(open(GOLDEN))["infeasibility_examples"][idx]
    lp = _lp(ex)
    rp, rd = O.infeasibility_ratios(lp, np.array(ex["ray_x"], float), np.array(ex["ray_y"], float))
    for got, want in ((rp, _f(ex["ratio_p"])), (rd, _f(ex["ratio_d"]))):
        if math.isinf(want):
            assert math.isinf(got), ex["name"]
        else:
            assert got == pytest.approx(want, rel=1e-15, abs=1e-15), ex["name"]


def test_rounding_bound_definition():
    u = 2.0 ** -53
    assert O.rounding_bound(1) == pytest.approx(u / (1 - u), rel=1e-15)
    assert O.rounding_bound(10 ** 6) == pytest.approx(1e6 * u / (1 - 1e6 * u), rel=1e-12)
    assert O.rounding_bound(0) == O.rounding_bound(1)


def test_monitor_trend_and_priority():
    o = O.Options()
    mon = O.InfeasibilityMonitor(o)
    # low-accuracy primal: ratio below 1e-12 with a rising dual objective at 3
    # consecutive checks; the first check has no previous objective
    assert mon.update(1e-13, math.inf, 0.0, 1.0) is None       # no trend yet
    assert mon.update(1e-13, math.inf, 0.0, 2.0) is None       # 1
    assert mon.update(1e-13, math.inf, 0.0, 3.0) is None       # 2
    assert mon.update(1e-13, math.inf, 0.0, 4.0) == O.EXIT_PRIMAL_INFEASIBLE_LOW_ACC
    mon = O.InfeasibilityMonitor(o)
    for dobj in (1.0, 2.0, 3.0):
        mon.update(1e-13, math.inf, 0.0, dobj)
    assert mon.update(1e-13, math.inf, 0.0, 2.5) is None       # not rising: the count restarts
    assert mon.trend_p == 0
    # high accuracy wins at once, primal before dual
    mon = O.InfeasibilityMonitor(o)
    assert mon.update(0.0, 0.0, 0.0, 0.0) == O.EXIT_PRIMAL_INFEASIBLE_HIGH_ACC
    mon = O.InfeasibilityMonitor(o)
    assert mon.update(math.inf, 1e-17, 0.0, 0.0) == O.EXIT_DUAL_INFEASIBLE_HIGH_ACC
    # dual low accuracy: the negated primal objective must rise
    mon = O.InfeasibilityMonitor(o)
    codes = [mon.update(math.inf, 1e-13, -k, 0.0) for k in range(4)]
    assert codes == [None, None, None, O.EXIT_DUAL_INFEASIBLE_LOW_ACC]
    # a tolerance of 0 switches its test off
    off = O.InfeasibilityMonitor(O.Options(eps_primal_infeasible_high_acc=0.0, eps_primal_infeasible_low_acc=0.0))
    assert all(off.update(0.0, math.inf, 0.0, float(k)) is None for k in range(6))


def _farkas_margin(lp: O.LPData, ray_y):
    """max over the box of ray_y^T (G x - h); negative (with ray_y in K_d)
    proves that no box point satisfies G x - h in K_d*, since y^T v >= 0 for
    y in K_d and v in K_d*.  The maximum of a linear function over a box is
    separable: each x_j sits at the bound its coefficient points to."""
    assert np.all(ray_y[lp.m_zero:] >= 0.0)
    g = lp.G.T @ ray_y
    lo = np.where(g > 0, lp.u, lp.l)
    terms = np.where(g == 0, 0.0, g * lo)
    return float(np.sum(terms) - lp.h @ ray_y)


@pytest.mark.parametrize("gen", ["infeasible_sum_row", "infeasible_geq_pair"])
def test_boxed_infeasible_lps_exit_with_farkas_ray(gen):
    lp = O.lpdata_from_instance(getattr(lpgen, gen)(0))
    assert _highs_status(lp) == 2
    r = O.solve(lp, O.Options(max_iter=20000))
    assert r.exit_code in (O.EXIT_PRIMAL_INFEASIBLE_LOW_ACC, O.EXIT_PRIMAL_INFEASIBLE_HIGH_ACC)
    assert _farkas_margin(lp, r.state["ray_y"]) < 0.0


def test_infeasible_with_free_columns_low_accuracy():
    lp = O.lpdata_from_instance(lpgen.infeasible_free_columns(0))
    assert _highs_status(lp) == 2
    r = O.solve(lp, O.Options(max_iter=20000))
    assert r.exit_code == O.EXIT_PRIMAL_INFEASIBLE_LOW_ACC
    ray_y = r.state["ray_y"]
    # the ray is a certificate up to its tiny Lambda violation on the unbounded
    # columns: dropping those columns' terms, the margin is negative by far more
    lam = -(lp.G.T @ ray_y)
    free = ~np.isfinite(lp.l) & ~np.isfinite(lp.u)
    lower_only = np.isfinite(lp.l) & ~np.isfinite(lp.u)
    viol = np.linalg.norm(np.concatenate([lam[free], np.minimum(lam[lower_only], 0.0)]))
    boxed = np.isfinite(lp.l) & np.isfinite(lp.u)
    g = -lam
    # boxed columns take the bound their coefficient points to; lower-only
    # columns sit at l (their g > 0 part is the violation counted above), free
    # columns drop out (their g is the violation)
    margin = float(np.sum(np.where(g[boxed] > 0, g[boxed] * lp.u[boxed], g[boxed] * lp.l[boxed]))
                   + np.sum(g[lower_only] * lp.l[lower_only]) - lp.h @ ray_y)
    assert margin < 0.0 and viol < 1e-12 * abs(margin)


def _unbounded_check(lp: O.LPData, ray_x, tol):
    """ray_x proves the LP unbounded (with a feasible point, which HiGHS's status
    confirms): it stays in the recession cone of the box, keeps G r in K_d*
    (within tol relative to the cost decrease) and lowers the cost."""
    lf, uf = np.isfinite(lp.l), np.isfinite(lp.u)
    assert np.all(ray_x[lf & uf] == 0.0) and np.all(ray_x[lf & ~uf] >= 0.0) and np.all(ray_x[~lf & uf] <= 0.0)
    gr = lp.G @ ray_x
    viol = np.concatenate([gr[: lp.m_zero], np.minimum(gr[lp.m_zero:], 0.0)])
    dec = -float(lp.c @ ray_x)
    assert dec > 0.0 and np.linalg.norm(viol) <= tol * dec


def test_unbounded_positive_columns_high_accuracy():
    lp = O.lpdata_from_instance(lpgen.unbounded_positive_columns(0))
    assert _highs_status(lp) == 3
    r = O.solve(lp, O.Options(max_iter=20000))
    assert r.exit_code == O.EXIT_DUAL_INFEASIBLE_HIGH_ACC
    _unbounded_check(lp, r.state["ray_x"], 1e-16)


def test_unbounded_free_pair_low_accuracy():
    lp = O.lpdata_from_instance(lpgen.unbounded_free_pair(0))
    assert _highs_status(lp) == 3
    r = O.solve(lp, O.Options(max_iter=20000, eps_dual_infeasible_low_acc=1e-4))
    assert r.exit_code == O.EXIT_DUAL_INFEASIBLE_LOW_ACC
    _unbounded_check(lp, r.state["ray_x"], 1e-4)


FEASIBLE = [("c0", lambda: lpgen.c0_instance(1)), ("c0", lambda: lpgen.c0_instance(2)),
            ("geq", lambda: lpgen.planted_lp(lpgen.rng_for(91, 0), 200, 500, per_col=5, m_zero=0)),
            ("dense_runs", lambda: lpgen.dense_runs_instance(0, m=32, run=8))]


@pytest.mark.parametrize("idx", range(len(FEASIBLE)))
def test_no_infeasibility_exit_on_feasible_lps(idx):
    lp = O.lpdata_from_instance(FEASIBLE[idx][1]())
    assert _highs_status(lp) == 0
    r = O.solve(lp, O.Options())
    assert r.exit_code == O.EXIT_OPTIMAL
    ratios = [c["ratio_p"] for c in r.checks_log if "ratio_p" in c]
    assert ratios and all(not (v < 1e-12) for v in ratios)


def test_feasible_with_free_columns_no_false_positive():
    inst = lpgen.c0_instance(0)
    inst.l[:50] = -np.inf
    inst.u[:50] = np.inf
    inst.u[50:100] = np.inf
    lp = O.lpdata_from_instance(inst)
    assert _highs_status(lp) == 0
    assert O.solve(lp, O.Options()).exit_code == O.EXIT_OPTIMAL


def test_kkt_metric_options_skip_the_gap_and_solve():
    lp = O.lpdata_from_instance(lpgen.c0_instance(3))
    for opts in (O.Options(use_duality_gap_restart=False), O.Options(use_kkt_restart=True)):
        r = O.solve(lp, opts)
        assert r.exit_code == 0
        assert all(c["use_kkt"] for c in r.checks_log)
        assert all(math.isnan(v) for c in r.checks_log for v in c["rho"].values())


def test_restart_frequency_options_set_the_check_period():
    lp = O.lpdata_from_instance(lpgen.c0_instance(3))
    r = O.solve(lp, O.Options(duality_gap_restart_freq=128, max_iter=1280))
    assert [c["kbar"] for c in r.checks_log] and all(c["kbar"] % 128 == 0 for c in r.checks_log)
    r = O.solve(lp, O.Options(use_kkt_restart=True, kkt_restart_freq=96, duality_gap_restart_freq=128,
                              max_iter=960))
    assert all(c["kbar"] % 96 == 0 for c in r.checks_log)
