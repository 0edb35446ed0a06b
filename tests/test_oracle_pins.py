"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these re-types an oracle formula to compare with itself: each checks a
hand-derived value, a closed form, an invariant, a brute-force optimum or a
library routine (HiGHS through scipy, numpy's SVD).
"""
import itertools
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


def _load_golden():
    with open(GOLDEN) as f:
        return yaml.safe_load(f)


def _lp_from_dense(d):
    G = sp.csr_matrix(np.array(d["G"], dtype=np.float64))
    f = lambda v: np.array([float(s) for s in v], dtype=np.float64)
    return O.LPData(G, f(d["h"]), f(d["c"]), f(d["l"]), f(d["u"]), int(d["m_zero"]))


def _highs(lp: O.LPData):
    """Optimum of the LP by HiGHS; returns (p*, x*, y*) in the paper's sign convention."""
    mz = lp.m_zero
    G = lp.G.toarray()
    kw = {}
    if mz > 0:
        kw["A_eq"], kw["b_eq"] = G[:mz], lp.h[:mz]
    if lp.m > mz:
        kw["A_ub"], kw["b_ub"] = -G[mz:], -lp.h[mz:]
    bounds = [(None if not np.isfinite(a) else a, None if not np.isfinite(b) else b)
              for a, b in zip(lp.l, lp.u)]
    res = linprog(lp.c, bounds=bounds, method="highs", **kw)
    assert res.status == 0, res.message
    y = np.zeros(lp.m)
    if mz > 0:
        y[:mz] = res.eqlin.marginals
    if lp.m > mz:
        y[mz:] = -res.ineqlin.marginals
    return float(res.fun), res.x, y


def _rel_kkt(err):
    return max(err["rel_p"], err["rel_d"], err["rel_gap"])


# ----------------------------------------------------------------------------
# Error metrics: hand-evaluated example (eq. tolerance-3, tolerance-2,
# adaptive_reflection, KKT_omega, Section 3 termination errors)
# ----------------------------------------------------------------------------
def test_error_metrics_hand_example():
    g = _load_golden()["error_example"]
    lp = _lp_from_dense(g)
    x = np.array(g["x"], float)
    y = np.array(g["y"], float)
    e = O.termination_errors(lp, x, y)
    for k, v in g["inf_norm"].items():
        assert e[k] == pytest.approx(v, rel=1e-14, abs=1e-14), k
    ep, ed, eg, pobj, dobj = O.abs_errors_l2(lp, x, y)
    L = g["l2"]
    assert ep == pytest.approx(L["err_p"], rel=1e-14)
    assert ed == pytest.approx(L["err_d"], rel=1e-14)
    assert eg == pytest.approx(L["err_gap"], rel=1e-14)
    rp, rd, rg = O.rel_errors_l2(lp, x, y)
    assert (rp, rd, rg) == pytest.approx((L["rel_p"], L["rel_d"], L["rel_gap"]), rel=1e-14)
    assert O.reflection_parameter(O.max_err(lp, x, y)) == pytest.approx(L["beta"], rel=1e-13)
    assert O.kkt_omega(ep, ed, eg, g["omega"]) == pytest.approx(L["kkt_omega"], rel=1e-14)


# ----------------------------------------------------------------------------
# Hand-solved LPs: the oracle's solve must land on the hand optimum, and the
# error metrics at the hand optimum must vanish.
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("idx", range(5))
def test_hand_lps(idx):
    d = _load_golden()["lps"][idx]
    lp = _lp_from_dense(d)
    xs = np.array([float(v) for v in d["x_opt"]])
    ys = np.array([float(v) for v in d["y_opt"]])
    e = O.termination_errors(lp, xs, ys)
    assert max(e["abs_p"], e["abs_d"], e["abs_gap"]) < 1e-12
    assert e["pobj"] == pytest.approx(d["p_opt"], abs=1e-12)
    r = O.solve(lp, O.Options(rel_tol=1e-9, abs_tol=1e-9, check_every=8))
    assert r.exit_code == O.EXIT_OPTIMAL
    assert r.pobj == pytest.approx(d["p_opt"], abs=1e-6)
    assert np.allclose(r.x, xs, atol=1e-5)


# ----------------------------------------------------------------------------
# Reflection parameter: closed-form values of eq. adaptive_reflection
# ----------------------------------------------------------------------------
def test_beta_closed_form():
    assert O.reflection_parameter(1.0) == pytest.approx(0.2)
    assert O.reflection_parameter(1e-2) == pytest.approx(0.4)
    assert O.reflection_parameter(1e-6) == pytest.approx(0.8)
    assert O.reflection_parameter(1e-8) == pytest.approx(1.0)
    assert O.reflection_parameter(1e-12) == 1.0
    assert O.reflection_parameter(100.0) == pytest.approx(0.0)
    assert O.reflection_parameter(1e5) == 0.0
    assert O.reflection_parameter(0.0) == 1.0


# ----------------------------------------------------------------------------
# Step size rule (Function 2): hand values of eta' and the eta_bar bound
# ----------------------------------------------------------------------------
def test_eta_next_hand_values():
    # kbar = 1: factors 1 - 2^-0.3 = 0.18775..., 1 + 2^-0.6 = 1.65975...
    f1 = 1.0 - 2.0 ** -0.3
    f2 = 1.0 + 2.0 ** -0.6
    assert f1 == pytest.approx(0.1877476, rel=1e-6)
    assert f2 == pytest.approx(1.6597540, rel=1e-6)
    assert O.eta_next(10.0, 1.0, 1) == pytest.approx(f2 * 1.0)       # growth-limited
    assert O.eta_next(1.0, 10.0, 1) == pytest.approx(f1 * 1.0)       # limit-bound
    # kbar = 2: 1 - 3^-0.3 = 0.28077..., 1 + 3^-0.6 = 1.51728...
    assert O.eta_next(100.0, 1.0, 2) == pytest.approx(1.5172818, rel=1e-6)
    assert O.eta_next(1.0, 100.0, 2) == pytest.approx(0.2807769, rel=1e-6)
    assert O.eta_next(math.inf, 2.0, 5) == pytest.approx(2.0 * (1 + 6 ** -0.6))


def test_eta_bar_at_least_inverse_spectral_norm():
    # |dy^T G dx| <= ||G||_2 ||dx|| ||dy|| <= ||G||_2 * (w||dx||^2 + ||dy||^2/w)/2,
    # so eta_bar >= 1/||G||_2 for every direction and weight.
    rng = np.random.default_rng(7)
    inst = lpgen.c0_instance(0, m=30, n=60, per_col=3)
    lp = O.lpdata_from_instance(inst)
    smax = np.linalg.svd(lp.G.toarray(), compute_uv=False)[0]
    for _ in range(50):
        dx = rng.standard_normal(lp.n)
        dy = rng.standard_normal(lp.m)
        w = 10.0 ** rng.uniform(-2, 2)
        assert O.eta_bar(lp, dx, dy, w) >= (1.0 - 1e-12) / smax
    # the bound is tight for the top singular pair with w = ||dy||/||dx||
    U, S, Vt = np.linalg.svd(lp.G.toarray())
    assert O.eta_bar(lp, Vt[0], U[:, 0], 1.0) == pytest.approx(1.0 / S[0], rel=1e-10)


def test_first_trial_accepted_below_inverse_norm():
    inst = lpgen.c0_instance(1, m=30, n=60, per_col=3)
    lp = O.lpdata_from_instance(inst)
    smax = np.linalg.svd(lp.G.toarray(), compute_uv=False)[0]
    x = np.zeros(lp.n)
    y = np.zeros(lp.m)
    xh, yh, eta, ep, kbar, trials = O.adaptive_step_pdhg(lp, x, y, 1.0, 0.99 / smax, 0)
    assert trials == 1 and kbar == 1


# ----------------------------------------------------------------------------
# Primal weight (Section 2.5): hand values
# ----------------------------------------------------------------------------
def test_primal_weight_hand_values():
    assert O.primal_weight_init(np.array([3.0, 4.0]), np.array([0.0, 2.0])) == pytest.approx(2.5)
    assert O.primal_weight_init(np.array([1e-11]), np.array([1.0])) == 1.0
    assert O.primal_weight_init(np.array([1.0]), np.zeros(3)) == 1.0
    # theta = 1/2: omega_new = sqrt(omega * dy/dx)
    assert O.primal_weight_update(1.0, 4.0, 1.0, 7.0) == pytest.approx(2.0)
    assert O.primal_weight_update(2.0, 8.0, 9.0, 7.0) == pytest.approx(6.0)
    # tiny movement keeps omega
    assert O.primal_weight_update(1e-11, 4.0, 3.0, 7.0) == 3.0
    # leaving [1e-5, 1e5] resets to the initial weight
    assert O.primal_weight_update(1.0, 1e12, 1.0, 7.0) == 7.0
    assert O.primal_weight_update(1e6, 1e-6, 1e-3, 7.0) == 7.0


# ----------------------------------------------------------------------------
# Restart conditions (Section 2.3): hand cases
# ----------------------------------------------------------------------------
def test_restart_rules_hand_cases():
    # first interval: only the artificial rule
    assert O.restart_decision(0, 10, 100, 0.0, None, None) == (False, 0)
    assert O.restart_decision(0, 23, 100, 5.0, None, None) == (True, 3)
    # sufficient decay
    assert O.restart_decision(2, 5, 1000, 0.39, 1.0, None) == (True, 1)
    assert O.restart_decision(2, 5, 1000, 0.41, 1.0, None) == (False, 0)
    # necessary decay + no local progress
    assert O.restart_decision(2, 5, 1000, 0.7, 1.0, 0.6) == (True, 2)
    assert O.restart_decision(2, 5, 1000, 0.7, 1.0, 0.75) == (False, 0)
    assert O.restart_decision(2, 5, 1000, 0.85, 1.0, 0.6) == (False, 0)
    # long inner loop: k >= 0.223 kbar
    assert O.restart_decision(2, 223, 1000, 0.99, 1.0, 0.5) == (True, 3)
    assert O.restart_decision(2, 222, 1000, 0.99, 1.0, 0.5) == (False, 0)


# ----------------------------------------------------------------------------
# Projections: special cases (eq. defn_Lambda1)
# ----------------------------------------------------------------------------
def test_proj_lambda_cases():
    l = np.array([-np.inf, -np.inf, 0.0, 0.0])
    u = np.array([np.inf, 1.0, np.inf, 1.0])
    lam = np.array([3.0, 3.0, -3.0, -3.0])
    assert np.array_equal(O.proj_Lambda(lam, l, u), [0.0, 0.0, 0.0, -3.0])
    lam = -lam
    assert np.array_equal(O.proj_Lambda(lam, l, u), [0.0, -3.0, 3.0, 3.0])


# ----------------------------------------------------------------------------
# Normalized duality gap (Algorithm 3): closed form and exact breakpoint method
# ----------------------------------------------------------------------------
def test_rho_closed_form_without_projection():
    # free x and equality rows: z(t) = z + t (tau b1, sigma b2), so the ball
    # constraint binds at t = r / sqrt(tau|b1|^2 + sigma|b2|^2) and
    # rho = sqrt(tau |b1|^2 + sigma |b2|^2) for every r.
    rng = np.random.default_rng(3)
    m, n = 7, 11
    G = sp.random(m, n, density=0.5, random_state=4, format="csr")
    lp = O.LPData(G, rng.standard_normal(m), rng.standard_normal(n), np.full(n, -np.inf),
                  np.full(n, np.inf), m)
    x = rng.standard_normal(n)
    y = rng.standard_normal(m)
    b1 = G.T @ y - lp.c
    b2 = lp.h - G @ x
    tau, sigma = 0.3, 2.0
    want = math.sqrt(tau * b1 @ b1 + sigma * b2 @ b2)
    for r in (1e-3, 0.5, 7.0):
        got = O.normalized_gap(lp, x, y, tau, sigma, r, rel_eps=1e-12)
        assert got == pytest.approx(want, rel=1e-9)


def _rho_exact_breakpoints(x, y, b1, b2, l, u, mz, tau, sigma, r):
    """Exact rho^N by sorting the breakpoints of ||z - z(t)||_N^2 (piecewise quadratic).

    Coordinate i moves linearly with slope s_i until it hits its bound at time
    T_i (possibly inf) and stays there; its N-weighted squared distance is
    w_i * min(t, T_i)^2 with w_i = s_i^2 / weight.  Solve sum = r^2 exactly.
    """
    s = np.concatenate([tau * b1, sigma * b2])
    wgt = np.concatenate([np.full(x.size, tau), np.full(y.size, sigma)])
    z = np.concatenate([x, y])
    lo = np.concatenate([l, np.where(np.arange(y.size) < mz, -np.inf, 0.0)])
    hi = np.concatenate([u, np.full(y.size, np.inf)])
    T = np.full(z.size, np.inf)
    pos = s > 0
    neg = s < 0
    T[pos] = (hi[pos] - z[pos]) / s[pos]
    T[neg] = (lo[neg] - z[neg]) / s[neg]
    w = s * s / wgt
    bv = np.concatenate([b1, b2])
    order = np.argsort(T)
    T, w, s, bv = T[order], w[order], s[order], bv[order]
    # sum_{T_i < t} w_i T_i^2 + t^2 sum_{T_i >= t} w_i = r^2
    done_sq = 0.0
    active = float(w.sum())
    t_prev = 0.0
    t_star = None
    for i in range(T.size):
        if active > 0:
            t_cand = math.sqrt(max(r * r - done_sq, 0.0) / active)
            if t_cand <= T[i]:
                t_star = max(t_cand, t_prev)
                break
        done_sq += w[i] * T[i] ** 2 if np.isfinite(T[i]) else 0.0
        active -= w[i]
        t_prev = T[i]
    if t_star is None:  # every coordinate saturates inside the ball
        t_star = np.inf
    move = np.where(np.isfinite(T), np.minimum(t_star, T), t_star) * s
    move = np.where(s == 0, 0.0, move)
    return float(bv @ move) / r


@pytest.mark.parametrize("seed", range(4))
def test_rho_bisection_matches_exact_breakpoints(seed):
    rng = np.random.default_rng(100 + seed)
    m, n, mz = 9, 14, 5
    G = sp.random(m, n, density=0.4, random_state=seed, format="csr")
    l = np.where(rng.random(n) < 0.2, -np.inf, 0.0)
    u = np.where(rng.random(n) < 0.2, np.inf, 3.0)
    lp = O.LPData(G, rng.standard_normal(m), rng.standard_normal(n), l, u, mz)
    x = O.proj_box(rng.uniform(-1, 4, n), l, u)
    y = O.proj_Kd(rng.standard_normal(m), mz)
    b1 = G.T @ y - lp.c
    b2 = lp.h - G @ x
    tau, sigma = 0.7, 1.3
    for r in (0.05, 0.4, 2.0):
        want = _rho_exact_breakpoints(x, y, b1, b2, l, u, mz, tau, sigma, r)
        got = O.normalized_gap(lp, x, y, tau, sigma, r, rel_eps=1e-12)
        assert got == pytest.approx(want, rel=1e-8, abs=1e-12)
        assert got >= 0.0


# ----------------------------------------------------------------------------
# Invariants at the HiGHS saddle point
# ----------------------------------------------------------------------------
def _small_lp(seed, m=12, n=30, mz=None):
    inst = lpgen.planted_lp(lpgen.rng_for(90, seed), m, n, per_col=3, m_zero=mz)
    return O.lpdata_from_instance(inst)


@pytest.mark.parametrize("seed,mz", [(0, None), (1, 6), (2, 0)])
def test_onepdhg_fixed_point_and_zero_gap_at_saddle(seed, mz):
    lp = _small_lp(seed, mz=mz)
    p, xs, ys = _highs(lp)
    e = O.termination_errors(lp, xs, ys)
    assert _rel_kkt(e) < 1e-8
    for tau, sigma in ((0.1, 0.1), (1.0, 0.01), (0.02, 3.0)):
        xh, yh = O.one_pdhg(lp, xs, ys, tau, sigma)
        assert np.allclose(xh, xs, atol=1e-7) and np.allclose(yh, ys, atol=1e-7)
    rho = O.normalized_gap(lp, xs, ys, 0.5, 0.5, 1.0)
    assert abs(rho) < 1e-6


def test_weak_duality_on_boxed_lp():
    # Every column is boxed, so Lambda = R and every y (>= 0 on the >= rows)
    # is dual feasible: dual objective <= p*.
    lp = _small_lp(3, mz=6)
    p, _, _ = _highs(lp)
    rng = np.random.default_rng(0)
    for _ in range(20):
        y = O.proj_Kd(rng.standard_normal(lp.m) * 3, lp.m_zero)
        lam = lp.c - lp.G.T @ y
        assert O.dual_objective(lp, y, lam) <= p + 1e-9


def test_primal_error_closed_form_perturbation():
    # Moving one coordinate of a feasible x by delta on equality rows gives a
    # primal residual of |delta| * max_i |G_ij|.
    lp = _small_lp(4)
    _, xs, ys = _highs(lp)
    j = 5
    col = lp.G.toarray()[:, j]
    for delta in (1e-3, -0.2):
        x = xs.copy()
        x[j] += delta
        e = O.termination_errors(lp, x, ys)
        assert e["abs_p"] == pytest.approx(abs(delta) * np.max(np.abs(col)), rel=1e-6)


# ----------------------------------------------------------------------------
# Scaling (Section 2.6): Ruiz fixed point and the Algorithm 4 round trip
# ----------------------------------------------------------------------------
def test_ruiz_equilibrates_rows_and_columns():
    inst = lpgen.c4_instance(0, m=40, n=90, per_col=4)
    G = inst.scipy_csr()
    D1, D2 = O.ruiz_l2_scaling(G, ruiz_iters=60, l2_pass=False)
    Gs = abs(sp.diags(D1) @ G @ sp.diags(D2)).tocsr()
    rmax = np.asarray(Gs.max(axis=1).todense()).ravel()
    cmax = np.asarray(Gs.max(axis=0).todense()).ravel()
    assert np.allclose(rmax, 1.0, atol=1e-6) and np.allclose(cmax, 1.0, atol=1e-6)


def test_l2_pass_on_diagonal_matrix():
    # For a diagonal matrix, Ruiz makes every entry 1 after one pass
    # (d -> d / sqrt(d) / sqrt(d)) and the L2 pass leaves it at 1.
    G = sp.diags([4.0, 0.25, 9.0]).tocsr()
    D1, D2 = O.ruiz_l2_scaling(G, ruiz_iters=1, l2_pass=True)
    assert np.allclose(D1 * np.array([4.0, 0.25, 9.0]) * D2, 1.0, rtol=1e-15)
    assert np.allclose(D1, [0.5, 2.0, 1.0 / 3.0], rtol=1e-15)


@pytest.mark.parametrize("precond", [True, False])
def test_scaling_round_trip_same_optimum(precond):
    lp = _small_lp(5, m=15, n=40)
    p, _, _ = _highs(lp)
    r = O.solve(lp, O.Options(use_preconditioner=precond, rel_tol=1e-8, abs_tol=1e-8))
    assert r.exit_code == 0
    assert abs(r.pobj - p) <= 1e-6 * (1 + abs(p))


# ----------------------------------------------------------------------------
# Vertex brute force on tiny LPs and closed forms
# ----------------------------------------------------------------------------
def _brute_force(G, h, c, l, u):
    """Best vertex of {Gx = h, l <= x <= u} by enumerating bases (all bounds finite)."""
    m, n = G.shape
    best = np.inf
    for B in itertools.combinations(range(n), m):
        GB = G[:, B]
        if abs(np.linalg.det(GB)) < 1e-10:
            continue
        N = [j for j in range(n) if j not in B]
        for pick in itertools.product((0, 1), repeat=len(N)):
            xN = np.array([u[j] if p else l[j] for j, p in zip(N, pick)])
            xB = np.linalg.solve(GB, h - G[:, N] @ xN)
            if np.all(xB >= l[list(B)] - 1e-9) and np.all(xB <= u[list(B)] + 1e-9):
                x = np.zeros(n)
                x[list(B)] = xB
                x[N] = xN
                best = min(best, float(c @ x))
    return best


@pytest.mark.parametrize("seed", range(4))
def test_tiny_lp_vertex_brute_force(seed):
    rng = np.random.default_rng(500 + seed)
    m, n = 3, 7
    G = rng.standard_normal((m, n))
    l = -rng.uniform(0, 2, n)
    u = rng.uniform(1, 3, n)
    x0 = rng.uniform(l, u)
    h = G @ x0
    c = rng.standard_normal(n)
    want = _brute_force(G, h, c, l, u)
    lp = O.LPData(sp.csr_matrix(G), h, c, l, u, m)
    r = O.solve(lp, O.Options(rel_tol=1e-9, abs_tol=1e-9, check_every=16))
    assert r.exit_code == 0
    assert r.pobj == pytest.approx(want, abs=1e-6 * (1 + abs(want)))


def test_knapsack_closed_form():
    # sum x = b, 0 <= x <= u: greedy by cost (fractional knapsack).
    rng = np.random.default_rng(11)
    n = 25
    c = rng.uniform(-1, 1, n)
    u = rng.uniform(0.5, 2, n)
    b = 0.4 * u.sum()
    order = np.argsort(c)
    x = np.zeros(n)
    left = b
    for j in order:
        x[j] = min(u[j], left)
        left -= x[j]
    want = float(c @ x)
    lp = O.LPData(sp.csr_matrix(np.ones((1, n))), np.array([b]), c, np.zeros(n), u, 1)
    r = O.solve(lp, O.Options(rel_tol=1e-9, abs_tol=1e-9, check_every=16))
    assert r.exit_code == 0
    assert r.pobj == pytest.approx(want, abs=1e-6)


def test_separable_closed_form_with_slack_rows():
    # Rows that can never bind (x >= -100 for boxed x) leave x_j = l_j if c_j > 0 else u_j.
    rng = np.random.default_rng(12)
    n = 20
    c = rng.standard_normal(n)
    l = -rng.uniform(0, 1, n)
    u = rng.uniform(0, 1, n)
    G = sp.csr_matrix(np.eye(n)[:4] + np.eye(n)[4:8])
    h = np.full(4, -100.0)
    lp = O.LPData(G, h, c, l, u, 0)
    r = O.solve(lp, O.Options(rel_tol=1e-9, abs_tol=1e-9, check_every=16))
    assert r.exit_code == 0
    assert np.allclose(r.x, np.where(c > 0, l, u), atol=1e-6)


# ----------------------------------------------------------------------------
# The whole method against HiGHS on config-0-shaped LPs
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1])
def test_c0_against_highs(seed):
    inst = lpgen.c0_instance(seed)
    lp = O.lpdata_from_instance(inst)
    p, _, _ = _highs(lp)
    r = O.solve(lp, O.Options())
    assert r.exit_code == 0
    assert _rel_kkt(r.errors) <= 1e-6
    assert abs(r.pobj - p) / (1 + abs(p)) <= 1e-6


@pytest.mark.parametrize("method", ["average", "halpern"])
def test_candidate_methods_against_highs(method):
    lp = _small_lp(6, m=20, n=50, mz=10)
    p, _, _ = _highs(lp)
    r = O.solve(lp, O.Options(method=method, rel_tol=1e-7, abs_tol=1e-7))
    assert r.exit_code == 0
    assert abs(r.pobj - p) / (1 + abs(p)) <= 1e-6


def test_kkt_restart_option_against_highs():
    # restart decisions on KKT_omega (the use_kkt_restart option of Section 3,
    # the fallback metric of Section 2.3) still reach the optimum
    lp = _small_lp(7, m=20, n=50, mz=10)
    p, _, _ = _highs(lp)
    r = O.solve(lp, O.Options(use_kkt_restart=True, rel_tol=1e-7, abs_tol=1e-7))
    assert r.exit_code == 0
    assert all(c["use_kkt"] for c in r.checks_log)
    assert abs(r.pobj - p) / (1 + abs(p)) <= 1e-6


def test_infinite_bounds_and_geq_rows_against_highs():
    rng = np.random.default_rng(21)
    inst = lpgen.planted_lp(lpgen.rng_for(91, 0), 15, 40, per_col=3, m_zero=8)
    l = inst.l.copy()
    u = inst.u.copy()
    u[rng.random(40) < 0.3] = np.inf      # one-sided columns
    lp = O.LPData(inst.scipy_csr(), inst.h, inst.c, l, u, inst.m_zero)
    p, _, _ = _highs(lp)
    r = O.solve(lp, O.Options(rel_tol=1e-7, abs_tol=1e-7))
    assert r.exit_code == 0
    assert abs(r.pobj - p) / (1 + abs(p)) <= 1e-6


def test_empty_rows_and_columns():
    # an all-zero row with h = 0 and an all-zero column (decided by its cost sign)
    G = sp.csr_matrix(np.array([[1.0, 1.0, 0.0, 0.0], [0.0, 0.0, 0.0, 0.0], [1.0, -1.0, 0.0, 1.0]]))
    lp = O.LPData(G, np.array([2.0, 0.0, 0.5]), np.array([1.0, 2.0, -1.0, 0.5]),
                  np.zeros(4), np.full(4, 5.0), 2)
    p, _, _ = _highs(lp)
    r = O.solve(lp, O.Options(rel_tol=1e-9, abs_tol=1e-9, check_every=16))
    assert r.exit_code == 0
    assert r.pobj == pytest.approx(p, abs=1e-6)
    assert r.x[2] == pytest.approx(5.0, abs=1e-6)


def test_warm_start_from_optimum_returns_immediately():
    lp = _small_lp(7)
    p, xs, ys = _highs(lp)
    r = O.solve(lp, O.Options(use_preconditioner=False), x0=xs, y0=ys)
    assert r.exit_code == 0 and r.iters == 0


def test_max_iter_and_time_limit_exit_codes():
    lp = _small_lp(8)
    r = O.solve(lp, O.Options(max_iter=10))
    assert r.exit_code == O.EXIT_MAX_ITER and r.iters == 10
    r = O.solve(lp, O.Options(time_limit=0.0))
    assert r.exit_code == O.EXIT_TIME_LIMIT


def test_scaling_hand_example_non_diagonal():
    # one Ruiz pass and the square-root-of-Euclidean-norm pass on a 2 x 3 matrix,
    # evaluated by hand in closed form (tests/golden/hand_lps.yaml): a different
    # L2 formula (the norm itself, the L1 norm) or a pass taken from a stale
    # matrix gives other numbers
    g = _load_golden()["scaling_example"]
    G = sp.csr_matrix(np.array(g["G"], dtype=np.float64))
    D1, D2 = O.ruiz_l2_scaling(G, int(g["ruiz_iters"]), True)
    np.testing.assert_allclose(D1, g["D1"], rtol=1e-14)
    np.testing.assert_allclose(D2, g["D2"], rtol=1e-14)
