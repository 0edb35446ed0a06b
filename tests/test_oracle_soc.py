"""Pins of the oracle's second-order-cone rows (socG option of Section 3;
rescaled-cone projection of Section 2.6) against facts it does not compute
itself: the closed-form projection onto the cone, Moreau's decomposition
(which ties the projection onto E K to the one onto E^{-1} K, a different
call), a search over the cone's boundary, SciPy's SLSQP on whole problems, hand-solved
problems, and invariance of the optimum under the diagonal rescaling.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import minimize

import lpgen
from oracle import pdcs_oracle as O


def in_scaled_cone(p, e, tol=1e-12):
    return np.linalg.norm(p[1:] / e[1:]) <= p[0] / e[0] + tol * (1.0 + np.abs(p).max())


def test_proj_soc_hand_values():
    # (1, 2, 0): outside, ||w|| = 2 > 1 > -2: ((1 + 2) / 2) (1, w / ||w||)
    assert np.allclose(O.proj_soc([1.0, 2.0, 0.0]), [1.5, 1.5, 0.0], rtol=0, atol=1e-15)
    assert np.array_equal(O.proj_soc([3.0, 1.0, 1.0]), [3.0, 1.0, 1.0])      # inside
    assert np.array_equal(O.proj_soc([-3.0, 1.0, 1.0]), [0.0, 0.0, 0.0])     # polar
    assert np.allclose(O.proj_soc([0.0, 3.0, 4.0]), [2.5, 1.5, 2.0], rtol=0, atol=1e-15)
    assert np.array_equal(O.proj_soc([-1.0]), [0.0]) and np.array_equal(O.proj_soc([2.0]), [2.0])


def test_proj_soc_moreau_decomposition():
    rng = np.random.default_rng(1)
    for d in (1, 2, 3, 7, 20):
        for _ in range(50):
            v = rng.standard_normal(d) * 3
            p, q = O.proj_soc(v), O.proj_soc(-v)   # the cone is self-dual: polar = -K
            assert np.allclose(v, p - q, rtol=0, atol=1e-13)
            assert abs(p @ q) <= 1e-12 * (1 + v @ v)
            assert in_scaled_cone(p, np.ones(d)) and in_scaled_cone(q, np.ones(d))


def test_proj_scaled_soc_uniform_factor_is_the_cone_itself():
    rng = np.random.default_rng(2)
    for d in (2, 3, 9):
        for _ in range(30):
            v = rng.standard_normal(d) * 2
            e = np.full(d, rng.uniform(0.1, 10.0))
            assert np.allclose(O.proj_scaled_soc(v, e), O.proj_soc(v), rtol=0, atol=1e-12 * (1 + abs(v).max()))


def test_proj_scaled_soc_moreau_between_E_and_its_inverse():
    # (E K)^* = E^{-1} K, so v = P_{E K}(v) - P_{E^{-1} K}(-v) with the two parts orthogonal
    rng = np.random.default_rng(3)
    for d in (2, 3, 5, 12):
        for _ in range(60):
            v = rng.standard_normal(d) * rng.uniform(0.1, 10)
            e = np.exp(rng.uniform(-3, 3, size=d))
            p = O.proj_scaled_soc(v, e)
            q = O.proj_scaled_soc(-v, 1.0 / e)
            scale = 1.0 + np.abs(v).max()
            assert np.allclose(v, p - q, rtol=0, atol=1e-10 * scale)
            assert abs(p @ q) <= 1e-10 * scale * scale
            assert in_scaled_cone(p, e, 1e-10) and in_scaled_cone(q, 1.0 / e, 1e-10)


def _project_by_boundary_search(v, e):
    """Projection onto E K_soc in dimension 3 by searching its boundary: points
    E (r, r cos a, r sin a), r >= 0; for fixed a the best r is the clipped
    least-squares value, and a is searched on a fine grid, then refined by
    golden sections.  Interior points of the cone project onto themselves."""
    if np.hypot(v[1] / e[1], v[2] / e[2]) <= v[0] / e[0]:
        return v.copy()

    def best(a):
        d = np.array([e[0], e[1] * np.cos(a), e[2] * np.sin(a)])
        r = max(0.0, d @ v / (d @ d))
        return np.sum((r * d - v) ** 2), r * d

    grid = np.linspace(-np.pi, np.pi, 20001)
    k = int(np.argmin([best(a)[0] for a in grid]))
    lo, hi = grid[max(k - 1, 0)], grid[min(k + 1, grid.size - 1)]
    g = (math.sqrt(5) - 1) / 2
    for _ in range(200):
        a1, a2 = hi - g * (hi - lo), lo + g * (hi - lo)
        if best(a1)[0] < best(a2)[0]:
            hi = a2
        else:
            lo = a1
    return best(0.5 * (lo + hi))[1]


def test_proj_scaled_soc_matches_boundary_search():
    rng = np.random.default_rng(4)
    for _ in range(40):
        v = rng.standard_normal(3) * 2
        e = np.exp(rng.uniform(-1.5, 1.5, size=3))
        got = O.proj_scaled_soc(v, e)
        want = _project_by_boundary_search(v, e)
        assert np.allclose(got, want, rtol=0, atol=1e-7 * (1 + abs(v).max()))
    # dimension 2: the cone is the wedge |p1 / e1| <= p0 / e0, whose boundary
    # rays are (e0, +-e1); the projection is the closest of v (inside), 0 and
    # the projections onto the two rays
    for _ in range(40):
        v = rng.standard_normal(2) * 2
        e = np.exp(rng.uniform(-1.5, 1.5, size=2))
        if abs(v[1] / e[1]) <= v[0] / e[0]:
            want = v
        else:
            cands = [np.zeros(2)] + [max(0.0, d @ v / (d @ d)) * d for d in (np.array([e[0], e[1]]),
                                                                          np.array([e[0], -e[1]]))]
            want = min(cands, key=lambda p: np.sum((p - v) ** 2))
        assert np.allclose(O.proj_scaled_soc(v, e), want, rtol=0, atol=1e-12 * (1 + abs(v).max()))


def _lp(G, h, c, l, u, m_zero, soc):
    return O.LPData(sp.csr_matrix(np.asarray(G, float)), np.asarray(h, float), np.asarray(c, float),
                    np.asarray(l, float), np.asarray(u, float), m_zero, tuple(soc))


def test_hand_problem_nearest_point_of_a_line():
    # x = (t, w1, w2): min t s.t. w1 + w2 = 1, (t, w) in K_soc, 0 <= t <= 10, w free.
    # The smallest ||w|| on the line is at w = (1/2, 1/2): p* = 1/sqrt(2).
    lp = _lp([[0, 1, 1], [1, 0, 0], [0, 1, 0], [0, 0, 1]], [1, 0, 0, 0], [1, 0, 0],
             [0, -np.inf, -np.inf], [10, np.inf, np.inf], 1, (3,))
    r = O.solve(lp, O.Options(rel_tol=1e-9, abs_tol=1e-9))
    assert r.exit_code == 0
    assert r.pobj == pytest.approx(1 / math.sqrt(2), rel=1e-7)
    assert np.allclose(r.x, [1 / math.sqrt(2), 0.5, 0.5], atol=1e-6)


def test_hand_problem_unit_ball():
    # max w1 + w2 over ||w|| <= t <= 1: w = (1, 1)/sqrt(2), p* = -sqrt(2)
    lp = _lp(np.eye(3), [0, 0, 0], [0, -1, -1], [0, -np.inf, -np.inf], [1, np.inf, np.inf], 0, (3,))
    r = O.solve(lp, O.Options(rel_tol=1e-9, abs_tol=1e-9))
    assert r.exit_code == 0
    assert r.pobj == pytest.approx(-math.sqrt(2), rel=1e-7)


def test_termination_errors_soc_residual_by_hand():
    # x = (1, 2, 0) with G = I, h = 0: the residual (1, 2, 0) is 0.5 * (1, 1, 0)-far
    # from its projection (1.5, 1.5, 0); ||h||_inf = 0, ||Gx||_inf = 2, ||proj||_inf = 1.5
    lp = _lp(np.eye(3), [0, 0, 0], [1, 0, 0], [-5, -5, -5], [5, 5, 5], 0, (3,))
    e = O.termination_errors(lp, np.array([1.0, 2.0, 0.0]), np.zeros(3))
    assert e["abs_p"] == pytest.approx(0.5, abs=1e-15)
    assert e["rel_p"] == pytest.approx(0.5 / 3.0, abs=1e-15)


def _slsqp_objective(inst):
    """SciPy's SLSQP on the same problem, each block as t - ||w|| >= 0, started
    from the planted strictly feasible point (the squared form t^2 >= ||w||^2
    stalls at spurious stationary points)."""
    G = inst.scipy_csr().toarray()
    h, c, mz = inst.h, inst.c, inst.m_zero
    cons = [{"type": "eq", "fun": lambda x: G[:mz] @ x - h[:mz], "jac": lambda x: G[:mz]}]
    a = mz
    for d in inst.soc:
        Gb, hb = G[a:a + d], h[a:a + d]

        def fq(x, Gb=Gb, hb=hb):
            r = Gb @ x - hb
            return np.array([r[0] - np.linalg.norm(r[1:])])

        def jq(x, Gb=Gb, hb=hb):
            r = Gb @ x - hb
            nw = np.linalg.norm(r[1:])
            return (Gb[0] - (r[1:] @ Gb[1:]) / max(nw, 1e-300))[None, :]

        cons.append({"type": "ineq", "fun": fq, "jac": jq})
        a += d
    res = minimize(lambda x: c @ x, inst.x_planted, jac=lambda x: c, bounds=list(zip(inst.l, inst.u)),
                   constraints=cons, method="SLSQP", options={"ftol": 1e-14, "maxiter": 3000})
    # status 8 (no descent direction for the line search) also ends at the
    # optimum here; either way SLSQP's point must be feasible
    assert res.status in (0, 8), res.message
    viol = max([abs(float(np.max(np.abs(cn["fun"](res.x))))) if cn["type"] == "eq" else
                max(0.0, -float(np.min(cn["fun"](res.x)))) for cn in cons])
    assert viol <= 1e-8 * (1 + np.abs(h).max())
    return float(res.fun)


@pytest.mark.parametrize("seed", [0, 1])
def test_soc_instance_matches_slsqp(seed):
    inst = lpgen.soc_instance(seed, m_zero=12, n=60, blocks=(3, 5, 8), per_col=3)
    lp = O.lpdata_from_instance(inst)
    r = O.solve(lp, O.Options(rel_tol=1e-8, abs_tol=1e-8, time_limit=120))
    assert r.exit_code == 0
    want = _slsqp_objective(inst)
    assert abs(r.pobj - want) / (1 + abs(want)) <= 1e-6
    # the answer is feasible to the tolerance in the oracle's own unscaled test
    assert max(r.errors["rel_p"], r.errors["rel_d"], r.errors["rel_gap"]) <= 1e-8


def test_soc_optimum_invariant_under_rescaling():
    inst = lpgen.soc_instance(2, m_zero=12, n=60, blocks=(4, 6), per_col=3)
    lp = O.lpdata_from_instance(inst)
    a = O.solve(lp, O.Options(rel_tol=1e-8, abs_tol=1e-8, use_preconditioner=True, time_limit=120))
    b = O.solve(lp, O.Options(rel_tol=1e-8, abs_tol=1e-8, use_preconditioner=False, time_limit=120))
    assert a.exit_code == 0 and b.exit_code == 0
    assert abs(a.pobj - b.pobj) / (1 + abs(b.pobj)) <= 1e-6


def test_rescaled_cones_follow_the_row_factors():
    # data rescaled by D1 has K_d* blocks diag(D1) K and K_d blocks diag(1/D1) K:
    # Proj_{K_d*} of the rescaled residual is D1 times a point of K, and the
    # rescaled problem's dual projection of D1^{-1} y lies in diag(1/D1) K
    inst = lpgen.soc_instance(3, m_zero=4, n=30, blocks=(5,), per_col=2)
    lp = O.lpdata_from_instance(inst)
    D1 = np.exp(np.random.default_rng(5).uniform(-2, 2, size=lp.m))
    sl = O.rescale(lp, D1, np.ones(lp.n))
    v = np.random.default_rng(6).standard_normal(lp.m) * 3
    p = sl.proj_Kd_star(v)
    blk = slice(lp.m - 5, lp.m)
    assert in_scaled_cone(p[blk], D1[blk], 1e-10)
    q = sl.proj_Kd(v)
    assert in_scaled_cone(q[blk], 1.0 / D1[blk], 1e-10)
    # zero and nonnegative rows keep their plain projections
    assert np.all(p[:4] == 0.0) and np.array_equal(q[:4], v[:4])
