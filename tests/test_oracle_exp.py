"""Pins of the oracle's exponential-cone rows (expG and dual_expG options of
Section 3; rescaled-cone projection of Section 2.6) against facts it does not
compute itself: points whose projection is known by construction (a boundary
ray of the cone plus a multiple of its normal), the textbook case of the
projection onto K_exp when the first two coordinates are nonpositive, the
characterization of a projection onto a closed convex cone (the point in the
cone, the residual in the polar cone, the two orthogonal), SciPy's SLSQP on the
projection and on whole problems, hand-solved problems, and invariance of the
optimum under the diagonal rescaling.

Convention: K_exp = closure {(x, y, z): y > 0, y e^(x / y) <= z}, its dual
K_exp* = closure {(u, v, w): u < 0, -u e^(v / u) <= e w}.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import minimize

import lpgen
from oracle import pdcs_oracle as O


def near_exp(q, tol):
    """q within about tol (in the max norm, relative to its size) of K_exp: some
    point moved by at most s = tol (1 + ||q||) in each coordinate lies in the
    cone (x down, z up, y tried at y and y +- s)."""
    x, y, z = (float(t) for t in q)
    s = tol * (1.0 + max(abs(x), abs(y), abs(z)))
    if y <= s and x <= s and z >= -s and y >= -s:
        return True
    return any(yy > 0.0 and yy * math.exp(min((x - s) / yy, 700.0)) <= z + s for yy in (y - s, y, y + s))


def near_exp_dual(q, tol):
    """q within about tol of K_exp*, in the same sense (v and w up, u tried at
    u and u +- s)."""
    u, v, w = (float(t) for t in q)
    s = tol * (1.0 + max(abs(u), abs(v), abs(w)))
    if u >= -s and u <= s and v >= -s and w >= -s:
        return True
    return any(uu < 0.0 and -uu * math.exp(min((v + s) / uu, 700.0)) <= math.e * (w + s) for uu in (u - s, u, u + s))


def ray(r):
    """Boundary ray of K_exp: (r, 1, e^r)."""
    return np.array([r, 1.0, math.exp(r)])


def normal(r):
    """Element of K_exp* orthogonal to ray(r): u = -1 puts it on the boundary
    e w = e^-v, and <(-1, v, e^(-v-1)), (r, 1, e^r)> = 0 at v = r - 1."""
    return np.array([-1.0, r - 1.0, math.exp(-r)])


def test_memberships_by_hand():
    assert O.in_exp_cone([0.0, 1.0, 1.0]) and O.in_exp_cone([-5.0, 0.0, 0.0])
    assert not O.in_exp_cone([1.0, 1.0, 2.0])          # 1 * e^1 > 2
    assert O.in_exp_cone([1.0, 1.0, 3.0])
    assert not O.in_exp_cone([1.0, 0.0, 5.0])          # y = 0 needs x <= 0
    assert O.in_exp_dual([-1.0, 0.0, 1.0 / math.e]) and O.in_exp_dual([0.0, 2.0, 3.0])
    assert not O.in_exp_dual([-1.0, 0.0, 0.3])         # e * 0.3 < 1
    assert not O.in_exp_dual([0.0, -1.0, 1.0])
    # the two cones are dual: <K, K*> >= 0 on samples of each boundary
    for r in np.linspace(-4, 4, 17):
        for t in np.linspace(-4, 4, 17):
            assert ray(r) @ normal(t) >= -1e-12


@pytest.mark.parametrize("seed", range(4))
def test_projection_of_ray_plus_normal_is_the_ray_point(seed):
    # p = s F a(r) lies on the boundary of F K_exp and w = -t F^-1 n(r) in its
    # polar (-F w = t n(r) in K_exp*) with <p, w> = s t <a, n> = 0: P(p + w) = p
    # (the normal taken times min(1, e^r), to keep it finite for r << 0)
    rng = np.random.default_rng(seed)
    for k in range(60):
        f = np.exp(rng.uniform(-2, 2, size=3)) if seed else np.ones(3)
        r = rng.uniform(-6, 4) if k % 2 else rng.uniform(-60, 40)
        s, t = rng.uniform(0.05, 5.0), rng.uniform(0.0, 5.0)
        p = s * f * ray(r)
        v = p - t * normal(r) * min(1.0, math.exp(r)) / f
        got = O.proj_scaled_exp(v, f)
        assert np.allclose(got, p, rtol=0, atol=1e-9 * (1 + np.abs(v).max())), (f, r, s, t)


@pytest.mark.parametrize("seed", range(3))
def test_projection_near_the_apex_is_the_ray_point(seed):
    # the same construction with s a billionth of t: the projection p is
    # within 1e-7 |v| of the apex, so its distance from v and that of the face
    # clip 0 agree to rounding (|v|^2 - |v - p|^2 = |p|^2), while the points
    # differ by |p|; the optimality conditions, not the distances, single p
    # out, and the projection is 1-Lipschitz, so rounding v moves it by as much
    rng = np.random.default_rng(100 + seed)
    for k in range(40):
        f = np.exp(rng.uniform(-2, 2, size=3)) if seed else np.ones(3)
        r = rng.uniform(-8, 5)
        t = rng.uniform(0.1, 10.0)
        s = t * 10.0 ** rng.uniform(-10, -7)
        p = s * f * ray(r)
        v = p - t * normal(r) * min(1.0, math.exp(r)) / f
        got = O.proj_scaled_exp(v, f)
        assert np.abs(got - p).max() <= 1e-13 * np.abs(v).max(), (f, r, s, t, got, p)


@pytest.mark.parametrize("r", [-300.5, -400.0, -700.0, -2000.0])
def test_projection_onto_far_negative_rays(r):
    # the rays (r, 1, e^r) approach the face edge (-1, 0, 0) only like 1 / |r|:
    # with e^r F^-1 n(r) = F^-1 (-e^r, (r - 1) e^r, 1) as the normal, the point
    # s F a(r) - t F^-1 (-e^r, (r - 1) e^r, 1) projects onto s F a(r), which is
    # s f1 away from the face's clip
    rng = np.random.default_rng(int(-r))
    for _ in range(20):
        f = np.exp(rng.uniform(-2, 2, size=3))
        s, t = rng.uniform(0.05, 5.0), rng.uniform(0.1, 5.0)
        E = math.exp(r)
        p = s * f * np.array([r, 1.0, E])
        v = p - t * np.array([-E, (r - 1.0) * E, 1.0]) / f
        got = O.proj_scaled_exp(v, f)
        assert np.allclose(got, p, rtol=0, atol=1e-9 * (1 + np.abs(v).max())), (f, s, t, got, p)


def test_textbook_case_both_leading_coordinates_nonpositive():
    # with x <= 0 and y <= 0 (and v outside K_exp and its polar) the projection
    # onto K_exp is (x, 0, max(z, 0))
    rng = np.random.default_rng(7)
    hits = 0
    for _ in range(300):
        v = np.array([-rng.uniform(0, 3), -rng.uniform(0, 3), rng.normal() * 3])
        if O.in_exp_cone(v) or O.in_exp_dual(-v):
            continue
        hits += 1
        assert np.allclose(O.proj_scaled_exp(v, np.ones(3)), [v[0], 0.0, max(v[2], 0.0)], rtol=0, atol=1e-14)
    assert hits > 100


def test_inside_and_polar_cases():
    f = np.array([2.0, 0.5, 3.0])
    v = f * np.array([0.2, 1.0, 2.0])                     # (0.2, 1, 2) in K_exp
    assert np.array_equal(O.proj_scaled_exp(v, f), v)
    w = -np.array([-1.0, 0.0, 1.0]) / f                   # -F w = (-1, 0, 1) in K_exp*
    assert np.array_equal(O.proj_scaled_exp(w, f), np.zeros(3))


@pytest.mark.parametrize("seed", range(3))
def test_projection_characterization_random(seed):
    # p = P_{F K}(v) iff p in F K, v - p in the polar (-F (v - p) in K*), <p, v - p> = 0
    rng = np.random.default_rng(100 + seed)
    for _ in range(80):
        v = rng.standard_normal(3) * rng.uniform(0.1, 10)
        f = np.exp(rng.uniform(-2, 2, size=3)) if seed else np.ones(3)
        p = O.proj_scaled_exp(v, f)
        d = v - p
        assert near_exp(p / f, 1e-10), (v, f, p)
        assert near_exp_dual(-f * d, 1e-10), (v, f, p)
        assert abs(p @ d) <= 1e-10 * (1 + v @ v)


@pytest.mark.parametrize("seed", range(3))
def test_dual_projection_characterization_random(seed):
    # q = P_{F K*}(v): q in F K*, -F (v - q) in (K*)* = K, <q, v - q> = 0
    rng = np.random.default_rng(200 + seed)
    for _ in range(80):
        v = rng.standard_normal(3) * rng.uniform(0.1, 10)
        f = np.exp(rng.uniform(-2, 2, size=3)) if seed else np.ones(3)
        q = O.proj_scaled_exp_dual(v, f)
        d = v - q
        assert near_exp_dual(q / f, 1e-10), (v, f, q)
        assert near_exp(-f * d, 1e-10), (v, f, q)
        assert abs(q @ d) <= 1e-10 * (1 + v @ v)


def _slsqp_distance(v, f):
    """Distance from v to F K_exp by SLSQP over q = (x, y, z) with y, z > 0 and
    y log(z / y) - x >= 0 (from four starts), against the face {y = 0} by its
    clip; the smallest wins."""
    best = float(np.linalg.norm(v - np.array([min(v[0], 0.0), 0.0, max(v[2], 0.0)])))
    for y0 in (1e-3, 0.1, 1.0, 10.0):
        x0 = np.array([min(v[0] / f[0], 0.0) - 1.0, y0, max(v[2] / f[2], 1.0) + 1.0])
        res = minimize(lambda q: float(np.sum((f * q - v) ** 2)), x0,
                       jac=lambda q: 2 * f * (f * q - v),
                       constraints=[{"type": "ineq", "fun": lambda q: np.array([q[1] * math.log(q[2] / q[1]) - q[0]])}],
                       bounds=[(None, None), (1e-12, None), (1e-12, None)], method="SLSQP",
                       options={"ftol": 1e-15, "maxiter": 2000})
        q = res.x
        if q[1] * math.log(q[2] / q[1]) - q[0] >= -1e-9:
            best = min(best, float(np.linalg.norm(f * q - v)))
    return best


def test_projection_distance_matches_slsqp():
    rng = np.random.default_rng(11)
    for _ in range(40):
        v = rng.standard_normal(3) * 2
        f = np.exp(rng.uniform(-1, 1, size=3))
        if O.in_exp_cone(v / f) or O.in_exp_dual(-f * v):
            continue
        got = float(np.linalg.norm(v - O.proj_scaled_exp(v, f)))
        want = _slsqp_distance(v, f)
        assert abs(got - want) <= 1e-7 * (1 + np.abs(v).max())


def _lp(G, h, c, l, u, m_zero, n_exp=0, n_dexp=0, m_nonneg=0):
    G = sp.csr_matrix(np.asarray(G, dtype=np.float64))
    return O.lpdata_from_arrays(G.shape[0], G.shape[1], m_zero, G.indptr, G.indices, G.data,
                                h, c, l, u, (), n_exp, n_dexp)


def test_hand_problem_exp_epigraph():
    # min z s.t. (0.5, 1, z) in K_exp: z* = e^0.5
    lp = _lp([[0], [0], [1]], [-0.5, -1.0, 0.0], [1.0], [0.0], [10.0], 0, n_exp=1)
    r = O.solve(lp, O.Options(rel_tol=1e-9, abs_tol=1e-9))
    assert r.exit_code == 0
    assert r.pobj == pytest.approx(math.exp(0.5), rel=1e-7)


def test_hand_problem_exp_log():
    # max x s.t. (x, 1, z) in K_exp, z <= 2: x* = log 2
    lp = _lp([[1, 0], [0, 0], [0, 1]], [0.0, -1.0, 0.0], [-1.0, 0.0], [-10.0, 0.0], [10.0, 2.0], 0, n_exp=1)
    r = O.solve(lp, O.Options(rel_tol=1e-9, abs_tol=1e-9))
    assert r.exit_code == 0
    assert r.pobj == pytest.approx(-math.log(2.0), rel=1e-7)
    assert r.x[0] == pytest.approx(math.log(2.0), abs=1e-6)


def test_hand_problem_dual_exp():
    # min w s.t. (-1, 0, w) in K_exp*: 1 <= e w, w* = 1/e
    lp = _lp([[0], [0], [1]], [1.0, 0.0, 0.0], [1.0], [0.0], [10.0], 0, n_dexp=1)
    r = O.solve(lp, O.Options(rel_tol=1e-9, abs_tol=1e-9))
    assert r.exit_code == 0
    assert r.pobj == pytest.approx(1.0 / math.e, rel=1e-7)


def _slsqp_objective(inst):
    """SciPy's SLSQP on the same problem, started from the planted strictly
    feasible point, with each block in a concave form: (x, y, z) in K_exp as
    y log(z / y) - x >= 0, y >= 0, z >= 0, and (u, v, w) in K_exp* as
    v + t - t log(t / w) >= 0 with t = -u >= 0, w >= 0 (the logarithm of
    t e^(-v / t) <= e w, times t)."""
    G = inst.scipy_csr().toarray()
    h, c, mz = inst.h, inst.c, inst.m_zero
    m_cone = inst.m - 3 * (inst.n_exp + inst.n_dexp)
    cons = [{"type": "eq", "fun": lambda x: G[:mz] @ x - h[:mz], "jac": lambda x: G[:mz]},
            {"type": "ineq", "fun": lambda x: G[mz:m_cone] @ x - h[mz:m_cone], "jac": lambda x: G[mz:m_cone]}]
    a = m_cone
    for kind in ["exp"] * inst.n_exp + ["dexp"] * inst.n_dexp:
        Gb, hb = G[a:a + 3], h[a:a + 3]
        if kind == "exp":
            def fq(x, Gb=Gb, hb=hb):
                p, q, r = Gb @ x - hb
                qq, rr = max(q, 1e-12), max(r, 1e-12)
                return np.array([qq * math.log(rr / qq) - p, q, r])

            def jq(x, Gb=Gb, hb=hb):
                p, q, r = Gb @ x - hb
                qq, rr = max(q, 1e-12), max(r, 1e-12)
                return np.vstack([np.array([-1.0, math.log(rr / qq) - 1.0, qq / rr]) @ Gb, Gb[1], Gb[2]])
        else:
            def fq(x, Gb=Gb, hb=hb):
                p, q, r = Gb @ x - hb
                t, rr = max(-p, 1e-12), max(r, 1e-12)
                return np.array([q + t - t * math.log(t / rr), -p, r])

            def jq(x, Gb=Gb, hb=hb):
                p, q, r = Gb @ x - hb
                t, rr = max(-p, 1e-12), max(r, 1e-12)
                return np.vstack([np.array([math.log(t / rr), 1.0, t / rr]) @ Gb, -Gb[0], Gb[2]])
        cons.append({"type": "ineq", "fun": fq, "jac": jq})
        a += 3
    res = minimize(lambda x: c @ x, inst.x_planted, jac=lambda x: c, bounds=list(zip(inst.l, inst.u)),
                   constraints=cons, method="SLSQP", options={"ftol": 1e-14, "maxiter": 3000})
    assert res.status in (0, 8), res.message
    viol = max([float(np.max(np.abs(cn["fun"](res.x)))) if cn["type"] == "eq" else
                max(0.0, -float(np.min(cn["fun"](res.x)))) for cn in cons])
    assert viol <= 1e-7 * (1 + np.abs(h).max())
    return float(res.fun)


def test_exp_instance_planted_point_is_interior():
    inst = lpgen.exp_instance(0, m_zero=8, n=40, m_nonneg=6, n_exp=4, n_dexp=3)
    lp = O.lpdata_from_instance(inst)
    r = lp.G @ inst.x_planted - lp.h
    assert np.allclose(r[:8], 0.0, atol=1e-12)
    assert (r[8:14] > 0).all()
    for kind, a, b in O._cone_blocks(lp.m, (), 4, 3):
        q = r[a:b]
        if kind == "exp":
            assert q[1] > 0 and q[1] * math.exp(q[0] / q[1]) < q[2]
        else:
            assert q[0] < 0 and -q[0] * math.exp(q[1] / q[0]) < math.e * q[2]


@pytest.mark.parametrize("seed", [0, 1])
def test_exp_instance_matches_slsqp(seed):
    inst = lpgen.exp_instance(seed, m_zero=8, n=40, m_nonneg=6, n_exp=4, n_dexp=3)
    lp = O.lpdata_from_instance(inst)
    r = O.solve(lp, O.Options(rel_tol=1e-8, abs_tol=1e-8, time_limit=120))
    assert r.exit_code == 0
    want = _slsqp_objective(inst)
    assert abs(r.pobj - want) / (1 + abs(want)) <= 1e-6
    assert max(r.errors["rel_p"], r.errors["rel_d"], r.errors["rel_gap"]) <= 1e-8


def test_exp_optimum_invariant_under_rescaling():
    inst = lpgen.exp_instance(2, m_zero=8, n=40, m_nonneg=6, n_exp=4, n_dexp=3)
    lp = O.lpdata_from_instance(inst)
    a = O.solve(lp, O.Options(rel_tol=1e-8, abs_tol=1e-8, use_preconditioner=True, time_limit=120))
    b = O.solve(lp, O.Options(rel_tol=1e-8, abs_tol=1e-8, use_preconditioner=False, time_limit=120))
    assert a.exit_code == 0 and b.exit_code == 0
    assert abs(a.pobj - b.pobj) / (1 + abs(b.pobj)) <= 1e-6


def test_rescaled_exp_cones_follow_the_row_factors():
    # rows multiplied by D1: K_d* blocks become diag(D1) K_exp (or K_exp*), K_d
    # blocks diag(1/D1) K_exp* (or K_exp)
    inst = lpgen.exp_instance(3, m_zero=4, n=30, m_nonneg=3, n_exp=2, n_dexp=2)
    lp = O.lpdata_from_instance(inst)
    D1 = np.exp(np.random.default_rng(5).uniform(-2, 2, size=lp.m))
    sl = O.rescale(lp, D1, np.ones(lp.n))
    rng = np.random.default_rng(6)
    for _ in range(20):
        v = rng.standard_normal(lp.m) * 3
        p, q = sl.proj_Kd_star(v), sl.proj_Kd(v)
        for kind, a, b in O._cone_blocks(lp.m, (), 2, 2):
            e = D1[a:b]
            if kind == "exp":
                assert near_exp(p[a:b] / e, 1e-10) and near_exp_dual(q[a:b] * e, 1e-10)
            else:
                assert near_exp_dual(p[a:b] / e, 1e-10) and near_exp(q[a:b] * e, 1e-10)
            # K_d and K_d* blocks are dual cones: their projections of v and -v split v
            r = sl.proj_Kd(-v)
            assert np.allclose(p[a:b] - r[a:b], v[a:b], rtol=0, atol=1e-9 * (1 + np.abs(v[a:b]).max()))


def test_termination_errors_exp_residual_by_hand():
    # rows (0.5, 1, z): at z = e^0.5 the residual is on the boundary; at z = 0 it
    # is 0.5 (0, 1, 1) - 0.5 (-1, -1, 1) = ray(0) / 2 - normal(0) / 2, so its
    # projection is (0, 0.5, 0.5) and the gap (0.5, 0.5, -0.5): abs_p = 0.5,
    # rel_p = 0.5 / (1 + max(||h|| = 1, ||Gx|| = 0, ||proj|| = 0.5))
    lp = _lp([[0], [0], [1]], [-0.5, -1.0, 0.0], [1.0], [0.0], [10.0], 0, n_exp=1)
    e0 = O.termination_errors(lp, np.array([math.exp(0.5)]), np.zeros(3))
    assert e0["abs_p"] <= 1e-12
    e1 = O.termination_errors(lp, np.array([0.0]), np.zeros(3))
    assert e1["abs_p"] == pytest.approx(0.5, abs=1e-12)
    assert e1["rel_p"] == pytest.approx(0.25, abs=1e-12)
