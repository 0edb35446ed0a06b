"""GPU parity of exponential-cone rows (expG and dual_expG options of
Section 3; the rescaled-cone projection of Section 2.6) against the FP64
oracle, through the C ABI.

The projection itself (pdcs_project_cone, the device function the solver
calls) is compared element by element with the oracle's on random points and
factors, and with points whose projection is known by construction.  Before
the first restart check an FP64 solve follows the oracle trial by trial (step
sizes, acceptance and reflection parameters to 1e-9, the state after 63 trials
to 1e-9 of its scale, the first check's radii to 1e-9 and normalized gaps to
2e-5, the bisection tolerance).  Whole solves are compared through what is
unique: the oracle's termination test of the GPU's answer, and the objective
against the oracle's or a closed form.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import lpgen
from oracle import pdcs_oracle as O

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_15504_amd")


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if P.pdcs_device_count() < 1:
        pytest.skip("no GPU visible")


def _points(seed, count, scaled):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((count, 3)) * rng.uniform(0.1, 10, size=(count, 1))
    f = np.exp(rng.uniform(-2, 2, size=(count, 3))) if scaled else np.ones((count, 3))
    return v, f


@pytest.mark.parametrize("dual", [0, 1])
@pytest.mark.parametrize("scaled", [False, True])
def test_projection_matches_oracle_elementwise(dual, scaled):
    v, f = _points(10 + dual + 2 * scaled, 700, scaled)
    got = P.pdcs_project_cone("exp_dual" if dual else "exp", v, f)
    ref = O.proj_scaled_exp_dual if dual else O.proj_scaled_exp
    for q in range(v.shape[0]):
        want = ref(v[q], f[q])
        assert np.max(np.abs(got[q] - want)) <= 1e-10 * (1 + np.abs(v[q]).max()), (q, v[q], f[q], got[q], want)


def test_projection_of_ray_plus_normal_is_the_ray_point():
    # s F (r, 1, e^r) - t F^-1 (-1, r - 1, e^-r) projects onto s F (r, 1, e^r)
    rng = np.random.default_rng(3)
    n = 300
    r = rng.uniform(-6, 4, size=n)
    s, t = rng.uniform(0.05, 5.0, size=n), rng.uniform(0.0, 5.0, size=n)
    f = np.exp(rng.uniform(-2, 2, size=(n, 3)))
    a = np.stack([r, np.ones(n), np.exp(r)], axis=1)
    nr = np.stack([-np.ones(n), r - 1.0, np.exp(-r)], axis=1)
    p = s[:, None] * f * a
    v = p - t[:, None] * nr / f
    got = P.pdcs_project_cone("exp", v, f)
    assert np.all(np.abs(got - p) <= 1e-9 * (1 + np.abs(v).max(axis=1, keepdims=True)))
    # Moreau: the dual cone of F K_exp is F^-1 K_exp*, and P_{F^-1 K_exp*}(-v) = P_{F K_exp}(v) - v
    got_d = P.pdcs_project_cone("exp_dual", -v, 1.0 / f)
    assert np.all(np.abs(got_d - (-v + p)) <= 1e-9 * (1 + np.abs(v).max(axis=1, keepdims=True)))


def test_projection_near_the_apex_is_the_ray_point():
    # the same construction with s a billionth of t: p is within 1e-7 |v| of
    # the apex, where its distance from v and the face clip's agree to
    # rounding; the certificate, not the distance, must pick p
    rng = np.random.default_rng(11)
    n = 400
    r = rng.uniform(-8, 5, size=n)
    t = rng.uniform(0.1, 10.0, size=n)
    s = t * 10.0 ** rng.uniform(-10, -7, size=n)
    f = np.exp(rng.uniform(-2, 2, size=(n, 3)))
    a = np.stack([r, np.ones(n), np.exp(r)], axis=1)
    nr = np.stack([-np.minimum(1.0, np.exp(r)), (r - 1.0) * np.minimum(1.0, np.exp(r)),
                   np.minimum(1.0, np.exp(r)) * np.exp(-r)], axis=1)
    p = s[:, None] * f * a
    v = p - t[:, None] * nr / f
    scale = np.abs(v).max(axis=1, keepdims=True)
    got = P.pdcs_project_cone("exp", v, f)
    assert np.all(np.abs(got - p) <= 1e-12 * scale)
    want = np.array([O.proj_scaled_exp(v[i], f[i]) for i in range(n)])
    assert np.all(np.abs(got - want) <= 1e-12 * scale)
    got_d = P.pdcs_project_cone("exp_dual", -v, 1.0 / f)
    assert np.all(np.abs(got_d - (-v + p)) <= 1e-12 * scale)


def test_projection_onto_far_negative_and_far_positive_rays():
    # rays below the scanned range (r < -300) and near its ends; the normal
    # taken times min(1, e^r) to stay finite
    rng = np.random.default_rng(4)
    r = np.concatenate([-rng.uniform(290, 2000, size=200), rng.uniform(-60, 40, size=200)])
    n = r.size
    s, t = rng.uniform(0.05, 5.0, size=n), rng.uniform(0.1, 5.0, size=n)
    f = np.exp(rng.uniform(-2, 2, size=(n, 3)))
    E = np.exp(r)
    a = np.stack([r, np.ones(n), E], axis=1)
    sc = np.minimum(1.0, E)
    nr = np.stack([-sc, (r - 1.0) * sc, np.where(r < 0, 1.0, np.exp(-np.maximum(r, 0.0)))], axis=1)
    p = s[:, None] * f * a
    v = p - t[:, None] * nr / f
    got = P.pdcs_project_cone("exp", v, f)
    tol = 1e-9 * (1 + np.abs(v).max(axis=1))
    bad = np.nonzero(np.abs(got - p).max(axis=1) > tol)[0]
    assert bad.size == 0, (r[bad[:5]], got[bad[:5]], p[bad[:5]])


def test_projection_special_cases():
    f = np.ones(3)
    v = np.array([[0.2, 1.0, 2.0],        # inside K_exp: itself
                  [1.0, 1.0, -3.0],       # -v = (-1, -1, 3) in K_exp*: the polar, 0
                  [-1.0, -2.0, 0.5],      # x, y <= 0: (x, 0, max(z, 0))
                  [-1.0, -2.0, -0.5],
                  [0.0, 0.0, 0.0]])
    got = P.pdcs_project_cone("exp", v, f)
    assert np.array_equal(got[0], v[0])
    assert np.array_equal(got[1], np.zeros(3))
    assert np.allclose(got[2], [-1.0, 0.0, 0.5], rtol=0, atol=1e-15)
    assert np.allclose(got[3], [-1.0, 0.0, 0.0], rtol=0, atol=1e-15)
    assert np.array_equal(got[4], np.zeros(3))
    assert P.pdcs_project_cone("exp", np.zeros((0, 3)), f).shape == (0, 3)
    with pytest.raises(P.PdcsError):
        P.pdcs_project_cone("exp", v, np.array([1.0, 0.0, 1.0]))
    with pytest.raises(P.PdcsError):
        P.pdcs_project_cone("exp", np.ones((2, 4)), np.ones(4))   # exponential cones have dimension 3


def _with_soc(inst, k):
    # the last k nonnegative rows as second-order-cone blocks of dimension 1
    # (K_soc of dimension 1 is R+): the same problem, with all three cone kinds
    inst.soc = (1,) * k
    return inst


INSTANCES = {
    "small": lambda: lpgen.exp_instance(0),
    # several row ranges, exponential blocks across a range boundary, and
    # second-order-cone blocks before them
    "mixed": lambda: _with_soc(lpgen.exp_instance(4, m_zero=1500, n=3000, m_nonneg=600, n_exp=60, n_dexp=40), 9),
}


def near_exp(q, tol):
    x, y, z = (float(t) for t in q)
    s = tol * (1.0 + max(abs(x), abs(y), abs(z)))
    if y <= s and x <= s and z >= -s and y >= -s:
        return True
    return any(yy > 0.0 and yy * math.exp(min((x - s) / yy, 700.0)) <= z + s for yy in (y - s, y, y + s))


def near_exp_dual(q, tol):
    u, v, w = (float(t) for t in q)
    s = tol * (1.0 + max(abs(u), abs(v), abs(w)))
    if u >= -s and u <= s and v >= -s and w >= -s:
        return True
    return any(uu < 0.0 and -uu * math.exp(min((v + s) / uu, 700.0)) <= math.e * (w + s) for uu in (u - s, u, u + s))


@pytest.fixture(scope="module", params=list(INSTANCES))
def case(request):
    inst = INSTANCES[request.param]()
    lp = O.lpdata_from_instance(inst)
    ref64 = O.solve(lp, O.Options(max_iter=64, check_every=64), trace=True)
    ref63 = O.solve(lp, O.Options(max_iter=63, check_every=1000))
    return request.param, inst, ref64, ref63


def test_exp_first_trials_and_check_match_oracle(case):
    name, inst, ref, _ = case
    sol = P.Problem.from_instance(inst).solve(precision="fp64", max_iter=64, check_every=64, trace_trials=64,
                                              keep_state=True)
    assert len(sol.trace) == 64 == len(ref.trace)
    for row, t in zip(sol.trace, ref.trace):
        assert int(row[0]) == t["kbar"] and bool(row[6]) == t["accepted"], name
        assert row[1] == pytest.approx(t["eta"], rel=1e-9)
        assert row[7] == pytest.approx(t["eta_next"], rel=1e-9)
        if t["accepted"]:
            assert row[8] == pytest.approx(t["beta"], rel=1e-9, abs=1e-12)
    c = ref.checks_log[0]
    st = sol.state
    assert st["r_cur"] == pytest.approx(c["r"]["cur"], rel=1e-9)
    assert st["r_avg"] == pytest.approx(c["r"]["avg"], rel=1e-9)
    assert st["rho_cur"] == pytest.approx(c["rho"]["cur"], rel=2e-5)
    assert st["rho_avg"] == pytest.approx(c["rho"]["avg"], rel=2e-5)
    assert st["chosen"] == (0 if c["chosen"] == "cur" else 1)


def test_exp_state_after_63_trials_matches_oracle(case):
    name, inst, _, ref = case
    sol = P.Problem.from_instance(inst).solve(precision="fp64", max_iter=63, check_every=1000, keep_state=True,
                                              with_scaling=True)
    st = sol.state
    assert st["kbar"] == ref.state["kbar"] == 63 and st["k"] == ref.state["k"]
    for key in ("x", "y", "x_hat", "y_hat"):
        a, b = st[key], ref.state[key]
        assert np.max(np.abs(a - b)) <= 1e-9 * (1.0 + np.abs(b).max()), (name, key)
    # the unscaled dual iterate lies in the dual cone of each block
    yu = sol.D1 * st["y_hat"]
    for kind, a, b in O._cone_blocks(inst.m, inst.soc, inst.n_exp, inst.n_dexp):
        if kind == "exp":
            assert near_exp_dual(yu[a:b], 1e-12), (a, yu[a:b])
        elif kind == "dexp":
            assert near_exp(yu[a:b], 1e-12), (a, yu[a:b])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_exp_solve_matches_oracle(precision):
    inst = lpgen.exp_instance(1)
    lp = O.lpdata_from_instance(inst)
    ref = O.solve(lp, O.Options(rel_tol=1e-8, abs_tol=1e-8, time_limit=300))
    assert ref.exit_code == 0
    prob = P.Problem.from_instance(inst)
    for tol in (1e-6, 1e-7):
        sol = prob.solve(precision=precision, time_limit=60.0, rel_tol=tol, abs_tol=tol)
        err = O.termination_errors(lp, sol.x, sol.y)
        print(f"{precision} tol {tol}: exit {sol.info['exit_code']} trials {sol.info['iters']} "
              f"rel KKT {max(err['rel_p'], err['rel_d'], err['rel_gap']):.2e}", flush=True)
        assert sol.info["exit_code"] == 0, sol.info
        assert max(err["rel_p"], err["rel_d"], err["rel_gap"]) <= tol * 1.0001
    assert abs(err["pobj"] - ref.pobj) / (1 + abs(ref.pobj)) <= 2e-6


def _small_lp(G, h, c, l, u, n_exp=0, n_dexp=0):
    G = sp.csr_matrix(np.asarray(G, float))
    return P.Problem(G.shape[0], G.shape[1], 0, G.indptr.astype(np.int64), G.indices, G.data,
                     np.asarray(h, float), np.asarray(c, float), np.asarray(l, float), np.asarray(u, float),
                     n_exp=n_exp, n_dexp=n_dexp)


def test_exp_hand_problems_on_gpu():
    # min z s.t. (0.5, 1, z) in K_exp: e^0.5
    sol = _small_lp([[0], [0], [1]], [-0.5, -1.0, 0.0], [1.0], [0.0], [10.0], n_exp=1).solve(
        precision="fp64", rel_tol=1e-9, abs_tol=1e-9, time_limit=30.0)
    assert sol.info["exit_code"] == 0 and sol.info["pobj"] == pytest.approx(math.exp(0.5), rel=1e-7)
    # max x s.t. (x, 1, z) in K_exp, z <= 2: log 2
    sol = _small_lp([[1, 0], [0, 0], [0, 1]], [0.0, -1.0, 0.0], [-1.0, 0.0], [-10.0, 0.0], [10.0, 2.0],
                    n_exp=1).solve(precision="fp64", rel_tol=1e-9, abs_tol=1e-9, time_limit=30.0)
    assert sol.info["exit_code"] == 0 and sol.info["pobj"] == pytest.approx(-math.log(2.0), rel=1e-7)
    # min w s.t. (-1, 0, w) in K_exp*: 1/e
    sol = _small_lp([[0], [0], [1]], [1.0, 0.0, 0.0], [1.0], [0.0], [10.0], n_dexp=1).solve(
        precision="fp64", rel_tol=1e-9, abs_tol=1e-9, time_limit=30.0)
    assert sol.info["exit_code"] == 0 and sol.info["pobj"] == pytest.approx(1.0 / math.e, rel=1e-7)


def test_exp_batch_with_lp_and_soc_members_matches_oracle():
    insts = [lpgen.exp_instance(s, m_zero=20, n=120, m_nonneg=10, n_exp=6, n_dexp=5) for s in (5, 6)]
    insts += [lpgen.soc_instance(7, m_zero=30, n=150, blocks=(3, 4, 9)), lpgen.c0_instance(7)]
    sols = P.Batch([P.Problem.from_instance(i) for i in insts]).solve(precision="fp64", time_limit=60.0)
    for inst, sol in zip(insts, sols):
        lp = O.lpdata_from_instance(inst)
        err = O.termination_errors(lp, sol.x, sol.y)
        assert sol.info["exit_code"] == 0, sol.info
        assert max(err["rel_p"], err["rel_d"], err["rel_gap"]) <= 1e-6 * 1.0001
        ref = O.solve(lp, O.Options(rel_tol=1e-9, abs_tol=1e-9, time_limit=300))
        assert abs(err["pobj"] - ref.pobj) / (1 + abs(ref.pobj)) <= 2e-6


def test_cones_create_rejects_bad_blocks():
    inst = lpgen.exp_instance(0)
    free = inst.m - inst.m_zero
    for n_exp, n_dexp in ((-1, 0), (0, -1), (free // 3 + 1, 0), (free // 3, 1)):
        with pytest.raises(P.PdcsError):
            P.Problem(inst.m, inst.n, inst.m_zero, inst.row_ptr, inst.col_idx, inst.val, inst.h, inst.c,
                      inst.l, inst.u, n_exp=n_exp, n_dexp=n_dexp)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_infeasible_exp_lp_exit_code_and_ratios_match_oracle(precision):
    # an exponential-cone LP with an equality row beyond the box: the
    # infeasibility rays cross the cone rows (projections onto K_exp and K_exp*)
    inst = lpgen.infeasible_exp_sum_row(1)
    ref = O.solve(O.lpdata_from_instance(inst), O.Options(max_iter=20000))
    assert ref.exit_code == O.EXIT_PRIMAL_INFEASIBLE_HIGH_ACC and ref.iters == 64
    sol = P.Problem.from_instance(inst).solve(precision=precision, max_iter=20000, time_limit=60.0, keep_state=True)
    assert sol.info["exit_code"] == ref.exit_code and sol.info["iters"] == 64
    if precision == "fp64":
        c = ref.checks_log[0]
        for key in ("ratio_p", "ratio_d"):
            want, got = c[key], sol.state[key]
            if math.isinf(want):
                assert math.isinf(got), (key, got)
            else:
                assert got == pytest.approx(want, rel=1e-9, abs=1e-300), key
