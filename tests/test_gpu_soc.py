"""GPU parity of second-order-cone rows (socG option of Section 3; the
rescaled-cone projection of Section 2.6) against the FP64 oracle, through the
C ABI.

Before the first restart check an FP64 solve follows the oracle trial by trial:
the per-trial step sizes, acceptance and reflection parameters (1e-9), the
state after 63 trials (1e-9 of its scale) and the first check's radii (1e-9)
and normalized duality gaps (2e-5, the bisection tolerance) are compared.  Whole
solves are compared through what is unique: the oracle's own termination test
of the GPU's answer, and the objective against the oracle's (or a closed form).
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


INSTANCES = {
    # small blocks of several dimensions after equality rows
    "small": lambda: lpgen.soc_instance(0),
    # a 3000-row block (larger than a row range), many 3-row blocks, and
    # equality rows: several row ranges, blocks never split across them
    "wide": lambda: lpgen.soc_instance(4, m_zero=800, n=12000, blocks=(3000,) + (3,) * 20 + (17, 1), per_col=3),
}


@pytest.fixture(scope="module", params=list(INSTANCES))
def case(request):
    inst = INSTANCES[request.param]()
    lp = O.lpdata_from_instance(inst)
    ref64 = O.solve(lp, O.Options(max_iter=64, check_every=64), trace=True)
    ref63 = O.solve(lp, O.Options(max_iter=63, check_every=1000))
    return request.param, inst, ref64, ref63


def test_soc_first_trials_and_check_match_oracle(case):
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


def test_soc_state_after_63_trials_matches_oracle(case):
    name, inst, _, ref = case
    sol = P.Problem.from_instance(inst).solve(precision="fp64", max_iter=63, check_every=1000, keep_state=True,
                                              with_scaling=True)
    st = sol.state
    assert st["kbar"] == ref.state["kbar"] == 63 and st["k"] == ref.state["k"]
    for key in ("x", "y", "x_hat", "y_hat"):
        a, b = st[key], ref.state[key]
        assert np.max(np.abs(a - b)) <= 1e-9 * (1.0 + np.abs(b).max()), (name, key)
    # the dual iterate lies in the rescaled cone: D1 y_hat in K_soc per block
    D1 = sol.D1 if sol.D1 is not None else None
    if D1 is not None:
        yu = D1 * st["y_hat"]
        r = inst.m - sum(inst.soc)
        for d in inst.soc:
            blk = yu[r:r + d]
            assert np.linalg.norm(blk[1:]) <= blk[0] * (1 + 1e-12) + 1e-12
            r += d


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_soc_solve_matches_oracle(precision):
    inst = lpgen.soc_instance(1)
    lp = O.lpdata_from_instance(inst)
    ref = O.solve(lp, O.Options(rel_tol=1e-9, abs_tol=1e-9, time_limit=300))
    assert ref.exit_code == 0
    prob = P.Problem.from_instance(inst)
    for tol in (1e-6, 1e-7):
        sol = prob.solve(precision=precision, time_limit=60.0, rel_tol=tol, abs_tol=tol)
        err = O.termination_errors(lp, sol.x, sol.y)
        print(f"{precision} tol {tol}: exit {sol.info['exit_code']} trials {sol.info['iters']} "
              f"rel KKT {max(err['rel_p'], err['rel_d'], err['rel_gap']):.2e}", flush=True)
        assert sol.info["exit_code"] == 0, sol.info
        assert max(err["rel_p"], err["rel_d"], err["rel_gap"]) <= tol * 1.0001
    # solved to 1e-7 the objective is within 1e-6 of the oracle's 1e-9 answer
    assert abs(err["pobj"] - ref.pobj) / (1 + abs(ref.pobj)) <= 1e-6


def _small_lp(G, h, c, l, u, m_zero, soc):
    G = sp.csr_matrix(np.asarray(G, float))
    return P.Problem(G.shape[0], G.shape[1], m_zero, G.indptr.astype(np.int64), G.indices, G.data,
                     np.asarray(h, float), np.asarray(c, float), np.asarray(l, float), np.asarray(u, float),
                     soc=soc)


def test_soc_hand_problems_on_gpu():
    # nearest point of the line w1 + w2 = 1 to the origin: min t over (t, w) in K_soc
    prob = _small_lp([[0, 1, 1], [1, 0, 0], [0, 1, 0], [0, 0, 1]], [1, 0, 0, 0], [1, 0, 0],
                     [0, -np.inf, -np.inf], [10, np.inf, np.inf], 1, (3,))
    sol = prob.solve(precision="fp64", rel_tol=1e-9, abs_tol=1e-9, time_limit=30.0)
    assert sol.info["exit_code"] == 0 and sol.info["pobj"] == pytest.approx(1 / math.sqrt(2), rel=1e-7)
    # max w1 + w2 over the unit ball
    prob = _small_lp(np.eye(3), [0, 0, 0], [0, -1, -1], [0, -np.inf, -np.inf], [1, np.inf, np.inf], 0, (3,))
    sol = prob.solve(precision="fp64", rel_tol=1e-9, abs_tol=1e-9, time_limit=30.0)
    assert sol.info["exit_code"] == 0 and sol.info["pobj"] == pytest.approx(-math.sqrt(2), rel=1e-7)


def test_soc_batch_with_lp_members_matches_oracle():
    # conic and plain LP instances in one batch (the band layout, per-instance cones)
    insts = [lpgen.soc_instance(s, m_zero=30, n=150, blocks=(3, 4, 9)) for s in (5, 6)]
    insts += [lpgen.c0_instance(7)]
    sols = P.Batch([P.Problem.from_instance(i) for i in insts]).solve(precision="fp64", time_limit=60.0)
    for inst, sol in zip(insts, sols):
        lp = O.lpdata_from_instance(inst)
        err = O.termination_errors(lp, sol.x, sol.y)
        assert sol.info["exit_code"] == 0, sol.info
        assert max(err["rel_p"], err["rel_d"], err["rel_gap"]) <= 1e-6 * 1.0001
        ref = O.solve(lp, O.Options(rel_tol=1e-9, abs_tol=1e-9, time_limit=300))
        # a relative KKT error of 1e-6 bounds the gap by 1e-6 (1 + max |obj|), and the
        # residuals move the objective by as much again: 2e-6 against the 1e-9 answer
        assert abs(err["pobj"] - ref.pobj) / (1 + abs(ref.pobj)) <= 2e-6


def test_conic_create_rejects_bad_blocks():
    inst = lpgen.soc_instance(0)
    for soc in ((0,), (inst.m,), (inst.m - inst.m_zero + 1,)):
        with pytest.raises(P.PdcsError):
            P.Problem(inst.m, inst.n, inst.m_zero, inst.row_ptr, inst.col_idx, inst.val, inst.h, inst.c,
                      inst.l, inst.u, soc=soc)


@pytest.mark.parametrize("d", [1, 2, 3, 9, 50, 64, 65, 200])
def test_soc_projection_matches_oracle_elementwise(d):
    # the device projection onto diag(e) K_soc against the oracle's, on random
    # points and factors, with zero leading entries and zero entries of w
    # among them (v_0 = 0 starts the multiplier search at a zero denominator)
    rng = np.random.default_rng(d)
    cnt = 300
    v = rng.standard_normal((cnt, d)) * rng.uniform(0.1, 10, size=(cnt, 1))
    e = np.exp(rng.uniform(-3, 3, size=(cnt, d)))
    v[::3, 0] = 0.0
    if d > 2:
        v[::2, 1] = 0.0
    e[::4] = 1.0
    got = P.pdcs_project_cone("soc", v, e)
    for q in range(cnt):
        want = O.proj_scaled_soc(v[q], e[q])
        assert np.all(np.isfinite(got[q]))
        assert np.max(np.abs(got[q] - want)) <= 1e-10 * (1 + np.abs(v[q]).max()), (q, v[q], got[q], want)
