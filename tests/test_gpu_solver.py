"""GPU parity of the HIP solver (through the C ABI) against the FP64 CPU oracle.

Tolerances: the method is an iteration whose restart decisions are
discontinuous in rounding, so full solves are compared through what is unique
(the optimal objective, to 1e-6 relative as the stated bar) and through the
oracle's own evaluation of the KKT errors of the GPU's answer (<= the
requested tolerance).  Deterministic pieces (scaling, the first trials before
any restart check, SpMV) are compared element by element.
"""
import math

import numpy as np
import pytest

import lpgen
from oracle import pdcs_oracle as O

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_15504_amd")


def _gpu_ok():
    return P.pdcs_device_count() > 0


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not _gpu_ok():
        pytest.skip("no GPU visible")


def _rel_kkt(err):
    return max(err["rel_p"], err["rel_d"], err["rel_gap"])


def _check_solution(inst, sol, p_ref, tol=1e-6, obj_tol=1e-6):
    lp = O.lpdata_from_instance(inst)
    err = O.termination_errors(lp, sol.x, sol.y)
    assert sol.info["exit_code"] == 0, sol.info
    assert _rel_kkt(err) <= tol * 1.0001, err
    assert abs(err["pobj"] - p_ref) / (1.0 + abs(p_ref)) <= obj_tol, (err["pobj"], p_ref)
    # the returned slack is c - G^T y of the returned y
    lam = inst.c - lp.G.T @ sol.y
    assert np.allclose(sol.lam, lam, rtol=1e-9, atol=1e-9 * (1 + np.abs(lam).max()))
    return err


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_c0_fp64_matches_oracle(seed):
    inst = lpgen.c0_instance(seed)
    ref = O.solve(O.lpdata_from_instance(inst), O.Options())
    assert ref.exit_code == 0
    prob = P.Problem.from_instance(inst)
    sol = prob.solve(precision="fp64", time_limit=60.0)
    print(f"seed {seed}: gpu iters {sol.info['iters']} restarts {sol.info['restarts']} "
          f"oracle iters {ref.iters} restarts {ref.restarts} time {sol.info['time_sec']:.3f}s", flush=True)
    _check_solution(inst, sol, ref.pobj)


@pytest.mark.parametrize("seed", [0, 1])
def test_c0_mixed_matches_oracle(seed):
    inst = lpgen.c0_instance(seed)
    ref = O.solve(O.lpdata_from_instance(inst), O.Options())
    prob = P.Problem.from_instance(inst)
    sol = prob.solve(precision="mixed", time_limit=60.0)
    print(f"mixed seed {seed}: iters {sol.info['iters']} fp64 iters {sol.info['fp64_iters']}", flush=True)
    _check_solution(inst, sol, ref.pobj)


def test_scaling_matches_oracle():
    inst = lpgen.c4_instance(0, m=300, n=700, per_col=6)
    D1o, D2o = O.ruiz_l2_scaling(inst.scipy_csr(), 10, True)
    prob = P.Problem.from_instance(inst)
    sol = prob.solve(max_iter=1, with_scaling=True)
    assert np.allclose(sol.D1, D1o, rtol=1e-13, atol=0)
    assert np.allclose(sol.D2, D2o, rtol=1e-13, atol=0)


def _edge_lp():
    # >= rows, an empty row, an empty column, and every kind of bound:
    # [l, u], [l, inf), (-inf, u], free
    inst = lpgen.planted_lp(lpgen.rng_for(78, 0), 90, 200, per_col=4, m_zero=50)
    rp, ci, v = inst.row_ptr.copy(), inst.col_idx.copy(), inst.val.copy()
    # empty row 7 and empty column 11
    keep = np.ones(v.size, bool)
    rows = np.repeat(np.arange(inst.m), np.diff(rp))
    keep &= rows != 7
    keep &= ci != 11
    rows, ci, v = rows[keep], ci[keep], v[keep]
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=inst.m))]).astype(np.int64)
    l, u = inst.l.copy(), inst.u.copy()
    j = np.arange(inst.n)
    l[j % 4 == 1] = -np.inf
    u[j % 4 == 2] = np.inf
    l[j % 4 == 3], u[j % 4 == 3] = -np.inf, np.inf
    x0 = inst.x_planted
    h = np.zeros(inst.m)
    np.add.at(h, rows, v * x0[ci])
    h[inst.m_zero:] -= 0.5       # >= rows hold with slack at x0
    # costs that keep the LP bounded: no recession direction lowers c^T x
    c = inst.c.copy()
    c[j % 4 == 1] *= -1.0         # (-inf, u]: decreasing x raises the cost
    c[j % 4 == 3] = 0.0           # free columns
    return lpgen.LPInstance(inst.m, inst.n, inst.m_zero, rp, ci.astype(np.int32), v, h, c, l, u, name="edge")


@pytest.mark.parametrize("layout", ["rows", "bands", "workgroup"])
@pytest.mark.parametrize("mz", [None, 60, "edge"])
def test_first_trials_match_oracle_elementwise(mz, layout):
    # Before the first restart check the iteration is deterministic: after N
    # trials the GPU state must equal the oracle's up to rounding.
    if mz == "edge":
        inst = _edge_lp()
    else:
        inst = lpgen.planted_lp(lpgen.rng_for(77, 1), 120, 300, per_col=4, m_zero=mz)
    lp = O.lpdata_from_instance(inst)
    N = 40
    ref = O.solve(lp, O.Options(max_iter=N, check_every=1000))
    prob = P.Problem.from_instance(inst)
    prob.set_layout(layout)
    sol = prob.solve(precision="fp64", max_iter=N, check_every=1000, keep_state=True)
    st = sol.state
    assert st["kbar"] == ref.state["kbar"] == N
    assert st["k"] == ref.state["k"]
    assert st["omega"] == pytest.approx(ref.state["omega"], rel=1e-14)
    assert st["eta_hat"] == pytest.approx(ref.state["eta_hat"], rel=1e-9)
    for key, okey in (("x", "x"), ("y", "y"), ("x_hat", "x_hat"), ("y_hat", "y_hat"),
                      ("x_a", "x_anchor"), ("y_a", "y_anchor")):
        a, b = st[key], ref.state[okey]
        scale = 1.0 + np.abs(b).max()
        assert np.max(np.abs(a - b)) <= 1e-9 * scale, key


def test_spmv_matches_scipy_power_law():
    torch = pytest.importorskip("torch")
    inst = lpgen.c1_instance(0, m=20000, n=40000, s=1.5, max_len=3000)
    A = inst.scipy_csr()
    prob = P.Problem.from_instance(inst)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(inst.n)
    y = rng.standard_normal(inst.m)
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    yd = torch.tensor(y, dtype=torch.float64, device="cuda")
    out_m = torch.empty(inst.m, dtype=torch.float64, device="cuda")
    out_n = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    prob.spmv(xd.data_ptr(), out_m.data_ptr(), transpose=False, precision="fp64")
    prob.spmv(yd.data_ptr(), out_n.data_ptr(), transpose=True, precision="fp64")
    torch.cuda.synchronize()
    ax = A @ x
    aty = A.T @ y
    bound_m = np.abs(A) @ np.abs(x)
    bound_n = np.abs(A.T) @ np.abs(y)
    # FP64 accumulation in a different order: error <= n_row * eps * sum|a x|
    assert np.all(np.abs(out_m.cpu().numpy() - ax) <= 1e-13 * (1 + bound_m) * 64)
    assert np.all(np.abs(out_n.cpu().numpy() - aty) <= 1e-13 * (1 + bound_n) * 64)
    # FP32 values and vectors, FP64 accumulation
    x32 = torch.tensor(x, dtype=torch.float32, device="cuda")
    o32 = torch.empty(inst.m, dtype=torch.float32, device="cuda")
    prob.spmv(x32.data_ptr(), o32.data_ptr(), transpose=False, precision="mixed")
    torch.cuda.synchronize()
    A32 = A.astype(np.float32).astype(np.float64)
    exact32 = A32 @ x.astype(np.float32).astype(np.float64)
    assert np.all(np.abs(o32.cpu().numpy().astype(np.float64) - exact32) <= 6e-8 * (1 + np.abs(exact32)) + 1e-12 * bound_m)


@pytest.mark.parametrize("seed,m", [(0, 300), (1, 1000)])
def test_first_restart_check_matches_oracle(seed, m):
    # The trajectory is deterministic up to the first restart check, so the
    # radii and normalized duality gaps of both candidates there must agree
    # (bisection tolerance 1e-6 relative), and so must the state.
    inst = lpgen.c1_instance(seed, m=m, n=2 * m)
    lp = O.lpdata_from_instance(inst)
    ref = O.solve(lp, O.Options(max_iter=64, check_every=64))
    assert ref.checks == 1, "the reference must reach its first check"
    c = ref.checks_log[0]
    prob = P.Problem.from_instance(inst)
    sol = prob.solve(precision="fp64", max_iter=64, check_every=64, keep_state=True)
    st = sol.state
    print("gpu", st["r_cur"], st["r_avg"], st["rho_cur"], st["rho_avg"], "oracle", c["r"], c["rho"])
    assert st["r_cur"] == pytest.approx(c["r"]["cur"], rel=1e-9)
    assert st["r_avg"] == pytest.approx(c["r"]["avg"], rel=1e-9)
    assert st["rho_cur"] == pytest.approx(c["rho"]["cur"], rel=2e-5)
    assert st["rho_avg"] == pytest.approx(c["rho"]["avg"], rel=2e-5)


@pytest.mark.parametrize("seed,m", [(0, 300)])
def test_state_before_first_check_matches_oracle(seed, m):
    inst = lpgen.c1_instance(seed, m=m, n=2 * m)
    lp = O.lpdata_from_instance(inst)
    ref = O.solve(lp, O.Options(max_iter=63, check_every=1000))
    prob = P.Problem.from_instance(inst)
    sol = prob.solve(precision="fp64", max_iter=63, check_every=1000, keep_state=True)
    st = sol.state
    assert st["k"] == ref.state["k"] and st["kbar"] == ref.state["kbar"]
    # each eta depends on norms reduced in a different order on the two sides,
    # so the sum of 63 of them agrees to about 1e-12 relative
    assert st["sum_eta"] == pytest.approx(ref.state["SH"], rel=1e-10)
    for key, okey in (("x", "x"), ("y", "y"), ("x_hat", "x_hat"), ("y_hat", "y_hat")):
        a, b = st[key], ref.state[okey]
        assert np.max(np.abs(a - b)) <= 1e-9 * (1.0 + np.abs(b).max()), key


@pytest.mark.parametrize("seed,m,layout", [(0, 300, "rows"), (1, 1000, "rows"), (0, 300, "workgroup")])
def test_first_trials_scalars_match_oracle(seed, m, layout):
    # Per-trial step sizes, acceptance and reflection parameters of the first
    # 64 trials (deterministic up to the first restart check) on a power-law
    # LP, whose SpMV schedules have many workgroups per instance.
    inst = lpgen.c1_instance(seed, m=m, n=2 * m)
    lp = O.lpdata_from_instance(inst)
    ref = O.solve(lp, O.Options(max_iter=64, check_every=64), trace=True)
    prob = P.Problem.from_instance(inst)
    prob.set_layout(layout)
    sol = prob.solve(precision="fp64", max_iter=64, check_every=64, trace_trials=64)
    tr = sol.trace
    assert len(tr) == 64 == len(ref.trace)
    for row, t in zip(tr, ref.trace):
        assert int(row[0]) == t["kbar"]
        assert bool(row[6]) == t["accepted"]
        assert row[1] == pytest.approx(t["eta"], rel=1e-9)
        assert row[7] == pytest.approx(t["eta_next"], rel=1e-9)
        if t["accepted"]:
            assert row[8] == pytest.approx(t["beta"], rel=1e-9, abs=1e-12)


# ---------------------------------------------------------------------------
# Band-tile layout (forced on instances small enough for the oracle)
# ---------------------------------------------------------------------------
def _band_problem(inst):
    prob = P.Problem.from_instance(inst)
    prob.set_layout("bands")
    return prob


@pytest.mark.parametrize("seed,m", [(0, 300), (1, 3000)])
def test_band_layout_first_trials_match_oracle(seed, m):
    inst = lpgen.c1_instance(seed, m=m, n=2 * m)
    lp = O.lpdata_from_instance(inst)
    ref = O.solve(lp, O.Options(max_iter=64, check_every=64), trace=True)
    sol = _band_problem(inst).solve(precision="fp64", max_iter=64, check_every=64, trace_trials=64)
    for row, t in zip(sol.trace, ref.trace):
        assert int(row[0]) == t["kbar"] and bool(row[6]) == t["accepted"]
        assert row[1] == pytest.approx(t["eta"], rel=1e-9)
        assert row[7] == pytest.approx(t["eta_next"], rel=1e-9)
        if t["accepted"]:
            assert row[8] == pytest.approx(t["beta"], rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("maker", ["c1", "dense_runs"])
def test_band_layout_state_matches_oracle(maker):
    # dense_runs puts 64 consecutive gathered indices in one row, so every
    # 64-entry group of its tiles repeats a row: extra accumulator slots, and
    # (256 rows x 63 extras > slot capacity) a band split, are exercised
    inst = lpgen.c1_instance(2, m=2000, n=4000) if maker == "c1" else lpgen.dense_runs_instance(0)
    lp = O.lpdata_from_instance(inst)
    ref = O.solve(lp, O.Options(max_iter=63, check_every=1000))
    sol = _band_problem(inst).solve(precision="fp64", max_iter=63, check_every=1000, keep_state=True)
    st = sol.state
    assert st["k"] == ref.state["k"] and st["kbar"] == ref.state["kbar"]
    # dense_runs amplifies rounding: in the oracle itself, a 1e-16 relative
    # perturbation of its values moves y by 2.6e-11 after 63 trials (c1: 2.6e-13),
    # and its rows of 64 nearly cancelling terms are summed in another order here
    tol = 1e-9 if maker == "c1" else 1e-7
    for key in ("x", "y", "x_hat", "y_hat"):
        a, b = st[key], ref.state[key]
        assert np.max(np.abs(a - b)) <= tol * (1.0 + np.abs(b).max()), key
    # the maintained product G^T y_hat against a direct product of the GPU's own
    # y_hat (its y_hat may differ from the oracle's by the tolerance above)
    D1, D2 = O.ruiz_l2_scaling(lp.G, 10, True)
    Gs = (lp.G.multiply(D1[:, None]).multiply(D2[None, :])).tocsr()
    gty = Gs.T @ st["y_hat"]
    bound = abs(Gs).T @ np.abs(st["y_hat"])
    assert np.all(np.abs(st["gty_hat"] - gty) <= 1e-12 * (1.0 + bound))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_band_layout_solves_c0(precision):
    inst = lpgen.c0_instance(3)
    ref = O.solve(O.lpdata_from_instance(inst), O.Options())
    sol = _band_problem(inst).solve(precision=precision, time_limit=60.0)
    _check_solution(inst, sol, ref.pobj)


def test_band_layout_solves_dense_runs():
    inst = lpgen.dense_runs_instance(1)
    ref = O.solve(O.lpdata_from_instance(inst), O.Options(time_limit=120))
    assert ref.exit_code == 0
    sol = _band_problem(inst).solve(precision="mixed", time_limit=60.0)
    _check_solution(inst, sol, ref.pobj)


@pytest.mark.parametrize("maker", ["c1", "dense_runs", "c1_wide", "dense_cols"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_band_layout_spmv_elementwise(maker, precision):
    # The band SpMV itself, both directions, against scipy.  Each row is summed
    # sequentially per accumulator slot and window, the window sums are stored
    # in the value type and added in FP64, so with u the unit roundoff of the
    # value type the error is at most (len + 4) u sum_j |a_ij x_j|.
    torch = pytest.importorskip("torch")
    if maker == "c1":
        inst = lpgen.c1_instance(3, m=5000, n=10000)
    elif maker == "c1_wide":      # more than 2^18 gathered columns: several windows
        inst = lpgen.c1_instance(4, m=20000, n=600000, max_len=400)
    elif maker == "dense_cols":   # one gathered index with more entries per band than a chunk holds
        inst = lpgen.dense_columns_instance(0)
    else:
        inst = lpgen.dense_runs_instance(2)
    A = inst.scipy_csr()
    prob = _band_problem(inst)
    rng = np.random.default_rng(7)
    dt = torch.float64 if precision == "fp64" else torch.float32
    u = 2.0 ** -53 if precision == "fp64" else 2.0 ** -24
    for transpose in (False, True):
        M = (A.T if transpose else A).tocsr()
        x = rng.standard_normal(M.shape[1])
        if precision == "mixed":
            x = x.astype(np.float32).astype(np.float64)
            M.data = M.data.astype(np.float32).astype(np.float64)
        want = M @ x
        bound = abs(M) @ np.abs(x)
        xin = torch.tensor(x, dtype=dt, device="cuda")
        out = torch.empty(M.shape[0], dtype=dt, device="cuda")
        prob.spmv(xin.data_ptr(), out.data_ptr(), transpose=transpose, precision=precision)
        torch.cuda.synchronize()
        got = out.double().cpu().numpy()
        lens = np.diff(M.indptr)
        err = np.abs(got - want)
        assert np.all(err <= (lens + 4) * u * bound), (transpose, np.max(err / (bound + 1e-300)))



@pytest.fixture(scope="module")
def edge_ref():
    inst = _edge_lp()
    ref = O.solve(O.lpdata_from_instance(inst), O.Options(time_limit=120))
    assert ref.exit_code == 0
    return inst, ref


@pytest.mark.parametrize("layout", ["rows", "bands", "workgroup"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_edge_lp_solves(edge_ref, layout, precision):
    inst, ref = edge_ref
    prob = P.Problem.from_instance(inst)
    prob.set_layout(layout)
    sol = prob.solve(precision=precision, time_limit=60.0)
    _check_solution(inst, sol, ref.pobj)



@pytest.mark.parametrize("variant", ["average", "halpern", "kkt"])
@pytest.mark.parametrize("layout", ["rows", "bands", "workgroup"])
def test_restart_variants_match_oracle(variant, layout):
    # the candidate rules of Section 2.3 (average only, Halpern only) and the
    # KKT restart option, each against the oracle run with the same option
    inst = lpgen.c0_instance(4)
    lp = O.lpdata_from_instance(inst)
    kw = dict(use_kkt_restart=True) if variant == "kkt" else dict(method=variant)
    ref = O.solve(lp, O.Options(time_limit=120, **kw))
    assert ref.exit_code == 0
    prob = P.Problem.from_instance(inst)
    prob.set_layout(layout)
    gkw = dict(use_kkt_restart=1) if variant == "kkt" else dict(method=variant)
    sol = prob.solve(precision="fp64", time_limit=60.0, **gkw)
    print(f"{variant} {layout}: gpu trials {sol.info['iters']} restarts {sol.info['restarts']}, "
          f"oracle {ref.iters} / {ref.restarts}", flush=True)
    _check_solution(inst, sol, ref.pobj)


@pytest.mark.parametrize("variant", ["average", "halpern", "kkt"])
def test_restart_variants_first_check_matches_oracle(variant):
    # deterministic up to the first check: the chosen candidate and restart
    inst = lpgen.c1_instance(0, m=300, n=600)
    lp = O.lpdata_from_instance(inst)
    kw = dict(use_kkt_restart=True) if variant == "kkt" else dict(method=variant)
    ref = O.solve(lp, O.Options(max_iter=64, check_every=64, **kw))
    c = ref.checks_log[0]
    gkw = dict(use_kkt_restart=1) if variant == "kkt" else dict(method=variant)
    sol = P.Problem.from_instance(inst).solve(precision="fp64", max_iter=64, check_every=64, keep_state=True, **gkw)
    st = sol.state
    assert st["chosen"] == (0 if c["chosen"] == "cur" else 1)
    assert sol.info["restarts"] == ref.restarts
    assert st["omega"] == pytest.approx(ref.state["omega"], rel=1e-9)



@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_workgroup_layout_on_global_memory_is_bit_identical_to_rows(precision):
    # an instance too large for LDS: the chunk kernel runs the row-block passes
    # over the same blocks, separated by barriers instead of launches, so every
    # iterate agrees bit for bit, across restart checks too
    inst = lpgen.planted_lp(lpgen.rng_for(5, 0), 2000, 4000, per_col=8, m_zero=600)
    states = {}
    for layout in ("rows", "workgroup"):
        prob = P.Problem.from_instance(inst)
        prob.set_layout(layout)
        states[layout] = prob.solve(precision=precision, max_iter=700, check_every=64, keep_state=True)
    a, b = states["rows"], states["workgroup"]
    assert a.info["iters"] == b.info["iters"] and a.info["restarts"] == b.info["restarts"]
    for key in ("x", "y", "x_hat", "y_hat", "x_a", "y_a"):
        assert np.array_equal(a.state[key], b.state[key]), key


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_workgroup_layout_in_lds_matches_rows(precision):
    # C0 runs out of LDS with one thread per row: the same arithmetic in another
    # summation order, so before the first restart check the iterates agree to
    # rounding (FP64 1e-12, FP32 storage 1e-5 of their scale)
    inst = lpgen.c0_instance(3)
    states = {}
    for layout in ("rows", "workgroup"):
        prob = P.Problem.from_instance(inst)
        prob.set_layout(layout)
        states[layout] = prob.solve(precision=precision, max_iter=63, check_every=1000, keep_state=True)
    a, b = states["rows"], states["workgroup"]
    assert a.info["iters"] == b.info["iters"] == 63
    tol = 1e-12 if precision == "fp64" else 1e-5
    for key in ("x", "y", "x_hat", "y_hat"):
        scale = 1.0 + np.abs(a.state[key]).max()
        assert np.max(np.abs(a.state[key] - b.state[key])) <= tol * scale, key


def test_workgroup_layout_batch_matches_oracle():
    # uneven small instances, one workgroup each, with restarts and compaction
    insts = [lpgen.planted_lp(lpgen.rng_for(90, s), m, 2 * m, per_col=4, m_zero=m // 3)
             for s, m in enumerate((30, 75, 160, 240))]
    b = P.Batch([P.Problem.from_instance(i) for i in insts])
    b.set_layout("workgroup")
    for inst, sol in zip(insts, b.solve(precision="fp64", time_limit=60.0)):
        lp = O.lpdata_from_instance(inst)
        ref = O.solve(lp, O.Options(rel_tol=1e-9, abs_tol=1e-9, time_limit=300))
        err = O.termination_errors(lp, sol.x, sol.y)
        assert sol.info["exit_code"] == 0, sol.info
        assert max(err["rel_p"], err["rel_d"], err["rel_gap"]) <= 1e-6 * 1.0001
        assert abs(err["pobj"] - ref.pobj) / (1 + abs(ref.pobj)) <= 2e-6
