"""GPU parity of the batched solver (many LPs of uneven size in one
block-diagonal launch sequence with per-instance state) against the FP64 CPU
oracle run on each instance alone.

Each instance of a batch must reach what it reaches alone: the oracle's KKT
evaluation of its answer within the tolerance and the objective within 1e-6 of
the oracle's.  Deterministic pieces are compared exactly: the first trials of a
batch member against the oracle's trace, and graph-captured against eagerly
launched chunks (same kernels, same order: identical bits).
"""
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


def _small_c2(count, seed, m_lo=40, m_hi=400):
    # the C2 recipe (8 distinct rows per column, n = 2m, m log-uniform) at sizes
    # the oracle finishes in seconds
    return lpgen.c2_batch(count=count, m_lo=m_lo, m_hi=m_hi, per_col=8, seed=seed)


@pytest.fixture(scope="module")
def refs():
    insts = _small_c2(6, 7)
    out = []
    for inst in insts:
        r = O.solve(O.lpdata_from_instance(inst), O.Options(time_limit=120))
        assert r.exit_code == 0, inst.name
        out.append(r)
    return insts, out


def _check(inst, sol, p_ref, tol=1e-6):
    lp = O.lpdata_from_instance(inst)
    err = O.termination_errors(lp, sol.x, sol.y)
    assert sol.info["exit_code"] == 0, sol.info
    assert max(err["rel_p"], err["rel_d"], err["rel_gap"]) <= tol * 1.0001, err
    assert abs(err["pobj"] - p_ref) / (1.0 + abs(p_ref)) <= 1e-6


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_matches_oracle_per_instance(refs, precision):
    insts, rs = refs
    probs = [P.Problem.from_instance(i) for i in insts]
    sols = P.Batch(probs).solve(precision=precision, time_limit=120.0)
    for inst, sol, r in zip(insts, sols, rs):
        print(f"{inst.name} m={inst.m}: gpu trials {sol.info['iters']} oracle {r.iters}", flush=True)
        _check(inst, sol, r.pobj)
    # instances finish on their own schedules
    assert len({s.info["iters"] for s in sols}) > 1


def test_batch_member_first_trials_match_oracle(refs):
    insts, _ = refs
    lp = O.lpdata_from_instance(insts[0])
    ref = O.solve(lp, O.Options(max_iter=64, check_every=64), trace=True)
    sols = P.Batch([P.Problem.from_instance(i) for i in insts]).solve(
        precision="fp64", max_iter=64, check_every=64, trace_trials=64)
    tr = sols[0].trace
    assert len(tr) == len(ref.trace) == 64
    for row, t in zip(tr, ref.trace):
        assert int(row[0]) == t["kbar"] and bool(row[6]) == t["accepted"]
        assert row[1] == pytest.approx(t["eta"], rel=1e-9)
        assert row[7] == pytest.approx(t["eta_next"], rel=1e-9)


def test_batch_graph_equals_eager(refs):
    insts, _ = refs
    b = P.Batch([P.Problem.from_instance(i) for i in insts])
    g = b.solve(precision="mixed", max_iter=3000, use_graph=1)
    e = b.solve(precision="mixed", max_iter=3000, use_graph=0)
    for sg, se in zip(g, e):
        assert sg.info["iters"] == se.info["iters"]
        assert np.array_equal(sg.x, se.x) and np.array_equal(sg.y, se.y)


def test_batch_autotuned_schedule_still_matches(refs):
    insts, rs = refs
    b = P.Batch([P.Problem.from_instance(i) for i in insts])
    sched = b.autotune(200.0)
    assert all(v > 0 for v in sched)
    sols = b.solve(precision="mixed", time_limit=120.0)
    for inst, sol, r in zip(insts, sols, rs):
        _check(inst, sol, r.pobj)


def test_batch_band_schedule_autotuned_still_matches(refs):
    # with band tiles the autotuner also times band height, tile minimum and
    # entry cap (rebuilding the band layouts); the chosen one is a candidate and
    # the batch still solves to the oracle's answers
    insts, rs = refs
    b = P.Batch([P.Problem.from_instance(i) for i in insts])
    b.set_layout("bands")
    before = b.band_schedule()
    b.autotune(60000.0)
    after = b.band_schedule()
    cands = {(before["rows"], before["min_tiles"], before["entry_cap"]),
             (before["rows"], before["min_tiles"], max(1024, before["entry_cap"] // 2)),
             (before["rows"], before["min_tiles"], before["entry_cap"] * 2),
             (before["rows"], before["min_tiles"] * 2, before["entry_cap"]),
             (max(256, before["rows"] // 2), before["min_tiles"], before["entry_cap"])}
    assert (after["rows"], after["min_tiles"], after["entry_cap"]) in cands
    assert after["built_rows"] > 0
    sols = b.solve(precision="mixed", time_limit=120.0)
    for inst, sol, r in zip(insts, sols, rs):
        _check(inst, sol, r.pobj)


@pytest.mark.parametrize("sched", [(1, 1024, 256), (64, 65536, 8192)])
def test_batch_schedule_extremes(refs, sched):
    insts, rs = refs
    b = P.Batch([P.Problem.from_instance(i) for i in insts[:3]])
    b.set_schedule(*sched)
    sols = b.solve(precision="fp64", time_limit=120.0)
    for inst, sol, r in zip(insts[:3], sols, rs[:3]):
        _check(inst, sol, r.pobj)


def test_batch_warm_start_from_solutions(refs):
    insts, rs = refs
    b = P.Batch([P.Problem.from_instance(i) for i in insts])
    cold = b.solve(precision="fp64", time_limit=120.0)
    warm = b.solve([r.x for r in rs], [r.y for r in rs], precision="fp64", time_limit=120.0)
    for inst, c, w, r in zip(insts, cold, warm, rs):
        _check(inst, w, r.pobj)
        assert w.info["iters"] <= c.info["iters"]


def test_batch_of_one_equals_single_solve(refs):
    insts, _ = refs
    p = P.Problem.from_instance(insts[1])
    s1 = p.solve(precision="fp64", max_iter=2000)
    s2 = P.Batch([P.Problem.from_instance(insts[1])]).solve(precision="fp64", max_iter=2000)[0]
    assert s1.info["iters"] == s2.info["iters"]
    assert np.array_equal(s1.x, s2.x) and np.array_equal(s1.y, s2.y)


def test_batch_compaction_is_exact():
    # 12 LPs of uneven difficulty: the schedules are rebuilt over the active
    # instances as they finish; every instance keeps exactly its own blocks,
    # so results are bitwise those of the uncompacted run
    insts = _small_c2(12, 9, m_lo=30, m_hi=300)
    b = P.Batch([P.Problem.from_instance(i) for i in insts])
    a = b.solve(precision="mixed", compact=1, time_limit=120.0)
    c = b.solve(precision="mixed", compact=0, time_limit=120.0)
    its = [s.info["iters"] for s in a]
    assert max(its) > 2 * min(its)
    for sa, sc in zip(a, c):
        assert sa.info["iters"] == sc.info["iters"] and sa.info["exit_code"] == sc.info["exit_code"]
        assert np.array_equal(sa.x, sc.x) and np.array_equal(sa.y, sc.y)
    for inst, sa in list(zip(insts, a))[:3]:
        ref = O.solve(O.lpdata_from_instance(inst), O.Options(time_limit=120))
        _check(inst, sa, ref.pobj)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_band_layout_matches_oracle(refs, precision):
    # band tiles per instance (own bands and windows), per-instance gating of
    # the band kernel, window sums combined by the instance-aware epilogues
    insts, rs = refs
    b = P.Batch([P.Problem.from_instance(i) for i in insts])
    b.set_layout("bands")
    sols = b.solve(precision=precision, time_limit=120.0)
    for inst, sol, r in zip(insts, sols, rs):
        _check(inst, sol, r.pobj)


def test_batch_band_layout_first_trials_match_oracle(refs):
    insts, _ = refs
    lp = O.lpdata_from_instance(insts[0])
    ref = O.solve(lp, O.Options(max_iter=64, check_every=64), trace=True)
    b = P.Batch([P.Problem.from_instance(i) for i in insts])
    b.set_layout("bands")
    tr = b.solve(precision="fp64", max_iter=64, check_every=64, trace_trials=64)[0].trace
    for row, t in zip(tr, ref.trace):
        assert int(row[0]) == t["kbar"] and bool(row[6]) == t["accepted"]
        assert row[1] == pytest.approx(t["eta"], rel=1e-9)
        if t["accepted"]:
            assert row[8] == pytest.approx(t["beta"], rel=1e-9, abs=1e-12)


def test_batch_band_layout_mixed_precisions_and_compaction():
    # 12 instances, mixed precision with an early polish switch: instances run
    # in FP32 and FP64 side by side, finish at different times, and the band
    # kernels skip instances in the other precision
    insts = _small_c2(12, 10, m_lo=30, m_hi=300)
    b = P.Batch([P.Problem.from_instance(i) for i in insts])
    b.set_layout("bands")
    sols = b.solve(precision="mixed", polish_switch_tol=1e-4, time_limit=120.0)
    assert any(0 < s.info["fp64_iters"] < s.info["iters"] for s in sols)
    for inst, s in zip(insts, sols):
        lp = O.lpdata_from_instance(inst)
        err = O.termination_errors(lp, s.x, s.y)
        assert s.info["exit_code"] == 0
        assert max(err["rel_p"], err["rel_d"], err["rel_gap"]) <= 1e-6 * 1.0001
