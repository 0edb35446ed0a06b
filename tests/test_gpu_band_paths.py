"""Oracle parity on the band-tile paths that full-size runs take.

The C1 workload runs full-height (8192-row) bands, several gathered-index
windows of 2^18 columns (so the dual and dual-slack epilogues sum P > 1 window
partials inside every trial), and a batch routes small instances' tiles to one
XCD each.  These tests force those shapes at sizes the oracle runs in seconds
and compare what the iteration fixes before its first restart check
(Algorithm 1, Function 2, Algorithm 3): per-trial step sizes, acceptance and
reflection parameters (1e-9), the state after 63 trials (1e-9 of its scale),
and the first check's radii (1e-9) and normalized duality gaps (2e-5, the
bisection tolerance).
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


@pytest.fixture(scope="module")
def wide():
    # 1.2e6 columns: ceil(1.2e6 / 2^18) = 5 windows for G x; 60000 rows in
    # 8 bands of at most 8192 rows (the tile minimum lifted to keep full height)
    inst = lpgen.c1_instance(5, m=60000, n=1_200_000, max_len=400)
    lp = O.lpdata_from_instance(inst)
    ref64 = O.solve(lp, O.Options(max_iter=64, check_every=64), trace=True)
    ref63 = O.solve(lp, O.Options(max_iter=63, check_every=1000))
    return inst, ref64, ref63


def _full_height(inst):
    prob = P.Problem.from_instance(inst)
    prob.set_layout("bands")
    prob.set_band_schedule(rows=8192, min_tiles=1)
    bs = prob.band_schedule()
    assert bs["built_rows"] == 8192 and bs["windows"] == 5, bs
    return prob


def test_full_height_bands_trial_scalars_and_first_check(wide):
    inst, ref, _ = wide
    sol = _full_height(inst).solve(precision="fp64", max_iter=64, check_every=64, trace_trials=64,
                                   keep_state=True)
    assert len(sol.trace) == 64 == len(ref.trace)
    for row, t in zip(sol.trace, ref.trace):
        assert int(row[0]) == t["kbar"] and bool(row[6]) == t["accepted"]
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


def test_full_height_bands_state_after_63_trials(wide):
    inst, _, ref = wide
    sol = _full_height(inst).solve(precision="fp64", max_iter=63, check_every=1000, keep_state=True)
    st = sol.state
    assert st["kbar"] == ref.state["kbar"] == 63 and st["k"] == ref.state["k"]
    for key in ("x", "y", "x_hat", "y_hat"):
        a, b = st[key], ref.state[key]
        assert np.max(np.abs(a - b)) <= 1e-9 * (1.0 + np.abs(b).max()), key


def test_batch_band_routing_state_after_63_trials():
    # one instance with 3 windows (more than 1/16 of the work: spread over the
    # XCDs like a single problem) and 20 small ones (one window each, empty
    # tiles for windows 1-2, every tile of an instance on one XCD)
    big = lpgen.c1_instance(6, m=20000, n=600_000, max_len=400)
    small = lpgen.c2_batch(count=20, m_lo=200, m_hi=2000, seed=7)
    insts = [big] + small
    batch = P.Batch([P.Problem.from_instance(i) for i in insts])
    batch.set_layout("bands")
    assert batch.band_schedule()["windows"] == 3
    sols = batch.solve(precision="fp64", max_iter=63, check_every=1000, keep_state=True, trace_trials=63)
    for k, (inst, sol) in enumerate(zip(insts, sols)):
        ref = O.solve(O.lpdata_from_instance(inst), O.Options(max_iter=63, check_every=1000), trace=(k == 0))
        st = sol.state
        assert st["kbar"] == ref.state["kbar"] and st["k"] == ref.state["k"], k
        for key in ("x", "y", "x_hat", "y_hat"):
            a, b = st[key], ref.state[key]
            assert np.max(np.abs(a - b)) <= 1e-9 * (1.0 + np.abs(b).max()), (k, key)
        if k == 0:
            for row, t in zip(sol.trace, ref.trace):
                assert bool(row[6]) == t["accepted"] and row[1] == pytest.approx(t["eta"], rel=1e-9)
