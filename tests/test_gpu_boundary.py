"""The C ABI's device-pointer calls and restart options on the GPU.

* pdcs_solve_device / pdcs_batch_solve_device (warm start read from device
  memory, FP64 or FP32) give the same solve as the host warm-start calls on
  the same values: the solver is deterministic, so iterates, trial counts and
  outputs match exactly.
* pdcs_result_*_device copy the same outputs as the host getters.
* use_duality_gap_restart = 0 selects the KKT_omega metric like the oracle's
  option, and the restart-frequency options set the check period (option list
  of Section 3); print_freq sets the progress-line period.
"""
import numpy as np
import pytest

import lpgen
from oracle import pdcs_oracle as O

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_15504_amd")
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if P.pdcs_device_count() < 1:
        pytest.skip("no GPU visible")


def _warm(inst, seed=0, noise=0.05):
    """A start near the oracle's solution (the shape of a learned prediction)."""
    ref = O.solve(O.lpdata_from_instance(inst), O.Options())
    rng = np.random.default_rng(seed)
    x0 = ref.x * (1.0 + noise * rng.standard_normal(inst.n))
    y0 = ref.y * (1.0 + noise * rng.standard_normal(inst.m))
    return x0, y0


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("layout", ["rows", "bands", "workgroup"])
def test_device_warm_start_equals_host_warm_start(dtype, layout):
    inst = lpgen.c0_instance(5)
    x0, y0 = _warm(inst)
    if dtype == "float32":   # the device values are FP32: give the host call the same values
        x0 = x0.astype(np.float32).astype(np.float64)
        y0 = y0.astype(np.float32).astype(np.float64)
    prob = P.Problem.from_instance(inst)
    prob.set_layout(layout)
    host = prob.solve(x0=x0, y0=y0, precision="mixed", time_limit=60.0)
    tdt = getattr(torch, dtype)
    dev = prob.solve(x0=torch.tensor(x0, dtype=tdt, device="cuda"),
                     y0=torch.tensor(y0, dtype=tdt, device="cuda"), precision="mixed", time_limit=60.0)
    assert dev.info["exit_code"] == host.info["exit_code"] == 0
    assert dev.info["iters"] == host.info["iters"]
    np.testing.assert_array_equal(dev.x, host.x)
    np.testing.assert_array_equal(dev.y, host.y)


def test_device_warm_start_only_primal_and_nan_rejected():
    inst = lpgen.c0_instance(6)
    x0, _ = _warm(inst)
    prob = P.Problem.from_instance(inst)
    host = prob.solve(x0=x0, precision="fp64", time_limit=60.0)
    dev = prob.solve(x0=torch.tensor(x0, device="cuda"), precision="fp64", time_limit=60.0)
    assert dev.info["iters"] == host.info["iters"]
    np.testing.assert_array_equal(dev.x, host.x)
    bad = torch.tensor(x0, device="cuda")
    bad[7] = float("nan")
    with pytest.raises(P.PdcsError) as e:
        prob.solve(x0=bad, precision="fp64", time_limit=60.0)
    assert e.value.code == -1
    with pytest.raises(ValueError):
        prob.solve(x0=torch.tensor(x0[:-1], device="cuda"))


def test_batch_device_warm_start_from_one_network_output():
    # one [count x (n + m)] FP32 tensor, as the warm-start network produces:
    # each instance reads its row's x and y parts in place
    insts = lpgen.c2_batch(count=6, m_lo=40, m_hi=120, seed=3)
    starts = [_warm(i, seed=k) for k, i in enumerate(insts)]
    width = max(i.n + i.m for i in insts)
    Z = np.zeros((len(insts), width), dtype=np.float32)
    for k, (i, (x0, y0)) in enumerate(zip(insts, starts)):
        Z[k, : i.n] = x0
        Z[k, i.n: i.n + i.m] = y0
    Zd = torch.tensor(Z, device="cuda")
    probs = [P.Problem.from_instance(i) for i in insts]
    batch = P.Batch(probs)
    xs = [Z[k, : i.n].astype(np.float64) for k, i in enumerate(insts)]
    ys = [Z[k, i.n: i.n + i.m].astype(np.float64) for k, i in enumerate(insts)]
    xs[2] = None   # one instance without a primal start
    host = batch.solve(x0s=xs, y0s=ys, precision="mixed", time_limit=60.0)
    dxs = [Zd[k, : i.n] for k, i in enumerate(insts)]
    dys = [Zd[k, i.n: i.n + i.m] for k, i in enumerate(insts)]
    dxs[2] = None
    dev = batch.solve(x0s=dxs, y0s=dys, precision="mixed", time_limit=60.0)
    for h, d in zip(host, dev):
        assert d.info["exit_code"] == h.info["exit_code"] == 0
        assert d.info["iters"] == h.info["iters"]
        np.testing.assert_array_equal(d.x, h.x)
        np.testing.assert_array_equal(d.y, h.y)


def test_host_batch_warm_start_lengths_checked():
    insts = lpgen.c2_batch(count=2, m_lo=40, m_hi=60, seed=4)
    batch = P.Batch([P.Problem.from_instance(i) for i in insts])
    with pytest.raises(ValueError):
        batch.solve(x0s=[np.zeros(insts[0].n - 1), None])
    with pytest.raises(ValueError):
        batch.solve(x0s=[np.zeros(insts[0].n)])


@pytest.mark.parametrize("layout", ["rows", "bands", "workgroup"])
def test_device_results_equal_host_results(layout):
    inst = lpgen.c0_instance(7)
    prob = P.Problem.from_instance(inst)
    prob.set_layout(layout)
    host = prob.solve(precision="fp64", time_limit=60.0)
    dev = prob.solve(precision="fp64", time_limit=60.0, device_out=True)
    assert dev.info["iters"] == host.info["iters"]
    for a, b in ((dev.x, host.x), (dev.y, host.y), (dev.lam, host.lam)):
        assert a.is_cuda and a.dtype == torch.float64
        np.testing.assert_array_equal(a.cpu().numpy(), b)


def test_gap_metric_off_matches_oracle_at_first_check():
    inst = lpgen.c1_instance(0, m=300, n=600)
    lp = O.lpdata_from_instance(inst)
    ref = O.solve(lp, O.Options(max_iter=64, check_every=64, use_duality_gap_restart=False))
    c = ref.checks_log[0]
    sol = P.Problem.from_instance(inst).solve(precision="fp64", max_iter=64, check_every=64, keep_state=True,
                                              use_duality_gap_restart=0)
    st = sol.state
    assert c["use_kkt"] and np.isnan(st["rho_cur"]) and np.isnan(st["rho_avg"])
    assert st["chosen"] == (0 if c["chosen"] == "cur" else 1)
    assert sol.info["restarts"] == ref.restarts
    assert st["omega"] == pytest.approx(ref.state["omega"], rel=1e-9)


def test_gap_metric_off_solves():
    inst = lpgen.c0_instance(3)
    ref = O.solve(O.lpdata_from_instance(inst), O.Options(use_duality_gap_restart=False))
    sol = P.Problem.from_instance(inst).solve(precision="fp64", time_limit=60.0, use_duality_gap_restart=0)
    assert sol.info["exit_code"] == 0
    err = O.termination_errors(O.lpdata_from_instance(inst), sol.x, sol.y)
    assert max(err["rel_p"], err["rel_d"], err["rel_gap"]) <= 1e-6 * 1.0001
    assert abs(err["pobj"] - ref.pobj) / (1 + abs(ref.pobj)) <= 1e-6


def test_restart_frequency_options_set_the_check_period():
    inst = lpgen.c0_instance(3)
    sol = P.Problem.from_instance(inst).solve(precision="fp64", time_limit=60.0, duality_gap_restart_freq=128,
                                              kkt_restart_freq=96)
    assert sol.info["exit_code"] == 0 and sol.info["iters"] % 128 == 0
    assert 0 < sol.info["checks"] <= sol.info["iters"] // 128
    sol = P.Problem.from_instance(inst).solve(precision="fp64", time_limit=60.0, use_kkt_restart=1,
                                              kkt_restart_freq=96, duality_gap_restart_freq=128)
    assert sol.info["exit_code"] == 0 and sol.info["iters"] % 96 == 0


def test_print_freq_sets_progress_lines(capfd):
    inst = lpgen.c0_instance(0)   # needs far more than 1024 trials
    P.Problem.from_instance(inst).solve(precision="fp64", max_iter=1024, check_every=64, verbose=1,
                                        print_freq=256)
    err = capfd.readouterr().err
    assert err.count("[pdcs]") == 4, err
