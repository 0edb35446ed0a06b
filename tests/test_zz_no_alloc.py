"""pdcs_problem_spmv_noalloc through the C ABI: the allocation-free plain
product gives exactly the output of pdcs_problem_spmv (same kernels, window
partial sums in the library's file-scope device array instead of the
problem's buffer), on two calls in a row where the second problem is smaller,
in both layouts, both precisions and both directions; a product whose partial
sums exceed the array is refused with PDCS_ERR_SIZE.
"""
import numpy as np
import pytest

import lpgen

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_15504_amd")
torch = pytest.importorskip("torch")

PDCS_ERR_SIZE = -5


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if P.pdcs_device_count() < 1:
        pytest.skip("no GPU visible")


def _both(prob, inst, transpose, precision, seed):
    """(pdcs_problem_spmv output, pdcs_problem_spmv_noalloc output, host FP64 product)."""
    dt = torch.float64 if precision == "fp64" else torch.float32
    n_in, n_out = (inst.m, inst.n) if transpose else (inst.n, inst.m)
    g = torch.Generator().manual_seed(seed)
    x = torch.randn(n_in, generator=g, dtype=torch.float64).to(dt).cuda()
    ref = torch.full((n_out,), float("nan"), dtype=dt, device="cuda")
    got = torch.full((n_out,), float("nan"), dtype=dt, device="cuda")
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        prob.spmv(x.data_ptr(), ref.data_ptr(), transpose=transpose, precision=precision, stream=st.cuda_stream)
        P.pdcs_problem_spmv_noalloc(prob.handle, 1 if transpose else 0, P.PRECISION[precision], x.data_ptr(),
                                    got.data_ptr(), st.cuda_stream)
    st.synchronize()
    G = inst.scipy_csr()
    xv = x.double().cpu().numpy()
    host = (G.T @ xv) if transpose else (G @ xv)
    return ref.cpu(), got.cpu(), host


def _problem(inst, layout):
    prob = P.Problem.from_instance(inst)
    prob.set_layout(layout)
    return prob


@pytest.mark.parametrize("layout", ["bands", "rows"])
def test_noalloc_matches_spmv_on_two_calls_second_smaller(layout):
    # first: 5 windows of 2^18 gathered columns for G x; second: a smaller
    # problem (2 windows), so stale partial sums of the first call would show
    big = lpgen.c1_instance(5, m=60000, n=1_200_000, max_len=400)
    small = lpgen.c1_instance(6, m=20000, n=300_000, max_len=200)
    for k, inst in enumerate((big, small)):
        prob = _problem(inst, layout)
        if layout == "bands":
            assert prob.band_schedule()["windows"] == (5 if k == 0 else 2)
        for transpose in (False, True):
            for precision in ("fp64", "mixed"):
                ref, got, host = _both(prob, inst, transpose, precision, seed=10 * k + 2 * transpose)
                print(f"problem {k} layout {layout} transpose {transpose} {precision}", flush=True)
                assert torch.isfinite(ref).all()
                assert torch.equal(ref, got), (k, transpose, precision)
                if precision == "fp64":
                    scale = np.abs(host).max() + 1.0
                    assert np.max(np.abs(got.numpy() - host)) <= 1e-12 * scale
        prob.close()


def test_noalloc_refuses_partial_sums_beyond_the_array():
    # FP64 G x with 9 windows of 2^18 columns over 1e6 rows needs
    # 9 x 1e6 x 8 B = 72 MB of partial sums (> 64 MiB); FP32 needs half
    m, n = 1_000_000, 9 * (1 << 18)
    inst = lpgen.planted_lp(lpgen.rng_for(77, 0), m, n, per_col=1, m_zero=m)
    prob = _problem(inst, "bands")
    assert prob.band_schedule()["windows"] == 9
    x = torch.randn(n, dtype=torch.float64, device="cuda")
    y = torch.empty(m, dtype=torch.float64, device="cuda")
    with pytest.raises(P.PdcsError) as e:
        P.pdcs_problem_spmv_noalloc(prob.handle, 0, P.PRECISION["fp64"], x.data_ptr(), y.data_ptr(), 0)
    assert e.value.code == PDCS_ERR_SIZE
    ref, got, _ = _both(prob, inst, False, "mixed", seed=5)
    assert torch.equal(ref, got)
    prob.close()
