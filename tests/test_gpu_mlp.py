"""GPU parity of the MLP kernels (BF16 MFMA forward/backward, Adam) against the
FP64 NumPy oracle that rounds the same GEMM operands to BF16.

Tolerance: both sides use identical BF16 operands; they differ only in FP32 vs
FP64 accumulation order, which can flip the BF16 rounding of an intermediate
activation by one unit (2^-8 relative).  Outputs and gradients are therefore
compared norm-wise to 2e-3 and element-wise to 2e-2 of the largest magnitude.
"""
import numpy as np
import pytest

from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_15504_amd")
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if P.pdcs_device_count() < 1:
        pytest.skip("no GPU visible")


def _close(a, b, norm_tol=2e-3, elem_tol=2e-2):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    scale = max(np.abs(b).max(), 1e-30)
    assert np.linalg.norm(a - b) <= norm_tol * max(np.linalg.norm(b), 1e-30), np.linalg.norm(a - b) / np.linalg.norm(b)
    assert np.abs(a - b).max() <= elem_tol * scale


@pytest.mark.parametrize("dims,batch", [((300, 96, 200), 37), ((130, 128, 257), 64), ((1000, 64, 33), 5)])
def test_forward_and_gradients_match_oracle(dims, batch):
    d_in, w, d_out = dims
    net = P.MLP(d_in, w, d_out, seed=3)
    rng = np.random.default_rng(1)
    u = rng.standard_normal((batch, d_in)).astype(np.float32)
    t = rng.standard_normal((batch, d_out)).astype(np.float32)
    ud = torch.tensor(u, device="cuda")
    td = torch.tensor(t, device="cuda")
    v = net.forward(ud).cpu().numpy()
    params = net.params.astype(np.float64)
    v_ref, _ = M.forward(params, u, d_in, w, d_out, bf16=True)
    _close(v, v_ref)
    loss, g = net.gradients(ud, td)
    loss_ref, g_ref = M.loss_and_grad(params, u, t, d_in, w, d_out, bf16=True)
    assert loss == pytest.approx(loss_ref, rel=2e-3)
    _close(g.cpu().numpy(), g_ref)


def test_full_width_forward_sampled_rows():
    # the warm-start network's real shape: 6e4 -> 512 -> 512 -> 6e4
    d_in, w, d_out = 60000, 512, 60000
    net = P.MLP(d_in, w, d_out, seed=7)
    rng = np.random.default_rng(2)
    u = rng.standard_normal((16, d_in)).astype(np.float32)
    v = net.forward(torch.tensor(u, device="cuda")).cpu().numpy()
    params = net.params.astype(np.float64)
    rows = [0, 7, 15]
    v_ref, _ = M.forward(params, u[rows], d_in, w, d_out, bf16=True)
    _close(v[rows], v_ref)


def test_adam_step_matches_textbook_update():
    d_in, w, d_out, batch = 50, 32, 20, 8
    net = P.MLP(d_in, w, d_out, seed=5)
    rng = np.random.default_rng(3)
    ud = torch.tensor(rng.standard_normal((batch, d_in)).astype(np.float32), device="cuda")
    td = torch.tensor(rng.standard_normal((batch, d_out)).astype(np.float32), device="cuda")
    p0 = net.params.astype(np.float64)
    _, g = net.gradients(ud, td)
    g = g.cpu().numpy().astype(np.float64)
    net.train_step(ud, td, 1e-3)
    p1 = net.params.astype(np.float64)
    want, _, _ = M.adam_step(p0, g, np.zeros_like(p0), np.zeros_like(p0), 1, 1e-3)
    assert np.allclose(p1, want, rtol=0, atol=2e-6)


def test_training_reduces_loss():
    d_in, w, d_out, batch = 64, 128, 48, 128
    net = P.MLP(d_in, w, d_out, seed=11)
    rng = np.random.default_rng(4)
    A = rng.standard_normal((d_out, d_in)) / np.sqrt(d_in)
    u = rng.standard_normal((batch, d_in)).astype(np.float32)
    t = (u @ A.T).astype(np.float32)
    ud = torch.tensor(u, device="cuda")
    td = torch.tensor(t, device="cuda")
    first = net.train_step(ud, td, 2e-3)
    for _ in range(200):
        last = net.train_step(ud, td, 2e-3)
    assert last < 0.05 * first
