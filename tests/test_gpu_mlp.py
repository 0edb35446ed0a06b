"""GPU parity of the MLP kernels (BF16 MFMA forward/backward with the loss,
ReLU masks and Adam fused into the products' epilogues) against the FP64 NumPy
oracle, through the C ABI.

Two levels:
  * end to end: outputs and gradients against the oracle's own BF16 pass.  The
    two sides can round an intermediate activation to different BF16 neighbours
    (FP32 vs FP64 sums near a rounding boundary), so this level is norm-wise
    2e-3 and element-wise 2e-2 of the largest magnitude;
  * layer by layer: each product recomputed in FP64 from the BF16 activations
    the GPU actually fed it (read back through pdcs_mlp_activation).  Then the
    only differences are FP32 summation order (bounded by TOL = 1e-5 of the
    product over absolute values) and the final rounding of an activation to
    BF16 (half a unit in the last place: 2^-8 relative).
Adam is checked against its textbook update at steps 1, 2 and 10, on shapes
whose weight matrices have whole interior tiles and ragged edge tiles.
"""
import numpy as np
import pytest

from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_15504_amd")
torch = pytest.importorskip("torch")

TOL = 1e-5       # FP32 summation error per unit of sum |a||b|
HALF_ULP = 2.0 ** -8


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


def _data(d_in, d_out, batch, seed):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((batch, d_in)).astype(np.float32)
    t = rng.standard_normal((batch, d_out)).astype(np.float32)
    return u, t, torch.tensor(u, device="cuda"), torch.tensor(t, device="cuda")


@pytest.mark.parametrize("dims,batch", [((300, 96, 200), 37), ((130, 128, 257), 64), ((1000, 64, 33), 5)])
def test_forward_and_gradients_match_oracle(dims, batch):
    d_in, w, d_out = dims
    net = P.MLP(d_in, w, d_out, seed=3)
    u, t, ud, td = _data(d_in, d_out, batch, 1)
    v = net.forward(ud).cpu().numpy()
    params = net.params.astype(np.float64)
    v_ref, _ = M.forward(params, u, d_in, w, d_out, bf16=True)
    _close(v, v_ref)
    loss, g = net.gradients(ud, td)
    loss_ref, g_ref = M.loss_and_grad(params, u, t, d_in, w, d_out, bf16=True)
    assert loss == pytest.approx(loss_ref, rel=2e-3)
    _close(g.cpu().numpy(), g_ref)


def _within(gpu, exact, scale, rel=0.0, name=""):
    gpu = np.asarray(gpu, np.float64)
    err = np.abs(gpu - exact)
    bound = TOL * scale + rel * np.abs(exact) + 1e-30
    assert np.all(err <= bound), (name, float((err / bound).max()))


def _rounded_relu(gpu, pre, scale, name):
    # gpu = BF16(ReLU(FP32 pre)); pre known to FP64 within TOL * scale
    exact = np.maximum(pre, 0.0)
    _within(gpu, exact, scale, HALF_ULP * (1 + 1e-6), name)
    assert np.all(gpu >= 0), name


@pytest.mark.parametrize("dims,batch", [((300, 96, 200), 37), ((130, 128, 257), 300), ((300, 256, 260), 40)])
def test_layers_match_oracle_on_gpu_activations(dims, batch):
    d_in, w, d_out = dims
    net = P.MLP(d_in, w, d_out, seed=4)
    u, t, ud, td = _data(d_in, d_out, batch, 2)
    loss, g = net.gradients(ud, td)
    g = g.cpu().numpy().astype(np.float64)
    p = net.params.astype(np.float64)
    acts = {k: net.activation(n, batch).astype(np.float64)
            for k, n in (("U", "input"), ("h1", "h1"), ("h2", "h2"), ("dv", "dv"), ("dz2", "dz2"), ("dz1", "dz1"))}
    o = M.layer_products(p, acts, d_in, w, d_out)
    n = batch * d_out
    # the input enters the products as its BF16 rounding, bit for bit
    assert np.array_equal(acts["U"], M.bf16_round(u))
    _rounded_relu(acts["h1"], o["z1"], o["z1_abs"], "h1")
    _rounded_relu(acts["h2"], o["z2"], o["z2_abs"], "h2")
    # loss gradient 2 (v - t) / n, rounded to BF16
    dv = 2.0 * (o["v"] - t) / n
    _within(acts["dv"], dv, 2.0 / n * o["v_abs"], HALF_ULP * (1 + 1e-6), "dv")
    # masked backward products: zero exactly where the GPU's activation is zero
    for dz, dh, h in (("dz2", "dh2", "h2"), ("dz1", "dh1", "h1")):
        on = acts[h] > 0
        assert np.all(acts[dz][~on] == 0), dz
        _within(acts[dz][on], o[dh][on], o[dh + "_abs"][on], HALF_ULP * (1 + 1e-6), dz)
    G = M.split_params(g, d_in, w, d_out)
    for k in ("W1", "W2", "W3"):
        _within(G[k], o["g" + k], o["g" + k + "_abs"], 0.0, "g" + k)
    # bias gradients: FP32 column sums of the (unrounded) FP32 gradients
    _within(G["b3"], dv.sum(0), (2.0 / n * (o["v_abs"] + np.abs(t))).sum(0), 0.0, "gb3")
    on2, on1 = acts["h2"] > 0, acts["h1"] > 0
    _within(G["b2"], (o["dh2"] * on2).sum(0), (o["dh2_abs"] * on2).sum(0), 0.0, "gb2")
    _within(G["b1"], (o["dh1"] * on1).sum(0), (o["dh1_abs"] * on1).sum(0), 0.0, "gb1")
    loss_ref = float(np.mean((o["v"] - t) ** 2))
    assert abs(loss - loss_ref) <= TOL * float(np.mean((o["v_abs"] + np.abs(t)) ** 2))


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


def _adam_tol(p, lr):
    # FP32 update (relative error ~1e-6 of a step of size <= lr) and FP32 weights
    return 1e-5 * lr + 2.0 ** -22 * np.abs(p)


@pytest.mark.parametrize("dims,batch", [((50, 32, 20), 8), ((300, 256, 260), 40)])
def test_adam_steps_match_textbook_update(dims, batch):
    d_in, w, d_out = dims
    lr = 1e-3
    net = P.MLP(d_in, w, d_out, seed=5)
    _, _, ud, td = _data(d_in, d_out, batch, 3)
    p = net.params.astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for step in range(1, 11):
        _, g = net.gradients(ud, td)  # the same products as inside the step
        net.train_step(ud, td, lr)
        p_gpu = net.params.astype(np.float64)
        want, m, v = M.adam_step(p, g.cpu().numpy().astype(np.float64), m, v, step, lr)
        if step in (1, 2, 10):
            err = np.abs(p_gpu - want)
            assert np.all(err <= _adam_tol(want, lr)), (step, float((err / _adam_tol(want, lr)).max()))
        p = p_gpu


def test_full_width_adam_step_sampled():
    # one step at the real shape (61.7M parameters, interior and edge tiles);
    # 20000 sampled parameters plus every bias against the textbook update
    d_in, w, d_out, batch, lr = 60000, 512, 60000, 16, 1e-3
    net = P.MLP(d_in, w, d_out, seed=8)
    _, _, ud, td = _data(d_in, d_out, batch, 4)
    p0 = net.params.astype(np.float64)
    _, g = net.gradients(ud, td)
    g = g.cpu().numpy().astype(np.float64)
    net.train_step(ud, td, lr)
    p1 = net.params.astype(np.float64)
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([rng.integers(0, p0.size, 20000),
                                    np.arange(w * d_in, w * d_in + w),              # b1
                                    np.arange(p0.size - d_out, p0.size)]))          # b3
    want, _, _ = M.adam_step(p0[idx], g[idx], np.zeros(idx.size), np.zeros(idx.size), 1, lr)
    assert np.all(np.abs(p1[idx] - want) <= _adam_tol(want, lr))
    # parameters whose gradient is exactly zero do not move
    zero = idx[g[idx] == 0]
    assert np.array_equal(p1[zero], p0[zero])


def test_asynchronous_steps_equal_waited_steps():
    d_in, w, d_out, batch = 300, 256, 260, 40
    _, _, ud, td = _data(d_in, d_out, batch, 6)
    a = P.MLP(d_in, w, d_out, seed=9)
    b = P.MLP(d_in, w, d_out, seed=9)
    for _ in range(3):
        a.train_step(ud, td, 1e-3)
        assert b.train_step(ud, td, 1e-3, wait=False) is None
    torch.cuda.synchronize()
    assert np.array_equal(a.params, b.params)


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
