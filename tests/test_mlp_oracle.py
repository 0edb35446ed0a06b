"""Pins of the MLP oracle: finite differences, textbook Adam, BF16 rounding."""
import numpy as np
import pytest

from oracle import mlp_oracle as M


def _rand_problem(seed, d_in=7, w=5, d_out=4, B=3):
    rng = np.random.default_rng(seed)
    npar = w * d_in + w + w * w + w + d_out * w + d_out
    p = rng.standard_normal(npar) * 0.7
    u = rng.standard_normal((B, d_in))
    t = rng.standard_normal((B, d_out))
    return p, u, t, (d_in, w, d_out)


@pytest.mark.parametrize("seed", range(3))
def test_gradient_matches_central_differences(seed):
    p, u, t, dims = _rand_problem(seed)
    loss, g = M.loss_and_grad(p, u, t, *dims)
    eps = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = eps
        fd[i] = (M.loss_and_grad(p + e, u, t, *dims)[0] - M.loss_and_grad(p - e, u, t, *dims)[0]) / (2 * eps)
    assert np.allclose(g, fd, rtol=1e-5, atol=1e-7)


def test_forward_hand_values():
    # d_in = w = d_out = 1: v = w3 relu(w2 relu(w1 u + b1) + b2) + b3
    p = np.array([2.0, -1.0, 3.0, 0.5, -2.0, 0.25])
    v, _ = M.forward(p, np.array([[1.5], [0.2]]), 1, 1, 1)
    # u=1.5: z1 = 2, z2 = 6.5, v = -12.75 ; u=0.2: z1 = relu(-0.6) = 0, z2 = 0.5, v = -0.75
    assert np.allclose(v.ravel(), [-12.75, -0.75])


def test_adam_first_step_is_sign_times_lr():
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = M.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    # bias-corrected first step: m_hat = g, v_hat = g^2  =>  -lr * g / (|g| + eps)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8))


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(0).standard_normal(10000).astype(np.float32) * 100
    x[:4] = [1.0, 1.00390625, 1.01171875, -3.3e-3]   # exact bf16 value and ties
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16_round(x), ref)


def _fd_grad(p, u, t, dims, eps=1e-6):
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = eps
        fd[i] = (M.loss_and_grad(p + e, u, t, *dims)[0] - M.loss_and_grad(p - e, u, t, *dims)[0]) / (2 * eps)
    return fd


@pytest.mark.parametrize("seed", range(2))
def test_layer_products_weight_gradients_match_central_differences(seed):
    # exact float64 activations of a pass (weights already BF16 values, so the
    # BF16 rounding inside layer_products changes nothing); dv, dz2, dz1 by the
    # chain rule of the squared error and ReLU
    p, u, t, dims = _rand_problem(seed)
    d_in, w, d_out = dims
    p = M.bf16_round(p)
    P = M.split_params(p, *dims)
    z1 = u @ P["W1"].T + P["b1"]
    h1 = np.maximum(z1, 0)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0)
    v = h2 @ P["W3"].T + P["b3"]
    dv = 2 * (v - t) / v.size
    dz2 = (dv @ P["W3"]) * (z2 > 0)
    dz1 = (dz2 @ P["W2"]) * (z1 > 0)
    out = M.layer_products(p, dict(U=u, h1=h1, h2=h2, dv=dv, dz2=dz2, dz1=dz1), *dims)
    fd = M.split_params(_fd_grad(p, u, t, dims), *dims)
    for k in ("W1", "W2", "W3"):
        assert np.allclose(out["g" + k], fd[k], rtol=1e-5, atol=1e-7), k
    assert np.allclose(out["v"], M.forward(p, u, *dims)[0], rtol=1e-12, atol=1e-12)
    # the scales bound the products
    for k in ("z1", "z2", "v", "dh2", "dh1", "gW1", "gW2", "gW3"):
        assert np.all(np.abs(out[k]) <= out[k + "_abs"] * (1 + 1e-12) + 1e-300)


def test_normalized_forms_hand_values():
    # d_in = w = d_out = 1, p = (w1, b1, w2, b2, w3, b3); input mean 1, scale 0.5,
    # output mean 10, scale 3.  u = 1.5 -> (1.5 - 1) / 0.5 = 1 -> z1 = 1, z2 = 3.5,
    # raw output -6.75 -> -6.75 * 3 + 10 = -10.25.  Target 1 -> (1 - 10) / 3 = -3:
    # loss (-6.75 + 3)^2 = 14.0625 and dL/db3 = 2 (-3.75) = -7.5.
    p = np.array([2.0, -1.0, 3.0, 0.5, -2.0, 0.25])
    norm = ([1.0], [0.5], [10.0], [3.0])
    out = M.forward_normalized(p, np.array([[1.5]]), 1, 1, 1, norm)
    assert np.allclose(out, [[-10.25]])
    loss, g = M.loss_and_grad_normalized(p, np.array([[1.5]]), np.array([[1.0]]), 1, 1, 1, norm)
    assert loss == pytest.approx(14.0625)
    assert g[-1] == pytest.approx(-7.5)
    # dL/dw3 = -7.5 * h2 = -26.25; dL/dw1 = -7.5 * w3 * w2 * u_std = -7.5 * -2 * 3 * 1 = 45
    assert g[4] == pytest.approx(-26.25) and g[0] == pytest.approx(45.0)
