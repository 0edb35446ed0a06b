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
