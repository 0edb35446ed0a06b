"""FP64 NumPy oracle of the warm-start MLP -- test infrastructure only.

The network (not part of the paper; it is the learned warm start built beside
the method) is

    z1 = W1 u + b1, h1 = relu(z1), z2 = W2 h1 + b2, h2 = relu(z2), v = W3 h2 + b3,
    loss = mean over batch and outputs of (v - t)^2.

Parameters are laid out W1[w x d_in], b1[w], W2[w x w], b2[w], W3[d_out x w],
b3[d_out] in one flat vector.  With ``bf16=True`` the oracle rounds, like the
GPU, the GEMM operands (inputs, weights, hidden activations, output gradients)
to bfloat16 before multiplying, and accumulates in float64.

Parity pinning: the analytic gradients are checked against central finite
differences of the FP64 loss, the per-layer products (layer_products) against
the same finite differences, the standardized forms against hand-computed
values, and Adam against its textbook first step (tests).
"""
from __future__ import annotations

import numpy as np


def bf16_round(a):
    """Round float32 values to bfloat16 (round to nearest, ties to even), as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    rounded = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def split_params(p, d_in, w, d_out):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    out = {}
    for name, shape in (("W1", (w, d_in)), ("b1", (w,)), ("W2", (w, w)), ("b2", (w,)),
                        ("W3", (d_out, w)), ("b3", (d_out,))):
        size = int(np.prod(shape))
        out[name] = p[o:o + size].reshape(shape)
        o += size
    return out


def _q(x, bf16):
    return bf16_round(x) if bf16 else np.asarray(x, dtype=np.float64)


def forward(params, u, d_in, w, d_out, bf16=False):
    """Forward pass; returns v and the cache used by backward."""
    P = split_params(params, d_in, w, d_out)
    W1, W2, W3 = (_q(P[k], bf16) for k in ("W1", "W2", "W3"))
    U = _q(u, bf16)
    z1 = np.maximum(U @ W1.T + P["b1"], 0.0)
    if bf16:
        z1 = z1.astype(np.float32).astype(np.float64)
    h1 = _q(z1, bf16)
    z2 = np.maximum(h1 @ W2.T + P["b2"], 0.0)
    if bf16:
        z2 = z2.astype(np.float32).astype(np.float64)
    h2 = _q(z2, bf16)
    v = h2 @ W3.T + P["b3"]
    return v, dict(U=U, W1=W1, W2=W2, W3=W3, z1=z1, h1=h1, z2=z2, h2=h2)


def loss_and_grad(params, u, t, d_in, w, d_out, bf16=False):
    """Mean squared error and its gradient with respect to the flat parameters."""
    v, c = forward(params, u, d_in, w, d_out, bf16)
    n = v.size
    diff = v - t
    loss = float(np.sum(diff * diff) / n)
    dv = 2.0 * diff / n
    if bf16:
        dv = dv.astype(np.float32).astype(np.float64)
    dvq = _q(dv, bf16)
    gW3 = dvq.T @ c["h2"]
    gb3 = dv.sum(axis=0)
    dz2 = (dvq @ c["W3"]) * (c["z2"] > 0)
    if bf16:
        dz2 = dz2.astype(np.float32).astype(np.float64)
    dz2q = _q(dz2, bf16)
    gW2 = dz2q.T @ c["h1"]
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2q @ c["W2"]) * (c["z1"] > 0)
    if bf16:
        dz1 = dz1.astype(np.float32).astype(np.float64)
    dz1q = _q(dz1, bf16)
    gW1 = dz1q.T @ c["U"]
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def layer_products(params, acts, d_in, w, d_out):
    """Every product of one forward and backward pass, in float64, from the
    activations that pass fed its products: acts = dict(U, h1, h2, dv, dz2, dz1)
    of arrays [batch x features] (the GPU's BF16 values, widened).  Weights are
    rounded to BF16 like the GPU's copies.

    Returns z1 = U W1^T + b1, z2 = h1 W2^T + b2, v = h2 W3^T + b3, the backward
    products dh2 = dv W3 and dh1 = dz2 W2 (before the ReLU masks), the weight
    gradients gW1 = dz1^T U, gW2 = dz2^T h1, gW3 = dv^T h2, and under the same
    names with suffix "_abs" each product taken over absolute values (biases
    included), the scale that bounds a sum's rounding error."""
    P = split_params(params, d_in, w, d_out)
    W1, W2, W3 = (bf16_round(P[k]) for k in ("W1", "W2", "W3"))
    a = {k: np.asarray(acts[k], np.float64) for k in ("U", "h1", "h2", "dv", "dz2", "dz1")}
    out = {}
    for name, x, y, b in (("z1", a["U"], W1.T, P["b1"]), ("z2", a["h1"], W2.T, P["b2"]),
                          ("v", a["h2"], W3.T, P["b3"]), ("dh2", a["dv"], W3, None),
                          ("dh1", a["dz2"], W2, None), ("gW1", a["dz1"].T, a["U"], None),
                          ("gW2", a["dz2"].T, a["h1"], None), ("gW3", a["dv"].T, a["h2"], None)):
        out[name] = x @ y + (b if b is not None else 0.0)
        out[name + "_abs"] = np.abs(x) @ np.abs(y) + (np.abs(b) if b is not None else 0.0)
    return out


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Textbook Adam (Kingma & Ba) with bias correction; returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def forward_normalized(params, u, d_in, w, d_out, norm, bf16=False):
    """Forward pass with feature standardization norm = (in_mean, in_scale,
    out_mean, out_scale): the network sees (u - in_mean) / in_scale and its
    output z is returned as z * out_scale + out_mean."""
    in_mean, in_scale, out_mean, out_scale = (np.asarray(a, np.float64) for a in norm)
    z, _ = forward(params, (np.asarray(u, np.float64) - in_mean) / in_scale, d_in, w, d_out, bf16)
    return z * out_scale + out_mean


def loss_and_grad_normalized(params, u, t, d_in, w, d_out, norm, bf16=False):
    """MSE in standardized units: inputs and targets standardized per feature."""
    in_mean, in_scale, out_mean, out_scale = (np.asarray(a, np.float64) for a in norm)
    return loss_and_grad(params, (np.asarray(u, np.float64) - in_mean) / in_scale,
                         (np.asarray(t, np.float64) - out_mean) / out_scale, d_in, w, d_out, bf16)
