"""Learned warm start for a family of LPs that share the constraint matrix.

A family member differs from the others in its right-hand side h and cost c.
The warm-start network (the pdcs_mlp kernels: BF16 MFMA forward and backward
passes with FP32 accumulation, Adam on FP32 master weights) maps u = (h, c) to
a primal-dual start z = (x, y).  It is trained on pairs the solver itself
produced for other members.  The solver projects the prediction onto the box
and the dual cone before its first trial, and the cold start (zero) remains
the fallback: a warm-started solve is held to the same termination test.

Host code here only arranges data: per-feature statistics for the
standardization that the library applies, one host-side shuffle, and pointer
offsets of contiguous minibatches.  Every arithmetic step of training and
inference runs in the library's kernels.
"""
from __future__ import annotations

import numpy as np

from ._binding import MLP


def pack_inputs(hs, cs) -> np.ndarray:
    """Rows u = (h, c) as float32 [N x (m + n)]."""
    return np.ascontiguousarray(np.hstack([np.asarray(hs), np.asarray(cs)]), dtype=np.float32)


def pack_targets(xs, ys) -> np.ndarray:
    """Rows z = (x, y) as float32 [N x (n + m)]."""
    return np.ascontiguousarray(np.hstack([np.asarray(xs), np.asarray(ys)]), dtype=np.float32)


def _stats(a: np.ndarray):
    mean = a.mean(axis=0, dtype=np.float64)
    std = a.std(axis=0, dtype=np.float64)
    # features that barely vary in the training set (e.g. a variable at a bound
    # in every member) get a floor of a tenth of the typical spread, so that a
    # member where they move does not dominate the standardized loss
    floor = 0.1 * max(float(np.median(std[std > 0])) if np.any(std > 0) else 1.0, 1e-12)
    return mean.astype(np.float32), np.maximum(std, floor).astype(np.float32)


class WarmStartNet:
    """u = (h, c) -> z = (x, y) for members of one LP family (m rows, n columns)."""

    def __init__(self, m: int, n: int, width: int = 512, seed: int = 0):
        self.m, self.n = int(m), int(n)
        self.net = MLP(m + n, width, n + m, seed=seed)

    def fit(self, U: np.ndarray, Z: np.ndarray, epochs: int = 50, batch: int = 256, lr: float = 1e-3,
            seed: int = 0, val_frac: float = 0.1, log=None) -> list[float]:
        """Adam on minibatches of the standardized MSE.  A fraction val_frac of
        the members is held out; the weights of the epoch with the lowest
        validation loss are kept (early stopping: the solution map of an LP
        family is piecewise linear and the network overfits it quickly).
        Returns the validation loss per epoch (the training loss without a
        validation set)."""
        import torch

        U = np.asarray(U, np.float32)
        Z = np.asarray(Z, np.float32)
        if U.shape[0] != Z.shape[0] or U.shape[1] != self.m + self.n or Z.shape[1] != self.n + self.m:
            raise ValueError("U must be [N x (m+n)] and Z [N x (n+m)]")
        rng = np.random.default_rng(seed)
        perm = rng.permutation(U.shape[0])
        nval = int(round(val_frac * U.shape[0])) if U.shape[0] >= 20 else 0
        tr, va = perm[nval:], perm[:nval]
        im, isd = _stats(U[tr])
        om, osd = _stats(Z[tr])
        self.net.set_normalization(im, isd, om, osd)
        Ud = torch.tensor(U[tr], device="cuda")
        Zd = torch.tensor(Z[tr], device="cuda")
        Uv = torch.tensor(U[va], device="cuda") if nval else None
        Zv = torch.tensor(Z[va], device="cuda") if nval else None
        nb = max(1, len(tr) // batch)
        losses, best, best_p = [], np.inf, None
        for ep in range(epochs):
            tot = 0.0
            for b in rng.permutation(nb):
                lo = int(b) * batch
                hi = len(tr) if b == nb - 1 else lo + batch
                tot += self.net.train_step(Ud[lo:hi], Zd[lo:hi], lr) * (hi - lo)
            cur = self.net.gradients(Uv, Zv)[0] if nval else tot / len(tr)
            losses.append(cur)
            if nval and cur < best:
                best, best_p = cur, self.net.params
            if log is not None:
                log(f"epoch {ep}: train {tot / len(tr):.4e} validation {cur:.4e}")
        if best_p is not None:
            self.net.params = best_p
        torch.cuda.synchronize()
        self.best_epoch = int(np.argmin(losses)) if losses else -1
        return losses

    def predict(self, U: np.ndarray, batch: int = 1024):
        """Predicted starts (x [N x n], y [N x m]) as float64 host arrays."""
        import torch

        U = np.asarray(U, np.float32)
        outs = []
        for lo in range(0, U.shape[0], batch):
            u = torch.tensor(U[lo:lo + batch], device="cuda")
            outs.append(self.net.forward(u).cpu().numpy())
        Z = np.vstack(outs).astype(np.float64)
        return Z[:, : self.n], Z[:, self.n:]
