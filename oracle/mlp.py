"""Oracle for the learned destroy proposal's network (test infrastructure only).

The network scores customers: per-customer features (64) -> 256 -> 256 ->
256 -> 1 with ReLU after the hidden layers; the score of a removal set is the
sum of its customers' scores, trained by mean squared error against the
set's observed makespan change.  (The paper names learned destroy operators
only as future work, Section 6; the architecture is this build's.)

Everything here is plain numpy in fp64.  Mixed precision is emulated where
the GPU path fixes it: GEMM operands rounded to bfloat16 (round to nearest,
ties to even), products accumulated exactly in fp64 (the GPU accumulates in
fp32, within the bound of `gemm_error_bound`).
"""
from __future__ import annotations

import numpy as np

DIMS = (64, 256, 256, 256, 1)


def bf16_round(x):
    """Round float values to the nearest bfloat16 (ties to even), returned as
    float32 carrying the bfloat16 value."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    nan = np.isnan(a)
    if nan.any():
        out = out.copy()
        out[nan] = np.nan
    return out


def gemm_ref(A, B):
    """C = A @ B in fp64 from the operands as given (already rounded)."""
    return np.asarray(A, np.float64) @ np.asarray(B, np.float64)


def gemm_error_bound(A, B, k_factor=2.0):
    """|fp32-accumulated C - exact C| <= K * 2^-24 * (|A| @ |B|) * ceil(log2 K)-ish;
    a conservative bound for K-term fp32 sums of exact products: K * u * sum|a||b|."""
    K = np.asarray(A).shape[1]
    mag = np.abs(np.asarray(A, np.float64)) @ np.abs(np.asarray(B, np.float64))
    return k_factor * K * 2.0 ** -24 * mag + 1e-30


class MLP:
    """fp64 reference of the scorer.  Weights W[l] have shape [in, out]."""

    def __init__(self, W, b):
        self.W = [np.asarray(w, np.float64) for w in W]
        self.b = [np.asarray(x, np.float64) for x in b]

    @staticmethod
    def init(seed=0, dims=DIMS):
        g = np.random.Generator(np.random.Philox(key=seed))
        W, b = [], []
        for i in range(len(dims) - 1):
            lim = np.sqrt(6.0 / (dims[i] + dims[i + 1]))
            W.append(g.uniform(-lim, lim, size=(dims[i], dims[i + 1])))
            b.append(np.zeros(dims[i + 1]))
        return MLP(W, b)

    def forward(self, X, bf16=False):
        """Scores of rows of X.  With bf16, every GEMM operand (input
        activations and weights) is first rounded to bfloat16."""
        h = np.asarray(X, np.float64)
        cache = []
        L = len(self.W)
        for i in range(L):
            a = bf16_round(h) if bf16 else h
            w = bf16_round(self.W[i]) if bf16 else self.W[i]
            z = np.asarray(a, np.float64) @ np.asarray(w, np.float64) + self.b[i]
            cache.append((a, z))
            h = np.maximum(z, 0.0) if i < L - 1 else z
        return h[:, 0], cache

    def loss_and_grads(self, X, seg, target):
        """Mean squared error of set scores.  X: [R, 64] rows of customers,
        seg: [S+1] row offsets of each set, target: [S].  Returns (loss,
        dW list, db list, per-row dL/dscore)."""
        y, cache = self.forward(X)
        S = len(target)
        score = np.array([y[seg[s]:seg[s + 1]].sum() for s in range(S)])
        err = score - np.asarray(target, np.float64)
        loss = float(np.mean(err ** 2))
        dscore = 2.0 * err / S
        dy = np.zeros_like(y)
        for s in range(S):
            dy[seg[s]:seg[s + 1]] = dscore[s]
        g = dy[:, None]
        dW, db = [None] * len(self.W), [None] * len(self.W)
        for i in reversed(range(len(self.W))):
            a, z = cache[i]
            if i < len(self.W) - 1:
                g = g * (z > 0)
            dW[i] = np.asarray(a, np.float64).T @ g
            db[i] = g.sum(axis=0)
            g = g @ self.W[i].T
        return loss, dW, db, dy
