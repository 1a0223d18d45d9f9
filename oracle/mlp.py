"""Oracle for the learned destroy proposal's scorer network (test
infrastructure only: only tests, the smoke check and the CPU baseline use it).

The paper names learned destroy operators as future work (Section 7.4) and fixes
no network; the one here is this project's: per-customer features (64) ->
256 -> 256 -> 256 -> 1 with ReLU after the hidden layers.  The score of a
removal set is the sum of its customers' scores, fitted by mean squared error
to the makespan change that destroying and repairing the set produced.

Plain numpy in fp64.  `forward` / `loss_and_grads` are the textbook network;
`forward_mixed` / `backward_mixed` follow the GPU path's precision recipe:
every GEMM operand is a bfloat16 value (round to nearest, ties to even), and
products are summed exactly here (the GPU sums them in fp32).

Parameter layout (flat fp32 vector, the GPU library's layout too):
W1 [256][64], b1 [256], W2 [256][256], b2 [256], W3 [256][256], b3 [256],
w4 [256], b4 [1]; W[l][out][in] (row = output unit).
"""
from __future__ import annotations

import numpy as np

DIMS = (64, 256, 256, 256, 1)
U_BF16 = 2.0 ** -8      # unit roundoff of bfloat16 (8-bit significand)
U_FP32 = 2.0 ** -24


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even); returned as float32
    carrying the bfloat16 value."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).reshape(a.shape)
    nan = np.isnan(a)
    if nan.any():
        out = out.copy()
        out[nan] = np.nan
    return out


def bf16_bits(x):
    """bfloat16 bit patterns (uint16) of the nearest-even rounding of x."""
    return (bf16_round(x).view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(b):
    return (np.asarray(b, np.uint16).astype(np.uint32) << 16).view(np.float32)


def param_shapes(dims=DIMS):
    shapes = []
    for i in range(len(dims) - 1):
        shapes.append((dims[i + 1], dims[i]))
        shapes.append((dims[i + 1],))
    return shapes


def num_params(dims=DIMS):
    return int(sum(np.prod(s) for s in param_shapes(dims)))


class MLP:
    """fp64 network.  W[l] has shape [out, in]; the last layer's weights are
    W[-1] of shape [1, 256]."""

    def __init__(self, W, b):
        self.W = [np.array(w, np.float64) for w in W]
        self.b = [np.array(x, np.float64) for x in b]

    @staticmethod
    def init(seed=0, dims=DIMS):
        """Glorot-uniform weights from a Philox stream, zero biases."""
        g = np.random.Generator(np.random.Philox(key=seed))
        W, b = [], []
        for i in range(len(dims) - 1):
            lim = np.sqrt(6.0 / (dims[i] + dims[i + 1]))
            W.append(g.uniform(-lim, lim, size=(dims[i + 1], dims[i])))
            b.append(np.zeros(dims[i + 1]))
        return MLP(W, b)

    # ---- flat layout -------------------------------------------------------
    def flat(self):
        parts = []
        for w, x in zip(self.W, self.b):
            parts += [w.ravel(), x.ravel()]
        return np.concatenate(parts)

    @staticmethod
    def from_flat(v, dims=DIMS):
        v = np.asarray(v, np.float64)
        W, b, o = [], [], 0
        for i in range(len(dims) - 1):
            k = dims[i + 1] * dims[i]
            W.append(v[o:o + k].reshape(dims[i + 1], dims[i]))
            o += k
            b.append(v[o:o + dims[i + 1]].copy())
            o += dims[i + 1]
        assert o == len(v)
        return MLP(W, b)

    # ---- textbook network --------------------------------------------------
    def forward(self, X):
        h = np.asarray(X, np.float64)
        cache = []
        L = len(self.W)
        for i in range(L):
            z = h @ self.W[i].T + self.b[i]
            cache.append((h, z))
            h = np.maximum(z, 0.0) if i < L - 1 else z
        return h[:, 0], cache

    def loss_and_grads(self, X, seg, target):
        """Set-sum mean squared error and its exact gradient.  X: [R, 64],
        seg: [S+1] row offsets of the sets, target: [S]."""
        y, cache = self.forward(X)
        loss, dy = set_loss(y, seg, target)
        g = dy[:, None]
        dW, db = [None] * len(self.W), [None] * len(self.W)
        for i in reversed(range(len(self.W))):
            a, z = cache[i]
            if i < len(self.W) - 1:
                g = g * (z > 0)
            dW[i] = g.T @ a
            db[i] = g.sum(axis=0)
            g = g @ self.W[i]
        return loss, dW, db, dy

    # ---- the GPU path's precision recipe -----------------------------------
    def forward_mixed(self, Xb):
        """Xb: bfloat16 features.  Hidden layer l: z = a @ bf16(W)^T + b with
        exact sums, h = bf16(relu(z)).  Head: y = h3 . bf16(w4) + b4."""
        h = np.asarray(Xb, np.float64)
        acts, pre = [h], []
        L = len(self.W)
        for i in range(L - 1):
            z = h @ bf16_round(self.W[i]).astype(np.float64).T + self.b[i]
            pre.append(z)
            h = bf16_round(np.maximum(z, 0.0)).astype(np.float64)
            acts.append(h)
        w4 = bf16_round(self.W[-1][0]).astype(np.float64)
        y = h @ w4 + self.b[-1][0]
        return y, acts, pre

    def backward_mixed(self, acts, dy):
        """Gradients along the GPU path: dz3 = bf16(dy * bf16(w4) * [h3 > 0]);
        for l = 3, 2, 1: dW_l = dz_l^T a_{l-1}, db_l = column sums of dz_l,
        and dz_{l-1} = bf16((dz_l @ bf16(W_l)) * [h_{l-1} > 0]); head:
        dw4 = dy^T h3, db4 = sum dy.  All sums exact."""
        L = len(self.W)
        dy = np.asarray(dy, np.float64)
        w4 = bf16_round(self.W[-1][0]).astype(np.float64)
        h3 = acts[L - 1]
        dW, db = [None] * L, [None] * L
        dW[L - 1] = (dy @ h3)[None, :]
        db[L - 1] = np.array([dy.sum()])
        dz = bf16_round(dy[:, None] * w4[None, :] * (h3 > 0)).astype(np.float64)
        for i in reversed(range(L - 1)):
            a = acts[i]
            dW[i] = dz.T @ a
            db[i] = dz.sum(axis=0)
            if i > 0:
                dh = dz @ bf16_round(self.W[i]).astype(np.float64)
                dz = bf16_round(dh * (acts[i] > 0)).astype(np.float64)
        return dW, db


def set_loss(y, seg, target):
    """Loss = mean over sets s of (sum of y over s - target_s)^2, and the
    derivative of the loss with respect to each row's score."""
    y = np.asarray(y, np.float64)
    seg = np.asarray(seg, np.int64)
    S = len(seg) - 1
    score = np.array([y[seg[s]:seg[s + 1]].sum() for s in range(S)])
    err = score - np.asarray(target, np.float64)
    dscore = 2.0 * err / S
    dy = np.zeros_like(y)
    for s in range(S):
        dy[seg[s]:seg[s + 1]] = dscore[s]
    return float(np.mean(err ** 2)), dy


def sgd_momentum(params, grads, vel, lr, mu):
    """Heavy-ball step on flat vectors: v <- mu v + g; p <- p - lr v."""
    vel = mu * np.asarray(vel, np.float64) + np.asarray(grads, np.float64)
    return np.asarray(params, np.float64) - lr * vel, vel


def flat_grads(dW, db):
    parts = []
    for w, x in zip(dW, db):
        parts += [np.asarray(w).ravel(), np.asarray(x).ravel()]
    return np.concatenate(parts)


def gemm_bound(A, B, K=None):
    """Elementwise bound on |fp32-summed A @ B - exact A @ B| for exact
    operands: K * 2^-24 * (|A| @ |B|) (any summation order, K terms)."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    K = A.shape[1] if K is None else K
    g = K * U_FP32 / (1.0 - K * U_FP32)
    return g * (np.abs(A) @ np.abs(B))
