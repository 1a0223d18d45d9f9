"""Elementwise error bounds for the scorer network's mixed-precision path,
propagated from the arithmetic (shared by the GPU tests; CPU only)."""
import numpy as np

from oracle import mlp as om

U8, U24 = 2.0 ** -8, 2.0 ** -24


def gemm_err(A, EA, B, EB):
    """Bound on |A~ B~ (fp32 sums) - A B| for |A~ - A| <= EA, |B~ - B| <= EB
    (A: [M, K], B: [K, N], all fp64 arrays)."""
    K = A.shape[1]
    gam = K * U24 / (1 - K * U24)
    aA, aB = np.abs(A) + EA, np.abs(B) + EB
    return EA @ np.abs(B) + np.abs(A) @ EB + EA @ EB + gam * (aA @ aB)


def round_err(x, E):
    """Bound on |bf16(x~) - bf16(x)| for |x~ - x| <= E."""
    return E * (1 + U8) + 2 * U8 * np.abs(x)


def forward_bounds(net, X):
    """Oracle forward (mixed recipe) plus elementwise bounds on the GPU's
    hidden activations and row scores, for inputs exact on both sides."""
    y, acts, pre = net.forward_mixed(X)
    Wb = [om.bf16_round(w).astype(np.float64) for w in net.W]
    E_a = [np.zeros_like(acts[0])]
    for l in range(3):
        Ez = gemm_err(acts[l], E_a[l], Wb[l].T, np.zeros_like(Wb[l].T))
        Ez += U24 * (np.abs(pre[l]) + Ez)           # + bias, rounded
        E_a.append(round_err(np.maximum(pre[l], 0), Ez))
    w4 = Wb[3][0]
    E_y = gemm_err(acts[3], E_a[3], w4[:, None], np.zeros((w4.shape[0], 1)))[:, 0]
    E_y += 4 * U24 * (np.abs(y) + E_y)            # four partial sums + b4
    return y, acts, pre, E_a, E_y
