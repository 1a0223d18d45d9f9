"""Pins for the scorer network's oracle (CPU only)."""
import numpy as np

from oracle import mlp


def test_bf16_rounding_known_values():
    x = np.array([1.0, 1.00390625, 1.005859375, 1.0078125, -2.5, 3.0e38, 1e-40], np.float32)
    r = mlp.bf16_round(x)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1.0
    assert r[0] == 1.0 and r[1] == 1.0
    # 1 + 1.5 * 2^-8 rounds up to 1 + 2^-7
    assert r[2] == np.float32(1.0078125) and r[3] == np.float32(1.0078125)
    assert r[4] == -2.5
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8 + 1e-38)


def test_gradients_match_finite_differences():
    g = np.random.Generator(np.random.Philox(key=3))
    net = mlp.MLP.init(seed=1, dims=(6, 5, 4, 3, 1))
    # nonzero biases keep every pre-activation away from the ReLU kink, where
    # a central difference is not the derivative
    for b in net.b:
        b[:] = g.uniform(0.05, 0.3, size=b.shape)
    X = g.normal(size=(11, 6))
    seg = np.array([0, 3, 7, 11])
    target = np.array([0.5, -1.0, 2.0])
    loss, dW, db, _ = net.loss_and_grads(X, seg, target)
    eps = 1e-6
    for li in range(4):
        for idx in [(0, 0), (1, 0), (net.W[li].shape[0] - 1, net.W[li].shape[1] - 1)]:
            w0 = net.W[li][idx]
            net.W[li][idx] = w0 + eps
            lp = net.loss_and_grads(X, seg, target)[0]
            net.W[li][idx] = w0 - eps
            lm = net.loss_and_grads(X, seg, target)[0]
            net.W[li][idx] = w0
            assert abs((lp - lm) / (2 * eps) - dW[li][idx]) < 1e-6 * max(1.0, abs(dW[li][idx]))
        b0 = net.b[li][0]
        net.b[li][0] = b0 + eps
        lp = net.loss_and_grads(X, seg, target)[0]
        net.b[li][0] = b0 - eps
        lm = net.loss_and_grads(X, seg, target)[0]
        net.b[li][0] = b0
        assert abs((lp - lm) / (2 * eps) - db[li][0]) < 1e-6 * max(1.0, abs(db[li][0]))


def test_linear_special_case():
    """With one layer the model is linear: the least-squares solution of the
    set-sum regression zeroes the gradient."""
    g = np.random.Generator(np.random.Philox(key=4))
    X = g.normal(size=(40, 5))
    seg = np.arange(0, 41, 4)
    Xs = np.add.reduceat(X, seg[:-1], axis=0)
    w_true = g.normal(size=5)
    target = Xs @ w_true
    net = mlp.MLP([w_true[:, None]], [np.zeros(1)])
    loss, dW, db, _ = net.loss_and_grads(X, seg, target)
    assert loss < 1e-20 and np.abs(dW[0]).max() < 1e-9
