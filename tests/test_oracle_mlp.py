"""Pins for the scorer network's oracle (CPU only): finite differences,
closed forms, exactly representable special cases and a real fp32 sum."""
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
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert mlp.bf16_round(np.float32(1.01171875)) == np.float32(1.015625)
    assert np.all(mlp.from_bf16_bits(mlp.bf16_bits(x)) == r)


def small_net(seed=1):
    g = np.random.Generator(np.random.Philox(key=3))
    net = mlp.MLP.init(seed=seed, dims=(6, 5, 4, 3, 1))
    # nonzero biases keep every pre-activation away from the ReLU kink, where
    # a central difference is not the derivative
    for b in net.b:
        b[:] = g.uniform(0.05, 0.3, size=b.shape)
    return net, g


def test_gradients_match_finite_differences():
    net, g = small_net()
    X = g.normal(size=(11, 6))
    seg = np.array([0, 3, 7, 11])
    target = np.array([0.5, -1.0, 2.0])
    loss, dW, db, _ = net.loss_and_grads(X, seg, target)
    eps = 1e-6

    def fd(arr, idx):
        w0 = arr[idx]
        arr[idx] = w0 + eps
        lp = net.loss_and_grads(X, seg, target)[0]
        arr[idx] = w0 - eps
        lm = net.loss_and_grads(X, seg, target)[0]
        arr[idx] = w0
        return (lp - lm) / (2 * eps)

    for li in range(4):
        o, i = net.W[li].shape
        for idx in {(0, 0), (o - 1, 0), (0, i - 1), (o - 1, i - 1)}:
            assert abs(fd(net.W[li], idx) - dW[li][idx]) < 1e-6 * max(1.0, abs(dW[li][idx]))
        for j in range(o):
            assert abs(fd(net.b[li], j) - db[li][j]) < 1e-6 * max(1.0, abs(db[li][j]))


def test_linear_special_case():
    """With one layer the model is linear: the least-squares solution of the
    set-sum regression zeroes the gradient."""
    g = np.random.Generator(np.random.Philox(key=4))
    X = g.normal(size=(40, 5))
    seg = np.arange(0, 41, 4)
    Xs = np.add.reduceat(X, seg[:-1], axis=0)
    w_true = g.normal(size=5)
    target = Xs @ w_true
    net = mlp.MLP([w_true[None, :]], [np.zeros(1)])
    loss, dW, db, _ = net.loss_and_grads(X, seg, target)
    assert loss < 1e-20 and np.abs(dW[0]).max() < 1e-9


def test_set_loss_hand_example():
    y = np.array([1.0, 2.0, -1.0, 0.5])
    seg = np.array([0, 2, 4])
    loss, dy = mlp.set_loss(y, seg, [2.0, 0.0])
    # scores 3 and -0.5, errors 1 and -0.5: loss (1 + 0.25) / 2
    assert loss == 0.625
    assert np.array_equal(dy, [1.0, 1.0, -0.5, -0.5])


def representable_net(g, dims=(8, 6, 6, 6, 1)):
    """Small-integer weights and features: every activation is an integer
    below 256 in magnitude, hence exact in bfloat16."""
    W = [g.integers(-1, 2, size=(dims[i + 1], dims[i])).astype(np.float64) for i in range(4)]
    b = [g.integers(-1, 2, size=dims[i + 1]).astype(np.float64) for i in range(4)]
    return mlp.MLP(W, b)


def test_mixed_recipe_equals_textbook_when_exact():
    """When every operand is exact in bfloat16 the mixed-precision forward and
    backward are the textbook ones (pins their transposes, masks and head)."""
    g = np.random.Generator(np.random.Philox(key=5))
    for trial in range(20):
        net = representable_net(g)
        X = g.integers(-2, 3, size=(16, 8)).astype(np.float64)
        seg = np.array([0, 4, 8, 12, 16])
        y_ref, _ = net.forward(X)
        y, acts, pre = net.forward_mixed(X)
        assert np.all(np.abs(np.concatenate([a.ravel() for a in acts])) < 256)
        assert np.array_equal(y, y_ref)
        target = g.integers(-4, 5, size=4).astype(np.float64)
        loss, dW_ref, db_ref, dy = net.loss_and_grads(X, seg, target)
        # dy = 2 err / 4: a multiple of 1/2, small, exact in bfloat16
        dW, db = net.backward_mixed(acts, dy)
        for l in range(4):
            assert np.array_equal(dW[l], dW_ref[l]), (trial, l)
            assert np.array_equal(db[l], db_ref[l]), (trial, l)


def test_gemm_bound_holds_for_a_real_fp32_sum():
    g = np.random.Generator(np.random.Philox(key=6))
    A = mlp.bf16_round(g.normal(size=(64, 512))).astype(np.float64)
    B = mlp.bf16_round(g.normal(size=(512, 48))).astype(np.float64)
    exact = A @ B
    # sequential fp32 accumulation of exact products (bf16 x bf16 fits fp32)
    acc = np.zeros((64, 48), np.float32)
    for k in range(512):
        acc = (acc + np.outer(A[:, k], B[k]).astype(np.float32)).astype(np.float32)
    err = np.abs(acc.astype(np.float64) - exact)
    bound = mlp.gemm_bound(A, B)
    assert np.all(err <= bound)
    assert err.max() > 0    # the bound is not vacuous for this case


def test_sgd_momentum_closed_form():
    p0 = np.array([1.0, -2.0, 0.5])
    g = np.array([0.5, 0.25, -1.0])
    p, v = p0.copy(), np.zeros(3)
    lr, mu = 0.1, 0.9
    for t in range(1, 6):
        p, v = mlp.sgd_momentum(p, g, v, lr, mu)
        # constant gradient: v_t = g (1 - mu^t) / (1 - mu)
        assert np.allclose(v, g * (1 - mu ** t) / (1 - mu), rtol=0, atol=1e-15)
    s = sum((1 - mu ** t) / (1 - mu) for t in range(1, 6))
    assert np.allclose(p, p0 - lr * g * s, rtol=0, atol=1e-14)


def test_flat_layout_round_trip():
    net = mlp.MLP.init(seed=2)
    v = net.flat()
    assert len(v) == mlp.num_params() == 64 * 256 + 256 + 2 * (256 * 256 + 256) + 256 + 1
    back = mlp.MLP.from_flat(v)
    for a, b in zip(net.W + net.b, back.W + back.b):
        assert np.array_equal(a, b)
