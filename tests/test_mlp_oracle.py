"""Pins of the FP64 network oracle of the learned activation proposal:
finite differences, a closed form and Adam's first step."""
import numpy as np

from oracle import mlp_oracle as M


def _data(seed, n=40):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.normal(size=(n, M.IN)) * 2.0 + 1.0
    y = (rng.random(n) < 0.4).astype(np.float64)
    mean = rng.normal(size=M.IN) * 0.5
    istd = 1.0 / (0.5 + rng.random(M.IN))
    p = M.init_params(seed, mean, istd)
    p[M.TRAINABLE_FROM:] += rng.normal(size=M.NPARAMS - M.TRAINABLE_FROM) * 0.05  # nonzero biases
    return p, x, y


def test_gradient_matches_central_differences():
    p, x, y = _data(1)
    g = M.grad(p, x, y)
    rng = np.random.Generator(np.random.PCG64(7))
    idx = np.concatenate([rng.choice(np.arange(M.TRAINABLE_FROM, M.NPARAMS), 60, replace=False),
                          [M.NPARAMS - 1, M.TRAINABLE_FROM, M.TRAINABLE_FROM + 64 * 12]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (M.loss(p + e, x, y) - M.loss(p - e, x, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])
    assert np.all(g[:M.TRAINABLE_FROM] == 0.0)


def test_constant_network_closed_form():
    """All weights zero: every logit is b3, the loss is the cross-entropy of
    a constant probability and d loss / d b3 = sigmoid(b3) - mean(y)."""
    p, x, y = _data(2)
    d = M.unpack(p)
    for k in ("W1", "b1", "W2", "b2", "w3"):
        d[k] = np.zeros_like(d[k])
    c = 0.7
    d["b3"] = np.array([c])
    q = M.pack(d)
    s = 1.0 / (1.0 + np.exp(-c))
    expect = -np.mean(y * np.log(s) + (1 - y) * np.log(1 - s))
    assert abs(M.loss(q, x, y) - expect) < 1e-14
    g = M.grad(q, x, y)
    assert abs(g[-1] - (s - y.mean())) < 1e-15
    assert np.all(g[M.TRAINABLE_FROM:-1] == 0.0)


def test_adam_first_step_is_signed_learning_rate():
    """After one step the bias-corrected moments are g and g^2, so every
    trainable parameter moves by lr * g / (|g| + eps)."""
    p, x, y = _data(3)
    g = M.grad(p, x, y)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    lr, eps = 1e-2, 1e-8
    q, m1, v1 = M.adam(p, g, m, v, 1, lr=lr, eps=eps)
    sl = slice(M.TRAINABLE_FROM, None)
    np.testing.assert_allclose(q[sl], p[sl] - lr * g[sl] / (np.abs(g[sl]) + eps), rtol=1e-12, atol=1e-15)
    assert np.array_equal(q[:M.TRAINABLE_FROM], p[:M.TRAINABLE_FROM])
