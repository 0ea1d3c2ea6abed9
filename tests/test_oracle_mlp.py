"""Pins of the float64 cost-model network: central finite differences,
closed forms of Adam's first step and of a network reduced to its bias."""
import numpy as np

import oracle.mlp as mlp


def _data(n, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, mlp.IN)), rng.normal(size=n)


def test_parameter_count():
    assert mlp.NPARAM == 64 * 13 + 64 + 64 * 64 + 64 + 64 + 1 == 5121


def test_gradient_matches_central_differences():
    X, t = _data(7, 0)
    p = mlp.init_params(1)
    _, g = mlp.loss_and_grad(p, X, t)
    rng = np.random.default_rng(2)
    idx = rng.choice(mlp.NPARAM, size=60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss_and_grad(p + e, X, t)[0] - mlp.loss_and_grad(p - e, X, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_zero_weights_output_is_bias_and_only_b3_moves():
    X, t = _data(5, 3)
    q = mlp.unflatten(np.zeros(mlp.NPARAM))
    q["b3"][:] = 0.75
    y, cache = mlp.forward(q, X)
    assert np.all(y == 0.75)
    g = mlp.backward(q, cache, y, t)
    assert np.isclose(g["b3"][0], 2.0 * np.mean(0.75 - t))
    for name in ("W1", "b1", "W2", "b2", "W3"):
        assert np.all(g[name] == 0.0)


def test_adam_first_step_is_lr_times_sign():
    opt = mlp.Adam(3, lr=0.01)
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([3.0, -0.25, 1e-3])
    new = opt.step(p, g)
    # after one step mhat = g and vhat = g^2, so the move is lr * g / (|g| + eps)
    assert np.allclose(new, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_fits_log_volume():
    # the network can learn y = ln M + ln N + ln K on standardised inputs
    rng = np.random.default_rng(4)
    dims = np.exp(rng.uniform(np.log(64), np.log(8192), size=(256, 3)))
    X = np.zeros((256, mlp.IN))
    X[:, :3] = np.log(dims)
    X = (X - X.mean(0)) / np.where(X.std(0) > 0, X.std(0), 1)
    t = np.log(dims).sum(1)
    t = (t - t.mean()) / t.std()
    p = mlp.init_params(5)
    opt = mlp.Adam(mlp.NPARAM, lr=3e-3)
    for _ in range(400):
        _, g = mlp.loss_and_grad(p, X, t)
        p = opt.step(p, g)
    assert mlp.loss_and_grad(p, X, t)[0] < 1e-3


def test_adam_bias_correction_constant_gradient_every_step():
    # under a constant gradient g the moments are m_t = (1 - b1^t) g and
    # v_t = (1 - b2^t) g^2, so bias correction restores mhat = g and
    # vhat = g^2 at every step t and each step moves lr * g / (|g| + eps);
    # dividing by 1 - b1 (or 1 - b2) instead of 1 - b1^t moves the parameters
    # by a different amount from t = 2 on
    opt = mlp.Adam(3, lr=0.01)
    p0 = np.array([0.5, -1.0, 2.0])
    g = np.array([0.3, -4.0, 1e-2])
    p = p0.copy()
    for t in range(1, 7):
        p = opt.step(p, g)
        assert np.allclose(p, p0 - t * 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-13), t


def test_adam_two_different_gradients_by_hand():
    # g1 = 1, g2 = -2, b1 = 0.9, b2 = 0.999, lr = 0.1, worked by hand:
    #   m1 = 0.1, v1 = 0.001 (step 1 moves by lr: mhat = 1, vhat = 1)
    #   m2 = 0.9 * 0.1 + 0.1 * (-2) = -0.11
    #   v2 = 0.999 * 0.001 + 0.001 * 4 = 0.004999
    #   mhat = -0.11 / (1 - 0.81) = -11/19
    #   vhat = 0.004999 / (1 - 0.998001) = 4999/1999
    opt = mlp.Adam(1, lr=0.1)
    p = np.array([0.25])
    p = opt.step(p, np.array([1.0]))
    assert np.isclose(p[0], 0.25 - 0.1 / (1.0 + 1e-8), rtol=0, atol=1e-15)
    p = opt.step(p, np.array([-2.0]))
    assert np.isclose(opt.m[0], -0.11, rtol=0, atol=1e-15)
    assert np.isclose(opt.v[0], 0.004999, rtol=0, atol=1e-15)
    want = 0.25 - 0.1 / (1.0 + 1e-8) + 0.1 * (11.0 / 19.0) / (np.sqrt(4999.0 / 1999.0) + 1e-8)
    assert np.isclose(p[0], want, rtol=0, atol=1e-14)
    assert np.isclose(p[0], 0.1866103534720751, rtol=0, atol=1e-13)
