"""Pins of the FP64 MLP reference (oracle/mlp.py): analytic gradients against central finite
differences, the loss derivative likewise, and Adam against its first-step closed form."""
import numpy as np

from oracle import mlp


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init(rng)
    X = rng.random((37, mlp.IN))
    w = rng.standard_normal(37)
    _, cache = mlp.forward(theta, X)
    g = mlp.backward(theta, cache, w)
    f = lambda t: float(w @ mlp.forward(t, X)[0])
    idx = rng.choice(mlp.NPARAMS, 300, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros(mlp.NPARAMS)
        e[k] = h
        fd = (f(theta + e) - f(theta - e)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_bce_derivative_matches_finite_differences():
    rng = np.random.default_rng(1)
    s = rng.standard_normal(50) * 3
    y = (rng.random(50) < 0.3).astype(float)
    loss, ds = mlp.bce(s, y, 4.0)
    h = 1e-6
    for k in range(50):
        e = np.zeros(50)
        e[k] = h
        fd = (mlp.bce(s + e, y, 4.0)[0] - mlp.bce(s - e, y, 4.0)[0]) / (2 * h)
        assert abs(fd - ds[k]) < 1e-8
    # y = 1 with a large positive score and y = 0 with a large negative score cost ~0
    assert mlp.bce(np.array([40.0, -40.0]), np.array([1.0, 0.0]), 1.0)[0] < 1e-15


def test_adam_first_step_is_signed_lr():
    g = np.array([0.5, -2.0, 1e-3])
    t, m1, m2 = mlp.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(t, -0.01 * np.sign(g))
