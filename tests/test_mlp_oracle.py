"""Pins of the numpy FP64 rank-MLP reference: central finite differences of the loss, the
parameter count, Adam on a convex quadratic, and features against the box geometry."""
import numpy as np

from oracle import mlp


def _data(n=37, seed=1):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 4))
    y = rng.standard_normal(n)
    return X, y


def test_parameter_count():
    assert mlp.N_PARAMS == 4545
    th = mlp.he_init(0)
    assert th.shape == (4545,)
    assert np.array_equal(mlp.pack(mlp.unpack(th)), th)


def test_gradient_matches_central_differences():
    X, y = _data()
    th = mlp.he_init(3)
    # move the biases off zero so that every ReLU is away from its kink
    p = mlp.unpack(th)
    p["b1"] += 0.05
    p["b2"] += 0.05
    th = mlp.pack(p)
    loss, g = mlp.loss_and_grad(th, X, y)
    rng = np.random.default_rng(5)
    idx = rng.choice(th.size, 120, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (mlp.loss_and_grad(th + e, X, y)[0] - mlp.loss_and_grad(th - e, X, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_zero_loss_at_exact_fit():
    X, y = _data()
    th = mlp.he_init(0)
    o, _ = mlp.forward(th, X)
    loss, g = mlp.loss_and_grad(th, X, o)
    assert loss == 0.0 and np.abs(g).max() == 0.0


def test_adam_minimises_quadratic():
    c = np.array([1.0, -2.0, 3.0])
    th = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    for t in range(1, 3001):
        th, m, v = mlp.adam_step(th, 2 * (th - c), m, v, t, lr=1e-2)
    assert np.abs(th - c).max() < 1e-3


def test_block_features():
    f = mlp.block_features([64, 32], [128, 32], [0.5, 0.1], [0.25, 0.3], [1.0, 0.6], 40.0)
    assert np.allclose(f[0], [6, 7, np.log(2.0), 40 * 0.5 / (2 * np.pi)])
    assert np.allclose(f[1], [5, 5, np.log(2.0), 40 * 0.3 / (2 * np.pi)])
