"""Pins of the oracle's MLP: the reverse-mode gradient against central
differences, a linear special case against least squares, and Adam against
its closed form on a quadratic."""
import numpy as np

from oracle import mlp


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    n_in, H, n_out, R = 7, 5, 4, 9
    th = rng.normal(size=mlp.n_params(n_in, H, n_out)) * 0.5
    X = rng.normal(size=(R, n_in))
    T = rng.normal(size=(R, n_out))
    g = mlp.grad(th, X, T, n_in, H, n_out)
    h = 1e-6
    for k in rng.choice(th.size, 40, replace=False):
        e = np.zeros_like(th)
        e[k] = h
        fd = (mlp.loss(th + e, X, T, n_in, H, n_out) - mlp.loss(th - e, X, T, n_in, H, n_out)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k]))


def test_small_weights_reduce_to_linear_model():
    """With tiny hidden pre-activations tanh is the identity to first order,
    so the network is the product of its matrices."""
    rng = np.random.default_rng(1)
    n_in, H, n_out = 6, 8, 3
    th = rng.normal(size=mlp.n_params(n_in, H, n_out)) * 1e-4
    W1, b1, W2, b2, W3, b3 = mlp.unpack(th, n_in, H, n_out)
    X = rng.normal(size=(5, n_in))
    Y, _ = mlp.forward(th, X, n_in, H, n_out)
    lin = ((X @ W1 + b1) @ W2 + b2) @ W3 + b3
    assert np.allclose(Y, lin, rtol=0, atol=1e-12)


def test_features_targets_guess_roundtrip():
    rng = np.random.default_rng(2)
    S = rng.normal(size=(4, 3, 5))
    inc1 = rng.normal(size=(4, 3, 5))
    inc2 = rng.normal(size=(4, 3, 5))
    s_inc = np.array([0.5, 0.25, 2.0])
    s_out = np.array([0.1, 3.0, 0.7])
    X = mlp.features(inc1, inc2, s_inc, s_out)
    assert X.shape == (4, 30)
    assert np.allclose(X[:, :15].reshape(4, 3, 5) * s_inc[None, :, None], inc1)
    assert np.allclose(X[:, 15:].reshape(4, 3, 5) * s_out[None, :, None], inc1 - inc2)
    inc_new = inc1 + rng.normal(size=inc1.shape) * 0.1
    y = mlp.targets(inc_new, inc1, s_out)
    assert np.allclose(mlp.guess(S, inc1, y, s_out), S + inc_new)
    # a zero prediction is the extrapolated guess
    assert np.allclose(mlp.guess(S, inc1, 0 * y, s_out), S + inc1)
    s2, s3 = mlp.scales([[inc2, inc2], [inc1, inc1]])
    assert np.allclose(s2, np.sqrt(np.mean(np.stack([inc2, inc1]) ** 2, axis=(0, 1, 3))))
    assert np.allclose(s3, np.sqrt(np.mean((inc1 - inc2) ** 2, axis=(0, 2))))


def test_adam_first_step_is_sign_step():
    th = np.array([1.0, -2.0, 3.0])
    g = np.array([0.3, -5.0, 1e-3])
    t1, m, v = mlp.adam(th, g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    assert np.allclose(t1, th - 0.1 * g / (np.abs(g) + 1e-8))
