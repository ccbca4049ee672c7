"""Pins of the oracle's MLP: the reverse-mode gradients (regression and
pooled-blend losses) against central differences, a linear special case,
the blend guess against extrapolation theory (exact for quadratic
increments), the pooled loss against least squares, and Adam against its
closed form."""
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


def test_features_and_scale():
    """Rows are the element's last two increment differences over the
    per-variable RMS of the first; a variable with no change gets scale 1."""
    rng = np.random.default_rng(2)
    i1, i2, i3 = (rng.normal(size=(4, 3, 5)) for _ in range(3))
    i2[:, 2, :] = i1[:, 2, :]                     # variable 2 unchanged
    X, s = mlp.features(i1, i2, i3)
    assert X.shape == (4, 30)
    assert s[2] == 1.0
    for v in (0, 1):
        assert np.isclose(s[v], np.sqrt(np.mean((i1[:, v] - i2[:, v]) ** 2)))
    assert np.allclose(X[:, :15].reshape(4, 3, 5) * s[None, :, None], i1 - i2)
    assert np.allclose(X[:, 15:].reshape(4, 3, 5) * s[None, :, None], i2 - i3)


def test_blend_guess_special_cases_and_polynomial_exactness():
    """c = 0 is the extrapolated guess S + 2 i1 - i2, c = (-1, 0) the
    one-step guess S + i1, c = (0, 1) third-order extrapolation
    S + 3 i1 - 3 i2 + i3, which reproduces increments quadratic in the step
    index exactly (its error is the third difference)."""
    rng = np.random.default_rng(3)
    S = rng.normal(size=(3, 4, 6))
    a, b, q = (rng.normal(size=(3, 4, 6)) for _ in range(3))
    inc = lambda k: a + b * k + q * k * k
    n = 7
    i1, i2, i3 = inc(n - 1), inc(n - 2), inc(n - 3)
    assert np.allclose(mlp.blend_guess(S, i1, i2, i3, (0.0, 0.0)), S + 2 * i1 - i2)
    assert np.allclose(mlp.blend_guess(S, i1, i2, i3, (-1.0, 0.0)), S + i1)
    assert np.allclose(mlp.blend_guess(S, i1, i2, i3, (0.0, 1.0)), S + 3 * i1 - 3 * i2 + i3)
    assert np.allclose(mlp.blend_guess(S, i1, i2, i3, (0.0, 1.0)), S + inc(n), rtol=0, atol=1e-9)
    # the extrapolated guess is exact only for increments linear in k
    assert not np.allclose(mlp.blend_guess(S, i1, i2, i3, (0.0, 0.0)), S + inc(n), atol=1e-3)


def test_pooled_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    n_in, H, n_out, R = 8, 6, 2, 7
    th = rng.normal(size=mlp.n_params(n_in, H, n_out)) * 0.5
    X = rng.normal(size=(R, n_in))
    inc, i1, i2, i3 = (rng.normal(size=(R, 2, 4)) for _ in range(4))
    terms = mlp.blend_terms(inc, i1, i2, i3)
    g, _ = mlp.pooled_grad(th, X, terms, n_in, H, n_out)
    h = 1e-6
    for k in range(th.size):
        e = np.zeros_like(th)
        e[k] = h
        fd = (mlp.pooled_loss(th + e, X, terms, n_in, H, n_out) -
              mlp.pooled_loss(th - e, X, terms, n_in, H, n_out)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k]))


def test_pooled_loss_is_the_least_squares_blend_error():
    """With a constant network output c (W3 = 0, b3 = c) the loss is
    ||F c - r||^2 / ||r||^2; its minimum over c is the least-squares blend of
    the two directions (numpy's lstsq), with the gradient zero there."""
    rng = np.random.default_rng(5)
    n_in, H, n_out, R = 6, 4, 2, 5
    inc, i1, i2, i3 = (rng.normal(size=(R, 3, 4)) for _ in range(4))
    terms = mlp.blend_terms(inc, i1, i2, i3)
    F = np.stack([(i1 - i2).ravel(), (i1 - 2 * i2 + i3).ravel()], axis=1)
    r = (inc - 2 * i1 + i2).ravel()
    cstar, *_ = np.linalg.lstsq(F, r, rcond=None)
    th = rng.normal(size=mlp.n_params(n_in, H, n_out))
    W1, b1, W2, b2, W3, b3 = mlp.unpack(th, n_in, H, n_out)
    o = th.size - n_out - H * n_out
    th[o:o + H * n_out] = 0.0
    th[-n_out:] = cstar
    X = rng.normal(size=(R, n_in))
    L = mlp.pooled_loss(th, X, terms, n_in, H, n_out)
    assert np.isclose(L, np.sum((F @ cstar - r) ** 2) / np.sum(r ** 2), rtol=1e-12)
    _, dLdc = mlp.pooled_grad(th, X, terms, n_in, H, n_out)
    assert np.allclose(dLdc, 0.0, atol=1e-12)
    for dc in ((1e-3, 0.0), (0.0, -1e-3)):
        th2 = th.copy()
        th2[-n_out:] = cstar + np.array(dc)
        assert mlp.pooled_loss(th2, X, terms, n_in, H, n_out) > L


def test_adam_first_step_is_sign_step():
    th = np.array([1.0, -2.0, 3.0])
    g = np.array([0.3, -5.0, 1e-3])
    t1, m, v = mlp.adam(th, g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    assert np.allclose(t1, th - 0.1 * g / (np.abs(g) + 1e-8))
