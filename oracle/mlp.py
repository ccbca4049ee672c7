"""Per-element MLP behind the learned Newton initial guess (not in the paper:
the paper starts Newton from S_m, Eq. 21).  TEST INFRASTRUCTURE ONLY.

With inc_n = (u^m - S_m)_n the converged increment of stage m at step n and
i_k = inc_{n-k}, the guess of stage m at step n is
    g = S_m + 2 i_1 - i_2 + c0 (i_1 - i_2) + c1 (i_1 - 2 i_2 + i_3)
(c = 0: the extrapolated guess, c = (0, 1): third-order extrapolation),
with the blend c the mean over the elements of the network's two outputs
for the element features
    x_e = [ (i_1 - i_2)[e] / s,  (i_2 - i_3)[e] / s ]    (2 nb values)
s the per-variable RMS of i_1 - i_2 over all elements (1 where it is zero),
broadcast over the modes of each variable.  One training sample (a recorded
stage) has the loss ||F c - r||^2 / ||r||^2 with F c the blend term above
and r = inc_n - (2 i_1 - i_2) the extrapolated guess's error.

Network: z1 = x W1 + b1, h1 = tanh z1, z2 = h1 W2 + b2, h2 = tanh z2,
y = h2 W3 + b3.  Parameters are packed flat as W1[n_in][H], b1[H], W2[H][H],
b2[H], W3[H][n_out], b3[n_out] (row-major, W[in][out]).
"""
from __future__ import annotations

import numpy as np


def sizes(n_in: int, hidden: int, n_out: int):
    return [(n_in, hidden), (hidden,), (hidden, hidden), (hidden,), (hidden, n_out), (n_out,)]


def n_params(n_in: int, hidden: int, n_out: int) -> int:
    return int(sum(np.prod(s) for s in sizes(n_in, hidden, n_out)))


def unpack(theta, n_in, hidden, n_out):
    out, o = [], 0
    for s in sizes(n_in, hidden, n_out):
        k = int(np.prod(s))
        out.append(np.asarray(theta[o:o + k], dtype=np.float64).reshape(s))
        o += k
    return out


def forward(theta, X, n_in, hidden, n_out):
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, hidden, n_out)
    h1 = np.tanh(X @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    return h2 @ W3 + b3, (X, h1, h2)


def backprop(theta, X, dY, n_in, hidden, n_out):
    """Gradient with respect to the parameters of a loss whose gradient with
    respect to the network outputs is dY (reverse-mode differentiation)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, hidden, n_out)
    _, (X, h1, h2) = forward(theta, X, n_in, hidden, n_out)
    gW3 = h2.T @ dY
    gb3 = dY.sum(0)
    dz2 = (dY @ W3.T) * (1.0 - h2 ** 2)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2.T) * (1.0 - h1 ** 2)
    gW1 = X.T @ dz1
    gb1 = dz1.sum(0)
    return np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def loss(theta, X, T, n_in, hidden, n_out):
    """Mean squared error against targets T (the generic regression loss)."""
    Y, _ = forward(theta, X, n_in, hidden, n_out)
    return float(np.mean((Y - T) ** 2))


def grad(theta, X, T, n_in, hidden, n_out):
    Y, _ = forward(theta, X, n_in, hidden, n_out)
    return backprop(theta, X, 2.0 * (Y - T) / Y.size, n_in, hidden, n_out)


# ---------------------------------------------------------------- the learned guess
def features(i1, i2, i3):
    """x rows per element ([e][v][m] increments) and the per-variable scale."""
    E, nv, nm = i1.shape
    d1 = i1 - i2
    s = np.sqrt(np.mean(d1 ** 2, axis=(0, 2)))
    s = np.where(s > 0.0, s, 1.0)
    a = d1 / s[None, :, None]
    b = (i2 - i3) / s[None, :, None]
    return np.concatenate([a.reshape(E, nv * nm), b.reshape(E, nv * nm)], axis=1), s


def blend_guess(S, i1, i2, i3, c):
    return S + 2.0 * i1 - i2 + c[0] * (i1 - i2) + c[1] * (i1 - 2.0 * i2 + i3)


def pooled(theta, X, n_in, hidden, n_out):
    """The blend: mean over the rows (elements) of the network's outputs."""
    Y, _ = forward(theta, X, n_in, hidden, n_out)
    return Y.mean(axis=0)


def blend_terms(inc, i1, i2, i3):
    """G = F^T F, h = F^T r, e2 = r^T r of one sample (F: the two blend
    directions as columns, r: the extrapolated guess's error)."""
    F = np.stack([(i1 - i2).ravel(), (i1 - 2.0 * i2 + i3).ravel()], axis=1)
    r = (inc - (2.0 * i1 - i2)).ravel()
    return F.T @ F, F.T @ r, float(r @ r)


def pooled_loss(theta, X, terms, n_in, hidden, n_out):
    G, h, e2 = terms
    c = pooled(theta, X, n_in, hidden, n_out)
    return float((c @ G @ c - 2.0 * h @ c + e2) / e2)


def pooled_grad(theta, X, terms, n_in, hidden, n_out):
    """Gradient of pooled_loss: dL/dc = 2 (G c - h) / e2, every row's output
    gradient dL/dc / R."""
    G, h, e2 = terms
    c = pooled(theta, X, n_in, hidden, n_out)
    dLdc = 2.0 * (G @ c - h) / e2
    R = X.shape[0]
    return backprop(theta, X, np.tile(dLdc / R, (R, 1)), n_in, hidden, n_out), dLdc


def adam(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
