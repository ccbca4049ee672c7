"""Per-element MLP that predicts the Newton initial guess (not in the paper:
the paper starts Newton from S_m, Eq. 21).  TEST INFRASTRUCTURE ONLY.

With inc_n = (u^m - S_m)_n the converged increment of stage m at step n,
the features of element e at stage m of step n are (all FP64 here)
    x = [ inc_{n-1}[e] / s_inc,  (inc_{n-1} - inc_{n-2})[e] / s_out ]   (2 nb values)
and the target / prediction is the correction of the extrapolated increment,
    y = (inc_n - inc_{n-1})[e] / s_out                                   (nb values)
with per-variable scales s_inc (RMS of the increments) and s_out (RMS of
their step-to-step change) broadcast over the modes of each variable; the
guess is S_m + inc_{n-1} + s_out * y (a zero output gives the extrapolated
guess S_m + inc_{n-1}).

Network: z1 = x W1 + b1, h1 = tanh z1, z2 = h1 W2 + b2, h2 = tanh z2,
y = h2 W3 + b3; loss = mean over rows and outputs of (y - t)^2.  Parameters
are packed flat as W1[n_in][H], b1[H], W2[H][H], b2[H], W3[H][n_out],
b3[n_out] (row-major, W[in][out]).
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


def loss(theta, X, T, n_in, hidden, n_out):
    Y, _ = forward(theta, X, n_in, hidden, n_out)
    return float(np.mean((Y - T) ** 2))


def grad(theta, X, T, n_in, hidden, n_out):
    """Gradient of the mean squared error by reverse-mode differentiation."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, hidden, n_out)
    Y, (X, h1, h2) = forward(theta, X, n_in, hidden, n_out)
    dY = 2.0 * (Y - T) / Y.size
    gW3 = h2.T @ dY
    gb3 = dY.sum(0)
    dz2 = (dY @ W3.T) * (1.0 - h2 ** 2)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2.T) * (1.0 - h1 ** 2)
    gW1 = X.T @ dz1
    gb1 = dz1.sum(0)
    return np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def features(inc_prev, inc_prev2, s_inc, s_out):
    """x rows per element from the two previous increments (layout [e][v][m])."""
    E, nv, nm = inc_prev.shape
    a = inc_prev / s_inc[None, :, None]
    b = (inc_prev - inc_prev2) / s_out[None, :, None]
    return np.concatenate([a.reshape(E, nv * nm), b.reshape(E, nv * nm)], axis=1)


def targets(inc, inc_prev, s_out):
    E, nv, nm = inc.shape
    return ((inc - inc_prev) / s_out[None, :, None]).reshape(E, nv * nm)


def guess(S, inc_prev, y, s_out):
    E, nv, nm = S.shape
    return S + inc_prev + y.reshape(E, nv, nm) * s_out[None, :, None]


def scales(inc_list):
    """Per-variable RMS of the increments and of their step-to-step change
    over recorded stages (list indexed [step][stage])."""
    def rms(arrs):
        a = np.stack(arrs)
        return np.sqrt(np.mean(a ** 2, axis=tuple(i for i in range(a.ndim) if i != a.ndim - 2)))
    inc_all = [x for step in inc_list for x in step]
    d_all = [inc_list[n][m] - inc_list[n - 1][m] for n in range(1, len(inc_list)) for m in range(len(inc_list[n]))]
    return rms(inc_all), rms(d_all)


def adam(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
