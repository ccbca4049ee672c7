"""Approximate inverses of the BRJ diagonal blocks (the paper names the block
inversion and PREC-DIAG as the costs that grow fastest with P, Sec. 5.1,
and better preconditioning as future work, Sec. 7).  TEST INFRASTRUCTURE
ONLY: evaluated against the exact blocks of the oracle's BRJ; no product
path uses it.

A block D_e of size nb = nv n^d acts on u[v][i_{d-1}]..[i_0] (flat index
v n^d + sum_k i_k n^k).  A Kronecker sum couples the variables with one
direction at a time:
    (K u)[v][i] = sum_k sum_{w, j} A_k[(v, i_k), (w, j)] u[w][i with i_k -> j]
with one (nv n) x (nv n) matrix A_k per direction k (rows and columns
ordered (variable, modal index)).  The fit takes the A_k minimising the
Frobenius norm ||D_e - K||_F, a linear least-squares problem.  Its normal
equations involve only partial traces: with P_k = ptrace_k(D) (the sum over
the modal indices of every direction but k) and tr(A) the trace of A over
its modal index (an nv x nv matrix),
    n^(d-1) A_k + n^(d-2) sum_{l != k} I_n (x) tr(A_l) = P_k,
whose solutions differ only by multiples of the identity moved between
directions; the fit takes tr(A_k) = T / d for every k, T = tr(P_k) / n^(d-1).
Because the variable index is shared by all directions, K has no cheap
exact inverse; the cheap alternating-direction form writes K = I + sum_k T_k
with T_k = A_k - I/d (along direction k) and approximates K^-1 by
prod_k (I + T_k)^-1, dropping the products of the T_k.
"""
from __future__ import annotations

import numpy as np


def _axis(d, k):
    """Tensor axis of direction k in the [v][i_{d-1}]..[i_0] layout."""
    return d - k


def apply_dir(A, X, nv, n, d, k):
    """A applied along direction k to the columns of X (X: [nb, m], every
    column a vector of the block's layout)."""
    m = X.shape[1]
    T = X.T.reshape((m, nv) + (n,) * d)                       # [col][v][i_{d-1}]..[i_0]
    ax = 1 + _axis(d, k)                                       # batch axis first
    T = np.moveaxis(T, ax, 2)                                  # [col][v][i_k][rest...]
    sh = T.shape
    T = T.reshape(m, nv * n, -1)                               # [col][(v, i_k)][rest]
    A4 = A.reshape(nv * n, nv * n)
    T = np.einsum('ab,cbr->car', A4, T)
    T = np.moveaxis(T.reshape(sh), 2, ax)
    return T.reshape(m, -1).T


def dir_operator(A, nv, n, d, k):
    """Dense nb x nb matrix of A acting along direction k."""
    nb = nv * n ** d
    return apply_dir(A, np.eye(nb), nv, n, d, k)


def kron_sum(A_list, nv, n, d):
    """K = sum over the directions of A_k acting along direction k."""
    return sum(dir_operator(A, nv, n, d, k) for k, A in enumerate(A_list))


def ptrace(D, nv, n, d, k):
    """Partial trace of a block over the modal indices of every direction
    but k: [(v, i_k), (w, j_k)] entries sum_{rest} D[(v, i_k, rest), (w, j_k, rest)]."""
    T = D.reshape((nv,) + (n,) * d + (nv,) + (n,) * d)
    ax = _axis(d, k)
    rows = [a for a in range(1, d + 1) if a != ax]
    cols = [d + 1 + a for a in rows]
    # sum over the matched (row, column) pairs of the other directions
    letters = 'abcdefghijklmnopqrstuvwxyz'
    sub_in = list(letters[:2 * (d + 1)])
    for r, c in zip(rows, cols):
        sub_in[c] = sub_in[r]
    out = [sub_in[0], sub_in[ax], sub_in[d + 1], sub_in[d + 1 + ax]]
    P = np.einsum(''.join(sub_in) + '->' + ''.join(out), T)
    return P.reshape(nv * n, nv * n)


def mode_trace(A, nv, n):
    """tr over the modal index of an (nv n) x (nv n) matrix: [v, w]."""
    return np.einsum('aibi->ab', A.reshape(nv, n, nv, n))


def fit_kron_sum(D, nv, n, d):
    """The least-squares Kronecker-sum fit of the block D from the normal
    equations above."""
    P = [ptrace(D, nv, n, d, k) for k in range(d)]
    T = mode_trace(P[0], nv, n) / n ** (d - 1)
    shift = np.kron(T, np.eye(n))        # [(v, i), (w, j)] = T[v, w] delta_ij
    return [(Pk - n ** (d - 2) * (d - 1) / d * shift) / n ** (d - 1) for Pk in P]


def fit_kron_sum_lstsq(D, nv, n, d):
    """The same fit by numpy.linalg.lstsq on the entries of the A_k (small
    blocks only: nb^2 equations in d (nv n)^2 unknowns); returns the fitted
    operator K, which is unique."""
    m = nv * n
    cols = []
    for k in range(d):
        for a in range(m):
            for b in range(m):
                E = np.zeros((m, m))
                E[a, b] = 1.0
                cols.append(dir_operator(E, nv, n, d, k).ravel())
    G = np.stack(cols, axis=1)
    x, *_ = np.linalg.lstsq(G, D.ravel(), rcond=None)
    return (G @ x).reshape(D.shape)


def adi_inverse(A_list, nv, n, d):
    """The alternating-direction approximation of kron_sum(A)^-1:
    prod_k (I + T_k)^-1 with T_k = A_k - I/d along direction k."""
    nb = nv * n ** d
    m = nv * n
    P = np.eye(nb)
    for k, A in enumerate(A_list):
        Tk = dir_operator(A - np.eye(m) / d, nv, n, d, k)
        P = P @ np.linalg.inv(np.eye(nb) + Tk)
    return P
