"""Orthonormal tensor-product Legendre basis and Gauss quadrature.

The paper leaves the expansion open (Sec. 4.3 lists nodal and modal bases);
this oracle uses the modal tensor space Q^P on quadrilaterals/hexahedra
with phi_i(xi) = sqrt((2i+1)/2) P_i(xi), and Gauss-Legendre quadrature with
nq points per direction (Eq. 10: N_Q volume and N_Q^Gamma face points).
The matrices built here are the backward transform B (B_iq = phi_q(x_i),
Sec. 3.1), the reference derivative matrices D_j B and the face matrices
B^Gamma of Eq. 13, evaluated directly at the face quadrature points.
"""
from __future__ import annotations

import itertools
from functools import lru_cache

import numpy as np
from numpy.polynomial import legendre as npleg


def phi1d(P: int, x: np.ndarray):
    """Values and derivatives of the orthonormal Legendre functions:
    V[i, k] = phi_i(x_k), dV[i, k] = phi_i'(x_k), i = 0..P."""
    x = np.asarray(x, dtype=np.float64)
    V = np.zeros((P + 1, x.size))
    dV = np.zeros((P + 1, x.size))
    for i in range(P + 1):
        c = np.zeros(i + 1)
        c[i] = np.sqrt((2 * i + 1) / 2.0)
        V[i] = npleg.legval(x, c)
        dV[i] = npleg.legval(x, npleg.legder(c)) if i > 0 else 0.0
    return V, dV


def gauss(nq: int):
    """Gauss-Legendre nodes and weights on [-1, 1]."""
    return npleg.leggauss(nq)


def mode_multi(dim: int, P: int):
    """Multi-indices of the modes, mode m = i0 + n*(i1 + n*i2)."""
    n = P + 1
    out = []
    for m in range(n ** dim):
        r, mi = m, []
        for _ in range(dim):
            mi.append(r % n)
            r //= n
        out.append(tuple(mi))
    return out


def point_multi(dim: int, nq: int):
    """Multi-indices of tensor quadrature points, q = a0 + nq*(a1 + nq*a2)."""
    return mode_multi(dim, nq - 1)


class RefElement:
    """Dense reference-element operators for dimension dim, order P and
    nq Gauss points per direction.

    B[q, m]          phi_m at volume point q
    D[j][q, m]       d phi_m / d xi_j at volume point q
    W[q]             tensor Gauss weight
    BF[f][p, m]      phi_m at point p of face f = 2*axis + side
    DF[f][j][p, m]   d phi_m / d xi_j at that face point
    WF[p]            tensor Gauss weight of the (dim-1)-dimensional face rule
    xi[q, :]         reference coordinates of the volume points
    xif[f][p, :]     reference coordinates of the face points
    Face points run over the tangential axes in increasing order, the first
    tangential axis fastest; the two faces across an interface therefore
    list their points in the same order.
    """

    def __init__(self, dim: int, P: int, nq: int):
        self.dim, self.P, self.nq = dim, P, nq
        self.n = P + 1
        x, w = gauss(nq)
        self.x1, self.w1 = x, w
        modes = mode_multi(dim, P)
        pts = point_multi(dim, nq)
        self.nm, self.nqv = len(modes), len(pts)

        def evalp(coords):
            # coords: [npts, dim] reference points -> (B, [D_j])
            npts = coords.shape[0]
            Vs, dVs = zip(*[phi1d(P, coords[:, a]) for a in range(dim)])
            Bm = np.ones((npts, len(modes)))
            Dm = [np.ones((npts, len(modes))) for _ in range(dim)]
            for mi, m in enumerate(modes):
                for a in range(dim):
                    Bm[:, mi] *= Vs[a][m[a]]
                    for j in range(dim):
                        Dm[j][:, mi] *= (dVs[a][m[a]] if j == a else Vs[a][m[a]])
            return Bm, Dm

        self.xi = np.array([[x[p[a]] for a in range(dim)] for p in pts])
        self.W = np.array([np.prod([w[p[a]] for a in range(dim)]) for p in pts])
        self.B, self.D = evalp(self.xi)
        fpts = point_multi(dim - 1, nq) if dim > 1 else [()]
        self.nqf = len(fpts)
        self.WF = np.array([np.prod([w[p[t]] for t in range(dim - 1)]) for p in fpts])
        self.BF, self.DF, self.xif = [], [], []
        for axis in range(dim):
            tang = [a for a in range(dim) if a != axis]
            for side in (0, 1):
                c = np.zeros((len(fpts), dim))
                c[:, axis] = -1.0 if side == 0 else 1.0
                for t, a in enumerate(tang):
                    c[:, a] = [x[p[t]] for p in fpts]
                Bf, Df = evalp(c)
                self.BF.append(Bf)
                self.DF.append(Df)
                self.xif.append(c)


@lru_cache(maxsize=None)
def ref_element(dim: int, P: int, nq: int) -> RefElement:
    return RefElement(dim, P, nq)
