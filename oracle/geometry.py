"""Element geometry for the oracle: per-point metrics of the map from the
reference element [-1,1]^d to each physical element (Sec. 3.1: the
integrals of Eq. 12-13 are taken on the reference element with the
Jacobian J of that map and its face counterpart J^Gamma).

Two kinds of element:
  * affine boxes x = origin + (xi + 1) h / 2 (closed forms);
  * isoparametric elements x(xi) = sum_i X_i l_i(xi), tensor-product Lagrange
    polynomials of order P_geo through equispaced nodes xi_i = -1 + 2i/P_geo
    (node index i0 + (P_geo+1)(i1 + (P_geo+1) i2), x fastest).

Arrays (e element, q volume point, p face point, k reference and j
physical direction):
  xq[e, q, j]        physical coordinates of the volume points
  Gq[e, q, k, j]     d xi_k / d x_j at the volume points
  wJ[e, q]           Gauss weight times |J|
  Gf[f][e, p, k, j]  d xi_k / d x_j at the points of face f (the element's own map)
  nf[f][e, p, j]     outward unit normal of face f
  wJf[f][e, p]       face Gauss weight times |J^Gamma| (area element)
  vol[e], area[f][e] element volume and face area (quadrature sums for
                     curved elements, closed forms for boxes)
The outward normal and area element follow Nanson's relation
n dA = |J| (d xi_a / d x) dxi_t for face f = 2a + side (sign + for side 1).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np


def lagrange1d(nodes: np.ndarray, x: np.ndarray):
    """Lagrange basis through `nodes` at points x: V[i, k] = l_i(x_k),
    dV[i, k] = l_i'(x_k) (product rule, written out)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = nodes.size
    V = np.ones((n, x.size))
    dV = np.zeros((n, x.size))
    for i in range(n):
        others = [m for m in range(n) if m != i]
        for m in others:
            V[i] *= (x - nodes[m]) / (nodes[i] - nodes[m])
        for m in others:
            t = np.full(x.size, 1.0 / (nodes[i] - nodes[m]))
            for r in others:
                if r != m:
                    t = t * (x - nodes[r]) / (nodes[i] - nodes[r])
            dV[i] += t
    return V, dV


def map_matrices(dim: int, geo_order: int, xi: np.ndarray):
    """Dense matrices Lw[pt, node] and dLw[k][pt, node] of the tensor
    Lagrange map and its reference derivatives at the points xi[pt, :]."""
    nodes1 = -1.0 + 2.0 * np.arange(geo_order + 1) / geo_order
    npt = xi.shape[0]
    ng = geo_order + 1
    per_axis = [lagrange1d(nodes1, xi[:, a]) for a in range(dim)]
    Lw = np.ones((npt, ng ** dim))
    dLw = [np.ones((npt, ng ** dim)) for _ in range(dim)]
    for c in range(ng ** dim):
        m = [(c // ng ** a) % ng for a in range(dim)]        # node index, x fastest
        for a in range(dim):
            V, dV = per_axis[a]
            Lw[:, c] *= V[m[a]]
            for k in range(dim):
                dLw[k][:, c] *= dV[m[a]] if k == a else V[m[a]]
    return Lw, dLw


def curved_metrics(nodes: np.ndarray, geo_order: int, xi: np.ndarray):
    """(x[e, pt, j], Jm[e, pt, j, k] = d x_j / d xi_k) at the points xi."""
    dim = xi.shape[1]
    Lw, dLw = map_matrices(dim, geo_order, xi)
    x = np.einsum('pc,ecj->epj', Lw, nodes)
    Jm = np.stack([np.einsum('pc,ecj->epj', dLw[k], nodes) for k in range(dim)], axis=-1)
    return x, Jm


class Geometry:
    """Per-point metrics of all elements (see the module docstring)."""

    def __init__(self, ref, dim, elem_origin=None, elem_h=None, geo_nodes=None, geo_order=1):
        self.dim = dim
        nf = 2 * dim
        if geo_nodes is None:
            h = np.asarray(elem_h, dtype=np.float64)
            E = h.shape[0]
            self.curved = False
            self.detJ = np.prod(h / 2.0, axis=1)
            self.dxi = 2.0 / h
            self.xq = elem_origin[:, None, :] + (ref.xi[None] + 1.0) * 0.5 * h[:, None, :]
            G = np.zeros((E, dim, dim))
            for j in range(dim):
                G[:, j, j] = self.dxi[:, j]
            self.Gq = np.broadcast_to(G[:, None], (E, ref.nqv, dim, dim))
            self.wJ = ref.W[None, :] * self.detJ[:, None]
            self.vol = np.prod(h, axis=1)
            self.Gf, self.nf, self.wJf, self.area = [], [], [], []
            for f in range(nf):
                a, s = divmod(f, 2)
                fd = np.prod(np.delete(h, a, axis=1) / 2.0, axis=1)
                self.Gf.append(np.broadcast_to(G[:, None], (E, ref.nqf, dim, dim)))
                n = np.zeros((E, ref.nqf, dim))
                n[..., a] = 1.0 if s == 1 else -1.0
                self.nf.append(n)
                self.wJf.append(ref.WF[None, :] * fd[:, None])
                self.area.append(np.prod(np.delete(h, a, axis=1), axis=1))
        else:
            nodes = np.asarray(geo_nodes, dtype=np.float64)
            self.curved = True
            self.detJ = None
            self.dxi = None
            self.xq, Jm = curved_metrics(nodes, geo_order, ref.xi)
            det = np.linalg.det(Jm)
            if np.any(det <= 0.0):
                raise ValueError("element map with non-positive Jacobian")
            self.Gq = np.linalg.inv(Jm)                      # [e, q, k, j] = d xi_k / d x_j
            self.wJ = ref.W[None, :] * det
            self.vol = self.wJ.sum(axis=1)
            self.Gf, self.nf, self.wJf, self.area = [], [], [], []
            for f in range(nf):
                a, s = divmod(f, 2)
                _, Jf = curved_metrics(nodes, geo_order, ref.xif[f])
                detf = np.linalg.det(Jf)
                Gf = np.linalg.inv(Jf)
                ga = Gf[:, :, a, :]                               # d xi_a / d x
                gn = np.linalg.norm(ga, axis=-1)
                self.Gf.append(Gf)
                self.nf.append((1.0 if s == 1 else -1.0) * ga / gn[..., None])
                w = ref.WF[None, :] * detf * gn
                self.wJf.append(w)
                self.area.append(w.sum(axis=1))
