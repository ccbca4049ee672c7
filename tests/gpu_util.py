"""Helpers of the GPU parity tests."""
import numpy as np

import workloads as W
from oracle.dg import Disc, make_disc
from oracle.physics import Gas


def rel_err_per_var(a, b):
    """max over variables of max|a_v - b_v| / max|b_v|."""
    errs = []
    for v in range(b.shape[1]):
        s = np.abs(b[:, v]).max()
        errs.append(np.abs(a[:, v] - b[:, v]).max() / (s if s > 0 else 1.0))
    return max(errs)


def setup(dim, cells, P, lengths=None, **over):
    """(cfg, mesh, oracle disc) for a periodic box."""
    import dataclasses
    base = W.config(1 if dim == 2 else 2)
    if lengths is None:
        lengths = tuple(1.0 + 0.3 * i for i in range(dim))
    cfg = dataclasses.replace(base, dim=dim, ncells=tuple(cells), lengths=tuple(lengths), P=P, nq=P + 2, **over)
    mesh = W.cartesian_mesh(cfg.ncells, cfg.lengths)
    disc = make_disc(cfg, mesh)
    return cfg, mesh, disc
