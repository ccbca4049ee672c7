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


def step_errs(a, b, vector_scale=False):
    """Per-variable relative error of a stepped state a against b:
    max|a_v - b_v| / max|b_v| for each conserved variable v.  vector_scale:
    the momentum components (a vector) share one scale, the largest of
    their maxima -- for states where one component vanishes in the exact
    solution and its discrete values are at the discretisation-error level."""
    nv = b.shape[1]
    scale = np.array([np.abs(b[:, v]).max() for v in range(nv)])
    if vector_scale:
        scale[1:nv - 1] = scale[1:nv - 1].max()
    scale[scale == 0] = 1.0
    return np.array([float(np.abs(a[:, v] - b[:, v]).max() / scale[v]) for v in range(nv)])


# Plain FP64 steps on the device and in the oracle take the same Newton and
# GMRES iteration counts; Newton contracts the rounding differences of the
# two summation orders, so the stepped states agree to this bar per variable.
STEP_TOL = 1e-12


def assert_step(a, b, label, tol=STEP_TOL, vector_scale=False):
    """Assert the per-variable step error and print it (the achieved value
    is reported with every plain-step parity case)."""
    e = step_errs(a, b, vector_scale)
    print(f"[step-parity] {label}: per-variable rel err {np.array2string(e, precision=2)} (bar {tol:.0e})",
          flush=True)
    assert np.all(e <= tol), (label, e)
    return e
