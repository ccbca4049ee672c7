"""Block inversions are deterministic and exact: the inverse mass matrices
of a curved mesh and the BRJ block inverses come out bitwise identical from
two separate contexts (a missing barrier in the Gauss-Jordan pivot step once
made a few blocks per launch differ), and sampled inverse mass matrices
equal numpy's inverse of the oracle's mass matrices.  The residual, stage
residual and matvec repeat bitwise on the cylinder's element shape."""
import dataclasses
import gc
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads as W
from tests.gpu_util import setup


def _case(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_curved_mass_inverse_repeatable_and_exact():
    _case("mass inverse, annulus 16x32x4 P=4")
    from paper_2002_04222_amd import Context
    from oracle.dg import restricted_disc
    from oracle.physics import Gas
    cfg = dataclasses.replace(W.config(4), ncells=(16, 32, 4), lengths=(1.0, 2 * np.pi, np.pi / 2))
    mesh = cfg.mesh()
    k, st = cfg.boundary()
    nm = (cfg.P + 1) ** 3
    out = []
    for _ in range(2):
        ctx = Context(mesh, cfg, bc_kind=k, bc_state=st)
        mi = torch.empty((mesh.n_elem, nm, nm), dtype=torch.float64, device="cuda")
        ctx.mass_inverse(mi)
        out.append(_host(mi))
        ctx.close()
        del ctx, mi
        gc.collect()
    assert np.array_equal(out[0], out[1])
    gas = Gas(gamma=cfg.gamma, Pr=cfg.Pr, Re=cfg.Re, Ma=cfg.Ma)
    sample = [0, 15, 511, 1024, 2047]
    d, keep, idx = restricted_disc(gas, 3, cfg.P, cfg.nq, mesh.face_nbr, sample, geo_nodes=mesh.geo_nodes,
                                   geo_order=mesh.geo_order, bc_kind=k, bc_state=st)
    for i, e in enumerate(sample):
        ref = np.linalg.inv(d.M[idx[i]])
        assert np.abs(out[0][e] - ref).max() <= 1e-11 * np.abs(ref).max(), e


def test_brj_block_inverses_repeatable():
    _case("BRJ blocks twice, 6^3 P=3")
    from paper_2002_04222_amd import Context
    cfg, mesh, disc = setup(3, (6, 6, 6), 3, Ma=0.3, Re=40.0)
    u = torch.tensor(W.random_state(mesh.n_elem, 3, 3, seed=61), dtype=torch.float64, device="cuda")
    nb = 5 * 64
    out = []
    for _ in range(2):
        ctx = Context(mesh, cfg)
        ctx.precond_build(u, 0.1)
        dinv = torch.empty((mesh.n_elem, nb, nb), dtype=torch.float64, device="cuda")
        ctx.precond_diag_inverse(dinv)
        out.append(_host(dinv))
        ctx.close()
        del ctx, dinv
        gc.collect()
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("fused", [True, False])
def test_residuals_repeatable_on_the_annulus(fused):
    """R, N and the matvec evaluated twice on a 3D P=4 annulus (wall and far
    field, the cylinder's element shape) come out bitwise equal: every sum in
    the residual kernels has a fixed order (no atomics, no races between the
    phases of a workgroup)."""
    _case(f"residual repeatability, annulus 3D P=4, fused={fused}")
    from paper_2002_04222_amd import Context
    cfg = dataclasses.replace(W.config(4), ncells=(2, 8, 2), lengths=(1.0, 2 * np.pi, 1.0), r1=3.0, Re=200.0)
    mesh = cfg.mesh()
    k, st = cfg.boundary()
    ctx = Context(mesh, cfg, bc_kind=k, bc_state=st)
    ctx.set_residual_kernels(fused)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda").reshape(ctx.shape)
    u = dev(W.freestream_state(cfg, mesh.n_elem)) * (1.0 + 1e-3 * dev(W.random_vector(mesh.n_elem, 3, cfg.P, seed=3)))
    S = 0.999 * u
    v = dev(W.random_vector(mesh.n_elem, 3, cfg.P, seed=4))
    outs = []
    for _ in range(2):
        R, N, J = ctx.empty(), ctx.empty(), ctx.empty()
        ctx.residual(u, R)
        ctx.stage_residual(u, S, 0.05, N)
        ctx.jfnk_matvec(u, N, S, 0.05, v, 1e-7, J)
        outs.append((_host(R), _host(N), _host(J)))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    ctx.close()
