"""The residual autotuner (workgroup sizes of the volume, face and lift
kernels chosen by timing): choices are valid, results on boxes are bitwise
unchanged, curved results keep parity with the oracle, and a tuned batch
gives the same residual as before."""
import dataclasses
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads as W
from tests.gpu_util import rel_err_per_var, setup


def _case(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("dim,cells,P", [(2, (5, 4), 3), (3, (3, 2, 2), 3)])
def test_autotune_boxes_bitwise(dim, cells, P):
    _case(f"autotune boxes dim={dim} P={P}")
    from paper_2002_04222_amd import Context
    cfg, mesh, disc = setup(dim, cells, P, Ma=0.3, Re=40.0)
    ctx = Context(mesh, cfg)
    u = _dev(W.random_state(mesh.n_elem, dim, P, seed=7))
    R0, R1 = ctx.empty(), ctx.empty()
    ctx.residual(u, R0)
    chosen, times = ctx.autotune(u, reps=5)
    assert all(c in (64, 128, 256) for c in chosen)
    assert all(t > 0.0 for row in times for t in row)
    for k in range(3):
        assert times[k][(64, 128, 256).index(chosen[k])] == min(times[k])
    ctx.residual(u, R1)
    assert np.array_equal(_host(R0), _host(R1))


def test_autotune_curved_keeps_parity():
    _case("autotune curved annulus")
    from paper_2002_04222_amd import Context
    from oracle.dg import Disc
    from oracle.physics import Gas
    cfg = dataclasses.replace(W.config(4), dim=3, ncells=(2, 6, 2), lengths=(1.0, 2 * np.pi, 1.0), P=3, nq=5,
                              r1=3.0, Re=200.0)
    mesh = cfg.mesh()
    k, st = cfg.boundary()
    ctx = Context(mesh, cfg, bc_kind=k, bc_state=st)
    u = W.freestream_state(dataclasses.replace(cfg, noise_amp=3e-2), mesh.n_elem)
    du = _dev(u)
    ctx.autotune(du, reps=5)
    R = ctx.empty()
    ctx.residual(du, R)
    gas = Gas(gamma=cfg.gamma, Pr=cfg.Pr, Re=cfg.Re, Ma=cfg.Ma, flux_mode=cfg.flux_mode, riemann=cfg.riemann)
    d = Disc(gas=gas, dim=3, P=cfg.P, nq=cfg.nq, elem_origin=None, elem_h=None, face_nbr=mesh.face_nbr,
             bc_kind=k, bc_state=st, geo_nodes=mesh.geo_nodes, geo_order=mesh.geo_order)
    assert rel_err_per_var(_host(R), d.residual(u)) <= 1e-12


def test_batch_autotune_same_residual():
    _case("batch autotune")
    from paper_2002_04222_amd import Batch
    cfgs = W.batch_configs(n=6, seed=9, nmin=3, nmax=6)
    b = Batch(cfgs)
    u = b.empty()
    noise = torch.tensor(W.noise((b.n_total,), 3), dtype=torch.float64, device="cuda")
    b.project_tgv(noise, 1e-3, u)
    R0, R1 = b.empty(), b.empty()
    b.residual(u, R0)
    chosen = b.autotune(u, reps=3)
    assert 1 <= len(chosen) <= len(cfgs)
    assert all(c in (64, 128, 256) for g in chosen for c in g)
    b.residual(u, R1)
    assert np.array_equal(_host(R0), _host(R1))
