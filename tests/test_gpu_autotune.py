"""The residual autotuner (the fused kernel's workgroup size, or the volume,
face and lift kernels' sizes of the three-kernel path, chosen by timing):
choices are valid, results on boxes are bitwise unchanged, curved results
keep parity with the oracle, and a tuned batch gives the same residual as
before.  The fused kernel and the three-kernel path agree to rounding."""
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


def _fused_tiles(dim, P):
    """(workgroup size, elements per workgroup) tiles the autotuner tries for
    the fused kernel, in its order."""
    npts = 2 * dim * (P + 2) ** (dim - 1)
    unit = 32 if dim == 2 else 64
    need = ((npts + unit - 1) // unit) * unit
    tiles = []
    for epw in (1, 2, 4, 8):
        for nt in (64, 128, 192, 256):
            per = nt // epw
            if nt % epw or per < need or per % 32 or (dim == 3 and epw != 1):
                continue
            if nt == 192 and (dim == 2 or epw != 1):
                continue
            tiles.append((nt, epw))
    return tiles


@pytest.mark.parametrize("dim,cells,P", [(2, (5, 4), 3), (3, (3, 2, 2), 3)])
def test_autotune_boxes_bitwise(dim, cells, P):
    _case(f"autotune boxes dim={dim} P={P}")
    from paper_2002_04222_amd import Context
    cfg, mesh, disc = setup(dim, cells, P, Ma=0.3, Re=40.0)
    ctx = Context(mesh, cfg)
    u = _dev(W.random_state(mesh.n_elem, dim, P, seed=7))
    R0, R1 = ctx.empty(), ctx.empty()
    ctx.residual(u, R0)
    # fused kernel: one tile (workgroup size, elements per workgroup)
    chosen, times = ctx.autotune(u, reps=5)
    tiles = _fused_tiles(dim, P)
    flat = [t for row in times for t in row][:len(tiles)]
    assert (chosen[0], chosen[1]) in tiles and chosen[2] == 0
    assert all(t > 0.0 for t in flat)
    assert flat[tiles.index((chosen[0], chosen[1]))] == min(flat)
    ctx.residual(u, R1)
    assert np.array_equal(_host(R0), _host(R1))
    # the three-kernel path: one size per kernel
    ctx.set_residual_kernels(False)
    R2, R3 = ctx.empty(), ctx.empty()
    ctx.residual(u, R2)
    chosen, times = ctx.autotune(u, reps=5)
    assert all(c in (64, 128, 256) for c in chosen)
    assert all(t > 0.0 for row in times for t in row)
    for k in range(3):
        assert times[k][(64, 128, 256).index(chosen[k])] == min(times[k])
    ctx.residual(u, R3)
    assert np.array_equal(_host(R2), _host(R3))


FUSED_CASES = [(2, (4, 3), 2, "box"), (2, (3, 3), 5, "box"), (3, (3, 2, 2), 3, "box"), (3, (2, 2, 2), 4, "box"),
               (3, (2, 2, 2), 2, "curved"), (2, (3, 3), 4, "curved")]


@pytest.mark.parametrize("dim,cells,P,geo", FUSED_CASES)
def test_fused_and_three_kernel_paths_agree(dim, cells, P, geo):
    """Residual, stage residual and Frechet matvec by the fused kernel and by
    the three-kernel path agree to rounding per variable, and the fused
    residual's element sums of the mode-0 component of M R cancel on
    periodic meshes (each interior flux bitwise the same from both sides)."""
    _case(f"fused vs three kernels dim={dim} cells={cells} P={P} {geo}")
    from paper_2002_04222_amd import Context
    cfg, mesh, disc = setup(dim, cells, P, Ma=0.3, Re=40.0)
    if geo == "curved":
        lengths = tuple(1.0 + 0.3 * i for i in range(dim))
        mesh = W.curved_box_mesh(cells, lengths, geo_order=2, amp=0.15, seed=17)
    ctx = Context(mesh, cfg)
    u = _dev(W.random_state(mesh.n_elem, dim, P, seed=71))
    v = _dev(W.random_vector(mesh.n_elem, dim, P, seed=72))
    out = {}
    for fused in (True, False):
        ctx.set_residual_kernels(fused)
        R, N, Jv = ctx.empty(), ctx.empty(), ctx.empty()
        ctx.residual(u, R)
        ctx.stage_residual(u, 0.999 * u, 0.05, N)
        ctx.jfnk_matvec(u, N, 0.999 * u, 0.05, v, 0.0, Jv)
        out[fused] = (_host(R), _host(N), _host(Jv))
    assert rel_err_per_var(out[True][0], out[False][0]) <= 1e-13
    assert rel_err_per_var(out[True][1], out[False][1]) <= 1e-13
    assert np.linalg.norm(out[True][2] - out[False][2]) <= 1e-6 * np.linalg.norm(out[False][2])
    if geo == "box":
        Rg = out[True][0]
        detJ = np.prod(mesh.elem_h, axis=1)[:, None] / 2.0 ** dim
        tot = (Rg[:, :, 0] * detJ).sum(0)
        assert np.all(np.abs(tot) <= 1e-14 * np.abs(Rg[:, :, 0] * detJ).sum(0) + 1e-300)


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
    # fused kernel per order group: one tile each
    assert all(g[0] in (64, 128, 256) and g[1] in (1, 2, 4, 8) and g[2] == 0 for g in chosen)
    b.residual(u, R1)
    assert np.array_equal(_host(R0), _host(R1))
