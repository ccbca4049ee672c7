"""Parity of the HIP path with the oracle on curved (isoparametric)
elements: periodic curved boxes and the cylinder annulus with wall and far
field.  Tolerances as for boxes: residual 1e-12 relative per variable,
matvec and BRJ 1e-6 (forward differences), SDIRK steps 1e-12 per variable; with far-field
faces the BRJ blocks 5e-6 and applies 1e-5 (see the boundary-condition
parity tests).  On curved
meshes the library stores (M_e - dt a A_e)^-1, which is compared with the
oracle's D_e^-1 M_e^-1."""
import dataclasses
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads as W
from oracle import solver as OS
from oracle.dg import Disc, restricted_disc
from oracle.physics import Gas, BC_FARFIELD, BC_WALL
from tests.gpu_util import assert_step, rel_err_per_var


def _case(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _gas(cfg):
    return Gas(gamma=cfg.gamma, Pr=cfg.Pr, Re=cfg.Re, Ma=cfg.Ma, visc_law=cfg.visc_law, T_ref_K=cfg.T_ref_K,
               flux_mode=cfg.flux_mode, riemann=cfg.riemann)


def _oracle(cfg, mesh, kinds=None, states=None):
    return Disc(gas=_gas(cfg), dim=mesh.dim, P=cfg.P, nq=cfg.nq, elem_origin=mesh.elem_origin,
                elem_h=mesh.elem_h, face_nbr=mesh.face_nbr, bc_kind=kinds, bc_state=states,
                geo_nodes=mesh.geo_nodes, geo_order=mesh.geo_order)


def _ctx(cfg, mesh, kinds=None, states=None):
    from paper_2002_04222_amd import Context
    return Context(mesh, cfg, bc_kind=kinds, bc_state=states)


def _box(dim, cells, P, **over):
    base = W.config(1 if dim == 2 else 2)
    lengths = tuple(1.0 + 0.3 * i for i in range(dim))
    cfg = dataclasses.replace(base, dim=dim, ncells=tuple(cells), lengths=lengths, P=P, nq=P + 2, Ma=0.3,
                              Re=40.0, **over)
    mesh = W.curved_box_mesh(cells, lengths, geo_order=2, amp=0.15, seed=17)
    return cfg, mesh


def _annulus(dim, nr, nth, nz, P, **over):
    base = W.config(4)
    cfg = dataclasses.replace(base, dim=dim, ncells=(nr, nth) + ((nz,) if dim == 3 else ()),
                              lengths=(1.0, 2 * np.pi) + ((1.0,) if dim == 3 else ()), P=P, nq=P + 2,
                              r1=3.0, Re=200.0, **over)
    mesh = cfg.mesh()
    kinds, states = cfg.boundary()
    return cfg, mesh, kinds, states


BOX_CASES = [(2, (3, 2), 2, 0, 0), (2, (2, 3), 4, 0, 1), (2, (3, 3), 3, 1, 0), (3, (2, 2, 3), 2, 0, 0),
             (3, (2, 2, 2), 3, 0, 0)]


@pytest.mark.parametrize("dim,cells,P,mode,riemann", BOX_CASES)
def test_curved_box_residual_parity(dim, cells, P, mode, riemann):
    _case(f"curved box residual dim={dim} cells={cells} P={P} mode={mode} riemann={riemann}")
    cfg, mesh = _box(dim, cells, P, flux_mode=mode, riemann=riemann)
    ctx = _ctx(cfg, mesh)
    u = W.random_state(mesh.n_elem, dim, P, seed=300 + P)
    R = ctx.empty()
    ctx.residual(_dev(u), R)
    assert rel_err_per_var(_host(R), _oracle(cfg, mesh).residual(u)) <= 1e-12


@pytest.mark.parametrize("dim,nr,nth,nz,P", [(2, 3, 8, 0, 3), (2, 2, 6, 0, 5), (3, 2, 6, 2, 2), (3, 2, 4, 2, 4)])
def test_annulus_residual_parity(dim, nr, nth, nz, P):
    _case(f"annulus residual dim={dim} nr={nr} nth={nth} nz={nz} P={P}")
    cfg, mesh, k, st = _annulus(dim, nr, nth, nz, P)
    ctx = _ctx(cfg, mesh, k, st)
    u = W.freestream_state(dataclasses.replace(cfg, noise_amp=3e-2), mesh.n_elem)
    R = ctx.empty()
    ctx.residual(_dev(u), R)
    assert rel_err_per_var(_host(R), _oracle(cfg, mesh, k, st).residual(u)) <= 1e-12


def test_annulus_matvec_and_precond_parity():
    _case("annulus matvec + precond 2D P=2")
    cfg, mesh, k, st = _annulus(2, 3, 8, 0, 2)
    ctx = _ctx(cfg, mesh, k, st)
    disc = _oracle(cfg, mesh, k, st)
    u = W.freestream_state(dataclasses.replace(cfg, noise_amp=3e-2), mesh.n_elem)
    S = 0.999 * u
    dt_a = 0.05
    No = disc.stage_residual(u, S, dt_a)
    v = W.random_vector(mesh.n_elem, 2, 2, seed=312)
    eps = OS.jfnk_eps(u)
    Jv = ctx.empty()
    ctx.jfnk_matvec(_dev(u), _dev(No), _dev(S), dt_a, _dev(v), eps, Jv)
    Jo = OS.jfnk_matvec(disc, u, No, S, dt_a, v, eps)
    assert np.linalg.norm(_host(Jv) - Jo) <= 1e-6 * np.linalg.norm(Jo)
    ctx.precond_build(_dev(u), dt_a)
    pc = OS.BRJ(disc, u, dt_a)
    nb = disc.nv * disc.ref.nm
    out = torch.empty((mesh.n_elem, nb, nb), dtype=torch.float64, device="cuda")
    ctx.precond_diag_inverse(out)
    Dg = _host(out)
    Do = np.einsum('eab,ebc->eac', pc.Dinv, np.stack([np.kron(np.eye(disc.nv), m) for m in pc.Minv]))
    # far-field faces in the inflow/outflow blend: see the tolerances of the
    # boundary-condition parity tests
    assert np.abs(Dg - Do).max() <= 5e-6 * np.abs(Do).max()
    q = W.random_vector(mesh.n_elem, 2, 2, seed=313)
    o = ctx.empty()
    ctx.precond_apply(_dev(q), o)
    ref = pc.apply(q)
    assert np.abs(_host(o) - ref).max() <= 1e-5 * np.abs(ref).max()


def test_curved_box_precond_parity_3d():
    _case("curved box precond 3D P=2")
    cfg, mesh = _box(3, (2, 2, 2), 2)
    ctx = _ctx(cfg, mesh)
    disc = _oracle(cfg, mesh)
    u = W.random_state(mesh.n_elem, 3, 2, seed=321)
    ctx.precond_build(_dev(u), 0.1)
    pc = OS.BRJ(disc, u, 0.1)
    q = W.random_vector(mesh.n_elem, 3, 2, seed=322)
    o = ctx.empty()
    ctx.precond_apply(_dev(q), o)
    ref = pc.apply(q)
    assert np.abs(_host(o) - ref).max() <= 1e-6 * np.abs(ref).max()


@pytest.mark.parametrize("scheme", ["sdirk2", "sdirk3"])
def test_annulus_sdirk_step_parity(scheme):
    _case(f"annulus sdirk step {scheme}")
    cfg, mesh, k, st = _annulus(2, 3, 8, 0, 2, scheme=scheme)
    ctx = _ctx(cfg, mesh, k, st)
    disc = _oracle(cfg, mesh, k, st)
    u0 = W.freestream_state(dataclasses.replace(cfg, noise_amp=1e-2), mesh.n_elem)
    du = _dev(u0)
    dt = 0.05
    stepper = OS.SDIRK(disc, OS.SolverOpts(scheme=scheme))
    uo = u0
    for k in range(2):
        s = ctx.sdirk_step(du, dt)
        uo, so = stepper.step(uo, dt)
        assert s["newton_its"] == [x.newton_its for x in so]
        assert s["gmres_its"] == [x.gmres_its for x in so]
        assert_step(_host(du), uo, f"annulus 3x8 P=2 {scheme} step {k}")


def test_cylinder_shaped_annulus_p4_blocks_apply_and_step():
    """The cylinder workload's shape at a size the oracle finishes: a 3D
    O-grid annulus r in [0.5, 10] of 2 x 4 x 2 hexes (span pi/4), P = 4
    (625 x 625 blocks), quadratic isoparametric maps, no-slip wall and far
    field, Re 3900, Ma 0.2.  The stored blocks (M_e - dt a A_e)^-1 against
    the oracle's D_e^-1 M_e^-1, one BRJ(7) apply, and one SDIRK2 step
    (identical Newton/GMRES counts, 1e-12 per variable)."""
    _case("cylinder-shaped annulus 2x4x2 P=4: blocks, apply, SDIRK2 step")
    cfg = dataclasses.replace(W.config(4), ncells=(2, 4, 2), lengths=(1.0, 2 * np.pi, np.pi / 4))
    mesh = cfg.mesh()
    k, st = cfg.boundary()
    disc = _oracle(cfg, mesh, k, st)
    u0 = W.freestream_state(dataclasses.replace(cfg, noise_amp=1e-2), mesh.n_elem)
    dt = 0.05
    dt_a = dt * (1.0 - np.sqrt(2.0) / 2.0)
    ctx = _ctx(cfg, mesh, k, st)
    ctx.precond_build(_dev(u0), dt_a)
    pc = OS.BRJ(disc, u0, dt_a)
    nb = disc.nv * disc.ref.nm
    out = torch.empty((mesh.n_elem, nb, nb), dtype=torch.float64, device="cuda")
    ctx.precond_diag_inverse(out)
    Do = np.einsum('eab,ebc->eac', pc.Dinv, np.stack([np.kron(np.eye(disc.nv), m) for m in pc.Minv]))
    blk = np.abs(_host(out) - Do).max() / np.abs(Do).max()
    q = W.random_vector(mesh.n_elem, 3, cfg.P, seed=331)
    o = ctx.empty()
    ctx.precond_apply(_dev(q), o)
    ref = pc.apply(q)
    app = np.abs(_host(o) - ref).max() / np.abs(ref).max()
    print(f"blocks rel err {blk:.2e}, apply rel err {app:.2e}", flush=True)
    # far-field faces: the tolerances of the boundary-condition parity tests
    assert blk <= 5e-6 and app <= 1e-5
    ctx2 = _ctx(cfg, mesh, k, st)
    du = _dev(u0)
    s = ctx2.sdirk_step(du, dt)
    uo, so = OS.SDIRK(disc, OS.SolverOpts(scheme="sdirk2")).step(u0, dt)
    print("newton", s["newton_its"], "gmres", s["gmres_its"], flush=True)
    assert s["newton_its"] == [x.newton_its for x in so]
    assert s["gmres_its"] == [x.gmres_its for x in so]
    assert_step(_host(du), uo, "cylinder-shaped annulus 2x4x2 P=4 SDIRK2")


def test_cylinder_annulus_full_size_sampled_residual():
    """The cylinder workload at full size (32 x 64 x 8 hexes, P=4, 10.24M
    unknowns): the device residual of the impulsive-start state against the
    oracle on sampled elements (wall, far field, interior, seam)."""
    cfg = W.config(4)
    _case(f"full-size sampled residual {cfg.name}")
    mesh = cfg.mesh()
    k, st = cfg.boundary()
    ctx = _ctx(cfg, mesh, k, st)
    u = W.freestream_state(cfg, mesh.n_elem)
    R = ctx.empty()
    ctx.residual(_dev(u), R)
    Rg = _host(R)
    nr, nth, nz = cfg.ncells
    rng = np.random.Generator(np.random.PCG64(41))
    picks = [0, nr - 1, nr * (nth - 1), nr * nth * nz - 1] + list(rng.integers(0, mesh.n_elem, size=12))
    sample = sorted(set(int(x) for x in picks))
    # the oracle on the sample elements and their neighbours only
    d, keep, idx = restricted_disc(_gas(cfg), mesh.dim, cfg.P, cfg.nq, mesh.face_nbr, sample,
                                   geo_nodes=mesh.geo_nodes, geo_order=mesh.geo_order, bc_kind=k, bc_state=st)
    Ro = d.residual(u[keep])[idx]
    assert np.all(np.isfinite(Rg))
    # As on the box workload, the single terms summed into R are of size
    # U (c+|u|)(P+1)^2 2/h (h the smallest element width, next to the
    # cylinder) and cancel down to |R|; FP64 rounding of such terms bounds
    # the agreement: 1e-12 of |R_v| plus 2e-16 of the largest term.
    h = cfg.r0 * ((cfg.r1 / cfg.r0) ** (1.0 / nr) - 1.0)
    term = np.abs(u).max() * (1.0 / cfg.Ma + 1.0) * (cfg.P + 1) ** 2 * 2.0 / h
    for v in range(cfg.dim + 2):
        err = np.abs(Rg[sample, v] - Ro[:, v]).max()
        rmax = np.abs(Ro[:, v]).max()
        print(f"var {v}: max err {err:.3e}  max |R| {rmax:.3e}  rel {err / rmax:.3e}  term {term:.3e}")
        assert err <= 1e-12 * rmax + 2e-16 * term, (v, err, rmax, term)


def test_curved_create_rejects_inverted_map():
    _case("curved create: inverted element")
    from paper_2002_04222_amd import DgjError
    cfg, mesh = _box(2, (3, 2), 2)
    bad = mesh.geo_nodes.copy()
    bad[0] = bad[0].reshape(3, 3, 2)[:, ::-1].reshape(9, 2)   # mirrored in xi_0: negative Jacobian
    m2 = dataclasses.replace(mesh, geo_nodes=bad)
    with pytest.raises(DgjError) as ei:
        _ctx(cfg, m2)
    assert ei.value.code == -1
    with pytest.raises(DgjError):
        c = _ctx(cfg, mesh)
        c.project_tgv(None, 0.0, c.empty())
