"""Pins of the oracle on curved (isoparametric) elements: a curved map that
is affine reproduces the box discretisation; the residual is covariant
under a rotation of the mesh and of the velocity; a uniform flow is
preserved; periodic meshes conserve every variable and walls conserve
mass and energy; the BRJ blocks equal exact Jacobian blocks (Euler)."""
import numpy as np
import pytest

import workloads as W
from oracle import solver as S
from oracle.dg import Disc
from oracle.physics import Gas, BC_FARFIELD, BC_WALL
from tests.test_oracle_solver import exact_jacobian


def _disc(mesh, P, **kw):
    gas = Gas(**{k: v for k, v in kw.items() if k in ("Ma", "Re", "flux_mode", "riemann")})
    extra = {k: v for k, v in kw.items() if k in ("bc_kind", "bc_state")}
    return Disc(gas=gas, dim=mesh.dim, P=P, nq=P + 2, elem_origin=mesh.elem_origin, elem_h=mesh.elem_h,
                face_nbr=mesh.face_nbr, geo_nodes=mesh.geo_nodes, geo_order=mesh.geo_order, **extra)


def _mean(dim):
    return W.DEFAULT_MEAN[dim]


@pytest.mark.parametrize("dim,cells,P", [(2, (3, 2), 2), (3, (2, 2, 2), 2)])
def test_affine_curved_map_reproduces_boxes(dim, cells, P):
    lengths = tuple(1.0 + 0.3 * i for i in range(dim))
    box = W.cartesian_mesh(cells, lengths)
    cur = W.curved_box_mesh(cells, lengths, geo_order=2, amp=0.0)
    db, dc = _disc(box, P, Ma=0.3, Re=40.0), _disc(cur, P, Ma=0.3, Re=40.0)
    assert dc.geo.curved and not db.geo.curved
    assert np.allclose(dc.M, db.M, rtol=1e-13, atol=1e-15)
    u = W.random_state(box.n_elem, dim, P, seed=5)
    Lb, Lc = db.L(u), dc.L(u)
    assert np.abs(Lc - Lb).max() <= 1e-12 * np.abs(Lb).max()
    pb, pc = S.BRJ(db, u, 0.1), S.BRJ(dc, u, 0.1)
    assert np.abs(pc.D - pb.D).max() <= 1e-8 * np.abs(pb.D).max()


def _rotation(dim, seed=3):
    if dim == 2:
        a = 0.7
        return np.array([[np.cos(a), -np.sin(a)], [np.sin(a), np.cos(a)]])
    q, r = np.linalg.qr(np.random.Generator(np.random.PCG64(seed)).normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    return q if np.linalg.det(q) > 0 else -q


@pytest.mark.parametrize("dim,cells,P,mode", [(2, (3, 3), 2, 0), (2, (3, 2), 3, 1), (3, (2, 2, 2), 2, 0)])
def test_rotation_covariance(dim, cells, P, mode):
    """Rotating the mesh nodes and the momentum by R rotates the momentum
    rows of L by R and leaves density and energy rows unchanged."""
    lengths = tuple(1.0 + 0.3 * i for i in range(dim))
    m = W.curved_box_mesh(cells, lengths, geo_order=2, amp=0.15, seed=11)
    R = _rotation(dim)
    mr = W.Mesh(dim=dim, ncells=m.ncells, elem_origin=None, elem_h=None, face_nbr=m.face_nbr,
                geo_nodes=m.geo_nodes @ R.T, geo_order=2)
    d, dr = _disc(m, P, Ma=0.3, Re=40.0, flux_mode=mode), _disc(mr, P, Ma=0.3, Re=40.0, flux_mode=mode)
    u = W.random_state(m.n_elem, dim, P, seed=9)
    ur = u.copy()
    ur[:, 1:1 + dim] = np.einsum('ij,ejm->eim', R, u[:, 1:1 + dim])
    L, Lr = d.L(u), dr.L(ur)
    expect = L.copy()
    expect[:, 1:1 + dim] = np.einsum('ij,ejm->eim', R, L[:, 1:1 + dim])
    assert np.abs(Lr - expect).max() <= 1e-12 * np.abs(L).max()


@pytest.mark.parametrize("dim,P", [(2, 3), (3, 2)])
def test_freestream_preserved_on_curved_periodic_mesh(dim, P):
    m = W.curved_box_mesh((3,) * dim, (1.0,) * dim, geo_order=2, amp=0.15, seed=2)
    d = _disc(m, P, Ma=0.3, Re=50.0)
    Uinf = np.array(_mean(dim))
    u = np.zeros(d.shape)
    u[:, :, 0] = Uinf * 2 ** (dim / 2)
    scale = np.abs(d.L(W.random_state(m.n_elem, dim, P, seed=1))).max()
    assert np.abs(d.L(u)).max() <= 1e-12 * scale


@pytest.mark.parametrize("nz", [0, 2])
def test_freestream_preserved_on_annulus_with_far_field(nz):
    m = W.annulus_mesh(3, 8, nz, r1=3.0, Lz=1.0, seed=4)
    dim = m.dim
    gas = Gas(Ma=0.2, Re=100.0)
    vel = np.zeros(dim)
    vel[0] = 1.0
    p = 1.0 / (gas.gamma * 0.04)
    Uinf = np.concatenate([[1.0], vel, [p / (gas.gamma - 1) + 0.5]])
    d = _disc(m, 2, Ma=0.2, Re=100.0, bc_kind=np.array([BC_FARFIELD, BC_FARFIELD]),
              bc_state=np.array([Uinf, Uinf]))
    u = np.zeros(d.shape)
    u[:, :, 0] = Uinf * 2 ** (dim / 2)
    noisy = u + 1e-2 * W.noise(u.shape, 3) * np.abs(Uinf + 0.1)[None, :, None]
    scale = np.abs(d.L(noisy)).max()
    assert np.abs(d.L(u)).max() <= 1e-12 * scale


def test_curved_periodic_mesh_conserves_every_variable():
    m = W.curved_box_mesh((3, 4), (1.0, 1.2), geo_order=3, amp=0.1, seed=5)
    d = _disc(m, 3, Ma=0.3, Re=30.0)
    L = d.L(W.random_state(m.n_elem, 2, 3, seed=6))
    for v in range(d.nv):
        assert abs(L[:, v, 0].sum()) <= 1e-13 * np.abs(L[:, v, 0]).sum()


@pytest.mark.parametrize("nz", [0, 2])
def test_annulus_walls_conserve_mass_and_energy(nz):
    m = W.annulus_mesh(2, 8, nz, r1=2.0, Lz=1.0, seed=6)
    dim = m.dim
    d = _disc(m, 2, Ma=0.3, Re=30.0, bc_kind=np.array([BC_WALL, BC_WALL]), bc_state=np.zeros((2, dim + 2)))
    mean = np.array(_mean(dim))
    L = d.L(W.random_state(m.n_elem, dim, 2, seed=7, mean=mean))
    for v in (0, dim + 1):
        assert abs(L[:, v, 0].sum()) <= 1e-13 * np.abs(L[:, v, 0]).sum(), v


def test_brj_blocks_exact_on_curved_mesh_euler():
    """P8a on curved elements: with Euler fluxes the BRJ diagonal blocks are
    the exact diagonal Jacobian blocks up to forward-difference error."""
    m = W.curved_box_mesh((3, 3), (1.0, 1.0), geo_order=2, amp=0.15, seed=8)
    d = _disc(m, 1, Ma=0.3, flux_mode=1)
    u = W.random_state(m.n_elem, 2, 1, seed=21)
    J = exact_jacobian(d, u, u, 0.2)
    pc = S.BRJ(d, u, 0.2)
    nb = d.nv * d.ref.nm
    for e in range(d.n_elem):
        blk = J[e * nb:(e + 1) * nb, e * nb:(e + 1) * nb]
        assert np.abs(pc.D[e] - blk).max() <= 1e-6 * np.abs(blk).max()


def test_curved_mass_matrix_projects_constants_exactly():
    m = W.annulus_mesh(2, 6, 0, r1=2.0, seed=9)
    d = _disc(m, 3, Ma=0.3)
    c = np.array([1.3, -0.2, 0.4, 7.0])
    u = d.project(lambda x: np.broadcast_to(c, x.shape[:-1] + (4,)))
    expect = np.zeros(d.shape)
    expect[:, :, 0] = c * 2.0
    assert np.abs(u - expect).max() <= 1e-13 * np.abs(c).max()
    # the summed element volumes converge to pi (r1^2 - r0^2) as the
    # quadratic arcs refine (interior node moves do not change the total)
    errs = []
    for nth in (6, 12):
        dd = _disc(W.annulus_mesh(2, nth, 0, r1=2.0, seed=9), 1, Ma=0.3)
        errs.append(abs(dd.vol.sum() - np.pi * 3.75) / (np.pi * 3.75))
    assert errs[0] < 1e-2 and errs[1] < errs[0] / 6.0, errs
