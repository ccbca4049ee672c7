"""Pins of the oracle's boundary conditions (far field by Riemann
invariants, adiabatic no-slip wall): characteristic relations of the ghost
state, freestream preservation, conservation of mass and energy with walls,
the exact wall flux of a fluid at rest, and the BRJ blocks against exact
Jacobian blocks with boundaries."""
import numpy as np
import pytest

import workloads as W
from oracle import solver as S
from oracle.dg import Disc
from oracle.physics import (Gas, BC_FARFIELD, BC_WALL, farfield_ghost, wall_ghost, primitives,
                            boundary_flux_own)
from tests.test_oracle_solver import exact_jacobian


def _cons(gas, rho, vel, p):
    vel = np.asarray(vel, dtype=float)
    return np.concatenate([[rho], rho * vel, [p / (gas.gamma - 1) + 0.5 * rho * vel @ vel]])


def _inv(gas, U, n):
    r, v, E, p = primitives(gas, U)
    c = np.sqrt(gas.gamma * p / r)
    un = v @ n
    return un + 2 * c / (gas.gamma - 1), un - 2 * c / (gas.gamma - 1), p / r ** gas.gamma, v - un * n


@pytest.mark.parametrize("un_sign", [1.0, -1.0])
def test_farfield_ghost_characteristics(un_sign):
    """Away from u_nb = 0 (|u_nb| >> 0.02 c_b) the ghost has R+ of the
    interior, R- of the freestream, and the upwind side's entropy and
    tangential velocity."""
    gas = Gas(Ma=0.3)
    n = np.array([0.6, 0.8])
    c = np.sqrt(1.4 * 8.5 / 1.1)
    t = np.array([-0.8, 0.6])
    Ui = _cons(gas, 1.1, un_sign * 0.6 * c * n + 0.25 * t, 8.5)
    Uo = _cons(gas, 1.0, un_sign * 0.6 * c * n - 0.3 * t, 7.9)
    Ub = farfield_ghost(gas, Ui, n, Uo)
    Rpi, _, si, vti = _inv(gas, Ui, n)
    _, Rmo, so, vto = _inv(gas, Uo, n)
    Rpb, Rmb, sb, vtb = _inv(gas, Ub, n)
    assert np.isclose(Rpb, Rpi, rtol=1e-13) and np.isclose(Rmb, Rmo, rtol=1e-13)
    out = (Rpb + Rmb) > 0
    assert out == (un_sign > 0)
    assert np.isclose(sb, si if out else so, rtol=1e-12)
    assert np.allclose(vtb, vti if out else vto, atol=1e-13)
    # a ghost computed from the freestream itself is the freestream
    assert np.allclose(farfield_ghost(gas, Uo, n, Uo), Uo, rtol=1e-13)


def test_farfield_blend_is_continuous_across_un_zero():
    """Where u_nb changes sign the entropy and tangential velocity are
    blended: at u_nb = 0 they are the two sides' means, and the ghost state
    changes continuously (no jump between the inflow and outflow choices)."""
    gas = Gas(Ma=0.3)
    n = np.array([1.0, 0.0])
    Uo = _cons(gas, 1.0, [0.0, 0.4], 8.0)
    Ri_of = lambda un: _cons(gas, 1.2, [un, -0.2], 9.0)
    # interior normal velocity giving u_nb = 0 exactly: R+ = -R-
    ro, vo, Eo, po = primitives(gas, Uo)
    co = np.sqrt(1.4 * po / ro)
    ci = np.sqrt(1.4 * 9.0 / 1.2)
    un0 = -(0.0 - 2 * co / 0.4) - 2 * ci / 0.4
    Ub = farfield_ghost(gas, Ri_of(un0), n, Uo)
    _, _, sb, vtb = _inv(gas, Ub, n)
    _, _, si, vti = _inv(gas, Ri_of(un0), n)
    _, _, so, vto = _inv(gas, Uo, n)
    assert np.isclose(sb, 0.5 * (si + so), rtol=1e-12)
    assert np.allclose(vtb, 0.5 * (vti + vto), atol=1e-12)
    h = 1e-7
    jump = np.abs(farfield_ghost(gas, Ri_of(un0 + h), n, Uo) - farfield_ghost(gas, Ri_of(un0 - h), n, Uo)).max()
    assert jump < 1e-3


def test_farfield_supersonic():
    gas = Gas(Ma=0.3)
    n = np.array([1.0, 0.0])
    Uo = _cons(gas, 1.0, [0.0, 0.0], 7.9)
    c = np.sqrt(1.4 * 7.9)
    Ui = _cons(gas, 1.0, [1.5 * c, 0.1], 7.9)
    assert np.allclose(farfield_ghost(gas, Ui, n, Uo), Ui)          # supersonic outflow
    Uin = _cons(gas, 1.0, [-1.5 * c, 0.1], 7.9)
    assert np.allclose(farfield_ghost(gas, Ui * 0.99, n, Uin), Uin)   # supersonic inflow


def test_wall_flux_of_fluid_at_rest():
    gas = Gas(Ma=0.3, Re=50.0)
    for d in (2, 3):
        n = np.zeros(d)
        n[d - 1] = -1.0
        U = _cons(gas, 1.2, np.zeros(d), 9.0)
        go = np.zeros((d, d + 2))
        H, Sv = boundary_flux_own(gas, BC_WALL, U[None], go[None], n[None], np.array([3.0]))
        expect = np.zeros(d + 2)
        expect[1:1 + d] = 9.0 * n
        assert np.allclose(H[0], expect, atol=1e-13)
        assert np.allclose(wall_ghost(U)[1:-1], -U[1:-1])


def _bc_disc(dim, cells, P, periodic, kinds, state, **gas):
    mesh = W.cartesian_mesh(cells, tuple(1.0 + 0.3 * i for i in range(dim)), periodic=periodic,
                            bc_ids=list(range(2 * dim)))
    return Disc(gas=Gas(**gas), dim=dim, P=P, nq=P + 2, elem_origin=mesh.elem_origin, elem_h=mesh.elem_h,
                face_nbr=mesh.face_nbr, bc_kind=np.array(kinds), bc_state=np.array(state))


@pytest.mark.parametrize("dim,P,speed", [(2, 2, 0.3), (2, 3, 3.0), (3, 2, 0.3)])
def test_freestream_preserved_with_farfield(dim, P, speed):
    gas = Gas(Ma=0.3, Re=50.0)
    vel = np.zeros(dim)
    vel[0] = speed
    vel[-1] = 0.5 * speed
    Uinf = _cons(gas, 1.0, vel, 1.0 / (1.4 * 0.09))
    d = _bc_disc(dim, (3,) * dim, P, False, [BC_FARFIELD] * (2 * dim), [Uinf] * (2 * dim), Ma=0.3, Re=50.0)
    u = np.zeros(d.shape)
    u[:, :, 0] = Uinf * 2 ** (dim / 2)
    scale = np.abs(d.L(W.random_state(d.n_elem, dim, P, seed=1, mean=Uinf))).max()
    assert np.abs(d.L(u)).max() <= 1e-13 * scale


@pytest.mark.parametrize("dim", [2, 3])
def test_walls_conserve_mass_and_energy(dim):
    kinds = [BC_WALL] * (2 * dim)
    per = [True] * dim
    per[-1] = False
    d = _bc_disc(dim, (3,) * dim, 2, per, kinds, [np.zeros(dim + 2)] * (2 * dim), Ma=0.3, Re=30.0)
    u = W.random_state(d.n_elem, dim, 2, seed=3)
    L = d.L(u)
    for v in (0, dim + 1):
        tot = L[:, v, 0].sum()
        assert abs(tot) <= 1e-13 * np.abs(L[:, v, 0]).sum(), v
    # wall-normal momentum is not conserved: the walls push
    assert abs(L[:, dim, 0].sum()) > 1e-6 * np.abs(L[:, dim, 0]).sum()


def test_brj_blocks_exact_with_boundaries_euler():
    """P8a with far-field and wall faces: the boundary conditions are inside
    the differenced flux (Eq. 31), so the BRJ diagonal blocks equal the exact
    Jacobian blocks to forward-difference accuracy.  The far-field blend
    varies on the scale 0.02 c_b ~ 0.07 in u_n here, so the forward
    difference's truncation (~ chi / (2 delta^2) relative) is ~5e-6, not the
    ~3e-7 of the other faces."""
    gas = dict(Ma=0.3, flux_mode=1)
    Uinf = _cons(Gas(**gas), 1.0, [0.3, 0.1], 20.0 * 0.4)
    d = _bc_disc(2, (3, 3), 1, [False, False], [BC_FARFIELD, BC_FARFIELD, BC_WALL, BC_WALL],
                 [Uinf] * 4, **gas)
    u = W.random_state(d.n_elem, 2, 1, seed=21, mean=Uinf)
    J = exact_jacobian(d, u, u, 0.2)
    pc = S.BRJ(d, u, 0.2)
    nb = d.nv * d.ref.nm
    for e in range(d.n_elem):
        blk = J[e * nb:(e + 1) * nb, e * nb:(e + 1) * nb]
        assert np.abs(pc.D[e] - blk).max() <= 2e-5 * np.abs(blk).max()
