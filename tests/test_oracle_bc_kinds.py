"""Pins of the remaining boundary kinds of the paper's list (Sec. 4.3):
slip wall / symmetry plane, isothermal no-slip wall, zero-order
extrapolation, pressure outflow and pressure inflow.  Uniform states that
satisfy a condition are preserved exactly; slip walls conserve mass, energy
and the wall-parallel momentum; an isothermal wall holds a fluid at rest at
its temperature and heats a colder one; the ghost states carry the given
quantities; BRJ blocks with these faces equal the exact Jacobian blocks."""
import numpy as np
import pytest

import workloads as W
from oracle import solver as S
from oracle.dg import Disc
from oracle.physics import (Gas, BC_SLIP, BC_ISOTHERMAL, BC_EXTRAPOLATE, BC_PRESSURE_OUT, BC_PRESSURE_IN,
                            ghost_state, primitives, temperature)
from tests.test_oracle_solver import exact_jacobian


def _cons(gamma, rho, vel, p):
    vel = np.asarray(vel, dtype=float)
    return np.concatenate([[rho], rho * vel, [p / (gamma - 1.0) + 0.5 * rho * vel @ vel]])


def _disc(dim, cells, P, periodic, kinds, states, **gas):
    mesh = W.cartesian_mesh(cells, tuple(1.0 + 0.3 * i for i in range(dim)), periodic=periodic,
                            bc_ids=list(range(2 * dim)))
    return Disc(gas=Gas(**gas), dim=dim, P=P, nq=P + 2, elem_origin=mesh.elem_origin, elem_h=mesh.elem_h,
                face_nbr=mesh.face_nbr, bc_kind=np.array(kinds), bc_state=np.array(states))


def _uniform(d, U):
    u = np.zeros(d.shape)
    u[:, :, 0] = U * 2 ** (d.dim / 2)
    return u


@pytest.mark.parametrize("dim,mode", [(2, 0), (2, 1), (3, 0)])
def test_uniform_states_preserved(dim, mode):
    gas = dict(Ma=0.3, Re=50.0, flux_mode=mode)
    p0 = 1.0 / (1.4 * 0.09)
    vel = np.zeros(dim)
    vel[0] = 0.4
    U = _cons(1.4, 1.1, vel, p0)
    # x: pressure inflow (given state) / pressure outflow (given pressure);
    # the other axes: slip walls on one side, extrapolation on the other
    kinds = [BC_PRESSURE_IN, BC_PRESSURE_OUT] + [BC_SLIP, BC_EXTRAPOLATE] * (dim - 1)
    d = _disc(dim, (3,) * dim, 2, False, kinds, [U] * (2 * dim), **gas)
    scale = np.abs(d.L(W.random_state(d.n_elem, dim, 2, seed=1, mean=U))).max()
    assert np.abs(d.L(_uniform(d, U))).max() <= 1e-13 * scale
    # a fluid at rest at the wall temperature between isothermal walls
    R0 = _cons(1.4, 0.9, np.zeros(dim), p0)
    kinds = [BC_ISOTHERMAL] * (2 * dim)
    d = _disc(dim, (3,) * dim, 2, False, kinds, [R0] * (2 * dim), **gas)
    assert np.abs(d.L(_uniform(d, R0))).max() <= 1e-13 * scale


def test_slip_walls_conserve_mass_energy_and_parallel_momentum():
    per = [True, False]
    d = _disc(2, (3, 3), 2, per, [BC_SLIP] * 4, [np.zeros(4)] * 4, Ma=0.3, Re=30.0)
    u = W.random_state(d.n_elem, 2, 2, seed=3)
    L = d.L(u)
    for v in (0, 1, 3):
        assert abs(L[:, v, 0].sum()) <= 1e-13 * np.abs(L[:, v, 0]).sum(), v
    assert abs(L[:, 2, 0].sum()) > 1e-6 * np.abs(L[:, 2, 0]).sum()     # the walls push


def test_isothermal_wall_heats_a_colder_fluid():
    dim = 2
    p0 = 1.0 / (1.4 * 0.09)
    hot = _cons(1.4, 1.0, [0.0, 0.0], 1.5 * p0)          # the wall state: temperature 1.5 x the fluid's
    d = _disc(dim, (3, 3), 2, [True, False], [BC_ISOTHERMAL] * 4, [hot] * 4, Ma=0.3, Re=30.0)
    u = _uniform(d, _cons(1.4, 1.0, [0.0, 0.0], p0))
    L = d.L(u)
    assert abs(L[:, 0, 0].sum()) <= 1e-13 * np.abs(L[:, 3, 0]).sum()   # no mass through the wall
    assert L[:, 3, 0].sum() > 0.0                                        # energy flows in


def test_ghost_states_carry_the_given_quantities():
    gas = Gas(Ma=0.3)
    rng = np.random.default_rng(5)
    n = rng.normal(size=(30, 3))
    n /= np.linalg.norm(n, axis=-1, keepdims=True)
    U = np.stack([_cons(1.4, rng.uniform(0.8, 1.2), rng.uniform(-0.3, 0.3, 3), 8.0) for _ in range(30)])
    Ub = _cons(1.4, 1.3, [0.2, -0.1, 0.05], 9.0)
    r, v, E, p = primitives(gas, U)
    rb, vb, Eb, pb = primitives(gas, Ub)
    G = ghost_state(gas, BC_PRESSURE_OUT, U, n, Ub)
    rg, vg, Eg, pg = primitives(gas, G)
    assert np.allclose(rg, r) and np.allclose(vg, v) and np.allclose(pg, pb)
    G = ghost_state(gas, BC_PRESSURE_IN, U, n, Ub)
    rg, vg, Eg, pg = primitives(gas, G)
    assert np.allclose(rg, rb) and np.allclose(vg, vb) and np.allclose(pg, p)
    G = ghost_state(gas, BC_SLIP, U, n, Ub)
    rg, vg, Eg, pg = primitives(gas, G)
    vn = np.sum(v * n, -1)
    assert np.allclose(vg, v - 2 * vn[:, None] * n) and np.allclose(pg, p) and np.allclose(rg, r)
    G = ghost_state(gas, BC_ISOTHERMAL, U, n, Ub)
    rg, vg, Eg, pg = primitives(gas, G)
    Tw = temperature(gas, Ub[None])[0]
    assert np.allclose(vg, -v) and np.allclose(pg, p)
    assert np.allclose(0.5 * (temperature(gas, G) + temperature(gas, U)), Tw)
    assert np.array_equal(ghost_state(gas, BC_EXTRAPOLATE, U, n, Ub), U)


def test_brj_blocks_exact_with_the_other_kinds_euler():
    gas = dict(Ma=0.3, flux_mode=1)
    U = _cons(1.4, 1.0, [0.3, 0.1], 20.0 * 0.4)
    Ub = _cons(1.4, 1.1, [0.25, 0.0], 21.0 * 0.4)
    d = _disc(2, (3, 3), 1, [False, False], [BC_PRESSURE_IN, BC_PRESSURE_OUT, BC_SLIP, BC_ISOTHERMAL],
              [Ub] * 4, **gas)
    u = W.random_state(d.n_elem, 2, 1, seed=21, mean=U)
    J = exact_jacobian(d, u, u, 0.2)
    pc = S.BRJ(d, u, 0.2)
    nb = d.nv * d.ref.nm
    for e in range(d.n_elem):
        blk = J[e * nb:(e + 1) * nb, e * nb:(e + 1) * nb]
        assert np.abs(pc.D[e] - blk).max() <= 2e-6 * np.abs(blk).max()
