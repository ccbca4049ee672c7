"""Pins of the Dirichlet boundary, the source term and the projection of
point values (the manufactured Poiseuille case of Sec. 6.1 and Appendix
B): a uniform state with matching Dirichlet data is preserved, BRJ blocks
with Dirichlet faces equal the exact Jacobian blocks, and the steady
solution of the manufactured problem converges at the designed order
P + 1 in the L2 norm, as the paper reports for the IP method."""
import numpy as np
import pytest

import workloads as W
from oracle import solver as S
from oracle.dg import Disc, make_disc
from oracle.physics import Gas, BC_DIRICHLET
from tests.test_oracle_solver import exact_jacobian


def _cons(gamma, rho, vel, p):
    vel = np.asarray(vel, dtype=float)
    return np.concatenate([[rho], rho * vel, [p / (gamma - 1.0) + 0.5 * rho * vel @ vel]])


def _dirichlet_disc(dim, cells, P, **gas):
    mesh = W.cartesian_mesh(cells, tuple(1.0 + 0.3 * i for i in range(dim)), periodic=False)
    return mesh, Disc(gas=Gas(**gas), dim=dim, P=P, nq=P + 2, elem_origin=mesh.elem_origin, elem_h=mesh.elem_h,
                      face_nbr=mesh.face_nbr, bc_kind=np.array([BC_DIRICHLET]),
                      bc_state=np.zeros((1, dim + 2)))


@pytest.mark.parametrize("dim,P", [(2, 2), (2, 4), (3, 2)])
def test_uniform_state_preserved_with_dirichlet_data(dim, P):
    gas = dict(Ma=0.3, Re=50.0)
    mesh, d = _dirichlet_disc(dim, (3,) * dim, P, **gas)
    U = _cons(1.4, 1.2, [0.4, -0.2, 0.1][:dim], 1.0 / (1.4 * 0.09))
    nqf = (P + 2) ** (dim - 1)
    d.bc_field = np.broadcast_to(U[None, None, :, None], (d.n_elem, 2 * dim, dim + 2, nqf)).copy()
    u = np.zeros(d.shape)
    u[:, :, 0] = U * 2 ** (dim / 2)
    scale = np.abs(d.L(W.random_state(d.n_elem, dim, P, seed=1, mean=U))).max()
    assert np.abs(d.L(u)).max() <= 1e-13 * scale


def test_brj_blocks_exact_with_dirichlet_faces():
    """The Dirichlet ghost state does not depend on the interior, so the BRJ
    diagonal blocks of elements on the boundary still equal the exact
    Jacobian blocks (Euler: no neglected gradient terms) to forward-
    difference accuracy."""
    gas = dict(Ma=0.3, flux_mode=1)
    mesh, d = _dirichlet_disc(2, (3, 3), 1, **gas)
    U = _cons(1.4, 1.0, [0.3, 0.1], 20.0 * 0.4)
    rng = np.random.default_rng(3)
    d.bc_field = U[None, None, :, None] * (1.0 + 0.01 * rng.uniform(-1, 1, size=(d.n_elem, 4, 4, 3)))
    u = W.random_state(d.n_elem, 2, 1, seed=21, mean=U)
    J = exact_jacobian(d, u, u, 0.2)
    pc = S.BRJ(d, u, 0.2)
    nb = d.nv * d.ref.nm
    for e in range(d.n_elem):
        blk = J[e * nb:(e + 1) * nb, e * nb:(e + 1) * nb]
        assert np.abs(pc.D[e] - blk).max() <= 2e-6 * np.abs(blk).max()


def mms_disc(P, n, viscous="ip"):
    cfg = W.mms_config(P, n)
    mesh = cfg.mesh()
    inp = W.mms_inputs(cfg, mesh)
    d = make_disc(cfg, mesh)
    d.viscous = viscous
    d.bc_kind, d.bc_state = cfg.boundary()
    d.bc_field = inp["bc_field"]
    d.source = d.project_values(inp["forcing"])
    return cfg, d, inp


def mms_steady(P, n, stepper_opts=None, viscous="ip"):
    """Backward-Euler pseudo-time steps from the initial state with the
    CFL number growing from 500 to 5000 over ten steps (as the paper's
    steady runs), until ||M^-1 L + s|| has dropped by 1e-9.  Returns the
    solution, the L2 error per variable at the Gauss points and the steps."""
    cfg, d, inp = mms_disc(P, n, viscous)
    u = d.project_values(inp["initial"])
    r0 = np.linalg.norm(d.residual(u))
    opts = stepper_opts or S.SolverOpts(scheme="beuler", pc_freeze=1, newton_rtol=1e-4)
    st = S.make_stepper(d, opts)
    dt0 = cfg.dt()
    for i in range(30):
        u, _ = st.step(u, dt0 * 10.0 ** min(1.0, i / 9.0))
        if np.linalg.norm(d.residual(u)) < 1e-9 * r0:
            break
    Q = np.einsum('qm,evm->evq', d.ref.B, u)
    err = np.sqrt(np.einsum('eq,evq->v', d.geo.wJ, (Q - inp["exact"]) ** 2))
    return u, err, i + 1


@pytest.mark.parametrize("viscous", ["ip", "ldg"])
@pytest.mark.parametrize("P,levels", [(2, (3, 4, 8)), (3, (4, 8))])
def test_manufactured_poiseuille_order_of_accuracy(P, levels, viscous):
    errs = [mms_steady(P, n, viscous=viscous)[1] for n in levels]
    for k in range(1, len(levels)):
        rate = np.log(errs[k - 1] / errs[k]) / np.log(levels[k] / levels[k - 1])
        print(P, levels[k], errs[k], rate)
        # momentum and energy at the designed order, density at least at order P
        assert np.all(rate[1:] > P + 1 - 0.35), rate
        assert rate[0] > P - 0.1, rate


def test_input_generator_matches_the_manufactured_solution():
    """The inputs the oracle and the library share: the exact state and the
    forcing from the problem module equal the manufactured field and the
    divergence of the oracle's fluxes at that field (complex step)."""
    from tests.oracle_util import flux_divergence
    from tests.test_oracle_physics import poiseuille
    gas = Gas(Re=100.0, Ma=0.1)
    field, _ = poiseuille(gas)
    exact, forcing = W.poiseuille_mms(gas.gamma, gas.Ma, gas.Re)
    x = np.random.default_rng(4).uniform(0, 1, size=(100, 2))
    U, _ = field(x)
    assert np.abs(exact(x) - U).max() <= 1e-13 * np.abs(U).max()
    f = forcing(x)
    div = flux_divergence(gas, field, x)
    assert np.abs(div - f).max() <= 1e-9 * np.abs(f).max()
    assert np.abs(div[:, 1] - f[:, 1]).max() <= 1e-9 * np.abs(f[:, 1]).max()
