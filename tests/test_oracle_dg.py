"""Pins of the oracle's DG residual (Eq. 9-13) against mathematics:
orthonormality, freestream preservation, conservation, mirror symmetry,
symmetry and definiteness of the interior-penalty operator, and the order
of the truncation error on exact solutions."""
import numpy as np
import pytest

import workloads as W
from oracle.basis import phi1d, gauss, ref_element
from oracle.physics import Gas
from tests.oracle_util import tiny_disc, conserved_with_gradient, flux_divergence, l2_coeff_norm


def test_basis_orthonormal_and_mass_matrix():
    for dim, P in ((2, 2), (3, 3), (2, 5)):
        d = tiny_disc(dim=dim, cells=(2,) * dim, P=P)
        M = d.M / d.detJ[:, None, None]
        assert np.allclose(M, np.eye(d.ref.nm)[None], atol=1e-13)
    # derivative of the Legendre functions against finite differences
    x = np.linspace(-0.9, 0.9, 7)
    V, dV = phi1d(4, x)
    Vp, _ = phi1d(4, x + 1e-6)
    Vm, _ = phi1d(4, x - 1e-6)
    assert np.allclose((Vp - Vm) / 2e-6, dV, atol=1e-7)
    # phi_i(1) = sqrt((2i+1)/2) and phi_i(-1) = (-1)^i sqrt((2i+1)/2)
    V1, _ = phi1d(4, np.array([-1.0, 1.0]))
    c = np.sqrt((2 * np.arange(5) + 1) / 2.0)
    assert np.allclose(V1[:, 1], c) and np.allclose(V1[:, 0], c * (-1.0) ** np.arange(5))
    xg, wg = gauss(5)
    assert abs(wg.sum() - 2.0) < 1e-14 and abs(np.sum(wg * xg ** 8) - 2.0 / 9.0) < 1e-14


@pytest.mark.parametrize("dim,cells,P", [(2, (3, 2), 2), (3, (2, 2, 3), 2), (2, (2, 2), 4)])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_freestream_and_conservation(dim, cells, P, mode):
    d = tiny_disc(dim=dim, cells=cells, P=P, Ma=0.3, Re=50.0, flux_mode=mode)
    ne = d.n_elem
    # P1: a constant state is preserved
    uc = W.random_state(ne, dim, P, seed=3, amp=0.0)
    vol = np.abs(d.L(W.random_state(ne, dim, P, seed=3))).max()
    assert np.abs(d.L(uc)).max() <= 1e-13 * vol
    # P2: element sums of the mode-0 component cancel on a periodic mesh
    u = W.random_state(ne, dim, P, seed=4)
    L = d.L(u)
    tot = L[:, :, 0].sum(axis=0)
    assert np.all(np.abs(tot) <= 1e-13 * np.abs(L[:, :, 0]).sum(axis=0) + 1e-300)


def _mirror(u, dim, P, cells, a, b):
    """Swap axes a and b of a state on a cube grid (elements, modes and
    the two momentum components)."""
    n = P + 1
    E, nv, nm = u.shape
    ue = u.reshape(cells[::-1] + (nv,) + (n,) * dim)        # [k,j,i, v, mk,mj,mi]
    ax_e = [dim - 1 - a, dim - 1 - b]
    ax_m = [dim + 1 + (dim - 1 - a), dim + 1 + (dim - 1 - b)]
    perm = list(range(ue.ndim))
    perm[ax_e[0]], perm[ax_e[1]] = perm[ax_e[1]], perm[ax_e[0]]
    perm[ax_m[0]], perm[ax_m[1]] = perm[ax_m[1]], perm[ax_m[0]]
    ue = ue.transpose(perm).reshape(E, nv, nm).copy()
    ue[:, [1 + a, 1 + b]] = ue[:, [1 + b, 1 + a]]
    return ue


@pytest.mark.parametrize("dim,P", [(2, 2), (3, 1)])
def test_axis_swap_symmetry(dim, P):
    cells = (3,) * dim
    d = tiny_disc(dim=dim, cells=cells, P=P, lengths=(1.3,) * dim, Ma=0.3, Re=20.0)
    u = W.random_state(d.n_elem, dim, P, seed=7)
    R = d.residual(u)
    for a, b in ((0, 1), (0, dim - 1)):
        if a == b:
            continue
        Rs = d.residual(_mirror(u, dim, P, cells, a, b))
        assert np.allclose(Rs, _mirror(R, dim, P, cells, a, b), rtol=1e-12, atol=1e-12 * np.abs(R).max())


@pytest.mark.parametrize("dim,cells,P", [(2, (3, 3), 2), (2, (2, 3), 3), (3, (2, 2, 2), 1)])
def test_interior_penalty_symmetric_negative(dim, cells, P):
    """P9: with G = nu grad U and F = 0 the operator -dL/du of Eq. 12 is
    symmetric and positive semi-definite (beta_s = 1, dissipative
    penalty)."""
    d = tiny_disc(dim=dim, cells=cells, P=P, Re=1.0, flux_mode=2)
    n = int(np.prod(d.shape))
    K = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        K[:, i] = -d.L(e.reshape(d.shape)).ravel()
    s = np.abs(K).max()
    assert np.abs(K - K.T).max() <= 1e-12 * s
    ev = np.linalg.eigvalsh(0.5 * (K + K.T))
    assert ev.min() >= -1e-11 * s
    # the kernel is exactly the piecewise... constants per variable
    assert np.sum(np.abs(ev) <= 1e-10 * s) == d.nv


def _vortex(gas, x0=5.0, y0=5.0, u0=1.0, v0=0.5, phi=5.0):
    """Isentropic vortex of Sec. 6.1 at t = 0, with the u-perturbation
    taken as -phi (y - y0) e^(1-r^2) / (2 pi): with the printed '+' on both
    perturbations the field is not a solution of the Euler equations."""
    g = gas.gamma

    def field(x):
        X, Y = x[..., 0] - x0, x[..., 1] - y0
        r2 = X * X + Y * Y
        ex = np.exp(1 - r2)
        A = phi ** 2 * (g - 1) / (16 * g * np.pi ** 2)
        base = 1 - A * ex ** 2
        rho = base ** (1 / (g - 1))
        drho_dr2 = (1 / (g - 1)) * base ** (1 / (g - 1) - 1) * (2 * A * ex ** 2)
        grho = np.stack([drho_dr2 * 2 * X, drho_dr2 * 2 * Y], -1)
        c = phi / (2 * np.pi)
        u = u0 - c * Y * ex
        v = v0 + c * X * ex
        gvel = np.zeros(X.shape + (2, 2), dtype=x.dtype)
        gvel[..., 0, 0] = -c * Y * ex * (-2 * X)
        gvel[..., 1, 0] = -c * ex - c * Y * ex * (-2 * Y)
        gvel[..., 0, 1] = c * ex + c * X * ex * (-2 * X)
        gvel[..., 1, 1] = c * X * ex * (-2 * Y)
        p = rho ** g
        gp = (g * rho ** (g - 1))[..., None] * grho
        return conserved_with_gradient(g, rho, grho, np.stack([u, v], -1), gvel, p, gp)
    return field


def _truncation_errors(gas, dim, P, Ns, field, lengths, origin=None):
    errs = []
    for N in Ns:
        mesh = W.cartesian_mesh((N,) * dim, lengths)
        from oracle.dg import Disc
        d = Disc(gas=gas, dim=dim, P=P, nq=P + 2, elem_origin=mesh.elem_origin, elem_h=mesh.elem_h,
                 face_nbr=mesh.face_nbr)
        u = d.project(lambda x: field(x)[0].real)
        rate = d.project(lambda x: -flux_divergence(gas, field, x))
        errs.append(l2_coeff_norm(d, d.residual(u) - rate))
    return np.array(errs)


@pytest.mark.parametrize("P,Ns", [(2, (10, 20)), (3, (20, 40))])
def test_isentropic_vortex_truncation_order(P, Ns):
    """P5: on the Euler equations the DG residual of the projected exact
    vortex converges to the projected exact rate at order >= P (meshes
    fine enough to be in the asymptotic range)."""
    gas = Gas(flux_mode=1, Ma=1.0 / np.sqrt(1.4))
    field = _vortex(gas)
    e = _truncation_errors(gas, 2, P, Ns, field, (10.0, 10.0))
    order = np.log2(e[0] / e[1])
    assert order >= P - 0.2, (e, order)


def _smooth_periodic(gas, dim):
    """A smooth periodic compressible field on [0, 2 pi]^d."""
    pinf = 1.0 / (gas.gamma * gas.Ma ** 2)

    def field(x):
        s = [x[..., j] for j in range(dim)]
        ph = sum((j + 1) * s[j] for j in range(dim))
        rho = 1.0 + 0.2 * np.sin(ph)
        grho = np.stack([0.2 * (j + 1) * np.cos(ph) for j in range(dim)], -1)
        vel = np.stack([0.3 * np.cos(s[(c + 1) % dim]) + 0.1 * c for c in range(dim)], -1)
        gvel = np.zeros(s[0].shape + (dim, dim), dtype=x.dtype)
        for c in range(dim):
            gvel[..., (c + 1) % dim, c] = -0.3 * np.sin(s[(c + 1) % dim])
        p = pinf * (1.0 + 0.1 * np.cos(s[0] - s[-1] + 0.3))
        gp = np.zeros(s[0].shape + (dim,), dtype=x.dtype)
        gp[..., 0] += -pinf * 0.1 * np.sin(s[0] - s[-1] + 0.3)
        gp[..., dim - 1] += pinf * 0.1 * np.sin(s[0] - s[-1] + 0.3)
        return conserved_with_gradient(gas.gamma, rho, grho, vel, gvel, p, gp)
    return field


@pytest.mark.parametrize("P", [2, 3])
def test_navier_stokes_truncation_converges(P):
    """The full NS residual (Roe + interior penalty) of a projected smooth
    periodic field converges to the projected exact rate; the interior
    penalty truncation error in L2 is O(h^(P-1)), so order >= P - 1."""
    gas = Gas(Re=5.0, Ma=0.5)
    field = _smooth_periodic(gas, 2)
    e = _truncation_errors(gas, 2, P, (6, 12, 24), field, (2 * np.pi, 2 * np.pi))
    orders = np.log2(e[:-1] / e[1:])
    assert orders[-1] >= P - 1 - 0.3, (e, orders)
    assert e[-1] < 0.5 * e[0]


def test_navier_stokes_truncation_3d():
    gas = Gas(Re=5.0, Ma=0.5)
    field = _smooth_periodic(gas, 3)
    e = _truncation_errors(gas, 3, 3, (4, 8), field, (2 * np.pi,) * 3)
    # pre-asymptotic on these meshes (P - 1 = 2 is approached from below)
    assert np.log2(e[0] / e[1]) >= 1.2, e


@pytest.mark.parametrize("dim,cells,P", [(2, (3, 3), 2), (2, (2, 3), 3), (3, (2, 2, 2), 1)])
def test_ldg_diffusion_symmetric_negative(dim, cells, P):
    """The LDG option (auxiliary gradient with lifted jumps, u_hat and q_hat
    from opposite sides, jump penalty): with G = nu grad U the operator
    -dL/du is symmetric and positive semi-definite with the constants as
    its kernel, as the LDG primal form is; it differs from the IP operator."""
    d = tiny_disc(dim=dim, cells=cells, P=P, Re=1.0, flux_mode=2)
    n = int(np.prod(d.shape))
    K = np.zeros((n, n))
    Kip = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        Kip[:, i] = -d.L(e.reshape(d.shape)).ravel()
    d.viscous = "ldg"
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        K[:, i] = -d.L(e.reshape(d.shape)).ravel()
    s = np.abs(K).max()
    assert np.abs(K - K.T).max() <= 1e-12 * s
    ev = np.linalg.eigvalsh(0.5 * (K + K.T))
    assert ev.min() >= -1e-11 * s
    assert np.sum(np.abs(ev) <= 1e-10 * s) == d.nv
    assert np.abs(K - Kip).max() > 1e-3 * s


@pytest.mark.parametrize("dim,P", [(2, 3), (3, 2)])
def test_ldg_navier_stokes_conservation_and_freestream(dim, P):
    d = tiny_disc(dim=dim, cells=(3,) * dim, P=P, Ma=0.3, Re=30.0)
    d.viscous = "ldg"
    u = W.random_state(d.n_elem, dim, P, seed=9)
    L = d.L(u)
    for v in range(d.nv):
        assert abs(L[:, v, 0].sum()) <= 1e-13 * np.abs(L[:, v, 0]).sum()
    U = W.DEFAULT_MEAN[dim]
    c = np.zeros(d.shape)
    c[:, :, 0] = np.asarray(U) * 2 ** (dim / 2)
    assert np.abs(d.L(c)).max() <= 1e-13 * np.abs(L).max()
