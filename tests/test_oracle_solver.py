"""Pins of the oracle's implicit solver (Sec. 3.2, Sec. 4.2.2, Appendix A):
order conditions of the tableaus, the printed SDIRK3 lambda and BRJ memory
table, the Jacobian-free matvec and the BRJ blocks against exact Jacobians
(complex step) on tiny meshes, BRJ and GMRES against dense linear algebra,
Newton against dense Newton, and the temporal order of the SDIRK steps."""
import math
import os

import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import solver as S
from oracle.butcher import tableau, sdirk3_lambda
from tests.oracle_util import tiny_disc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(line.split())
    return rows


# ---------------------------------------------------------------- tableaus
@pytest.mark.parametrize("name,order", [("sdirk2", 2), ("sdirk3", 3), ("erk2", 2)])
def test_butcher_order_conditions(name, order):
    A, b, c = tableau(name)
    assert abs(b.sum() - 1) < 1e-15
    assert abs(b @ c - 1 / 2) < 1e-15
    if order >= 3:
        assert abs(b @ c ** 2 - 1 / 3) < 1e-15
        assert abs(b @ (A @ c) - 1 / 6) < 1e-15
    # row sums are the abscissae; SDIRK tableaus are stiffly accurate
    assert np.allclose(A.sum(1), c)
    if name.startswith("sdirk"):
        assert np.allclose(A[-1], b) and np.allclose(np.diag(A), A[0, 0])


def test_printed_sdirk3_lambda():
    lam = float(dict(_golden_rows("butcher_printed.txt"))["sdirk3_lambda"])
    assert abs(sdirk3_lambda() - lam) < 5e-11
    assert abs(round(sdirk3_lambda(), 10) - lam) < 1e-15


def test_brj_memory_table():
    """Sec. 5.2 table: diagonal block (nv (P+1)^3)^2 single-precision values
    per hexahedron, face flux Jacobians nv x nv per face point on 6 faces for
    both trace sides with ceil(3(P+1)/2)^2 face points (over-integration),
    and the dense Jacobian as 7 double-precision blocks."""
    for P, diag, off, total, dense, _sparse in _golden_rows("brj_memory_table.txt"):
        P = int(P)
        nq = math.ceil(3 * (P + 1) / 2)
        d = tiny_disc(dim=3, cells=(2, 1, 1), P=P, nq=nq, flux_mode=1, Ma=0.3)
        u = W.random_state(d.n_elem, 3, P, seed=1)
        pc = S.BRJ(d, u, 0.1, chunk=1) if P <= 2 else None
        nb = d.nv * d.ref.nm
        if pc is not None:
            assert pc.Dinv.shape[1:] == (nb, nb)
            per_elem_face = sum(Jp.size for (_, _, _, _, Jp) in pc.face_jp.values()) / d.n_elem
        else:
            per_elem_face = 2 * d.dim * d.ref.nqf * d.nv * d.nv
        assert nb * nb * 4 == int(diag)
        assert 2 * per_elem_face * 4 == int(off)        # dH/dQ^- and dH/dQ^+
        assert int(diag) + int(off) == int(total)
        assert 7 * nb * nb * 8 == int(dense)


# ---------------------------------------------------------------- Jacobians
def exact_jacobian(disc, u, Sv, dt_a):
    n = u.size
    J = np.zeros((n, n))
    h = 1e-30
    for k in range(n):
        uc = u.astype(np.complex128)
        uc.flat[k] += 1j * h
        J[:, k] = disc.stage_residual(uc, Sv, dt_a).imag.ravel() / h
    return J


@pytest.mark.parametrize("dim,cells,P,mode", [(2, (2, 2), 1, 0), (2, (2, 2), 2, 0), (2, (3, 2), 2, 1),
                                              (3, (2, 2, 2), 1, 0)])
def test_jfnk_matvec_against_exact_jacobian(dim, cells, P, mode):
    """P7: the Frechet difference of Eq. 25-26 matches the exact Jacobian."""
    d = tiny_disc(dim=dim, cells=cells, P=P, Ma=0.3, Re=30.0, flux_mode=mode)
    u = W.random_state(d.n_elem, dim, P, seed=11)
    Sv = 0.999 * u
    dt_a = 0.05
    J = exact_jacobian(d, u, Sv, dt_a)
    Nu = d.stage_residual(u, Sv, dt_a)
    rng = np.random.default_rng(3)
    for _ in range(3):
        w = rng.normal(size=u.shape)
        w /= np.linalg.norm(w)
        Jw = S.jfnk_matvec(d, u, Nu, Sv, dt_a, w)
        ex = (J @ w.ravel()).reshape(u.shape)
        assert np.linalg.norm(Jw - ex) <= 1e-6 * np.linalg.norm(ex)


def _dense_offdiag(pc, shape):
    n = int(np.prod(shape))
    O = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        O[:, k] = pc.offdiag(e.reshape(shape)).ravel()
    return O


def test_brj_blocks_equal_exact_jacobian_blocks_euler():
    """P8a: without viscous terms the dropped terms of Eq. 30 vanish, so the
    BRJ blocks are the exact Jacobian blocks up to the forward-difference
    error of Eq. 31."""
    d = tiny_disc(dim=2, cells=(3, 3), P=1, Ma=0.3, flux_mode=1)
    u = W.random_state(d.n_elem, 2, 1, seed=21)
    dt_a = 0.2
    J = exact_jacobian(d, u, u, dt_a)
    pc = S.BRJ(d, u, dt_a)
    nb = d.nv * d.ref.nm
    for e in range(d.n_elem):
        blk = J[e * nb:(e + 1) * nb, e * nb:(e + 1) * nb]
        assert np.abs(pc.D[e] - blk).max() <= 1e-6 * np.abs(blk).max()
    O = _dense_offdiag(pc, d.shape)
    Jo = J.copy()
    for e in range(d.n_elem):
        Jo[e * nb:(e + 1) * nb, e * nb:(e + 1) * nb] = 0.0
    assert np.abs(O - Jo).max() <= 1e-6 * np.abs(Jo).max()


def _frozen_stage_residual(d, u, u_p, Sv, dt_a):
    """N(u) with the face-trace gradients and the symmetric flux frozen at
    u_p: the residual whose exact Jacobian the kept terms of Eq. 30
    describe."""
    import dataclasses
    from oracle.physics import face_flux_own
    dv = dataclasses.replace(d, face_nbr=-np.ones_like(d.face_nbr), bc=lambda disc, uu: 0.0)
    L = dv.L(u)
    ref = d.ref
    for axis in range(d.dim):
        eL, eR = d.interior_faces(axis)
        fL, fR = 2 * axis + 1, 2 * axis
        QL, _ = d.trace(u, eL, fL)
        QR, _ = d.trace(u, eR, fR)
        QLp, gL = d.trace(u_p, eL, fL)
        QRp, gR = d.trace(u_p, eR, fR)
        n = np.zeros(QLp.shape[:-1] + (d.dim,))
        n[..., axis] = 1.0
        beta = np.broadcast_to(d.beta_p(eL, eR, axis)[:, None], QLp.shape[:-1])
        Hn, _ = face_flux_own(d.gas, QL, QR, gL, gR, n, beta)
        _, Sf = face_flux_own(d.gas, QLp, QRp, gL, gR, n, beta)
        wf = ref.WF[None, :] * d.face_det(eL, axis)[:, None]
        cL = -np.einsum('pm,kpv->kvm', ref.BF[fL], Hn * wf[..., None])
        cR = np.einsum('pm,kpv->kvm', ref.BF[fR], Hn * wf[..., None])
        for j in range(d.dim):
            Sw = Sf[:, :, j, :] * wf[..., None]
            cL = cL + np.einsum('pm,kpv->kvm', ref.DF[fL][j], Sw) * d.dxi[eL, j, None, None]
            cR = cR + np.einsum('pm,kpv->kvm', ref.DF[fR][j], Sw) * d.dxi[eR, j, None, None]
        np.add.at(L, eL, cL)
        np.add.at(L, eR, cR)
    return u - Sv - dt_a * d.apply_Minv(L)


def test_brj_blocks_equal_frozen_jacobian_ns():
    """P8b: with viscous terms, the BRJ blocks are the exact Jacobian blocks
    of the residual whose trace gradients and symmetric flux are frozen (the
    terms Eq. 30 keeps), up to the forward-difference error of Eq. 31; the
    frozen residual itself equals the full one at u_p."""
    d = tiny_disc(dim=2, cells=(3, 3), P=2, Ma=0.3, Re=20.0)
    u = W.random_state(d.n_elem, 2, 2, seed=22)
    dt_a = 0.2
    assert np.allclose(_frozen_stage_residual(d, u, u, u, dt_a), d.stage_residual(u, u, dt_a),
                       rtol=1e-13, atol=1e-13)
    n = u.size
    J = np.zeros((n, n))
    for k in range(n):
        uc = u.astype(np.complex128)
        uc.flat[k] += 1j * 1e-30
        J[:, k] = _frozen_stage_residual(d, uc, u, u, dt_a).imag.ravel() / 1e-30
    pc = S.BRJ(d, u, dt_a)
    nb = d.nv * d.ref.nm
    for e in range(d.n_elem):
        blk = J[e * nb:(e + 1) * nb, e * nb:(e + 1) * nb]
        assert np.abs(pc.D[e] - blk).max() <= 1e-6 * np.abs(blk).max()
    O = _dense_offdiag(pc, d.shape)
    for e in range(d.n_elem):
        J[e * nb:(e + 1) * nb, e * nb:(e + 1) * nb] = 0.0
    assert np.abs(O - J).max() <= 1e-6 * np.abs(J).max()
    # and against the full Jacobian the dropped viscous terms show, scaling
    # with 1/Re
    Jf = exact_jacobian(d, u, u, dt_a)
    rel = np.abs(pc.D[0] - Jf[:nb, :nb]).max() / np.abs(Jf[:nb, :nb]).max()
    assert rel > 1e-3


def test_brj_apply_equals_dense_iteration():
    """P11a: the on-the-fly BRJ(J) sweeps equal the dense iteration of Eq. 28."""
    d = tiny_disc(dim=2, cells=(3, 2), P=2, Ma=0.3, Re=50.0)
    u = W.random_state(d.n_elem, 2, 2, seed=31)
    for omega in (1.0, 0.8):
        pc = S.BRJ(d, u, 0.3, sweeps=7, omega=omega)
        n = int(np.prod(d.shape))
        nb = d.nv * d.ref.nm
        Dinv = scipy.linalg.block_diag(*pc.Dinv)
        O = _dense_offdiag(pc, d.shape)
        q = np.random.default_rng(4).normal(size=n)
        x = np.zeros(n)
        for _ in range(7):
            x = omega * Dinv @ (q - O @ x) + (1 - omega) * x
        y = pc.apply(q.reshape(d.shape)).ravel()
        assert np.abs(x - y).max() <= 1e-12 * np.abs(x).max()


def test_gmres_solves_dense_system():
    """P11b: with a tight tolerance and no restart GMRES returns the solution
    of the linear system."""
    rng = np.random.default_rng(5)
    n = 40
    A = np.eye(n) * 4 + rng.normal(size=(n, n)) * 0.3
    b = rng.normal(size=n)
    M = np.diag(1.0 / np.diag(A))
    x, its, ok, hist = S.gmres(lambda v: A @ v, lambda v: M @ v, b, restart=n, rtol=1e-13, maxit=n)
    assert ok
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    # restarted variant converges to the same solution
    x2, its2, ok2, _ = S.gmres(lambda v: A @ v, lambda v: M @ v, b, restart=5, rtol=1e-11, maxit=400)
    assert ok2 and its2 > 5
    assert np.allclose(x2, np.linalg.solve(A, b), rtol=1e-8, atol=1e-10)
    # residual estimate equals the true residual at exit
    x3, its3, ok3, hist3 = S.gmres(lambda v: A @ v, lambda v: M @ v, b, restart=30, rtol=5e-2)
    assert np.isclose(np.linalg.norm(b - A @ x3), hist3[-1], rtol=1e-8)
    assert hist3[-1] <= 5e-2 * np.linalg.norm(b)


def test_newton_jfnk_matches_dense_newton():
    """P12: JFNK-Newton reaches the root that Newton with exact Jacobian
    solves reaches."""
    d = tiny_disc(dim=2, cells=(2, 2), P=2, Ma=0.3, Re=40.0)
    un = W.random_state(d.n_elem, 2, 2, seed=41)
    dt_a = 0.05
    opts = S.SolverOpts(newton_rtol=1e-11, gmres_rtol=1e-3)
    pc = S.BRJ(d, un, dt_a)
    u1, st = S.newton_solve(d, un, dt_a, pc, opts)
    assert st.converged and st.newton_its <= 8
    u2 = un.copy()
    for _ in range(8):
        N = d.stage_residual(u2, un, dt_a)
        u2 = u2 - np.linalg.solve(exact_jacobian(d, u2, un, dt_a), N.ravel()).reshape(u2.shape)
    n0 = np.linalg.norm(d.stage_residual(un, un, dt_a))
    assert np.linalg.norm(d.stage_residual(u2, un, dt_a)) < 1e-13 * n0
    assert np.abs(u1 - u2).max() <= 1e-9 * np.abs(u2).max()


@pytest.mark.parametrize("scheme,order", [("sdirk2", 2), ("sdirk3", 3)])
def test_sdirk_temporal_order_linear(scheme, order):
    """P13 on a linear problem: the scalar-diffusion test operator makes
    M du/dt = L u linear, so u(T) = expm(T M^-1 dL/du) u0 exactly."""
    d = tiny_disc(dim=2, cells=(2, 2), P=2, lengths=(2 * np.pi, 2 * np.pi), Re=2.0, flux_mode=2)
    n = int(np.prod(d.shape))
    K = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        K[:, i] = d.residual(e.reshape(d.shape)).ravel()
    u0 = W.random_state(d.n_elem, 2, 2, seed=51, decay=0.3)
    T = 0.4
    ref = (scipy.linalg.expm(T * K) @ u0.ravel()).reshape(u0.shape)
    errs = []
    for nsteps in (4, 8, 16):
        opts = S.SolverOpts(scheme=scheme, newton_rtol=1e-13, gmres_rtol=1e-12, gmres_restart=200,
                            gmres_max=2000, pc_freeze=1000)
        st = S.SDIRK(d, opts)
        u = u0.copy()
        for _ in range(nsteps):
            u, _ = st.step(u, T / nsteps)
        errs.append(np.abs(u - ref).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > order - 0.3), (errs, rates)


def test_sdirk_preconditioner_refresh_rule():
    """With pc_refresh_its = 1 every stage after one whose GMRES took more
    than one iteration rebuilds the blocks at its S_m; the step still meets
    the Newton tolerance and stays within it of the frozen-blocks step."""
    d = tiny_disc(dim=2, cells=(3, 3), P=2, Ma=0.3, Re=40.0)
    u0 = W.random_state(d.n_elem, 2, 2, seed=51)
    frozen = S.SDIRK(d, S.SolverOpts(scheme="sdirk3", pc_refresh_its=0))
    fresh = S.SDIRK(d, S.SolverOpts(scheme="sdirk3", pc_refresh_its=1))
    builds = []
    orig = fresh.build_pc

    def counting(u_p, dt_a):
        builds.append(u_p.copy())
        return orig(u_p, dt_a)
    fresh.build_pc = counting
    ua, sa = frozen.step(u0, 0.2)
    ub, sb = fresh.step(u0, 0.2)
    assert len(builds) >= 2                           # the step's own build plus refreshes
    assert all(x.converged for x in sb)
    assert np.linalg.norm(ub - ua) <= 1e-6 * np.linalg.norm(ua)
