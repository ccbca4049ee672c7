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
@pytest.mark.parametrize("name,order", [("sdirk2", 2), ("sdirk3", 3), ("sdirk4", 4), ("beuler", 1), ("erk2", 2)])
def test_butcher_order_conditions(name, order):
    A, b, c = tableau(name)
    assert abs(b.sum() - 1) < 1e-15
    if order >= 2:
        assert abs(b @ c - 1 / 2) < 1e-15
    if order >= 3:
        assert abs(b @ c ** 2 - 1 / 3) < 1e-15
        assert abs(b @ (A @ c) - 1 / 6) < 1e-15
    if order >= 4:
        assert abs(b @ c ** 3 - 1 / 4) < 1e-15
        assert abs(b @ (c * (A @ c)) - 1 / 8) < 1e-15
        assert abs(b @ (A @ c ** 2) - 1 / 12) < 1e-15
        assert abs(b @ (A @ (A @ c)) - 1 / 24) < 1e-15
    # row sums are the abscissae; the implicit tableaus are stiffly accurate
    # with a single nonzero diagonal value
    assert np.allclose(A.sum(1), c)
    if name != "erk2":
        d = np.diag(A)
        assert np.allclose(A[-1], b) and np.allclose(d[d != 0], d[-1])
        # L-stable: the stability function R(z) = 1 + z b (I - z A)^-1 1 vanishes at infinity
        for z in (-1e6, -1e8):
            R = 1 + z * b @ np.linalg.solve(np.eye(len(b)) - z * A, np.ones(len(b)))
            assert abs(R) < 1e2 / abs(z)
    else:
        assert np.all(np.triu(A) == 0)


def test_printed_sdirk3_lambda():
    lam = float(dict(r for r in _golden_rows("butcher_printed.txt") if len(r) == 2)["sdirk3_lambda"])
    assert abs(sdirk3_lambda() - lam) < 5e-11
    assert abs(round(sdirk3_lambda(), 10) - lam) < 1e-15


def test_printed_sdirk4_entries():
    """The six-stage SDIRK4 equals the printed entries a^{mk}, k >= 1; its
    first column repeats the second and its abscissae are the row sums, which
    agree with the printed ones except c_2 (printed (2 - sqrt 2)/2, here
    (2 - sqrt 2)/4, the reading under which the order conditions hold)."""
    A, b, c = tableau("sdirk4")
    r2 = math.sqrt(2.0)
    rows = [r for r in _golden_rows("butcher_printed.txt") if len(r) == 7]
    seen = set()
    for kind, m, k, f, p, q, r in rows:
        m, k = int(m), int(k)
        v = float(f) * (float(p) + float(q) * r2) / float(r)
        if kind == "a":
            assert abs(A[m, k] - v) < 1e-15, (m, k)
            seen.add((m, k))
        elif m == 2:
            assert abs(v - (2 - r2) / 2) < 1e-15 and abs(c[2] - (2 - r2) / 4) < 1e-15
        else:
            assert abs(c[m] - v) < 1e-14, m
    assert len(seen) == 15                              # every printed entry below and on the diagonal
    assert np.array_equal(A[1:, 0], A[1:, 1]) and A[0, 0] == 0.0
    assert np.all(np.triu(A, 1) == 0)


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


@pytest.mark.parametrize("ortho", ["mgs", "cgs2"])
def test_gmres_solves_dense_system(ortho):
    """P11b: with a tight tolerance and no restart GMRES returns the solution
    of the linear system, with either orthogonalisation."""
    rng = np.random.default_rng(5)
    n = 40
    A = np.eye(n) * 4 + rng.normal(size=(n, n)) * 0.3
    b = rng.normal(size=n)
    M = np.diag(1.0 / np.diag(A))
    x, its, ok, hist = S.gmres(lambda v: A @ v, lambda v: M @ v, b, restart=n, rtol=1e-13, maxit=n, ortho=ortho)
    assert ok
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    # restarted variant converges to the same solution
    x2, its2, ok2, _ = S.gmres(lambda v: A @ v, lambda v: M @ v, b, restart=5, rtol=1e-11, maxit=400, ortho=ortho)
    assert ok2 and its2 > 5
    assert np.allclose(x2, np.linalg.solve(A, b), rtol=1e-8, atol=1e-10)
    # residual estimate equals the true residual at exit
    x3, its3, ok3, hist3 = S.gmres(lambda v: A @ v, lambda v: M @ v, b, restart=30, rtol=5e-2, ortho=ortho)
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


@pytest.mark.parametrize("scheme,order", [("sdirk2", 2), ("sdirk3", 3), ("sdirk4", 4), ("beuler", 1),
                                          ("bdf2", 2), ("erk2", 2)])
def test_sdirk_temporal_order_linear(scheme, order):
    """P13 on a linear problem: the scalar-diffusion test operator makes
    M du/dt = L u linear, so u(T) = expm(T M^-1 dL/du) u0 exactly; each
    stepper converges at its order."""
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
    # BDF2's backward-Euler start leaves the asymptotic range at 4 steps
    for nsteps in ((8, 16, 32) if scheme == "bdf2" else (4, 8, 16)):
        opts = S.SolverOpts(scheme=scheme, newton_rtol=1e-13, gmres_rtol=1e-12, gmres_restart=200,
                            gmres_max=2000, pc_freeze=1000)
        st = S.make_stepper(d, opts)
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


def test_erk2_step_is_second_order_taylor_polynomial():
    """On a linear problem one ERK2 step multiplies by the stability
    polynomial of every two-stage second-order explicit method,
    I + dt K + (dt K)^2 / 2; the step builds no preconditioner and runs no
    Newton iteration."""
    d = tiny_disc(dim=2, cells=(2, 2), P=2, lengths=(2 * np.pi, 2 * np.pi), Re=2.0, flux_mode=2)
    n = int(np.prod(d.shape))
    K = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        K[:, i] = d.residual(e.reshape(d.shape)).ravel()
    u0 = W.random_state(d.n_elem, 2, 2, seed=52, decay=0.3)
    dt = 0.05
    st = S.make_stepper(d, S.SolverOpts(scheme="erk2"))
    u1, stats = st.step(u0, dt)
    Kd = dt * K
    ref = (u0.ravel() + Kd @ u0.ravel() + 0.5 * Kd @ (Kd @ u0.ravel())).reshape(u0.shape)
    assert np.abs(u1 - ref).max() <= 1e-13 * np.abs(ref).max()
    assert st.pc is None and all(x.newton_its == 0 for x in stats)



def test_cgs2_basis_orthonormal_where_single_cgs_is_not():
    """The second classical pass restores orthogonality that one pass loses
    on an ill-conditioned Krylov sequence (Giraud-Langou-Rozloznik): the
    basis GMRES builds with "cgs2" stays orthonormal to rounding."""
    rng = np.random.default_rng(7)
    n = 60
    U, _ = np.linalg.qr(rng.normal(size=(n, n)))
    A = U @ np.diag(np.logspace(0, 12, n)) @ U.T
    b = rng.normal(size=n)
    basis = []

    def mv(v):
        basis.append(v)
        return A @ v
    S.gmres(mv, lambda v: v, b, restart=25, rtol=1e-30, maxit=25, ortho="cgs2")
    Vb = np.array(basis).T
    G = Vb.T @ Vb
    assert np.abs(G - np.eye(G.shape[0])).max() < 1e-14      # one classical pass: ~2e-10 here
