"""Implicit solver of Sec. 3.2 and Sec. 4.2.2, step by step.

  * Jacobian-free matvec (Eq. 25-26):  J q ~ (N(u + eps q) - N(u)) / eps,
    eps = ||u||_2 sqrt(eps_hat), eps_hat = 2^-52 (the printed 2.22e-16 is its
    rounding), ||u||_2 over the whole coefficient vector of the current
    Newton iterate, q the vector actually multiplied (not normalised), N(u)
    stored, the difference taken on N itself.
  * Block-relaxed Jacobi BRJ(J) (Eq. 27-28): q^0 = 0,
    q^j = omega D^-1 [q - (L+U) q^(j-1)] + (1-omega) q^(j-1).
    D_e = I - dt a M^-1 A_e with A_e the element block of dL/du built from
    the first three terms of Eq. 30: analytic volume flux Jacobians
    (dH_j/dQ at fixed grad Q and dH_j/d grad_i Q = -K), and the own-side
    face term with dHhat/dQ^- from the forward difference of Eq. 31 at
    fixed trace gradients.  The sign of the face term follows Eq. 13 (the
    residual subtracts the face flux); the '+' printed between the terms of
    Eq. 30 is read as part of the sum, not as a sign.  The last two terms of
    Eq. 30 (gradient and symmetric-flux dependence on the trace) are
    dropped, as the paper does.  (L+U) q is applied on the fly from the
    stored face Jacobians dHhat/dQ^+ (Eq. 31) and the neighbour trace of q.
    chi_v = ||u^(v)||_2 sqrt(eps_hat) with u^(v) all coefficients of
    variable v (||u||_2 sqrt(eps_hat) for a variable that is zero
    everywhere, where the paper's rule gives no step).  D_e is inverted explicitly with LU and partial pivoting.
  * GMRES (Sec. 3.2): restarted right-preconditioned GMRES(m) of Saad and
    Schultz with modified Gram-Schmidt (or classical Gram-Schmidt twice) and
    Givens rotations, x0 = 0,
    stopping when the residual has dropped by the factor rtol (5e-2) or
    after gmres_max iterations in total.  x = x0 + P^-1 V y (the
    preconditioner is linear: a fixed number of sweeps from q^0 = 0).
  * Newton (Eq. 21-23): u^0 = S_m, full steps, stop when
    ||N(u^l)|| < alpha ||N(u^0)||, or ||N(u^l)|| <= 1e-14 ||u^l|| when the
    initial residual is already at rounding level.
  * SDIRK (Eq. 17-20): S_m = u^n + sum_{i<m} a^mi E^i; after the stage solve
    E^m = (u^m - S_m) / a^mm (equal to dt M^-1 L(u^m) at convergence);
    u^{n+1} = u^n + sum b^i E^i.  A stage with a^mm = 0 (the first stage of
    the six-stage SDIRK4, every stage of ERK2) is explicit: u^m = S_m and
    E^m = dt M^-1 L(S_m).  The preconditioner is built at u^n of the step
    where it is (re)built and kept for pc_freeze steps or until dt a^mm
    changes.
  * BDF2 (Sec. 4.3 lists it among the implicit integrators; the paper gives
    no formula, the constant-step form is used): u^{n+1} - (4/3) u^n
    + (1/3) u^{n-1} = (2/3) dt M^-1 L(u^{n+1}), i.e. Eq. 20 with
    S = (4 u^n - u^{n-1}) / 3 and dt a = 2 dt / 3; the first step, and a
    step whose dt differs from the previous one's, is a backward-Euler step.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from .butcher import tableau
from .physics import euler_flux, viscous_flux, face_flux_own

EPS_HAT = 2.0 ** -52


def l2(x) -> float:
    return float(np.sqrt(np.sum(np.asarray(x) ** 2)))


def jfnk_eps(u) -> float:
    """eps of Eq. 26."""
    return l2(u) * np.sqrt(EPS_HAT)


def jfnk_matvec(disc, u, N_u, S, dt_a, q, eps=None):
    """(N(u + eps q) - N(u)) / eps   (Eq. 25)."""
    if eps is None or eps <= 0:
        eps = jfnk_eps(u)
    return (disc.stage_residual(u + eps * q, S, dt_a) - N_u) / eps


# ------------------------------------------------------------------ preconditioner
def volume_flux_jacobians(gas, Q, gQ):
    """dH_j/dQ at fixed gradient ([..., j, k, l], complex step) and
    dH_j/d(grad_i Q) ([..., j, i, k, l], exact: G is linear in grad Q)."""
    d = Q.shape[-1] - 2
    nv = d + 2
    h = 1e-30
    dHdQ = np.zeros(Q.shape[:-1] + (d, nv, nv))
    gQc = gQ.astype(np.complex128)
    for l in range(nv):
        Qc = Q.astype(np.complex128)
        Qc[..., l] += 1j * h
        Hc = euler_flux(gas, Qc) - viscous_flux(gas, Qc, gQc)
        dHdQ[..., :, :, l] = Hc.imag / h
    dHdG = np.zeros(Q.shape[:-1] + (d, d, nv, nv))
    for i in range(d):
        for l in range(nv):
            E = np.zeros(gQ.shape)
            E[..., i, l] = 1.0
            dHdG[..., :, i, :, l] = -viscous_flux(gas, Q, E)
    return dHdQ, dHdG


def face_sides(disc):
    """For every element face: (elements, face f, neighbours, neighbour's face,
    outward normal sign) for the faces that have a neighbour."""
    out = []
    for f in range(2 * disc.dim):
        axis, side = divmod(f, 2)
        e = np.arange(disc.n_elem)
        nb = disc.face_nbr[:, f]
        keep = nb >= 0
        out.append((e[keep], f, nb[keep], 2 * axis + (1 - side), -1.0 if side == 0 else 1.0))
    return out


def face_fd_jacobians(disc, u, chi, elems, f, nbrs, fn, sign):
    """Own-side and neighbour-side forward differences of Eq. 31 for the
    faces (elems, f): returns (dH/dQ^-, dH/dQ^+) as [k, p, v, l]."""
    gas, d, nv = disc.gas, disc.dim, disc.nv
    axis = f // 2
    Qo, go = disc.trace(u, elems, f)
    Qn, gn = disc.trace(u, nbrs, fn)
    n = disc.geo.nf[f][elems]                       # own outward normal
    eL, eR = (elems, nbrs) if f % 2 == 1 else (nbrs, elems)
    beta = np.broadcast_to(disc.beta_p(eL, eR, axis)[:, None], Qo.shape[:-1])
    H0, _ = face_flux_own(gas, Qo, Qn, go, gn, n, beta)
    Jm = np.zeros(Qo.shape + (nv,))
    Jp = np.zeros(Qo.shape + (nv,))
    for l in range(nv):
        dq = np.zeros(nv)
        dq[l] = chi[l]
        Hm, _ = face_flux_own(gas, Qo + dq, Qn, go, gn, n, beta)
        Hp, _ = face_flux_own(gas, Qo, Qn + dq, go, gn, n, beta)
        Jm[..., l] = (Hm - H0) / chi[l]
        Jp[..., l] = (Hp - H0) / chi[l]
    return Jm, Jp


class BRJ:
    """Block-relaxed Jacobi preconditioner BRJ(J) built at state u_p."""

    def __init__(self, disc, u_p, dt_a, sweeps=7, omega=1.0, chunk=256):
        self.disc, self.dt_a, self.sweeps, self.omega = disc, dt_a, sweeps, omega
        ref, gas, d, nv, nm = disc.ref, disc.gas, disc.dim, disc.nv, disc.ref.nm
        E = disc.n_elem
        nb = nv * nm
        # a variable that is zero everywhere (a velocity component of a
        # parallel flow) takes the norm of the whole state instead
        norms = np.array([l2(u_p[:, v, :]) for v in range(nv)])
        self.chi = np.where(norms > 0.0, norms, l2(u_p)) * np.sqrt(EPS_HAT)
        A = np.zeros((E, nv, nm, nv, nm))
        # volume terms (first two terms of Eq. 30)
        for s in range(0, E, chunk):
            el = np.arange(s, min(E, s + chunk))
            Q, gQ = disc.vol_values(u_p[el], el)
            dHdQ, dHdG = volume_flux_jacobians(gas, Q, gQ)
            wq = disc.geo.wJ[el]
            # physical derivatives of the basis at the points: sum_k dxi_k/dx_j D_k B
            Dx = np.einsum('eqkj,kqm->ejqm', disc.geo.Gq[el], np.stack(ref.D))                # [e,j,q,m]
            # sum over j, q of (w Dx)[j,q,m] T[q,j,k,l,n], with the point
            # factor T = dH_j/dQ B (first term) + sum_i dH_j/d(grad_i Q) Dx_i
            # (second term), taken as one matrix product per element
            T = np.einsum('eqjkl,qn->eqjkln', dHdQ, ref.B) + np.einsum('eqjikl,eiqn->eqjkln', dHdG, Dx)
            WDx = np.einsum('ejqm,eq->emqj', Dx, wq)
            ne, nq = WDx.shape[0], WDx.shape[2]
            A[el] += np.matmul(WDx.reshape(ne, nm, nq * d), T.reshape(ne, nq * d, nv * nv * nm)).reshape(
                ne, nm, nv, nv, nm).transpose(0, 2, 1, 3, 4)
        # own-side face term (third term of Eq. 30) and stored neighbour Jacobians
        self.face_jp = {}
        for elems, f, nbrs, fn, sign in face_sides(disc):
            Jm, Jp = face_fd_jacobians(disc, u_p, self.chi, elems, f, nbrs, fn, sign)
            wf = disc.geo.wJf[f][elems]
            A[elems] -= np.einsum('pm,kp,kpvl,pn->kvmln', ref.BF[f], wf, Jm, ref.BF[f], optimize=True)
            self.face_jp[f] = (elems, nbrs, fn, wf, Jp)
        # boundary faces: the boundary condition is inside the flux that is
        # differenced (Eq. 31), so only the own-side Jacobian exists
        if disc.bc_kind is not None:
            for elems, f, bid in disc.boundary_faces():
                Qo, go = disc.trace(u_p, elems, f)
                H0, _ = disc.boundary_flux(u_p, elems, f, bid, Qo, go)
                Jm = np.zeros(Qo.shape + (nv,))
                for l in range(nv):
                    dq = np.zeros(nv)
                    dq[l] = self.chi[l]
                    H1, _ = disc.boundary_flux(u_p, elems, f, bid, Qo + dq, go)
                    Jm[..., l] = (H1 - H0) / self.chi[l]
                wf = disc.geo.wJf[f][elems]
                A[elems] -= np.einsum('pm,kp,kpvl,pn->kvmln', ref.BF[f], wf, Jm, ref.BF[f], optimize=True)
        self.A_diag = A.reshape(E, nb, nb)
        Minv = np.linalg.inv(disc.M)                                       # [E, nm, nm]
        MinvA = np.einsum('emn,eknlo->ekmlo', Minv, A).reshape(E, nb, nb)
        self.Minv = Minv
        self.D = np.eye(nb)[None] - dt_a * MinvA
        self.Dinv = np.linalg.inv(self.D)

    def offdiag(self, q):
        """(L+U) q = -dt a M^-1 sum_f dL_e/du_e' q_e' with
        dL_e/du_e' = -(B^G_f)^T diag(w^G |J^G| dHhat/dQ^+) B^G_f'."""
        disc, ref = self.disc, self.disc.ref
        acc = np.zeros(q.shape)
        for f, (elems, nbrs, fn, wf, Jp) in self.face_jp.items():
            t = np.einsum('pm,kvm->kpv', ref.BF[fn], q[nbrs])
            flux = np.einsum('kpvl,kpl->kpv', Jp, t) * wf[..., None]
            acc[elems] -= np.einsum('pm,kpv->kvm', ref.BF[f], flux)
        return -self.dt_a * np.einsum('emn,evn->evm', self.Minv, acc)

    def diag_solve(self, r):
        E, nv, nm = r.shape
        return np.einsum('eab,eb->ea', self.Dinv, r.reshape(E, nv * nm)).reshape(E, nv, nm)

    def apply(self, q, sweeps=None):
        J = self.sweeps if sweeps is None else sweeps
        w = self.omega
        qh = np.zeros_like(q)
        for j in range(J):
            r = q - self.offdiag(qh) if j > 0 else q
            qh = w * self.diag_solve(r) + (1.0 - w) * qh
        return qh


# ------------------------------------------------------------------ GMRES
def gmres(matvec, precond, b, restart=30, rtol=5e-2, maxit=300, ortho="mgs"):
    """Right-preconditioned restarted GMRES(m); returns (x, iterations,
    converged, residual history).  ortho: "mgs" (modified Gram-Schmidt, one
    projection at a time) or "cgs2" (classical Gram-Schmidt applied twice:
    all projections of a pass from the same vector, the second pass
    removing what rounding left of the first; the Hessenberg column is the
    sum of both passes' coefficients)."""
    x = np.zeros_like(b)
    beta0 = l2(b)
    hist = [beta0]
    total = 0
    if beta0 == 0.0:
        return x, 0, True, hist
    r = b
    converged = False
    while True:
        beta = l2(r)
        if beta <= rtol * beta0:
            converged = True
            break
        m = restart
        V = [r / beta]
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k_used = 0
        for k in range(m):
            z = precond(V[k])
            w = matvec(z)
            total += 1
            if ortho == "cgs2":
                for _ in range(2):
                    h = np.array([float(np.sum(w * V[i])) for i in range(k + 1)])
                    w = w - sum(h[i] * V[i] for i in range(k + 1))
                    H[:k + 1, k] += h
            else:
                for i in range(k + 1):
                    H[i, k] = float(np.sum(w * V[i]))
                    w = w - H[i, k] * V[i]
            H[k + 1, k] = l2(w)
            breakdown = H[k + 1, k] == 0.0
            V.append(w / H[k + 1, k] if not breakdown else np.zeros_like(w))
            for i in range(k):
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            den = np.hypot(H[k, k], H[k + 1, k])
            cs[k] = H[k, k] / den
            sn[k] = H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            k_used = k + 1
            hist.append(abs(g[k + 1]))
            if abs(g[k + 1]) <= rtol * beta0 or breakdown or total >= maxit:
                converged = abs(g[k + 1]) <= rtol * beta0 or breakdown
                break
        y = np.zeros(k_used)
        for i in range(k_used - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:k_used], y[i + 1:k_used])) / H[i, i]
        Vy = sum(y[i] * V[i] for i in range(k_used))
        x = x + precond(Vy)
        if converged or total >= maxit:
            break
        r = b - matvec(x)
    return x, total, converged, hist


# ------------------------------------------------------------------ Newton / SDIRK
@dataclasses.dataclass
class SolverOpts:
    scheme: str = "sdirk2"
    newton_rtol: float = 1e-8
    newton_max: int = 30
    gmres_restart: int = 30
    gmres_rtol: float = 5e-2
    gmres_max: int = 300
    brj_sweeps: int = 7
    brj_omega: float = 1.0
    pc_freeze: int = 10
    pc_refresh_its: int = 30      # rebuild before a stage when the last Newton step's GMRES took more (0: never)
    ortho: str = "mgs"            # GMRES orthogonalisation: "mgs" or "cgs2"
    use_pc: bool = True


@dataclasses.dataclass
class StageStats:
    newton_its: int = 0
    gmres_its: List[int] = dataclasses.field(default_factory=list)
    nres: List[float] = dataclasses.field(default_factory=list)
    converged: bool = True


class NotConverged(RuntimeError):
    pass


def newton_solve(disc, S, dt_a, pc, opts: SolverOpts, guess=None):
    """Solve N(u) = 0 of Eq. 20 by Newton (Eq. 21-23) with JFNK-GMRES."""
    u = S.copy() if guess is None else guess.copy()
    N = disc.stage_residual(u, S, dt_a)
    n0 = l2(N)
    st = StageStats(nres=[n0])
    precond = pc.apply if (pc is not None and opts.use_pc) else (lambda v: v)
    nrm = n0
    while True:
        if nrm < opts.newton_rtol * n0 or nrm <= 1e-14 * l2(u):
            break
        if st.newton_its >= opts.newton_max:
            st.converged = False
            break
        eps = jfnk_eps(u)
        Nu = N
        mv = lambda q, u=u, Nu=Nu, eps=eps: jfnk_matvec(disc, u, Nu, S, dt_a, q, eps)
        delta, its, ok, _ = gmres(mv, precond, -N, opts.gmres_restart, opts.gmres_rtol, opts.gmres_max,
                                  opts.ortho)
        st.gmres_its.append(its)
        u = u + delta
        N = disc.stage_residual(u, S, dt_a)
        nrm = l2(N)
        st.nres.append(nrm)
        st.newton_its += 1
        if not np.isfinite(nrm):
            st.converged = False
            break
    return u, st


class SDIRK:
    """Implicit Runge-Kutta stepper with a frozen BRJ preconditioner: built at
    u^n and kept for pc_freeze steps while dt a^mm is unchanged (Sec. 4.2.2).
    Two refresh rules beyond the paper's fixed freeze: before a stage, when
    the last Newton step's GMRES needed more than pc_refresh_its iterations,
    the blocks are rebuilt at the stage's S_m; a stage whose Newton solve
    fails is retried once from S_m with blocks rebuilt at S_m."""

    def __init__(self, disc, opts: SolverOpts):
        self.disc, self.opts = disc, opts
        self.A, self.b, self.c = tableau(opts.scheme)
        self.pc: Optional[BRJ] = None
        self.pc_age = 0
        self.pc_dta = None
        self.last_gmres_max = 0

    def build_pc(self, u_p, dt_a):
        self.pc = BRJ(self.disc, u_p, dt_a, self.opts.brj_sweeps, self.opts.brj_omega)
        self.pc_age = 0
        self.pc_dta = dt_a
        self.last_gmres_max = 0

    def ensure_pc(self, u_n, dt_a):
        if not self.opts.use_pc:
            return
        if self.pc is None or self.pc_age >= self.opts.pc_freeze or self.pc_dta != dt_a:
            self.build_pc(u_n, dt_a)

    def first_implicit(self):
        d = np.diag(self.A)
        nz = [m for m in range(len(d)) if d[m] != 0.0]
        return nz[0] if nz else None

    def solve_stage(self, S, dt_a, guess=None):
        """Newton solve of one implicit stage with the refresh rules."""
        refresh = self.opts.use_pc and self.opts.pc_refresh_its > 0
        if refresh and self.last_gmres_max > self.opts.pc_refresh_its:
            self.build_pc(S, dt_a)
        u_m, st = newton_solve(self.disc, S, dt_a, self.pc, self.opts, guess=guess)
        if not st.converged and refresh:
            self.build_pc(S, dt_a)
            u_m, st = newton_solve(self.disc, S, dt_a, self.pc, self.opts)
        self.last_gmres_max = max(st.gmres_its) if st.gmres_its else 0
        return u_m, st

    def step(self, u_n, dt, guesses=None):
        A, b = self.A, self.b
        s = A.shape[0]
        Es = []
        stats = []
        m0 = self.first_implicit()
        if m0 is not None:
            self.ensure_pc(u_n, dt * A[m0, m0])
        for m in range(s):
            S = u_n + sum(A[m, i] * Es[i] for i in range(m)) if m > 0 else u_n.copy()
            if A[m, m] == 0.0:
                # explicit stage: the stage value is S_m itself
                Es.append(dt * self.disc.residual(S))
                stats.append(StageStats())
                continue
            dt_a = dt * A[m, m]
            g = None if guesses is None else guesses[m]
            u_m, st = self.solve_stage(S, dt_a, g)
            stats.append(st)
            if not st.converged:
                raise NotConverged(f"stage {m}: Newton did not converge: {st.nres}")
            Es.append((u_m - S) / A[m, m])
        self.pc_age += 1
        u_new = u_n + sum(b[i] * Es[i] for i in range(s))
        return u_new, stats


class BDF2(SDIRK):
    """Constant-step BDF2 with a backward-Euler start (see the module notes);
    the preconditioner and its refresh rules are those of the RK steppers."""

    def __init__(self, disc, opts: SolverOpts):
        super().__init__(disc, dataclasses.replace(opts, scheme="beuler"))
        self.u_prev = None
        self.dt_prev = None

    def step(self, u_n, dt, guesses=None):
        if self.u_prev is None or self.dt_prev != dt:
            S, dt_a = u_n.copy(), dt
        else:
            S, dt_a = (4.0 * u_n - self.u_prev) / 3.0, 2.0 * dt / 3.0
        self.ensure_pc(u_n, dt_a)
        g = None if guesses is None else guesses[0]
        u_new, st = self.solve_stage(S, dt_a, g)
        if not st.converged:
            raise NotConverged(f"BDF2: Newton did not converge: {st.nres}")
        self.u_prev, self.dt_prev = u_n.copy(), dt
        self.pc_age += 1
        return u_new, [st]


def make_stepper(disc, opts: SolverOpts):
    """The time stepper named by opts.scheme: sdirk2, sdirk3, sdirk4, beuler,
    erk2 (Runge-Kutta tableaus) or bdf2."""
    if opts.scheme == "bdf2":
        return BDF2(disc, opts)
    return SDIRK(disc, opts)
