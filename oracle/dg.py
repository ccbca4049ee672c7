"""DG spatial residual R(u) = M^-1 L(u) of Eq. 13, written out densely.

Discretisation (Sec. 3.1): for element e with test function phi_p,

  L_e[p] =   sum_q w_q |J| grad phi_p(x_q) . (F - G)(Q_q, grad Q_q)          (volume)
           - sum_faces sum_i w^G_i |J^G| phi_p(x_i) Hhat^n_i                 (Riemann + IP)
           + sum_faces sum_i w^G_i |J^G| grad phi_p(x_i) . Shat_i           (symmetric IP term)

with Q = B u (Eq. 9), Hhat^n = Fhat^n - Ghat^n and the IP fluxes of
physics.ip_face_fluxes.  Each interior face is visited once and contributes
to the test functions on both of its sides (the sum over element
boundaries of Eq. 12 would otherwise count it twice).  The penalty is
beta_p = (P+1)^2 / h with h = min(|Omega_e|, |Omega_e'|) / |Gamma_f|, the
element width normal to the face on a Cartesian grid (the paper does not
define h).  Traces are evaluated directly at the face quadrature points
(equal to interpolation from the volume points on affine elements).

Geometry (oracle/geometry.py): affine boxes x = origin + (xi + 1) h / 2,
with d/dx_j = (2/h_j) d/dxi_j, |J| = prod(h)/2^d and |J^Gamma| the product
of the tangential half-widths; or isoparametric curved elements with the
metrics d xi / d x, |J|, the outward normal and |J^Gamma| taken pointwise,
gradients grad Q = (d xi/d x)^T grad_xi Q, and the dense mass matrix
M_e = B^T diag(w |J|) B.  On curved elements h = min(|Omega_e|,
|Omega_e'|) / |Gamma_f| uses quadrature volumes and areas.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np

from .basis import ref_element
from .geometry import Geometry
from .physics import Gas, euler_flux, viscous_flux, face_flux_own, BC_DIRICHLET


@dataclasses.dataclass
class Disc:
    """A DG discretisation on a structured mesh of affine boxes or of
    isoparametric curved elements (geo_nodes [E, (geo_order+1)^d, d])."""
    gas: Gas
    dim: int
    P: int
    nq: int
    elem_origin: Optional[np.ndarray]
    elem_h: Optional[np.ndarray]
    face_nbr: np.ndarray
    bc: Optional[Callable] = None   # extra boundary contribution hook (tests)
    bc_kind: Optional[np.ndarray] = None    # per boundary id: one of the BC_* kinds of physics.py
    bc_state: Optional[np.ndarray] = None   # per boundary id: freestream conserved state [nv]
    geo_nodes: Optional[np.ndarray] = None  # curved elements: isoparametric nodes
    geo_order: int = 1
    viscous: str = "ip"                     # viscous face terms: "ip" (Eq. 12) or "ldg"
    bc_field: Optional[np.ndarray] = None   # Dirichlet ghost states [E, 2d, nv, nqf] (faces of that kind)
    source: Optional[np.ndarray] = None     # modal source [E, nv, nm] added to M^-1 L

    def __post_init__(self):
        self.ref = ref_element(self.dim, self.P, self.nq)
        self.nv = self.dim + 2
        self.n_elem = self.face_nbr.shape[0]
        ref = self.ref
        self.geo = Geometry(ref, self.dim, self.elem_origin, self.elem_h, self.geo_nodes, self.geo_order)
        self.detJ = self.geo.detJ                                   # [E] (boxes only)
        self.dxi = self.geo.dxi                                     # [E, d] dxi_j/dx_j (boxes only)
        self.vol = self.geo.vol
        self._M = None

    @property
    def M(self):
        """Mass matrices M_e = B^T diag(w |J|) B (Eq. 13), formed on first use."""
        if self._M is None:
            ref = self.ref
            if self.geo.curved:
                self._M = np.einsum('qm,eq,qn->emn', ref.B, self.geo.wJ, ref.B)
            else:
                self._M = np.einsum('qm,q,qn->mn', ref.B, ref.W, ref.B)[None] * self.detJ[:, None, None]
        return self._M

    @property
    def shape(self):
        return (self.n_elem, self.nv, self.ref.nm)

    def face_det(self, e, axis):
        h = self.elem_h[e]
        return np.prod(np.delete(h, axis, axis=-1) / 2.0, axis=-1)

    def beta_p(self, eL, eR, axis):
        """Penalty of the faces between eL (side 1) and eR (side 0)."""
        area = self.geo.area[2 * axis + 1][eL]
        hf = np.minimum(self.vol[eL], self.vol[eR]) / area
        return (self.P + 1) ** 2 / hf

    def phys_grad(self, G, dref):
        """grad Q[..., j, v] = sum_k (d xi_k / d x_j) d Q_v / d xi_k."""
        return np.einsum('...kj,k...v->...jv', G, dref)

    def lift_S(self, f, elems, Sw):
        """sum_k (D_k B^G_f)^T (sum_j (d xi_k/d x_j) S_j w|J^G|) for the
        weighted symmetric-term flux Sw[k, p, j, v] of face f of elems."""
        ref = self.ref
        Gf = self.geo.Gf[f][elems]
        out = 0.0
        for k in range(self.dim):
            Sk = np.einsum('epj,epjv->epv', Gf[:, :, k, :], Sw)
            out = out + np.einsum('pm,kpv->kvm', ref.DF[f][k], Sk)
        return out

    # -- element-level evaluations ------------------------------------------------
    def vol_values(self, u, elems=None):
        """Q[e, q, v] and grad Q[e, q, j, v] at the volume points of the
        elements elems (all if None; u holds their coefficients)."""
        ref = self.ref
        Q = np.einsum('qm,evm->eqv', ref.B, u)
        dref = np.stack([np.einsum('qm,evm->eqv', ref.D[k], u) for k in range(self.dim)])
        Gq = self.geo.Gq if elems is None else self.geo.Gq[elems]
        return Q, self.phys_grad(Gq, dref)

    def trace(self, u, elems, f):
        """Trace value [k, p, v] and broken gradient [k, p, j, v] of the
        elements `elems` at the points of their face f."""
        ref = self.ref
        ue = u[elems]
        Q = np.einsum('pm,evm->epv', ref.BF[f], ue)
        dref = np.stack([np.einsum('pm,evm->epv', ref.DF[f][k], ue) for k in range(self.dim)])
        return Q, self.phys_grad(self.geo.Gf[f][elems], dref)

    def interior_faces(self, axis):
        """Interior faces normal to `axis` as (left elems, right elems): the
        left element meets the face with its side 1, the right one with
        side 0."""
        eL = np.arange(self.n_elem)
        eR = self.face_nbr[:, 2 * axis + 1]
        keep = eR >= 0
        return eL[keep], eR[keep]

    # -- the residual -------------------------------------------------------------
    def L(self, u):
        """L(u) of Eq. 16 (the right-hand side before M^-1)."""
        gas, ref, d = self.gas, self.ref, self.dim
        u = np.asarray(u)
        if self.viscous == "ldg":
            return self.L_ldg(u)
        Q, gQ = self.vol_values(u)
        H = euler_flux(gas, Q) - viscous_flux(gas, Q, gQ)                  # [e, q, j, v]
        wq = self.geo.wJ                                                     # [e, q]
        L = np.zeros(u.shape, dtype=np.result_type(u, np.float64))
        for k in range(d):
            Hk = np.einsum('eqj,eqjv->eqv', self.geo.Gq[:, :, k, :], H)      # contravariant flux
            L += np.einsum('qm,eqv->evm', ref.D[k], Hk * wq[:, :, None])
        for axis in range(d):
            eL, eR = self.interior_faces(axis)
            fL, fR = 2 * axis + 1, 2 * axis
            QL, gL = self.trace(u, eL, fL)
            QR, gR = self.trace(u, eR, fR)
            n = self.geo.nf[fL][eL]                                          # side 1's outward normal
            beta = np.broadcast_to(self.beta_p(eL, eR, axis)[:, None], QL.shape[:-1])
            Hn, S = face_flux_own(gas, QL, QR, gL, gR, n, beta)
            wf = self.geo.wJf[fL][eL]                                        # [k, p]
            contribL = -np.einsum('pm,kpv->kvm', ref.BF[fL], Hn * wf[..., None])
            contribR = np.einsum('pm,kpv->kvm', ref.BF[fR], Hn * wf[..., None])
            Sw = S * wf[..., None, None]
            contribL = contribL + self.lift_S(fL, eL, Sw)
            contribR = contribR + self.lift_S(fR, eR, Sw)
            np.add.at(L, eL, contribL)
            np.add.at(L, eR, contribR)
        if np.any(self.face_nbr < 0):
            if self.bc is not None:
                L += self.bc(self, u)
            elif self.bc_kind is not None:
                L += self.boundary_terms(u)
            else:
                raise ValueError("mesh has boundary faces but no boundary condition")
        return L

    # -- LDG (the viscous option "ldg"; readings in physics.py) ------------------
    def _boundary_data(self, u, e, f, bid, Qo):
        """Per-point given states Uinf [k, p, v] of boundary faces (e, f)."""
        out = np.zeros(Qo.shape)
        for b in np.unique(bid):
            k = bid == b
            if int(self.bc_kind[b]) == BC_DIRICHLET:
                out[k] = np.transpose(self.bc_field[e[k], f], (0, 2, 1))
            else:
                out[k] = self.bc_state[b]
        return out

    def ldg_lift(self, u):
        """r[e, j, v, m] with M_e r_j = sum over the faces of the integral of
        phi (u_hat - u^-) n_j: nonzero on faces where the element is the
        right one (u_hat from the left) and on boundary faces (u_hat the mean
        of interior and ghost states)."""
        from .physics import boundary_ghost
        ref, d = self.ref, self.dim
        rhs = np.zeros((self.n_elem, d) + self.shape[1:], dtype=np.result_type(u, np.float64))
        for axis in range(d):
            eL, eR = self.interior_faces(axis)
            fL, fR = 2 * axis + 1, 2 * axis
            QL, _ = self.trace(u, eL, fL)
            QR, _ = self.trace(u, eR, fR)
            n = -self.geo.nf[fL][eL]                        # outward from the right element
            wf = self.geo.wJf[fL][eL]
            c = np.einsum('pm,kpv,kp,kpj->kjvm', ref.BF[fR], QL - QR, wf, n)
            np.add.at(rhs, eR, c)
        if self.bc_kind is not None:
            for e, f, bid in self.boundary_faces():
                Qo, _ = self.trace(u, e, f)
                n = self.geo.nf[f][e]
                Ub = self._boundary_data(u, e, f, bid, Qo)
                Ug = np.zeros(Qo.shape, dtype=Qo.dtype)
                for b in np.unique(bid):
                    k = bid == b
                    Ug[k] = boundary_ghost(self.gas, int(self.bc_kind[b]), Qo[k], n[k], Ub[k])
                wf = self.geo.wJf[f][e]
                c = np.einsum('pm,kpv,kp,kpj->kjvm', ref.BF[f], 0.5 * (Ug - Qo), wf, n)
                np.add.at(rhs, e, c)
        Minv = np.linalg.inv(self.M)
        return np.einsum('emn,ejvn->ejvm', Minv, rhs)

    def L_ldg(self, u):
        from .physics import riemann_flux, ldg_viscous_flux_n, boundary_flux_own_ldg
        gas, ref, d = self.gas, self.ref, self.dim
        r = self.ldg_lift(u)
        Q, gQ = self.vol_values(u)
        gQ = gQ + np.einsum('qm,ejvm->eqjv', ref.B, r)
        H = euler_flux(gas, Q) - viscous_flux(gas, Q, gQ)
        wq = self.geo.wJ
        L = np.zeros(u.shape, dtype=np.result_type(u, np.float64))
        for k in range(d):
            Hk = np.einsum('eqj,eqjv->eqv', self.geo.Gq[:, :, k, :], H)
            L += np.einsum('qm,eqv->evm', ref.D[k], Hk * wq[:, :, None])
        for axis in range(d):
            eL, eR = self.interior_faces(axis)
            fL, fR = 2 * axis + 1, 2 * axis
            QL, _ = self.trace(u, eL, fL)
            QR, gR = self.trace(u, eR, fR)
            gR = gR + np.einsum('pm,kjvm->kpjv', ref.BF[fR], r[eR])
            n = self.geo.nf[fL][eL]
            beta = np.broadcast_to(self.beta_p(eL, eR, axis)[:, None], QL.shape[:-1])
            Hn = riemann_flux(gas, QL, QR, n) - ldg_viscous_flux_n(gas, QL, gR, QL - QR, n, beta)
            wf = self.geo.wJf[fL][eL]
            np.add.at(L, eL, -np.einsum('pm,kpv->kvm', ref.BF[fL], Hn * wf[..., None]))
            np.add.at(L, eR, np.einsum('pm,kpv->kvm', ref.BF[fR], Hn * wf[..., None]))
        if np.any(self.face_nbr < 0):
            if self.bc_kind is None:
                raise ValueError("mesh has boundary faces but no boundary condition")
            for e, f, bid in self.boundary_faces():
                Qo, go = self.trace(u, e, f)
                go = go + np.einsum('pm,kjvm->kpjv', ref.BF[f], r[e])
                n = self.geo.nf[f][e]
                beta = np.broadcast_to(self.boundary_beta(e, f)[:, None], Qo.shape[:-1])
                Ub = self._boundary_data(u, e, f, bid, Qo)
                Hb = np.zeros(Qo.shape, dtype=np.result_type(Qo, go))
                for b in np.unique(bid):
                    k = bid == b
                    Hb[k] = boundary_flux_own_ldg(gas, int(self.bc_kind[b]), Qo[k], go[k], n[k], beta[k], Ub[k])
                wf = self.geo.wJf[f][e]
                np.add.at(L, e, -np.einsum('pm,kpv->kvm', ref.BF[f], Hb * wf[..., None]))
        return L

    def boundary_faces(self):
        """(elements, face f, boundary id) of every boundary face."""
        out = []
        for f in range(2 * self.dim):
            e = np.nonzero(self.face_nbr[:, f] < 0)[0]
            if e.size:
                out.append((e, f, -self.face_nbr[e, f] - 1))
        return out

    def boundary_beta(self, e, f):
        return (self.P + 1) ** 2 / (self.vol[e] / self.geo.area[f][e])

    def boundary_flux(self, u, e, f, bid, Qo=None, go=None):
        """Flux (H^n, S) of the boundary faces (e, f) in e's orientation."""
        from .physics import boundary_flux_own
        if Qo is None:
            Qo, go = self.trace(u, e, f)
        n = self.geo.nf[f][e]
        beta = np.broadcast_to(self.boundary_beta(e, f)[:, None], Qo.shape[:-1])
        H = np.zeros(Qo.shape, dtype=np.result_type(Qo, go))
        S = np.zeros(go.shape, dtype=H.dtype)
        for b in np.unique(bid):
            k = bid == b
            kind = int(self.bc_kind[b])
            if kind == BC_DIRICHLET:
                Ub = np.transpose(self.bc_field[e[k], f], (0, 2, 1))       # [k, p, v]
            else:
                Ub = self.bc_state[b]
            Hb, Sb = boundary_flux_own(self.gas, kind, Qo[k], go[k], n[k], beta[k], Ub)
            H[k], S[k] = Hb, Sb
        return H, S

    def boundary_terms(self, u):
        """Lifted boundary face fluxes: -phi H + grad phi . S on each boundary face."""
        ref = self.ref
        L = np.zeros(u.shape, dtype=np.result_type(u, np.float64))
        for e, f, bid in self.boundary_faces():
            H, S = self.boundary_flux(u, e, f, bid)
            wf = self.geo.wJf[f][e]
            c = -np.einsum('pm,kpv->kvm', ref.BF[f], H * wf[..., None])
            c = c + self.lift_S(f, e, S * wf[..., None, None])
            np.add.at(L, e, c)
        return L

    def apply_Minv(self, L):
        """Solve M_e x = L_e for every element and variable."""
        return np.linalg.solve(self.M[:, None, :, :], L[..., None])[..., 0]

    def residual(self, u):
        """R(u) = M^-1 L(u), plus the modal source when one is set (a forcing
        f of the equations, projected: M^-1 of the integrals of phi f)."""
        R = self.apply_Minv(self.L(u))
        if self.source is not None:
            R = R + self.source
        return R

    def stage_residual(self, u, S, dt_a):
        """N(u) = u - S - dt a^mm M^-1 L(u)   (Eq. 20)."""
        return u - S - dt_a * self.residual(u)

    # -- initial conditions -------------------------------------------------------
    def points(self):
        """Physical coordinates of the volume quadrature points [e, q, j]."""
        return self.geo.xq

    def project_values(self, vals):
        """L2 projection of values [E, nv, nq^d] given at the volume points."""
        wq = self.geo.wJ
        rhs = np.einsum('qm,evq->evm', self.ref.B, vals * wq[:, None, :])
        return self.apply_Minv(rhs)

    def project(self, fn):
        """L2 projection of a pointwise field fn(x[..., d]) -> [..., nv]."""
        vals = fn(self.points())
        wq = self.geo.wJ
        rhs = np.einsum('qm,eqv->evm', self.ref.B, vals * wq[..., None])
        return self.apply_Minv(rhs)


def restricted_disc(gas, dim, P, nq, face_nbr, sample, elem_origin=None, elem_h=None, geo_nodes=None,
                    geo_order=1, bc_kind=None, bc_state=None) -> tuple:
    """Discretisation of the elements `sample` of a mesh and their face
    neighbours, in which faces that leave this set become far-field faces
    of an extra boundary id.  The residual of each sample element is then
    the full mesh's (its own and its neighbours' traces are all present);
    the other elements' are not meaningful.  Returns (sub, kept element
    ids, positions of the sample elements in sub)."""
    from .physics import BC_FARFIELD
    sample = [int(e) for e in sample]
    keep = sorted(set(sample) | {int(x) for e in sample for x in face_nbr[e] if x >= 0})
    loc = {e: i for i, e in enumerate(keep)}
    n_bc = 0 if bc_kind is None else len(bc_kind)
    sub = np.empty((len(keep), face_nbr.shape[1]), dtype=np.int32)
    for i, e in enumerate(keep):
        for f in range(face_nbr.shape[1]):
            x = int(face_nbr[e, f])
            sub[i, f] = x if x < 0 else (loc[x] if x in loc else -(n_bc + 1))
    free = np.zeros((1, dim + 2))
    free[0, 0] = 1.0
    free[0, -1] = 1.0 / (gas.gamma * gas.Ma ** 2) / (gas.gamma - 1.0)
    kinds = np.concatenate([[] if bc_kind is None else bc_kind, [BC_FARFIELD]]).astype(int)
    states = free if bc_state is None else np.concatenate([bc_state, free])
    pick = lambda a: None if a is None else np.asarray(a)[keep]
    d = Disc(gas=gas, dim=dim, P=P, nq=nq, elem_origin=pick(elem_origin), elem_h=pick(elem_h), face_nbr=sub,
             bc_kind=kinds, bc_state=states, geo_nodes=pick(geo_nodes), geo_order=geo_order)
    return d, keep, [loc[e] for e in sample]


def restrict(disc: Disc, sample) -> tuple:
    """restricted_disc of an existing discretisation."""
    return restricted_disc(disc.gas, disc.dim, disc.P, disc.nq, disc.face_nbr, sample, disc.elem_origin,
                           disc.elem_h, disc.geo_nodes, disc.geo_order, disc.bc_kind, disc.bc_state)


def make_disc(cfg, mesh, **gas_overrides) -> Disc:
    kw = dict(gamma=cfg.gamma, Pr=cfg.Pr, Re=cfg.Re, Ma=cfg.Ma, visc_law=cfg.visc_law,
              T_ref_K=cfg.T_ref_K, flux_mode=cfg.flux_mode, riemann=cfg.riemann)
    kw.update(gas_overrides)
    return Disc(gas=Gas(**kw), dim=mesh.dim, P=cfg.P, nq=cfg.nq, elem_origin=mesh.elem_origin,
                elem_h=mesh.elem_h, face_nbr=mesh.face_nbr, geo_nodes=getattr(mesh, "geo_nodes", None),
                geo_order=getattr(mesh, "geo_order", 1), viscous=getattr(cfg, "viscous", "ip"))


def conserved_from_primitive(gamma, rho, vel, p):
    """U = (rho, rho u, p/(gamma-1) + rho |u|^2 / 2)."""
    E = p / (gamma - 1.0) + 0.5 * rho * np.sum(vel * vel, axis=-1)
    return np.concatenate([rho[..., None], rho[..., None] * vel, E[..., None]], axis=-1)


def taylor_green(gas: Gas, dim: int):
    """Taylor-Green vortex field at T = 1 (rho = p / p_inf) with
    p_inf = 1/(gamma Ma^2).  2D: u = sin x cos y, v = -cos x sin y,
    p = p_inf + (cos 2x + cos 2y)/4.  3D: u = sin x cos y cos z,
    v = -cos x sin y cos z, w = 0, p = p_inf + (cos 2x + cos 2y)(cos 2z + 2)/16."""
    pinf = 1.0 / (gas.gamma * gas.Ma ** 2)

    def fn(x):
        if dim == 2:
            X, Y = x[..., 0], x[..., 1]
            vel = np.stack([np.sin(X) * np.cos(Y), -np.cos(X) * np.sin(Y)], axis=-1)
            p = pinf + (np.cos(2 * X) + np.cos(2 * Y)) / 4.0
        else:
            X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
            vel = np.stack([np.sin(X) * np.cos(Y) * np.cos(Z), -np.cos(X) * np.sin(Y) * np.cos(Z),
                            0.0 * X], axis=-1)
            p = pinf + (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0
        rho = p / pinf
        return conserved_from_primitive(gas.gamma, rho, vel, p)
    return fn


def initial_state(disc: Disc, noise: np.ndarray, noise_amp: float):
    """Taylor-Green field, L2-projected, plus noise_amp * sigma_v * noise on
    every modal coefficient with sigma = (1, 1, .., 1, E_ref) and
    E_ref = p_inf/(gamma-1) + 1/2."""
    gas = disc.gas
    u = disc.project(taylor_green(gas, disc.dim))
    pinf = 1.0 / (gas.gamma * gas.Ma ** 2)
    sigma = np.ones(disc.nv)
    sigma[-1] = pinf / (gas.gamma - 1.0) + 0.5
    return u + noise_amp * sigma[None, :, None] * noise
