"""Compressible Navier-Stokes fluxes (Sec. 2, Eq. 1-6) and face fluxes.

States have shape [..., nv] with nv = d + 2 conserved variables
(rho, rho u_1..rho u_d, E); gradients have shape [..., d, nv] with the
derivative direction first; flux tensors have shape [..., d, nv] with the
flux direction first.  Every function accepts complex arrays so that
complex-step derivatives can be taken (|x| is then x*sign(Re x)).

Readings of the paper used here:
  * the stress tensor of Sec. 2 carries the Kronecker delta on its
    2/3 mu div(u) term (Stokes hypothesis; the symbol is missing in print);
  * E is the total energy per unit volume, E = p/(gamma-1) + rho|u|^2/2;
  * Sutherland's law needs a reference temperature in kelvin, which the
    paper does not give: visc_law=1 uses Gas.T_ref_K (default 288.15 K);
    visc_law=0 (default) uses the constant mu = 1/Re;
  * the Riemann solver is not named for the test cases: Roe's flux without
    entropy fix is the default, local Lax-Friedrichs the alternative.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class Gas:
    gamma: float = 1.4
    Pr: float = 0.72
    Re: float = 100.0
    Ma: float = 0.1
    visc_law: int = 0       # 0 constant, 1 Sutherland
    T_ref_K: float = 288.15
    flux_mode: int = 0      # 0 Navier-Stokes, 1 Euler, 2 scalar diffusion test
    riemann: int = 0        # 0 Roe, 1 local Lax-Friedrichs, 2 HLL, 3 HLLC, 4 AUSM+


def cabs(x):
    """|x| that keeps the complex-step derivative: x * sign(Re x)."""
    if np.iscomplexobj(x):
        return x * np.sign(x.real)
    return np.abs(x)


def primitives(gas: Gas, U):
    d = U.shape[-1] - 2
    rho = U[..., 0]
    vel = U[..., 1:1 + d] / rho[..., None]
    E = U[..., d + 1]
    p = (gas.gamma - 1.0) * (E - 0.5 * rho * np.sum(vel * vel, axis=-1))
    return rho, vel, E, p


def temperature(gas: Gas, U):
    """Equation of state p = rho T / (gamma Ma^2)."""
    rho, vel, E, p = primitives(gas, U)
    return gas.gamma * gas.Ma ** 2 * p / rho


def viscosity(gas: Gas, U):
    if gas.visc_law == 0:
        return np.full(U.shape[:-1], 1.0 / gas.Re, dtype=U.dtype)
    T = temperature(gas, U)
    s = 110.0 / gas.T_ref_K
    return T ** 1.5 / gas.Re * (1.0 + s) / (T + s)


def euler_flux(gas: Gas, U):
    """F_i of Eq. 2, returned as F[..., i, v]."""
    d = U.shape[-1] - 2
    F = np.zeros(U.shape[:-1] + (d, d + 2), dtype=U.dtype)
    if gas.flux_mode == 2:
        return F
    rho, vel, E, p = primitives(gas, U)
    for i in range(d):
        F[..., i, 0] = rho * vel[..., i]
        for c in range(d):
            F[..., i, 1 + c] = rho * vel[..., i] * vel[..., c] + (p if c == i else 0.0)
        F[..., i, d + 1] = vel[..., i] * (E + p)
    return F


def viscous_flux(gas: Gas, U, gradU):
    """G_i of Eq. 2 from the conserved state and its gradient, returned as
    G[..., i, v].  Velocity and temperature gradients follow from the chain
    rule; G is linear in gradU for a fixed U (Eq. 11)."""
    d = U.shape[-1] - 2
    G = np.zeros(U.shape[:-1] + (d, d + 2), dtype=np.result_type(U, gradU))
    if gas.flux_mode == 1:
        return G
    if gas.flux_mode == 2:
        return gradU / gas.Re + 0.0 * G
    rho, vel, E, p = primitives(gas, U)
    mu = viscosity(gas, U)
    grho = gradU[..., :, 0]                     # [..., j]
    gvel = (gradU[..., :, 1:1 + d] - vel[..., None, :] * grho[..., :, None]) / rho[..., None, None]
    # gvel[..., j, c] = d u_c / d x_j
    div = sum(gvel[..., c, c] for c in range(d))
    gE = gradU[..., :, d + 1]
    # d(e)/dx_j with e = E/rho - |u|^2/2 ; T = gamma Ma^2 (gamma-1) e
    ge = (gE - (E / rho)[..., None] * grho) / rho[..., None] \
        - np.sum(vel[..., None, :] * gvel, axis=-1)
    # -q_j = mu/(Ma^2 Pr (gamma-1)) dT/dx_j = mu gamma / Pr * de/dx_j
    kappa = mu * gas.gamma / gas.Pr
    for i in range(d):
        for c in range(d):
            tau = mu * (gvel[..., c, i] + gvel[..., i, c])
            if c == i:
                tau = tau - (2.0 / 3.0) * mu * div
            G[..., i, 1 + c] = tau
        G[..., i, d + 1] = sum(vel[..., c] * G[..., i, 1 + c] for c in range(d)) + kappa * ge[..., i]
    return G


def normal_flux(Fdir, n):
    """n . F for F[..., i, v] and n[..., i]."""
    return np.einsum('...iv,...i->...v', Fdir, n)


def roe_flux(gas: Gas, UL, UR, n):
    """Roe's approximate Riemann flux F^n(UL, UR, n), n the unit normal
    pointing from L to R, without entropy fix."""
    d = UL.shape[-1] - 2
    g = gas.gamma
    rL, vL, EL, pL = primitives(gas, UL)
    rR, vR, ER, pR = primitives(gas, UR)
    HL = (EL + pL) / rL
    HR = (ER + pR) / rR
    sL, sR = np.sqrt(rL), np.sqrt(rR)
    rt = sL * sR
    vt = (sL[..., None] * vL + sR[..., None] * vR) / (sL + sR)[..., None]
    Ht = (sL * HL + sR * HR) / (sL + sR)
    q2 = np.sum(vt * vt, axis=-1)
    c2 = (g - 1.0) * (Ht - 0.5 * q2)
    ct = np.sqrt(c2)
    unt = np.sum(vt * n, axis=-1)
    dr = rR - rL
    dp = pR - pL
    dv = vR - vL
    dun = np.sum(dv * n, axis=-1)
    a1 = (dp - rt * ct * dun) / (2.0 * c2)
    a5 = (dp + rt * ct * dun) / (2.0 * c2)
    a2 = dr - dp / c2
    l1, l2, l5 = cabs(unt - ct), cabs(unt), cabs(unt + ct)
    diss = np.zeros(UL.shape, dtype=np.result_type(UL, UR))
    # acoustic waves
    for lam, a, sgn in ((l1, a1, -1.0), (l5, a5, 1.0)):
        coef = lam * a
        diss[..., 0] += coef
        diss[..., 1:1 + d] += coef[..., None] * (vt + sgn * ct[..., None] * n)
        diss[..., d + 1] += coef * (Ht + sgn * unt * ct)
    # entropy and shear waves (eigenvalue u.n)
    shear = dv - dun[..., None] * n
    diss[..., 0] += l2 * a2
    diss[..., 1:1 + d] += l2[..., None] * (a2[..., None] * vt + rt[..., None] * shear)
    diss[..., d + 1] += l2 * (a2 * 0.5 * q2 + rt * (np.sum(vt * dv, axis=-1) - unt * dun))
    FL = normal_flux(euler_flux(gas, UL), n)
    FR = normal_flux(euler_flux(gas, UR), n)
    return 0.5 * (FL + FR) - 0.5 * diss


def llf_flux(gas: Gas, UL, UR, n):
    rL, vL, EL, pL = primitives(gas, UL)
    rR, vR, ER, pR = primitives(gas, UR)
    cL = np.sqrt(gas.gamma * pL / rL)
    cR = np.sqrt(gas.gamma * pR / rR)
    lL = cabs(np.sum(vL * n, axis=-1)) + cL
    lR = cabs(np.sum(vR * n, axis=-1)) + cR
    if np.iscomplexobj(lL) or np.iscomplexobj(lR):
        lam = np.where(lL.real >= lR.real, lL, lR)
    else:
        lam = np.maximum(lL, lR)
    FL = normal_flux(euler_flux(gas, UL), n)
    FR = normal_flux(euler_flux(gas, UR), n)
    return 0.5 * (FL + FR) - 0.5 * lam[..., None] * (UR - UL)


def _normal_state(gas, U, n):
    r, v, E, p = primitives(gas, U)
    un = np.sum(v * n, axis=-1)
    c = np.sqrt(gas.gamma * p / r)
    return r, v, E, p, un, c


def _wave_speeds(gas, UL, UR, n):
    """Signal speeds S_L, S_R of the HLL family: the smaller (larger) of the
    left (right) acoustic speed u_n -+ c and the Roe-average one (Einfeldt's
    estimate)."""
    rL, vL, EL, pL, uL, cL = _normal_state(gas, UL, n)
    rR, vR, ER, pR, uR, cR = _normal_state(gas, UR, n)
    sL, sR = np.sqrt(rL), np.sqrt(rR)
    vt = (sL[..., None] * vL + sR[..., None] * vR) / (sL + sR)[..., None]
    Ht = (sL * (EL + pL) / rL + sR * (ER + pR) / rR) / (sL + sR)
    ct = np.sqrt((gas.gamma - 1.0) * (Ht - 0.5 * np.sum(vt * vt, axis=-1)))
    ut = np.sum(vt * n, axis=-1)
    return np.minimum(uL - cL, ut - ct), np.maximum(uR + cR, ut + ct)


def hll_flux(gas: Gas, UL, UR, n):
    """HLL flux (Harten, Lax and van Leer): one intermediate state between
    the signal speeds S_L, S_R; upwind when both have one sign."""
    SL, SR = _wave_speeds(gas, UL, UR, n)
    FL = normal_flux(euler_flux(gas, UL), n)
    FR = normal_flux(euler_flux(gas, UR), n)
    mid = (SR[..., None] * FL - SL[..., None] * FR + (SL * SR)[..., None] * (UR - UL)) / (SR - SL)[..., None]
    return np.where((SL >= 0.0)[..., None], FL, np.where((SR <= 0.0)[..., None], FR, mid))


def hllc_flux(gas: Gas, UL, UR, n):
    """HLLC flux (Toro, Spruce and Speares): HLL with the contact wave
    restored; the two star states share the contact speed S* and the
    pressure, and keep their side's tangential velocity."""
    SL, SR = _wave_speeds(gas, UL, UR, n)
    rL, vL, EL, pL, uL, _ = _normal_state(gas, UL, n)
    rR, vR, ER, pR, uR, _ = _normal_state(gas, UR, n)
    mL, mR = rL * (SL - uL), rR * (SR - uR)
    Ss = (pR - pL + mL * uL - mR * uR) / (mL - mR)

    def star(r, v, E, p, u, S, m):
        f = m / (S - Ss)
        Us = np.empty(np.broadcast_shapes(v.shape[:-1] + (v.shape[-1] + 2,)), dtype=np.result_type(r, v))
        Us[..., 0] = f
        Us[..., 1:-1] = f[..., None] * (v + (Ss - u)[..., None] * n)
        Us[..., -1] = f * (E / r + (Ss - u) * (Ss + p / m))
        return Us
    FL = normal_flux(euler_flux(gas, UL), n)
    FR = normal_flux(euler_flux(gas, UR), n)
    FsL = FL + SL[..., None] * (star(rL, vL, EL, pL, uL, SL, mL) - UL)
    FsR = FR + SR[..., None] * (star(rR, vR, ER, pR, uR, SR, mR) - UR)
    out = np.where((Ss >= 0.0)[..., None], FsL, FsR)
    out = np.where((SL >= 0.0)[..., None], FL, out)
    return np.where((SR <= 0.0)[..., None], FR, out)


AUSM_BETA, AUSM_ALPHA = 1.0 / 8.0, 3.0 / 16.0


def ausmp_flux(gas: Gas, UL, UR, n):
    """AUSM+ flux (Liou): the interface Mach number and pressure from the
    polynomial splittings M+-(M), P+-(M) of both sides (beta = 1/8,
    alpha = 3/16), the convected quantities (rho, rho u, rho H) taken
    upwind of the interface mass flux, and the interface sound speed the
    mean of the two sides' (read here; Liou's critical-speed variant is one
    of several)."""
    rL, vL, EL, pL, uL, cL = _normal_state(gas, UL, n)
    rR, vR, ER, pR, uR, cR = _normal_state(gas, UR, n)
    a = 0.5 * (cL + cR)
    ML, MR = uL / a, uR / a

    def split(M, sgn):
        big = np.abs(M) >= 1.0
        Mb = 0.5 * (M + sgn * np.abs(M))
        Pb = 0.5 * (1.0 + sgn * np.sign(M))
        q = M * M - 1.0
        Ms = sgn * 0.25 * (M + sgn) ** 2 + sgn * AUSM_BETA * q * q
        Ps = 0.25 * (M + sgn) ** 2 * (2.0 - sgn * M) + sgn * AUSM_ALPHA * M * q * q
        return np.where(big, Mb, Ms), np.where(big, Pb, Ps)
    MpL, PpL = split(ML, 1.0)
    MmR, PmR = split(MR, -1.0)
    m = MpL + MmR
    p = PpL * pL + PmR * pR

    def phi(r, v, E, pp):
        return np.concatenate([r[..., None], (r[..., None] * v), (E + pp)[..., None]], axis=-1)
    mp, mm = 0.5 * (m + np.abs(m)), 0.5 * (m - np.abs(m))
    F = a[..., None] * (mp[..., None] * phi(rL, vL, EL, pL) + mm[..., None] * phi(rR, vR, ER, pR))
    F[..., 1:-1] = F[..., 1:-1] + p[..., None] * n
    return F


RIEMANN = {0: "roe", 1: "llf", 2: "hll", 3: "hllc", 4: "ausm+"}


def riemann_flux(gas: Gas, UL, UR, n):
    """The Riemann flux chosen by gas.riemann: 0 Roe, 1 local
    Lax-Friedrichs, 2 HLL, 3 HLLC, 4 AUSM+ (the paper's solver offers these
    among others, Sec. 4.3)."""
    if gas.flux_mode == 2:
        return np.zeros(np.broadcast_shapes(UL.shape, UR.shape), dtype=np.result_type(UL, UR))
    fn = {0: roe_flux, 1: llf_flux, 2: hll_flux, 3: hllc_flux, 4: ausmp_flux}[gas.riemann]
    return fn(gas, UL, UR, n)


def ip_face_fluxes(gas: Gas, Uo, Un, go, gn, n, beta_p):
    """Interior-penalty face fluxes seen from the side 'o' (own), with n the
    outward normal of that side, Uo/Un the own/neighbour traces and go/gn
    their broken gradients ([..., d, nv]).

    Returns (Ghat_n, S) with
      Ghat_n = n . G(Ubar, {grad U}) - beta_p n . G(Ubar, dU (x) n)
      S[..., j, v] = 1/2 n . G(Ubar, dU (x) e_j)
    where Ubar = (Uo+Un)/2 and dU = Uo - Un.  This is Eq. 12 read with the
    penalty term dissipative (the printed '+' makes the operator
    anti-dissipative) and with the average of the test-function gradient
    carrying its 1/2, the form for which beta_s = 1 gives a symmetric,
    adjoint-consistent operator (the property Eq. 12 is stated to have);
    the symmetric term then enters the residual with a plus sign.
    """
    d = Uo.shape[-1] - 2
    Ubar = 0.5 * (Uo + Un)
    dU = Uo - Un
    gavg = 0.5 * (go + gn)
    Gn = normal_flux(viscous_flux(gas, Ubar, gavg), n)
    jump = n[..., :, None] * dU[..., None, :]           # [..., i, v] = dU_v n_i
    Gn = Gn - beta_p[..., None] * normal_flux(viscous_flux(gas, Ubar, jump), n)
    S = np.zeros(Uo.shape[:-1] + (d, d + 2), dtype=np.result_type(Uo, Un, go, gn))
    for j in range(d):
        e = np.zeros(Uo.shape[:-1] + (d, d + 2), dtype=S.dtype)
        e[..., j, :] = dU
        S[..., j, :] = 0.5 * normal_flux(viscous_flux(gas, Ubar, e), n)
    return Gn, S


def face_flux_own(gas: Gas, Uo, Un, go, gn, n, beta_p):
    """Total numerical normal flux H^n = F^n - G^n seen from the own side
    (outward normal n), and the symmetric flux S."""
    F = riemann_flux(gas, Uo, Un, n)
    Gn, S = ip_face_fluxes(gas, Uo, Un, go, gn, n, beta_p)
    return F - Gn, S


# ---------------------------------------------------------------- boundary ghost states
# The paper names its boundary conditions (Sec. 4.3) but gives no formulas.
# Readings: a boundary face takes the interior trace Q- and a ghost state Q+
# with the interior gradient, and the interior-face fluxes are applied.
# Dirichlet ("time dependent Dirichlet" in its list; the manufactured
# Poiseuille case applies the exact solution weakly): the ghost state is a
# given state at every face point.
BC_FARFIELD, BC_WALL, BC_DIRICHLET = 0, 1, 2
# The other kinds of its list, with readings that keep the number of
# conditions equal to the number of incoming characteristics:
#  slip wall / symmetry plane: the normal momentum mirrored; no heat flux
#    and no tangential viscous traction through the face;
#  isothermal no-slip wall: the velocity negated, the pressure kept and the
#    ghost temperature the interior's mirrored about the wall temperature
#    (that of the given state), so that their mean is the wall temperature
#    and a fluid at rest sees a stationary contact (no mass flux) -- the
#    viscous penalty then drives the wall temperature weakly;
#  zero-order extrapolation: the ghost is the interior state;
#  pressure outflow: the interior state with the given pressure where the
#    outflow is subsonic (the interior state where supersonic);
#  pressure inflow: the given density and velocity with the interior
#    pressure where the inflow is subsonic (the given state where supersonic).
BC_SLIP, BC_ISOTHERMAL, BC_EXTRAPOLATE, BC_PRESSURE_OUT, BC_PRESSURE_IN = 3, 4, 5, 6, 7


FARFIELD_BLEND = 0.02   # half-width of the inflow/outflow blend in u_nb, relative to c_b


def farfield_ghost(gas: Gas, U, n, Uinf):
    """Riemann-invariant far field: with u_n the outward normal velocity and
    c the sound speed, R+ = u_n + 2c/(gamma-1) from the interior, R- = u_n -
    2c/(gamma-1) from the freestream (for |u_n| < c); u_nb = (R+ + R-)/2,
    c_b = (gamma-1)(R+ - R-)/4; tangential velocity and entropy p/rho^gamma
    taken from the interior on outflow (u_nb > 0) and from the freestream on
    inflow, blended by w = (1 + tanh(u_nb / (0.02 c_b)))/2 so that the ghost
    state is differentiable where u_nb changes sign (w is 0 or 1 to double
    precision once |u_nb| > c_b).  Supersonic: all from the freestream
    (inflow, checked first) or the interior (outflow)."""
    g = gas.gamma
    Uinf = np.broadcast_to(Uinf, U.shape)
    ri, vi, Ei, pi = primitives(gas, U)
    ro, vo, Eo, po = primitives(gas, Uinf)
    ci, co = np.sqrt(g * pi / ri), np.sqrt(g * po / ro)
    uni = np.sum(vi * n, axis=-1)
    uno = np.sum(vo * n, axis=-1)
    Rp = uni + 2.0 * ci / (g - 1.0)
    Rm = uno - 2.0 * co / (g - 1.0)
    unb = 0.5 * (Rp + Rm)
    cb = 0.25 * (g - 1.0) * (Rp - Rm)
    w = 0.5 * (1.0 + np.tanh(unb / (FARFIELD_BLEND * cb)))
    s_i, s_o = pi / ri ** g, po / ro ** g
    s = w * s_i + (1.0 - w) * s_o
    vt = w[..., None] * (vi - uni[..., None] * n) + (1.0 - w)[..., None] * (vo - uno[..., None] * n)
    rb = (cb * cb / (g * s)) ** (1.0 / (g - 1.0))
    pb = rb * cb * cb / g
    vb = vt + unb[..., None] * n
    Ub = np.concatenate([rb[..., None], rb[..., None] * vb,
                         (pb / (g - 1.0) + 0.5 * rb * np.sum(vb * vb, axis=-1))[..., None]], axis=-1)
    sup_out = np.real(uni) >= np.real(ci)
    sup_in = np.real(uno) <= -np.real(co)
    Ub = np.where(sup_out[..., None], U, Ub)
    Ub = np.where(sup_in[..., None], Uinf, Ub)
    return Ub


def wall_ghost(U):
    """No-slip wall: the momentum mirrored, density and energy kept, so the
    face average has zero velocity and the interior temperature."""
    G = U.copy()
    G[..., 1:-1] = -U[..., 1:-1]
    return G


def ghost_state(gas: Gas, kind, U, n, Ub):
    """Ghost state of the kinds other than far field and Dirichlet (see the
    readings above); Ub is the boundary id's given state."""
    g = gas.gamma
    G = U.copy()
    r, v, E, p = primitives(gas, U)
    ke = 0.5 * r * np.sum(v * v, axis=-1)
    if kind == BC_WALL:
        return wall_ghost(U)
    if kind == BC_SLIP:
        mn = np.sum(U[..., 1:-1] * n, axis=-1)
        G[..., 1:-1] = U[..., 1:-1] - 2.0 * mn[..., None] * n
        return G
    if kind == BC_ISOTHERMAL:
        rb, vb, Eb, pb = primitives(gas, np.broadcast_to(Ub, U.shape))
        Tw, T = pb / rb, p / r                              # temperatures up to the same factor
        rg = r * T / (2.0 * Tw - T)                         # same pressure, mirrored temperature
        G[..., 0] = rg
        G[..., 1:-1] = -rg[..., None] * v
        G[..., -1] = p / (g - 1.0) + 0.5 * rg * np.sum(v * v, axis=-1)
        return G
    if kind == BC_EXTRAPOLATE:
        return G
    if kind == BC_PRESSURE_OUT:
        _, _, _, pb = primitives(gas, np.broadcast_to(Ub, U.shape))
        c = np.sqrt(g * p / r)
        sub = np.real(np.sum(v * n, axis=-1)) < np.real(c)
        G[..., -1] = np.where(sub, pb / (g - 1.0) + ke, E)
        return G
    if kind == BC_PRESSURE_IN:
        Ubb = np.broadcast_to(Ub, U.shape)
        rb, vb, Eb, pb = primitives(gas, Ubb)
        cb = np.sqrt(g * pb / rb)
        sup = np.real(np.sum(vb * n, axis=-1)) <= -np.real(cb)
        G = np.array(Ubb, dtype=np.result_type(U, Ubb))
        G[..., -1] = np.where(sup, Eb, p / (g - 1.0) + 0.5 * rb * np.sum(vb * vb, axis=-1))
        return G
    raise ValueError(f"unknown boundary kind {kind}")


def boundary_flux_own(gas: Gas, kind, Uo, go, n, beta_p, Uinf=None):
    """Boundary face flux (H^n, S) seen from the interior with outward normal
    n: ghost state per kind (Dirichlet: Uinf holds the ghost state of every
    point; far field, isothermal wall and the pressure kinds read their
    given state from Uinf), ghost gradient = interior gradient; at slip and
    no-slip adiabatic walls no heat flux crosses, at a slip wall no
    tangential traction either; at an
    adiabatic wall the heat flux through the wall is zero, so the energy
    components of the viscous face fluxes vanish (the work term vanishes with
    the zero wall velocity)."""
    Un = boundary_ghost(gas, kind, Uo, n, Uinf)
    F = riemann_flux(gas, Uo, Un, n)
    Gn, S = ip_face_fluxes(gas, Uo, Un, go, go, n, beta_p)
    Gn, S = wall_viscous_limits(kind, Gn, S, n)
    return F - Gn, S


def boundary_ghost(gas: Gas, kind, Uo, n, Uinf):
    """The ghost state of any boundary kind."""
    if kind == BC_DIRICHLET:
        return np.broadcast_to(Uinf, Uo.shape)
    if kind == BC_FARFIELD:
        return farfield_ghost(gas, Uo, n, Uinf)
    return ghost_state(gas, kind, Uo, n, Uinf)


def wall_viscous_limits(kind, Gn, S, n):
    """No heat flux (nor work) through slip and no-slip adiabatic walls; at a
    slip wall only the normal viscous traction remains."""
    if kind in (BC_WALL, BC_SLIP):
        Gn = Gn.copy()
        Gn[..., -1] = 0.0
        if S is not None:
            S = S.copy()
            S[..., -1] = 0.0
    if kind == BC_SLIP:
        gm = np.sum(Gn[..., 1:-1] * n, axis=-1)
        Gn[..., 1:-1] = gm[..., None] * n
        if S is not None:
            sm = np.einsum('...jc,...c->...j', S[..., 1:-1], n)
            S[..., 1:-1] = sm[..., None] * n[..., None, :]
    return Gn, S


# ---------------------------------------------------------------- LDG viscous fluxes
# Local discontinuous Galerkin (Sec. 4.3 lists it beside IP; the paper gives
# no formulas).  Reading: the auxiliary gradient is q = grad u + r, with the
# lifting r of the face jumps defined by M r_j = sum over faces of the
# integral of phi (u_hat - u^-) n_j; the switch takes u_hat from the face's
# left element (the one that meets it with side 1) and the viscous flux's
# gradient q_hat from the right one; a penalty beta_p n.G(u_hat, [u] (x) n)
# on the jump; no symmetric term.  On a boundary face u_hat is the mean of
# the interior and ghost states, q_hat the interior q.


def ldg_viscous_flux_n(gas: Gas, Uhat, qhat, jump, n, beta_p):
    """n.G(u_hat, q_hat) - beta_p n.G(u_hat, jump (x) n) with jump = u^- - u^+
    seen from the side whose outward normal is n."""
    Gn = normal_flux(viscous_flux(gas, Uhat, qhat), n)
    J = n[..., :, None] * jump[..., None, :]
    return Gn - beta_p[..., None] * normal_flux(viscous_flux(gas, Uhat, J), n)


def boundary_flux_own_ldg(gas: Gas, kind, Uo, qo, n, beta_p, Uinf=None):
    """LDG boundary face flux H^n seen from the interior (no symmetric term)."""
    Un = boundary_ghost(gas, kind, Uo, n, Uinf)
    F = riemann_flux(gas, Uo, Un, n)
    Gn = ldg_viscous_flux_n(gas, 0.5 * (Uo + Un), qo, Uo - Un, n, beta_p)
    Gn, _ = wall_viscous_limits(kind, Gn, None, n)
    return F - Gn
