"""Seeded synthetic workloads: meshes, flow parameters and random numbers.

This module is the only thing the CPU oracle and the device library share,
and it holds none of the discretisation's arithmetic: it produces mesh
connectivity, element sizes, flow and solver parameters, and seeded random
arrays.  Every array is plain data that both sides take as input.

Data layout contract (the same one the C header documents):
  * conserved variables per element, in the order (rho, rho*u_1..rho*u_d, E);
  * modal coefficients of the orthonormal tensor-product Legendre basis on
    the reference element [-1,1]^d, mode index i + n*(j + n*k), x fastest,
    n = P+1.  With that basis a constant field c has mode-0 coefficient
    c * 2**(d/2) and all other coefficients zero.
  * element index e = i + nx*(j + ny*k) on structured grids, x fastest.
  * face f = 2*axis + side, side 0 is the face at xi_axis = -1 and side 1
    the face at xi_axis = +1.  face_nbr[e, f] is the element across that
    face (it meets it with its face 2*axis + (1-side)), or -(bc_id + 1) for
    a boundary face.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclasses.dataclass
class Mesh:
    dim: int
    ncells: tuple
    elem_origin: Optional[np.ndarray]   # [n_elem, dim] float64, lower corner (boxes)
    elem_h: Optional[np.ndarray]        # [n_elem, dim] float64, edge lengths (boxes)
    face_nbr: np.ndarray                # [n_elem, 2*dim] int32
    geo_nodes: Optional[np.ndarray] = None   # [n_elem, (geo_order+1)^dim, dim] (curved)
    geo_order: int = 1

    @property
    def n_elem(self) -> int:
        return int(self.face_nbr.shape[0])


def cartesian_mesh(ncells: Sequence[int], lengths: Sequence[float],
                   periodic: Sequence[bool] | bool = True,
                   origin: Optional[Sequence[float]] = None,
                   bc_ids: Optional[Sequence[int]] = None) -> Mesh:
    """Structured grid of ncells[0] x ncells[1] (x ncells[2]) affine boxes.

    Non-periodic axes get boundary faces with id bc_ids[2*axis+side]
    (default 0)."""
    dim = len(ncells)
    if isinstance(periodic, bool):
        periodic = [periodic] * dim
    if origin is None:
        origin = [0.0] * dim
    if bc_ids is None:
        bc_ids = [0] * (2 * dim)
    nc = [int(c) for c in ncells]
    n_elem = int(np.prod(nc))
    h = np.array([lengths[a] / nc[a] for a in range(dim)], dtype=np.float64)
    idx = np.indices(nc[::-1]).reshape(dim, -1)[::-1].T  # [n_elem, dim], x fastest
    elem_origin = np.asarray(origin, dtype=np.float64)[None, :] + idx * h[None, :]
    elem_h = np.broadcast_to(h, (n_elem, dim)).copy()
    strides = [int(np.prod(nc[:a])) for a in range(dim)]
    face_nbr = np.zeros((n_elem, 2 * dim), dtype=np.int32)
    for a in range(dim):
        for side, step in ((0, -1), (1, +1)):
            j = idx[:, a] + step
            inside = (j >= 0) & (j < nc[a])
            jw = np.mod(j, nc[a])
            nb = np.arange(n_elem) + (jw - idx[:, a]) * strides[a]
            if periodic[a]:
                face_nbr[:, 2 * a + side] = nb
            else:
                face_nbr[:, 2 * a + side] = np.where(inside, nb, -(bc_ids[2 * a + side] + 1))
    return Mesh(dim=dim, ncells=tuple(nc), elem_origin=elem_origin, elem_h=elem_h,
                face_nbr=face_nbr)


def _lattice_elements(ncells, geo_order):
    """Global lattice indices [n_elem, (geo_order+1)^dim, dim] of the
    isoparametric nodes of each element of a structured grid (elements x
    fastest; nodes i0 + (g+1)(i1 + (g+1) i2) at equispaced reference
    positions -1 + 2 i / g)."""
    dim = len(ncells)
    g = geo_order
    eidx = np.indices(ncells[::-1]).reshape(dim, -1)[::-1].T           # [E, dim]
    nidx = np.indices((g + 1,) * dim).reshape(dim, -1)[::-1].T         # [nn, dim], x fastest
    return eidx[:, None, :] * g + nidx[None, :, :]


def curved_box_mesh(ncells: Sequence[int], lengths: Sequence[float], geo_order: int = 2,
                    amp: float = 0.1, seed: int = 7, periodic: Sequence[bool] | bool = True,
                    bc_ids: Optional[Sequence[int]] = None) -> Mesh:
    """Box [0, L]^d split as a structured grid, with curved elements: the
    isoparametric nodes of order geo_order are a Cartesian lattice moved by
    a smooth seeded displacement, periodic over the box,
      d_j(x) = amp h_j sum_{t<3} c_jt sin(2 pi m_t . x / L + phi_jt),
    h_j the cell size, c ~ U(-1/3, 1/3), integer wave numbers m_t in {0, 1, 2}
    (not all zero), phi ~ U(0, 2 pi).  Neighbours share their face nodes."""
    dim = len(ncells)
    nc = [int(c) for c in ncells]
    rng = np.random.Generator(np.random.PCG64(seed))
    h = np.array([lengths[a] / nc[a] for a in range(dim)])
    L = np.asarray(lengths, dtype=np.float64)
    m = rng.integers(0, 3, size=(3, dim))
    m[:, 0] = np.maximum(m[:, 0], 1)
    c = rng.uniform(-1.0 / 3.0, 1.0 / 3.0, size=(dim, 3))
    ph = rng.uniform(0.0, TWO_PI, size=(dim, 3))
    lat = _lattice_elements(nc, geo_order)                                   # [E, nn, dim]
    x0 = lat * (h / geo_order)[None, None, :]
    nodes = x0.copy()
    arg = TWO_PI * np.einsum('td,end->ent', m, x0 / L)                        # [E, nn, 3]
    for j in range(dim):
        nodes[..., j] += amp * h[j] * np.sum(c[j] * np.sin(arg + ph[j]), axis=-1)
    base = cartesian_mesh(nc, lengths, periodic=periodic, bc_ids=bc_ids)
    return Mesh(dim=dim, ncells=tuple(nc), elem_origin=None, elem_h=None, face_nbr=base.face_nbr,
                geo_nodes=nodes, geo_order=geo_order)


def annulus_mesh(nr: int, nth: int, nz: int = 0, r0: float = 0.5, r1: float = 10.0, Lz: float = math.pi,
                 geo_order: int = 2, amp: float = 0.1, seed: int = 4) -> Mesh:
    """O-grid around a cylinder of radius r0 out to r1, extruded over Lz
    (periodic) when nz > 0: axis 0 radial (face side 0 on r = r0: boundary
    id 0; side 1 on r = r1: id 1), axis 1 angular (periodic), axis 2
    spanwise (periodic).  Radial node positions r = r0 (r1/r0)^s, s
    uniform; nodes strictly inside are moved in r and theta by a smooth
    seeded field, amp times the local spacing times sin(pi s) (zero on both
    circles), periodic in theta and z.  Node x = r cos(theta), y = r
    sin(theta), z."""
    dim = 3 if nz > 0 else 2
    nc = [nr, nth] + ([nz] if nz > 0 else [])
    g = geo_order
    rng = np.random.Generator(np.random.PCG64(seed))
    lat = _lattice_elements(nc, g)
    s = lat[..., 0] / (nr * g)
    th = TWO_PI * (lat[..., 1] % (nth * g)) / (nth * g)    # the seam's nodes are theta = 0's
    zz = lat[..., 2] * (Lz / (nz * g)) if dim == 3 else None
    ratio = (r1 / r0) ** (1.0 / (nr * g))
    mth = rng.integers(1, 4, size=3)
    mz = rng.integers(0, 2, size=3)
    cr, ct = rng.uniform(-1.0 / 3.0, 1.0 / 3.0, size=(2, 3))
    pr, pt = rng.uniform(0.0, TWO_PI, size=(2, 3))
    wave_r = np.zeros(s.shape)
    wave_t = np.zeros(s.shape)
    for t in range(3):
        arg = mth[t] * th + (TWO_PI * mz[t] * zz / Lz if dim == 3 else 0.0)
        wave_r += cr[t] * np.sin(arg + pr[t])
        wave_t += ct[t] * np.sin(arg + pt[t])
    bump = np.sin(math.pi * s)
    r = r0 * (r1 / r0) ** s
    r = r + amp * r * (ratio - 1.0) * bump * wave_r
    th = th + amp * (TWO_PI / (nth * g)) * bump * wave_t
    cols = [r * np.cos(th), r * np.sin(th)] + ([zz] if dim == 3 else [])
    nodes = np.stack(cols, axis=-1)
    base = cartesian_mesh(nc, [1.0] * dim, periodic=[False] + [True] * (dim - 1),
                          bc_ids=[0, 1] + [0] * (2 * dim - 2))
    return Mesh(dim=dim, ncells=tuple(nc), elem_origin=None, elem_h=None, face_nbr=base.face_nbr,
                geo_nodes=nodes, geo_order=g)


@dataclasses.dataclass
class FlowConfig:
    """Physical, discretisation and solver parameters of one workload."""
    name: str
    dim: int
    ncells: tuple
    lengths: tuple
    P: int
    nq: int
    Re: float
    Ma: float
    gamma: float = 1.4
    Pr: float = 0.72
    flux_mode: int = 0        # 0 Navier-Stokes, 1 Euler, 2 scalar-diffusion test
    riemann: int = 0          # 0 Roe, 1 LLF, 2 HLL, 3 HLLC, 4 AUSM+
    viscous: str = "ip"       # viscous face terms: "ip" (interior penalty) or "ldg"
    visc_law: int = 0         # 0 constant mu = 1/Re, 1 Sutherland
    T_ref_K: float = 288.15
    scheme: str = "sdirk2"
    cfl: float = 20.0
    ic: str = "tgv"
    noise_amp: float = 1e-3
    seed: int = 1
    newton_rtol: float = 1e-8
    newton_max: int = 30
    gmres_restart: int = 30
    gmres_rtol: float = 5e-2
    gmres_max: int = 300
    brj_sweeps: int = 7
    brj_omega: float = 1.0
    pc_freeze: int = 10
    pc_refresh_its: int = 30
    ortho: str = "mgs"        # GMRES orthogonalisation: "mgs" or "cgs2"
    pc_precision: str = "f64"
    geometry: str = "box"     # "box" (periodic affine boxes), "annulus" (curved O-grid, walls + far
                              # field) or "channel" (affine boxes, Dirichlet on every side)
    r0: float = 0.5
    r1: float = 10.0

    @property
    def nv(self) -> int:
        return self.dim + 2

    @property
    def n_modes(self) -> int:
        return (self.P + 1) ** self.dim

    def mesh(self) -> Mesh:
        if self.geometry == "annulus":
            return annulus_mesh(self.ncells[0], self.ncells[1], self.ncells[2] if self.dim == 3 else 0,
                                r0=self.r0, r1=self.r1, Lz=self.lengths[-1], seed=self.seed)
        if self.geometry == "channel":
            return cartesian_mesh(self.ncells, self.lengths, periodic=False)
        return cartesian_mesh(self.ncells, self.lengths, periodic=True)

    def freestream(self) -> np.ndarray:
        """Freestream in conserved variables: rho = 1, velocity (1, 0, ..),
        p = 1/(gamma Ma^2), so E = p/(gamma-1) + 1/2."""
        p = 1.0 / (self.gamma * self.Ma ** 2)
        return np.array([1.0, 1.0] + [0.0] * (self.dim - 1) + [p / (self.gamma - 1.0) + 0.5])

    def boundary(self):
        """(bc_kind, bc_state) of the boundary ids: annulus id 0 = no-slip
        adiabatic wall on the cylinder, id 1 = far field; channel: id 0 =
        Dirichlet on all four sides; none on periodic boxes."""
        if self.geometry == "channel":
            # one id, Dirichlet (ghost states per face point from mms_inputs)
            return np.array([2], dtype=np.int32), self.freestream()[None]
        if self.geometry != "annulus":
            return None, None
        U = self.freestream()
        return np.array([1, 0], dtype=np.int32), np.stack([U, U])

    def dofs(self) -> int:
        """Degrees of freedom per variable, N_e (P+1)^d."""
        return int(np.prod(self.ncells)) * self.n_modes

    def dt(self, umax: float = 1.0) -> float:
        """Time step from the standard CFL number (c_lambda = 0.2,
        d_RK = 2) with the freestream estimate c + |u| = 1/Ma + umax and
        dx the element edge."""
        if self.geometry == "annulus":
            dx = self.r0 * ((self.r1 / self.r0) ** (1.0 / self.ncells[0]) - 1.0)   # first radial cell
        else:
            dx = min(self.lengths[a] / self.ncells[a] for a in range(self.dim))
        lam = 1.0 / self.Ma + umax
        return self.cfl * 2.0 * dx / (0.2 * lam * self.P ** 2)


def config(i: int, **overrides) -> FlowConfig:
    """Workloads: 1 = 2D 8x8 P=2 Taylor-Green (Re 100, Ma 0.1, SDIRK2);
    2 = 3D 16^3 P=3 Taylor-Green (Re 1600, Ma 0.1, SDIRK3);
    3 = workload 2 with a reduced-precision preconditioner;
    4 = flow past a cylinder: curved O-grid annulus r in [0.5, 10], 32
    radial x 64 angular x 8 spanwise hexes (span pi), P=4, Re 3900, Ma 0.2,
    wall + far field, SDIRK2."""
    if i == 1:
        c = FlowConfig(name="tgv2d-8x8-p2", dim=2, ncells=(8, 8), lengths=(TWO_PI, TWO_PI),
                       P=2, nq=4, Re=100.0, Ma=0.1, scheme="sdirk2", seed=1)
    elif i == 2:
        c = FlowConfig(name="tgv3d-16c-p3", dim=3, ncells=(16, 16, 16),
                       lengths=(TWO_PI, TWO_PI, TWO_PI), P=3, nq=5, Re=1600.0, Ma=0.1,
                       scheme="sdirk3", seed=2)
    elif i == 3:
        c = FlowConfig(name="tgv3d-16c-p3-f32pc", dim=3, ncells=(16, 16, 16),
                       lengths=(TWO_PI, TWO_PI, TWO_PI), P=3, nq=5, Re=1600.0, Ma=0.1,
                       scheme="sdirk3", seed=3, pc_precision="f32")
    elif i == 4:
        c = FlowConfig(name="cylinder-annulus-64x32x8-p4", dim=3, ncells=(32, 64, 8),
                       lengths=(1.0, TWO_PI, math.pi), P=4, nq=6, Re=3900.0, Ma=0.2, scheme="sdirk2", seed=4,
                       geometry="annulus", ic="freestream")
    else:
        raise ValueError(f"unknown workload {i}")
    return dataclasses.replace(c, **overrides)


def batch_configs(n: int = 64, seed: int = 5, nmin: int = 4, nmax: int = 32, pmin: int = 2, pmax: int = 5):
    """Independent 2D periodic Taylor-Green problems on [0, 2 pi]^2:
    N_x, N_y ~ U{nmin..nmax}, P ~ U{pmin..pmax}, Ma ~ U[0.1, 0.5],
    Re ~ logU[100, 2000], SDIRK2 at CFL 20 (seeded)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        nx, ny = (int(x) for x in rng.integers(nmin, nmax + 1, size=2))
        P = int(rng.integers(pmin, pmax + 1))
        Ma = float(rng.uniform(0.1, 0.5))
        Re = float(np.exp(rng.uniform(np.log(100.0), np.log(2000.0))))
        out.append(FlowConfig(name=f"tgv2d-batch{i}", dim=2, ncells=(nx, ny), lengths=(TWO_PI, TWO_PI), P=P,
                              nq=P + 2, Re=Re, Ma=Ma, scheme="sdirk2", seed=seed * 1000 + i))
    return out


def freestream_state(cfg: FlowConfig, n_elem: int, at_rest: bool = False) -> np.ndarray:
    """Uniform freestream (mode-0 coefficient U_inf 2^(d/2)) plus
    cfg.noise_amp * sigma_v * noise(seed) on every coefficient, sigma =
    (1, .., 1, E_inf): an impulsive start.  at_rest: the fluid starts at
    rest (rho = 1, p = p_inf) and the far field sets it moving."""
    U = cfg.freestream()
    if at_rest:
        U = U.copy()
        U[1:1 + cfg.dim] = 0.0
        U[-1] -= 0.5
    shape = (n_elem, cfg.dim + 2, (cfg.P + 1) ** cfg.dim)
    u = np.zeros(shape)
    u[:, :, 0] = U * 2.0 ** (cfg.dim / 2.0)
    sigma = np.ones(cfg.dim + 2)
    sigma[-1] = U[-1]
    return u + cfg.noise_amp * sigma[None, :, None] * noise(shape, cfg.seed)


def noise(shape, seed: int) -> np.ndarray:
    """Seeded uniform(-1, 1) array (PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, size=shape)


DEFAULT_MEAN = {2: (1.0, 0.3, -0.2, 20.0), 3: (1.0, 0.3, -0.2, 0.1, 20.0)}


def random_state(n_elem: int, dim: int, P: int, seed: int,
                 mean: Optional[Sequence[float]] = None,
                 amp: float = 0.05, decay: float = 0.5) -> np.ndarray:
    """Smooth-ish random modal state u[e, v, m] around a constant
    conserved state `mean` (density and pressure stay positive for the
    default amplitude).  Coefficient of total degree s gets a uniform
    random perturbation of size amp*|mean_v|*decay**s (plus element-to-
    element jumps on mode 0), so the field is discontinuous across
    elements, as DG states are."""
    nv = dim + 2
    n = P + 1
    if mean is None:
        mean = DEFAULT_MEAN[dim]
    mean = np.asarray(mean, dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(seed))
    nm = n ** dim
    deg = np.zeros(nm)
    for m in range(nm):
        r, s = m, 0
        for _ in range(dim):
            s += r % n
            r //= n
        deg[m] = s
    scale = amp * np.abs(mean)[None, :, None] * (decay ** deg)[None, None, :]
    scale[:, :, 0] *= 2.0 ** (dim / 2.0)
    u = rng.uniform(-1.0, 1.0, size=(n_elem, nv, nm)) * scale
    u[:, :, 0] += mean[None, :] * 2.0 ** (dim / 2.0)
    return u


def random_vector(n_elem: int, dim: int, P: int, seed: int) -> np.ndarray:
    """Seeded uniform(-1,1) vector in the state layout, for matvec tests."""
    nv = dim + 2
    return noise((n_elem, nv, (P + 1) ** dim), seed)


def mlp_init(n_in: int, hidden: int, n_out: int, seed: int, out_scale: float = 1e-2) -> np.ndarray:
    """Seeded initial MLP parameters, packed W1[n_in][H], b1[H], W2[H][H],
    b2[H], W3[H][n_out], b3[n_out] (FP32): Glorot-uniform weights, zero
    biases, the output layer scaled by out_scale so that the first
    predictions are near zero."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def glorot(a, b):
        lim = np.sqrt(6.0 / (a + b))
        return rng.uniform(-lim, lim, size=(a, b))
    parts = [glorot(n_in, hidden), np.zeros(hidden), glorot(hidden, hidden), np.zeros(hidden),
             glorot(hidden, n_out) * out_scale, np.zeros(n_out)]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


# ---------------------------------------------------------------- manufactured Poiseuille flow
def poiseuille_mms(gamma: float, Ma: float, Re: float, L: float = 1.0, theta: float = 0.01):
    """Manufactured compressible Poiseuille flow of Sec. 6.1 and Appendix B:
    rho = 1, u = -(dp/dx)/(2 mu) [y(L-y) + theta y^2 (L-y)^2], v = 0,
    p = 1/(gamma Ma^2) + (dp/dx) x, mu = 1/Re, dp/dx = -8 mu / L^2; and the
    forcing f that makes it a steady solution (dU/dt + div(F - G) = f).
    f_4 carries the factor (1 + theta y (L - y)) in its first term, which
    the printed expression lacks (with it f follows from the exact
    solution).  Returns (exact(x) -> U[..., 4], forcing(x) -> f[..., 4])."""
    mu = 1.0 / Re
    dpdx = -8.0 * mu / L ** 2

    def exact(x):
        X, Y = x[..., 0], x[..., 1]
        s = Y * (L - Y)
        u = -(dpdx / (2.0 * mu)) * (s + theta * s * s)
        p = 1.0 / (gamma * Ma ** 2) + dpdx * X
        E = p / (gamma - 1.0) + 0.5 * u * u
        return np.stack([np.ones_like(X), u, np.zeros_like(X), E], axis=-1)

    def forcing(x):
        Y = x[..., 1]
        c = L ** 2 - 6.0 * Y * L + 6.0 * Y ** 2
        f2 = dpdx * theta * c
        f4 = (dpdx ** 2 / (2.0 * mu)) * Y * (L - Y) * (1.0 + theta * Y * (L - Y)) \
            * (1.0 - theta * c - gamma / (gamma - 1.0)) \
            - (dpdx ** 2 / (4.0 * mu)) * (L - 2.0 * Y) ** 2 * (2.0 * theta * Y * L - 2.0 * theta * Y ** 2 + 1.0) ** 2
        return np.stack([np.zeros_like(Y), f2, np.zeros_like(Y), f4], axis=-1)

    return exact, forcing


def mms_config(P: int, n: int, **overrides) -> FlowConfig:
    """The manufactured Poiseuille case on [0, 1]^2 with n x n elements:
    Re 100, Ma 0.1 (maximum velocity about 1), Dirichlet data from the exact
    solution on every side, backward-Euler pseudo-time steps."""
    c = FlowConfig(name=f"poiseuille-mms-{n}x{n}-p{P}", dim=2, ncells=(n, n), lengths=(1.0, 1.0), P=P, nq=P + 2,
                   Re=100.0, Ma=0.1, scheme="beuler", geometry="channel", ic="mms", cfl=500.0, seed=6)
    return dataclasses.replace(c, **overrides)


def box_points(mesh: Mesh, nq: int):
    """Physical coordinates where inputs given at quadrature points are
    sampled, on affine boxes: volume points [E, nq^d, d] (Gauss-Legendre
    points, x fastest) and face points [E, 2d, nq^(d-1), d] (face f =
    2 axis + side; the tangential axes in increasing order, the first
    fastest)."""
    x1, _ = np.polynomial.legendre.leggauss(nq)
    d = mesh.dim
    org, h = mesh.elem_origin, mesh.elem_h
    idx = np.indices((nq,) * d).reshape(d, -1)[::-1].T          # [nq^d, d], first axis fastest
    xi = x1[idx]
    xv = org[:, None, :] + (xi[None] + 1.0) * 0.5 * h[:, None, :]
    nqf = nq ** (d - 1)
    tid = np.indices((nq,) * (d - 1)).reshape(d - 1, -1)[::-1].T if d > 1 else np.zeros((1, 0), int)
    xf = np.zeros((mesh.face_nbr.shape[0], 2 * d, nqf, d))
    for axis in range(d):
        tang = [a for a in range(d) if a != axis]
        for side in (0, 1):
            ref = np.zeros((nqf, d))
            ref[:, axis] = 1.0 if side else -1.0
            for t, a in enumerate(tang):
                ref[:, a] = x1[tid[:, t]]
            xf[:, 2 * axis + side] = org[:, None, :] + (ref[None] + 1.0) * 0.5 * h[:, None, :]
    return xv, xf


def mms_inputs(cfg: FlowConfig, mesh: Mesh) -> Dict[str, np.ndarray]:
    """Inputs of the manufactured Poiseuille case, sampled at the
    quadrature points: 'bc_field' [E, 2d, nv, nqf] the exact solution at the
    face points (the Dirichlet ghost states); 'forcing', 'exact' and
    'initial' [E, nv, nq^d] at the volume points; the initial state has the
    exact density and pressure and a uniform velocity 1."""
    exact, forcing = poiseuille_mms(cfg.gamma, cfg.Ma, cfg.Re)
    xv, xf = box_points(mesh, cfg.nq)
    U = exact(xv)
    U0 = U.copy()
    U0[..., 1] = 1.0
    U0[..., 2] = 0.0
    p = (U[..., 3] - 0.5 * U[..., 1] ** 2) * (cfg.gamma - 1.0)
    U0[..., 3] = p / (cfg.gamma - 1.0) + 0.5
    return {"bc_field": np.ascontiguousarray(np.transpose(exact(xf), (0, 1, 3, 2))),
            "forcing": np.ascontiguousarray(np.transpose(forcing(xv), (0, 2, 1))),
            "exact": np.ascontiguousarray(np.transpose(U, (0, 2, 1))),
            "initial": np.ascontiguousarray(np.transpose(U0, (0, 2, 1)))}
