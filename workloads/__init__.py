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
    elem_origin: np.ndarray   # [n_elem, dim] float64, lower corner
    elem_h: np.ndarray        # [n_elem, dim] float64, edge lengths
    face_nbr: np.ndarray      # [n_elem, 2*dim] int32

    @property
    def n_elem(self) -> int:
        return int(self.elem_h.shape[0])


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
    riemann: int = 0          # 0 Roe, 1 local Lax-Friedrichs
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
    pc_precision: str = "f64"

    @property
    def nv(self) -> int:
        return self.dim + 2

    @property
    def n_modes(self) -> int:
        return (self.P + 1) ** self.dim

    def mesh(self) -> Mesh:
        return cartesian_mesh(self.ncells, self.lengths, periodic=True)

    def dofs(self) -> int:
        """Degrees of freedom per variable, N_e (P+1)^d."""
        return int(np.prod(self.ncells)) * self.n_modes

    def dt(self, umax: float = 1.0) -> float:
        """Time step from the standard CFL number (c_lambda = 0.2,
        d_RK = 2) with the freestream estimate c + |u| = 1/Ma + umax and
        dx the element edge."""
        dx = min(self.lengths[a] / self.ncells[a] for a in range(self.dim))
        lam = 1.0 / self.Ma + umax
        return self.cfl * 2.0 * dx / (0.2 * lam * self.P ** 2)


def config(i: int, **overrides) -> FlowConfig:
    """Workloads: 1 = 2D 8x8 P=2 Taylor-Green (Re 100, Ma 0.1, SDIRK2);
    2 = 3D 16^3 P=3 Taylor-Green (Re 1600, Ma 0.1, SDIRK3);
    3 = workload 2 with a reduced-precision preconditioner."""
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
