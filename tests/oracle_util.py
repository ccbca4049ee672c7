"""Helpers for the oracle pin tests: tiny discretisations and exact
fields given in primitive variables with analytic gradients."""
from __future__ import annotations

import numpy as np

import workloads as W
from oracle.dg import Disc
from oracle.physics import Gas


def tiny_disc(dim=2, cells=(3, 3), P=2, nq=None, lengths=None, **gas):
    nq = P + 2 if nq is None else nq
    if lengths is None:
        lengths = tuple(1.0 + 0.3 * i for i in range(dim))
    mesh = W.cartesian_mesh(cells, lengths)
    return Disc(gas=Gas(**gas), dim=dim, P=P, nq=nq, elem_origin=mesh.elem_origin,
                elem_h=mesh.elem_h, face_nbr=mesh.face_nbr)


def conserved_with_gradient(gamma, rho, grho, vel, gvel, p, gp):
    """U and grad U from primitive fields and their gradients (product rule).
    rho, p: [...]; grho, gp: [..., j]; vel: [..., c]; gvel: [..., j, c]."""
    d = vel.shape[-1]
    E = p / (gamma - 1.0) + 0.5 * rho * np.sum(vel * vel, axis=-1)
    gE = gp / (gamma - 1.0) + 0.5 * np.sum(vel * vel, axis=-1)[..., None] * grho \
        + rho[..., None] * np.einsum('...c,...jc->...j', vel, gvel)
    U = np.concatenate([rho[..., None], rho[..., None] * vel, E[..., None]], axis=-1)
    gU = np.zeros(vel.shape[:-1] + (d, d + 2), dtype=np.result_type(U, gvel))
    gU[..., :, 0] = grho
    gU[..., :, 1:1 + d] = grho[..., :, None] * vel[..., None, :] + rho[..., None, None] * gvel
    gU[..., :, d + 1] = gE
    return U, gU


def flux_divergence(gas, field, x, h=1e-20):
    """sum_j d/dx_j H_j(U(x), grad U(x)) by complex step in x_j, where
    field(x) -> (U, gradU) is complex-analytic."""
    from oracle.physics import euler_flux, viscous_flux
    d = x.shape[-1]
    out = 0.0
    for j in range(d):
        xc = x.astype(np.complex128)
        xc[..., j] += 1j * h
        U, gU = field(xc)
        H = euler_flux(gas, U) - viscous_flux(gas, U, gU)
        out = out + H[..., j, :].imag / h
    return out


def l2_coeff_norm(disc, c):
    """L2 norm of the field with modal coefficients c (orthonormal basis)."""
    return float(np.sqrt(np.sum(disc.detJ[:, None, None] * c ** 2)))
