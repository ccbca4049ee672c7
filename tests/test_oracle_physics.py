"""Pins of the oracle's pointwise physics (Sec. 2, Eq. 1-6) against closed
forms: the manufactured Poiseuille forcing the paper prints (Appendix B)
and exact rates of change for special states derived by hand from the
governing equations."""
import numpy as np
import pytest

from oracle.physics import Gas, roe_flux, llf_flux, normal_flux, euler_flux
from tests.oracle_util import conserved_with_gradient, flux_divergence


def poiseuille(gas, L=1.0, theta=0.01):
    mu = 1.0 / gas.Re
    dpdx = -8.0 * mu / L ** 2

    def field(x):
        X, Y = x[..., 0], x[..., 1]
        s = Y * (L - Y)
        ds = L - 2 * Y
        u = -(1 / (2 * mu)) * dpdx * (s + theta * s ** 2)
        du = -(1 / (2 * mu)) * dpdx * (ds + 2 * theta * s * ds)
        rho = 1.0 + 0 * X
        grho = np.zeros(X.shape + (2,), dtype=x.dtype)
        vel = np.stack([u, 0 * u], -1)
        gvel = np.zeros(X.shape + (2, 2), dtype=x.dtype)
        gvel[..., 1, 0] = du
        p = 1.0 / (gas.gamma * gas.Ma ** 2) + dpdx * X
        gp = np.stack([dpdx + 0 * X, 0 * X], -1)
        return conserved_with_gradient(gas.gamma, rho, grho, vel, gvel, p, gp)

    def forcing(x):
        # Appendix B.  f4 carries the factor (1 + theta y (L - y)) in its
        # first term, which the printed expression lacks; with it the forcing
        # follows from the printed exact solution (checked by hand).
        g = gas.gamma
        Y = x[..., 1]
        c = L ** 2 - 6 * Y * L + 6 * Y ** 2
        f2 = dpdx * theta * c
        f4 = (1 / (2 * mu)) * dpdx ** 2 * Y * (L - Y) * (1 + theta * Y * (L - Y)) * (1 - theta * c - g / (g - 1)) \
            - (1 / (4 * mu)) * dpdx ** 2 * (L - 2 * Y) ** 2 * (2 * theta * Y * L - 2 * theta * Y ** 2 + 1) ** 2
        return np.stack([0 * Y, f2, 0 * Y, f4], -1)
    return field, forcing


def test_poiseuille_forcing_matches_appendix_b():
    gas = Gas(Re=100.0, Ma=0.1)
    field, forcing = poiseuille(gas)
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, size=(200, 2))
    div = flux_divergence(gas, field, x)
    f = forcing(x)
    scale = np.abs(f).max(axis=0) + 1e-300
    assert np.abs(div - f).max() <= 1e-9 * np.abs(f).max()
    # the momentum forcing alone is small; check it separately
    assert np.abs(div[:, 1] - f[:, 1]).max() <= 1e-9 * scale[1]


def _mu_closed_form(gas, T):
    """Viscosity and dmu/dT written out by hand: constant 1/Re, or
    Sutherland's law mu = (1/Re) T^(3/2) (1 + s) / (T + s), s = 110 K / T_ref
    (nondimensional T = 1 at the reference state, where mu = 1/Re)."""
    if gas.visc_law == 0:
        return 1.0 / gas.Re + 0.0 * T, 0.0 * T
    s = 110.0 / gas.T_ref_K
    mu = T ** 1.5 * (1.0 + s) / (T + s) / gas.Re
    dmu = (1.0 + s) / gas.Re * np.sqrt(T) * (0.5 * T + 1.5 * s) / (T + s) ** 2
    return mu, dmu


def _special(kind, axis, dim, gas, a=0.3, k=2.0):
    p0 = 1.0 / (gas.gamma * gas.Ma ** 2)

    def field(x):
        s = x[..., axis]
        Z = 0 * s
        gz = np.zeros(s.shape + (dim,), dtype=x.dtype)
        vel = np.zeros(s.shape + (dim,), dtype=x.dtype)
        gvel = np.zeros(s.shape + (dim, dim), dtype=x.dtype)
        if kind == "heat":
            T = 1.0 + a * np.sin(k * s)
            dT = a * k * np.cos(k * s)
            rho = gas.gamma * gas.Ma ** 2 * p0 / T
            grho = gz.copy()
            grho[..., axis] = -gas.gamma * gas.Ma ** 2 * p0 * dT / T ** 2
        else:
            rho = 1.0 + Z
            grho = gz.copy()
            comp = axis if kind == "long" else (axis + 1) % dim
            vel[..., comp] = a * np.sin(k * s)
            gvel[..., axis, comp] = a * k * np.cos(k * s)
        return conserved_with_gradient(gas.gamma, rho, grho, vel, gvel, p0 + Z, gz.copy())

    def exact_div(x):
        # d/dx_j H_j derived by hand from Eq. 1-6 for each special state
        s = x[..., axis]
        mu = 1.0 / gas.Re
        out = np.zeros(s.shape + (dim + 2,))
        if kind == "heat":
            # -(kappa(T) T')' = -(kappa' T'^2 + kappa T''), kappa = mu / (Ma^2 Pr (gamma - 1))
            T = 1.0 + a * np.sin(k * s)
            dT = a * k * np.cos(k * s)
            d2T = -a * k ** 2 * np.sin(k * s)
            mu_T, dmu_T = _mu_closed_form(gas, T)
            c = 1.0 / (gas.Ma ** 2 * gas.Pr * (gas.gamma - 1))
            out[..., dim + 1] = -c * (dmu_T * dT * dT + mu_T * d2T)
        elif kind == "long":
            u = a * np.sin(k * s)
            ux = a * k * np.cos(k * s)
            uxx = -a * k ** 2 * np.sin(k * s)
            g = gas.gamma
            out[..., 0] = ux
            out[..., 1 + axis] = 2 * u * ux - (4.0 / 3.0) * mu * uxx
            out[..., dim + 1] = ux * g * p0 / (g - 1) + 1.5 * u * u * ux - (4.0 / 3.0) * mu * (ux * ux + u * uxx)
        else:  # shear: v = a sin(k x)
            comp = (axis + 1) % dim
            v = a * np.sin(k * s)
            vx = a * k * np.cos(k * s)
            vxx = -a * k ** 2 * np.sin(k * s)
            out[..., 1 + comp] = -mu * vxx
            out[..., dim + 1] = -mu * (vx * vx + v * vxx)
        return out
    return field, exact_div


@pytest.mark.parametrize("visc_law", [0, 1])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("kind", ["heat", "long", "shear"])
def test_special_state_rates(kind, dim, visc_law):
    """Sutherland's law (visc_law 1) is pinned by the heat-conduction state,
    whose temperature varies (kappa(T) differentiated by hand), and by the
    two velocity states at T = 1, where it must reduce to mu = 1/Re."""
    gas = Gas(Re=7.0, Ma=0.3, Pr=0.72, visc_law=visc_law)
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 3, size=(50, dim))
    for axis in range(dim):
        field, exact = _special(kind, axis, dim, gas)
        div = flux_divergence(gas, field, x)
        ex = exact(x)
        assert np.abs(div - ex).max() <= 1e-9 * (np.abs(ex).max() + 1.0), (kind, axis)


@pytest.mark.parametrize("flux", [roe_flux, llf_flux])
def test_riemann_consistency_and_conservation(flux):
    gas = Gas(Ma=0.3)
    rng = np.random.default_rng(2)
    for d in (2, 3):
        U = np.concatenate([rng.uniform(0.8, 1.2, (20, 1)), rng.uniform(-0.5, 0.5, (20, d)),
                            rng.uniform(25, 30, (20, 1))], -1)
        V = U * (1 + 0.05 * rng.uniform(-1, 1, U.shape))
        n = rng.normal(size=(20, d))
        n /= np.linalg.norm(n, axis=-1, keepdims=True)
        # consistency F(U, U, n) = F(U).n
        assert np.allclose(flux(gas, U, U, n), normal_flux(euler_flux(gas, U), n), rtol=1e-13, atol=1e-12)
        # conservation F(U, V, n) = -F(V, U, -n)
        assert np.allclose(flux(gas, U, V, n), -flux(gas, V, U, -n), rtol=1e-12, atol=1e-11)


def test_roe_resolves_isolated_contact():
    """Roe's flux is exact for a stationary contact discontinuity (only the
    density jumps, u.n = 0 and p equal): the flux is then pure pressure."""
    gas = Gas(Ma=0.3)
    d = 2
    p = 10.0
    UL = np.array([1.0, 0.0, 0.0, p / 0.4])
    UR = np.array([2.0, 0.0, 0.0, p / 0.4])
    n = np.array([1.0, 0.0])
    F = roe_flux(gas, UL, UR, n)
    assert np.allclose(F, [0.0, p, 0.0, 0.0], atol=1e-13)
