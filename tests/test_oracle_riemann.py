"""Pins of the oracle's Riemann fluxes (Roe, local Lax-Friedrichs, HLL,
HLLC, AUSM+; the paper's solver offers these among others, Sec. 4.3)
against properties their definitions fix: consistency with the physical
flux, conservation (the flux seen from the other side is the negative),
pure upwinding of supersonic states, and exact resolution of stationary
and moving contact discontinuities by the solvers that keep the contact
wave (Roe, HLLC, AUSM+) but not by the two-wave ones (HLL, LLF)."""
import numpy as np
import pytest

from oracle.physics import Gas, euler_flux, normal_flux, riemann_flux

KINDS = {"roe": 0, "llf": 1, "hll": 2, "hllc": 3, "ausm+": 4}


def _states(rng, dim, k, mach=0.5):
    rho = rng.uniform(0.5, 2.0, size=k)
    p = rng.uniform(0.5, 2.0, size=k)
    c = np.sqrt(1.4 * p / rho)
    vel = rng.uniform(-1, 1, size=(k, dim)) * (mach * c)[:, None]
    E = p / 0.4 + 0.5 * rho * np.sum(vel * vel, -1)
    return np.concatenate([rho[:, None], rho[:, None] * vel, E[:, None]], -1)


def _normals(rng, dim, k):
    n = rng.normal(size=(k, dim))
    return n / np.linalg.norm(n, axis=-1, keepdims=True)


@pytest.mark.parametrize("kind", list(KINDS))
@pytest.mark.parametrize("dim", [2, 3])
def test_consistency_and_conservation(kind, dim):
    gas = Gas(riemann=KINDS[kind])
    rng = np.random.default_rng(1)
    U, V = _states(rng, dim, 50, 1.5), _states(rng, dim, 50, 1.5)
    n = _normals(rng, dim, 50)
    F = riemann_flux(gas, U, U, n)
    exact = normal_flux(euler_flux(gas, U), n)
    assert np.abs(F - exact).max() <= 1e-13 * np.abs(exact).max()
    A = riemann_flux(gas, U, V, n)
    B = riemann_flux(gas, V, U, -n)
    assert np.abs(A + B).max() <= 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("kind", ["roe", "hll", "hllc", "ausm+"])
def test_supersonic_states_are_upwinded(kind):
    gas = Gas(riemann=KINDS[kind])
    rng = np.random.default_rng(2)
    n = _normals(rng, 3, 40)
    U, V = _states(rng, 3, 40, 0.2), _states(rng, 3, 40, 0.2)
    for W_ in (U, V):                      # both sides move along n at Mach 2 .. 3
        r = W_[:, 0]
        p = 0.4 * (W_[:, 4] - 0.5 * np.sum(W_[:, 1:4] ** 2, -1) / r)
        c = np.sqrt(1.4 * p / r)
        vel = W_[:, 1:4] / r[:, None] + (rng.uniform(2.0, 3.0, 40) * c)[:, None] * n
        W_[:, 1:4] = r[:, None] * vel
        W_[:, 4] = p / 0.4 + 0.5 * r * np.sum(vel * vel, -1)
    F = riemann_flux(gas, U, V, n)
    exact = normal_flux(euler_flux(gas, U), n)
    assert np.abs(F - exact).max() <= 1e-12 * np.abs(exact).max()


def _contact(u_n, dim=3, k=20):
    rng = np.random.default_rng(3)
    n = _normals(rng, dim, k)
    p = 1.3
    out = []
    for rho in (rng.uniform(0.5, 1.0, k), rng.uniform(1.5, 3.0, k)):
        t = rng.normal(size=(k, dim))
        t = t - np.sum(t * n, -1, keepdims=True) * n        # tangential velocity differs across the contact
        vel = u_n * n + 0.3 * t
        E = p / 0.4 + 0.5 * rho * np.sum(vel * vel, -1)
        out.append(np.concatenate([rho[:, None], rho[:, None] * vel, E[:, None]], -1))
    return out[0], out[1], n


@pytest.mark.parametrize("kind", list(KINDS))
def test_contact_discontinuities(kind):
    gas = Gas(riemann=KINDS[kind])
    # stationary contact: the exact flux is the pressure alone, but a
    # tangential slip makes it a shear layer too; take zero slip for it
    UL, UR, n = _contact(0.0)
    for U in (UL, UR):
        r = U[:, 0]
        U[:, 4] = 1.3 / 0.4
        U[:, 1:-1] = 0.0
    F = riemann_flux(gas, UL, UR, n)
    pn = np.concatenate([np.zeros((len(n), 1)), 1.3 * n, np.zeros((len(n), 1))], -1)
    err = np.abs(F - pn).max() / 1.3
    if kind in ("roe", "hllc", "ausm+"):
        assert err <= 1e-13
    else:
        assert err > 1e-3                  # two-wave solvers smear the contact
    # moving contact with slip (u_n > 0): the exact flux is the left state's
    UL, UR, n = _contact(0.4)
    F = riemann_flux(gas, UL, UR, n)
    FL = normal_flux(euler_flux(gas, UL), n)
    err = np.abs(F - FL).max() / np.abs(FL).max()
    if kind in ("roe", "hllc", "ausm+"):
        assert err <= 1e-13
    else:
        assert err > 1e-3
