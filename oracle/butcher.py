"""Butcher tableaus of Appendix A (SDIRK2, SDIRK3, ERK2).

SDIRK3: the printed 10-digit lambda = 0.4358665215 is the rounded root of
lambda^3 - 3 lambda^2 + 3/2 lambda - 1/6 = 0 that makes the three-stage
tableau third order; the exact root is used here so that the order
conditions hold to rounding.
"""
from __future__ import annotations

import numpy as np


def sdirk3_lambda() -> float:
    roots = np.roots([1.0, -3.0, 1.5, -1.0 / 6.0])
    r = [x.real for x in roots if abs(x.imag) < 1e-12 and 0.4 < x.real < 0.5][0]
    # one Newton polish in float64
    for _ in range(3):
        f = ((r - 3.0) * r + 1.5) * r - 1.0 / 6.0
        df = (3.0 * r - 6.0) * r + 1.5
        r -= f / df
    return float(r)


def tableau(name: str):
    """(A, b, c) of the named scheme."""
    name = name.lower()
    if name == "sdirk2":
        lam = 1.0 - np.sqrt(2.0) / 2.0
        A = np.array([[lam, 0.0], [1.0 - lam, lam]])
    elif name == "sdirk3":
        lam = sdirk3_lambda()
        A = np.array([[lam, 0.0, 0.0],
                      [(1.0 - lam) / 2.0, lam, 0.0],
                      [(-6 * lam ** 2 + 16 * lam - 1) / 4.0, (6 * lam ** 2 - 20 * lam + 5) / 4.0, lam]])
    elif name == "erk2":
        A = np.array([[0.0, 0.0], [1.0, 0.0]])
        return A, np.array([0.5, 0.5]), A.sum(axis=1)
    else:
        raise ValueError(name)
    return A, A[-1].copy(), A.sum(axis=1)
