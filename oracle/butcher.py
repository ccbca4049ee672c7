"""Butcher tableaus of Appendix A (ERK2, SDIRK2, SDIRK3, the six-stage
SDIRK4) and backward Euler (Sec. 4.3 lists it among the implicit
integrators).

SDIRK3: the printed 10-digit lambda = 0.4358665215 is the rounded root of
lambda^3 - 3 lambda^2 + 3/2 lambda - 1/6 = 0 that makes the three-stage
tableau third order; the exact root is used here so that the order
conditions hold to rounding.

SDIRK4 (an ESDIRK: explicit first stage, diagonal 1/4, stiffly accurate):
the printed table leaves its first column as symbols and gives the third
abscissa as (2 - sqrt 2)/2.  Read here: the first column repeats the second
(a^{m0} = a^{m1}, as in the Kennedy-Carpenter family it is taken from) and
the abscissae are the row sums, so c_2 = (2 - sqrt 2)/4.  With that reading
all eight fourth-order conditions hold to rounding; with the printed c_2
(and the first column from the row sums) the second-order condition is
already off by 5.7e-2.
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
    elif name == "sdirk4":
        r2 = np.sqrt(2.0)
        A = np.zeros((6, 6))
        for m in range(1, 6):
            A[m, m] = 0.25
        A[2, 1] = (1.0 - r2) / 8.0
        A[3, 1] = (5.0 - 7.0 * r2) / 64.0
        A[3, 2] = 7.0 * (1.0 + r2) / 32.0
        A[4, 1] = (-13796.0 - 54539.0 * r2) / 125000.0
        A[4, 2] = (506605.0 + 132109.0 * r2) / 437500.0
        A[4, 3] = 166.0 * (-97.0 + 376.0 * r2) / 109375.0
        A[5, 1] = (1181.0 - 987.0 * r2) / 13782.0
        A[5, 2] = 47.0 * (-267.0 + 1783.0 * r2) / 273343.0
        A[5, 3] = -16.0 * (-22922.0 + 3525.0 * r2) / 571953.0
        A[5, 4] = -15625.0 * (97.0 + 376.0 * r2) / 90749876.0
        A[1:, 0] = A[1:, 1]
    elif name == "beuler":
        A = np.array([[1.0]])
    elif name == "erk2":
        A = np.array([[0.0, 0.0], [1.0, 0.0]])
        return A, np.array([0.5, 0.5]), A.sum(axis=1)
    else:
        raise ValueError(name)
    return A, A[-1].copy(), A.sum(axis=1)
