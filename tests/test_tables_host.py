"""The compile-time basis and quadrature tables of the HIP path
(paper_2002_04222_amd/csrc/dgj_tables.h: orthonormal Legendre functions and
their derivatives at the Gauss points and at xi = +-1, Gauss weights, Lagrange
weights of the Gauss points at +-1; the 1D operators of the sum-factorised
residual, Sec. 3.1), compiled on the host with g++ and pinned against closed
forms: Gauss-Legendre nodes are the roots of P_Q and integrate polynomials of
degree 2Q-1 exactly, phi_n = sqrt((2n+1)/2) P_n is orthonormal under the rule,
phi_n(+-1) = sqrt((2n+1)/2) (+-1)^n and phi_n'(+-1) = sqrt((2n+1)/2)
(+-1)^(n+1) n(n+1)/2, and the Lagrange weights reproduce x^k at +-1 for k < Q.
The device kernels use these same constexpr objects (and the host copies them
into the flat table array the other kernels read)."""
import json
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from numpy.polynomial import legendre as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2002_04222_amd", "csrc", "dgj_tables.h")
SHAPES = [(2, 3), (3, 4), (4, 5), (5, 6), (6, 7)]   # (N, Q) of the built shapes: Q = N + 1

PROG = r"""
#include <cstdio>
#include "%s"
template <int N, int Q> void dump(bool last) {
  constexpr dgj::TabK<N, Q> t = dgj::make_tabk<N, Q>();
  constexpr dgj::GaussRule<Q> g = dgj::gauss_rule<Q>();
  const double* p = &t.B[0][0];
  std::printf("{\"N\": %%d, \"Q\": %%d, \"x\": [", N, Q);
  for (int q = 0; q < Q; ++q) std::printf("%%s%%.17g", q ? ", " : "", g.x[q]);
  std::printf("], \"gw\": [");
  for (int q = 0; q < Q; ++q) std::printf("%%s%%.17g", q ? ", " : "", g.w[q]);
  std::printf("], \"tab\": [");
  const int n = (int)(sizeof(t) / sizeof(double));
  for (int i = 0; i < n; ++i) std::printf("%%s%%.17g", i ? ", " : "", p[i]);
  std::printf("]}%%s\n", last ? "" : ",");
}
int main() {
  std::printf("[\n");
  dump<2, 3>(false); dump<3, 4>(false); dump<4, 5>(false); dump<5, 6>(false); dump<6, 7>(true);
  std::printf("]\n");
  return 0;
}
"""


@pytest.fixture(scope="module")
def tables():
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.cpp")
        exe = os.path.join(d, "t")
        with open(src, "w") as f:
            f.write(PROG % HDR)
        subprocess.run([gxx, "-std=c++17", "-O1", "-o", exe, src], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    res = {}
    for rec in json.loads(out):
        N, Q = rec["N"], rec["Q"]
        t = np.array(rec["tab"])
        o = 0
        B = t[o:o + Q * N].reshape(Q, N); o += Q * N
        Dq = t[o:o + Q * N].reshape(Q, N); o += Q * N
        w = t[o:o + Q]; o += Q
        phiE = t[o:o + 2 * N].reshape(2, N); o += 2 * N
        dphiE = t[o:o + 2 * N].reshape(2, N); o += 2 * N
        lag = t[o:o + 2 * Q].reshape(2, Q); o += 2 * Q
        assert o == t.size
        res[(N, Q)] = dict(x=np.array(rec["x"]), gw=np.array(rec["gw"]), B=B, Dq=Dq, w=w, phiE=phiE,
                           dphiE=dphiE, lag=lag)
    return res


def _c(n):
    return np.sqrt((2.0 * n + 1.0) / 2.0)


@pytest.mark.parametrize("N,Q", SHAPES)
def test_gauss_rule(tables, N, Q):
    t = tables[(N, Q)]
    x, w = t["x"], t["w"]
    assert np.array_equal(w, t["gw"])
    assert np.all(np.diff(x) > 0) and -1 < x[0] and x[-1] < 1
    eQ = np.zeros(Q + 1)
    eQ[Q] = 1.0
    assert np.max(np.abs(L.legval(x, eQ))) < 1e-14               # roots of P_Q
    assert np.max(np.abs(x + x[::-1])) < 1e-15                    # symmetric nodes
    for k in range(2 * Q):                                        # exact up to degree 2Q-1
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14


@pytest.mark.parametrize("N,Q", SHAPES)
def test_basis_at_gauss_points(tables, N, Q):
    t = tables[(N, Q)]
    x, w, B, Dq = t["x"], t["w"], t["B"], t["Dq"]
    for n in range(N):
        en = np.zeros(n + 1)
        en[n] = 1.0
        assert np.max(np.abs(B[:, n] - _c(n) * L.legval(x, en))) < 1e-14
        assert np.max(np.abs(Dq[:, n] - _c(n) * L.legval(x, L.legder(en)))) < 1e-13
    # orthonormal under the rule (degree 2N-2 < 2Q)
    G = B.T @ (w[:, None] * B)
    assert np.max(np.abs(G - np.eye(N))) < 1e-14


@pytest.mark.parametrize("N,Q", SHAPES)
def test_end_values_and_lagrange_weights(tables, N, Q):
    t = tables[(N, Q)]
    for n in range(N):
        assert abs(t["phiE"][1][n] - _c(n)) < 1e-15
        assert abs(t["dphiE"][1][n] - _c(n) * n * (n + 1) / 2.0) < 1e-13
        # the parity of P_n holds bitwise: the two faces of an element use exact mirror values
        assert t["phiE"][0][n] == (-1.0) ** n * t["phiE"][1][n]
        assert t["dphiE"][0][n] == (-1.0) ** (n + 1) * t["dphiE"][1][n]
    x, lag = t["x"], t["lag"]
    for s, xe in ((0, -1.0), (1, 1.0)):
        for k in range(Q):
            assert abs(np.dot(lag[s], x ** k) - xe ** k) < 1e-12
