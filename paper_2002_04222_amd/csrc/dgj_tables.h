// 1D basis and quadrature tables of the tensor-product DG discretisation
// (Sec. 3.1): the orthonormal Legendre functions phi_n = sqrt((2n+1)/2) P_n
// and their derivatives at the Q Gauss-Legendre points and at xi = -1, +1,
// the Gauss weights, and the Lagrange basis of the Gauss points at xi = -1, +1.
//
// Everything here is constexpr.  kTab<N, Q> is a compile-time constant, so
// the fully unrolled sum-factorised contractions of the residual kernels see
// each table entry as an immediate value (no kernel argument, no register
// held across the kernel); the host copies the very same object into the
// table array the other kernels read, so every kernel uses identical values.
#pragma once

namespace dgj {

// cos by its Taylor series (a Newton starting guess only)
constexpr double tab_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 40; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

// square root by Newton's iteration, which decreases monotonically after the
// first step: stop at the first iterate that does not decrease
constexpr double tab_sqrt(double x) {
  if (x <= 0.0) return 0.0;
  double r = x > 1.0 ? x : 1.0;
  for (int i = 0; i < 2000; ++i) {
    const double nx = 0.5 * (r + x / r);
    if (!(nx < r)) break;
    r = nx;
  }
  return r;
}

constexpr double tab_abs(double x) { return x < 0.0 ? -x : x; }

// Legendre P_k(x) and P_k'(x), k = 0..P, by the three-term recurrence
// k P_k = (2k-1) x P_{k-1} - (k-1) P_{k-2} and P_k' = P_{k-2}' + (2k-1) P_{k-1};
// phi_k = sqrt((2k+1)/2) P_k
template <int N>
constexpr void tab_legendre(double x, double (&v)[N], double (&d)[N]) {
  double p[N] = {}, dp[N] = {};
  p[0] = 1.0;
  if (N > 1) { p[1] = x; dp[1] = 1.0; }
  for (int k = 2; k < N; ++k) {
    p[k] = ((2.0 * k - 1.0) * x * p[k - 1] - (k - 1.0) * p[k - 2]) / k;
    dp[k] = dp[k - 2] + (2.0 * k - 1.0) * p[k - 1];
  }
  for (int k = 0; k < N; ++k) {
    const double c = tab_sqrt((2.0 * k + 1.0) / 2.0);
    v[k] = c * p[k];
    d[k] = c * dp[k];
  }
}

// P_n(z) and P_{n-1}(z)
constexpr void tab_leg_pair(int n, double z, double& pn, double& pm) {
  double p0 = 1.0, p1 = z;
  if (n == 0) { pn = 1.0; pm = 0.0; return; }
  for (int j = 2; j <= n; ++j) {
    const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pm = p0;
}

template <int Q>
struct GaussRule {
  double x[Q];   // ascending nodes on (-1, 1)
  double w[Q];
};

// Gauss-Legendre rule: Newton's iteration on P_Q from the usual cosine guess,
// weights 2 / ((1 - z^2) P_Q'(z)^2)
template <int Q>
constexpr GaussRule<Q> gauss_rule() {
  GaussRule<Q> g{};
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < Q; ++k) {
    double z = tab_cos(pi * (k + 0.75) / (Q + 0.5));
    double pn = 0.0, pm = 0.0, dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      tab_leg_pair(Q, z, pn, pm);
      dp = Q * (z * pn - pm) / (z * z - 1.0);
      const double dz = pn / dp;
      z -= dz;
      if (tab_abs(dz) <= 1e-16) break;
    }
    tab_leg_pair(Q, z, pn, pm);
    dp = Q * (z * pn - pm) / (z * z - 1.0);
    g.x[Q - 1 - k] = z;
    g.w[Q - 1 - k] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  return g;
}

// The residual kernels' tables.  The member order is also the layout of the
// flat table array in device memory that the preconditioner kernels read.
template <int N, int Q>
struct TabK {
  double B[Q][N];      // phi_n(xi_q)
  double Dq[Q][N];     // phi_n'(xi_q)
  double w[Q];
  double phiE[2][N];   // phi_n(-1), phi_n(+1)
  double dphiE[2][N];
  double lag[2][Q];    // Lagrange basis of the Gauss points at xi = -1, +1
};

template <int N, int Q>
constexpr TabK<N, Q> make_tabk() {
  TabK<N, Q> t{};
  const GaussRule<Q> g = gauss_rule<Q>();
  for (int q = 0; q < Q; ++q) {
    double v[N] = {}, d[N] = {};
    tab_legendre<N>(g.x[q], v, d);
    for (int n = 0; n < N; ++n) { t.B[q][n] = v[n]; t.Dq[q][n] = d[n]; }
    t.w[q] = g.w[q];
  }
  for (int s = 0; s < 2; ++s) {
    double v[N] = {}, d[N] = {};
    tab_legendre<N>(s == 0 ? -1.0 : 1.0, v, d);
    for (int n = 0; n < N; ++n) { t.phiE[s][n] = v[n]; t.dphiE[s][n] = d[n]; }
    const double xe = s == 0 ? -1.0 : 1.0;
    for (int a = 0; a < Q; ++a) {
      double l = 1.0;
      for (int b = 0; b < Q; ++b)
        if (b != a) l *= (xe - g.x[b]) / (g.x[a] - g.x[b]);
      t.lag[s][a] = l;
    }
  }
  return t;
}

template <int N, int Q>
inline constexpr TabK<N, Q> kTab = make_tabk<N, Q>();

}  // namespace dgj
