// Host-side metrics of isoparametric curved elements (arxiv 2002.04222,
// Sec. 3.1: the element integrals are taken on the reference element with
// the Jacobian of its map and the face Jacobian).
//
// Element map x(xi) = sum_c X_c l_c(xi), tensor-product Lagrange polynomials
// of order g through equispaced nodes xi_i = -1 + 2 i / g, node index
// c = i0 + (g+1)(i1 + (g+1) i2).  At every Gauss point the library stores
//   vg[e][c][q], c < D*D: G[k][j] = d xi_k / d x_j at c = k*D + j,
//                c = D*D:  w_q |J_q|
//   fg[e][f][c][p], c < D*D: G at face point p of face f (the element's map),
//                   D*D <= c < D*D+D: outward unit normal,
//                   c = D*D+D: w^G_p |J^G_p|
// with the normal and area element from Nanson's relation
// n dA = |J| (d xi_a / d x) dxi_t on face f = 2a + side (+ for side 1).
// Face points: tangential axes in increasing order, the first fastest.
#pragma once
#include <algorithm>
#include <cmath>
#include <string>
#include <thread>
#include <vector>

namespace dgj_geo {

// 1D Lagrange basis through n equispaced nodes on [-1, 1] at x: l[i], dl[i]
inline void lagrange_eq(int g, double x, double* l, double* dl) {
  const int n = g + 1;
  double nodes[8];
  for (int i = 0; i < n; ++i) nodes[i] = -1.0 + 2.0 * i / g;
  for (int i = 0; i < n; ++i) {
    double v = 1.0, d = 0.0;
    for (int m = 0; m < n; ++m) {
      if (m == i) continue;
      const double inv = 1.0 / (nodes[i] - nodes[m]);
      // product rule: d(v * (x - x_m) inv) = d (x - x_m) inv + v inv
      d = d * (x - nodes[m]) * inv + v * inv;
      v = v * (x - nodes[m]) * inv;
    }
    l[i] = v;
    dl[i] = d;
  }
}

struct Curved {
  std::vector<double> vg, fg, vol, area;   // area[e][f]
};

// Jm[j][k] = d x_j / d xi_k at the point whose per-axis 1D tables are
// (lv[a], ld[a]); nodes X[c][j] of one element.
inline void map_jacobian(int D, int g, const double* X, const double* const* lv, const double* const* ld,
                         double Jm[3][3]) {
  const int n = g + 1;
  const int nn = D == 3 ? n * n * n : n * n;
  for (int j = 0; j < D; ++j)
    for (int k = 0; k < D; ++k) Jm[j][k] = 0.0;
  for (int c = 0; c < nn; ++c) {
    int mi[3] = {c % n, (c / n) % n, c / (n * n)};
    for (int k = 0; k < D; ++k) {
      double w = 1.0;
      for (int a = 0; a < D; ++a) w *= (a == k) ? ld[a][mi[a]] : lv[a][mi[a]];
      for (int j = 0; j < D; ++j) Jm[j][k] += w * X[c * D + j];
    }
  }
}

// G = Jm^-1 (G[k][j] = d xi_k / d x_j), returns det Jm
inline double invert_small(int D, const double Jm[3][3], double G[3][3]) {
  if (D == 2) {
    const double det = Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0];
    G[0][0] = Jm[1][1] / det;
    G[0][1] = -Jm[0][1] / det;
    G[1][0] = -Jm[1][0] / det;
    G[1][1] = Jm[0][0] / det;
    return det;
  }
  double C[3][3];   // cofactors
  for (int r = 0; r < 3; ++r)
    for (int s = 0; s < 3; ++s) {
      const int r1 = (r + 1) % 3, r2 = (r + 2) % 3, s1 = (s + 1) % 3, s2 = (s + 2) % 3;
      C[r][s] = Jm[r1][s1] * Jm[r2][s2] - Jm[r1][s2] * Jm[r2][s1];
    }
  const double det = Jm[0][0] * C[0][0] + Jm[0][1] * C[0][1] + Jm[0][2] * C[0][2];
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) G[k][j] = C[j][k] / det;
  return det;
}

// Metrics of all elements; xg, wg: the Q Gauss nodes and weights.  Returns
// an empty string, or the reason the map is not valid.
inline std::string curved_metrics(int D, int g, int Q, long E, const double* nodes, const std::vector<double>& xg,
                                  const std::vector<double>& wg, Curved& out) {
  if (g < 1 || g > 7) return "geo_order must be in 1..7";
  const int n = g + 1;
  const int nn = D == 3 ? n * n * n : n * n;
  const int NQ = D == 3 ? Q * Q * Q : Q * Q, NQF = D == 3 ? Q * Q : Q, NF = 2 * D;
  const int CV = D * D + 1, CF = D * D + D + 1;
  // 1D tables at the Gauss points and at -1, +1 (indices Q, Q+1)
  std::vector<double> lv((Q + 2) * n), ld((Q + 2) * n);
  for (int i = 0; i < Q + 2; ++i) {
    const double x = i < Q ? xg[i] : (i == Q ? -1.0 : 1.0);
    lagrange_eq(g, x, &lv[i * n], &ld[i * n]);
  }
  out.vg.assign((size_t)E * CV * NQ, 0.0);
  out.fg.assign((size_t)E * NF * CF * NQF, 0.0);
  out.vol.assign(E, 0.0);
  out.area.assign((size_t)E * NF, 0.0);
  std::vector<long> bad;
  const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<long> bad_t(nt, -1);
  auto work = [&](unsigned t) {
    for (long e = t; e < E; e += nt) {
      const double* X = nodes + (size_t)e * nn * D;
      const double* pv[3];
      const double* pd[3];
      double vol = 0.0;
      for (int q = 0; q < NQ; ++q) {
        int aq[3] = {q % Q, (q / Q) % Q, q / (Q * Q)};
        double w = 1.0;
        for (int a = 0; a < D; ++a) {
          pv[a] = &lv[aq[a] * n];
          pd[a] = &ld[aq[a] * n];
          w *= wg[aq[a]];
        }
        double Jm[3][3], G[3][3];
        map_jacobian(D, g, X, pv, pd, Jm);
        const double det = invert_small(D, Jm, G);
        if (!(det > 0.0)) { bad_t[t] = e; return; }
        double* o = out.vg.data() + (size_t)e * CV * NQ;
        for (int k = 0; k < D; ++k)
          for (int j = 0; j < D; ++j) o[(k * D + j) * NQ + q] = G[k][j];
        o[D * D * NQ + q] = w * det;
        vol += w * det;
      }
      out.vol[e] = vol;
      for (int f = 0; f < NF; ++f) {
        const int ax = f >> 1, s = f & 1;
        int tax[2] = {0, 0}, k2 = 0;
        for (int x = 0; x < D; ++x)
          if (x != ax) tax[k2++] = x;
        double area = 0.0;
        for (int p = 0; p < NQF; ++p) {
          int idx[3] = {0, 0, 0};
          idx[ax] = Q + s;
          idx[tax[0]] = p % Q;
          double w = wg[p % Q];
          if (D == 3) { idx[tax[1]] = p / Q; w *= wg[p / Q]; }
          for (int a = 0; a < D; ++a) { pv[a] = &lv[idx[a] * n]; pd[a] = &ld[idx[a] * n]; }
          double Jm[3][3], G[3][3];
          map_jacobian(D, g, X, pv, pd, Jm);
          const double det = invert_small(D, Jm, G);
          if (!(det > 0.0)) { bad_t[t] = e; return; }
          double gn = 0.0;
          for (int j = 0; j < D; ++j) gn += G[ax][j] * G[ax][j];
          gn = std::sqrt(gn);
          double* o = out.fg.data() + ((size_t)e * NF + f) * CF * NQF;
          for (int k = 0; k < D; ++k)
            for (int j = 0; j < D; ++j) o[(k * D + j) * NQF + p] = G[k][j];
          const double sg = s == 1 ? 1.0 : -1.0;
          for (int j = 0; j < D; ++j) o[(D * D + j) * NQF + p] = sg * G[ax][j] / gn;
          o[(D * D + D) * NQF + p] = w * det * gn;
          area += w * det * gn;
        }
        out.area[(size_t)e * NF + f] = area;
      }
    }
  };
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t) th.emplace_back(work, t);
  for (auto& x : th) x.join();
  for (long b : bad_t)
    if (b >= 0) return "element " + std::to_string(b) + ": map with non-positive Jacobian";
  return "";
}

}  // namespace dgj_geo
