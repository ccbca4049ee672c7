// Device kernels of the DG residual and the block-relaxed-Jacobi
// preconditioner, templated on dimension D, modes per direction N = P+1 and
// Gauss points per direction Q.
//
// Layouts (element-major, coalesced per element):
//   state   u[e][v][m], m = i0 + N*(i1 + N*i2), v over (rho, rho u.., E)
//   geo     geo[e][GEO]: dxi_0..dxi_{D-1} (= 2/h_j), detJ, 1/detJ, fdet_0..fdet_{D-1}
//           (face Jacobian |J^Gamma| of the faces normal to axis a)
//   nbr     nbr[e][2D]: element across face f = 2a+s (it meets it with face 2a+1-s)
//   beta    beta[e][2D]: interior-penalty beta_p of that face
//   tables  B[Q][N] = phi_n(xi_q), Dq[Q][N] = phi_n'(xi_q), w[Q],
//           phiE[2][N] = phi_n(-1), phi_n(+1), dphiE[2][N] the derivatives.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include "dgj_physics.h"

namespace dgj {

constexpr __host__ __device__ int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

template <int D, int N, int Q>
struct Shape {
  static constexpr int NV = D + 2;
  static constexpr int NM = ipow(N, D);
  static constexpr int NQ = ipow(Q, D);
  static constexpr int NQF = ipow(Q, D - 1);
  static constexpr int NMF = ipow(N, D - 1);
  static constexpr int NF = 2 * D;
  static constexpr int GEO = 2 * D + 2;
  static constexpr int NB = NV * NM;
  static constexpr int TAB = 2 * Q * N + Q + 4 * N;
};

struct Tab {
  const double* B;
  const double* Dq;
  const double* w;
  const double* phiE;
  const double* dphiE;
};

template <int N, int Q>
__device__ __forceinline__ Tab load_tables(const double* __restrict__ g, double* s) {
  constexpr int T = 2 * Q * N + Q + 4 * N;
  for (int i = threadIdx.x; i < T; i += blockDim.x) s[i] = g[i];
  Tab t;
  t.B = s;
  t.Dq = s + Q * N;
  t.w = s + 2 * Q * N;
  t.phiE = s + 2 * Q * N + Q;
  t.dphiE = s + 2 * Q * N + Q + 2 * N;
  return t;
}

// tangential axes of the face normal to axis a
template <int D>
__device__ __forceinline__ void tang_axes(int a, int* t) {
  int k = 0;
  for (int x = 0; x < D; ++x)
    if (x != a) t[k++] = x;
}

// multi-index helpers
template <int D, int N>
__device__ __forceinline__ void split(int m, int* i) {
#pragma unroll
  for (int k = 0; k < D; ++k) { i[k] = m % N; m /= N; }
}

// mode index from the normal index in axis a and the tangential face-mode index tm
template <int D, int N>
__device__ __forceinline__ int mode_of(int a, int ia, int tm) {
  int idx[3] = {0, 0, 0};
  int t[2];
  tang_axes<D>(a, t);
  idx[a] = ia;
  int r = tm;
  for (int k = 0; k < D - 1; ++k) { idx[t[k]] = r % N; r /= N; }
  int m = 0;
  for (int k = D - 1; k >= 0; --k) m = m * N + idx[k];
  return m;
}

// ---------------------------------------------------------------- state access
struct StateIn {
  const double* u;    // base state
  const double* v;    // perturbation direction (matvec) or nullptr
  double eps;
  __device__ __forceinline__ double operator()(long i) const {
    if (v == nullptr) return u[i];
    // u + eps v rounded as two separate operations (no contraction)
    return __dadd_rn(u[i], __dmul_rn(eps, v[i]));
  }
};

enum ResMode { RES_R = 0, RES_N = 1, RES_JV = 2 };

struct ResArgs {
  StateIn in;
  const double* S;     // stage source (modes N, JV)
  const double* Nu;    // stored N(u) (mode JV)
  double dt_a;
  double* out;
  int mode;
  const int* nbr;
  const double* geo;
  const double* beta;
  const double* tables;
  Phys ph;
  long n_elem;
};

// ---------------------------------------------------------------- residual kernel
// One workgroup per element.  Volume: sum-factorised backward transform and
// reference gradients at the Q^D Gauss points, pointwise H_j = F_j - G_j
// scaled by w |J| dxi_j, transposed sum-factorised inner product with the
// derivative bases.  Faces: each element evaluates both traces of each of
// its faces, the numerical flux in the face's canonical orientation (left =
// the element with side 1, normal +e_a) and uses +/- of it, so both sides of
// a face see bitwise identical fluxes; then lifts -phi H + grad phi . S.
template <int D, int N, int Q>
struct ResidualLDS {
  using S = Shape<D, N, Q>;
  static constexpr int TABSZ = S::TAB;
  // volume phase
  static constexpr int V_T1 = (D == 3) ? 2 * S::NV * Q * N * N : 2 * S::NV * Q * N;
  static constexpr int V_T2 = (D == 3) ? 3 * S::NV * Q * Q * N : 0;
  static constexpr int V_QG = (D + 1) * S::NV * S::NQ;
  static constexpr int VOL = V_T1 + V_T2 + V_QG;
  // face phase (one face at a time)
  static constexpr int F_TV = 2 * 2 * S::NV * S::NMF;
  static constexpr int F_TR = 2 * (D + 1) * S::NV * S::NQF;
  static constexpr int F_X = (D + 1) * S::NV * S::NQF;
  static constexpr int FACE = F_TV + F_TR + F_X;
  static constexpr int WORK = VOL > FACE ? VOL : FACE;
  static constexpr int TOTAL = TABSZ + S::NB /*sU*/ + S::NB /*sL*/ + WORK;
};

// Sum-factorised backward transform Q = B u and reference gradients
// d Q / d xi_j at the Q^D Gauss points: sQ[0][v][q] values, sQ[1+j][v][q]
// derivatives.  W is scratch of ResidualLDS::V_T1 + V_T2 doubles.
template <int D, int N, int Q, int NT>
__device__ __forceinline__ void vol_forward(const Tab& tb, const double* sU, double* W, double* sQ) {
  using S = Shape<D, N, Q>;
  using L = ResidualLDS<D, N, Q>;
  constexpr int NV = S::NV, NM = S::NM, NQ = S::NQ;
  const int tid = threadIdx.x;
  if constexpr (D == 2) {
    double* T1 = W;                          // [2][NV][Q][N]
    for (int it = tid; it < NV * Q * N; it += NT) {
      int i1 = it % N, a0 = (it / N) % Q, v = it / (N * Q);
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int i0 = 0; i0 < N; ++i0) {
        double uu = sU[v * NM + i0 + N * i1];
        s0 += tb.B[a0 * N + i0] * uu;
        s1 += tb.Dq[a0 * N + i0] * uu;
      }
      T1[it] = s0;
      T1[NV * Q * N + it] = s1;
    }
    __syncthreads();
    for (int it = tid; it < NV * NQ; it += NT) {
      int q = it % NQ, v = it / NQ;
      int a0 = q % Q, a1 = q / Q;
      double s0 = 0.0, sx = 0.0, sy = 0.0;
#pragma unroll
      for (int i1 = 0; i1 < N; ++i1) {
        double t = T1[(v * Q + a0) * N + i1];
        double td = T1[NV * Q * N + (v * Q + a0) * N + i1];
        s0 += tb.B[a1 * N + i1] * t;
        sx += tb.B[a1 * N + i1] * td;
        sy += tb.Dq[a1 * N + i1] * t;
      }
      sQ[it] = s0;
      sQ[NV * NQ + it] = sx;
      sQ[2 * NV * NQ + it] = sy;
    }
  } else {
    double* T1 = W;                          // [2][NV][Q][N][N]  (a0, i1, i2)
    double* T2 = W + L::V_T1;                // [3][NV][Q][Q][N]  (a0, a1, i2)
    constexpr int n1 = NV * Q * N * N;
    for (int it = tid; it < n1; it += NT) {
      int i2 = it % N, i1 = (it / N) % N, a0 = (it / (N * N)) % Q, v = it / (N * N * Q);
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int i0 = 0; i0 < N; ++i0) {
        double uu = sU[v * NM + i0 + N * (i1 + N * i2)];
        s0 += tb.B[a0 * N + i0] * uu;
        s1 += tb.Dq[a0 * N + i0] * uu;
      }
      T1[it] = s0;
      T1[n1 + it] = s1;
    }
    __syncthreads();
    constexpr int n2 = NV * Q * Q * N;
    for (int it = tid; it < n2; it += NT) {
      int i2 = it % N, a1 = (it / N) % Q, a0 = (it / (N * Q)) % Q, v = it / (N * Q * Q);
      double s0 = 0.0, sx = 0.0, sy = 0.0;
#pragma unroll
      for (int i1 = 0; i1 < N; ++i1) {
        int src = ((v * Q + a0) * N + i1) * N + i2;
        double t = T1[src], td = T1[n1 + src];
        s0 += tb.B[a1 * N + i1] * t;
        sx += tb.B[a1 * N + i1] * td;
        sy += tb.Dq[a1 * N + i1] * t;
      }
      T2[it] = s0;
      T2[n2 + it] = sx;
      T2[2 * n2 + it] = sy;
    }
    __syncthreads();
    for (int it = tid; it < NV * NQ; it += NT) {
      int q = it % NQ, v = it / NQ;
      int a0 = q % Q, a1 = (q / Q) % Q, a2 = q / (Q * Q);
      double s0 = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
      for (int i2 = 0; i2 < N; ++i2) {
        int src = ((v * Q + a0) * Q + a1) * N + i2;
        double b = tb.B[a2 * N + i2], dq = tb.Dq[a2 * N + i2];
        s0 += b * T2[src];
        sx += b * T2[n2 + src];
        sy += b * T2[2 * n2 + src];
        sz += dq * T2[src];
      }
      sQ[it] = s0;
      sQ[NV * NQ + it] = sx;
      sQ[2 * NV * NQ + it] = sy;
      sQ[3 * NV * NQ + it] = sz;
    }
  }
}

template <int D, int N, int Q, int NT>
__global__ __launch_bounds__(NT) void k_residual(ResArgs a) {
  using S = Shape<D, N, Q>;
  using L = ResidualLDS<D, N, Q>;
  constexpr int NV = S::NV, NM = S::NM, NQ = S::NQ, NQF = S::NQF, NMF = S::NMF;
  __shared__ double smem[L::TOTAL];
  const long e = blockIdx.x;
  if (e >= a.n_elem) return;
  Tab tb = load_tables<N, Q>(a.tables, smem);
  double* sU = smem + L::TABSZ;
  double* sL = sU + S::NB;
  double* W = sL + S::NB;
  const int tid = threadIdx.x;
  const double* g = a.geo + e * S::GEO;
  double dxi[D];
#pragma unroll
  for (int j = 0; j < D; ++j) dxi[j] = g[j];
  const double detJ = g[D], invdetJ = g[D + 1];

  for (int i = tid; i < S::NB; i += NT) { sU[i] = a.in(e * S::NB + i); sL[i] = 0.0; }
  __syncthreads();

  // ---------------- volume: backward transform + reference gradients
  double* sQ = W + L::V_T1 + L::V_T2;     // [D+1][NV][NQ]: value, d/dxi_0..
  vol_forward<D, N, Q, NT>(tb, sU, W, sQ);
  __syncthreads();

  // ---------------- pointwise volume flux, scaled by w |J| dxi_j
  for (int q = tid; q < NQ; q += NT) {
    double U[NV], gU[D][NV], F[D][NV], G[D][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      U[v] = sQ[v * NQ + q];
#pragma unroll
      for (int j = 0; j < D; ++j) gU[j][v] = sQ[(1 + j) * NV * NQ + v * NQ + q] * dxi[j];
    }
    euler_flux<D, double>(a.ph, U, F);
    viscous_flux<D, double, double>(a.ph, U, gU, G);
    double wq = detJ;
    {
      int r = q;
#pragma unroll
      for (int k = 0; k < D; ++k) { wq *= tb.w[r % Q]; r /= Q; }
    }
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int v = 0; v < NV; ++v) sQ[(1 + j) * NV * NQ + v * NQ + q] = (F[j][v] - G[j][v]) * (wq * dxi[j]);
  }
  __syncthreads();

  // ---------------- transposed contraction with derivative bases
  const double* Hx = sQ + NV * NQ;
  const double* Hy = sQ + 2 * NV * NQ;
  if constexpr (D == 2) {
    double* U1 = W;   // [2][NV][Q][N] (a0, i1)
    for (int it = tid; it < NV * Q * N; it += NT) {
      int i1 = it % N, a0 = (it / N) % Q, v = it / (N * Q);
      double sx = 0.0, sy = 0.0;
#pragma unroll
      for (int a1 = 0; a1 < Q; ++a1) {
        int q = a0 + Q * a1;
        sx += tb.B[a1 * N + i1] * Hx[v * NQ + q];
        sy += tb.Dq[a1 * N + i1] * Hy[v * NQ + q];
      }
      U1[it] = sx;
      U1[NV * Q * N + it] = sy;
    }
    __syncthreads();
    for (int it = tid; it < NV * NM; it += NT) {
      int m = it % NM, v = it / NM;
      int i0 = m % N, i1 = m / N;
      double s = 0.0;
#pragma unroll
      for (int a0 = 0; a0 < Q; ++a0) {
        int src = (v * Q + a0) * N + i1;
        s += tb.Dq[a0 * N + i0] * U1[src] + tb.B[a0 * N + i0] * U1[NV * Q * N + src];
      }
      sL[it] = s;
    }
  } else {
    const double* Hz = sQ + 3 * NV * NQ;
    double* U1 = W;                      // [3][NV][Q][Q][N] (a0, a1, i2)
    double* U2 = W + 3 * NV * Q * Q * N; // [2][NV][Q][N][N] (a0, i1, i2)
    constexpr int n1 = NV * Q * Q * N;
    for (int it = tid; it < n1; it += NT) {
      int i2 = it % N, a1 = (it / N) % Q, a0 = (it / (N * Q)) % Q, v = it / (N * Q * Q);
      double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
      for (int a2 = 0; a2 < Q; ++a2) {
        int q = a0 + Q * (a1 + Q * a2);
        double b = tb.B[a2 * N + i2];
        sx += b * Hx[v * NQ + q];
        sy += b * Hy[v * NQ + q];
        sz += tb.Dq[a2 * N + i2] * Hz[v * NQ + q];
      }
      U1[it] = sx;
      U1[n1 + it] = sy;
      U1[2 * n1 + it] = sz;
    }
    __syncthreads();
    constexpr int n2 = NV * Q * N * N;
    for (int it = tid; it < n2; it += NT) {
      int i2 = it % N, i1 = (it / N) % N, a0 = (it / (N * N)) % Q, v = it / (N * N * Q);
      double sa = 0.0, sb = 0.0;
#pragma unroll
      for (int a1 = 0; a1 < Q; ++a1) {
        int src = ((v * Q + a0) * Q + a1) * N + i2;
        sa += tb.B[a1 * N + i1] * U1[src];
        sb += tb.Dq[a1 * N + i1] * U1[n1 + src] + tb.B[a1 * N + i1] * U1[2 * n1 + src];
      }
      U2[it] = sa;
      U2[n2 + it] = sb;
    }
    __syncthreads();
    for (int it = tid; it < NV * NM; it += NT) {
      int m = it % NM, v = it / NM;
      int i0 = m % N, i1 = (m / N) % N, i2 = m / (N * N);
      double s = 0.0;
#pragma unroll
      for (int a0 = 0; a0 < Q; ++a0) {
        int src = ((v * Q + a0) * N + i1) * N + i2;
        s += tb.Dq[a0 * N + i0] * U2[src] + tb.B[a0 * N + i0] * U2[n2 + src];
      }
      sL[it] = s;
    }
  }
  __syncthreads();

  // ---------------- faces, one at a time
  double* fTV = W;                        // [side][2 (val, dn)][NV][NMF]
  double* fTR = W + L::F_TV;              // [side][D+1][NV][NQF]  value, physical gradient
  double* fX = fTR + L::F_TR;             // [D+1][NV][NQF]: -w H, w dxi_j S_j
  for (int f = 0; f < S::NF; ++f) {
    const int ax = f >> 1, s = f & 1;
    const long en = a.nbr[e * S::NF + f];
    int tax[2] = {0, 0};
    tang_axes<D>(ax, tax);
    // face-modal contraction along the normal axis, for own (side 0) and neighbour (side 1)
    for (int it = tid; it < 2 * NV * NMF; it += NT) {
      int tm = it % NMF, v = (it / NMF) % NV, side = it / (NMF * NV);
      long X = side == 0 ? e : en;
      int sg = side == 0 ? s : 1 - s;
      double sv = 0.0, sd = 0.0;
#pragma unroll
      for (int ia = 0; ia < N; ++ia) {
        double uu = a.in(X * S::NB + v * NM + mode_of<D, N>(ax, ia, tm));
        sv += tb.phiE[sg * N + ia] * uu;
        sd += tb.dphiE[sg * N + ia] * uu;
      }
      fTV[((side * 2 + 0) * NV + v) * NMF + tm] = sv;
      fTV[((side * 2 + 1) * NV + v) * NMF + tm] = sd;
    }
    __syncthreads();
    // tangential expansion to face points: value and physical gradient
    for (int it = tid; it < 2 * NV * NQF; it += NT) {
      int p = it % NQF, v = (it / NQF) % NV, side = it / (NQF * NV);
      long X = side == 0 ? e : en;
      const double* gX = a.geo + X * S::GEO;
      int b0 = p % Q, b1 = (D == 3) ? p / Q : 0;
      double val = 0.0, dn = 0.0, dt0 = 0.0, dt1 = 0.0;
      for (int tm = 0; tm < NMF; ++tm) {
        int j0 = tm % N, j1 = (D == 3) ? tm / N : 0;
        double B0 = tb.B[b0 * N + j0], D0 = tb.Dq[b0 * N + j0];
        double B1 = (D == 3) ? tb.B[b1 * N + j1] : 1.0;
        double D1 = (D == 3) ? tb.Dq[b1 * N + j1] : 0.0;
        double tv = fTV[((side * 2 + 0) * NV + v) * NMF + tm];
        double td = fTV[((side * 2 + 1) * NV + v) * NMF + tm];
        val += B0 * B1 * tv;
        dn += B0 * B1 * td;
        dt0 += D0 * B1 * tv;
        if (D == 3) dt1 += B0 * D1 * tv;
      }
      double* o = fTR + (side * (D + 1)) * NV * NQF;
      o[v * NQF + p] = val;
      o[(1 + ax) * NV * NQF + v * NQF + p] = dn * gX[ax];
      o[(1 + tax[0]) * NV * NQF + v * NQF + p] = dt0 * gX[tax[0]];
      if (D == 3) o[(1 + tax[1]) * NV * NQF + v * NQF + p] = dt1 * gX[tax[1]];
    }
    __syncthreads();
    // numerical flux at each face point
    for (int p = tid; p < NQF; p += NT) {
      double Uo[NV], Un[NV], go[D][NV], gn[D][NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Uo[v] = fTR[v * NQF + p];
        Un[v] = fTR[(D + 1) * NV * NQF + v * NQF + p];
#pragma unroll
        for (int j = 0; j < D; ++j) {
          go[j][v] = fTR[(1 + j) * NV * NQF + v * NQF + p];
          gn[j][v] = fTR[(D + 1 + 1 + j) * NV * NQF + v * NQF + p];
        }
      }
      double nrm[D];
#pragma unroll
      for (int j = 0; j < D; ++j) nrm[j] = (j == ax) ? 1.0 : 0.0;
      double H[NV], Sf[D][NV];
      const double beta = a.beta[e * S::NF + f];
      if (s == 1) face_flux<D>(a.ph, Uo, Un, go, gn, nrm, beta, H, Sf);
      else face_flux<D>(a.ph, Un, Uo, gn, go, nrm, beta, H, Sf);
      double wf = g[D + 2 + ax];
      {
        int b0 = p % Q, b1 = (D == 3) ? p / Q : 0;
        wf *= tb.w[b0];
        if (D == 3) wf *= tb.w[b1];
      }
      const double sgn = (s == 1) ? 1.0 : -1.0;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        fX[v * NQF + p] = -wf * sgn * H[v];
#pragma unroll
        for (int j = 0; j < D; ++j) fX[(1 + j) * NV * NQF + v * NQF + p] = wf * dxi[j] * Sf[j][v];
      }
    }
    __syncthreads();
    // lift into the own modes
    for (int it = tid; it < NV * NM; it += NT) {
      int m = it % NM, v = it / NM;
      int mi[3] = {0, 0, 0};
      split<D, N>(m, mi);
      int ia = mi[ax];
      int j0 = mi[tax[0]], j1 = (D == 3) ? mi[tax[1]] : 0;
      double acc0 = 0.0, accn = 0.0;
      for (int p = 0; p < NQF; ++p) {
        int b0 = p % Q, b1 = (D == 3) ? p / Q : 0;
        double B0 = tb.B[b0 * N + j0], D0 = tb.Dq[b0 * N + j0];
        double B1 = (D == 3) ? tb.B[b1 * N + j1] : 1.0;
        double D1 = (D == 3) ? tb.Dq[b1 * N + j1] : 0.0;
        double bb = B0 * B1;
        acc0 += bb * fX[v * NQF + p] + D0 * B1 * fX[(1 + tax[0]) * NV * NQF + v * NQF + p];
        if (D == 3) acc0 += B0 * D1 * fX[(1 + tax[1]) * NV * NQF + v * NQF + p];
        accn += bb * fX[(1 + ax) * NV * NQF + v * NQF + p];
      }
      sL[it] += tb.phiE[s * N + ia] * acc0 + tb.dphiE[s * N + ia] * accn;
    }
    __syncthreads();
  }

  // ---------------- epilogue
  for (int i = tid; i < S::NB; i += NT) {
    const long gi = e * S::NB + i;
    double R = sL[i] * invdetJ;
    if (a.mode == RES_R) {
      a.out[gi] = R;
    } else {
      double Nw = (sU[i] - a.S[gi]) - a.dt_a * R;
      if (a.mode == RES_N) a.out[gi] = Nw;
      else a.out[gi] = (Nw - a.Nu[gi]) / a.in.eps;
    }
  }
}

}  // namespace dgj
