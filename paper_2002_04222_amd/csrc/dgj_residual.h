// DG residual R(u) = M^-1 L(u) of arxiv 2002.04222 (Sec. 3.1, Eq. 13) as
// three kernels:
//   k_res_vol   per element: sum-factorised backward transform and reference
//               gradients at the Gauss points, pointwise H_j = F_j - G_j
//               scaled by w|J| dxi_j, transposed contraction with the
//               derivative bases -> Lvol[e]; and the element's own face
//               traces (value and physical gradient at every face point,
//               by exact Lagrange interpolation from the Gauss points to
//               xi = +-1) -> trace[e][f][c][v][p].
//   k_res_face  one thread per face point, each interior face once, in its
//               canonical orientation (left = the element that meets it
//               with side 1, normal +e_axis): Roe/LLF flux and interior-
//               penalty fluxes -> X[e][axis][k][v][p] = w^G|J^G| (Hhat, Shat_j).
//   k_res_lift  per element: Lvol plus lifting of -phi Hhat_own + grad phi . Shat
//               over the 2D faces, times 1/|J| (M^-1 of the orthonormal basis on
//               affine elements), then the R / N / Jv epilogue.
// Each face flux is computed once, so the element sums of the residual
// cancel exactly across interior faces.  The 1D tables are compile-time
// constants of each kernel (make_tabk): the fully unrolled contractions take
// their entries as immediate operands.
#pragma once
#include "dgj_kernels.h"
#include "dgj_tables.h"

namespace dgj {

template <int D, int N, int Q>
struct ResK {
  using S = Shape<D, N, Q>;
  static constexpr int NV = S::NV, NM = S::NM, NQ = S::NQ, NQF = S::NQF, NMF = S::NMF, NF = S::NF, NB = S::NB;
  // sizes of the per-element scratch arrays
  static constexpr int TRACE = NF * (D + 1) * NV * NQF;    // trace[e]
  static constexpr int XF = 2 * D * (D + 1) * NV * NQF;    // X[e][f]: the flux of each face e computes
  static constexpr int T1 = (D == 3) ? 2 * NV * Q * N * N : 2 * NV * Q * N;
  static constexpr int T2 = (D == 3) ? 3 * NV * Q * Q * N : 0;
  static constexpr int QG = (D + 1) * NV * NQ;
};

// ---------------------------------------------------------------- volume phases
// Sum-factorised backward transform and reference gradients at the Gauss
// points: sQ[0][v][q] values, sQ[1+j][v][q] d/dxi_j (W: scratch of
// ResK::T1 + T2 doubles).  Thread tid of the NT that work on the element;
// every loop strides by NT.
template <int D, int N, int Q>
__device__ __forceinline__ void res_vol_forward(const TabK<N, Q>& tk, const double* __restrict__ sU,
                                                double* __restrict__ W, double* __restrict__ sQ, int tid, int NT) {
  using K = ResK<D, N, Q>;
  constexpr int NV = K::NV, NM = K::NM, NQ = K::NQ;
  (void)NM;
  if constexpr (D == 3) {
    double* T1 = W;                  // [2][v][a0][i1 + N i2]
    double* T2 = W + K::T1;          // [3][v][i2][a0 + Q a1]
    constexpr int n1 = NV * Q * N * N, n2 = NV * N * Q * Q;
    for (int pc = tid; pc < NV * N * N; pc += NT) {
      const int v = pc / (N * N), r = pc % (N * N);
      double x[N];
#pragma unroll
      for (int i0 = 0; i0 < N; ++i0) x[i0] = sU[v * NM + i0 + N * r];
#pragma unroll
      for (int a0 = 0; a0 < Q; ++a0) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int i0 = 0; i0 < N; ++i0) { s0 += tk.B[a0][i0] * x[i0]; s1 += tk.Dq[a0][i0] * x[i0]; }
        T1[(v * Q + a0) * N * N + r] = s0;
        T1[n1 + (v * Q + a0) * N * N + r] = s1;
      }
    }
    __syncthreads();
    for (int pc = tid; pc < NV * Q * N; pc += NT) {
      const int v = pc / (Q * N), a0 = (pc / N) % Q, i2 = pc % N;
      double x[N], xd[N];
#pragma unroll
      for (int i1 = 0; i1 < N; ++i1) {
        x[i1] = T1[(v * Q + a0) * N * N + i1 + N * i2];
        xd[i1] = T1[n1 + (v * Q + a0) * N * N + i1 + N * i2];
      }
#pragma unroll
      for (int a1 = 0; a1 < Q; ++a1) {
        double s0 = 0.0, sx = 0.0, sy = 0.0;
#pragma unroll
        for (int i1 = 0; i1 < N; ++i1) {
          s0 += tk.B[a1][i1] * x[i1];
          sx += tk.B[a1][i1] * xd[i1];
          sy += tk.Dq[a1][i1] * x[i1];
        }
        const int o = (v * N + i2) * Q * Q + a0 + Q * a1;
        T2[o] = s0;
        T2[n2 + o] = sx;
        T2[2 * n2 + o] = sy;
      }
    }
    __syncthreads();
    for (int pc = tid; pc < NV * Q * Q; pc += NT) {
      const int v = pc / (Q * Q), r = pc % (Q * Q);
      double x[N], xx[N], xy[N];
#pragma unroll
      for (int i2 = 0; i2 < N; ++i2) {
        const int o = (v * N + i2) * Q * Q + r;
        x[i2] = T2[o];
        xx[i2] = T2[n2 + o];
        xy[i2] = T2[2 * n2 + o];
      }
#pragma unroll
      for (int a2 = 0; a2 < Q; ++a2) {
        double s0 = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
        for (int i2 = 0; i2 < N; ++i2) {
          s0 += tk.B[a2][i2] * x[i2];
          sx += tk.B[a2][i2] * xx[i2];
          sy += tk.B[a2][i2] * xy[i2];
          sz += tk.Dq[a2][i2] * x[i2];
        }
        const int q = r + Q * Q * a2;
        sQ[v * NQ + q] = s0;
        sQ[NV * NQ + v * NQ + q] = sx;
        sQ[2 * NV * NQ + v * NQ + q] = sy;
        sQ[3 * NV * NQ + v * NQ + q] = sz;
      }
    }
  } else {
    double* T1 = W;                  // [2][v][i1][a0]
    constexpr int n1 = NV * N * Q;
    for (int pc = tid; pc < NV * N; pc += NT) {
      const int v = pc / N, i1 = pc % N;
      double x[N];
#pragma unroll
      for (int i0 = 0; i0 < N; ++i0) x[i0] = sU[v * NM + i0 + N * i1];
#pragma unroll
      for (int a0 = 0; a0 < Q; ++a0) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int i0 = 0; i0 < N; ++i0) { s0 += tk.B[a0][i0] * x[i0]; s1 += tk.Dq[a0][i0] * x[i0]; }
        T1[(v * N + i1) * Q + a0] = s0;
        T1[n1 + (v * N + i1) * Q + a0] = s1;
      }
    }
    __syncthreads();
    for (int pc = tid; pc < NV * Q; pc += NT) {
      const int v = pc / Q, a0 = pc % Q;
      double x[N], xd[N];
#pragma unroll
      for (int i1 = 0; i1 < N; ++i1) { x[i1] = T1[(v * N + i1) * Q + a0]; xd[i1] = T1[n1 + (v * N + i1) * Q + a0]; }
#pragma unroll
      for (int a1 = 0; a1 < Q; ++a1) {
        double s0 = 0.0, sx = 0.0, sy = 0.0;
#pragma unroll
        for (int i1 = 0; i1 < N; ++i1) {
          s0 += tk.B[a1][i1] * x[i1];
          sx += tk.B[a1][i1] * xd[i1];
          sy += tk.Dq[a1][i1] * x[i1];
        }
        const int q = a0 + Q * a1;
        sQ[v * NQ + q] = s0;
        sQ[NV * NQ + v * NQ + q] = sx;
        sQ[2 * NV * NQ + v * NQ + q] = sy;
      }
    }
  }
}

// Pointwise volume flux H_j = F_j - G_j scaled by w|J| dxi_j (boxes) or the
// contravariant w|J| sum_j (d xi_k / d x_j) H_j (curved), written over the
// gradient slots of sQ.
template <int D, int N, int Q, bool CV>
__device__ __forceinline__ void res_vol_flux(const ResArgs& a, const TabK<N, Q>& tk, const ElemParams& ep, long e,
                                             const double* dxi, double detJ, double* __restrict__ sQ, int tid,
                                             int NT) {
  using K = ResK<D, N, Q>;
  constexpr int NV = K::NV, NM = K::NM, NQ = K::NQ;
  (void)NM;
  // pointwise volume flux, scaled by w |J| dxi_j (overwrites the gradients);
  // curved: the contravariant flux w|J| sum_j (d xi_k/d x_j) H_j
  if constexpr (CV) {
    const double* vge = a.vg + e * (long)(D * D + 1) * NQ;
    for (int q = tid; q < NQ; q += NT) {
      double U[NV], gU[D][NV], F[D][NV], G[D][NV], Gm[D][D];
#pragma unroll
      for (int kk = 0; kk < D; ++kk)
#pragma unroll
        for (int j = 0; j < D; ++j) Gm[kk][j] = vge[(kk * D + j) * NQ + q];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        U[v] = sQ[v * NQ + q];
        double dr[D];
#pragma unroll
        for (int kk = 0; kk < D; ++kk) dr[kk] = sQ[(1 + kk) * NV * NQ + v * NQ + q];
#pragma unroll
        for (int j = 0; j < D; ++j) {
          double s = 0.0;
#pragma unroll
          for (int kk = 0; kk < D; ++kk) s += Gm[kk][j] * dr[kk];
          gU[j][v] = s;
        }
      }
      euler_flux<D, double>(ep.ph, U, F);
      viscous_flux<D, double, double>(ep.ph, U, gU, G);
      const double wJ = vge[D * D * NQ + q];
#pragma unroll
      for (int kk = 0; kk < D; ++kk)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double s = 0.0;
#pragma unroll
          for (int j = 0; j < D; ++j) s += Gm[kk][j] * (F[j][v] - G[j][v]);
          sQ[(1 + kk) * NV * NQ + v * NQ + q] = wJ * s;
        }
    }
  } else
  for (int q = tid; q < NQ; q += NT) {
    double U[NV], gU[D][NV], F[D][NV], G[D][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      U[v] = sQ[v * NQ + q];
#pragma unroll
      for (int j = 0; j < D; ++j) gU[j][v] = sQ[(1 + j) * NV * NQ + v * NQ + q] * dxi[j];
    }
    euler_flux<D, double>(ep.ph, U, F);
    viscous_flux<D, double, double>(ep.ph, U, gU, G);
    double wq = detJ;
    {
      int r = q;
#pragma unroll
      for (int k = 0; k < D; ++k) { wq *= tk.w[r % Q]; r /= Q; }
    }
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int v = 0; v < NV; ++v) sQ[(1 + j) * NV * NQ + v * NQ + q] = (F[j][v] - G[j][v]) * (wq * dxi[j]);
  }
}

// Transposed contraction with the derivative bases: out[v][m] =
// sum_j sum_q d(phi_m)/d(xi_j) H_j (W: scratch of ResK::T1 + T2 doubles).
template <int D, int N, int Q>
__device__ __forceinline__ void res_vol_transpose(const TabK<N, Q>& tk, const double* __restrict__ sQ,
                                                  double* __restrict__ W, double* __restrict__ out, int tid,
                                                  int NT) {
  using K = ResK<D, N, Q>;
  constexpr int NV = K::NV, NM = K::NM, NQ = K::NQ;
  if constexpr (D == 3) {
    const double* Hx = sQ + NV * NQ;
    const double* Hy = sQ + 2 * NV * NQ;
    const double* Hz = sQ + 3 * NV * NQ;
    double* U1 = W;                              // [3][v][i2][a0 + Q a1]
    double* U2 = W + 3 * NV * N * Q * Q;         // [2][v][a0][i1 + N i2]
    constexpr int n1 = NV * N * Q * Q, n2 = NV * Q * N * N;
    for (int pc = tid; pc < NV * Q * Q; pc += NT) {
      const int v = pc / (Q * Q), r = pc % (Q * Q);
      double hx[Q], hy[Q], hz[Q];
#pragma unroll
      for (int a2 = 0; a2 < Q; ++a2) {
        hx[a2] = Hx[v * NQ + r + Q * Q * a2];
        hy[a2] = Hy[v * NQ + r + Q * Q * a2];
        hz[a2] = Hz[v * NQ + r + Q * Q * a2];
      }
#pragma unroll
      for (int i2 = 0; i2 < N; ++i2) {
        double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
        for (int a2 = 0; a2 < Q; ++a2) {
          sx += tk.B[a2][i2] * hx[a2];
          sy += tk.B[a2][i2] * hy[a2];
          sz += tk.Dq[a2][i2] * hz[a2];
        }
        const int o = (v * N + i2) * Q * Q + r;
        U1[o] = sx;
        U1[n1 + o] = sy;
        U1[2 * n1 + o] = sz;
      }
    }
    __syncthreads();
    for (int pc = tid; pc < NV * Q * N; pc += NT) {
      const int v = pc / (Q * N), a0 = (pc / N) % Q, i2 = pc % N;
      double x[Q], y[Q], z[Q];
#pragma unroll
      for (int a1 = 0; a1 < Q; ++a1) {
        const int o = (v * N + i2) * Q * Q + a0 + Q * a1;
        x[a1] = U1[o];
        y[a1] = U1[n1 + o];
        z[a1] = U1[2 * n1 + o];
      }
#pragma unroll
      for (int i1 = 0; i1 < N; ++i1) {
        double sa = 0.0, sb = 0.0;
#pragma unroll
        for (int a1 = 0; a1 < Q; ++a1) {
          sa += tk.B[a1][i1] * x[a1];
          sb += tk.Dq[a1][i1] * y[a1] + tk.B[a1][i1] * z[a1];
        }
        const int o = (v * Q + a0) * N * N + i1 + N * i2;
        U2[o] = sa;
        U2[n2 + o] = sb;
      }
    }
    __syncthreads();
    for (int pc = tid; pc < NV * N * N; pc += NT) {
      const int v = pc / (N * N), r = pc % (N * N);
      double x[Q], y[Q];
#pragma unroll
      for (int a0 = 0; a0 < Q; ++a0) {
        x[a0] = U2[(v * Q + a0) * N * N + r];
        y[a0] = U2[n2 + (v * Q + a0) * N * N + r];
      }
#pragma unroll
      for (int i0 = 0; i0 < N; ++i0) {
        double s = 0.0;
#pragma unroll
        for (int a0 = 0; a0 < Q; ++a0) s += tk.Dq[a0][i0] * x[a0] + tk.B[a0][i0] * y[a0];
        out[v * NM + i0 + N * r] = s;
      }
    }
  } else {
    const double* Hx = sQ + NV * NQ;
    const double* Hy = sQ + 2 * NV * NQ;
    double* U1 = W;                              // [2][v][i1][a0]
    constexpr int n1 = NV * N * Q;
    for (int pc = tid; pc < NV * Q; pc += NT) {
      const int v = pc / Q, a0 = pc % Q;
      double hx[Q], hy[Q];
#pragma unroll
      for (int a1 = 0; a1 < Q; ++a1) { hx[a1] = Hx[v * NQ + a0 + Q * a1]; hy[a1] = Hy[v * NQ + a0 + Q * a1]; }
#pragma unroll
      for (int i1 = 0; i1 < N; ++i1) {
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int a1 = 0; a1 < Q; ++a1) { sx += tk.B[a1][i1] * hx[a1]; sy += tk.Dq[a1][i1] * hy[a1]; }
        U1[(v * N + i1) * Q + a0] = sx;
        U1[n1 + (v * N + i1) * Q + a0] = sy;
      }
    }
    __syncthreads();
    for (int pc = tid; pc < NV * N; pc += NT) {
      const int v = pc / N, i1 = pc % N;
      double x[Q], y[Q];
#pragma unroll
      for (int a0 = 0; a0 < Q; ++a0) { x[a0] = U1[(v * N + i1) * Q + a0]; y[a0] = U1[n1 + (v * N + i1) * Q + a0]; }
#pragma unroll
      for (int i0 = 0; i0 < N; ++i0) {
        double s = 0.0;
#pragma unroll
        for (int a0 = 0; a0 < Q; ++a0) s += tk.Dq[a0][i0] * x[a0] + tk.B[a0][i0] * y[a0];
        out[v * NM + i0 + N * i1] = s;
      }
    }
  }
}

// ---------------------------------------------------------------- volume + traces
// Block size (runtime, a multiple of 64, at most 256) is chosen per shape by
// the autotuner; every loop strides by blockDim.x.
template <int D, int N, int Q, bool CV>
__global__ __launch_bounds__(256) void k_res_vol(ResArgs a, double* __restrict__ trace,
                                                double* __restrict__ Lvol) {
  static constexpr TabK<N, Q> tk = make_tabk<N, Q>();
  using K = ResK<D, N, Q>;
  constexpr int NV = K::NV, NM = K::NM, NQ = K::NQ, NQF = K::NQF, NF = K::NF, NB = K::NB;
  __shared__ double sU[NB];
  __shared__ double W[K::T1 + K::T2];
  __shared__ double sQ[K::QG];
  const long e = blockIdx.x;
  if (e >= a.n_elem) return;
  ElemParams ep;
  if (!elem_params(a, e, ep)) return;
  const int tid = threadIdx.x;
  const int NT = blockDim.x;
  const double* g = a.geo + e * K::S::GEO;
  double dxi[D];
#pragma unroll
  for (int j = 0; j < D; ++j) dxi[j] = g[j];
  const double detJ = g[D];
  for (int i = tid; i < NB; i += NT) sU[i] = ep.in(e * NB + i);
  __syncthreads();

  res_vol_forward<D, N, Q>(tk, sU, W, sQ, tid, NT);
  __syncthreads();

  // LDG (affine boxes): the auxiliary gradient is grad u plus the lifted
  // face jumps, so the traces and the volume flux below see q
  if (!CV && a.ldg_r) {
    const double* r = a.ldg_r + e * (long)D * NV * NQ;
    for (int it = tid; it < D * NV * NQ; it += NT) {
      const int j = it / (NV * NQ);
      sQ[(1 + j) * NV * NQ + it % (NV * NQ)] += r[it] / dxi[j];
    }
    __syncthreads();
  }

  // own face traces: value and physical gradient at the face points
  if constexpr (CV) {
    // curved: interpolate value and reference gradient, then grad = G^T grad_xi
    constexpr int CF = D * D + D + 1;
    double* tr = trace + e * (long)K::TRACE;
    const double* fge = a.fg + e * (long)NF * CF * NQF;
    for (int it = tid; it < NF * NV * NQF; it += NT) {
      const int p = it % NQF;
      const int v = (it / NQF) % NV;
      const int f = it / (NQF * NV);
      const int ax = f >> 1, s = f & 1;
      int qstride = 1, base = 0;
      {
        int t[2] = {0, 0};
        tang_axes<D>(ax, t);
        int st[3] = {1, Q, Q * Q};
        qstride = st[ax];
        base = (p % Q) * st[t[0]];
        if (D == 3) base += (p / Q) * st[t[1]];
      }
      double rv[D + 1];
#pragma unroll
      for (int c = 0; c <= D; ++c) {
        const double* y = sQ + c * NV * NQ + v * NQ + base;
        double acc = 0.0;
#pragma unroll
        for (int aa = 0; aa < Q; ++aa) acc += tk.lag[s][aa] * y[aa * qstride];
        rv[c] = acc;
      }
      const double* Gp = fge + f * CF * NQF + p;
      tr[((f * (D + 1)) * NV + v) * NQF + p] = rv[0];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        double gj = 0.0;
#pragma unroll
        for (int kk = 0; kk < D; ++kk) gj += Gp[(kk * D + j) * NQF] * rv[1 + kk];
        tr[((f * (D + 1) + 1 + j) * NV + v) * NQF + p] = gj;
      }
    }
  } else {
    double* tr = trace + e * (long)K::TRACE;
    for (int it = tid; it < K::TRACE; it += NT) {
      const int p = it % NQF;
      const int v = (it / NQF) % NV;
      const int c = (it / (NQF * NV)) % (D + 1);
      const int f = it / (NQF * NV * (D + 1));
      const int ax = f >> 1, s = f & 1;
      // volume point index of (a along ax, tangential p)
      int qstride = 1, base = 0;
      {
        int t[2] = {0, 0};
        tang_axes<D>(ax, t);
        int st[3] = {1, Q, Q * Q};
        qstride = st[ax];
        base = (p % Q) * st[t[0]];
        if (D == 3) base += (p / Q) * st[t[1]];
      }
      const double* y = sQ + c * NV * NQ + v * NQ + base;
      double acc = 0.0;
#pragma unroll
      for (int aa = 0; aa < Q; ++aa) acc += tk.lag[s][aa] * y[aa * qstride];
      tr[it] = (c == 0) ? acc : acc * dxi[c - 1];
    }
  }
  __syncthreads();   // the flux loop below overwrites the gradients read above

  // pointwise volume flux (overwrites the gradients)
  res_vol_flux<D, N, Q, CV>(a, tk, ep, e, dxi, detJ, sQ, tid, NT);
  __syncthreads();

  // transposed contraction with the derivative bases
  res_vol_transpose<D, N, Q>(tk, sQ, W, Lvol + e * (long)NB, tid, NT);
}

// ---------------------------------------------------------------- LDG lifting
// Lifted face jumps of the LDG auxiliary gradient at the volume points of
// an affine box: rq[e][j][v][q] = r_j(x_q), M_e r_j = sum over the faces of
// the integral of phi (u_hat - u^-) n_j.  u_hat comes from the face's left
// element, so only the element's side-0 interior faces (u_hat = the
// neighbour's trace) and its boundary faces (u_hat = the mean of interior
// and ghost states) contribute.  With the orthonormal basis M_e = |J| I and
// |J_f| / |J| = 2 / h_axis, so for face f of axis j and side s
//   r_j(x_q) += (2/h_j) n_j sum_p K_f(q, p) w_p delta_p,
// K_f(q, p) = sum_m phi_m(x_q) phi_m(x_p) = kE[a_j(q)][s] prod_t k1[a_t(q)][a_t(p)]
// with the 1D kernels k1[a][b] = sum_i B[a][i] B[b][i] (Gauss points) and
// kE[a][s] = sum_i B[a][i] phi_i(+-1).
template <int D, int N, int Q>
__global__ __launch_bounds__(256) void k_ldg_lift(ResArgs a, double* __restrict__ rq) {
  static constexpr TabK<N, Q> tk = make_tabk<N, Q>();
  using K = ResK<D, N, Q>;
  constexpr int NV = K::NV, NM = K::NM, NQ = K::NQ, NQF = K::NQF, NF = K::NF, NB = K::NB;
  __shared__ double sU[NB], sN[NB];
  __shared__ double sD[NF * NV * NQF];
  __shared__ double k1[Q][Q], kE[Q][2];
  const long e = blockIdx.x;
  if (e >= a.n_elem) return;
  ElemParams ep;
  if (!elem_params(a, e, ep)) return;
  const int tid = threadIdx.x, NT = blockDim.x;
  const double* g = a.geo + e * K::S::GEO;
  for (int i = tid; i < NB; i += NT) sU[i] = ep.in(e * NB + i);
  for (int i = tid; i < Q * Q; i += NT) {
    const int x = i / Q, y = i % Q;
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) s += tk.B[x][m] * tk.B[y][m];
    k1[x][y] = s;
  }
  for (int i = tid; i < 2 * Q; i += NT) {
    const int x = i / 2, sd = i % 2;
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) s += tk.B[x][m] * tk.phiE[sd][m];
    kE[x][sd] = s;
  }
  for (int f = 0; f < NF; ++f) {
    const long en = a.nbr[e * NF + f];
    const int ax = f >> 1, sd = f & 1;
    const bool active = en < 0 || sd == 0;
    __syncthreads();
    if (active && en >= 0)
      for (int i = tid; i < NB; i += NT) sN[i] = ep.in(en * NB + i);
    __syncthreads();
    for (int p = tid; p < NQF; p += NT) {
      double* dj = sD + f * NV * NQF + p;
      if (!active) {
#pragma unroll
        for (int v = 0; v < NV; ++v) dj[v * NQF] = 0.0;
        continue;
      }
      int t[2] = {0, 0};
      tang_axes<D>(ax, t);
      const int ap0 = p % Q, ap1 = p / Q;
      double Uo[NV], Uo2[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) { Uo[v] = 0.0; Uo2[v] = 0.0; }
      for (int m = 0; m < NM; ++m) {
        int mi[3] = {0, 0, 0};
        split<D, N>(m, mi);
        double bt = tk.B[ap0][mi[t[0]]];
        if (D == 3) bt *= tk.B[ap1][mi[t[1]]];
        const double po = bt * tk.phiE[sd][mi[ax]];
        const double pn = bt * tk.phiE[sd ^ 1][mi[ax]];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          Uo[v] += po * sU[v * NM + m];
          if (en >= 0) Uo2[v] += pn * sN[v * NM + m];
        }
      }
      if (en >= 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) dj[v * NQF] = Uo2[v] - Uo[v];
      } else {
        const int bid = -(int)en - 1;
        const int kind = a.bc_kind[bid];
        double nrm[D], UD[NV], Ug[NV];
#pragma unroll
        for (int j = 0; j < D; ++j) nrm[j] = (j == ax) ? (sd == 1 ? 1.0 : -1.0) : 0.0;
        const double* Ub = a.bc_state + bid * NV;
        if (kind == BC_DIRICHLET) {
          const double* gb = a.bc_field + (e * NF + f) * (long)NV * NQF + p;
#pragma unroll
          for (int v = 0; v < NV; ++v) UD[v] = gb[v * NQF];
          Ub = UD;
        }
        ghost_state<D>(ep.ph, kind, Uo, nrm, Ub, Ug);
#pragma unroll
        for (int v = 0; v < NV; ++v) dj[v * NQF] = 0.5 * (Ug[v] - Uo[v]);
      }
    }
  }
  __syncthreads();
  double* out = rq + e * (long)D * NV * NQ;
  for (int it = tid; it < D * NV * NQ; it += NT) {
    const int q = it % NQ, v = (it / NQ) % NV, j = it / (NV * NQ);
    int aq[3] = {0, 0, 0};
    {
      int r = q;
#pragma unroll
      for (int k = 0; k < D; ++k) { aq[k] = r % Q; r /= Q; }
    }
    int t[2] = {0, 0};
    tang_axes<D>(j, t);
    double acc = 0.0;
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const double* dj = sD + (2 * j + sd) * NV * NQF + v * NQF;
      double s = 0.0;
      for (int p = 0; p < NQF; ++p) {
        const int ap0 = p % Q, ap1 = p / Q;
        double kk = k1[aq[t[0]]][ap0] * tk.w[ap0];
        if (D == 3) kk *= k1[aq[t[1]]][ap1] * tk.w[ap1];
        s += kk * dj[p];
      }
      acc += (sd == 1 ? 1.0 : -1.0) * kE[aq[j]][sd] * s;
    }
    out[it] = g[j] * acc;   // g[j] = d xi_j / d x_j = 2 / h_j
  }
}

// ---------------------------------------------------------------- face fluxes
// Flux of face f of element e at face point p, weighted by w^G |J^G|, into
// X[e][f]: (H^n, S_j) in e's orientation (outward normal of face f).
template <int D, int N, int Q, bool CV>
__device__ __forceinline__ void face_point_flux(const ResArgs& a, const TabK<N, Q>& tk, const Phys& ph,
                                                const double* __restrict__ trace, double* __restrict__ X, long e,
                                                int f, long en, int p) {
  using K = ResK<D, N, Q>;
  constexpr int NV = K::NV, NQF = K::NQF;
  const int ax = f >> 1, s = f & 1;
  const double* tL = trace + e * (long)K::TRACE + f * (D + 1) * NV * NQF;
  double UL[NV], gL[D][NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    UL[v] = tL[v * NQF + p];
#pragma unroll
    for (int j = 0; j < D; ++j) gL[j][v] = tL[((1 + j) * NV + v) * NQF + p];
  }
  double nrm[D];
  double wf;
  if constexpr (CV) {
    constexpr int CF = D * D + D + 1;
    const double* Gp = a.fg + (e * K::NF + f) * (long)CF * NQF + p;
#pragma unroll
    for (int j = 0; j < D; ++j) nrm[j] = Gp[(D * D + j) * NQF];
    wf = Gp[(D * D + D) * NQF];
  } else {
#pragma unroll
    for (int j = 0; j < D; ++j) nrm[j] = (j == ax) ? (s == 1 ? 1.0 : -1.0) : 0.0;
    wf = a.geo[e * K::S::GEO + D + 2 + ax] * tk.w[p % Q];
    if (D == 3) wf *= tk.w[p / Q];
  }
  double H[NV], Sf[D][NV];
  const double beta = a.beta[e * K::NF + f];
  if (a.ldg_r) {
    // LDG: the traces' gradients are the auxiliary q; no symmetric term
    if (en >= 0) {
      const double* tR = trace + en * (long)K::TRACE + (f ^ 1) * (D + 1) * NV * NQF;
      double UR[NV], qR[D][NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        UR[v] = tR[v * NQF + p];
#pragma unroll
        for (int j = 0; j < D; ++j) qR[j][v] = tR[((1 + j) * NV + v) * NQF + p];
      }
      face_flux_ldg<D>(ph, UL, UR, qR, nrm, beta, H);
    } else {
      const int bid = -(int)en - 1;
      const int kind = a.bc_kind[bid];
      double UD[NV];
      const double* Ub = a.bc_state + bid * NV;
      if (kind == BC_DIRICHLET) {
        const double* g = a.bc_field + (e * K::NF + f) * (long)NV * NQF + p;
#pragma unroll
        for (int v = 0; v < NV; ++v) UD[v] = g[v * NQF];
        Ub = UD;
      }
      boundary_flux_ldg<D>(ph, kind, UL, gL, nrm, beta, Ub, H);
    }
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int v = 0; v < NV; ++v) Sf[j][v] = 0.0;
  } else if (en >= 0) {
    const double* tR = trace + en * (long)K::TRACE + (f ^ 1) * (D + 1) * NV * NQF;
    double UR[NV], gR[D][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      UR[v] = tR[v * NQF + p];
#pragma unroll
      for (int j = 0; j < D; ++j) gR[j][v] = tR[((1 + j) * NV + v) * NQF + p];
    }
    face_flux<D>(ph, UL, UR, gL, gR, nrm, beta, H, Sf);
  } else {
    const int bid = -(int)en - 1;
    const int kind = a.bc_kind[bid];
    double UD[NV];
    const double* Ub = a.bc_state + bid * NV;
    if (kind == BC_DIRICHLET) {
      const double* g = a.bc_field + (e * K::NF + f) * (long)NV * NQF + p;
#pragma unroll
      for (int v = 0; v < NV; ++v) UD[v] = g[v * NQF];
      Ub = UD;
    }
    boundary_flux<D>(ph, kind, UL, gL, nrm, beta, Ub, H, Sf);
  }
  double* o = X + e * (long)K::XF + f * (D + 1) * NV * NQF;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    o[v * NQF + p] = wf * H[v];
#pragma unroll
    for (int j = 0; j < D; ++j) o[((1 + j) * NV + v) * NQF + p] = wf * Sf[j][v];
  }
}

// One thread per (element, axis, point).  Each interior face is computed
// once, by the element that meets it with side 1 (normal +e_axis); a
// boundary face by its element, in its own orientation, so the thread of
// axis a also computes its element's side-0 face when that is a boundary.
template <int D, int N, int Q, bool CV>
__global__ __launch_bounds__(256) void k_res_face(ResArgs a, const double* __restrict__ trace,
                                                  double* __restrict__ X) {
  static constexpr TabK<N, Q> tk = make_tabk<N, Q>();
  using K = ResK<D, N, Q>;
  constexpr int NQF = K::NQF, NF = K::NF;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= a.n_elem * D * NQF) return;
  const int p = gid % NQF;
  const int ax = (gid / NQF) % D;
  const long e = gid / (NQF * D);
  ElemParams ep;
  if (!elem_params(a, e, ep)) return;
  face_point_flux<D, N, Q, CV>(a, tk, ep.ph, trace, X, e, 2 * ax + 1, a.nbr[e * NF + 2 * ax + 1], p);
  const long e0 = a.nbr[e * NF + 2 * ax];
  if (e0 < 0) face_point_flux<D, N, Q, CV>(a, tk, ep.ph, trace, X, e, 2 * ax, e0, p);
}

// the operands of the epilogue of unknown gi other than R: the state w
// (the caller's copy), and S and N_u as the mode needs them, so that a
// kernel can load them ahead of the result
struct EpiIn {
  double w, S, Nu;
};
__device__ __forceinline__ EpiIn epi_load(const ResArgs& a, long gi, double w) {
  EpiIn x{w, 0.0, 0.0};
  if (a.mode != RES_R) x.S = a.S[gi];
  if (a.mode == RES_JV) x.Nu = a.Nu[gi];
  return x;
}
// the epilogue below with its operands given (the same arithmetic)
__device__ __forceinline__ void epilogue_pre(const ResArgs& a, const ElemParams& ep, long gi, double R,
                                             const EpiIn& x) {
  if (a.src) R += a.src[gi];
  if (a.mode == RES_R) {
    a.out[gi] = R;
  } else {
    const double Nw = (x.w - x.S) - ep.dt_a * R;
    if (a.mode == RES_N) a.out[gi] = Nw;
    else a.out[gi] = (Nw - x.Nu) / ep.in.eps;
  }
}

// output of the residual kernels for unknown gi with R = (M^-1 L)_gi
__device__ __forceinline__ void epilogue(const ResArgs& a, const ElemParams& ep, long gi, double R) {
  if (a.src) R += a.src[gi];
  if (a.mode == RES_R) {
    a.out[gi] = R;
  } else {
    const double w = ep.in(gi);
    const double Nw = (w - a.S[gi]) - ep.dt_a * R;
    if (a.mode == RES_N) a.out[gi] = Nw;
    else a.out[gi] = (Nw - a.Nu[gi]) / ep.in.eps;
  }
}

// ---------------------------------------------------------------- lift + epilogue
template <int D, int N, int Q, bool CV>
__global__ __launch_bounds__(256) void k_res_lift(ResArgs a, const double* __restrict__ Lvol,
                                                 const double* __restrict__ X) {
  static constexpr TabK<N, Q> tk = make_tabk<N, Q>();
  using K = ResK<D, N, Q>;
  constexpr int NV = K::NV, NM = K::NM, NQF = K::NQF, NMF = K::NMF, NF = K::NF, NB = K::NB;
  __shared__ double sA[NF * (D + 1) * NV * NQF];
  __shared__ double sF[NF * 2 * NV * NMF];
  const long e = blockIdx.x;
  if (e >= a.n_elem) return;
  ElemParams ep;
  if (!elem_params(a, e, ep)) return;
  const int tid = threadIdx.x;
  const int NT = blockDim.x;
  const double* g = a.geo + e * K::S::GEO;
  // where each face's flux is stored: this element's slot (side-1 and
  // boundary faces, own orientation) or the neighbour's side-1 slot
  __shared__ long s_src[NF];
  __shared__ int s_fs[NF], s_mine[NF];
  if (tid < NF) {
    const long en = a.nbr[e * NF + tid];
    const bool mine = (tid & 1) == 1 || en < 0;
    s_src[tid] = mine ? e : en;
    s_fs[tid] = mine ? tid : (tid ^ 1);
    s_mine[tid] = mine;
  }
  __syncthreads();
  // this thread's volume terms, loaded early (read after the face phases)
  constexpr int LPT = (NB + 63) / 64;           // at most this many per thread (NT >= 64)
  double lv[LPT];
#pragma unroll
  for (int u = 0; u < LPT; ++u) {
    const int i = tid + u * NT;
    lv[u] = i < NB ? Lvol[e * NB + i] : 0.0;
  }
  // face data in the element's own orientation and scaling
  constexpr int TOT = NF * (D + 1) * NV * NQF;
  if constexpr (CV) {
    for (int it = tid; it < TOT; it += NT) {
      const int p = it % NQF;
      const int v = (it / NQF) % NV;
      const int k = (it / (NQF * NV)) % (D + 1);
      const int f = it / (NQF * NV * (D + 1));
      const bool mine = s_mine[f];
      const double* Xs = X + s_src[f] * (long)K::XF + (s_fs[f] * (D + 1) * NV + v) * NQF + p;
      // k = 0: -Hhat_own (the neighbour's flux has the opposite orientation);
      // k >= 1: sum_j (d xi_{k-1} / d x_j) Shat_j
      if (k == 0) {
        const double x = Xs[0];
        sA[it] = mine ? -x : x;
      } else {
        constexpr int CF = D * D + D + 1;
        const double* Gp = a.fg + (e * NF + f) * (long)CF * NQF + p;
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) s += Gp[((k - 1) * D + j) * NQF] * Xs[(1 + j) * NV * NQF];
        sA[it] = s;
      }
    }
  } else {
    // affine boxes: each face's data is one contiguous run of X; issue a
    // batch of independent loads per thread before any is used
    constexpr int FB = (D + 1) * NV * NQF;
    constexpr int UB = 8;
    for (int base = 0; base < TOT; base += UB * NT) {
      double x[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int it = base + u * NT + tid;
        if (it < TOT) {
          const int f = it / FB;
          x[u] = X[s_src[f] * (long)K::XF + s_fs[f] * FB + it % FB];
        }
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int it = base + u * NT + tid;
        if (it < TOT) {
          const int f = it / FB;
          const int k = (it % FB) / (NV * NQF);
          sA[it] = (k == 0) ? (s_mine[f] ? -x[u] : x[u]) : x[u] * g[k - 1];
        }
      }
    }
  }
  __syncthreads();
  // tangential contraction to face modes: F0 (multiplies phi(+-1)), F1 (phi'(+-1))
  for (int it = tid; it < NF * NV * NMF; it += NT) {
    const int tm = it % NMF;
    const int v = (it / NMF) % NV;
    const int f = it / (NMF * NV);
    const int ax = f >> 1;
    int t[2] = {0, 0};
    tang_axes<D>(ax, t);
    const int j0 = tm % N, j1 = (D == 3) ? tm / N : 0;
    const double* A = sA + f * (D + 1) * NV * NQF;
    double f0 = 0.0, f1 = 0.0;
#pragma unroll
    for (int p = 0; p < NQF; ++p) {
      const int b0 = p % Q, b1 = (D == 3) ? p / Q : 0;
      const double B0 = tk.B[b0][j0], D0 = tk.Dq[b0][j0];
      const double B1 = (D == 3) ? tk.B[b1][j1] : 1.0;
      const double D1 = (D == 3) ? tk.Dq[b1][j1] : 0.0;
      const double bb = B0 * B1;
      f0 += bb * A[v * NQF + p] + D0 * B1 * A[((1 + t[0]) * NV + v) * NQF + p];
      if (D == 3) f0 += B0 * D1 * A[((1 + t[1]) * NV + v) * NQF + p];
      f1 += bb * A[((1 + ax) * NV + v) * NQF + p];
    }
    sF[(f * 2 + 0) * NV * NMF + v * NMF + tm] = f0;
    sF[(f * 2 + 1) * NV * NMF + v * NMF + tm] = f1;
  }
  __syncthreads();
  const double invdetJ = g[D + 1];
  double* sL = sA;   // curved: L staged for the dense M^-1 (sA is no longer read)
  constexpr bool curved = CV;
#pragma unroll
  for (int u = 0; u < LPT; ++u) {
    const int i = tid + u * NT;
    if (i >= NB) break;
    const int m = i % NM, v = i / NM;
    int mi[3] = {0, 0, 0};
    split<D, N>(m, mi);
    double L = lv[u];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int ax = f >> 1, s = f & 1;
      int t[2] = {0, 0};
      tang_axes<D>(ax, t);
      const int tm = mi[t[0]] + ((D == 3) ? N * mi[t[1]] : 0);
      L += tk.phiE[s][mi[ax]] * sF[(f * 2 + 0) * NV * NMF + v * NMF + tm] +
           tk.dphiE[s][mi[ax]] * sF[(f * 2 + 1) * NV * NMF + v * NMF + tm];
    }
    if constexpr (curved) sL[i] = L;
    else epilogue(a, ep, e * NB + i, L * invdetJ);
  }
  if constexpr (curved) {
    __syncthreads();
    constexpr int NSC = (NF * (D + 1) * NV * NQF - NB) / NB;   // groups whose partial sums fit in sA
    static_assert(NSC >= 1, "LDS staging of the mass-matrix product");
    mass_inv_dense<NM, NV>(a.minv + e * (long)NM * mass_ld(NM), sL, sA + NB, tid, NT, NSC,
                           [&](int i, double R, int) { epilogue(a, ep, e * NB + i, R); });
  }
}

}  // namespace dgj
