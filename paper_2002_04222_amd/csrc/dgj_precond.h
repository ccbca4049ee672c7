// Block-relaxed-Jacobi preconditioner BRJ(J) of arxiv 2002.04222
// (Sec. 4.2.2, Eq. 27-31): build of the element blocks
//   D_e = I - dt a M^-1 A_e,
//   A_e = sum_j (D_j B)^T diag(w|J| dH_j/dQ) B + sum_ij (D_j B)^T diag(w|J| dH_j/d grad_i Q) (D_i B)
//         - sum_f (B^G_f)^T diag(w^G |J^G| dHhat/dQ^-) B^G_f,
// the forward-difference face flux Jacobians dHhat/dQ^+- of Eq. 31, the
// explicit inverse of D_e by blocked Gauss-Jordan elimination with partial
// pivoting, and the apply of Eq. 28 (diagonal GEMV with the stored inverse,
// off-diagonal product on the fly from neighbour traces).
//
// Storage: Dinv[e][col][row] (column-major per element, nb = NV*NM rows) in
// double, float or bfloat16; face Jacobians Jp[e][f][p][k][l] (unscaled) in
// double or float.
#pragma once
#include "dgj_kernels.h"

namespace dgj {

// value of the element's trace at face point p of its face f: sum over modes;
// the gradient by dxi_j = gX[j] (boxes) or by the face-point metrics fgF
// (curved: the element's fg block of face f, or null)
template <int D, int N, int Q>
__device__ __forceinline__ void trace_point(const Tab& tb, const StateIn& in, long X, const double* gX, int f,
                                            int p, double* U, double (*gU)[D + 2],
                                            const double* fgF = nullptr) {
  using S = Shape<D, N, Q>;
  constexpr int NV = S::NV, NM = S::NM;
  const int ax = f >> 1, s = f & 1;
  int tax[2] = {0, 0};
  tang_axes<D>(ax, tax);
  int bq[3] = {0, 0, 0};
  bq[tax[0]] = p % Q;
  if (D == 3) bq[tax[1]] = p / Q;
  double dref[D][NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    U[v] = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) dref[j][v] = 0.0;
  }
  for (int m = 0; m < NM; ++m) {
    int mi[3] = {0, 0, 0};
    split<D, N>(m, mi);
    double val[D], der[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      if (k == ax) { val[k] = tb.phiE[s * N + mi[k]]; der[k] = tb.dphiE[s * N + mi[k]]; }
      else { val[k] = tb.B[bq[k] * N + mi[k]]; der[k] = tb.Dq[bq[k] * N + mi[k]]; }
    }
    double phi = 1.0;
#pragma unroll
    for (int k = 0; k < D; ++k) phi *= val[k];
    double dphi[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double t = 1.0;
#pragma unroll
      for (int k = 0; k < D; ++k) t *= (k == j) ? der[k] : val[k];
      dphi[j] = t;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double uu = in(X * S::NB + v * NM + m);
      U[v] += phi * uu;
#pragma unroll
      for (int j = 0; j < D; ++j) dref[j][v] += dphi[j] * uu;
    }
  }
  if (fgF) {
    constexpr int NQF = S::NQF;
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) s += fgF[(k * D + j) * NQF + p] * dref[k][v];
        gU[j][v] = s;
      }
    return;
  }
#pragma unroll
  for (int j = 0; j < D; ++j)
#pragma unroll
    for (int v = 0; v < NV; ++v) gU[j][v] = dref[j][v] * gX[j];
}

// ---------------------------------------------------------------- volume flux Jacobians
// Wt[e][q][j][b][k][l]: b = 0 -> dH_j,k/dQ_l at fixed gradient (exact, forward-mode
// duals), b = 1+i -> dH_j,k/d(d_i Q_l) = -K (exact, G is linear in grad Q);
// in reference directions j, i: scaled by w_q |J| dxi_j (and dxi_i for b > 0)
// on boxes; on curved elements (vg) contracted with d xi/d x on both sides,
// w|J| sum_j' G[j][j'] dH_j'/dQ and w|J| sum_j' G[j][j'] dH_j'/d(grad Q) . G[i].
template <int D, int N, int Q, int NT>
__global__ __launch_bounds__(NT) void k_pc_volume(const double* __restrict__ u, const double* __restrict__ geo,
                                                  const double* __restrict__ tables, Phys ph, long n_elem,
                                                  double* __restrict__ Wt, long e0, const double* __restrict__ vg) {
  using S = Shape<D, N, Q>;
  using L = ResidualLDS<D, N, Q>;
  constexpr int NV = S::NV, NQ = S::NQ;
  __shared__ double smem[L::TABSZ + S::NB + L::VOL];
  const long e = e0 + blockIdx.x;
  if (blockIdx.x >= n_elem) return;
  Tab tb = load_tables<N, Q>(tables, smem);
  double* sU = smem + L::TABSZ;
  double* W = sU + S::NB;
  double* sQ = W + L::V_T1 + L::V_T2;
  for (int i = threadIdx.x; i < S::NB; i += NT) sU[i] = u[e * S::NB + i];
  __syncthreads();
  vol_forward<D, N, Q, NT>(tb, sU, W, sQ);
  __syncthreads();
  const double* g = geo + e * S::GEO;
  constexpr int PER_Q = D * (D + 1) * NV * NV;
  const double* vge = vg ? vg + e * (long)(D * D + 1) * NQ : nullptr;
  for (int q = threadIdx.x; q < NQ; q += NT) {
    double U[NV], gU[D][NV], Gm[D][D];
    double wq;
    if (vge) {
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int j = 0; j < D; ++j) Gm[k][j] = vge[(k * D + j) * NQ + q];
      wq = vge[D * D * NQ + q];
    } else {
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int j = 0; j < D; ++j) Gm[k][j] = (k == j) ? g[j] : 0.0;
      wq = g[D];
      int r = q;
#pragma unroll
      for (int k = 0; k < D; ++k) { wq *= tb.w[r % Q]; r /= Q; }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      U[v] = sQ[v * NQ + q];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) s += Gm[k][j] * sQ[(1 + k) * NV * NQ + v * NQ + q];
        gU[j][v] = s;
      }
    }
    double* out = Wt + ((long)blockIdx.x * NQ + q) * PER_Q;   // Wt holds the launch's elements
    // dH/dQ via duals, one flux direction at a time to bound register use
    Dual<NV> Ud[NV];
#pragma unroll
    for (int l = 0; l < NV; ++l) { Ud[l] = Dual<NV>(U[l]); Ud[l].d[l] = 1.0; }
    {
      Dual<NV> F[D][NV], G[D][NV];
      euler_flux<D, Dual<NV>>(ph, Ud, F);
      viscous_flux<D, Dual<NV>, double>(ph, Ud, gU, G);
#pragma unroll
      for (int j = 0; j < D; ++j) {
#pragma unroll
        for (int k = 0; k < NV; ++k)
#pragma unroll
          for (int l = 0; l < NV; ++l) {
            double s = 0.0;
#pragma unroll
            for (int jj = 0; jj < D; ++jj) s += Gm[j][jj] * (F[jj][k].d[l] - G[jj][k].d[l]);
            out[((j * (D + 1) + 0) * NV + k) * NV + l] = s * wq;
          }
      }
    }
    // dH/d grad Q = -K: probe the linear viscous flux with the physical
    // gradient of a unit reference derivative, d_x Q_l = G[i][.]
    for (int i = 0; i < D; ++i) {
      for (int l = 0; l < NV; ++l) {
        double E[D][NV], G[D][NV];
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int v = 0; v < NV; ++v) E[a][v] = (v == l) ? Gm[i][a] : 0.0;
        viscous_flux<D, double, double>(ph, U, E, G);
#pragma unroll
        for (int j = 0; j < D; ++j) {
#pragma unroll
          for (int k = 0; k < NV; ++k) {
            double s = 0.0;
#pragma unroll
            for (int jj = 0; jj < D; ++jj) s += Gm[j][jj] * G[jj][k];
            out[((j * (D + 1) + 1 + i) * NV + k) * NV + l] = -s * wq;
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------- face flux Jacobians
// One thread per (element, face, face point): forward differences of Eq. 31
// of the own-side numerical flux (outward normal of the element) with respect
// to the own trace (JmW, weighted by w^G |J^G|, feeds the diagonal block) and
// to the neighbour trace (Jp, stored for the off-diagonal product), at fixed
// trace gradients.
template <int D, int N, int Q, typename TJ>
__global__ __launch_bounds__(128) void k_pc_face(const double* __restrict__ u, const int* __restrict__ nbr,
                                                 const double* __restrict__ geo,
                          const double* __restrict__ beta, const double* __restrict__ tables, Phys ph, long n_elem,
                          const double* __restrict__ chi_dev, double* __restrict__ JmW, TJ* __restrict__ Jp,
                          long e0, const int* __restrict__ bc_kind, const double* __restrict__ bc_state,
                          const double* __restrict__ fg, const double* __restrict__ bc_field) {
  using S = Shape<D, N, Q>;
  constexpr int NV = S::NV, NQF = S::NQF, NF = S::NF;
  __shared__ double st[S::TAB];
  Tab tb = load_tables<N, Q>(tables, st);
  __syncthreads();
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n_elem * NF * NQF) return;
  const int p = gid % NQF;
  const int f = (gid / NQF) % NF;
  const long e = e0 + gid / (NQF * NF);
  const long en = nbr[e * NF + f];
  const int ax = f >> 1, s = f & 1;
  StateIn in{u, 0.0};
  double Uo[NV], Un[NV], go[D][NV], gn[D][NV];
  constexpr int CF = D * D + D + 1;
  const double* fgo = fg ? fg + (e * NF + f) * (long)CF * NQF : nullptr;
  trace_point<D, N, Q>(tb, in, e, geo + e * S::GEO, f, p, Uo, go, fgo);
  double nrm[D];
  double wf;
  if (fgo) {
#pragma unroll
    for (int j = 0; j < D; ++j) nrm[j] = fgo[(D * D + j) * NQF + p];
    wf = fgo[(D * D + D) * NQF + p];
  } else {
#pragma unroll
    for (int j = 0; j < D; ++j) nrm[j] = (j == ax) ? (s == 1 ? 1.0 : -1.0) : 0.0;
    wf = geo[e * S::GEO + D + 2 + ax] * tb.w[p % Q];
    if (D == 3) wf *= tb.w[p / Q];
  }
  const double b = beta[e * NF + f];
  const long base = ((e * NF + f) * NQF + p) * NV * NV;
  const long lbase = gid * (long)(NV * NV);   // JmW holds the launch's elements
  double H0[NV], H1[NV];
  double Sd[D][NV];   // not written (the Jacobian needs no test-gradient terms)
  if (en < 0) {
    // boundary face: the condition is inside the differenced flux (Eq. 31);
    // no neighbour, so no off-diagonal Jacobian
    const int bid = -en - 1;
    const int kind = bc_kind[bid];
    const double* Uinf = bc_state + bid * NV;
    double UD[NV];
    if (kind == BC_DIRICHLET) {
      const double* g = bc_field + (e * NF + f) * (long)NV * NQF + p;
#pragma unroll
      for (int v = 0; v < NV; ++v) UD[v] = g[v * NQF];
      Uinf = UD;
    }
    boundary_flux<D, false>(ph, kind, Uo, go, nrm, b, Uinf, H0, Sd);
    for (int l = 0; l < NV; ++l) {
      const double chi = chi_dev[l];
      const double save = Uo[l];
      Uo[l] = save + chi;
      boundary_flux<D, false>(ph, kind, Uo, go, nrm, b, Uinf, H1, Sd);
      Uo[l] = save;
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        JmW[lbase + k * NV + l] = wf * ((H1[k] - H0[k]) / chi);
        Jp[base + k * NV + l] = (TJ)0.0;
      }
    }
    return;
  }
  trace_point<D, N, Q>(tb, in, en, geo + en * S::GEO, f ^ 1, p, Un, gn,
                       fg ? fg + (en * NF + (f ^ 1)) * (long)CF * NQF : nullptr);
  face_flux<D, false>(ph, Uo, Un, go, gn, nrm, b, H0, Sd);
  for (int l = 0; l < NV; ++l) {
    const double chi = chi_dev[l];
    double save = Uo[l];
    Uo[l] = save + chi;
    face_flux<D, false>(ph, Uo, Un, go, gn, nrm, b, H1, Sd);
    Uo[l] = save;
#pragma unroll
    for (int k = 0; k < NV; ++k) JmW[lbase + k * NV + l] = wf * ((H1[k] - H0[k]) / chi);
    save = Un[l];
    Un[l] = save + chi;
    face_flux<D, false>(ph, Uo, Un, go, gn, nrm, b, H1, Sd);
    Un[l] = save;
#pragma unroll
    for (int k = 0; k < NV; ++k) Jp[base + k * NV + l] = (TJ)((H1[k] - H0[k]) / chi);
  }
}

// ---------------------------------------------------------------- block assembly
// Sum-factorised assembly: one workgroup per (element, k, l) computes the
// whole NM x NM sub-block A_kl.  The volume term
//   A_kl[m][n] = sum_j sum_b sum_q f_j(q, m) W_jb(q) g_b(q, n),
// f_j = d phi_m / d xi_j, g_0 = phi_n, g_{1+i} = d phi_n / d xi_i, is
// contracted one tensor direction at a time (the 1D factors are B or its
// derivative Dq per direction); terms that continue with the same 1D
// factors are merged after each direction, so the cost per sub-block is
// about N^(2d) Q instead of the dense N^(2d) Q^d.  The partial sums of each
// direction j go straight into the output block (coalesced over rows), so
// no per-thread accumulators are kept.  The own-side face term of face f
// (normal axis a, side s) factorises as phi_s(m_a) phi_s(n_a) times a
// contraction over the tangential face points; the last pass adds it and
// writes D = I - dt_a / |J| A (boxes) or D = M_e - dt_a A (curved) column-
// major into Dm[e][col][row].
template <int D, int N, int Q>
struct AssembleSF {
  using S = Shape<D, N, Q>;
  static constexpr int NM = S::NM, NQ = S::NQ, NQF = S::NQF, NF = S::NF;
  static constexpr int NM2 = NM * NM;
  static constexpr int NTR = ((NM2 / 16 + 63) / 64) * 64;
  static constexpr int NT = NTR < 64 ? 64 : (NTR > 512 ? 512 : NTR);
  static constexpr int SW = D * (D + 1) * NQ;                                 // W_jb(q)
  static constexpr int S1 = (D == 3) ? 3 * N * N * Q * Q : 2 * N * N * Q;     // after the first direction
  static constexpr int S2 = (D == 3) ? 2 * N * N * N * N * Q : 0;             // after the second (3D)
  static constexpr int FF = NF * ((D == 3) ? N * N * N * N : N * N);          // face blocks
  static constexpr int FG = (D == 3) ? N * N * Q : 0;                         // face scratch
  static constexpr int WORK = (S1 + S2) > (FF + FG) ? (S1 + S2) : (FF + FG);
};

template <int D, int N, int Q>
__global__ __launch_bounds__((AssembleSF<D, N, Q>::NT)) void k_pc_assemble_sf(
    const double* __restrict__ Wt, const double* __restrict__ JmW, const double* __restrict__ geo,
    const double* __restrict__ tables, double dt_a, long n_elem, double* __restrict__ Dm, long e0,
    const double* __restrict__ mass, int ld) {
  using S = Shape<D, N, Q>;
  using A = AssembleSF<D, N, Q>;
  constexpr int NV = S::NV, NM = S::NM, NQ = S::NQ, NQF = S::NQF, NF = S::NF, NB = S::NB;
  constexpr int PER_Q = D * (D + 1) * NV * NV;
  constexpr int NT = A::NT;
  __shared__ double st[S::TAB];
  __shared__ double sW[A::SW];
  __shared__ double wk[A::WORK];
  __shared__ double sJ[NF * NQF];
  Tab tb = load_tables<N, Q>(tables, st);
  const long blk = blockIdx.x;
  if (blk / (NV * NV) >= n_elem) return;
  const long le = blk / (NV * NV);   // Wt, JmW and Dm hold the launch's elements
  const long e = e0 + le;
  const int kl = blk % (NV * NV);
  const int k = kl / NV, l = kl % NV;
  const int tid = threadIdx.x;
  for (int i = tid; i < A::SW; i += NT) {
    const int q = i % NQ, jb = i / NQ;
    sW[i] = Wt[(le * NQ + q) * (long)PER_Q + (jb * NV + k) * NV + l];
  }
  for (int i = tid; i < NF * NQF; i += NT) sJ[i] = JmW[(le * NF * NQF + i) * (long)NV * NV + k * NV + l];
  const double* B = tb.B;     // B[q * N + m]
  const double* Dq = tb.Dq;
  // output sub-block: entry (m, n) of A_kl at Dm[e][l NM + n][k NM + m]
  // (columns ld apart, ld >= nb)
  double* out = Dm + le * (long)NB * ld + (long)(l * NM) * ld + k * NM;
  __syncthreads();
  for (int j = 0; j < D; ++j) {
    const double* F1 = (j == 0) ? Dq : B;
    const double* F2 = (j == 1) ? Dq : B;
    const double* W0 = sW + (j * (D + 1)) * NQ;
    if constexpr (D == 3) {
      const double* F3 = (j == 2) ? Dq : B;
      double* s1a = wk;                          // [m1][n1][q2 q3]: g = (B|Dq, B, B)
      double* s1b = wk + N * N * Q * Q;          // (B, Dq, B)
      double* s1c = wk + 2 * N * N * Q * Q;      // (B, B, Dq)
      double* s2b = wk + A::S1;                  // [m1][n1][m2][n2][q3]: g3 = B
      double* s2d = s2b + N * N * N * N * Q;     // g3 = Dq
      for (int it = tid; it < N * N * Q * Q; it += NT) {
        const int r = it % (Q * Q), n1 = (it / (Q * Q)) % N, m1 = it / (Q * Q * N);
        double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1) {
          const double f = F1[q1 * N + m1];
          const int q = q1 + Q * r;
          a += f * (B[q1 * N + n1] * W0[q] + Dq[q1 * N + n1] * W0[NQ + q]);
          b += f * B[q1 * N + n1] * W0[2 * NQ + q];
          c += f * B[q1 * N + n1] * W0[3 * NQ + q];
        }
        s1a[it] = a;
        s1b[it] = b;
        s1c[it] = c;
      }
      __syncthreads();
      for (int it = tid; it < N * N * N * N * Q; it += NT) {
        const int q3 = it % Q, n2 = (it / Q) % N, m2 = (it / (Q * N)) % N, mn1 = it / (Q * N * N);
        double b3 = 0.0, d3 = 0.0;
#pragma unroll
        for (int q2 = 0; q2 < Q; ++q2) {
          const double f = F2[q2 * N + m2];
          const int o = mn1 * Q * Q + q2 + Q * q3;
          b3 += f * (B[q2 * N + n2] * s1a[o] + Dq[q2 * N + n2] * s1b[o]);
          d3 += f * B[q2 * N + n2] * s1c[o];
        }
        s2b[it] = b3;
        s2d[it] = d3;
      }
      __syncthreads();
      for (int oi = tid; oi < NM * NM; oi += NT) {
        const int m = oi % NM, n = oi / NM;
        const int m1 = m % N, m2 = (m / N) % N, m3 = m / (N * N);
        const int n1 = n % N, n2 = (n / N) % N, n3 = n / (N * N);
        const int base = (((m1 * N + n1) * N + m2) * N + n2) * Q;
        double t = 0.0;
#pragma unroll
        for (int q3 = 0; q3 < Q; ++q3)
          t += F3[q3 * N + m3] * (B[q3 * N + n3] * s2b[base + q3] + Dq[q3 * N + n3] * s2d[base + q3]);
        double* o = out + (long)n * ld + m;
        *o = (j == 0) ? t : *o + t;
      }
      __syncthreads();
    } else {
      double* s1a = wk;                // [m1][n1][q2]: g = (B|Dq, B)
      double* s1b = wk + N * N * Q;    // (B, Dq)
      for (int it = tid; it < N * N * Q; it += NT) {
        const int q2 = it % Q, n1 = (it / Q) % N, m1 = it / (Q * N);
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1) {
          const double f = F1[q1 * N + m1];
          const int q = q1 + Q * q2;
          a += f * (B[q1 * N + n1] * W0[q] + Dq[q1 * N + n1] * W0[NQ + q]);
          b += f * B[q1 * N + n1] * W0[2 * NQ + q];
        }
        s1a[it] = a;
        s1b[it] = b;
      }
      __syncthreads();
      for (int oi = tid; oi < NM * NM; oi += NT) {
        const int m = oi % NM, n = oi / NM;
        const int m1 = m % N, m2 = m / N, n1 = n % N, n2 = n / N;
        const int base = (m1 * N + n1) * Q;
        double t = 0.0;
#pragma unroll
        for (int q2 = 0; q2 < Q; ++q2)
          t += F2[q2 * N + m2] * (B[q2 * N + n2] * s1a[base + q2] + Dq[q2 * N + n2] * s1b[base + q2]);
        double* o = out + (long)n * ld + m;
        *o = (j == 0) ? t : *o + t;
      }
      __syncthreads();
    }
  }
  // own-side face terms: tangential contraction per face, then the normal factors
  constexpr int FB = (D == 3) ? N * N * N * N : N * N;
  double* ff = wk;
  for (int f = 0; f < NF; ++f) {
    const double* jw = sJ + f * NQF;
    if constexpr (D == 3) {
      double* g = wk + A::FF;                  // [mt0][nt0][p1]
      for (int it = tid; it < N * N * Q; it += NT) {
        const int p1 = it % Q, n0 = (it / Q) % N, m0 = it / (Q * N);
        double t = 0.0;
#pragma unroll
        for (int p0 = 0; p0 < Q; ++p0) t += B[p0 * N + m0] * B[p0 * N + n0] * jw[p0 + Q * p1];
        g[it] = t;
      }
      __syncthreads();
      for (int it = tid; it < FB; it += NT) {
        const int n1 = it % N, m1 = (it / N) % N, mn0 = it / (N * N);
        double t = 0.0;
#pragma unroll
        for (int p1 = 0; p1 < Q; ++p1) t += B[p1 * N + m1] * B[p1 * N + n1] * g[mn0 * Q + p1];
        ff[f * FB + it] = t;                   // [mt0][nt0][mt1][nt1]
      }
      __syncthreads();
    } else {
      for (int it = tid; it < FB; it += NT) {
        const int n0 = it % N, m0 = it / N;
        double t = 0.0;
#pragma unroll
        for (int p = 0; p < Q; ++p) t += B[p * N + m0] * B[p * N + n0] * jw[p];
        ff[f * FB + it] = t;                   // [mt][nt]
      }
    }
  }
  __syncthreads();
  const double sc = mass ? dt_a : dt_a * geo[e * S::GEO + D + 1];
  for (int oi = tid; oi < NM * NM; oi += NT) {
    const int m = oi % NM, n = oi / NM;
    int mi[3] = {0, 0, 0}, ni[3] = {0, 0, 0};
    split<D, N>(m, mi);
    split<D, N>(n, ni);
    double fsum = 0.0;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int ax = f >> 1, sd = f & 1;
      int t[2] = {0, 0};
      tang_axes<D>(ax, t);
      const double nf = tb.phiE[sd * N + mi[ax]] * tb.phiE[sd * N + ni[ax]];
      const int fi = (D == 3) ? ((mi[t[0]] * N + ni[t[0]]) * N + mi[t[1]]) * N + ni[t[1]] : mi[t[0]] * N + ni[t[0]];
      fsum += nf * ff[f * FB + fi];
    }
    double* o = out + (long)n * ld + m;
    const double dg = mass ? ((k == l) ? mass[(e * NM + m) * (long)mass_ld(NM) + n] : 0.0)
                           : ((k == l && m == n) ? 1.0 : 0.0);
    *o = dg - sc * (*o - fsum);
  }
}

// ---------------------------------------------------------------- blocked Gauss-Jordan inverse
// In-place inversion of each nb x nb block (column-major, columns ld apart,
// blocks nb ld apart) by Gauss-Jordan elimination with partial pivoting,
// processed in column panels of width KB held in LDS: the panel is eliminated
// on all rows (one thread per row, one workgroup barrier per pivot: a row
// stays where it is inside the panel, the pivot row is scaled by its own
// thread at the next step, and the row swaps of the panel are derived from
// the pivots chosen afterwards), then the other columns take the panel's row
// swaps and the rank-KB update x <- x(non-pivot rows) + Panel * x(pivot rows)
// on FP64 MFMA; finally the columns are unscrambled in reverse order of the
// swaps.  status[e] = 1 if a zero pivot was met.
template <typename T, int KB>
__global__ void k_gj_invert(T* __restrict__ A, int nb, int ld, long n_elem, int* __restrict__ status) {
  static_assert(sizeof(T) == 8, "the trailing update runs on FP64 MFMA");
  extern __shared__ unsigned char smraw[];
  T* Pan = reinterpret_cast<T*>(smraw);                       // [nb][KB+1]
  int* piv = reinterpret_cast<int*>(Pan + (size_t)nb * (KB + 1));
  int* perm = piv + nb;
  T* redv = reinterpret_cast<T*>(perm + nb);                   // [2][32] per-wave pivot candidates (by step parity)
  int* redi = reinterpret_cast<int*>(redv + 64);               // [2][32]
  int* srow = redi + 64;                                       // [2 KB] rows the panel's swaps touch
  int* nsrow = srow + 2 * KB;                                  // [1] their number
  int* pphys = nsrow + 1;                                      // [KB] the panel's pivot rows (rows as loaded)
  const long e = blockIdx.x;
  if (e >= n_elem) return;
  T* Ae = A + e * (long)nb * ld;
  const int r = threadIdx.x;
  const int nw = (blockDim.x + 63) / 64;
  const int lane = r & 63, wid = r >> 6;
  int bad = 0;
  for (int k0 = 0; k0 < nb; k0 += KB) {
    const int kb = (nb - k0) < KB ? (nb - k0) : KB;
    if (r < nb)
      for (int c = 0; c < kb; ++c) Pan[r * (KB + 1) + c] = Ae[(long)(k0 + c) * ld + r];
    // candidates: the rows from k0 on that are not yet pivots of this panel
    bool elig = r < nb && r >= k0;
    int prev = -1;        // the previous step's pivot row, scaled at this step by its thread
    T prev_inv = (T)0;
    for (int t = 0; t < kb; ++t) {
      // pivot candidate of this thread's own row (rows are only ever written
      // by their own thread), reduced over the wave
      T best = (T)-1;
      int bi = nb;
      if (elig) { T x = Pan[r * (KB + 1) + t]; best = x < (T)0 ? -x : x; bi = r; }
      for (int off = 32; off > 0; off >>= 1) {
        T ob = __shfl_down(best, off, 64);
        int oi = __shfl_down(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      T* rv = redv + (t & 1) * 32;
      int* ri = redi + (t & 1) * 32;
      if (lane == 0) { rv[wid] = best; ri[wid] = bi; }
      __syncthreads();   // the wave candidates, and every row's update of the previous step
      if (r == prev) {
        // the previous pivot row, which no other thread reads at this step
        for (int c = 0; c < kb; ++c)
          Pan[r * (KB + 1) + c] = (c == t - 1) ? prev_inv : Pan[r * (KB + 1) + c] * prev_inv;
      }
      // the pivot: largest |value| (smallest row on ties), the same in every thread
      T b = rv[0];
      int p = ri[0];
      for (int w = 1; w < nw; ++w)
        if (rv[w] > b || (rv[w] == b && ri[w] < p)) { b = rv[w]; p = ri[w]; }
      if (!(b > (T)0)) bad = 1;
      const T pinv = bad ? (T)0 : (T)1 / Pan[p * (KB + 1) + t];
      if (r == 0) pphys[t] = p;
      // eliminate column t from every other row with the scaled pivot row
      // (its entries scaled here; the row itself is scaled at the next step)
      if (r < nb && r != p) {
        const T fct = Pan[r * (KB + 1) + t];
        for (int c = 0; c < kb; ++c) {
          if (c == t) continue;
          Pan[r * (KB + 1) + c] -= fct * (Pan[p * (KB + 1) + c] * pinv);
        }
        Pan[r * (KB + 1) + t] = -fct * pinv;
      }
      if (r == p) { elig = false; prev_inv = pinv; }
      prev = p;
    }
    __syncthreads();   // every read of the last pivot row
    if (r == prev)
      for (int c = 0; c < kb; ++c)
        Pan[r * (KB + 1) + c] = (c == kb - 1) ? prev_inv : Pan[r * (KB + 1) + c] * prev_inv;
    if (r < nb) perm[r] = r;
    __syncthreads();
    if (r == 0) {
      // the equivalent row swaps: step t moves its pivot row (at the position
      // the earlier swaps left it) to position k0 + t; perm[pos] = the row
      // (as loaded) that ends at pos
      for (int t = 0; t < kb; ++t) {
        int q = pphys[t];
        for (int u = 0; u < t; ++u) {
          const int a0 = k0 + u, a1 = piv[k0 + u];
          if (q == a0) q = a1;
          else if (q == a1) q = a0;
        }
        piv[k0 + t] = q;
        const int k = k0 + t;
        int tmp = perm[k]; perm[k] = perm[q]; perm[q] = tmp;
      }
      // every row a swap moved: the pivot range and the rows below it that
      // were exchanged with it (rows below only ever receive pivot-range rows)
      int ns = 0;
      for (int t = 0; t < kb; ++t) srow[ns++] = k0 + t;
      for (int t = 0; t < kb; ++t) {
        const int p = piv[k0 + t];
        if (p >= k0 + kb) {
          bool seen = false;
          for (int i = kb; i < ns; ++i) seen = seen || srow[i] == p;
          if (!seen) srow[ns++] = p;
        }
      }
      *nsrow = ns;
    }
    __syncthreads();
    // write the panel back in the swapped row order
    if (r < nb) {
      const int src = perm[r];
      for (int c = 0; c < kb; ++c) Ae[(long)(k0 + c) * ld + r] = Pan[src * (KB + 1) + c];
    }
    // FP64 MFMA trailing update over tiles of 16 columns, one tile per wave
    // at a time: (a) the panel's row swaps are applied to the tile's
    // columns in memory (each touched row's source read before any write),
    // so that (c) reads x'(r) = x(perm[r]); (b) the pivot rows x'(k0 + t)
    // of the 16 columns are held as the A operand; (c) per 16-row tile,
    // x(r) <- [r not a pivot row] x'(r) + sum_t Panel[r][t] x'(k0 + t) by
    // v_mfma_f64_16x16x4 (lane l: A[l%16][l/16], B[l/16][l%16], D[l/16 + 4v][l%16]).
    typedef double dgj_d4 __attribute__((ext_vector_type(4)));
    constexpr int NK = (KB + 3) / 4;
    const int ns = *nsrow;
    const int ncol = nb - kb;
    const int ntile = (ncol + 15) >> 4;
    const int nrt = (nb + 15) >> 4;
    const int li = lane & 15, lq = lane >> 4;
    for (int jt = wid; jt < ntile; jt += nw) {
      double tmp[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int idx = lane + 64 * i;
        tmp[i] = 0.0;
        if (idx < 16 * ns) {
          const int c = idx / ns, sidx = idx - c * ns;
          const int jj = jt * 16 + c;
          if (jj < ncol) tmp[i] = Ae[(long)(jj < k0 ? jj : jj + kb) * ld + perm[srow[sidx]]];
        }
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int idx = lane + 64 * i;
        if (idx < 16 * ns) {
          const int c = idx / ns, sidx = idx - c * ns;
          const int jj = jt * 16 + c;
          if (jj < ncol) Ae[(long)(jj < k0 ? jj : jj + kb) * ld + srow[sidx]] = tmp[i];
        }
      }
      __threadfence_block();
      const int jjA = jt * 16 + li;
      const bool okA = jjA < ncol;
      const T* colA = Ae + (long)(okA ? (jjA < k0 ? jjA : jjA + kb) : 0) * ld;
      double a[NK];
#pragma unroll
      for (int kk = 0; kk < NK; ++kk) {
        const int t = 4 * kk + lq;
        a[kk] = (okA && t < kb) ? colA[k0 + t] : 0.0;
      }
      T* colD[4];
      bool okD[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int jj = jt * 16 + lq + 4 * v;
        okD[v] = jj < ncol;
        colD[v] = Ae + (long)(okD[v] ? (jj < k0 ? jj : jj + kb) : 0) * ld;
      }
      // RB row tiles at a time: all their loads in flight together, then
      // RB independent MFMA chains, then the stores
      constexpr int RB = 4;
      for (int rt0 = 0; rt0 < nrt; rt0 += RB) {
        dgj_d4 acc[RB];
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          const int n = (rt0 + b) * 16 + li;
          const bool rowok = n < nb;
          const bool piv_row = n >= k0 && n < k0 + kb;
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[b][v] = (okD[v] && rowok && !piv_row) ? colD[v][n] : 0.0;
        }
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          const int n = (rt0 + b) * 16 + li;
          const bool rowok = n < nb;
          const int pn = rowok ? perm[n] : 0;   // the panel row (as loaded) at position n
#pragma unroll
          for (int kk = 0; kk < NK; ++kk) {
            const int t = 4 * kk + lq;
            const double bv = (rowok && t < kb) ? Pan[pn * (KB + 1) + t] : 0.0;
            acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk], bv, acc[b], 0, 0, 0);
          }
        }
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          const int n = (rt0 + b) * 16 + li;
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (okD[v] && n < nb) colD[v][n] = acc[b][v];
        }
      }
    }
    __syncthreads();
  }
  // unscramble columns
  for (int k = nb - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k && r < nb) {
      T a0 = Ae[(long)k * ld + r], a1 = Ae[(long)p * ld + r];
      Ae[(long)k * ld + r] = a1;
      Ae[(long)p * ld + r] = a0;
    }
    __syncthreads();
  }
  if (r == 0) status[e] = bad;
}

// ---------------------------------------------------------------- apply
template <typename T> __device__ __forceinline__ float to_f(T x) { return (float)x; }
template <> __device__ __forceinline__ float to_f<__hip_bfloat16>(__hip_bfloat16 x) { return __bfloat162float(x); }

template <typename T> struct AccT { using type = float; };
template <> struct AccT<double> { using type = double; };

template <typename T>
__device__ __forceinline__ typename AccT<T>::type ld_acc(const T* p) { return (typename AccT<T>::type)to_f<T>(*p); }
template <>
__device__ __forceinline__ double ld_acc<double>(const double* p) { return *p; }

template <typename T> __device__ __forceinline__ double jp_ld(const T* p) { return (double)(*p); }

// Column stride of the stored block inverses, so that the sweep reads them
// with 16-byte loads: columns of at least 1 KB start on a 128-byte boundary
// (whole cache lines, none shared by two columns: the sweep streams the
// blocks with the nontemporal hint, and a shared line was fetched twice),
// smaller ones on a 16-byte boundary (padding rows are zero or unused; e.g.
// 3D P = 4: nb = 625 -> 640 in every precision; 3D P = 3: 320 unchanged).
template <typename T> __host__ __device__ constexpr int stored_ld(int nb) {
  const int g = nb * (int)sizeof(T) >= 1024 ? 128 / (int)sizeof(T) : 16 / (int)sizeof(T);
  return (nb + g - 1) / g * g;
}

// 16-byte load of 16/sizeof(T) consecutive entries (p 16-byte aligned),
// widened to the accumulation type.  The block inverses are streamed once
// per sweep with no reuse, so the loads carry the nontemporal hint (FP64
// sweep on 16^3 P = 3: 0.58 -> 0.51 ms).
typedef float dgj_f4 __attribute__((ext_vector_type(4)));
typedef unsigned dgj_u4 __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ void ld16(const T* p, typename AccT<T>::type* v);
template <>
__device__ __forceinline__ void ld16<double>(const double* p, double* v) {
  const dgj_d2 x = __builtin_nontemporal_load(reinterpret_cast<const dgj_d2*>(p));
  v[0] = x[0];
  v[1] = x[1];
}
template <>
__device__ __forceinline__ void ld16<float>(const float* p, float* v) {
  const dgj_f4 x = __builtin_nontemporal_load(reinterpret_cast<const dgj_f4*>(p));
  v[0] = x[0];
  v[1] = x[1];
  v[2] = x[2];
  v[3] = x[3];
}
template <>
__device__ __forceinline__ void ld16<__hip_bfloat16>(const __hip_bfloat16* p, float* v) {
  const dgj_u4 x = __builtin_nontemporal_load(reinterpret_cast<const dgj_u4*>(p));
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[2 * i] = __uint_as_float(x[i] << 16);              // bfloat16 -> float: the high half of the bits
    v[2 * i + 1] = __uint_as_float(x[i] & 0xffff0000u);
  }
}

// One BRJ sweep for element e (one workgroup, blockDim >= nb):
//   r = q - (L+U) qold   (skipped when first),  out = omega Dinv r + (1-omega) qold.
// (L+U) qold = -dt_a / |J| sum_f -(B^G_f)^T diag(w^G|J^G| Jp (B^G_f' qold_nbr)).
// Curved elements (fg): q holds M_e q, Dinv holds (M_e - dt_a A_e)^-1, the
// face weights are per point and r = M_e q + dt_a sum_f (...), which equals
// M_e times the r above (M_e^-1 is not applied).
template <int D, int N, int Q, int NT, typename T, typename TJ>
__global__ __launch_bounds__(NT) void k_brj_sweep(const double* __restrict__ q, const double* __restrict__ qold,
                                                   double* __restrict__ out, const T* __restrict__ Dinv,
                                                   const TJ* __restrict__ Jp, const int* __restrict__ nbr,
                                                   const double* __restrict__ geo, const double* __restrict__ tables,
                                                   double dt_a, double omega, int first, long n_elem,
                                                   const int* __restrict__ inst, const double* __restrict__ dtav,
                                                   const int* __restrict__ active, const double* __restrict__ fg) {
  using S = Shape<D, N, Q>;
  constexpr int NV = S::NV, NM = S::NM, NQF = S::NQF, NMF = S::NMF, NF = S::NF, NB = S::NB;
  __shared__ double st[S::TAB];
  __shared__ double sr[NB];
  __shared__ double tvf[NF * NV * NMF];
  __shared__ double tpt[NF * NV * NQF];
  __shared__ double flx[NF * NV * NQF];
  __shared__ long snb[NF];
  Tab tb = load_tables<N, Q>(tables, st);
  const long e = blockIdx.x;
  if (e >= n_elem) return;
  if (inst) {
    const int ii = inst[e];
    if (active && !active[ii]) return;
    dt_a = dtav[ii];
  }
  const int tid = threadIdx.x;
  const double* g = geo + e * S::GEO;
  for (int i = tid; i < NB; i += NT) sr[i] = q[e * NB + i];
  if (tid < NF) snb[tid] = nbr[e * NF + tid];
  __syncthreads();
  if (!first) {
    // all faces at once (boundary faces have no neighbour block and add 0):
    // neighbour trace in face modes, at the face points, times the stored
    // flux Jacobian and weight, lifted back onto this element's modes
    for (int it = tid; it < NF * NV * NMF; it += NT) {
      const int tm = it % NMF, v = (it / NMF) % NV, f = it / (NMF * NV);
      const long en = snb[f];
      double sv = 0.0;
      if (en >= 0) {
        const int ax = f >> 1, sg = 1 - (f & 1);
#pragma unroll
        for (int ia = 0; ia < N; ++ia) sv += tb.phiE[sg * N + ia] * qold[en * NB + v * NM + mode_of<D, N>(ax, ia, tm)];
      }
      tvf[it] = sv;
    }
    __syncthreads();
    for (int it = tid; it < NF * NV * NQF; it += NT) {
      const int p = it % NQF, f = it / (NQF * NV);
      const int b0 = p % Q, b1 = (D == 3) ? p / Q : 0;
      const double* tv = tvf + (it / NQF) * NMF;
      double val = 0.0;
      if (snb[f] >= 0)
        for (int tm = 0; tm < NMF; ++tm) {
          const int j0 = tm % N, j1 = (D == 3) ? tm / N : 0;
          val += tb.B[b0 * N + j0] * ((D == 3) ? tb.B[b1 * N + j1] : 1.0) * tv[tm];
        }
      tpt[it] = val;
    }
    __syncthreads();
    for (int it = tid; it < NF * NV * NQF; it += NT) {
      const int p = it % NQF, k = (it / NQF) % NV, f = it / (NQF * NV);
      double val = 0.0;
      if (snb[f] >= 0) {
        const int ax = f >> 1;
        const TJ* J = Jp + ((e * NF + f) * NQF + p) * NV * NV + k * NV;
        const double* tp = tpt + f * NV * NQF + p;
        double sacc2 = 0.0;
#pragma unroll
        for (int l = 0; l < NV; ++l) sacc2 += jp_ld<TJ>(J + l) * tp[l * NQF];
        double wf;
        if (fg) {
          wf = fg[((e * NF + f) * (long)(D * D + D + 1) + D * D + D) * NQF + p];
        } else {
          wf = g[D + 2 + ax] * tb.w[p % Q];
          if (D == 3) wf *= tb.w[p / Q];
        }
        val = sacc2 * wf;
      }
      flx[it] = val;
    }
    __syncthreads();
    // r = q - (L+U) qold, (L+U) qold = -dt_a / |J| sacc (curved: times M_e),
    // sacc = -sum_f phi_s(m_ax) sum_p B B flx
    const double sc = fg ? dt_a : dt_a * g[D + 1];
    for (int it = tid; it < NB; it += NT) {
      const int m = it % NM, v = it / NM;
      int mi[3] = {0, 0, 0};
      split<D, N>(m, mi);
      double sacc = 0.0;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        if (snb[f] < 0) continue;
        const int ax = f >> 1, s = f & 1;
        int tax[2] = {0, 0};
        tang_axes<D>(ax, tax);
        const int j0 = mi[tax[0]], j1 = (D == 3) ? mi[tax[1]] : 0;
        const double* fl = flx + (f * NV + v) * NQF;
        double s2 = 0.0;
        for (int p = 0; p < NQF; ++p) {
          const int b0 = p % Q, b1 = (D == 3) ? p / Q : 0;
          s2 += tb.B[b0 * N + j0] * ((D == 3) ? tb.B[b1 * N + j1] : 1.0) * fl[p];
        }
        sacc -= tb.phiE[s * N + mi[ax]] * s2;
      }
      sr[it] = sr[it] + sc * sacc;
    }
    __syncthreads();
  }
  using A = typename AccT<T>::type;
  constexpr int LD = stored_ld<T>(NB);                     // column stride of the stored blocks
  const T* De = Dinv + e * (long)NB * LD;
  constexpr int VW = 16 / (int)sizeof(T);                 // rows per 16-byte load
  if constexpr (LD % VW == 0 && (LD * (int)sizeof(T)) % 16 == 0) {
    // every thread busy: VW rows by one 16-byte load per column, the
    // columns split into SEG segments, partial sums added in LDS in a fixed
    // order; the padding rows of an odd FP64 block (row nb) are summed and
    // dropped
    constexpr int NR = LD / VW;
    constexpr int SEG = NT / NR >= 1 ? NT / NR : 1;
    __shared__ A part[SEG * LD];
    for (int t = tid; t < SEG * NR; t += NT) {
      const int rg = t % NR, sg = t / NR;
      const int c0 = sg * NB / SEG, c1 = (sg + 1) * NB / SEG;
      A acc[VW];
#pragma unroll
      for (int i = 0; i < VW; ++i) acc[i] = (A)0;
#pragma unroll 4
      for (int c = c0; c < c1; ++c) {
        A v[VW];
        ld16<T>(De + (long)c * LD + rg * VW, v);
        const A x = (A)sr[c];
#pragma unroll
        for (int i = 0; i < VW; ++i) acc[i] += v[i] * x;
      }
#pragma unroll
      for (int i = 0; i < VW; ++i) part[sg * LD + rg * VW + i] = acc[i];
    }
    __syncthreads();
    for (int row = tid; row < NB; row += NT) {
      A acc = (A)0;
#pragma unroll
      for (int sg = 0; sg < SEG; ++sg) acc += part[sg * LD + row];
      double res = omega * (double)acc;
      if (!first && omega != 1.0) res += (1.0 - omega) * qold[e * NB + row];
      out[e * NB + row] = res;
    }
  } else {
    for (int row = tid; row < NB; row += NT) {
      A acc = (A)0;
      for (int c = 0; c < NB; ++c) acc += ld_acc<T>(De + (long)c * LD + row) * (A)sr[c];
      double res = omega * (double)acc;
      if (!first && omega != 1.0) res += (1.0 - omega) * qold[e * NB + row];
      out[e * NB + row] = res;
    }
  }
}

}  // namespace dgj
