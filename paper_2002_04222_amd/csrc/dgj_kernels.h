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
//   curved elements (instead of geo): vg[e][c][q] (c < D*D: d xi_k/d x_j at
//           c = k*D + j; c = D*D: w_q |J_q|), fg[e][f][c][p] (c < D*D: d xi/d x;
//           D*D + j: outward unit normal; D*D + D: w^G_p |J^G_p|), minv[e][n][m]
//           (column-major, columns mass_ld(NM) apart).
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
  const double* u;    // the state the residual is evaluated at (the matvec's u + eps v)
  double eps;         // the matvec's eps (mode RES_JV)
  __device__ __forceinline__ double operator()(long i) const { return u[i]; }
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
  // boundary conditions: kind and freestream state per boundary id
  // (face_nbr = -(id + 1))
  const int* bc_kind;
  const double* bc_state;
  // Dirichlet ghost states at the face points, bc_field[e][NF][NV][NQF]
  // (read at faces whose id has the Dirichlet kind; may be null otherwise)
  const double* bc_field;
  // modal source [e][NV][NM] added to M^-1 L (null: none)
  const double* src;
  // LDG: lifted jump gradient r_j at the volume points, rq[e][D][NV][NQ]
  // (written by k_ldg_lift; null for the interior-penalty form)
  double* ldg_r;
  // curved elements (all null for affine boxes): per-point metrics
  // vg[e][D*D+1][NQ], fg[e][NF][D*D+D+1][NQF] and the dense inverse mass
  // matrix minv[e][NM][mass_ld(NM)] (column-major, padding rows zero)
  const double* vg;
  const double* fg;
  const double* minv;
  // batches of independent instances: per-element instance index and
  // per-instance gas parameters, eps, dt a^mm and active flag (all null for
  // a single instance, which then uses ph, in.eps and dt_a)
  const int* inst;
  const Phys* phs;
  const double* epsv;
  const double* dtav;
  const int* active;
};

// instance-resolved view of ResArgs for element e; false if e's instance is inactive
struct ElemParams {
  Phys ph;
  StateIn in;
  double dt_a;
};
__device__ __forceinline__ bool elem_params(const ResArgs& a, long e, ElemParams& p) {
  p.ph = a.ph;
  p.in = a.in;
  p.dt_a = a.dt_a;
  if (a.inst) {
    const int i = a.inst[e];
    if (a.active && !a.active[i]) return false;
    p.ph = a.phs[i];
    if (a.epsv) p.in.eps = a.epsv[i];
    if (a.dtav) p.dt_a = a.dtav[i];
  }
  return true;
}

// ---------------------------------------------------------------- volume transform in LDS
// LDS sizes of the volume transform used by the preconditioner build.
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

// ---------------------------------------------------------------- curved mass inverse
// Column stride of the stored inverse mass matrices of curved elements: NM
// rounded up to even, so that every column starts on a 16-byte boundary
// (padding rows zero).
__host__ __device__ constexpr int mass_ld(int nm) { return (nm + 1) & ~1; }

typedef double dgj_d2 __attribute__((ext_vector_type(2)));

// R[v][m] = sum_n Minv[m][n] L[v][n] on one curved element (the M^-1 of
// Eq. 13), Minv column-major with columns mass_ld(NM) apart.  The NT threads
// form NS <= NSmax groups of whole wavefronts; a thread of group h owns the
// row pair (2p, 2p+1) and reads it from the columns n = h, h + NS, ... with
// 16-byte nontemporal loads, 16 in flight (the matrix is streamed once per
// evaluation with no reuse), and the groups' partial sums meet in
// part[NS][NV][NM] (LDS).  Every thread of the element calls it once L[v][n]
// (LDS) is complete; out(i, R, k) receives result i = v NM + m once, with k
// the ordinal of i among the thread's results (i = tid + k NT) for the first
// MINV_OUTK of them and -1 for the rest, so that a caller can use values it
// loaded ahead for them.
constexpr int MINV_OUTK = 4;

template <int NM, int NV, class Out>
__device__ __forceinline__ void mass_inv_dense(const double* __restrict__ Mi, const double* sL, double* part,
                                               int tid, int NT, int NSmax, Out out) {
  constexpr int NP = mass_ld(NM) / 2;
  constexpr int GP = ((NP + 63) / 64) * 64;
  const int NS = NT / GP < 1 ? 1 : (NT / GP > NSmax ? NSmax : NT / GP);
  const dgj_d2* M2 = reinterpret_cast<const dgj_d2*>(Mi);
  for (int t = tid; t < NS * GP; t += NT) {
    const int p = t % GP, h = t / GP;
    if (p >= NP) continue;
    double r0[NV], r1[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) r0[v] = r1[v] = 0.0;
    constexpr int BK = 16;
    for (int n0 = h; n0 < NM; n0 += BK * NS) {
      dgj_d2 w[BK];
#pragma unroll
      for (int k = 0; k < BK; ++k) {
        const int n = n0 + k * NS;
        w[k] = n < NM ? __builtin_nontemporal_load(M2 + (long)n * NP + p) : dgj_d2{0.0, 0.0};
      }
#pragma unroll
      for (int k = 0; k < BK; ++k) {
        const int n = n0 + k * NS;
        if (n < NM) {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const double x = sL[v * NM + n];
            r0[v] += w[k][0] * x;
            r1[v] += w[k][1] * x;
          }
        }
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      part[(h * NV + v) * NM + 2 * p] = r0[v];
      if (2 * p + 1 < NM) part[(h * NV + v) * NM + 2 * p + 1] = r1[v];
    }
  }
  __syncthreads();
  auto result = [&](int i, int k) {
    const int m = i % NM, v = i / NM;
    double R = 0.0;
    for (int h = 0; h < NS; ++h) R += part[(h * NV + v) * NM + m];
    out(i, R, k);
  };
#pragma unroll
  for (int k = 0; k < MINV_OUTK; ++k)
    if (tid + k * NT < NV * NM) result(tid + k * NT, k);
  for (int i = tid + MINV_OUTK * NT; i < NV * NM; i += NT) result(i, -1);
}

}  // namespace dgj
