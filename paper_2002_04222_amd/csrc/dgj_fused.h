// Fused DG residual R(u) = M^-1 L(u) of arxiv 2002.04222 (Sec. 3.1, Eq. 13)
// for the interior-penalty form: one workgroup per element, one kernel, and
// nothing in HBM but the state read (the element's own coefficients, and its
// face neighbours' through the L2) and the result written.
//
// Phases, separated by workgroup barriers, on LDS:
//   volume  sum-factorised values and reference gradients at the Gauss
//           points, pointwise H_j = F_j - G_j, transposed contraction with
//           the derivative bases -> sL (as the three-kernel path).
//   traces  modal face traces of both sides of every face: the value
//           sum_i phi_i(+-1) u and the normal derivative sum_i phi_i'(+-1) u
//           over the normal index (n^(d-1) coefficients each per variable),
//           computed from the modal coefficients of the element and of its
//           neighbour by the same code; then, tangentially, values and
//           reference gradients at the face points.
//   fluxes  one thread per face point: Riemann flux and interior-penalty
//           terms (Eq. 12) in the face's canonical orientation (left = the
//           element that meets it with side 1, its normal and weights), so
//           that the two elements of an interior face compute bitwise the
//           same flux and the element sums cancel exactly, as when each face
//           is computed once; boundary faces in the element's orientation.
//   lift    -phi H_own + grad phi . S over the 2d faces, sum-factorised to
//           face modes and expanded along the normal index, added to sL;
//           times 1/|J| (orthonormal basis on affine elements) or the dense
//           M_e^-1 (curved elements), then the R / N / Jv epilogue.
// Each interior face flux is evaluated by both of its elements (twice the
// face arithmetic of the three-kernel path), which replaces the round trips
// of the per-point traces and face fluxes through HBM.
#pragma once
#include "dgj_residual.h"

namespace dgj {

// tangential axes of the face normal to axis ax (the first is the faster
// one in face-point and face-mode indices), without a runtime-indexed array
template <int D>
__device__ __forceinline__ int tang0(int ax) { return D == 3 ? (ax == 0 ? 1 : 0) : 1 - ax; }
template <int D>
__device__ __forceinline__ int tang1(int ax) { return D == 3 ? (ax == 2 ? 1 : 2) : 0; }
template <int N>
__device__ __forceinline__ int npow(int x) { return x == 0 ? 1 : (x == 1 ? N : N * N); }

template <int D, int N, int Q>
struct FusedK {
  using K = ResK<D, N, Q>;
  static constexpr int NV = K::NV, NM = K::NM, NQ = K::NQ, NQF = K::NQF, NMF = K::NMF, NF = K::NF, NB = K::NB;
  static constexpr int VOL = K::T1 + K::T2 + K::QG;                    // volume phase (W + sQ)
  static constexpr int TR = 2 * NF * 2 * NV * NMF;                     // modal traces [side][f][kind][v][tm]
  static constexpr int SA = (D == 3) ? 2 * NF * 3 * NV * Q * N : 0;    // first tangential stage [side][f][c][v][a][j]
  static constexpr int AF = NF * (D + 1) * NV * NQF;                   // weighted face data [f][k][v][p]
  static constexpr int Y = (D == 3) ? NF * NV * Q * 3 * N : 0;         // lift, first stage [f][v][a][c][j]
  static constexpr int FM = NF * 2 * NV * NMF;                         // face modes [f][c][v][tm]
  static constexpr int FACE = TR + SA;
  static constexpr int LIFT = AF + Y + FM;
  static constexpr int U1 = VOL > FACE ? VOL : FACE;
  static constexpr int U = U1 > LIFT ? U1 : LIFT;
  static constexpr int NPTS = NF * NQF;   // face points: one thread each in the flux phase
  // LDS of a workgroup of EPW elements, and the workgroups of 256 threads
  // per CU the register budget is set for: as many as the LDS holds (at most 3)
  static constexpr int lds_bytes(int epw) { return epw * 8 * (2 * NB + U + NF) + 8 * (4 * N + 2 * Q * N + Q); }
  static constexpr int minb(int epw) {
    return (160 * 1024 / lds_bytes(epw)) >= 3 ? 3 : ((160 * 1024 / lds_bytes(epw)) >= 2 ? 2 : 1);
  }
};

// smallest number of threads per element: a thread per face point, in
// whole half-wavefronts (2D) or wavefronts (3D)
template <int D, int N, int Q>
constexpr int fused_min_threads() {
  return D == 2 ? ((FusedK<D, N, Q>::NPTS + 31) / 32) * 32 : ((FusedK<D, N, Q>::NPTS + 63) / 64) * 64;
}

// EPW elements per workgroup, blockDim.x / EPW threads per element (the
// workgroup-size and elements-per-workgroup tile the autotuner chooses; the
// arithmetic of each element does not depend on it)
template <int D, int N, int Q, bool CV, int EPW>
__global__ __launch_bounds__(256, (FusedK<D, N, Q>::minb(EPW))) void k_res_fused(ResArgs a) {
  static constexpr TabK<N, Q> tk = make_tabk<N, Q>();
  using F = FusedK<D, N, Q>;
  using K = ResK<D, N, Q>;
  constexpr int NV = F::NV, NM = F::NM, NQF = F::NQF, NMF = F::NMF, NF = F::NF, NB = F::NB;
  constexpr int CF = D * D + D + 1;
  constexpr int GEO = K::S::GEO;
  __shared__ double sUa[EPW][NB];
  __shared__ double sLa[EPW][NB];
  __shared__ double WSa[EPW][F::U];
  __shared__ double sE[4 * N];         // phi(-1), phi(+1), phi'(-1), phi'(+1)
  __shared__ double sB[Q * N], sD[Q * N], sW[Q];
  __shared__ long s_nba[EPW][NF];
  const int NT = blockDim.x / EPW;                 // threads of this element
  const int sub = threadIdx.x / NT;
  const int tid = threadIdx.x - sub * NT;
  const long e_raw = (long)blockIdx.x * EPW + sub;
  // an element past the end or of an inactive instance computes on a valid
  // index (every load in bounds, every barrier reached) and writes nothing
  const long e = e_raw < a.n_elem ? e_raw : a.n_elem - 1;
  ElemParams ep;
  const bool ok = elem_params(a, e, ep) && e_raw < a.n_elem;
  double* sU = sUa[sub];
  double* sL = sLa[sub];
  double* WS = WSa[sub];
  long* s_nb = s_nba[sub];
  const double* g = a.geo + e * GEO;
  double dxi[D];
#pragma unroll
  for (int j = 0; j < D; ++j) dxi[j] = g[j];
  const double detJ = g[D];
  for (int i = tid; i < NB; i += NT) sU[i] = ep.in(e * NB + i);
  if (tid < NF) s_nb[tid] = a.nbr[e * NF + tid];
  if (threadIdx.x < 2 * N) {
    sE[threadIdx.x] = tk.phiE[threadIdx.x / N][threadIdx.x % N];
    sE[2 * N + threadIdx.x] = tk.dphiE[threadIdx.x / N][threadIdx.x % N];
  }
  for (int i = threadIdx.x; i < Q * N; i += blockDim.x) {
    sB[i] = tk.B[i / N][i % N];
    sD[i] = tk.Dq[i / N][i % N];
  }
  if (threadIdx.x < Q) sW[threadIdx.x] = tk.w[threadIdx.x];
  __syncthreads();

  // ---- volume terms -> sL
  {
    double* W = WS;
    double* sQ = WS + K::T1 + K::T2;
    res_vol_forward<D, N, Q>(tk, sU, W, sQ, tid, NT);
    __syncthreads();
    res_vol_flux<D, N, Q, CV>(a, tk, ep, e, dxi, detJ, sQ, tid, NT);
    __syncthreads();
    res_vol_transpose<D, N, Q>(tk, sQ, W, sL, tid, NT);
    __syncthreads();
  }

  // ---- modal face traces of both sides: TR[side][f][kind][v][tm] (side 0:
  // this element on face f; side 1: the neighbour on its face f^1, zero on
  // boundary faces); item it = (f, v, tm), tm = i + N j with i along the
  // first tangential axis
  double* TR = WS;
  double* SA = WS + F::TR;
  constexpr int NI = NF * NV * NMF;
  auto tr_item = [&](int it, int& f, int& v, int& tm, int& mt, int& st) {
    tm = it % NMF;
    v = (it / NMF) % NV;
    f = it / (NMF * NV);
    const int ax = f >> 1;
    mt = (tm % N) * npow<N>(tang0<D>(ax)) + (D == 3 ? (tm / N) * npow<N>(tang1<D>(ax)) : 0);
    st = npow<N>(ax);
  };
  // the neighbours' modes come from memory: a thread's loads for up to 4
  // items are issued together, then contracted
  for (int i0 = tid; i0 < NI; i0 += 4 * NT) {
    double x[4][N];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int it = i0 + k * NT;
      int f, v, tm, mt, st;
      tr_item(it < NI ? it : 0, f, v, tm, mt, st);
      const long en = s_nb[f];
      const bool ld = it < NI && en >= 0;
#pragma unroll
      for (int ia = 0; ia < N; ++ia) x[k][ia] = ld ? ep.in(en * NB + v * NM + mt + ia * st) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int it = i0 + k * NT;
      if (it < NI) {
        int f, v, tm, mt, st;
        tr_item(it, f, v, tm, mt, st);
        const int ss = (f & 1) ^ 1;
        double tv = 0.0, tn = 0.0;
#pragma unroll
        for (int ia = 0; ia < N; ++ia) {
          tv += sE[ss * N + ia] * x[k][ia];
          tn += sE[2 * N + ss * N + ia] * x[k][ia];
        }
        TR[((NF + f) * 2 + 0) * NV * NMF + v * NMF + tm] = tv;
        TR[((NF + f) * 2 + 1) * NV * NMF + v * NMF + tm] = tn;
      }
    }
  }
  for (int it = tid; it < NI; it += NT) {
    int f, v, tm, mt, st;
    tr_item(it, f, v, tm, mt, st);
    const int ss = f & 1;
    double tv = 0.0, tn = 0.0;
#pragma unroll
    for (int ia = 0; ia < N; ++ia) {
      const double x = sU[v * NM + mt + ia * st];
      tv += sE[ss * N + ia] * x;
      tn += sE[2 * N + ss * N + ia] * x;
    }
    TR[(f * 2 + 0) * NV * NMF + v * NMF + tm] = tv;
    TR[(f * 2 + 1) * NV * NMF + v * NMF + tm] = tn;
  }
  __syncthreads();
  if constexpr (D == 3) {
    // first tangential direction t0: SA[side][f][c][v][a][j], c = 0: B tv,
    // 1: Dq tv, 2: B tn (tm = i + N j, i along t0)
    for (int it = tid; it < 2 * NF * NV * N; it += NT) {
      const int j = it % N;
      const int v = (it / N) % NV;
      const int sf = it / (N * NV);           // side * NF + f
      const double* tv = TR + (sf * 2 + 0) * NV * NMF + v * NMF + N * j;
      const double* tn = TR + (sf * 2 + 1) * NV * NMF + v * NMF + N * j;
      double xv[N], xn[N];
#pragma unroll
      for (int i = 0; i < N; ++i) { xv[i] = tv[i]; xn[i] = tn[i]; }
      double* o = SA + (sf * 3 * NV + v) * Q * N + j;
#pragma unroll
      for (int aa = 0; aa < Q; ++aa) {
        double b0 = 0.0, d0 = 0.0, bn = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          b0 += tk.B[aa][i] * xv[i];
          d0 += tk.Dq[aa][i] * xv[i];
          bn += tk.B[aa][i] * xn[i];
        }
        o[aa * N] = b0;
        o[NV * Q * N + aa * N] = d0;
        o[2 * NV * Q * N + aa * N] = bn;
      }
    }
    __syncthreads();
  }

  // ---- face points: both sides' values and physical gradients, the face
  // flux, and the weighted data the lift contracts: AF[f][k][v][p] with
  // k = 0: -w H_own, k >= 1: sum_j (d xi_{k-1} / d x_j) w S_j (curved) or
  // w S_{k-1} dxi_{k-1} (boxes)
  double Af[D + 1][NV];
  const bool pt = tid < F::NPTS;
  const int f = pt ? tid / NQF : 0;
  const int p = pt ? tid % NQF : 0;
  if (pt) {
    const int ax = f >> 1, s = f & 1;
    const int t0 = tang0<D>(ax), t1 = tang1<D>(ax);
    const int pa = p % Q, pb = (D == 3) ? p / Q : 0;
    const long en = s_nb[f];
    // curved elements: the metric d xi_k / d x_j at the point of both sides
    // (Mo: this element on face f, Mn: the neighbour on its face f^1) and the
    // normal and face weight of the canonical side (the side-1 element on
    // interior faces), all loads issued before any use
    double Mo[CV ? D * D : 1], Mn[CV ? D * D : 1], nrm[D], wf;
    if constexpr (CV) {
      const double* Go = a.fg + (e * NF + f) * (long)CF * NQF + p;
#pragma unroll
      for (int c = 0; c < D * D; ++c) Mo[c] = Go[c * NQF];
      const double* Gn = a.fg + ((en >= 0 ? en : e) * NF + (en >= 0 ? (f ^ 1) : f)) * (long)CF * NQF + p;
#pragma unroll
      for (int c = 0; c < D * D; ++c) Mn[c] = Gn[c * NQF];
      const double* G1 = (en >= 0 && !s) ? Gn : Go;
#pragma unroll
      for (int j = 0; j < D; ++j) nrm[j] = G1[(D * D + j) * NQF];
      wf = G1[(D * D + D) * NQF];
    }
    // values and physical gradients of one side at the point: side 0 this
    // element on face f, side 1 the neighbour on its face f^1 (the same code
    // for both, so the two elements of a face see bitwise the same data)
    // (accumulate: the gradient is added into G, which then holds the sum
    // of both sides' gradients, left first, as the face flux takes it)
    auto side_data = [&](int side, double* U, double (*G)[NV], bool accumulate) {
      const long ee = side == 0 ? e : en;
      const double* Ms = side == 0 ? Mo : Mn;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double val = 0.0, dt0 = 0.0, dt1 = 0.0, dn = 0.0;
        if constexpr (D == 3) {
          const double* o = SA + ((side * NF + f) * 3 * NV + v) * Q * N + pa * N;
#pragma unroll
          for (int j = 0; j < N; ++j) {
            const double bj = sB[pb * N + j];
            val += bj * o[j];
            dt0 += bj * o[NV * Q * N + j];
            dt1 += sD[pb * N + j] * o[j];
            dn += bj * o[2 * NV * Q * N + j];
          }
        } else {
          const double* tv = TR + ((side * NF + f) * 2 + 0) * NV * NMF + v * NMF;
          const double* tn = TR + ((side * NF + f) * 2 + 1) * NV * NMF + v * NMF;
#pragma unroll
          for (int i = 0; i < N; ++i) {
            val += sB[pa * N + i] * tv[i];
            dt0 += sD[pa * N + i] * tv[i];
            dn += sB[pa * N + i] * tn[i];
          }
        }
        // reference gradient component k: d/dn along ax, the tangential ones
        double gr[D];
#pragma unroll
        for (int k = 0; k < D; ++k) gr[k] = (k == ax) ? dn : ((k == t0) ? dt0 : dt1);
        U[v] = val;
        if constexpr (CV) {
#pragma unroll
          for (int j = 0; j < D; ++j) {
            double sg = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) sg += Ms[k * D + j] * gr[k];
            G[j][v] = accumulate ? G[j][v] + sg : sg;
          }
        } else {
          const double* ge = a.geo + ee * GEO;
#pragma unroll
          for (int j = 0; j < D; ++j) {
            const double gj = gr[j] * ge[j];
            G[j][v] = accumulate ? G[j][v] + gj : gj;
          }
        }
      }
    };
    // left = the side-1 element's data (this element's when s = 1); a
    // boundary face has this element's only
    double UL[NV], UR[NV], GS[D][NV];
    const int sideL = (en >= 0 && !s) ? 1 : 0;
    side_data(sideL, UL, GS, false);
    if (en >= 0) side_data(1 - sideL, UR, GS, true);
    double H[NV], Sf[D][NV];
    if (en >= 0) {
      // canonical orientation: the side-1 element's normal, weights and penalty
      const long e1 = s ? e : en;
      const int f1 = s ? f : (f ^ 1);
      if constexpr (!CV) {
#pragma unroll
        for (int j = 0; j < D; ++j) nrm[j] = (j == ax) ? 1.0 : 0.0;
        wf = a.geo[e1 * GEO + D + 2 + ax] * sW[pa];
        if (D == 3) wf *= sW[pb];
      }
      const double beta = a.beta[e1 * NF + f1];
      face_flux_gsum<D>(ep.ph, UL, UR, GS, nrm, beta, H, Sf);
      if (!s) {
#pragma unroll
        for (int v = 0; v < NV; ++v) H[v] = -H[v];
      }
    } else {
      const int bid = -(int)en - 1;
      const int kind = a.bc_kind[bid];
      if constexpr (!CV) {
#pragma unroll
        for (int j = 0; j < D; ++j) nrm[j] = (j == ax) ? (s == 1 ? 1.0 : -1.0) : 0.0;
        wf = g[D + 2 + ax] * sW[pa];
        if (D == 3) wf *= sW[pb];
      }
      // the id's state, or the Dirichlet ghost state at the point
      double Ub[NV];
      const bool dir = kind == BC_DIRICHLET;
      const double* gb = dir ? a.bc_field + (e * NF + f) * (long)NV * NQF + p : a.bc_state + bid * NV;
      const int gstride = dir ? NQF : 1;
#pragma unroll
      for (int v = 0; v < NV; ++v) Ub[v] = gb[v * gstride];
      boundary_flux<D>(ep.ph, kind, UL, GS, nrm, a.beta[e * NF + f], Ub, H, Sf);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) Af[0][v] = -H[v];
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if constexpr (CV) {
          double sg = 0.0;
#pragma unroll
          for (int j = 0; j < D; ++j) sg += Mo[k * D + j] * Sf[j][v];
          Af[1 + k][v] = sg;
        } else {
          Af[1 + k][v] = Sf[k][v] * dxi[k];
        }
      }
    // face weight: w^G |J^G| at the point (boxes: |J^G| times the tensor Gauss weight)
#pragma unroll
    for (int k = 0; k <= D; ++k)
#pragma unroll
      for (int v = 0; v < NV; ++v) Af[k][v] *= wf;
  }
  __syncthreads();   // traces and first-stage data are dead from here
  double* AF = WS;
  double* Yb = WS + F::AF;
  double* FMb = WS + F::AF + F::Y;
  if (pt) {
#pragma unroll
    for (int k = 0; k <= D; ++k)
#pragma unroll
      for (int v = 0; v < NV; ++v) AF[((f * (D + 1) + k) * NV + v) * NQF + p] = Af[k][v];
  }
  __syncthreads();

  // ---- lift: tangential contraction to face modes FM[f][c][v][tm]
  // (c = 0 multiplies phi(+-1), c = 1 phi'(+-1) of the normal index)
  if constexpr (D == 3) {
    for (int it = tid; it < NF * NV * Q; it += NT) {
      const int aa = it % Q;
      const int v = (it / Q) % NV;
      const int ff = it / (Q * NV);
      const int ax = ff >> 1;
      const double* A0 = AF + ((ff * (D + 1) + 0) * NV + v) * NQF + aa;
      const double* At0 = AF + ((ff * (D + 1) + 1 + tang0<D>(ax)) * NV + v) * NQF + aa;
      const double* At1 = AF + ((ff * (D + 1) + 1 + tang1<D>(ax)) * NV + v) * NQF + aa;
      const double* Aax = AF + ((ff * (D + 1) + 1 + ax) * NV + v) * NQF + aa;
      double x0[Q], xt0[Q], xt1[Q], xax[Q];
#pragma unroll
      for (int b = 0; b < Q; ++b) {
        x0[b] = A0[b * Q];
        xt0[b] = At0[b * Q];
        xt1[b] = At1[b * Q];
        xax[b] = Aax[b * Q];
      }
      double* o = Yb + ((ff * NV + v) * Q + aa) * 3 * N;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        double y0 = 0.0, y1 = 0.0, y2 = 0.0;
#pragma unroll
        for (int b = 0; b < Q; ++b) {
          y0 += tk.B[b][j] * x0[b] + tk.Dq[b][j] * xt1[b];
          y1 += tk.B[b][j] * xt0[b];
          y2 += tk.B[b][j] * xax[b];
        }
        o[j] = y0;
        o[N + j] = y1;
        o[2 * N + j] = y2;
      }
    }
    __syncthreads();
    for (int it = tid; it < NF * NV * N; it += NT) {
      const int j1 = it % N;
      const int v = (it / N) % NV;
      const int ff = it / (N * NV);
      double y0[Q], y1[Q], y2[Q];
#pragma unroll
      for (int aa = 0; aa < Q; ++aa) {
        const double* o = Yb + ((ff * NV + v) * Q + aa) * 3 * N + j1;
        y0[aa] = o[0];
        y1[aa] = o[N];
        y2[aa] = o[2 * N];
      }
#pragma unroll
      for (int j0 = 0; j0 < N; ++j0) {
        double f0 = 0.0, f1 = 0.0;
#pragma unroll
        for (int aa = 0; aa < Q; ++aa) {
          f0 += tk.B[aa][j0] * y0[aa] + tk.Dq[aa][j0] * y1[aa];
          f1 += tk.B[aa][j0] * y2[aa];
        }
        FMb[((ff * 2 + 0) * NV + v) * NMF + j0 + N * j1] = f0;
        FMb[((ff * 2 + 1) * NV + v) * NMF + j0 + N * j1] = f1;
      }
    }
  } else {
    for (int it = tid; it < NF * NV; it += NT) {
      const int v = it % NV;
      const int ff = it / NV;
      const int ax = ff >> 1;
      const int t0 = 1 - ax;
      const double* A0 = AF + ((ff * (D + 1) + 0) * NV + v) * NQF;
      const double* At0 = AF + ((ff * (D + 1) + 1 + t0) * NV + v) * NQF;
      const double* Aax = AF + ((ff * (D + 1) + 1 + ax) * NV + v) * NQF;
#pragma unroll
      for (int j0 = 0; j0 < N; ++j0) {
        double f0 = 0.0, f1 = 0.0;
#pragma unroll
        for (int aa = 0; aa < Q; ++aa) {
          f0 += tk.B[aa][j0] * A0[aa] + tk.Dq[aa][j0] * At0[aa];
          f1 += tk.B[aa][j0] * Aax[aa];
        }
        FMb[((ff * 2 + 0) * NV + v) * NMF + j0] = f0;
        FMb[((ff * 2 + 1) * NV + v) * NMF + j0] = f1;
      }
    }
  }
  __syncthreads();

  // ---- expansion along the normal index, mass inverse, epilogue
  // The epilogue's operands of this thread's first MINV_OUTK unknowns
  // (i = tid + k NT) are loaded here, ahead of their results (the stage
  // residual and the matvec; R alone needs none); the state is the
  // element's copy in LDS.
  EpiIn pre[MINV_OUTK];
  const bool need = ok && a.mode != RES_R;
#pragma unroll
  for (int k = 0; k < MINV_OUTK; ++k) {
    const int i = tid + k * NT;
    pre[k] = (need && i < NB) ? epi_load(a, e * NB + i, sU[i]) : EpiIn{0.0, 0.0, 0.0};
  }
  const double invdetJ = g[D + 1];
  auto expand = [&](int i) {
    const int m = i % NM, v = i / NM;
    int mi[3] = {0, 0, 0};
    split<D, N>(m, mi);
    double Lm = sL[i];
#pragma unroll
    for (int ff = 0; ff < NF; ++ff) {
      const int ax = ff >> 1, s = ff & 1;
      int t[2] = {0, 0};
      tang_axes<D>(ax, t);
      const int tm = mi[t[0]] + ((D == 3) ? N * mi[t[1]] : 0);
      Lm += sE[s * N + mi[ax]] * FMb[((ff * 2 + 0) * NV + v) * NMF + tm] +
            sE[2 * N + s * N + mi[ax]] * FMb[((ff * 2 + 1) * NV + v) * NMF + tm];
    }
    return Lm;
  };
  if constexpr (CV) {
    for (int i = tid; i < NB; i += NT) sL[i] = expand(i);
    __syncthreads();
    static_assert(F::U / NB >= 1, "LDS staging of the mass-matrix product");
    mass_inv_dense<NM, NV>(a.minv + e * (long)NM * mass_ld(NM), sL, WS, tid, NT, F::U / NB,
                           [&](int i, double R, int k) {
                             if (!ok) return;
                             const long gi = e * NB + i;
                             epilogue_pre(a, ep, gi, R, k >= 0 ? pre[k] : epi_load(a, gi, sU[i]));
                           });
  } else {
#pragma unroll
    for (int k = 0; k < MINV_OUTK; ++k) {
      const int i = tid + k * NT;
      if (i < NB && ok) epilogue_pre(a, ep, e * NB + i, expand(i) * invdetJ, pre[k]);
    }
    for (int i = tid + MINV_OUTK * NT; i < NB; i += NT)
      if (ok) epilogue_pre(a, ep, e * NB + i, expand(i) * invdetJ, epi_load(a, e * NB + i, sU[i]));
  }
}

}  // namespace dgj
