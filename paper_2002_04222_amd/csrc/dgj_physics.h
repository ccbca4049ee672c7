// Pointwise physics of the compressible Navier-Stokes equations (arxiv
// 2002.04222, Sec. 2, Eq. 1-6) as device functions templated on the scalar
// type, so the same source evaluates fluxes in double precision and, with
// the forward-mode Dual type below, their exact derivatives with respect to
// the conserved state (the analytic volume flux Jacobians of Sec. 4.2.2).
//
// Conserved state U = (rho, rho u_1..rho u_D, E); E = p/(gamma-1) + rho|u|^2/2;
// p = rho T / (gamma Ma^2); tau_ij = mu (du_i/dx_j + du_j/dx_i) - 2/3 mu
// div(u) delta_ij; q_i = -mu/(Ma^2 Pr (gamma-1)) dT/dx_i.  Gradients enter
// as gradients of conserved variables, gU[j][v] = d U_v / d x_j.
#pragma once
#include <hip/hip_runtime.h>

namespace dgj {

struct Phys {
  double gamma, Pr, Re, Ma, T_ref_K;
  int visc_law;    // 0 constant mu = 1/Re, 1 Sutherland
  int flux_mode;   // 0 Navier-Stokes, 1 Euler, 2 scalar diffusion test (G = grad U / Re, F = 0)
  int riemann;     // 0 Roe, 1 local Lax-Friedrichs, 2 HLL, 3 HLLC, 4 AUSM+
};

// ---------------------------------------------------------------- dual numbers
template <int M>
struct Dual {
  double v;
  double d[M];
  __host__ __device__ Dual() {}
  __host__ __device__ Dual(double x) : v(x) {
#pragma unroll
    for (int i = 0; i < M; ++i) d[i] = 0.0;
  }
};
template <int M> __device__ __forceinline__ Dual<M> operator+(const Dual<M>& a, const Dual<M>& b) {
  Dual<M> r; r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int M> __device__ __forceinline__ Dual<M> operator-(const Dual<M>& a, const Dual<M>& b) {
  Dual<M> r; r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int M> __device__ __forceinline__ Dual<M> operator-(const Dual<M>& a) {
  Dual<M> r; r.v = -a.v;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int M> __device__ __forceinline__ Dual<M> operator*(const Dual<M>& a, const Dual<M>& b) {
  Dual<M> r; r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int M> __device__ __forceinline__ Dual<M> operator/(const Dual<M>& a, const Dual<M>& b) {
  Dual<M> r; double ib = 1.0 / b.v; r.v = a.v * ib;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
  return r;
}
template <int M> __device__ __forceinline__ Dual<M> operator*(double a, const Dual<M>& b) {
  Dual<M> r; r.v = a * b.v;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = a * b.d[i];
  return r;
}
template <int M> __device__ __forceinline__ Dual<M> operator*(const Dual<M>& b, double a) { return a * b; }
template <int M> __device__ __forceinline__ Dual<M> operator+(const Dual<M>& a, double b) {
  Dual<M> r = a; r.v += b; return r;
}
template <int M> __device__ __forceinline__ Dual<M> operator+(double b, const Dual<M>& a) { return a + b; }
template <int M> __device__ __forceinline__ Dual<M> operator-(const Dual<M>& a, double b) {
  Dual<M> r = a; r.v -= b; return r;
}
template <int M> __device__ __forceinline__ Dual<M> operator-(double b, const Dual<M>& a) {
  Dual<M> r = -a; r.v += b; return r;
}
template <int M> __device__ __forceinline__ Dual<M> operator/(const Dual<M>& a, double b) {
  return a * (1.0 / b);
}
template <int M> __device__ __forceinline__ Dual<M> operator/(double a, const Dual<M>& b) {
  return Dual<M>(a) / b;
}
template <int M> __device__ __forceinline__ Dual<M> dsqrt(const Dual<M>& a) {
  Dual<M> r; r.v = sqrt(a.v); double h = 0.5 / r.v;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = a.d[i] * h;
  return r;
}
__device__ __forceinline__ double dsqrt(double a) { return sqrt(a); }

// 1/x for the positive, normal quantities of the pointwise fluxes (densities,
// c^2, sums of square roots): the hardware reciprocal estimate refined by two
// Newton steps, within about an ulp of the quotient, in place of the full
// IEEE division sequence.  Dual numbers keep their quotient rule.
__device__ __forceinline__ double rcp_pos(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
template <int M> __device__ __forceinline__ Dual<M> rcp_pos(const Dual<M>& x) { return 1.0 / x; }

// ---------------------------------------------------------------- fluxes
template <typename T>
__device__ __forceinline__ T viscosity(const Phys& ph, const T& rho, const T& p) {
  if (ph.visc_law == 0) return T(1.0 / ph.Re);
  T Tk = ph.gamma * ph.Ma * ph.Ma * p / rho;
  double s = 110.0 / ph.T_ref_K;
  return (Tk * dsqrt(Tk)) * ((1.0 + s) / ph.Re) / (Tk + s);
}

// F_j(U) of Eq. 2: F[j][v]
template <int D, typename T>
__device__ __forceinline__ void euler_flux(const Phys& ph, const T* U, T (*F)[D + 2]) {
  constexpr int NV = D + 2;
  if (ph.flux_mode == 2) {
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int v = 0; v < NV; ++v) F[j][v] = T(0.0);
    return;
  }
  T rho = U[0];
  T irho = rcp_pos(rho);
  T vel[D];
  T ke = T(0.0);
#pragma unroll
  for (int c = 0; c < D; ++c) { vel[c] = U[1 + c] * irho; ke = ke + vel[c] * U[1 + c]; }
  T p = (ph.gamma - 1.0) * (U[D + 1] - 0.5 * ke);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    F[j][0] = U[1 + j];
#pragma unroll
    for (int c = 0; c < D; ++c) F[j][1 + c] = U[1 + j] * vel[c];
    F[j][1 + j] = F[j][1 + j] + p;
    F[j][D + 1] = vel[j] * (U[D + 1] + p);
  }
}

// G_j(U, grad U) of Eq. 2 (viscous flux): G[j][v]; gU[j][v] = d U_v / d x_j.
template <int D, typename T, typename TG>
__device__ __forceinline__ void viscous_flux(const Phys& ph, const T* U, const TG (*gU)[D + 2], T (*G)[D + 2]) {
  constexpr int NV = D + 2;
  if (ph.flux_mode == 1) {
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int v = 0; v < NV; ++v) G[j][v] = T(0.0);
    return;
  }
  if (ph.flux_mode == 2) {
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int v = 0; v < NV; ++v) G[j][v] = T(0.0) + gU[j][v] * (1.0 / ph.Re);
    return;
  }
  T rho = U[0];
  T irho = rcp_pos(rho);
  T vel[D];
  T ke = T(0.0);
#pragma unroll
  for (int c = 0; c < D; ++c) { vel[c] = U[1 + c] * irho; ke = ke + vel[c] * U[1 + c]; }
  T E = U[D + 1];
  T p = (ph.gamma - 1.0) * (E - 0.5 * ke);
  T mu = viscosity<T>(ph, rho, p);
  // gvel[j][c] = d u_c / d x_j
  T gvel[D][D];
  T div = T(0.0);
#pragma unroll
  for (int j = 0; j < D; ++j) {
#pragma unroll
    for (int c = 0; c < D; ++c) gvel[j][c] = (gU[j][1 + c] - vel[c] * gU[j][0]) * irho;
    div = div + gvel[j][j];
  }
  T Eor = E * irho;
  T kappa = mu * (ph.gamma / ph.Pr);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    T work = T(0.0);
#pragma unroll
    for (int c = 0; c < D; ++c) {
      T tau = mu * (gvel[c][i] + gvel[i][c]);
      if (c == i) tau = tau - (2.0 / 3.0) * mu * div;
      G[i][1 + c] = tau;
      work = work + vel[c] * tau;
    }
    // d e / d x_i with e = E/rho - |u|^2/2
    T ge = (gU[i][D + 1] - Eor * gU[i][0]) * irho;
#pragma unroll
    for (int c = 0; c < D; ++c) ge = ge - vel[c] * gvel[i][c];
    G[i][0] = T(0.0);
    G[i][D + 1] = work + kappa * ge;
  }
}

// Normal viscous fluxes of rank-one gradients d (x) dU (grad U_v = d dU_v),
// the interior-penalty and symmetric terms of Eq. 12: with
// w_c = (dU_{1+c} - u_c dU_0) / rho (then grad u = d (x) w) and
// e~ = (dU_E - (E/rho) dU_0) / rho - u . w,
//   n . G[1+c] = mu ((n.d) w_c + (n.w) d_c) - 2/3 mu (d.w) n_c,
//   n . G[E]   = u . (n . G[mom]) + kappa (n.d) e~,      n . G[0] = 0,
// the same flux as viscous_flux (Eq. 2-6) without forming the gradient.
// Pn = n . G(U, n (x) dU) and, if WS, S[j] = 1/2 n . G(U, e_j (x) dU).
template <int D, bool WS = true>
__device__ __forceinline__ void viscous_normal_rank1(const Phys& ph, const double* U, const double* dU,
                                                     const double* n, double* Pn, double (&S)[D][D + 2]) {
  constexpr int NV = D + 2;
  if (ph.flux_mode == 1) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Pn[v] = 0.0;
    if constexpr (WS) {
#pragma unroll
      for (int j = 0; j < D; ++j)
#pragma unroll
        for (int v = 0; v < NV; ++v) S[j][v] = 0.0;
    }
    return;
  }
  if (ph.flux_mode == 2) {
    double nn = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) nn += n[j] * n[j];
#pragma unroll
    for (int v = 0; v < NV; ++v) Pn[v] = nn * dU[v] * (1.0 / ph.Re);
    if constexpr (WS) {
#pragma unroll
      for (int j = 0; j < D; ++j)
#pragma unroll
        for (int v = 0; v < NV; ++v) S[j][v] = 0.5 * (n[j] * dU[v] * (1.0 / ph.Re));
    }
    return;
  }
  const double rho = U[0];
  const double irho = rcp_pos(rho);
  double vel[D], w[D];
  double ke = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) { vel[c] = U[1 + c] * irho; ke = ke + vel[c] * U[1 + c]; }
  const double E = U[D + 1];
  const double p = (ph.gamma - 1.0) * (E - 0.5 * ke);
  const double mu = viscosity<double>(ph, rho, p);
  const double kappa = mu * (ph.gamma / ph.Pr);
  double nw = 0.0, uw = 0.0, nn = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    w[c] = (dU[1 + c] - vel[c] * dU[0]) * irho;
    nw += n[c] * w[c];
    uw += vel[c] * w[c];
    nn += n[c] * n[c];
  }
  const double et = (dU[D + 1] - (E * irho) * dU[0]) * irho - uw;
  // d = n
  {
    double work = 0.0;
    Pn[0] = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double t = mu * (nn * w[c] + nw * n[c]) - (2.0 / 3.0) * mu * nw * n[c];
      Pn[1 + c] = t;
      work += vel[c] * t;
    }
    Pn[D + 1] = work + kappa * nn * et;
  }
  if constexpr (WS) {
    // d = e_j: n.d = n_j, d.w = w_j
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double work = 0.0;
      S[j][0] = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const double t = mu * (n[j] * w[c] + ((c == j) ? nw : 0.0)) - (2.0 / 3.0) * mu * w[j] * n[c];
        S[j][1 + c] = 0.5 * t;
        work += vel[c] * t;
      }
      S[j][D + 1] = 0.5 * (work + kappa * n[j] * et);
    }
  }
}

// n . G for G[j][v]
template <int D>
__device__ __forceinline__ void dot_normal(const double (*G)[D + 2], const double* n, double* out) {
#pragma unroll
  for (int v = 0; v < D + 2; ++v) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) s += n[j] * G[j][v];
    out[v] = s;
  }
}

__device__ __forceinline__ double fabs_(double x) { return x < 0.0 ? -x : x; }

// Roe's flux without entropy fix; n points from L to R (unit).
template <int D>
__device__ __forceinline__ void roe_flux(const Phys& ph, const double* UL, const double* UR, const double* n,
                                         double* Fn) {
  constexpr int NV = D + 2;
  const double g = ph.gamma;
  // one division per reciprocal (1/rho of each side, 1/c^2) instead of per quotient
  double rL = UL[0], rR = UR[0];
  const double irL = rcp_pos(rL), irR = rcp_pos(rR);
  double vL[D], vR[D], kL = 0.0, kR = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    vL[c] = UL[1 + c] * irL; vR[c] = UR[1 + c] * irR;
    kL += vL[c] * UL[1 + c]; kR += vR[c] * UR[1 + c];
  }
  double pL = (g - 1.0) * (UL[D + 1] - 0.5 * kL);
  double pR = (g - 1.0) * (UR[D + 1] - 0.5 * kR);
  double HL = (UL[D + 1] + pL) * irL, HR = (UR[D + 1] + pR) * irR;
  double sL = sqrt(rL), sR = sqrt(rR);
  double rt = sL * sR;
  double isum = rcp_pos(sL + sR);
  double vt[D], q2 = 0.0, unt = 0.0, dun = 0.0, dv[D], unL = 0.0, unR = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    vt[c] = (sL * vL[c] + sR * vR[c]) * isum;
    q2 += vt[c] * vt[c];
    unt += vt[c] * n[c];
    dv[c] = vR[c] - vL[c];
    dun += dv[c] * n[c];
    unL += vL[c] * n[c];
    unR += vR[c] * n[c];
  }
  double Ht = (sL * HL + sR * HR) * isum;
  double c2 = (g - 1.0) * (Ht - 0.5 * q2);
  double ct = sqrt(c2);
  double dr = rR - rL, dp = pR - pL;
  const double ic2 = rcp_pos(c2);
  double a1 = (dp - rt * ct * dun) * (0.5 * ic2);
  double a5 = (dp + rt * ct * dun) * (0.5 * ic2);
  double a2 = dr - dp * ic2;
  double l1 = fabs_(unt - ct), l2 = fabs_(unt), l5 = fabs_(unt + ct);
  double diss[NV];
  double c1 = l1 * a1, c5 = l5 * a5;
  diss[0] = c1 + c5 + l2 * a2;
  double vdv = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    diss[1 + c] = c1 * (vt[c] - ct * n[c]) + c5 * (vt[c] + ct * n[c]) +
                  l2 * (a2 * vt[c] + rt * (dv[c] - dun * n[c]));
    vdv += vt[c] * dv[c];
  }
  diss[D + 1] = c1 * (Ht - unt * ct) + c5 * (Ht + unt * ct) + l2 * (a2 * 0.5 * q2 + rt * (vdv - unt * dun));
  // central part n.F(UL), n.F(UR)
  double FL[NV], FR[NV];
  FL[0] = rL * unL; FR[0] = rR * unR;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    FL[1 + c] = UL[1 + c] * unL + pL * n[c];
    FR[1 + c] = UR[1 + c] * unR + pR * n[c];
  }
  FL[D + 1] = unL * (UL[D + 1] + pL);
  FR[D + 1] = unR * (UR[D + 1] + pR);
#pragma unroll
  for (int v = 0; v < NV; ++v) Fn[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * diss[v];
}

template <int D>
__device__ __forceinline__ void llf_flux(const Phys& ph, const double* UL, const double* UR, const double* n,
                                         double* Fn) {
  constexpr int NV = D + 2;
  double F[2][NV];
  double lam[2];
  const double* Us[2] = {UL, UR};
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const double* U = Us[s];
    double r = U[0], ke = 0.0, un = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) { ke += U[1 + c] * U[1 + c] / r; un += U[1 + c] / r * n[c]; }
    double p = (ph.gamma - 1.0) * (U[D + 1] - 0.5 * ke);
    lam[s] = fabs_(un) + sqrt(ph.gamma * p / r);
    F[s][0] = r * un;
#pragma unroll
    for (int c = 0; c < D; ++c) F[s][1 + c] = U[1 + c] * un + p * n[c];
    F[s][D + 1] = un * (U[D + 1] + p);
  }
  double lm = lam[0] >= lam[1] ? lam[0] : lam[1];
#pragma unroll
  for (int v = 0; v < NV; ++v) Fn[v] = 0.5 * (F[0][v] + F[1][v]) - 0.5 * lm * (UR[v] - UL[v]);
}

// side state along n: density, velocity, pressure, normal velocity, sound speed
template <int D>
struct SideState {
  double r, v[D], p, E, un, c;
};
template <int D>
__device__ __forceinline__ SideState<D> side_state(const Phys& ph, const double* U, const double* n) {
  SideState<D> s;
  s.r = U[0];
  s.E = U[D + 1];
  double ke = 0.0, un = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    s.v[c] = U[1 + c] / s.r;
    ke += s.v[c] * U[1 + c];
    un += s.v[c] * n[c];
  }
  s.p = (ph.gamma - 1.0) * (U[D + 1] - 0.5 * ke);
  s.un = un;
  s.c = sqrt(ph.gamma * s.p / s.r);
  return s;
}
template <int D>
__device__ __forceinline__ void phys_normal_flux(const double* U, const SideState<D>& s, const double* n, double* F) {
  F[0] = s.r * s.un;
#pragma unroll
  for (int c = 0; c < D; ++c) F[1 + c] = U[1 + c] * s.un + s.p * n[c];
  F[D + 1] = s.un * (U[D + 1] + s.p);
}
// Einfeldt's signal speeds: the smaller (larger) of the left (right)
// acoustic speed and the Roe-average one
template <int D>
__device__ __forceinline__ void wave_speeds(const Phys& ph, const SideState<D>& L, const SideState<D>& R,
                                            const double* n, double& SL, double& SR) {
  const double sL = sqrt(L.r), sR = sqrt(R.r), is = 1.0 / (sL + sR);
  double q2 = 0.0, ut = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double vt = (sL * L.v[c] + sR * R.v[c]) * is;
    q2 += vt * vt;
    ut += vt * n[c];
  }
  const double Ht = (sL * (L.E + L.p) / L.r + sR * (R.E + R.p) / R.r) * is;
  const double ct = sqrt((ph.gamma - 1.0) * (Ht - 0.5 * q2));
  SL = fmin(L.un - L.c, ut - ct);
  SR = fmax(R.un + R.c, ut + ct);
}

// HLL (Harten, Lax, van Leer): one state between the signal speeds
template <int D>
__device__ __forceinline__ void hll_flux(const Phys& ph, const double* UL, const double* UR, const double* n,
                                         double* Fn) {
  constexpr int NV = D + 2;
  const SideState<D> L = side_state<D>(ph, UL, n), R = side_state<D>(ph, UR, n);
  double SL, SR;
  wave_speeds<D>(ph, L, R, n, SL, SR);
  double FL[NV], FR[NV];
  phys_normal_flux<D>(UL, L, n, FL);
  phys_normal_flux<D>(UR, R, n, FR);
  if (SL >= 0.0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Fn[v] = FL[v];
  } else if (SR <= 0.0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Fn[v] = FR[v];
  } else {
    const double id = 1.0 / (SR - SL);
#pragma unroll
    for (int v = 0; v < NV; ++v) Fn[v] = (SR * FL[v] - SL * FR[v] + SL * SR * (UR[v] - UL[v])) * id;
  }
}

// HLLC (Toro, Spruce, Speares): HLL with the contact wave; the star states
// share the contact speed S* and keep their side's tangential velocity
template <int D>
__device__ __forceinline__ void hllc_flux(const Phys& ph, const double* UL, const double* UR, const double* n,
                                          double* Fn) {
  constexpr int NV = D + 2;
  const SideState<D> L = side_state<D>(ph, UL, n), R = side_state<D>(ph, UR, n);
  double SL, SR;
  wave_speeds<D>(ph, L, R, n, SL, SR);
  const bool left = SL >= 0.0, right = SR <= 0.0;
  const double mL = L.r * (SL - L.un), mR = R.r * (SR - R.un);
  const double Ss = (R.p - L.p + mL * L.un - mR * R.un) / (mL - mR);
  const bool useL = left || (!right && Ss >= 0.0);
  const SideState<D>& K = useL ? L : R;
  const double* UK = useL ? UL : UR;
  const double SK = useL ? SL : SR, mK = useL ? mL : mR;
  double F[NV];
  phys_normal_flux<D>(UK, K, n, F);
  if (left || right) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Fn[v] = F[v];
    return;
  }
  const double f = mK / (SK - Ss);
  double Us[NV];
  Us[0] = f;
#pragma unroll
  for (int c = 0; c < D; ++c) Us[1 + c] = f * (K.v[c] + (Ss - K.un) * n[c]);
  Us[D + 1] = f * (K.E / K.r + (Ss - K.un) * (Ss + K.p / mK));
#pragma unroll
  for (int v = 0; v < NV; ++v) Fn[v] = F[v] + SK * (Us[v] - UK[v]);
}

// AUSM+ (Liou): interface Mach number and pressure from the polynomial
// splittings (beta = 1/8, alpha = 3/16), quantities convected upwind of
// the interface mass flux, interface sound speed the mean of the sides'
__device__ __forceinline__ void ausm_split(double M, double sgn, double& Ms, double& Ps) {
  if (fabs_(M) >= 1.0) {
    Ms = 0.5 * (M + sgn * fabs_(M));
    Ps = 0.5 * (1.0 + sgn * (M > 0.0 ? 1.0 : (M < 0.0 ? -1.0 : 0.0)));
  } else {
    const double q = M * M - 1.0;
    Ms = sgn * 0.25 * (M + sgn) * (M + sgn) + sgn * 0.125 * q * q;
    Ps = 0.25 * (M + sgn) * (M + sgn) * (2.0 - sgn * M) + sgn * 0.1875 * M * q * q;
  }
}
template <int D>
__device__ __forceinline__ void ausmp_flux(const Phys& ph, const double* UL, const double* UR, const double* n,
                                           double* Fn) {
  const SideState<D> L = side_state<D>(ph, UL, n), R = side_state<D>(ph, UR, n);
  const double a = 0.5 * (L.c + R.c);
  double MpL, PpL, MmR, PmR;
  ausm_split(L.un / a, 1.0, MpL, PpL);
  ausm_split(R.un / a, -1.0, MmR, PmR);
  const double m = MpL + MmR;
  const double p = PpL * L.p + PmR * R.p;
  const double mp = 0.5 * (m + fabs_(m)), mm = 0.5 * (m - fabs_(m));
  Fn[0] = a * (mp * L.r + mm * R.r);
#pragma unroll
  for (int c = 0; c < D; ++c) Fn[1 + c] = a * (mp * UL[1 + c] + mm * UR[1 + c]) + p * n[c];
  Fn[D + 1] = a * (mp * (L.E + L.p) + mm * (R.E + R.p));
}

// the Riemann flux chosen by ph.riemann (0 Roe, 1 LLF, 2 HLL, 3 HLLC, 4 AUSM+)
template <int D>
__device__ __forceinline__ void riemann_flux(const Phys& ph, const double* UL, const double* UR, const double* n,
                                             double* Fn) {
  switch (ph.riemann) {
    case 0: roe_flux<D>(ph, UL, UR, n, Fn); break;
    case 1: llf_flux<D>(ph, UL, UR, n, Fn); break;
    case 2: hll_flux<D>(ph, UL, UR, n, Fn); break;
    case 3: hllc_flux<D>(ph, UL, UR, n, Fn); break;
    default: ausmp_flux<D>(ph, UL, UR, n, Fn); break;
  }
}

// Numerical normal flux seen from side 'o' with outward normal n:
//   H = Fhat(Uo, Un, n) - [ n.G(Ubar, {gU}) - beta n.G(Ubar, dU (x) n) ]
//   S[j] = 1/2 n.G(Ubar, dU (x) e_j)
// with Ubar = (Uo+Un)/2, dU = Uo - Un (interior penalty, Eq. 12 with a
// dissipative penalty and the 1/2 of the test-gradient average).
// S is written only when WS (a non-null array reference keeps it in registers).
// The same face flux from the sum gs = go + gn of the two sides' gradients.
template <int D, bool WS = true>
__device__ __forceinline__ void face_flux_gsum(const Phys& ph, const double* Uo, const double* Un,
                                               const double (*gs)[D + 2], const double* n, double beta, double* H,
                                               double (&S)[D][D + 2]) {
  constexpr int NV = D + 2;
  double F[NV];
  if (ph.flux_mode == 2) {
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = 0.0;
  } else {
    riemann_flux<D>(ph, Uo, Un, n, F);
  }
  if (ph.flux_mode == 1) {
#pragma unroll
    for (int v = 0; v < NV; ++v) H[v] = F[v];
    if constexpr (WS) {
#pragma unroll
      for (int j = 0; j < D; ++j)
#pragma unroll
        for (int v = 0; v < NV; ++v) S[j][v] = 0.0;
    }
    return;
  }
  double Ub[NV], dU[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) { Ub[v] = 0.5 * (Uo[v] + Un[v]); dU[v] = Uo[v] - Un[v]; }
  double Gn[NV], Pn[NV];
  {
    double ga[D][NV], G[D][NV];
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int v = 0; v < NV; ++v) ga[j][v] = 0.5 * gs[j][v];
    viscous_flux<D, double, double>(ph, Ub, ga, G);
    dot_normal<D>(G, n, Gn);
  }
  // penalty and symmetric terms: viscous fluxes of the rank-one gradients n (x) dU, e_j (x) dU
  viscous_normal_rank1<D, WS>(ph, Ub, dU, n, Pn, S);
#pragma unroll
  for (int v = 0; v < NV; ++v) H[v] = F[v] - (Gn[v] - beta * Pn[v]);
}

template <int D, bool WS = true>
__device__ __forceinline__ void face_flux(const Phys& ph, const double* Uo, const double* Un,
                                          const double (*go)[D + 2], const double (*gn)[D + 2],
                                          const double* n, double beta, double* H, double (&S)[D][D + 2]) {
  double gs[D][D + 2];
#pragma unroll
  for (int j = 0; j < D; ++j)
#pragma unroll
    for (int v = 0; v < D + 2; ++v) gs[j][v] = go[j][v] + gn[j][v];
  face_flux_gsum<D, WS>(ph, Uo, Un, gs, n, beta, H, S);
}

// ---------------------------------------------------------------- boundary conditions
// A boundary face takes the interior trace and a ghost state with the
// interior gradient, and the interior-face fluxes apply.  Far field: 1D
// characteristic (Riemann-invariant) state against the freestream Uinf,
// with the inflow/outflow choice of entropy and tangential velocity blended
// by w = (1 + tanh(u_nb / (0.02 c_b)))/2;
// no-slip wall: mirrored momentum (zero wall velocity), with the heat flux
// through the wall zero (adiabatic), so the viscous energy fluxes vanish.
enum { BC_FARFIELD = 0, BC_WALL = 1, BC_DIRICHLET = 2, BC_SLIP = 3, BC_ISOTHERMAL = 4, BC_EXTRAPOLATE = 5,
       BC_PRESSURE_OUT = 6, BC_PRESSURE_IN = 7 };

template <int D>
__device__ __forceinline__ void farfield_ghost(const Phys& ph, const double* Ui, const double* n, const double* Uo,
                                               double* Ub) {
  constexpr int NV = D + 2;
  const double g = ph.gamma;
  double ri = Ui[0], ro = Uo[0];
  double vi[D], vo[D], ki = 0.0, ko = 0.0, uni = 0.0, uno = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    vi[c] = Ui[1 + c] / ri; vo[c] = Uo[1 + c] / ro;
    ki += vi[c] * vi[c]; ko += vo[c] * vo[c];
    uni += vi[c] * n[c]; uno += vo[c] * n[c];
  }
  const double pi = (g - 1.0) * (Ui[D + 1] - 0.5 * ri * ki);
  const double po = (g - 1.0) * (Uo[D + 1] - 0.5 * ro * ko);
  const double ci = sqrt(g * pi / ri), co = sqrt(g * po / ro);
  if (uno <= -co) {   // supersonic inflow (takes precedence)
#pragma unroll
    for (int v = 0; v < NV; ++v) Ub[v] = Uo[v];
    return;
  }
  if (uni >= ci) {    // supersonic outflow
#pragma unroll
    for (int v = 0; v < NV; ++v) Ub[v] = Ui[v];
    return;
  }
  const double Rp = uni + 2.0 * ci / (g - 1.0);
  const double Rm = uno - 2.0 * co / (g - 1.0);
  const double unb = 0.5 * (Rp + Rm);
  const double cb = 0.25 * (g - 1.0) * (Rp - Rm);
  // entropy and tangential velocity upwinded (interior on outflow,
  // freestream on inflow), blended smoothly where u_nb changes sign
  const double w = 0.5 * (1.0 + tanh(unb / (0.02 * cb)));
  const double s = w * (pi / pow(ri, g)) + (1.0 - w) * (po / pow(ro, g));
  const double rb = pow(cb * cb / (g * s), 1.0 / (g - 1.0));
  const double pb = rb * cb * cb / g;
  double vb[D], kb = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double vt = w * (vi[c] - uni * n[c]) + (1.0 - w) * (vo[c] - uno * n[c]);
    vb[c] = vt + unb * n[c];
    kb += vb[c] * vb[c];
  }
  Ub[0] = rb;
#pragma unroll
  for (int c = 0; c < D; ++c) Ub[1 + c] = rb * vb[c];
  Ub[D + 1] = pb / (g - 1.0) + 0.5 * rb * kb;
}

// Ghost state of boundary kind `kind` for the interior state Uo at a face
// point with outward normal n; Ub is the id's given state (Dirichlet: the
// point's state).  Far field by characteristics; no-slip adiabatic wall:
// momentum negated; slip wall: normal momentum mirrored; isothermal wall:
// velocity negated, pressure kept, temperature mirrored about the given
// state's; extrapolation: the interior; pressure outflow: the given
// pressure where the outflow is subsonic; pressure inflow: the given
// density and velocity with the interior pressure where the inflow is
// subsonic, the given state where supersonic.
template <int D>
__device__ __forceinline__ void ghost_state(const Phys& ph, int kind, const double* Uo, const double* n,
                                            const double* Ub, double* Un) {
  constexpr int NV = D + 2;
  const double g = ph.gamma;
  if (kind == BC_DIRICHLET) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Un[v] = Ub[v];
    return;
  }
  if (kind == BC_FARFIELD) {
    farfield_ghost<D>(ph, Uo, n, Ub, Un);
    return;
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) Un[v] = Uo[v];
  if (kind == BC_WALL) {
#pragma unroll
    for (int c = 0; c < D; ++c) Un[1 + c] = -Uo[1 + c];
    return;
  }
  if (kind == BC_EXTRAPOLATE) return;
  const double r = Uo[0];
  double ke = 0.0, un = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    ke += Uo[1 + c] * Uo[1 + c];
    un += Uo[1 + c] * n[c];
  }
  ke *= 0.5 / r;
  const double p = (g - 1.0) * (Uo[D + 1] - ke);
  if (kind == BC_SLIP) {
#pragma unroll
    for (int c = 0; c < D; ++c) Un[1 + c] = Uo[1 + c] - 2.0 * un * n[c];
    return;
  }
  double keb = 0.0, unb = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    keb += Ub[1 + c] * Ub[1 + c];
    unb += Ub[1 + c] * n[c];
  }
  keb *= 0.5 / Ub[0];
  const double pb = (g - 1.0) * (Ub[D + 1] - keb);
  if (kind == BC_ISOTHERMAL) {
    const double Tw = pb / Ub[0], T = p / r;
    const double rg = r * T / (2.0 * Tw - T);
    double kg = 0.0;
    Un[0] = rg;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double vc = Uo[1 + c] / r;
      Un[1 + c] = -rg * vc;
      kg += vc * vc;
    }
    Un[D + 1] = p / (g - 1.0) + 0.5 * rg * kg;
  } else if (kind == BC_PRESSURE_OUT) {
    const double c = sqrt(g * p / r);
    if (un / r < c) Un[D + 1] = pb / (g - 1.0) + ke;
  } else {   // BC_PRESSURE_IN
    const double cb = sqrt(g * pb / Ub[0]);
#pragma unroll
    for (int v = 0; v < NV; ++v) Un[v] = Ub[v];
    if (!(unb / Ub[0] <= -cb)) Un[D + 1] = p / (g - 1.0) + keb;
  }
}

// boundary face flux seen from the interior (outward normal n)
template <int D, bool WS = true>
__device__ __forceinline__ void boundary_flux(const Phys& ph, int kind, const double* Uo, const double (*go)[D + 2],
                                              const double* n, double beta, const double* Uinf, double* H,
                                              double (&S)[D][D + 2]) {
  constexpr int NV = D + 2;
  double Un[NV];
  ghost_state<D>(ph, kind, Uo, n, Uinf, Un);
  face_flux<D, WS>(ph, Uo, Un, go, go, n, beta, H, S);
  if (kind == BC_WALL || kind == BC_SLIP) {
    // no heat flux (and no work) through the wall: the energy components
    // keep only the Riemann flux; a slip wall also takes no tangential
    // viscous traction
    double F[NV];
    if (ph.flux_mode == 2) {
#pragma unroll
      for (int v = 0; v < NV; ++v) F[v] = 0.0;
    } else {
      riemann_flux<D>(ph, Uo, Un, n, F);
    }
    H[D + 1] = F[D + 1];
    if constexpr (WS) {
#pragma unroll
      for (int j = 0; j < D; ++j) S[j][D + 1] = 0.0;
    }
    if (kind == BC_SLIP) {
      // viscous momentum flux G = F - H, keep its normal part
      double gn = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) gn += (F[1 + c] - H[1 + c]) * n[c];
#pragma unroll
      for (int c = 0; c < D; ++c) H[1 + c] = F[1 + c] - gn * n[c];
      if constexpr (WS) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
          double sn = 0.0;
#pragma unroll
          for (int c = 0; c < D; ++c) sn += S[j][1 + c] * n[c];
#pragma unroll
          for (int c = 0; c < D; ++c) S[j][1 + c] = sn * n[c];
        }
      }
    }
  }
}

// LDG viscous normal flux n.G(u_hat, q_hat) - beta n.G(u_hat, jump (x) n)
template <int D>
__device__ __forceinline__ void ldg_viscous_n(const Phys& ph, const double* Uh, const double (*q)[D + 2],
                                              const double* jump, const double* n, double beta, double* Gn) {
  constexpr int NV = D + 2;
  double G[D][NV], J[D][NV], Pn[NV];
  viscous_flux<D, double, double>(ph, Uh, q, G);
  dot_normal<D>(G, n, Gn);
#pragma unroll
  for (int j = 0; j < D; ++j)
#pragma unroll
    for (int v = 0; v < NV; ++v) J[j][v] = n[j] * jump[v];
  viscous_flux<D, double, double>(ph, Uh, J, G);
  dot_normal<D>(G, n, Pn);
#pragma unroll
  for (int v = 0; v < NV; ++v) Gn[v] -= beta * Pn[v];
}

// LDG interior face flux seen from the left element (the one that meets the
// face with side 1, outward normal n): u_hat = U_L, q_hat = the right
// element's auxiliary gradient qR, penalty on U_L - U_R; no symmetric term
template <int D>
__device__ __forceinline__ void face_flux_ldg(const Phys& ph, const double* UL, const double* UR,
                                              const double (*qR)[D + 2], const double* n, double beta, double* H) {
  constexpr int NV = D + 2;
  double F[NV];
  if (ph.flux_mode == 2) {
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = 0.0;
  } else {
    riemann_flux<D>(ph, UL, UR, n, F);
  }
  if (ph.flux_mode == 1) {
#pragma unroll
    for (int v = 0; v < NV; ++v) H[v] = F[v];
    return;
  }
  double jump[NV], Gn[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) jump[v] = UL[v] - UR[v];
  ldg_viscous_n<D>(ph, UL, qR, jump, n, beta, Gn);
#pragma unroll
  for (int v = 0; v < NV; ++v) H[v] = F[v] - Gn[v];
}

// LDG boundary face flux: u_hat the mean of interior and ghost states, q_hat
// the interior auxiliary gradient, the same wall limits as the IP form
template <int D>
__device__ __forceinline__ void boundary_flux_ldg(const Phys& ph, int kind, const double* Uo,
                                                  const double (*qo)[D + 2], const double* n, double beta,
                                                  const double* Uinf, double* H) {
  constexpr int NV = D + 2;
  double Un[NV], F[NV];
  ghost_state<D>(ph, kind, Uo, n, Uinf, Un);
  if (ph.flux_mode == 2) {
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = 0.0;
  } else {
    riemann_flux<D>(ph, Uo, Un, n, F);
  }
  if (ph.flux_mode == 1) {
#pragma unroll
    for (int v = 0; v < NV; ++v) H[v] = F[v];
    return;
  }
  double Uh[NV], jump[NV], Gn[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) { Uh[v] = 0.5 * (Uo[v] + Un[v]); jump[v] = Uo[v] - Un[v]; }
  ldg_viscous_n<D>(ph, Uh, qo, jump, n, beta, Gn);
  if (kind == BC_WALL || kind == BC_SLIP) Gn[D + 1] = 0.0;
  if (kind == BC_SLIP) {
    double gn = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) gn += Gn[1 + c] * n[c];
#pragma unroll
    for (int c = 0; c < D; ++c) Gn[1 + c] = gn * n[c];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) H[v] = F[v] - Gn[v];
}

}  // namespace dgj
