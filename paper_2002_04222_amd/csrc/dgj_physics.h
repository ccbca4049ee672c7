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
  int riemann;     // 0 Roe, 1 local Lax-Friedrichs
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
  T irho = 1.0 / rho;
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
  T irho = 1.0 / rho;
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
  double rL = UL[0], rR = UR[0];
  double vL[D], vR[D], kL = 0.0, kR = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    vL[c] = UL[1 + c] / rL; vR[c] = UR[1 + c] / rR;
    kL += vL[c] * UL[1 + c]; kR += vR[c] * UR[1 + c];
  }
  double pL = (g - 1.0) * (UL[D + 1] - 0.5 * kL);
  double pR = (g - 1.0) * (UR[D + 1] - 0.5 * kR);
  double HL = (UL[D + 1] + pL) / rL, HR = (UR[D + 1] + pR) / rR;
  double sL = sqrt(rL), sR = sqrt(rR);
  double rt = sL * sR;
  double isum = 1.0 / (sL + sR);
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
  double a1 = (dp - rt * ct * dun) / (2.0 * c2);
  double a5 = (dp + rt * ct * dun) / (2.0 * c2);
  double a2 = dr - dp / c2;
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

// Numerical normal flux seen from side 'o' with outward normal n:
//   H = Fhat(Uo, Un, n) - [ n.G(Ubar, {gU}) - beta n.G(Ubar, dU (x) n) ]
//   S[j] = 1/2 n.G(Ubar, dU (x) e_j)
// with Ubar = (Uo+Un)/2, dU = Uo - Un (interior penalty, Eq. 12 with a
// dissipative penalty and the 1/2 of the test-gradient average).
// S is optional (nullptr skips it).
template <int D>
__device__ __forceinline__ void face_flux(const Phys& ph, const double* Uo, const double* Un,
                                          const double (*go)[D + 2], const double (*gn)[D + 2],
                                          const double* n, double beta, double* H, double (*S)[D + 2]) {
  constexpr int NV = D + 2;
  double F[NV];
  if (ph.flux_mode == 2) {
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = 0.0;
  } else if (ph.riemann == 0) {
    roe_flux<D>(ph, Uo, Un, n, F);
  } else {
    llf_flux<D>(ph, Uo, Un, n, F);
  }
  if (ph.flux_mode == 1) {
#pragma unroll
    for (int v = 0; v < NV; ++v) H[v] = F[v];
    if (S) {
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
  double ga[D][NV], G[D][NV], Gn[NV], Pn[NV];
#pragma unroll
  for (int j = 0; j < D; ++j)
#pragma unroll
    for (int v = 0; v < NV; ++v) ga[j][v] = 0.5 * (go[j][v] + gn[j][v]);
  viscous_flux<D, double, double>(ph, Ub, ga, G);
  dot_normal<D>(G, n, Gn);
#pragma unroll
  for (int j = 0; j < D; ++j)
#pragma unroll
    for (int v = 0; v < NV; ++v) ga[j][v] = n[j] * dU[v];
  viscous_flux<D, double, double>(ph, Ub, ga, G);
  dot_normal<D>(G, n, Pn);
#pragma unroll
  for (int v = 0; v < NV; ++v) H[v] = F[v] - (Gn[v] - beta * Pn[v]);
  if (S) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int v = 0; v < NV; ++v) ga[i][v] = (i == j) ? dU[v] : 0.0;
      viscous_flux<D, double, double>(ph, Ub, ga, G);
      double t[NV];
      dot_normal<D>(G, n, t);
#pragma unroll
      for (int v = 0; v < NV; ++v) S[j][v] = 0.5 * t[v];
    }
  }
}

// ---------------------------------------------------------------- boundary conditions
// A boundary face takes the interior trace and a ghost state with the
// interior gradient, and the interior-face fluxes apply.  Far field: 1D
// characteristic (Riemann-invariant) state against the freestream Uinf,
// with the inflow/outflow choice of entropy and tangential velocity blended
// by w = (1 + tanh(u_nb / (0.02 c_b)))/2;
// no-slip wall: mirrored momentum (zero wall velocity), with the heat flux
// through the wall zero (adiabatic), so the viscous energy fluxes vanish.
enum { BC_FARFIELD = 0, BC_WALL = 1, BC_DIRICHLET = 2 };

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

// boundary face flux seen from the interior (outward normal n)
template <int D>
__device__ __forceinline__ void boundary_flux(const Phys& ph, int kind, const double* Uo, const double (*go)[D + 2],
                                              const double* n, double beta, const double* Uinf, double* H,
                                              double (*S)[D + 2]) {
  constexpr int NV = D + 2;
  double Un[NV];
  if (kind == BC_DIRICHLET) {
    // the given state at this face point (Uinf points at it)
#pragma unroll
    for (int v = 0; v < NV; ++v) Un[v] = Uinf[v];
  } else if (kind == BC_FARFIELD) {
    farfield_ghost<D>(ph, Uo, n, Uinf, Un);
  } else {
    Un[0] = Uo[0];
#pragma unroll
    for (int c = 0; c < D; ++c) Un[1 + c] = -Uo[1 + c];
    Un[D + 1] = Uo[D + 1];
  }
  face_flux<D>(ph, Uo, Un, go, go, n, beta, H, S);
  if (kind == BC_WALL) {
    double F[NV];
    if (ph.flux_mode == 2) {
#pragma unroll
      for (int v = 0; v < NV; ++v) F[v] = 0.0;
    } else if (ph.riemann == 0) {
      roe_flux<D>(ph, Uo, Un, n, F);
    } else {
      llf_flux<D>(ph, Uo, Un, n, F);
    }
    H[D + 1] = F[D + 1];
    if (S) {
#pragma unroll
      for (int j = 0; j < D; ++j) S[j][D + 1] = 0.0;
    }
  }
}

}  // namespace dgj
