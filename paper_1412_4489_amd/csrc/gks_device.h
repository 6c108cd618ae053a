// gks_device.h -- device arithmetic of the compact third-order gas-kinetic
// scheme (Pan & Xu, arXiv:1412.4489) for gfx950.
//
// The interface evaluation is split by magnitude.  In double precision: the
// interface values of the two reconstructed cells (Sec. 3.2 polynomials at the
// interface centre), their half-space moments (erfc, exp), the equilibrium
// state U0 (eq. compatibility2), its quadratic (Sec. 3.3), the collision time
// (Sec. 4), the exponential time integrals of C1..C8 (Sec. 2.2), and the
// leading flux and point-value terms (C1 g0 and C7 g_k, i.e. the Euler flux of
// U0 and the free-transport flux of the two sides).  In the compute type TC
// (float or double): everything that carries a derivative -- the expansion
// coefficients and the remaining moments of eq. dis1 / eq. dis2, generated
// in interface_gen.h in the peculiar frame of each Maxwellian.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "interface_gen.h"

namespace gks {

constexpr double kPi = 3.14159265358979323846;
constexpr double kGaussOffset = 0.28867513459481288225;  // sqrt(3)/6

// Physical and numerical constants of one problem (kernel argument).
struct Phys {
  double gamma;
  double K;        // internal degrees of freedom
  double nth;      // thermal degrees of freedom: K + 2 (2D), K + 1 (1D)
  double kp[4];    // kp[e] = K (K+2) ... (K+2e-2)
  double tau_eps, tau_c, mu, prfix;  // prfix = 1/Pr - 1
  double weno_eps, weno_c, cfl;
  int viscous;
};

// ---------------------------------------------------------------------------
// closed-form time integrals of C1..C8 (Sec. 2.2) over [0, dt] and their
// values at dt.  Index: 1..8 = C1..C8, 9 = C7 t, 10 = C7 t^2.
// ---------------------------------------------------------------------------
struct TimeWeights {
  double I[11];  // integrals
  double C[11];  // values at t = dt
};

__device__ __forceinline__ void time_weights(double tau, double dt, TimeWeights& w) {
  const double E = tau > 0.0 ? exp(-dt / tau) : 0.0;
  const double omE = 1.0 - E;
  const double t2 = tau * tau, t3 = t2 * tau, d2 = dt * dt;
  w.I[1] = dt - tau * omE;
  w.I[2] = 2.0 * t2 * omE - tau * dt * (1.0 + E);
  w.I[3] = 0.5 * d2 - tau * dt + t2 * omE;
  const double dp = dt + 2.0 * tau;
  w.I[4] = tau * dp * dp * E - 4.0 * t3;
  w.I[5] = d2 * dt * (1.0 / 3.0) - tau * d2;
  w.I[6] = t2 * dt * E - 0.5 * tau * d2 - t3 * omE;
  w.I[7] = tau * omE;
  w.I[8] = tau * (dt + tau) * E - t2;
  w.I[9] = t2 - tau * (dt + tau) * E;
  w.I[10] = 2.0 * t3 - tau * (d2 + 2.0 * tau * dt + 2.0 * t2) * E;
  w.C[1] = omE;
  w.C[2] = (dt + tau) * E - tau;
  w.C[3] = dt - tau * omE;
  w.C[4] = -(d2 + 2.0 * dt * tau) * E;
  w.C[5] = d2 - 2.0 * dt * tau;
  w.C[6] = -dt * tau * (1.0 + E);
  w.C[7] = E;
  w.C[8] = -dt * E;
  w.C[9] = dt * E;
  w.C[10] = d2 * E;
}

// ---------------------------------------------------------------------------
// Maxwellian helpers
// ---------------------------------------------------------------------------

// Lab-frame half-space moments <u^n>, n = 0..3, of a unit-density Maxwellian
// (U, lambda) over u > 0 (sgn = +1) or u < 0 (sgn = -1); also the peculiar
// first moment h1 = <u - U> over the same half space.
struct Half {
  double M0, M1, M2, M3, h1;
};

__device__ __forceinline__ Half half_moments(double U, double lam, double sgn) {
  Half m;
  const double sl = sqrt(lam);
  const double th = 0.5 / lam;
  m.M0 = 0.5 * erfc(-sgn * sl * U);
  m.h1 = sgn * 0.5 * exp(-lam * U * U) / sqrt(kPi * lam);
  m.M1 = U * m.M0 + m.h1;
  m.M2 = U * m.M1 + th * m.M0;
  m.M3 = U * m.M2 + 2.0 * th * m.M1;
  return m;
}

// Peculiar-frame transform of a moment target b (lab basis psi) for a
// Maxwellian moving with (U, V): b' = L^{-1} b.
__device__ __forceinline__ void to_frame_2d(const double* b, double U, double V, double* o) {
  o[0] = b[0];
  o[1] = b[1] - U * b[0];
  o[2] = b[2] - V * b[0];
  o[3] = b[3] - U * o[1] - V * o[2] - 0.5 * (U * U + V * V) * b[0];
}
__device__ __forceinline__ void to_frame_1d(const double* b, double U, double* o) {
  o[0] = b[0];
  o[1] = b[1] - U * b[0];
  o[2] = b[2] - U * o[1] - 0.5 * U * U * b[0];
}

// moment target of a derivative vector d (conservative variables) for the
// Maxwellian of density rho = 1/ir moving with (U, V), in its frame
template <typename T>
__device__ __forceinline__ void frame_rhs_2d(const double* d, double ir, double U, double V, T* o) {
  double b[4], f[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) b[v] = d[v] * ir;
  to_frame_2d(b, U, V, f);
#pragma unroll
  for (int v = 0; v < 4; ++v) o[v] = (T)f[v];
}

// lab-basis moments from peculiar-basis moments: m = L m'
template <typename T>
__device__ __forceinline__ void from_frame_2d(const T* m, double U, double V, double* o) {
  const double m0 = (double)m[0], m1 = (double)m[1], m2 = (double)m[2], m3 = (double)m[3];
  o[0] = m0;
  o[1] = m1 + U * m0;
  o[2] = m2 + V * m0;
  o[3] = m3 + U * m1 + V * m2 + 0.5 * (U * U + V * V) * m0;
}
template <typename T>
__device__ __forceinline__ void from_frame_1d(const T* m, double U, double* o) {
  const double m0 = (double)m[0], m1 = (double)m[1], m2 = (double)m[2];
  o[0] = m0;
  o[1] = m1 + U * m0;
  o[2] = m2 + U * m1 + 0.5 * U * U * m0;
}

// peculiar half-space moment table h[n] = <c^n>, c = u - U, n = 0..9
template <typename T>
__device__ __forceinline__ void half_table(const Half& m, double U, double lam, T* h) {
  double hd[10];
  const double th = 0.5 / lam;
  hd[0] = m.M0;
  hd[1] = m.h1;
  double mu_pow = 1.0;  // (-U)^n
  for (int n = 1; n < 9; ++n) {
    mu_pow *= -U;
    hd[n + 1] = n * th * hd[n - 1] + mu_pow * m.h1;
  }
#pragma unroll
  for (int n = 0; n < 10; ++n) h[n] = (T)hd[n];
}

template <typename T>
__device__ __forceinline__ void theta_powers(double th, T* t) {
  t[0] = T(1);
  double p = 1.0;
#pragma unroll
  for (int k = 1; k < 5; ++k) {
    p *= th;
    t[k] = (T)p;
  }
}

// ---------------------------------------------------------------------------
// one interface, 2D, in the interface frame (n normal, s tangential)
//   Wc[s][v], p[s][v][0..4] = (p_n, p_s, p_nn, p_ss, p_ns): cell averages and
//   reconstruction coefficients of the left (s = 0) and right (s = 1) cells;
//   Ueq[m][n][v]: averages of the six cells around the interface
//   (m: normal column, n: tangential row -1, 0, +1).
// Outputs: flux (time- and interface-integrated), point values at the
// tangential Gauss points -delta and +delta, heat flux (Navier-Stokes).
// Returns false for a nonphysical interface state.
// ---------------------------------------------------------------------------
template <typename TC>
__device__ __forceinline__ bool interface_2d(const Phys& P, double dt, double hn, double hs,
                                             const double (&Wc)[2][4], const double (&pc)[2][4][5],
                                             const double (&Ueq)[2][3][4], double (&flux)[4],
                                             double (&pvm)[4], double (&pvp)[4]) {
  const double g1 = P.gamma - 1.0;
  // interface values and derivatives of the two cell polynomials
  double W[2][4], Wn[2][4], Ws[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const double xn = s == 0 ? 0.5 * hn : -0.5 * hn;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double* p = pc[s][v];
      W[s][v] = Wc[s][v] + p[0] * xn + p[2] * (hn * hn * (1.0 / 12.0)) - p[3] * (hs * hs * (1.0 / 24.0));
      Wn[s][v] = p[0] + p[2] * xn;
      Ws[s][v] = p[1] + p[4] * xn;
    }
  }
  double rho[2], U[2], V[2], pr[2], lam[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    rho[s] = W[s][0];
    U[s] = W[s][1] / rho[s];
    V[s] = W[s][2] / rho[s];
    pr[s] = g1 * (W[s][3] - 0.5 * rho[s] * (U[s] * U[s] + V[s] * V[s]));
    lam[s] = 0.5 * rho[s] / pr[s];
  }
  if (!(rho[0] > 0.0) || !(rho[1] > 0.0) || !(pr[0] > 0.0) || !(pr[1] > 0.0)) return false;
  // U0 from the two half-space Maxwellians; free-transport flux of the sides
  const Half hm[2] = {half_moments(U[0], lam[0], 1.0), half_moments(U[1], lam[1], -1.0)};
  double W0[4] = {0, 0, 0, 0}, Fk[4] = {0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const double th = 0.5 / lam[s];
    const double e2 = V[s] * V[s] + (1.0 + P.K) * th;  // <v^2> + <xi^2>
    const Half& m = hm[s];
    W0[0] += rho[s] * m.M0;
    W0[1] += rho[s] * m.M1;
    W0[2] += rho[s] * V[s] * m.M0;
    W0[3] += rho[s] * 0.5 * (m.M2 + e2 * m.M0);
    Fk[0] += rho[s] * m.M1;
    Fk[1] += rho[s] * m.M2;
    Fk[2] += rho[s] * V[s] * m.M1;
    Fk[3] += rho[s] * 0.5 * (m.M3 + e2 * m.M1);
  }
  const double rho0 = W0[0], U0 = W0[1] / rho0, V0 = W0[2] / rho0;
  const double p0 = g1 * (W0[3] - 0.5 * rho0 * (U0 * U0 + V0 * V0));
  if (!(p0 > 0.0)) return false;
  const double lam0 = 0.5 * rho0 / p0;
  // equilibrium quadratic (Sec. 3.3): slopes / curvatures of U0 + b2 x + b3 y + ...
  double q[5][4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double L0 = Ueq[0][0][v], L1 = Ueq[0][1][v], L2 = Ueq[0][2][v];
    const double R0 = Ueq[1][0][v], R1 = Ueq[1][1][v], R2 = Ueq[1][2][v];
    q[0][v] = ((R2 - L2) + 2.0 * (R1 - L1) + (R0 - L0)) / (4.0 * hn);
    q[1][v] = (R2 - R0 + L2 - L0) / (4.0 * hs);
    q[2][v] = (26.0 * (R1 + L1) - (R2 + L2 + R0 + L0) - 48.0 * W0[v]) / (8.0 * hn * hn);
    q[3][v] = (R2 - 2.0 * R1 + R0 + L2 - 2.0 * L1 + L0) / (2.0 * hs * hs);
    q[4][v] = (R2 - L2 - R0 + L0) / (2.0 * hn * hs);
  }
  // collision time (Sec. 4)
  const double jump = fabs((pr[0] - pr[1]) / (pr[0] + pr[1]));
  const double tau = P.viscous ? P.mu / p0 + P.tau_c * jump * dt : (P.tau_eps + P.tau_c * jump) * dt;
  TimeWeights w;
  time_weights(tau, dt, w);
  // leading terms: Euler flux of U0 and free transport of the sides
  {
    const double pe = p0;
    const double FE[4] = {W0[1], W0[1] * U0 + pe, W0[1] * V0, U0 * (W0[3] + pe)};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      flux[v] = hs * (w.I[1] * FE[v] + w.I[7] * Fk[v]);
      pvm[v] = W0[v];
      pvp[v] = W0[v];
    }
  }
  double Edens[4];  // time- and interface-integrated <psi f> (for the heat flux)
#pragma unroll
  for (int v = 0; v < 4; ++v) Edens[v] = hs * dt * W0[v];

  TC kp[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) kp[e] = (TC)P.kp[e];
  const TC nth = (TC)P.nth;
  const double delta = kGaussOffset * hs;

  // ---- hydrodynamic part, g0 -------------------------------------------
  {
    TC th[5];
    theta_powers(0.5 / lam0, th);
    const double ir = 1.0 / rho0;
    TC bx[4], by[4], bxx[4], bxy[4], byy[4];
    frame_rhs_2d(q[0], ir, U0, V0, bx);
    frame_rhs_2d(q[1], ir, U0, V0, by);
    frame_rhs_2d(q[2], ir, U0, V0, bxx);
    frame_rhs_2d(q[4], ir, U0, V0, bxy);
    frame_rhs_2d(q[3], ir, U0, V0, byy);
    TC ax[4], ay[4], At[4], dxx[4], dxy[4], dyy[4], bxt[4], byt[4], Bt[4];
    coef_g0_2d<TC>(th, kp, nth, (TC)U0, (TC)V0, bx, by, bxx, bxy, byy, ax, ay, At, dxx, dxy, dyy, bxt, byt, Bt);
    TC wI[7], wC[7];
#pragma unroll
    for (int k = 1; k < 7; ++k) {
      wI[k] = (TC)w.I[k];
      wC[k] = (TC)w.C[k];
    }
    const TC wI1y = (TC)(w.I[1] * hs * hs * (1.0 / 24.0));
    TC AF[4], BF[4], V0m[4], V1m[4], V2m[4];
    hydro_2d<TC>(th, kp, (TC)U0, (TC)V0, ax, ay, At, dxx, dxy, dyy, bxt, byt, Bt, wI, wI1y, wC, AF, BF, V0m, V1m,
                 V2m);
    TC fl[4], pm[4], pp[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      fl[v] = BF[v] + (TC)U0 * AF[v];
      pm[v] = V0m[v] - (TC)delta * V1m[v] + (TC)(delta * delta) * V2m[v];
      pp[v] = V0m[v] + (TC)delta * V1m[v] + (TC)(delta * delta) * V2m[v];
    }
    double a[4];
    from_frame_2d(fl, U0, V0, a);
#pragma unroll
    for (int v = 0; v < 4; ++v) flux[v] += hs * rho0 * a[v];
    from_frame_2d(pm, U0, V0, a);
#pragma unroll
    for (int v = 0; v < 4; ++v) pvm[v] += rho0 * a[v];
    from_frame_2d(pp, U0, V0, a);
#pragma unroll
    for (int v = 0; v < 4; ++v) pvp[v] += rho0 * a[v];
    if (P.viscous) {
      from_frame_2d(AF, U0, V0, a);
#pragma unroll
      for (int v = 0; v < 4; ++v) Edens[v] += hs * rho0 * a[v];
    }
  }

  // ---- kinetic parts of the two sides ----------------------------------
  const TC kI8 = (TC)w.I[8], kI72 = (TC)(0.5 * w.I[10]), kI7y = (TC)(w.I[7] * hs * hs * (1.0 / 24.0));
  const TC kI7tau = (TC)(tau * w.I[7]), kI8tau = (TC)(tau * w.I[8]);
  const TC kC8 = (TC)w.C[8], kC72 = (TC)(0.5 * w.C[10]), kC7 = (TC)w.C[7], kC7t = (TC)w.C[9];
  const TC kC7tau = (TC)(tau * w.C[7]), kC8tau = (TC)(tau * w.C[8]);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    TC th[5];
    theta_powers(0.5 / lam[s], th);
    const double ir = 1.0 / rho[s];
    TC bx[4], by[4], bxx[4], bxy[4], byy[4];
    {
      double dnn[4], dns[4], dss[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        dnn[v] = pc[s][v][2];
        dns[v] = pc[s][v][4];
        dss[v] = pc[s][v][3];
      }
      frame_rhs_2d(Wn[s], ir, U[s], V[s], bx);
      frame_rhs_2d(Ws[s], ir, U[s], V[s], by);
      frame_rhs_2d(dnn, ir, U[s], V[s], bxx);
      frame_rhs_2d(dns, ir, U[s], V[s], bxy);
      frame_rhs_2d(dss, ir, U[s], V[s], byy);
    }
    TC ax[4], ay[4], At[4], dxx[4], dxy[4], dyy[4], bxt[4], byt[4], Bt[4];
    TC h[10];
    half_table(hm[s], U[s], lam[s], h);
    TC AF[4], BF[4], V0m[4], V1m[4], V2m[4];
    if (P.viscous) {
      coef_side_ns_2d<TC>(th, kp, nth, (TC)U[s], (TC)V[s], bx, by, bxx, bxy, byy, ax, ay, At, dxx, dxy, dyy, bxt,
                          byt, Bt);
      kin_ns_2d<TC>(th, kp, h, (TC)U[s], (TC)V[s], ax, ay, At, dxx, dxy, dyy, bxt, byt, kI8, kI72, kI7y, kI7tau,
                    kI8tau, kC8, kC72, kC7, kC7t, kC7tau, kC8tau, AF, BF, V0m, V1m, V2m);
    } else {
      coef_side_euler_2d<TC>(th, kp, nth, (TC)U[s], (TC)V[s], bx, by, bxx, bxy, byy, ax, ay, At, dxx, dxy, dyy,
                             bxt, byt, Bt);
      kin_euler_2d<TC>(th, kp, h, (TC)U[s], (TC)V[s], ax, ay, At, dxx, dxy, dyy, bxt, byt, kI8, kI72, kI7y, kI7tau,
                       kI8tau, kC8, kC72, kC7, kC7t, kC7tau, kC8tau, AF, BF, V0m, V1m, V2m);
    }
    TC fl[4], pm[4], pp[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      fl[v] = BF[v] + (TC)U[s] * AF[v];
      pm[v] = V0m[v] - (TC)delta * V1m[v] + (TC)(delta * delta) * V2m[v];
      pp[v] = V0m[v] + (TC)delta * V1m[v] + (TC)(delta * delta) * V2m[v];
    }
    double a[4];
    from_frame_2d(fl, U[s], V[s], a);
#pragma unroll
    for (int v = 0; v < 4; ++v) flux[v] += hs * rho[s] * a[v];
    from_frame_2d(pm, U[s], V[s], a);
#pragma unroll
    for (int v = 0; v < 4; ++v) pvm[v] += rho[s] * a[v];
    from_frame_2d(pp, U[s], V[s], a);
#pragma unroll
    for (int v = 0; v < 4; ++v) pvp[v] += rho[s] * a[v];
    if (P.viscous) {
      from_frame_2d(AF, U[s], V[s], a);
#pragma unroll
      for (int v = 0; v < 4; ++v) Edens[v] += hs * rho[s] * a[v];
    }
  }
  if (P.viscous) {
    // heat flux relative to the velocity of g0, added with weight 1/Pr - 1
    const double k2 = 0.5 * (U0 * U0 + V0 * V0);
    const double qh = flux[3] - U0 * flux[1] - V0 * flux[2] + k2 * flux[0] -
                      U0 * (Edens[3] - U0 * Edens[1] - V0 * Edens[2] + k2 * Edens[0]);
    flux[3] += P.prfix * qh;
  }
  return true;
}

// ---------------------------------------------------------------------------
// compact reconstruction of one scalar (Sec. 3.1 / 3.2)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double mm2(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return fabs(a) < fabs(b) ? a : b;
}

// 2D: c = cell average; e, w, n, s = face-neighbour averages; E+-, W+-, N+-, S+-
// = Gauss-point values on the four interfaces.  p = (p2..p6).
// The quantities that decide branches (the one-sided estimates, the minmod
// arguments and the cross-derivative candidates) are formed in the order of
// their printed formulas and without FMA contraction, so that a tie or a sign
// is decided from the same rounded values as in a plain evaluation.
__device__ __forceinline__ void recon_2d(double c, double e, double w, double n, double s, double Ep, double Em,
                                         double Wp, double Wm, double Np, double Nm, double Sp, double Sm, double h,
                                         double k, double eps, double Cw, double* p) {
#pragma clang fp contract(off)
  // eq. over-sys: normal (x) and tangential (y) pairs of the one-sided stencils
  const double cxE = 3.0 * ((c + e) - (Ep + Em)) / (h * h), sxE = (Ep + Em - 2.0 * c) / h;
  const double cxW = 3.0 * ((c + w) - (Wp + Wm)) / (h * h), sxW = (Wp + Wm - 2.0 * c) / h;
  const double cyN = 3.0 * ((c + n) - (Np + Nm)) / (k * k), syN = (Np + Nm - 2.0 * c) / k;
  const double cyS = 3.0 * ((c + s) - (Sp + Sm)) / (k * k), syS = (Sp + Sm - 2.0 * c) / k;
  // eq. limiter on each pair
  const double a4 = mm2(cxW, cxE);
  const double a2 = mm2(-sxW + a4 * h / 6.0, sxE - a4 * h / 6.0);
  const double a5 = mm2(cyS, cyN);
  const double a3 = mm2(-syS + a5 * k / 6.0, syN - a5 * k / 6.0);
  // cross term of the stencils NE, NW, SW, SE with the limited slopes; the one
  // of smallest magnitude (the earlier one on an exact tie)
  const double s3 = 1.7320508075688772;  // sqrt(3)
  const double dE = Ep - Em, dW = Wp - Wm, dN = Np - Nm, dS = Sp - Sm;
  const double hk = h * k;
  double a6 = s3 * (dE + dN) / hk - (a2 / k + a3 / h);
  double cand = s3 * (dN - dW) / hk - (a2 / k - a3 / h);
  if (fabs(cand) < fabs(a6)) a6 = cand;
  cand = -s3 * (dS + dW) / hk + (a2 / k + a3 / h);
  if (fabs(cand) < fabs(a6)) a6 = cand;
  cand = s3 * (dE - dS) / hk + (a2 / k - a3 / h);
  if (fabs(cand) < fabs(a6)) a6 = cand;
  // central stencil
  const double c2 = (e - w) / (2.0 * h), c4 = (e - 2.0 * c + w) / (h * h);
  const double c3 = (n - s) / (2.0 * k), c5 = (n - 2.0 * c + s) / (k * k);
  const double c6 = s3 * ((dE - dW) + (dN - dS)) / (2.0 * hk);
  // nonlinear weights, I(U1) = C |cell|, I(U2) from the derivatives of U2
  const double A = hk;
  const double I1 = Cw * A;
  const double I2 = A * (c2 * c2 + c3 * c3) + A * (c4 * c4 * (h * h / 12.0 + A) + c5 * c5 * (k * k / 12.0 + A) +
                                                  c6 * c6 * ((h * h + k * k) / 12.0 + A));
  const double b1 = 1.0 / ((eps + I1) * (eps + I1)), b2 = 1.0 / ((eps + I2) * (eps + I2));
  const double w1 = b1 / (b1 + b2), w2 = b2 / (b1 + b2);
  p[0] = w1 * a2 + w2 * c2;
  p[1] = w1 * a3 + w2 * c3;
  p[2] = w1 * a4 + w2 * c4;
  p[3] = w1 * a5 + w2 * c5;
  p[4] = w1 * a6 + w2 * c6;
}

}  // namespace gks
