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

__device__ __forceinline__ double decay(double tau, double dt) { return tau > 0.0 ? exp(-dt / tau) : 0.0; }

// E = decay(tau, dt) = e^{-dt/tau}
__device__ __forceinline__ void time_weights(double tau, double dt, double E, TimeWeights& w) {
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

// the recurrence from <u^0> and h1
__device__ __forceinline__ Half half_moments_from(double M0, double h1, double U, double lam) {
  Half m;
  const double th = 0.5 / lam;
  m.M0 = M0;
  m.h1 = h1;
  m.M1 = U * m.M0 + m.h1;
  m.M2 = U * m.M1 + th * m.M0;
  m.M3 = U * m.M2 + 2.0 * th * m.M1;
  return m;
}
__device__ __forceinline__ Half half_moments(double U, double lam, double sgn) {
  const double sl = sqrt(lam);
  return half_moments_from(0.5 * erfc(-sgn * sl * U), sgn * 0.5 * exp(-lam * U * U) / sqrt(kPi * lam), U, lam);
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

// Knudsen reading of eq. dis2 (Navier-Stokes): the correction
// -tau (a1 u + a2 v + A) g_k of a side's initial distribution is the
// first-order Chapman-Enskog expansion, valid while the side's cell Knudsen
// number tau s is below one, s the rate at which its equilibrium changes for
// a particle at the sound speed c: the sum over the normal and tangential
// derivatives of c |d rho| / rho + |d u| + |d v| + |d (rho e)| / (rho c).
// Where tau s exceeds one the correction takes tau capped at 1 / s (the
// relaxation keeps tau); in resolved flow it is the printed bracket.
// rate_term: one direction's share from the frame derivatives f of
// to_frame (f0 = d rho / rho, f1, f2 = d u, d v, f3 = d (rho e) / rho).
__device__ __forceinline__ double rate_term(double c, double f0, double fu, double fv, double fe) {
  return c * fabs(f0) + fabs(fu) + fabs(fv) + fabs(fe) / c;
}
__device__ __forceinline__ double bracket_tau(double tau, double s) { return tau * s > 1.0 ? 1.0 / s : tau; }

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

// Accumulators of the correction moments of one Maxwellian in its frame:
// flux moments AF = <psi' P_F>, BF = <c psi' P_F>, and the point values at the
// two Gauss points y = -delta (PM) and +delta (PP) of the interface, to which
// the y^0, y^1, y^2 parts contribute with weights 1, -+delta, delta^2.
template <typename TC>
struct Acc {
  TC AF[4] = {0, 0, 0, 0}, BF[4] = {0, 0, 0, 0}, PM[4] = {0, 0, 0, 0}, PP[4] = {0, 0, 0, 0};
  TC d, d2;
  __device__ __forceinline__ explicit Acc(double delta) : d((TC)delta), d2((TC)(delta * delta)) {}
  __device__ __forceinline__ void flux(const TC* m0, const TC* m1, TC w) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      AF[v] += w * m0[v];
      BF[v] += w * m1[v];
    }
  }
  __device__ __forceinline__ void pv0(const TC* m0, TC w) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const TC a = w * m0[v];
      PM[v] += a;
      PP[v] += a;
    }
  }
  __device__ __forceinline__ void pv1(const TC* m0, TC w) {
    const TC wd = w * d;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const TC a = wd * m0[v];
      PM[v] -= a;
      PP[v] += a;
    }
  }
  __device__ __forceinline__ void pv2(const TC* m0, TC w) {
    const TC wd = w * d2;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const TC a = wd * m0[v];
      PM[v] += a;
      PP[v] += a;
    }
  }
  // back to lab-frame moments, times rho (and the interface length for the
  // integrated flux), added to the double-precision totals
  __device__ __forceinline__ void add_to(double U, double V, double rho, double hs, double* flux, double* pvm,
                                         double* pvp, double* Edens) const {
    TC fl[4];
    const TC u = (TC)U;
#pragma unroll
    for (int v = 0; v < 4; ++v) fl[v] = BF[v] + u * AF[v];
    double a[4];
    from_frame_2d(fl, U, V, a);
#pragma unroll
    for (int v = 0; v < 4; ++v) flux[v] += hs * rho * a[v];
    from_frame_2d(PM, U, V, a);
#pragma unroll
    for (int v = 0; v < 4; ++v) pvm[v] += rho * a[v];
    from_frame_2d(PP, U, V, a);
#pragma unroll
    for (int v = 0; v < 4; ++v) pvp[v] += rho * a[v];
    if (Edens) {
      from_frame_2d(AF, U, V, a);
#pragma unroll
      for (int v = 0; v < 4; ++v) Edens[v] += hs * rho * a[v];
    }
  }
};

// ---------------------------------------------------------------------------
// One 2D interface is evaluated by one thread in four sections, each holding
// only its own working set in registers; what passes between them (the frame
// record of g0) lives in the thread's slots of LDS:
//   prologue  (double)  interface values of the two cell polynomials, their
//                       half-space moments, U0 (eq. compatibility2), the
//                       equilibrium quadratic (Sec. 3.3), tau (Sec. 4); the
//                       leading flux and point values; (TC) the expansion
//                       coefficients of g0 (FP32-mixed); the record of g0;
//   hydro     (TC)      the terms of eq. dis1 (FP64: after solving the
//                       coefficients of g0 from the recorded targets);
//   kinetic   (double)  the side's interface state and targets (single
//                       precision: from the record, where the prologue put
//                       them; double: again from its cell, same arithmetic
//                       as in the prologue), its half-space moments from the
//                       prologue's <u^0> and h1 in the record, (TC) the
//                       coefficients of g_k and the terms of eq. dis2 (once
//                       per side).
// The later sections take e^{-dt/tau} from the record too.
// The sums keep the order ((prologue + hydrodynamic) + side 0) + side 1.
// The record is a structure of arrays over the threads of a block.
// ---------------------------------------------------------------------------
enum HydroW { HW_I2, HW_I3, HW_I4H, HW_I5H, HW_I6, HW_I1Y, HW_C2, HW_C3, HW_C4H, HW_C5H, HW_C6, HW_C1, HW_C1H };
enum KinW { KW_ICONV, KW_CCONV, KW_IQUAD, KW_CQUAD, KW_IY, KW_C7H, KW_C7, KW_CINNER, KW_AI, KW_AC, KW_TI, KW_TC };
enum RecD {  // double fields
  D_RHO0, D_U0, D_V0, D_LAM0,
  D_TAU,                    // collision time (the sections rebuild the time weights)
  D_E0, D_E1, D_E2, D_E3,  // time- and interface-integrated <psi f> (heat flux; Navier-Stokes only)
  D_RATE0, D_RATE1,        // each side's rate s (Knudsen reading; Navier-Stokes only; kinetic sections)
  D_DECAY,                  // e^{-dt/tau} (the time weights of the later sections)
  D_HM0, D_HH1, D_HM1, D_HH2,  // each side's half-space <u^0> and h1 (its half-space moments, eq. compatibility2)
  D_SIDE,                   // single-precision compute type: each side's interface state rho, U, V, p, lambda (10)
  ND_REC = D_SIDE + 10
};
enum RecT {  // compute-type fields
  T_CG = 0,  // g0 coefficients ax, ay, A, dxx, dxy, dyy, bx, by, B (9 x 4), peculiar frame; in double
             // precision its targets bx, by, bxx, bxy, byy (5 x 4)
  T_SB = 36  // single precision: each side's expansion targets (2 x 5 x 4, peculiar frame)
};

// Where the coefficient systems of g0 are solved: in the prologue for a
// single-precision compute type (it then leaves the hydrodynamic phase within
// two waves per SIMD), in the hydrodynamic phase for double precision (where
// the prologue would lose its second wave).
template <typename TC>
constexpr bool g0_solved_in_prologue() {
  return sizeof(TC) == 4;
}
// Whether the prologue hands each side's interface state and targets to its
// kinetic section through the record (single-precision compute type: 240 B
// more per thread still leave room in LDS for four waves per compute unit),
// or the kinetic section reloads its cell and rebuilds them (double: the
// record would halve the waves a compute unit holds).
template <typename TC>
constexpr bool sides_in_record() {
  return sizeof(TC) == 4;
}
// compute-type fields of the record: 36 coefficients (+ 40 side targets) or
// 20 targets
template <typename TC>
constexpr int nt_rec() {
  return g0_solved_in_prologue<TC>() ? (sides_in_record<TC>() ? 76 : 36) : 20;
}

// weights of the terms of eq. dis1 (hydro) and eq. dis2 (kinetic) from the
// time integrals (flux) and values at dt (point values) of C1..C8
__device__ __forceinline__ void hydro_weights(const TimeWeights& w, double hs, double (&hw)[13]) {
  const double hs2 = hs * hs * (1.0 / 24.0);
  hw[HW_I2] = w.I[2];
  hw[HW_I3] = w.I[3];
  hw[HW_I4H] = 0.5 * w.I[4];
  hw[HW_I5H] = 0.5 * w.I[5];
  hw[HW_I6] = w.I[6];
  hw[HW_I1Y] = w.I[1] * hs2;
  hw[HW_C2] = w.C[2];
  hw[HW_C3] = w.C[3];
  hw[HW_C4H] = 0.5 * w.C[4];
  hw[HW_C5H] = 0.5 * w.C[5];
  hw[HW_C6] = w.C[6];
  hw[HW_C1] = w.C[1];
  hw[HW_C1H] = 0.5 * w.C[1];
}
__device__ __forceinline__ void kinetic_weights(const TimeWeights& w, double tau, double tv, double hs,
                                                double (&kw)[12]) {
  const double hs2 = hs * hs * (1.0 / 24.0);
  kw[KW_ICONV] = w.I[8] - tv * w.I[7];
  kw[KW_CCONV] = w.C[8] - tv * w.C[7];
  kw[KW_IQUAD] = 0.5 * w.I[10] - tv * w.I[8];
  kw[KW_CQUAD] = 0.5 * w.C[10] - tv * w.C[8];
  kw[KW_IY] = w.I[7] * hs2;
  kw[KW_C7H] = 0.5 * w.C[7];
  kw[KW_C7] = w.C[7];
  kw[KW_CINNER] = -w.C[9] - tv * w.C[7];
  kw[KW_AI] = -tau * w.I[7];
  kw[KW_AC] = -tau * w.C[7];
  kw[KW_TI] = -tau * w.I[8];
  kw[KW_TC] = -tau * w.C[8];
}

// the frame record of the threads of a block (structure of arrays: field k
// of thread f at k * nf + f)
template <typename TC>
struct Rec {
  double* d;
  TC* t;
  unsigned nf;
  __device__ __forceinline__ double& D(int k, unsigned f) const { return d[(unsigned)k * nf + f]; }
  __device__ __forceinline__ TC& T(int k, unsigned f) const { return t[(unsigned)k * nf + f]; }
};

// coefficient-set arrays of one Maxwellian (peculiar frame)
template <typename TC>
struct Coefs {
  TC ax[4], ay[4], At[4], dxx[4], dxy[4], dyy[4], bxt[4], byt[4], Bt[4];
};

// Division by a divisor b with a precomputed reciprocal rb = RN(1/b): the
// quotient q = RN(a rb) is within one ulp of a/b, its remainder a - q b is
// exact with an FMA, and q + remainder rb rounded once is the correctly
// rounded a/b (Markstein's correction step; finite normal operands), the
// same bits as the division itself in three dependent operations.
struct Divisor {
  double b, rb;
};
__device__ __forceinline__ Divisor divisor(double b) { return Divisor{b, 1.0 / b}; }
__device__ __forceinline__ double div_by(double a, const Divisor& d) {
#pragma clang fp contract(off)
  const double q = a * d.rb;
  const double r = fma(-q, d.b, a);
  return fma(r, d.rb, q);
}

// State of side s (0: left cell, 1: right cell) at the interface centre from
// its cell average Wc and reconstruction pc = (p_n, p_s, p_nn, p_ss, p_ns) in
// the interface frame; false if nonphysical.
struct Side {
  double rho, U, V, pr, lam;
};
__device__ __forceinline__ bool side_state_2d(const Phys& P, int s, double hn, double hs, const double (&Wc)[4],
                                              const double (&pc)[4][5], Side& o) {
  const double xn = s == 0 ? 0.5 * hn : -0.5 * hn;
  double W[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double* p = pc[v];
    W[v] = Wc[v] + p[0] * xn + p[2] * (hn * hn * (1.0 / 12.0)) - p[3] * (hs * hs * (1.0 / 24.0));
  }
  o.rho = W[0];
  const Divisor dr = divisor(o.rho);
  o.U = div_by(W[1], dr);
  o.V = div_by(W[2], dr);
  o.pr = (P.gamma - 1.0) * (W[3] - 0.5 * o.rho * (o.U * o.U + o.V * o.V));
  o.lam = 0.5 * o.rho / o.pr;
  return o.rho > 0.0 && o.pr > 0.0;
}

template <typename TC>
__device__ __forceinline__ void side_targets_2d(int s, double hn, const Side& S, const double (&pc)[4][5],
                                                TC (&b)[5][4]) {
  const double ir = 1.0 / S.rho, xn = s == 0 ? 0.5 * hn : -0.5 * hn;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double d[4], f[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double* p = pc[v];
      d[v] = (k == 0 ? p[0] + p[2] * xn : k == 1 ? p[1] + p[4] * xn : k == 2 ? p[2] : k == 3 ? p[4] : p[3]) * ir;
    }
    to_frame_2d(d, S.U, S.V, f);
#pragma unroll
    for (int v = 0; v < 4; ++v) b[k][v] = (TC)f[v];
  }
}

// Prologue of interface f.  Wc[s][v], pc[s][v][0..4] = (p_n, p_s, p_nn, p_ss,
// p_ns): averages and reconstruction coefficients of the left (s = 0) and
// right (s = 1) cells in the interface frame; Ueq[m][n][v]: the six averages
// around the interface.  Writes the record of g0 (state, tau, expansion
// coefficients) and returns the leading flux (C1 g0 and C7 g_k terms) and the
// leading point value U0.
// kCurv (an interface of a curvilinear grid): Ueq are the six averages in
// the grid's logical orientation with frame momentum components; the
// equilibrium quadratic is formed with unit spacing and turned into frame
// derivatives with the metric Gm = (G_nn, G_ns, G_tt) (d/dn = G_nn d/dxi +
// G_ns d/deta, d/dt = G_tt d/deta).
template <typename TC, bool kCurv = false>
__device__ __forceinline__ bool iface_prologue_2d(const Phys& P, double dt, double hn, double hs,
                                                  const double (&Wc)[2][4], const double (&pc)[2][4][5],
                                                  const double (&Ueq)[2][3][4], const Rec<TC>& R, unsigned f,
                                                  double (&flux)[4], double (&pv)[4],
                                                  const double* Gm = nullptr) {
  const double g1 = P.gamma - 1.0;
  Side S[2];
  const bool okl = side_state_2d(P, 0, hn, hs, Wc[0], pc[0], S[0]);
  const bool okr = side_state_2d(P, 1, hn, hs, Wc[1], pc[1], S[1]);
  if (!okl || !okr) return false;
  if constexpr (sides_in_record<TC>()) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      R.D(D_SIDE + 5 * s + 0, f) = S[s].rho;
      R.D(D_SIDE + 5 * s + 1, f) = S[s].U;
      R.D(D_SIDE + 5 * s + 2, f) = S[s].V;
      R.D(D_SIDE + 5 * s + 3, f) = S[s].pr;
      R.D(D_SIDE + 5 * s + 4, f) = S[s].lam;
      TC b[5][4];
      side_targets_2d(s, hn, S[s], pc[s], b);
#pragma unroll
      for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int v = 0; v < 4; ++v) R.T(T_SB + 20 * s + 4 * k + v, f) = b[k][v];
    }
  }
  double W0[4] = {0, 0, 0, 0}, Fk[4] = {0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const Half m = half_moments(S[s].U, S[s].lam, s == 0 ? 1.0 : -1.0);
    R.D(D_HM0 + 2 * s, f) = m.M0;
    R.D(D_HH1 + 2 * s, f) = m.h1;
    const double th = 0.5 / S[s].lam, rho = S[s].rho, V = S[s].V;
    const double e2 = V * V + (1.0 + P.K) * th;  // <v^2> + <xi^2>
    W0[0] += rho * m.M0;
    W0[1] += rho * m.M1;
    W0[2] += rho * V * m.M0;
    W0[3] += rho * 0.5 * (m.M2 + e2 * m.M0);
    Fk[0] += rho * m.M1;
    Fk[1] += rho * m.M2;
    Fk[2] += rho * V * m.M1;
    Fk[3] += rho * 0.5 * (m.M3 + e2 * m.M1);
  }
  const Divisor d0 = divisor(W0[0]);
  const double rho0 = W0[0], U0 = div_by(W0[1], d0), V0 = div_by(W0[2], d0);
  const double p0 = g1 * (W0[3] - 0.5 * rho0 * (U0 * U0 + V0 * V0));
  if (!(p0 > 0.0)) return false;
  const double lam0 = 0.5 * rho0 / p0;
  R.D(D_RHO0, f) = rho0;
  R.D(D_U0, f) = U0;
  R.D(D_V0, f) = V0;
  R.D(D_LAM0, f) = lam0;
  // equilibrium quadratic (Sec. 3.3) -> targets and coefficients of g0
  {
    const double ir = 1.0 / rho0;
    TC b[5][4];
    if constexpr (kCurv) {
      double q[5][4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double L0 = Ueq[0][0][v], L1 = Ueq[0][1][v], L2 = Ueq[0][2][v];
        const double R0 = Ueq[1][0][v], R1 = Ueq[1][1][v], R2 = Ueq[1][2][v];
        // logical derivatives (unit spacing)
        const double lx = 0.25 * ((R2 - L2) + 2.0 * (R1 - L1) + (R0 - L0));
        const double ly = 0.25 * (R2 - R0 + L2 - L0);
        const double lxx = 0.125 * (26.0 * (R1 + L1) - (R2 + L2 + R0 + L0) - 48.0 * W0[v]);
        const double lxy = 0.5 * (R2 - L2 - R0 + L0);
        const double lyy = 0.5 * (R2 - 2.0 * R1 + R0 + L2 - 2.0 * L1 + L0);
        const double g00 = Gm[0], g01 = Gm[1], g11 = Gm[2];
        q[0][v] = (g00 * lx + g01 * ly) * ir;
        q[1][v] = g11 * ly * ir;
        q[2][v] = (g00 * g00 * lxx + 2.0 * g00 * g01 * lxy + g01 * g01 * lyy) * ir;
        q[3][v] = g11 * (g00 * lxy + g01 * lyy) * ir;
        q[4][v] = g11 * g11 * lyy * ir;
      }
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        double bf[4];
        to_frame_2d(q[k], U0, V0, bf);
#pragma unroll
        for (int v = 0; v < 4; ++v) b[k][v] = (TC)bf[v];
      }
    }
    // the divisors of the five derivatives (uniform over a launch)
    const Divisor qdiv[5] = {divisor(4.0 * hn), divisor(4.0 * hs), divisor(8.0 * hn * hn), divisor(2.0 * hn * hs),
                             divisor(2.0 * hs * hs)};
#pragma unroll
    for (int k = 0; k < (kCurv ? 0 : 5); ++k) {
      double qd[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double L0 = Ueq[0][0][v], L1 = Ueq[0][1][v], L2 = Ueq[0][2][v];
        const double R0 = Ueq[1][0][v], R1 = Ueq[1][1][v], R2 = Ueq[1][2][v];
        const double num = k == 0   ? (R2 - L2) + 2.0 * (R1 - L1) + (R0 - L0)                    // U_x
                           : k == 1 ? R2 - R0 + L2 - L0                                            // U_y
                           : k == 2 ? 26.0 * (R1 + L1) - (R2 + L2 + R0 + L0) - 48.0 * W0[v]      // U_xx
                           : k == 3 ? R2 - L2 - R0 + L0                                            // U_xy
                                    : R2 - 2.0 * R1 + R0 + L2 - 2.0 * L1 + L0;                   // U_yy
        qd[v] = div_by(num, qdiv[k]) * ir;
      }
      double bf[4];
      to_frame_2d(qd, U0, V0, bf);
#pragma unroll
      for (int v = 0; v < 4; ++v) b[k][v] = (TC)bf[v];
    }
    if constexpr (g0_solved_in_prologue<TC>()) {
      TC th[5], kp[4];
      theta_powers(0.5 / lam0, th);
#pragma unroll
      for (int e = 0; e < 4; ++e) kp[e] = (TC)P.kp[e];
      Coefs<TC> c;
      coef_g0_2d<TC>(th, kp, (TC)P.nth, (TC)U0, (TC)V0, b[0], b[1], b[2], b[3], b[4], c.ax, c.ay, c.At, c.dxx,
                     c.dxy, c.dyy, c.bxt, c.byt, c.Bt);
      const TC* sets[9] = {c.ax, c.ay, c.At, c.dxx, c.dxy, c.dyy, c.bxt, c.byt, c.Bt};
#pragma unroll
      for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int v = 0; v < 4; ++v) R.T(T_CG + 4 * k + v, f) = sets[k][v];
    } else {
#pragma unroll
      for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int v = 0; v < 4; ++v) R.T(T_CG + 4 * k + v, f) = b[k][v];
    }
  }
  // collision time (Sec. 4)
  const double jump = fabs((S[0].pr - S[1].pr) / (S[0].pr + S[1].pr));
  const double tau = P.viscous ? P.mu / p0 + P.tau_c * jump * dt : (P.tau_eps + P.tau_c * jump) * dt;
  R.D(D_TAU, f) = tau;
  // leading terms: Euler flux of U0 (C1 g0) and free transport of the sides
  // (C7 g_k); only the two time integrals of the leading terms are needed here
  const double E = decay(tau, dt);
  R.D(D_DECAY, f) = E;
  const double I7 = tau * (1.0 - E), I1 = dt - I7;
  const double FE[4] = {W0[1], W0[1] * U0 + p0, W0[1] * V0, U0 * (W0[3] + p0)};
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    flux[v] = hs * (I1 * FE[v] + I7 * Fk[v]);
    pv[v] = W0[v];  // C1 + C7 = 1
    if (P.viscous) R.D(D_E0 + v, f) = hs * dt * W0[v];
  }
  return true;
}

// Hydrodynamic phase of interface f: corrections to flux, point values and
// the integrated density (lab frame, interface frame components).
template <typename TC>
__device__ __forceinline__ void iface_hydro_2d(const Phys& P, double dt, double hs, const Rec<TC>& R, unsigned f,
                                               double (&flux)[4], double (&pvm)[4], double (&pvp)[4],
                                               double (&E)[4]) {
  const double rho0 = R.D(D_RHO0, f), U0 = R.D(D_U0, f), V0 = R.D(D_V0, f), lam0 = R.D(D_LAM0, f);
  TC th[5], kp[4];
  theta_powers(0.5 / lam0, th);
#pragma unroll
  for (int e = 0; e < 4; ++e) kp[e] = (TC)P.kp[e];
  const TC u0 = (TC)U0, v0 = (TC)V0;
  Coefs<TC> c;
  if constexpr (g0_solved_in_prologue<TC>()) {
    TC* sets[9] = {c.ax, c.ay, c.At, c.dxx, c.dxy, c.dyy, c.bxt, c.byt, c.Bt};
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
      for (int v = 0; v < 4; ++v) sets[k][v] = R.T(T_CG + 4 * k + v, f);
  } else {
    TC b[5][4];
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
      for (int v = 0; v < 4; ++v) b[k][v] = R.T(T_CG + 4 * k + v, f);
    coef_g0_2d<TC>(th, kp, (TC)P.nth, u0, v0, b[0], b[1], b[2], b[3], b[4], c.ax, c.ay, c.At, c.dxx, c.dxy, c.dyy,
                   c.bxt, c.byt, c.Bt);
  }
  TC w[13];
  {
    TimeWeights tw;
    time_weights(R.D(D_TAU, f), dt, R.D(D_DECAY, f), tw);
    double hw[13];
    hydro_weights(tw, hs, hw);
#pragma unroll
    for (int k = 0; k < 13; ++k) w[k] = (TC)hw[k];
  }
  Acc<TC> A(kGaussOffset * hs);
  TC m0[4], m1[4];
  // C2 g0 (a1 u + a2 v)
  mom_full_conv_2d<TC>(th, kp, u0, v0, c.ax, c.ay, m0, m1);
  A.flux(m0, m1, w[HW_I2]);
  A.pv0(m0, w[HW_C2]);
  // C3 g0 A
  mom_full_A_2d<TC>(th, kp, u0, v0, c.At, m0, m1);
  A.flux(m0, m1, w[HW_I3]);
  A.pv0(m0, w[HW_C3]);
  // 1/2 C4 g0 [(a1^2 + d11) u^2 + 2 (a1 a2 + d12) u v + (a2^2 + d22) v^2]
  mom_full_quad_2d<TC>(th, kp, u0, v0, c.ax, c.ay, c.dxx, c.dxy, c.dyy, m0, m1);
  A.flux(m0, m1, w[HW_I4H]);
  A.pv0(m0, w[HW_C4H]);
  // 1/2 C5 g0 (A^2 + B)
  mom_full_ttt_2d<TC>(th, kp, u0, v0, c.At, c.Bt, m0, m1);
  A.flux(m0, m1, w[HW_I5H]);
  A.pv0(m0, w[HW_C5H]);
  // C6 g0 [(A a1 + b1) u + (A a2 + b2) v]
  mom_full_tlin_2d<TC>(th, kp, u0, v0, c.ax, c.ay, c.At, c.bxt, c.byt, m0, m1);
  A.flux(m0, m1, w[HW_I6]);
  A.pv0(m0, w[HW_C6]);
  // 1/2 C1 g0 (a2^2 + d22) y^2: int y^2 dy over the interface = ds^3/12
  mom_full_dyy_2d<TC>(th, kp, u0, v0, c.ay, c.dyy, m0, m1);
  A.flux(m0, m1, w[HW_I1Y]);
  A.pv2(m0, w[HW_C1H]);
  // terms linear in y vanish in the flux; point values:
  // C1 g0 a2 y + C2 g0 [(a2^2 + d22) v + (a1 a2 + d12) u] y + C3 g0 (A a2 + b2) y
  mom_full_ay_2d<TC>(th, kp, u0, v0, c.ay, m0);
  A.pv1(m0, w[HW_C1]);
  mom_full_inner_2d<TC>(th, kp, u0, v0, c.ax, c.ay, c.dxy, c.dyy, m0);
  A.pv1(m0, w[HW_C2]);
  mom_full_ty_2d<TC>(th, kp, u0, v0, c.ay, c.At, c.byt, m0);
  A.pv1(m0, w[HW_C3]);
#pragma unroll
  for (int v = 0; v < 4; ++v) flux[v] = pvm[v] = pvp[v] = E[v] = 0.0;
  A.add_to(U0, V0, rho0, hs, flux, pvm, pvp, P.viscous ? E : nullptr);
}

// Kinetic phase of interface f, side s (0: g_l on u > 0, 1: g_r on u < 0);
// Wc, pc: average and reconstruction of the side's cell in the interface frame.
template <typename TC>
__device__ __forceinline__ void iface_kinetic_2d(const Phys& P, double dt, double hn, double hs, int s,
                                                 const double (&Wc)[4], const double (&pc)[4][5], const Rec<TC>& R,
                                                 unsigned f, double (&flux)[4], double (&pvm)[4], double (&pvp)[4],
                                                 double (&E)[4]) {
  Side S;
  if constexpr (sides_in_record<TC>()) {
    S.rho = R.D(D_SIDE + 5 * s + 0, f);
    S.U = R.D(D_SIDE + 5 * s + 1, f);
    S.V = R.D(D_SIDE + 5 * s + 2, f);
    S.pr = R.D(D_SIDE + 5 * s + 3, f);
    S.lam = R.D(D_SIDE + 5 * s + 4, f);
  } else {
    side_state_2d(P, s, hn, hs, Wc, pc, S);  // physical: the prologue checked it
  }
  const double rho = S.rho, U = S.U, V = S.V, lam = S.lam;
  const Half hm = half_moments_from(R.D(D_HM0 + 2 * s, f), R.D(D_HH1 + 2 * s, f), U, lam);  // the prologue's
  TC th[5], kp[4], h[10];
  theta_powers(0.5 / lam, th);
  half_table(hm, U, lam, h);
#pragma unroll
  for (int e = 0; e < 4; ++e) kp[e] = (TC)P.kp[e];
  const TC us = (TC)U, vs = (TC)V;
  Coefs<TC> c;
  {
    TC b[5][4];
    if constexpr (sides_in_record<TC>()) {
#pragma unroll
      for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int v = 0; v < 4; ++v) b[k][v] = R.T(T_SB + 20 * s + 4 * k + v, f);
    } else {
      side_targets_2d(s, hn, S, pc, b);
    }
    // the side's rate for the Knudsen reading from its first derivatives
    if (P.viscous) {
      const double cs = sqrt(P.gamma * S.pr / S.rho);
      R.D(D_RATE0 + s, f) = rate_term(cs, (double)b[0][0], (double)b[0][1], (double)b[0][2], (double)b[0][3]) +
                            rate_term(cs, (double)b[1][0], (double)b[1][1], (double)b[1][2], (double)b[1][3]);
    }
    if (P.viscous)
      coef_side_ns_2d<TC>(th, kp, (TC)P.nth, us, vs, b[0], b[1], b[2], b[3], b[4], c.ax, c.ay, c.At, c.dxx, c.dxy,
                          c.dyy, c.bxt, c.byt, c.Bt);
    else
      coef_side_euler_2d<TC>(th, kp, (TC)P.nth, us, vs, b[0], b[1], b[2], b[3], b[4], c.ax, c.ay, c.At, c.dxx,
                             c.dxy, c.dyy, c.bxt, c.byt, c.Bt);
  }
  TC w[12];
  {
    const double tau = R.D(D_TAU, f);
    TimeWeights tw;
    time_weights(tau, dt, R.D(D_DECAY, f), tw);
    // collision time of the Chapman-Enskog correction
    const double tb = P.viscous ? bracket_tau(tau, R.D(D_RATE0 + s, f)) : tau;
    double kw[12];
    kinetic_weights(tw, tb, P.viscous ? tb : 0.0, hs, kw);  // Euler: f_G = g_k
#pragma unroll
    for (int k = 0; k < 12; ++k) w[k] = (TC)kw[k];
  }
  Acc<TC> A(kGaussOffset * hs);
  TC m0[4], m1[4];
  // C8 g (a1 u + a2 v)  [and -tau C7 g (a1 u + a2 v)]
  mom_half_conv_2d<TC>(th, kp, h, us, vs, c.ax, c.ay, m0, m1);
  A.flux(m0, m1, w[KW_ICONV]);
  A.pv0(m0, w[KW_CCONV]);
  // 1/2 C7 t^2 g [(a1^2+d11) u^2 + 2 (a1 a2+d12) u v + (a2^2+d22) v^2]  [and -tau C8 g (same)]
  mom_half_quad_2d<TC>(th, kp, h, us, vs, c.ax, c.ay, c.dxx, c.dxy, c.dyy, m0, m1);
  A.flux(m0, m1, w[KW_IQUAD]);
  A.pv0(m0, w[KW_CQUAD]);
  // 1/2 C7 g (a2^2 + d22) y^2
  mom_half_dyy_2d<TC>(th, kp, h, us, vs, c.ay, c.dyy, m0, m1);
  A.flux(m0, m1, w[KW_IY]);
  A.pv2(m0, w[KW_C7H]);
  // point values, linear in y: C7 g a2 y - C7 t g [(a1 a2+d12) u + (a2^2+d22) v] y
  //   [and -tau C7 g ((a1 a2+d12) u + (a2^2+d22) v + A a2 + b2) y]
  mom_half_ay_2d<TC>(th, kp, h, us, vs, c.ay, m0);
  A.pv1(m0, w[KW_C7]);
  mom_half_inner_2d<TC>(th, kp, h, us, vs, c.ax, c.ay, c.dxy, c.dyy, m0);
  A.pv1(m0, w[KW_CINNER]);
  if (P.viscous) {
    // -tau C7 g A, -tau C8 g [(A a1 + b1) u + (A a2 + b2) v], -tau C7 g (A a2 + b2) y
    mom_half_A_2d<TC>(th, kp, h, us, vs, c.At, m0, m1);
    A.flux(m0, m1, w[KW_AI]);
    A.pv0(m0, w[KW_AC]);
    mom_half_tlin_2d<TC>(th, kp, h, us, vs, c.ax, c.ay, c.At, c.bxt, c.byt, m0, m1);
    A.flux(m0, m1, w[KW_TI]);
    A.pv0(m0, w[KW_TC]);
    mom_half_ty_2d<TC>(th, kp, h, us, vs, c.ay, c.At, c.byt, m0);
    A.pv1(m0, w[KW_AC]);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) flux[v] = pvm[v] = pvp[v] = E[v] = 0.0;
  A.add_to(U, V, rho, hs, flux, pvm, pvp, P.viscous ? E : nullptr);
}

// ---------------------------------------------------------------------------
// compact reconstruction of one scalar (Sec. 3.1 / 3.2)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double mm2(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return fabs(a) < fabs(b) ? a : b;
}

// the divisors of the 2D reconstruction of a cell of size h x k
struct ReconDiv {
  Divisor h, k, hh, kk, hk, h2, k2, hk2, six;
  __device__ __forceinline__ explicit ReconDiv(double h_, double k_)
      : h(divisor(h_)), k(divisor(k_)), hh(divisor(h_ * h_)), kk(divisor(k_ * k_)), hk(divisor(h_ * k_)),
        h2(divisor(2.0 * h_)), k2(divisor(2.0 * k_)), hk2(divisor(2.0 * (h_ * k_))), six(divisor(6.0)) {}
};

// 2D reconstruction (Sec. 3.2).  Stencil values of one component: c = cell
// average; e, w, n, s = face-neighbour averages; E+-, W+-, N+-, S+- =
// Gauss-point values on the four interfaces.  The quantities that decide
// branches (the one-sided estimates, the minmod arguments and the
// cross-derivative candidates) are formed in the order of their printed
// formulas and without FMA contraction, so that a tie or a sign is decided
// from the same rounded values as in a plain evaluation (every quotient is the
// correctly rounded one, see div_by).

// eq. over-sys and the limiter along one direction: the normal pair (first,
// second derivative) of the one-sided stencils on the positive side (up, the
// neighbour average; Pp, Pm, the Gauss-point values of the interface between)
// and on the negative side (um; Mp, Mm), limited.  hd = cell size along the
// direction.
__device__ __forceinline__ void recon_pair(double c, double up, double um, double Pp, double Pm, double Mp, double Mm,
                                           double hd, const Divisor& Dh, const Divisor& Dhh, const Divisor& six,
                                           double& d1, double& d2) {
#pragma clang fp contract(off)
  const double cP = div_by(3.0 * ((c + up) - (Pp + Pm)), Dhh), sP = div_by(Pp + Pm - 2.0 * c, Dh);
  const double cM = div_by(3.0 * ((c + um) - (Mp + Mm)), Dhh), sM = div_by(Mp + Mm - 2.0 * c, Dh);
  d2 = mm2(cM, cP);
  d1 = mm2(-sM + div_by(d2 * hd, six), sP - div_by(d2 * hd, six));
}

// the rest of Sec. 3.2 once the pairs a2, a4 (x) and a3, a5 (y) are limited:
// the cross term, the central stencil and the nonlinear weights.  p = p2..p6.
__device__ __forceinline__ void recon_finish(double c, double e, double w, double n, double s, double Ep, double Em,
                                             double Wp, double Wm, double Np, double Nm, double Sp, double Sm,
                                             double h, double k, double eps, double Cw, const ReconDiv& D, double a2,
                                             double a3, double a4, double a5, double tie_rel, double* p) {
#pragma clang fp contract(off)
  // cross term of the stencils NE, NW, SW, SE with the limited slopes; the one
  // of smallest magnitude.  A relative perturbation d of the Gauss values and
  // slopes moves every candidate by at most d M, M = sqrt(3) sum|G| / (h k) +
  // |a2| / k + |a3| / h: candidates within tie_rel M of the smallest
  // magnitude (tie_rel: the relative rounding noise of the stored point
  // values) are tied, and a tie of both signs gives zero (so that mirrored
  // data give the mirrored term)
  const double s3 = 1.7320508075688772;  // sqrt(3)
  const double dE = Ep - Em, dW = Wp - Wm, dN = Np - Nm, dS = Sp - Sm;
  const double ak = div_by(a2, D.k), ah = div_by(a3, D.h);
  const double cand[4] = {div_by(s3 * (dE + dN), D.hk) - (ak + ah), div_by(s3 * (dN - dW), D.hk) - (ak - ah),
                          div_by(-s3 * (dS + dW), D.hk) + (ak + ah), div_by(s3 * (dE - dS), D.hk) + (ak - ah)};
  double a6 = cand[0], m6 = fabs(cand[0]);
#pragma unroll
  for (int q = 1; q < 4; ++q)
    if (fabs(cand[q]) < m6) {
      m6 = fabs(cand[q]);
      a6 = cand[q];
    }
  const double sumG = fabs(Ep) + fabs(Em) + fabs(Wp) + fabs(Wm) + fabs(Np) + fabs(Nm) + fabs(Sp) + fabs(Sm);
  const double band = m6 + tie_rel * (div_by(s3 * sumG, D.hk) + fabs(ak) + fabs(ah));
  int pos = 0, neg = 0;  // bitwise logic: no branches
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int near = fabs(cand[q]) <= band;
    pos |= near & (cand[q] > 0.0);
    neg |= near & (cand[q] < 0.0);
  }
  a6 = (pos & neg) ? 0.0 : a6;
  // central stencil
  const double c2 = div_by(e - w, D.h2), c4 = div_by((e + w) - 2.0 * c, D.hh);
  const double c3 = div_by(n - s, D.k2), c5 = div_by((n + s) - 2.0 * c, D.kk);
  const double c6 = div_by(s3 * ((dE - dW) + (dN - dS)), D.hk2);
  // nonlinear weights, I(U1) = C |cell|, I(U2) from the derivatives of U2
  const double hk = h * k;
  const double A = hk;
  const double I1 = Cw * A;
  const double I2 = A * (c2 * c2 + c3 * c3) + A * (c4 * c4 * (h * h / 12.0 + A) + c5 * c5 * (k * k / 12.0 + A) +
                                                  c6 * c6 * ((h * h + k * k) / 12.0 + A));
  const double b1 = 1.0 / ((eps + I1) * (eps + I1)), b2 = 1.0 / ((eps + I2) * (eps + I2));
  const Divisor sb = divisor(b1 + b2);
  const double w1 = div_by(b1, sb), w2 = div_by(b2, sb);
  p[0] = w1 * a2 + w2 * c2;
  p[1] = w1 * a3 + w2 * c3;
  p[2] = w1 * a4 + w2 * c4;
  p[3] = w1 * a5 + w2 * c5;
  p[4] = w1 * a6 + w2 * c6;
}

// one component in conservative variables
__device__ __forceinline__ void recon_2d(double c, double e, double w, double n, double s, double Ep, double Em,
                                         double Wp, double Wm, double Np, double Nm, double Sp, double Sm, double h,
                                         double k, double eps, double Cw, const ReconDiv& D, double tie_rel,
                                         double* p) {
  double a2, a3, a4, a5;
  recon_pair(c, e, w, Ep, Em, Wp, Wm, h, D.h, D.hh, D.six, a2, a4);
  recon_pair(c, n, s, Np, Nm, Sp, Sm, k, D.k, D.kk, D.six, a3, a5);
  recon_finish(c, e, w, n, s, Ep, Em, Wp, Wm, Np, Nm, Sp, Sm, h, k, eps, Cw, D, a2, a3, a4, a5, tie_rel, p);
}

// Eigenvectors of the 2D Euler flux Jacobian along x (kX) or y at the
// conservative state W: columns of R for the waves un - c, un (entropy),
// un (shear), un + c; L = R^-1 in closed form (b1 = (gamma - 1) / c^2,
// b2 = b1 q, q = |u|^2 / 2).  False for a nonphysical state.
template <bool kX>
__device__ __forceinline__ bool euler_eigen_2d(double gamma, const double* W, double (&R)[4][4],
                                               double (&L)[4][4]) {
  const double rho = W[0];
  if (!(rho > 0.0)) return false;
  const double u = W[1] / rho, v = W[2] / rho, q = 0.5 * (u * u + v * v);
  const double p = (gamma - 1.0) * (W[3] - rho * q);
  if (!(p > 0.0)) return false;
  const double c = sqrt(gamma * p / rho), H = (W[3] + p) / rho, ic = 1.0 / c;
  const double un = kX ? u : v, ut = kX ? v : u;  // normal and tangential velocity
  const int in = kX ? 1 : 2, it = kX ? 2 : 1;      // their momentum components
  const double b1 = (gamma - 1.0) / (c * c), b2 = b1 * q;
  // R: columns (1, u - c n, H - un c), (1, u, q), (0, tangential unit vector,
  // ut), (1, u + c n, H + un c); rows 0 (density), in / it (normal and
  // tangential momentum), 3 (energy)
  const double rcol[4][4] = {{1.0, un - c, ut, H - un * c},
                             {1.0, un, ut, q},
                             {0.0, 0.0, 1.0, ut},
                             {1.0, un + c, ut, H + un * c}};  // (rho, normal, tangential, energy)
  // L rows in the same order of components: 0.5 (b2 + un/c, -b1 un - 1/c,
  // -b1 ut, b1); (1 - b2, b1 un, b1 ut, -b1); (-ut, 0, 1, 0);
  // 0.5 (b2 - un/c, -b1 un + 1/c, -b1 ut, b1)
  const double lrow[4][4] = {{0.5 * (b2 + un * ic), -0.5 * (b1 * un + ic), -0.5 * (b1 * ut), 0.5 * b1},
                             {1.0 - b2, b1 * un, b1 * ut, -b1},
                             {-ut, 0.0, 1.0, 0.0},
                             {0.5 * (b2 - un * ic), -0.5 * (b1 * un - ic), -0.5 * (b1 * ut), 0.5 * b1}};
  const int comp[4] = {0, in, it, 3};  // frame component -> conservative component
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      R[comp[f]][r] = rcol[r][f];
      L[r][comp[f]] = lrow[r][f];
    }
  return true;
}

// The limited pair of one direction in the characteristic variables of that
// direction at the cell average S[0] (the remark on characteristic variables
// in Sec. 4, carried to 2D direction by direction): the direction's stencil
// data are multiplied by L, each field's pair is limited as a scalar, and the
// limited pairs are multiplied back by R.  S[13][4] in the order c, e, w, n,
// s, E+, E-, W+, W-, N+, N-, S+, S-.  a[v] = (a2, a3, a4, a5) of component v;
// this direction's two entries are written.  False for a nonphysical average.
template <bool kX>
__device__ __forceinline__ bool recon_pair_characteristic(double gamma, const double (&S)[13][4], double hd,
                                                          const Divisor& Dh, const Divisor& Dhh, const Divisor& six,
                                                          double (&a)[4][4]) {
#pragma clang fp contract(off)
  double R[4][4], L[4][4];
  if (!euler_eigen_2d<kX>(gamma, S[0], R, L)) return false;
  constexpr int e0 = 0, e1 = kX ? 1 : 3, e2 = kX ? 2 : 4, e3 = kX ? 5 : 9;  // c, up, um, first Gauss value
  const int ent[7] = {e0, e1, e2, e3, e3 + 1, e3 + 2, e3 + 3};
  double ch[7][4];
#pragma unroll
  for (int e = 0; e < 7; ++e)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc += L[r][v] * S[ent[e]][v];
      ch[e][r] = acc;
    }
  double d1[4], d2[4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
    recon_pair(ch[0][r], ch[1][r], ch[2][r], ch[3][r], ch[4][r], ch[5][r], ch[6][r], hd, Dh, Dhh, six, d1[r], d2[r]);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      s1 += R[v][r] * d1[r];
      s2 += R[v][r] * d2[r];
    }
    a[v][kX ? 0 : 1] = s1;
    a[v][kX ? 2 : 3] = s2;
  }
  return true;
}

// Admissibility of a reconstructed cell polynomial (a robustness reading; the
// paper leaves robust reconstruction open at the end of Sec. 3.3): at the
// centre of every interface of the cell, density and pressure must be
// positive (mode 0: the interface Maxwellians exist), and in mode 1 also lie
// within a factor two of the range of the averages of the cell and its face
// neighbours,
//   rho_min / 2 <= rho <= 2 rho_max,  p_min / 2 <= p <= 2 p_max;
// otherwise the cell is reconstructed as its constant average for this step.
struct Range {
  double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};  // rho, p
  __device__ __forceinline__ void add(double rho, double p) {
    lo[0] = fmin(lo[0], rho);
    hi[0] = fmax(hi[0], rho);
    lo[1] = fmin(lo[1], p);
    hi[1] = fmax(hi[1], p);
  }
  __device__ __forceinline__ bool admits(double rho, double p, int mode) const {
    return rho > 0.0 && p > 0.0 &&
           (mode == 0 || (!(rho < 0.5 * lo[0]) && !(rho > 2.0 * hi[0]) && !(p < 0.5 * lo[1]) && !(p > 2.0 * hi[1])));
  }
};

__device__ __forceinline__ double pressure_2d(double gamma, const double* W) {
  return (gamma - 1.0) * (W[3] - 0.5 * (W[1] * W[1] + W[2] * W[2]) / W[0]);
}
__device__ __forceinline__ double pressure_1d(double gamma, const double* W) {
  return (gamma - 1.0) * (W[2] - 0.5 * (W[1] * W[1]) / W[0]);
}

// the cell polynomial Wc + p2 x + p3 y + p4 w_x + p5 w_y + p6 x y (per
// conservative variable) at the centres of the four interfaces of the cell
__device__ __forceinline__ bool recon_admissible_2d(const double (&Wc)[4], const double (&p)[4][5], double h,
                                                    double k, double gamma, const Range& R, int mode) {
  bool ok = true;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const double x = f == 0 ? 0.5 * h : f == 1 ? -0.5 * h : 0.0;
    const double y = f == 2 ? 0.5 * k : f == 3 ? -0.5 * k : 0.0;
    double W[4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
      W[v] = Wc[v] + p[v][0] * x + p[v][1] * y + p[v][2] * 0.5 * (x * x - h * h / 12.0) +
             p[v][3] * 0.5 * (y * y - k * k / 12.0) + p[v][4] * x * y;
    ok = ok && R.admits(W[0], pressure_2d(gamma, W), mode);
  }
  return ok;
}

// 1D: the polynomial Wc + p2 x + p4 (x^2/2 - h^2/24) at x = -h/2, +h/2
__device__ __forceinline__ bool recon_admissible_1d(const double (&Wc)[3], const double (&p)[3][2], double h,
                                                    double gamma, const Range& R, int mode) {
  bool ok = true;
#pragma unroll
  for (int sd = 0; sd < 2; ++sd) {
    const double x = sd == 0 ? -0.5 * h : 0.5 * h;
    double W[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) W[v] = Wc[v] + p[v][0] * x + p[v][1] * 0.5 * (x * x - h * h / 12.0);
    ok = ok && R.admits(W[0], pressure_1d(gamma, W), mode);
  }
  return ok;
}

// ---------------------------------------------------------------------------
// 1D (Sec. 3.1): compact reconstruction of one scalar and the fused
// interface evaluation
// ---------------------------------------------------------------------------

// c = cell average, e, w = neighbour averages, Fp, Fm = point values at the
// right and left interfaces.  p = (p2, p4): U = c + p2 x + p4 (x^2/2 - h^2/24).
// Branch-deciding quantities in the order of the printed formulas, no FMA.
__device__ __forceinline__ void recon_1d(double c, double e, double w, double Fp, double Fm, double h, double eps,
                                         double Cw, double* p) {
#pragma clang fp contract(off)
  // one-sided stencils {U_{i-1}, U_{i-1/2}, U_i} and {U_i, U_{i+1/2}, U_{i+1}}
  const double a3W = 3.0 * (c + w - 2.0 * Fm) / (h * h), a3E = 3.0 * (c + e - 2.0 * Fp) / (h * h);
  const double s2W = 2.0 * (Fm - c) / h, s2E = 2.0 * (Fp - c) / h;
  // eq. limiter
  const double a3 = mm2(a3W, a3E);
  const double a2 = mm2(-s2W + a3 * h / 6.0, s2E - a3 * h / 6.0);
  // central stencil: averages of U2 over the three cells
  const double c2 = (e - w) / (2.0 * h), c4 = ((e + w) - 2.0 * c) / (h * h);
  // weights: I(U1) = C h^2, I(U2) = h^2 c2^2 + 13/12 h^4 c4^2
  const double I1 = Cw * h * h;
  const double I2 = h * h * c2 * c2 + 13.0 / 12.0 * h * h * h * h * c4 * c4;
  const double b1 = 1.0 / ((eps + I1) * (eps + I1)), b2 = 1.0 / ((eps + I2) * (eps + I2));
  const double w1 = b1 / (b1 + b2), w2 = b2 / (b1 + b2);
  p[0] = w1 * a2 + w2 * c2;
  p[1] = w1 * a3 + w2 * c4;
}

// Eigenvectors of the 1D Euler flux Jacobian at the state W (columns of R:
// waves u - c, u, u + c) and the rows of L = R^-1 in closed form.  False for a
// nonphysical state.
__device__ __forceinline__ bool euler_eigen_1d(double gamma, const double* W, double (&R)[3][3], double (&L)[3][3]) {
  const double rho = W[0], u = W[1] / rho, p = (gamma - 1.0) * (W[2] - 0.5 * rho * u * u);
  if (!(rho > 0.0) || !(p > 0.0)) return false;
  const double c = sqrt(gamma * p / rho), H = (W[2] + p) / rho;
  R[0][0] = 1.0;
  R[0][1] = 1.0;
  R[0][2] = 1.0;
  R[1][0] = u - c;
  R[1][1] = u;
  R[1][2] = u + c;
  R[2][0] = H - u * c;
  R[2][1] = 0.5 * u * u;
  R[2][2] = H + u * c;
  const double b1 = (gamma - 1.0) / (c * c), b2 = 0.5 * u * u * b1, ic = 1.0 / c;
  L[0][0] = 0.5 * (b2 + u * ic);
  L[0][1] = -0.5 * (b1 * u + ic);
  L[0][2] = 0.5 * b1;
  L[1][0] = 1.0 - b2;
  L[1][1] = b1 * u;
  L[1][2] = -b1;
  L[2][0] = 0.5 * (b2 - u * ic);
  L[2][1] = -0.5 * (b1 * u - ic);
  L[2][2] = 0.5 * b1;
  return true;
}

// moment target of a derivative vector d for the Maxwellian of density
// 1/ir moving with U, in its frame (1D)
template <typename T>
__device__ __forceinline__ void frame_rhs_1d(const double* d, double ir, double U, T* o) {
  double b[3], f[3];
#pragma unroll
  for (int v = 0; v < 3; ++v) b[v] = d[v] * ir;
  to_frame_1d(b, U, f);
#pragma unroll
  for (int v = 0; v < 3; ++v) o[v] = (T)f[v];
}

// One 1D interface.  Wc[s][v], pc[s][v] = (p2, p4): averages and
// reconstruction of the left (s = 0) and right (s = 1) cells; h = dx.
// Returns the time-integrated flux (eq. finite) and the interface value at
// t + dt (eq. point); false if an interface state is nonphysical.  Leading
// terms, U0, the equilibrium slopes, tau and the time integrals in double;
// coefficients and correction moments in TC.
template <typename TC>
__device__ __forceinline__ bool iface_1d(const Phys& P, double dt, double h, const double (&Wc)[2][3],
                                         const double (&pc)[2][3][2], double (&flux)[3], double (&pv)[3]) {
  const double g1 = P.gamma - 1.0;
  double W[2][3], Dn[2][3], Dnn[2][3], rho[2], U[2], pr[2], lam[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const double xn = s == 0 ? 0.5 * h : -0.5 * h;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      W[s][v] = Wc[s][v] + pc[s][v][0] * xn + pc[s][v][1] * (h * h * (1.0 / 12.0));
      Dn[s][v] = pc[s][v][0] + pc[s][v][1] * xn;
      Dnn[s][v] = pc[s][v][1];
    }
    rho[s] = W[s][0];
    U[s] = W[s][1] / rho[s];
    pr[s] = g1 * (W[s][2] - 0.5 * rho[s] * U[s] * U[s]);
    lam[s] = 0.5 * rho[s] / pr[s];
  }
  if (!(rho[0] > 0.0) || !(rho[1] > 0.0) || !(pr[0] > 0.0) || !(pr[1] > 0.0)) return false;
  Half hm[2];
  double W0[3] = {0, 0, 0}, Fk[3] = {0, 0, 0};
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    hm[s] = half_moments(U[s], lam[s], s == 0 ? 1.0 : -1.0);
    const double e2 = P.K * (0.5 / lam[s]);  // <xi^2>
    W0[0] += rho[s] * hm[s].M0;
    W0[1] += rho[s] * hm[s].M1;
    W0[2] += rho[s] * 0.5 * (hm[s].M2 + e2 * hm[s].M0);
    Fk[0] += rho[s] * hm[s].M1;
    Fk[1] += rho[s] * hm[s].M2;
    Fk[2] += rho[s] * 0.5 * (hm[s].M3 + e2 * hm[s].M1);
  }
  const double rho0 = W0[0], U0 = W0[1] / rho0;
  const double p0 = g1 * (W0[2] - 0.5 * rho0 * U0 * U0);
  if (!(p0 > 0.0)) return false;
  const double lam0 = 0.5 * rho0 / p0;
  // equilibrium slopes of the two cells sharing the interface (Sec. 3.3 in 1D)
  double q2[3], q4[3];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    q2[v] = (Wc[1][v] - Wc[0][v]) / h;
    q4[v] = 3.0 * (Wc[0][v] + Wc[1][v] - 2.0 * W0[v]) / (h * h);
  }
  const double jump = fabs((pr[0] - pr[1]) / (pr[0] + pr[1]));
  const double tau = P.viscous ? P.mu / p0 + P.tau_c * jump * dt : (P.tau_eps + P.tau_c * jump) * dt;
  TimeWeights w;
  time_weights(tau, dt, decay(tau, dt), w);
  const double tv = P.viscous ? tau : 0.0;
  TC kp[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) kp[e] = (TC)P.kp[e];
  const TC zero[3] = {0, 0, 0};
  double E[3];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    flux[v] = w.I[1] * (v == 0 ? W0[1] : v == 1 ? W0[1] * U0 + p0 : U0 * (W0[2] + p0)) + w.I[7] * Fk[v];
    pv[v] = W0[v];
    E[v] = dt * W0[v];
  }
  // accumulate the correction moments of one Maxwellian (peculiar frame) in
  // the lab frame
  auto add = [&](const TC* AF, const TC* BF, const TC* V0, double Us, double rs) {
    TC fl[3];
    const TC us = (TC)Us;
#pragma unroll
    for (int v = 0; v < 3; ++v) fl[v] = BF[v] + us * AF[v];
    double a[3];
    from_frame_1d(fl, Us, a);
#pragma unroll
    for (int v = 0; v < 3; ++v) flux[v] += rs * a[v];
    from_frame_1d(V0, Us, a);
#pragma unroll
    for (int v = 0; v < 3; ++v) pv[v] += rs * a[v];
    from_frame_1d(AF, Us, a);
#pragma unroll
    for (int v = 0; v < 3; ++v) E[v] += rs * a[v];
  };
  // hydrodynamic part (eq. dis1, g0 over the whole space)
  {
    TC th[5];
    theta_powers(0.5 / lam0, th);
    TC bx[3], bxx[3];
    frame_rhs_1d(q2, 1.0 / rho0, U0, bx);
    frame_rhs_1d(q4, 1.0 / rho0, U0, bxx);
    TC ax[3], ay[3] = {0, 0, 0}, At[3], dxx[3], dxy[3] = {0, 0, 0}, dyy[3] = {0, 0, 0}, bxt[3], byt[3] = {0, 0, 0},
                                                                                           Bt[3];
    const TC u0 = (TC)U0;
    coef_g0_1d<TC>(th, kp, (TC)P.nth, u0, TC(0), bx, zero, bxx, zero, zero, ax, ay, At, dxx, dxy, dyy, bxt, byt, Bt);
    TC AF[3] = {0, 0, 0}, BF[3] = {0, 0, 0}, V0[3] = {0, 0, 0}, m0[3], m1[3];
    auto acc = [&](TC wi, TC wc) {
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        AF[v] += wi * m0[v];
        BF[v] += wi * m1[v];
        V0[v] += wc * m0[v];
      }
    };
    mom_full_conv_1d<TC>(th, kp, u0, TC(0), ax, ay, m0, m1);  // C2 g0 a1 u
    acc((TC)w.I[2], (TC)w.C[2]);
    mom_full_A_1d<TC>(th, kp, u0, TC(0), At, m0, m1);  // C3 g0 A
    acc((TC)w.I[3], (TC)w.C[3]);
    mom_full_quad_1d<TC>(th, kp, u0, TC(0), ax, ay, dxx, dxy, dyy, m0, m1);  // 1/2 C4 g0 (a1^2 + d11) u^2
    acc((TC)(0.5 * w.I[4]), (TC)(0.5 * w.C[4]));
    mom_full_ttt_1d<TC>(th, kp, u0, TC(0), At, Bt, m0, m1);  // 1/2 C5 g0 (A^2 + B)
    acc((TC)(0.5 * w.I[5]), (TC)(0.5 * w.C[5]));
    mom_full_tlin_1d<TC>(th, kp, u0, TC(0), ax, ay, At, bxt, byt, m0, m1);  // C6 g0 (A a1 + b1) u
    acc((TC)w.I[6], (TC)w.C[6]);
    add(AF, BF, V0, U0, rho0);
  }
  // kinetic part (eq. dis2) of each side over its half space
#pragma unroll 1
  for (int s = 0; s < 2; ++s) {
    TC th[5], ht[10];
    theta_powers(0.5 / lam[s], th);
    half_table(hm[s], U[s], lam[s], ht);
    TC bx[3], bxx[3];
    const double ir = 1.0 / rho[s];
    frame_rhs_1d(Dn[s], ir, U[s], bx);
    frame_rhs_1d(Dnn[s], ir, U[s], bxx);
    double tb = tau;  // collision time of the Chapman-Enskog correction (Knudsen reading)
    if (P.viscous) {
      double d[3], fr[3];
#pragma unroll
      for (int v = 0; v < 3; ++v) d[v] = Dn[s][v] * ir;
      to_frame_1d(d, U[s], fr);
      tb = bracket_tau(tau, rate_term(sqrt(P.gamma * pr[s] * ir), fr[0], fr[1], 0.0, fr[2]));
    }
    const double tvb = P.viscous ? tb : 0.0;
    TC ax[3], ay[3] = {0, 0, 0}, At[3] = {0, 0, 0}, dxx[3], dxy[3] = {0, 0, 0}, dyy[3] = {0, 0, 0},
                                 bxt[3] = {0, 0, 0}, byt[3] = {0, 0, 0}, Bt[3] = {0, 0, 0};
    const TC us = (TC)U[s];
    if (P.viscous)
      coef_side_ns_1d<TC>(th, kp, (TC)P.nth, us, TC(0), bx, zero, bxx, zero, zero, ax, ay, At, dxx, dxy, dyy, bxt,
                          byt, Bt);
    else
      coef_side_euler_1d<TC>(th, kp, (TC)P.nth, us, TC(0), bx, zero, bxx, zero, zero, ax, ay, At, dxx, dxy, dyy,
                             bxt, byt, Bt);
    TC AF[3] = {0, 0, 0}, BF[3] = {0, 0, 0}, V0[3] = {0, 0, 0}, m0[3], m1[3];
    auto acc = [&](double wi, double wc) {
      const TC a = (TC)wi, b = (TC)wc;
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        AF[v] += a * m0[v];
        BF[v] += a * m1[v];
        V0[v] += b * m0[v];
      }
    };
    // C8 g a1 u  [and -tau C7 g a1 u]
    mom_half_conv_1d<TC>(th, kp, ht, us, TC(0), ax, ay, m0, m1);
    acc(w.I[8] - tvb * w.I[7], w.C[8] - tvb * w.C[7]);
    // 1/2 C7 t^2 g (a1^2 + d11) u^2  [and -tau C8 g (a1^2 + d11) u^2]
    mom_half_quad_1d<TC>(th, kp, ht, us, TC(0), ax, ay, dxx, dxy, dyy, m0, m1);
    acc(0.5 * w.I[10] - tvb * w.I[8], 0.5 * w.C[10] - tvb * w.C[8]);
    if (P.viscous) {
      // -tau C7 g A, -tau C8 g (A a1 + b1) u
      mom_half_A_1d<TC>(th, kp, ht, us, TC(0), At, m0, m1);
      acc(-tb * w.I[7], -tb * w.C[7]);
      mom_half_tlin_1d<TC>(th, kp, ht, us, TC(0), ax, ay, At, bxt, byt, m0, m1);
      acc(-tb * w.I[8], -tb * w.C[8]);
    }
    add(AF, BF, V0, U[s], rho[s]);
  }
  if (P.viscous) {
    // Prandtl-number fix: energy flux += (1/Pr - 1) q, q the heat flux
    // relative to the velocity of g0
    const double k2 = 0.5 * U0 * U0;
    const double qh = flux[2] - U0 * flux[1] + k2 * flux[0] - U0 * (E[2] - U0 * E[1] + k2 * E[0]);
    flux[2] += P.prfix * qh;
  }
  return true;
}

}  // namespace gks
