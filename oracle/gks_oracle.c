/*
 * gks_oracle.c -- plain FP64 CPU oracle for the compact third-order
 * gas-kinetic scheme of Pan & Xu (arXiv:1412.4489).
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py.  It shares no code with the HIP library.
 *
 * Style: literal and slow.  Every velocity-dependent quantity is a polynomial
 * in (u, v, xi^2) (struct vpoly), products are formed term by term, and each
 * moment is sum(coef * <u^a><v^b><xi^2e>) from Gaussian moment tables.  The
 * expansion coefficients come from a Gaussian elimination on the Gram matrix
 * <psi psi^T>.  The distribution function at the interface is assembled term
 * by term as printed in eq. dis1 (hydrodynamic part) and eq. dis2 (kinetic
 * part).  Readings of silent or garbled passages are marked "reading:".
 *
 * Built with -O2 -ffp-contract=off (no FMA contraction, no fast-math).
 */
#include "gks_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Polynomials in the particle velocity: sum c[a][b][e] u^a v^b (xi^2)^e.    */
/* ------------------------------------------------------------------------ */

#define VD 10 /* total degree bound, u and v count 1, xi^2 counts 2 */

typedef struct {
  int deg;
  double c[VD + 1][VD + 1][VD / 2 + 1];
} vpoly;

static void vp_zero(vpoly* p) { memset(p, 0, sizeof(*p)); }

static void vp_const(vpoly* p, double s) {
  vp_zero(p);
  p->c[0][0][0] = s;
}

/* u^a v^b */
static void vp_mono(vpoly* p, int a, int b, double s) {
  vp_zero(p);
  p->c[a][b][0] = s;
  p->deg = a + b;
}

/* coefficient vector -> polynomial.
 * 2D: a0 + a1 u + a2 v + a3 (u^2 + v^2 + xi^2)/2 ; 1D: a0 + a1 u + a2 (u^2 + xi^2)/2
 * (the expansion form of Sec. 2.2 in terms of psi). */
static void vp_lin(vpoly* p, int dim, const double* a) {
  vp_zero(p);
  p->deg = 2;
  p->c[0][0][0] = a[0];
  p->c[1][0][0] = a[1];
  if (dim == 2) {
    p->c[0][1][0] = a[2];
    p->c[2][0][0] = 0.5 * a[3];
    p->c[0][2][0] = 0.5 * a[3];
    p->c[0][0][1] = 0.5 * a[3];
  } else {
    p->c[2][0][0] = 0.5 * a[2];
    p->c[0][0][1] = 0.5 * a[2];
  }
}

static void vp_mul(vpoly* r, const vpoly* p, const vpoly* q) {
  vpoly t;
  vp_zero(&t);
  t.deg = p->deg + q->deg;
  if (t.deg > VD) abort();
  for (int a1 = 0; a1 <= p->deg; ++a1)
    for (int b1 = 0; a1 + b1 <= p->deg; ++b1)
      for (int e1 = 0; a1 + b1 + 2 * e1 <= p->deg; ++e1) {
        double x = p->c[a1][b1][e1];
        if (x == 0.0) continue;
        for (int a2 = 0; a2 <= q->deg; ++a2)
          for (int b2 = 0; a2 + b2 <= q->deg; ++b2)
            for (int e2 = 0; a2 + b2 + 2 * e2 <= q->deg; ++e2) {
              double y = q->c[a2][b2][e2];
              if (y == 0.0) continue;
              t.c[a1 + a2][b1 + b2][e1 + e2] += x * y;
            }
      }
  *r = t;
}

/* r += s * p */
static void vp_axpy(vpoly* r, double s, const vpoly* p) {
  if (p->deg > r->deg) r->deg = p->deg;
  for (int a = 0; a <= p->deg; ++a)
    for (int b = 0; a + b <= p->deg; ++b)
      for (int e = 0; a + b + 2 * e <= p->deg; ++e) r->c[a][b][e] += s * p->c[a][b][e];
}

static double vp_eval(const vpoly* p, double u, double v, double xi2) {
  double pu[VD + 1], pv[VD + 1], px[VD / 2 + 1];
  pu[0] = pv[0] = px[0] = 1.0;
  for (int a = 1; a <= VD; ++a) {
    pu[a] = pu[a - 1] * u;
    pv[a] = pv[a - 1] * v;
  }
  for (int e = 1; e <= VD / 2; ++e) px[e] = px[e - 1] * xi2;
  double s = 0.0;
  for (int a = 0; a <= p->deg; ++a)
    for (int b = 0; a + b <= p->deg; ++b)
      for (int e = 0; a + b + 2 * e <= p->deg; ++e)
        if (p->c[a][b][e] != 0.0) s += p->c[a][b][e] * pu[a] * pv[b] * px[e];
  return s;
}

/* ------------------------------------------------------------------------ */
/* Maxwellian and its moments (Sec. 2.1; moment formulas are the textbook    */
/* Gaussian and half-Gaussian integrals, which the paper does not print).    */
/* ------------------------------------------------------------------------ */

typedef struct {
  int dim;
  double rho, U, V, lam, K;
  double Mu[16], Mv[16], Mx[8];
  double G[4][4]; /* Gram matrix <psi_i psi_j>, filled for whole-space tables */
} mtab;

/* K internal degrees of freedom: 2D as printed in Sec. 2.1; 1D reading: the
 * same relation gamma = (N+2)/N with N = K+1 total thermal degrees of freedom. */
static double internal_dof(int dim, double gamma) {
  return dim == 2 ? (4.0 - 2.0 * gamma) / (gamma - 1.0) : (3.0 - gamma) / (gamma - 1.0);
}

/* (rho, U, V, lambda) of a conservative state; lambda = rho / (2p). */
static int primitive(int dim, double gamma, const double* W, double* prim) {
  double rho = W[0];
  if (!(rho > 0.0)) return -1;
  double U = W[1] / rho;
  double V = dim == 2 ? W[2] / rho : 0.0;
  double rE = dim == 2 ? W[3] : W[2];
  double p = (gamma - 1.0) * (rE - 0.5 * rho * (U * U + V * V));
  if (!(p > 0.0)) return -1;
  prim[0] = rho;
  prim[1] = U;
  prim[2] = V;
  prim[3] = rho / (2.0 * p);
  return 0;
}

static double mom(const mtab* m, int a, int b, int e) { return m->Mu[a] * m->Mv[b] * m->Mx[e]; }

/* out_i = < u^s psi_i P >, normalised by rho */
static void vp_psi_moment(const vpoly* P, int s, const mtab* m, double* out) {
  int nv = m->dim + 2;
  for (int i = 0; i < nv; ++i) out[i] = 0.0;
  for (int a = 0; a <= P->deg; ++a)
    for (int b = 0; a + b <= P->deg; ++b)
      for (int e = 0; a + b + 2 * e <= P->deg; ++e) {
        double c = P->c[a][b][e];
        if (c == 0.0) continue;
        int as = a + s;
        out[0] += c * mom(m, as, b, e);
        out[1] += c * mom(m, as + 1, b, e);
        if (m->dim == 2) {
          out[2] += c * mom(m, as, b + 1, e);
          out[3] += 0.5 * c * (mom(m, as + 2, b, e) + mom(m, as, b + 2, e) + mom(m, as, b, e + 1));
        } else {
          out[2] += 0.5 * c * (mom(m, as + 2, b, e) + mom(m, as, b, e + 1));
        }
      }
}

/* scalar moment < P > */
static double vp_moment(const vpoly* P, const mtab* m) {
  double s = 0.0;
  for (int a = 0; a <= P->deg; ++a)
    for (int b = 0; a + b <= P->deg; ++b)
      for (int e = 0; a + b + 2 * e <= P->deg; ++e)
        if (P->c[a][b][e] != 0.0) s += P->c[a][b][e] * mom(m, a, b, e);
  return s;
}

static int mtab_init(mtab* m, int dim, double gamma, const double* W, int half) {
  double prim[4];
  if (primitive(dim, gamma, W, prim)) return -1;
  m->dim = dim;
  m->rho = prim[0];
  m->U = prim[1];
  m->V = prim[2];
  m->lam = prim[3];
  m->K = internal_dof(dim, gamma);
  double lam = m->lam, U = m->U, V = m->V;
  /* u: whole space <u^0> = 1, <u> = U; half spaces via erfc and exp. */
  if (half == 0) {
    m->Mu[0] = 1.0;
    m->Mu[1] = U;
  } else if (half > 0) {
    m->Mu[0] = 0.5 * erfc(-sqrt(lam) * U);
    m->Mu[1] = U * m->Mu[0] + 0.5 * exp(-lam * U * U) / sqrt(M_PI * lam);
  } else {
    m->Mu[0] = 0.5 * erfc(sqrt(lam) * U);
    m->Mu[1] = U * m->Mu[0] - 0.5 * exp(-lam * U * U) / sqrt(M_PI * lam);
  }
  /* <u^(n+2)> = U <u^(n+1)> + (n+1)/(2 lambda) <u^n> holds for all three. */
  for (int n = 0; n + 2 < 16; ++n) m->Mu[n + 2] = U * m->Mu[n + 1] + (n + 1) / (2.0 * lam) * m->Mu[n];
  m->Mv[0] = 1.0;
  m->Mv[1] = dim == 2 ? V : 0.0;
  for (int n = 0; n + 2 < 16; ++n)
    m->Mv[n + 2] = (dim == 2 ? V * m->Mv[n + 1] + (n + 1) / (2.0 * lam) * m->Mv[n] : 0.0);
  /* xi: K independent Gaussian components, <xi^2e> = prod_{i<e} (K + 2i)/(2 lambda) */
  m->Mx[0] = 1.0;
  for (int e = 0; e + 1 < 8; ++e) m->Mx[e + 1] = m->Mx[e] * (m->K + 2.0 * e) / (2.0 * lam);
  /* Gram matrix <psi_i psi_j> */
  int nv = dim + 2;
  for (int j = 0; j < nv; ++j) {
    double ej[4] = {0, 0, 0, 0}, col[4];
    ej[j] = 1.0;
    vpoly pj;
    vp_lin(&pj, dim, ej);
    vp_psi_moment(&pj, 0, m, col);
    for (int i = 0; i < nv; ++i) m->G[i][j] = col[i];
  }
  return 0;
}

/* Gaussian elimination with partial pivoting: G a = b */
static int gauss_solve(int n, double A[4][4], const double* b, double* x) {
  double M[4][5];
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) M[i][j] = A[i][j];
    M[i][n] = b[i];
  }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
    if (M[piv][c] == 0.0) return -1;
    if (piv != c)
      for (int j = 0; j <= n; ++j) {
        double t = M[c][j];
        M[c][j] = M[piv][j];
        M[piv][j] = t;
      }
    for (int r = c + 1; r < n; ++r) {
      double f = M[r][c] / M[c][c];
      for (int j = c; j <= n; ++j) M[r][j] -= f * M[c][j];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = M[i][n];
    for (int j = i + 1; j < n; ++j) s -= M[i][j] * x[j];
    x[i] = s / M[i][i];
  }
  return 0;
}

/* S(b): the coefficient vector a with <a psi> = b */
static void solve_tab(const mtab* m, const double* b, double* a) {
  double G[4][4];
  memcpy(G, m->G, sizeof(G));
  gauss_solve(m->dim + 2, G, b, a);
}

/* ------------------------------------------------------------------------ */
/* Coefficient systems (the system after eq. dis3).                          */
/* ------------------------------------------------------------------------ */

enum { CAX = 0, CAY, CA, CDXX, CDXY, CDYY, CBX, CBY, CB };

/* which: 0 = g0 (all nine), 1 = side Euler (ax..dyy), 2 = side NS (+ A, bx, by) */
static void coefficients_tab(const mtab* m, const double* Wx, const double* Wy, const double* Wxx,
                             const double* Wxy, const double* Wyy, int which, double coef[9][4]) {
  int dim = m->dim, nv = dim + 2;
  double rho = m->rho, rhs[4] = {0, 0, 0, 0}, mm[4];
  memset(coef, 0, sizeof(double) * 36);
  vpoly a1, a2, A, d11, d12, d22, b1, b2, u, v, t1, t2, t3, S;
  vp_mono(&u, 1, 0, 1.0);
  vp_mono(&v, 0, 1, 1.0);
  vp_zero(&a2);
  vp_zero(&d12);
  vp_zero(&d22);
  vp_zero(&b2);

  /* <a1> = dU/dx, <a2> = dU/dy */
  for (int i = 0; i < nv; ++i) rhs[i] = Wx[i] / rho;
  solve_tab(m, rhs, coef[CAX]);
  vp_lin(&a1, dim, coef[CAX]);
  if (dim == 2) {
    for (int i = 0; i < nv; ++i) rhs[i] = Wy[i] / rho;
    solve_tab(m, rhs, coef[CAY]);
    vp_lin(&a2, dim, coef[CAY]);
  }
  /* <a1^2 + d11> = d2U/dx2, <a2^2 + d22> = d2U/dy2, <a1 a2 + d12> = d2U/dxdy */
  vp_mul(&t1, &a1, &a1);
  vp_psi_moment(&t1, 0, m, mm);
  for (int i = 0; i < nv; ++i) rhs[i] = Wxx[i] / rho - mm[i];
  solve_tab(m, rhs, coef[CDXX]);
  vp_lin(&d11, dim, coef[CDXX]);
  if (dim == 2) {
    vp_mul(&t1, &a1, &a2);
    vp_psi_moment(&t1, 0, m, mm);
    for (int i = 0; i < nv; ++i) rhs[i] = Wxy[i] / rho - mm[i];
    solve_tab(m, rhs, coef[CDXY]);
    vp_lin(&d12, dim, coef[CDXY]);
    vp_mul(&t1, &a2, &a2);
    vp_psi_moment(&t1, 0, m, mm);
    for (int i = 0; i < nv; ++i) rhs[i] = Wyy[i] / rho - mm[i];
    solve_tab(m, rhs, coef[CDYY]);
    vp_lin(&d22, dim, coef[CDYY]);
  }
  if (which == 1) return;

  /* <A + a1 u + a2 v> = 0 */
  vp_mul(&t1, &a1, &u);
  vp_mul(&t2, &a2, &v);
  vp_axpy(&t1, 1.0, &t2);
  vp_psi_moment(&t1, 0, m, mm);
  for (int i = 0; i < nv; ++i) rhs[i] = -mm[i];
  solve_tab(m, rhs, coef[CA]);
  vp_lin(&A, dim, coef[CA]);

  /* <(a1^2 + d11) u + (a1 a2 + d12) v + (A a1 + b1)> = 0 */
  vp_mul(&t1, &a1, &a1);
  vp_axpy(&t1, 1.0, &d11);
  vp_mul(&S, &t1, &u);
  vp_mul(&t1, &a1, &a2);
  vp_axpy(&t1, 1.0, &d12);
  vp_mul(&t2, &t1, &v);
  vp_axpy(&S, 1.0, &t2);
  vp_mul(&t3, &A, &a1);
  vp_axpy(&S, 1.0, &t3);
  vp_psi_moment(&S, 0, m, mm);
  for (int i = 0; i < nv; ++i) rhs[i] = -mm[i];
  solve_tab(m, rhs, coef[CBX]);
  vp_lin(&b1, dim, coef[CBX]);

  /* <(a1 a2 + d12) u + (a2^2 + d22) v + (A a2 + b2)> = 0 */
  if (dim == 2) {
    vp_mul(&t1, &a1, &a2);
    vp_axpy(&t1, 1.0, &d12);
    vp_mul(&S, &t1, &u);
    vp_mul(&t1, &a2, &a2);
    vp_axpy(&t1, 1.0, &d22);
    vp_mul(&t2, &t1, &v);
    vp_axpy(&S, 1.0, &t2);
    vp_mul(&t3, &A, &a2);
    vp_axpy(&S, 1.0, &t3);
    vp_psi_moment(&S, 0, m, mm);
    for (int i = 0; i < nv; ++i) rhs[i] = -mm[i];
    solve_tab(m, rhs, coef[CBY]);
    vp_lin(&b2, dim, coef[CBY]);
  }
  if (which == 2) return;

  /* <(A a1 + b1) u + (A a2 + b2) v + (A^2 + B)> = 0 */
  vp_mul(&t1, &A, &a1);
  vp_axpy(&t1, 1.0, &b1);
  vp_mul(&S, &t1, &u);
  vp_mul(&t1, &A, &a2);
  vp_axpy(&t1, 1.0, &b2);
  vp_mul(&t2, &t1, &v);
  vp_axpy(&S, 1.0, &t2);
  vp_mul(&t3, &A, &A);
  vp_axpy(&S, 1.0, &t3);
  vp_psi_moment(&S, 0, m, mm);
  for (int i = 0; i < nv; ++i) rhs[i] = -mm[i];
  solve_tab(m, rhs, coef[CB]);
}

/* ------------------------------------------------------------------------ */
/* Time coefficients C_1..C_8 (Sec. 2.2, after eq. dis1) and their integrals */
/* ------------------------------------------------------------------------ */

enum { T_C1 = 0, T_C2, T_C3, T_C4, T_C5, T_C6, T_C7, T_C8, T_C7T, T_C7T2, T_NFN };

static double expo(double t, double tau) { return tau > 0.0 ? exp(-t / tau) : 0.0; }

void orc_time_coefficients(double tau, double t, int exact_c, double* C) {
  double e = expo(t, tau);
  C[T_C1] = 1.0 - e;
  C[T_C2] = (t + tau) * e - tau;
  C[T_C3] = t - tau + tau * e;
  C[T_C4] = -(t * t + 2.0 * t * tau) * e;
  C[T_C5] = t * t - 2.0 * t * tau;
  C[T_C6] = -t * tau * (1.0 + e);
  C[T_C7] = e;
  C[T_C8] = -t * e;
  C[T_C7T] = t * e;
  C[T_C7T2] = t * t * e;
  if (exact_c) { /* the exact exponential integrals keep a 2 tau^2 (1 - e) term */
    double x = 2.0 * tau * tau * (1.0 - e);
    C[T_C4] += x;
    C[T_C5] += x;
    C[T_C6] += x;
  }
}

/* closed-form integrals over [0, dt] of the functions above */
void orc_time_integrals(double tau, double dt, int exact_c, double* I) {
  double E = expo(dt, tau);
  double t2 = tau * tau, t3 = t2 * tau, d2 = dt * dt;
  I[T_C1] = dt - tau * (1.0 - E);
  I[T_C2] = -tau * dt * (1.0 + E) + 2.0 * t2 * (1.0 - E);
  I[T_C3] = 0.5 * d2 - tau * dt + t2 * (1.0 - E);
  I[T_C4] = tau * (dt + 2.0 * tau) * (dt + 2.0 * tau) * E - 4.0 * t3;
  I[T_C5] = d2 * dt / 3.0 - tau * d2;
  I[T_C6] = -0.5 * tau * d2 + t2 * dt * E - t3 * (1.0 - E);
  I[T_C7] = tau * (1.0 - E);
  I[T_C8] = tau * (dt + tau) * E - t2;
  I[T_C7T] = t2 - tau * (dt + tau) * E;
  I[T_C7T2] = 2.0 * t3 - tau * (d2 + 2.0 * tau * dt + 2.0 * t2) * E;
  if (exact_c) {
    double x = 2.0 * t2 * (dt - tau * (1.0 - E));
    I[T_C4] += x;
    I[T_C5] += x;
    I[T_C6] += x;
  }
}

/* ------------------------------------------------------------------------ */
/* Assembly of the interface distribution function                          */
/* ------------------------------------------------------------------------ */

/* A set of consumers; each accumulates sum_terms wfn[fn] * wy[ypow] * s * P. */
#define NACC 3
typedef struct {
  int n;
  double wfn[NACC][T_NFN];
  double wy[NACC][3];
  vpoly acc[NACC];
} accset;

static void acc_add(accset* S, int fn, int ypow, double s, const vpoly* P) {
  for (int k = 0; k < S->n; ++k) {
    double w = S->wfn[k][fn] * S->wy[k][ypow] * s;
    if (w != 0.0) vp_axpy(&S->acc[k], w, P);
  }
}

typedef struct {
  vpoly a1, a2, A, d11, d12, d22, b1, b2, B;
} cpolys;

static void make_cpolys(cpolys* c, int dim, double coef[9][4]) {
  vp_lin(&c->a1, dim, coef[CAX]);
  vp_lin(&c->a2, dim, coef[CAY]);
  vp_lin(&c->A, dim, coef[CA]);
  vp_lin(&c->d11, dim, coef[CDXX]);
  vp_lin(&c->d12, dim, coef[CDXY]);
  vp_lin(&c->d22, dim, coef[CDYY]);
  vp_lin(&c->b1, dim, coef[CBX]);
  vp_lin(&c->b2, dim, coef[CBY]);
  vp_lin(&c->B, dim, coef[CB]);
}

/* x*y + z */
static void pmuladd(vpoly* r, const vpoly* x, const vpoly* y, const vpoly* z) {
  vp_mul(r, x, y);
  vp_axpy(r, 1.0, z);
}
static void pmul3(vpoly* r, const vpoly* x, const vpoly* y, const vpoly* z) {
  vpoly t;
  vp_mul(&t, x, y);
  vp_mul(r, &t, z);
}

/* eq. dis1: hydrodynamic part, weight g0, whole velocity space */
static void assemble_hydro(accset* S, int dim, const cpolys* c) {
  vpoly one, u, v, t, Dxx, Dxy, Dyy, Tx, Ty, Ttt;
  vp_const(&one, 1.0);
  vp_mono(&u, 1, 0, 1.0);
  vp_mono(&v, 0, 1, 1.0);
  pmuladd(&Dxx, &c->a1, &c->a1, &c->d11); /* a1^2 + d11 */
  pmuladd(&Tx, &c->A, &c->a1, &c->b1);    /* A a1 + b1  */
  pmuladd(&Ttt, &c->A, &c->A, &c->B);     /* A^2 + B    */

  /* C1 g0 + C2 g0 a1 u + C2 g0 a2 v + C1 g0 a2 y + C3 g0 A */
  acc_add(S, T_C1, 0, 1.0, &one);
  vp_mul(&t, &c->a1, &u);
  acc_add(S, T_C2, 0, 1.0, &t);
  if (dim == 2) {
    vp_mul(&t, &c->a2, &v);
    acc_add(S, T_C2, 0, 1.0, &t);
    acc_add(S, T_C1, 1, 1.0, &c->a2);
  }
  acc_add(S, T_C3, 0, 1.0, &c->A);
  /* + 1/2 C4 g0 (a1^2 + d11) u^2 + C6 g0 (A a1 + b1) u + 1/2 C5 g0 (A^2 + B) */
  pmul3(&t, &Dxx, &u, &u);
  acc_add(S, T_C4, 0, 0.5, &t);
  vp_mul(&t, &Tx, &u);
  acc_add(S, T_C6, 0, 1.0, &t);
  acc_add(S, T_C5, 0, 0.5, &Ttt);
  if (dim == 1) return;

  pmuladd(&Dxy, &c->a1, &c->a2, &c->d12); /* a1 a2 + d12 */
  pmuladd(&Dyy, &c->a2, &c->a2, &c->d22); /* a2^2 + d22 */
  pmuladd(&Ty, &c->A, &c->a2, &c->b2);    /* A a2 + b2  */
  /* + 1/2 C1 g0 (a2^2 + d22) y^2 + C2 g0 (a2^2 + d22) v y + 1/2 C4 g0 (a2^2 + d22) v^2 */
  acc_add(S, T_C1, 2, 0.5, &Dyy);
  vp_mul(&t, &Dyy, &v);
  acc_add(S, T_C2, 1, 1.0, &t);
  pmul3(&t, &Dyy, &v, &v);
  acc_add(S, T_C4, 0, 0.5, &t);
  /* + C2 g0 (a1 a2 + d12) u y + C4 g0 (a1 a2 + d12) u v */
  vp_mul(&t, &Dxy, &u);
  acc_add(S, T_C2, 1, 1.0, &t);
  pmul3(&t, &Dxy, &u, &v);
  acc_add(S, T_C4, 0, 1.0, &t);
  /* + C3 g0 (A a2 + b2) y + C6 g0 (A a2 + b2) v */
  acc_add(S, T_C3, 1, 1.0, &Ty);
  vp_mul(&t, &Ty, &v);
  acc_add(S, T_C6, 0, 1.0, &t);
}

/* eq. dis2: kinetic part of side k, weight g_k on its half space.
 * Euler reading: f_G = g_k, i.e. the tau(...) brackets are absent (tv = 0),
 * while C7, C8 keep their tau. */
static void assemble_kinetic(accset* S, int dim, const cpolys* c, double tv) {
  vpoly one, u, v, t, br, Dxx, Dxy, Dyy, Tx, Ty;
  vp_const(&one, 1.0);
  vp_mono(&u, 1, 0, 1.0);
  vp_mono(&v, 0, 1, 1.0);
  pmuladd(&Dxx, &c->a1, &c->a1, &c->d11);
  pmuladd(&Tx, &c->A, &c->a1, &c->b1);
  if (dim == 2) {
    pmuladd(&Dxy, &c->a1, &c->a2, &c->d12);
    pmuladd(&Dyy, &c->a2, &c->a2, &c->d22);
    pmuladd(&Ty, &c->A, &c->a2, &c->b2);
  }

  /* C7 g [1 - tau (a1 u + a2 v + A)] */
  acc_add(S, T_C7, 0, 1.0, &one);
  if (tv != 0.0) {
    vp_mul(&br, &c->a1, &u);
    if (dim == 2) {
      vp_mul(&t, &c->a2, &v);
      vp_axpy(&br, 1.0, &t);
    }
    vp_axpy(&br, 1.0, &c->A);
    acc_add(S, T_C7, 0, -tv, &br);
  }
  /* C8 g [a1 u - tau ((a1^2 + d11) u^2 + (a1 a2 + d12) u v + (A a1 + b1) u)] */
  vp_mul(&t, &c->a1, &u);
  acc_add(S, T_C8, 0, 1.0, &t);
  if (tv != 0.0) {
    pmul3(&br, &Dxx, &u, &u);
    if (dim == 2) {
      pmul3(&t, &Dxy, &u, &v);
      vp_axpy(&br, 1.0, &t);
    }
    vp_mul(&t, &Tx, &u);
    vp_axpy(&br, 1.0, &t);
    acc_add(S, T_C8, 0, -tv, &br);
  }
  if (dim == 2) {
    /* C8 g [a2 v - tau ((a1 a2 + d12) u v + (a2^2 + d22) v^2 + (A a2 + b2) v)] */
    vp_mul(&t, &c->a2, &v);
    acc_add(S, T_C8, 0, 1.0, &t);
    if (tv != 0.0) {
      pmul3(&br, &Dxy, &u, &v);
      pmul3(&t, &Dyy, &v, &v);
      vp_axpy(&br, 1.0, &t);
      vp_mul(&t, &Ty, &v);
      vp_axpy(&br, 1.0, &t);
      acc_add(S, T_C8, 0, -tv, &br);
    }
    /* C7 g [a2 - tau ((a1 a2 + d12) u + (a2^2 + d22) v + (A a2 + b2))] y */
    acc_add(S, T_C7, 1, 1.0, &c->a2);
    if (tv != 0.0) {
      vp_mul(&br, &Dxy, &u);
      vp_mul(&t, &Dyy, &v);
      vp_axpy(&br, 1.0, &t);
      vp_axpy(&br, 1.0, &Ty);
      acc_add(S, T_C7, 1, -tv, &br);
    }
  }
  /* 1/2 C7 g [(a1^2+d11)(-ut)^2 + 2(a1 a2+d12)(-ut)(y-vt) + (a2^2+d22)(y-vt)^2]
   * expanded in powers of t and y:
   *   (-ut)^2          -> t^2 u^2
   *   2(-ut)(y - vt)   -> -2 t y u + 2 t^2 u v
   *   (y - vt)^2       -> y^2 - 2 t y v + t^2 v^2                     */
  pmul3(&t, &Dxx, &u, &u);
  acc_add(S, T_C7T2, 0, 0.5, &t);
  if (dim == 2) {
    vp_mul(&t, &Dxy, &u);
    acc_add(S, T_C7T, 1, -1.0, &t);
    pmul3(&t, &Dxy, &u, &v);
    acc_add(S, T_C7T2, 0, 1.0, &t);
    acc_add(S, T_C7, 2, 0.5, &Dyy);
    vp_mul(&t, &Dyy, &v);
    acc_add(S, T_C7T, 1, -1.0, &t);
    pmul3(&t, &Dyy, &v, &v);
    acc_add(S, T_C7T2, 0, 0.5, &t);
  }
}

/* ------------------------------------------------------------------------ */
/* Equilibrium quadratic (Sec. 3.3)                                          */
/* ------------------------------------------------------------------------ */

/* Ueq[m][n][var]: m = 0 left column, 1 right column; n = 0, 1, 2 tangential
 * index -1, 0, +1.  q[0..4] = b2..b6 (normal slope, tangential slope, normal
 * curvature, tangential curvature, cross).  1D: b2 = q[0], b4 = q[2]. */
void orc_equilibrium_poly(int dim, const double* Ueq, const double* U0, double h, double k, double* q) {
  int nv = dim + 2;
#define UE(m, n, v) Ueq[((m)*3 + (n)) * 4 + (v)]
  for (int v = 0; v < nv; ++v) {
    if (dim == 2) {
      q[0 * 4 + v] = ((UE(1, 2, v) - UE(0, 2, v)) + 2.0 * (UE(1, 1, v) - UE(0, 1, v)) + (UE(1, 0, v) - UE(0, 0, v))) /
                     (4.0 * h);
      q[1 * 4 + v] = (UE(1, 2, v) - UE(1, 0, v) + UE(0, 2, v) - UE(0, 0, v)) / (4.0 * k);
      q[2 * 4 + v] = (26.0 * (UE(1, 1, v) + UE(0, 1, v)) - (UE(1, 2, v) + UE(0, 2, v) + UE(1, 0, v) + UE(0, 0, v)) -
                      48.0 * U0[v]) /
                     (8.0 * h * h);
      q[3 * 4 + v] =
          (UE(1, 2, v) - 2.0 * UE(1, 1, v) + UE(1, 0, v) + UE(0, 2, v) - 2.0 * UE(0, 1, v) + UE(0, 0, v)) / (2.0 * k * k);
      q[4 * 4 + v] = (UE(1, 2, v) - UE(0, 2, v) - UE(1, 0, v) + UE(0, 0, v)) / (2.0 * h * k);
    } else {
      /* the same least-squares conditions on the two cells sharing the interface */
      q[0 * 4 + v] = (UE(1, 1, v) - UE(0, 1, v)) / h;
      q[1 * 4 + v] = 0.0;
      q[2 * 4 + v] = 3.0 * (UE(0, 1, v) + UE(1, 1, v) - 2.0 * U0[v]) / (h * h);
      q[3 * 4 + v] = 0.0;
      q[4 * 4 + v] = 0.0;
    }
  }
#undef UE
}

/* ------------------------------------------------------------------------ */
/* One interface: eq. compatibility2, Sec. 3.3, Sec. 4 tau, systems, flux    */
/* (eq. finite), point values (eq. point).                                   */
/* ------------------------------------------------------------------------ */

static double pressure(int dim, double gamma, const double* W) {
  double rho = W[0], ru = W[1], rv = dim == 2 ? W[2] : 0.0, rE = dim == 2 ? W[3] : W[2];
  return (gamma - 1.0) * (rE - 0.5 * (ru * ru + rv * rv) / rho);
}

/* Reading (eq. dis2 for the Navier-Stokes equations): the correction
 * -tau (a1 u + a2 v + A) g_k of the initial distribution of side k is the
 * first-order Chapman-Enskog expansion, valid while the side's cell
 * Knudsen number tau s is below one, s the rate at which its equilibrium
 * changes for a particle at the sound speed c: the sum over the normal and
 * the tangential direction of c |d rho| / rho + |d u| + |d v| +
 * |d (rho e)| / (rho c), from the side's interface values and derivatives
 * (rho e = p / (gamma - 1)).  Where tau s exceeds one, the correction is
 * taken with tau capped at 1 / s; the relaxation (the time integrals) keeps
 * tau.  In resolved flow (tau s < 1) this is the printed bracket.  Without
 * the cap the shock of the viscous shock tube (Sec. 4.7) at cell Knudsen
 * numbers near two (300 x 150 at Re 200, 1000 x 500 at Re 1000) drives the
 * scheme out of the physical states within its first 20-65 steps. */
static long g_capped = 0;
static double kinetic_bracket_tau(int dim, double gamma, double tau, const double* W, const double* Wn,
                                  const double* Ws) {
  double rho = W[0], u = W[1] / rho, v = dim == 2 ? W[2] / rho : 0.0;
  double p = pressure(dim, gamma, W), c = sqrt(gamma * p / rho), s = 0.0;
  for (int k = 0; k < dim; ++k) {
    const double* d = k == 0 ? Wn : Ws;
    double dr = d[0], du = (d[1] - u * dr) / rho, dv = dim == 2 ? (d[2] - v * dr) / rho : 0.0;
    double de = d[dim + 1] - u * d[1] - (dim == 2 ? v * d[2] : 0.0) + 0.5 * (u * u + v * v) * dr;
    s += c * fabs(dr) / rho + fabs(du) + fabs(dv) + fabs(de) / (rho * c);
  }
  if (!(tau * s > 1.0)) return tau;
#pragma omp atomic
  g_capped += 1;
  return 1.0 / s;
}

int orc_face(const orc_problem* P, const orc_face_input* in, double dt, orc_face_output* out) {
  int dim = P->dim, nv = dim + 2;
  double gamma = P->gamma;
  memset(out, 0, sizeof(*out));

  /* eq. compatibility2: U0 = int_{u>0} psi g_l + int_{u<0} psi g_r */
  mtab hl, hr, fl, fr, f0;
  if (mtab_init(&hl, dim, gamma, in->W[0], +1)) return -1;
  if (mtab_init(&hr, dim, gamma, in->W[1], -1)) return -1;
  double ml[4], mr[4], one_c[4] = {1, 0, 0, 0};
  vpoly one;
  vp_lin(&one, dim, one_c);
  vp_psi_moment(&one, 0, &hl, ml);
  vp_psi_moment(&one, 0, &hr, mr);
  for (int i = 0; i < nv; ++i) out->W0[i] = hl.rho * ml[i] + hr.rho * mr[i];

  /* Sec. 3.3: equilibrium quadratic from the six cell averages and U0 */
  if (in->curv) {
    /* logical coordinates (unit spacing), then the interface frame through
     * the metric (curvilinear grids) */
    double ql[5][4];
    orc_equilibrium_poly(dim, &in->Ueq[0][0][0], out->W0, 1.0, 1.0, &ql[0][0]);
    double G[2][2] = {{in->G[0], in->G[1]}, {0.0, in->G[2]}};
    for (int v = 0; v < nv; ++v) {
      double grad[2] = {ql[0][v], ql[1][v]}, hess[2][2] = {{ql[2][v], ql[4][v]}, {ql[4][v], ql[3][v]}};
      double hf[2][2];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          hf[a][b] = 0.0;
          for (int c = 0; c < 2; ++c)
            for (int e = 0; e < 2; ++e) hf[a][b] += G[a][c] * hess[c][e] * G[b][e];
        }
      out->q[0][v] = G[0][0] * grad[0] + G[0][1] * grad[1];
      out->q[1][v] = G[1][0] * grad[0] + G[1][1] * grad[1];
      out->q[2][v] = hf[0][0];
      out->q[3][v] = hf[1][1];
      out->q[4][v] = hf[0][1];
    }
  } else {
    orc_equilibrium_poly(dim, &in->Ueq[0][0][0], out->W0, in->dn, in->ds, &out->q[0][0]);
  }

  /* Sec. 4: collision time (reading: p_l, p_r of the two interface values,
   * p of U0) */
  double pl = pressure(dim, gamma, in->W[0]), pr = pressure(dim, gamma, in->W[1]);
  double p0 = pressure(dim, gamma, out->W0);
  double jump = fabs((pl - pr) / (pl + pr));
  double tau = P->viscous ? P->mu / p0 + P->tau_c * jump * dt : P->tau_eps * dt + P->tau_c * jump * dt;
  out->tau = tau;

  /* coefficient systems for g0 (all nine) and the two sides */
  if (mtab_init(&f0, dim, gamma, out->W0, 0)) return -2;
  if (mtab_init(&fl, dim, gamma, in->W[0], 0)) return -1;
  if (mtab_init(&fr, dim, gamma, in->W[1], 0)) return -1;
  double c0[9][4], cl[9][4], cr[9][4];
  coefficients_tab(&f0, out->q[0], out->q[1], out->q[2], out->q[4], out->q[3], 0, c0);
  int side_which = P->viscous ? 2 : 1;
  coefficients_tab(&fl, in->Wn[0], in->Ws[0], in->Wnn[0], in->Wns[0], in->Wss[0], side_which, cl);
  coefficients_tab(&fr, in->Wn[1], in->Ws[1], in->Wnn[1], in->Wns[1], in->Wss[1], side_which, cr);

  /* consumers: [0] time- and face-integrated f, [1], [2] f at t = dt and
   * y = -delta, +delta (Gauss points of the interface, delta = sqrt(3)/6 ds) */
  accset S;
  memset(&S, 0, sizeof(S));
  double Iw[T_NFN], Cw[T_NFN];
  orc_time_integrals(tau, dt, P->exact_c, Iw);
  orc_time_coefficients(tau, dt, P->exact_c, Cw);
  double ds = in->ds, delta = sqrt(3.0) / 6.0 * ds;
  if (dim == 2) {
    S.n = 3;
    for (int f = 0; f < T_NFN; ++f) {
      S.wfn[0][f] = Iw[f];
      S.wfn[1][f] = Cw[f];
      S.wfn[2][f] = Cw[f];
    }
    /* int_{-ds/2}^{ds/2} y^p dy = ds, 0, ds^3/12 */
    S.wy[0][0] = ds;
    S.wy[0][1] = 0.0;
    S.wy[0][2] = ds * ds * ds / 12.0;
    S.wy[1][0] = 1.0;
    S.wy[1][1] = -delta;
    S.wy[1][2] = delta * delta;
    S.wy[2][0] = 1.0;
    S.wy[2][1] = delta;
    S.wy[2][2] = delta * delta;
  } else {
    S.n = 2;
    for (int f = 0; f < T_NFN; ++f) {
      S.wfn[0][f] = Iw[f];
      S.wfn[1][f] = Cw[f];
    }
    S.wy[0][0] = 1.0;
    S.wy[1][0] = 1.0;
  }
  double tv = P->viscous ? tau : 0.0;
  double tvk[2] = {tv, tv};
  if (P->viscous)
    for (int k = 0; k < 2; ++k) tvk[k] = kinetic_bracket_tau(dim, gamma, tau, in->W[k], in->Wn[k], in->Ws[k]);
  double flux[4] = {0, 0, 0, 0}, pv[2][4] = {{0}}, heat = 0.0;
  const mtab* tabs[3] = {&f0, &hl, &hr};
  double* coefs[3] = {&c0[0][0], &cl[0][0], &cr[0][0]};
  vpoly H; /* heat-flux weight 1/2 (u - U0) ((u - U0)^2 + (v - V0)^2 + xi^2) */
  {
    double U0 = f0.U, V0 = f0.V;
    vpoly cu, cv, cc, xi2, t;
    double cuv[4] = {-U0, 1.0, 0.0, 0.0};
    vp_zero(&cu);
    cu.deg = 1;
    cu.c[0][0][0] = cuv[0];
    cu.c[1][0][0] = 1.0;
    vp_zero(&cv);
    cv.deg = 1;
    cv.c[0][0][0] = -V0;
    cv.c[0][1][0] = 1.0;
    vp_zero(&xi2);
    xi2.deg = 2;
    xi2.c[0][0][1] = 1.0;
    vp_mul(&cc, &cu, &cu);
    if (dim == 2) {
      vp_mul(&t, &cv, &cv);
      vp_axpy(&cc, 1.0, &t);
    }
    vp_axpy(&cc, 1.0, &xi2);
    vp_mul(&H, &cu, &cc);
    for (int a = 0; a <= H.deg; ++a)
      for (int b = 0; a + b <= H.deg; ++b)
        for (int e = 0; a + b + 2 * e <= H.deg; ++e) H.c[a][b][e] *= 0.5;
  }
  for (int r = 0; r < 3; ++r) {
    cpolys cp;
    double cf[9][4];
    memcpy(cf, coefs[r], sizeof(cf));
    make_cpolys(&cp, dim, cf);
    for (int k = 0; k < S.n; ++k) vp_zero(&S.acc[k]);
    if (r == 0)
      assemble_hydro(&S, dim, &cp);
    else
      assemble_kinetic(&S, dim, &cp, tvk[r - 1]);
    double m[4];
    const mtab* T = tabs[r];
    vp_psi_moment(&S.acc[0], 1, T, m); /* F = int u psi f */
    for (int i = 0; i < nv; ++i) flux[i] += T->rho * m[i];
    for (int g = 0; g < S.n - 1; ++g) { /* eq. point: U = int psi f */
      vp_psi_moment(&S.acc[1 + g], 0, T, m);
      for (int i = 0; i < nv; ++i) pv[g][i] += T->rho * m[i];
    }
    if (P->viscous) {
      vpoly Hf;
      vp_mul(&Hf, &H, &S.acc[0]);
      heat += T->rho * vp_moment(&Hf, T);
    }
  }
  /* Prandtl-number fix (reading: energy flux += (1/Pr - 1) q, q the heat
   * flux relative to the velocity of g0; Pr = 1 leaves the BGK flux). */
  if (P->viscous) flux[nv - 1] += (1.0 / P->prandtl - 1.0) * heat;
  out->heat = heat;
  memcpy(out->flux, flux, sizeof(flux));
  memcpy(out->pv, pv, sizeof(pv));
  return 0;
}

void orc_f_assembled(int dim, double gamma, int viscous, int exact_c, double tau, const double* prim,
                     const double* coef, double y, double t, int n, const double* u, const double* v,
                     const double* xi2, double* out) {
  double C[T_NFN];
  orc_time_coefficients(tau, t, exact_c, C);
  accset S;
  memset(&S, 0, sizeof(S));
  S.n = 1;
  for (int f = 0; f < T_NFN; ++f) S.wfn[0][f] = C[f];
  S.wy[0][0] = 1.0;
  S.wy[0][1] = y;
  S.wy[0][2] = y * y;
  double tv = viscous ? tau : 0.0, K = internal_dof(dim, gamma);
  double N = dim == 2 ? K + 2.0 : K + 1.0;
  for (int q = 0; q < n; ++q) out[q] = 0.0;
  /* r = 0: left side on u > 0; r = 1: right side on u < 0; r = 2: g0 */
  for (int r = 0; r < 3; ++r) {
    const double* pr = prim + 4 * r;
    double rho = pr[0], U = pr[1], V = pr[2], lam = pr[3];
    cpolys cp;
    double cf[9][4];
    memcpy(cf, coef + 36 * r, sizeof(cf));
    make_cpolys(&cp, dim, cf);
    vp_zero(&S.acc[0]);
    if (r == 2)
      assemble_hydro(&S, dim, &cp);
    else
      assemble_kinetic(&S, dim, &cp, tv);
    for (int q = 0; q < n; ++q) {
      if (r == 0 && !(u[q] > 0.0)) continue;
      if (r == 1 && !(u[q] < 0.0)) continue;
      double vv = dim == 2 ? v[q] : 0.0;
      double c2 = (u[q] - U) * (u[q] - U) + (dim == 2 ? (vv - V) * (vv - V) : 0.0) + xi2[q];
      /* Maxwellian density at one point of (u, v, xi) space, xi in R^K */
      double g = rho * pow(lam / M_PI, 0.5 * N) * exp(-lam * c2);
      out[q] += g * vp_eval(&S.acc[0], u[q], vv, xi2[q]);
    }
  }
}

/* exported building blocks ------------------------------------------------ */

int orc_moment_tables(int dim, double gamma, const double* W, int half, double* Mu, double* Mv, double* Mx,
                      double* prim) {
  mtab m;
  if (mtab_init(&m, dim, gamma, W, half)) return -1;
  memcpy(Mu, m.Mu, sizeof(m.Mu));
  memcpy(Mv, m.Mv, sizeof(m.Mv));
  memcpy(Mx, m.Mx, sizeof(m.Mx));
  prim[0] = m.rho;
  prim[1] = m.U;
  prim[2] = m.V;
  prim[3] = m.lam;
  return 0;
}

int orc_solve(int dim, double gamma, const double* W, const double* b, double* a) {
  mtab m;
  if (mtab_init(&m, dim, gamma, W, 0)) return -1;
  solve_tab(&m, b, a);
  return 0;
}

int orc_coefficients(int dim, double gamma, const double* W, const double* Wx, const double* Wy, const double* Wxx,
                     const double* Wxy, const double* Wyy, int which, double* coef) {
  mtab m;
  if (mtab_init(&m, dim, gamma, W, 0)) return -1;
  double c[9][4];
  coefficients_tab(&m, Wx, Wy, Wxx, Wxy, Wyy, which, c);
  memcpy(coef, c, sizeof(c));
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Compact reconstruction (Sec. 3.1, 3.2)                                    */
/* ------------------------------------------------------------------------ */

/* relative rounding noise of FP64 inputs taken as a tie of the cross
 * derivative's candidates: 2^-46 */
#define TIE_REL 1.4210854715202004e-14

static double minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return a > 0.0 ? (a < b ? a : b) : (a > b ? a : b);
}

/* Sec. 3.1.  Uw = Ubar_{i-1}, Ue = Ubar_{i+1}, Fm = U_{i-1/2}, Fp = U_{i+1/2}. */
void orc_recon1d_scalar(double Uc, double Ue, double Uw, double Fp, double Fm, double h, double eps, double C,
                        double* p) {
  /* one-sided stencils S1 = {U_{i-1}, U_{i-1/2}, U_i}, S2 = {U_i, U_{i+1/2}, U_{i+1}} */
  double a3_1 = 3.0 * (Uc + Uw - 2.0 * Fm) / (h * h);
  double a3_2 = 3.0 * (Uc + Ue - 2.0 * Fp) / (h * h);
  double ta2_1 = 2.0 * (Fm - Uc) / h;
  double ta2_2 = 2.0 * (Fp - Uc) / h;
  /* eq. limiter */
  double a3 = minmod(a3_1, a3_2);
  double a2 = minmod(-ta2_1 + a3 * h / 6.0, ta2_2 - a3 * h / 6.0);
  /* central stencil S3: cell averages of U2 on I_{i-1}, I_i, I_{i+1} */
  double c2 = (Ue - Uw) / (2.0 * h);
  double c4 = ((Ue + Uw) - 2.0 * Uc) / (h * h);
  /* eq. average with I(U1) = C h^2 and I = sum_l int h^(2l-1) (U^(l))^2 */
  double I1 = C * h * h;
  double I2 = h * h * c2 * c2 + 13.0 / 12.0 * h * h * h * h * c4 * c4;
  double al1 = 1.0 / ((eps + I1) * (eps + I1));
  double al2 = 1.0 / ((eps + I2) * (eps + I2));
  double w1 = al1 / (al1 + al2), w2 = al2 / (al1 + al2);
  p[0] = w1 * a2 + w2 * c2;
  p[1] = w1 * a3 + w2 * c4;
}

/* Sec. 3.2, eq. over-sys and the limiter, one direction: from the cell
 * average Uc, the neighbour averages Up (positive side) and Um (negative side)
 * and the two Gauss-point values on each of the cell's two interfaces across
 * that direction (Pp, Pm on the positive side, Mp, Mm on the negative side),
 * the one-sided normal pairs (first, second derivative) of the two stencils,
 * limited.  h is the cell size along the direction. */
static void limited_normal_pair(double Uc, double Up, double Um, double Pp, double Pm, double Mp, double Mm, double h,
                                double* d1, double* d2) {
  double a4P = 3.0 * ((Uc + Up) - (Pp + Pm)) / (h * h);
  double ta2P = (Pp + Pm - 2.0 * Uc) / h;
  double a4M = 3.0 * ((Uc + Um) - (Mp + Mm)) / (h * h);
  double ta2M = (Mp + Mm - 2.0 * Uc) / h;
  double a4 = minmod(a4M, a4P);
  *d2 = a4;
  *d1 = minmod(-ta2M + a4 * h / 6.0, ta2P - a4 * h / 6.0);
}

/* Sec. 3.2 after the limiter: the cross derivative of the one-sided stencils
 * with the limited slopes a2, a3, the central stencil S5 and the nonlinear
 * weights.  Output p2..p6. */
static void recon2d_finish(double Uc, double Ue, double Uw, double Un, double Us, double Ep, double Em, double Wp,
                           double Wm, double Np, double Nm, double Sp, double Sm, double h, double k, double eps,
                           double C, double a2, double a3, double a4, double a5, double* p) {
  double s3 = sqrt(3.0);
  /* cross derivative of each one-sided stencil with the limited a2, a3;
   * stencil 1 (NE) as printed, NW / SW / SE by the same least squares */
  double dE = Ep - Em, dW = Wp - Wm, dN = Np - Nm, dS = Sp - Sm;
  double cand[4];
  cand[0] = s3 * (dE + dN) / (h * k) - (a2 / k + a3 / h); /* NE */
  cand[1] = s3 * (dN - dW) / (h * k) - (a2 / k - a3 / h); /* NW */
  cand[2] = -s3 * (dS + dW) / (h * k) + (a2 / k + a3 / h); /* SW */
  cand[3] = s3 * (dE - dS) / (h * k) + (a2 / k - a3 / h); /* SE */
  /* the one with the smallest absolute value.  Reading for ties: the
   * candidates are differences of the Gauss-point values (and of the limited
   * slopes), so a relative perturbation d of those inputs moves each one by at
   * most d * M, M = sqrt(3) (sum of the eight |Gauss values|) / (h k) +
   * |a2| / k + |a3| / h.  Candidates within TIE_REL * M of the smallest
   * magnitude are tied: the rounding of FP64 arithmetic (TIE_REL = 2^-46, 128
   * units of rounding) cannot order them.  When the tied candidates have both
   * signs, a6 = 0 (their mean), so that the mirror image of the data
   * (x -> -x or y -> -y maps the candidates onto their negated set) gives the
   * mirror image of a6. */
  double m = fabs(cand[0]);
  int best = 0;
  for (int s = 1; s < 4; ++s)
    if (fabs(cand[s]) < m) {
      m = fabs(cand[s]);
      best = s;
    }
  double M = s3 * (fabs(Ep) + fabs(Em) + fabs(Wp) + fabs(Wm) + fabs(Np) + fabs(Nm) + fabs(Sp) + fabs(Sm)) / (h * k) +
             fabs(a2) / k + fabs(a3) / h;
  double band = m + TIE_REL * M;
  int pos = 0, neg = 0;
  for (int s = 0; s < 4; ++s)
    if (fabs(cand[s]) <= band) {
      if (cand[s] > 0.0) pos = 1;
      if (cand[s] < 0.0) neg = 1;
    }
  double a6 = (pos && neg) ? 0.0 : cand[best];
  /* central stencil S5 (reading of the garbled passage: x pair from the
   * (i+-1, j) averages, y pair from the (i, j+-1) averages, cross term from
   * the eight interface Gauss-point differences) */
  double c2 = (Ue - Uw) / (2.0 * h);
  double c4 = ((Ue + Uw) - 2.0 * Uc) / (h * h);
  double c3 = (Un - Us) / (2.0 * k);
  double c5 = ((Un + Us) - 2.0 * Uc) / (k * k);
  double c6 = s3 * ((dE - dW) + (dN - dS)) / (2.0 * h * k);
  /* weights (reading: I = sum_{|alpha|=1,2} |K|^(|alpha|-1) int (D^alpha U)^2,
   * I(U1) = C |K|) */
  double A = h * k;
  double I1 = C * A;
  double I2 = A * (c2 * c2 + c3 * c3) +
              A * (c4 * c4 * (h * h / 12.0 + A) + c5 * c5 * (k * k / 12.0 + A) + c6 * c6 * ((h * h + k * k) / 12.0 + A));
  double al1 = 1.0 / ((eps + I1) * (eps + I1));
  double al2 = 1.0 / ((eps + I2) * (eps + I2));
  double w1 = al1 / (al1 + al2), w2 = al2 / (al1 + al2);
  p[0] = w1 * a2 + w2 * c2;
  p[1] = w1 * a3 + w2 * c3;
  p[2] = w1 * a4 + w2 * c4;
  p[3] = w1 * a5 + w2 * c5;
  p[4] = w1 * a6 + w2 * c6;
}

/* Sec. 3.2.  E+-, W+-: x-interface values at y_j +- sqrt(3)/6 k; N+-, S+-:
 * y-interface values at x_i +- sqrt(3)/6 h.  Output p2..p6. */
void orc_recon2d_scalar(double Uc, double Ue, double Uw, double Un, double Us, double Ep, double Em, double Wp,
                        double Wm, double Np, double Nm, double Sp, double Sm, double h, double k, double eps, double C,
                        double* p) {
  /* eq. over-sys and the limiter on the normal (a2, a4) and tangential
   * (a3, a5) pairs */
  double a2, a3, a4, a5;
  limited_normal_pair(Uc, Ue, Uw, Ep, Em, Wp, Wm, h, &a2, &a4);
  limited_normal_pair(Uc, Un, Us, Np, Nm, Sp, Sm, k, &a3, &a5);
  recon2d_finish(Uc, Ue, Uw, Un, Us, Ep, Em, Wp, Wm, Np, Nm, Sp, Sm, h, k, eps, C, a2, a3, a4, a5, p);
}

/* Right eigenvectors of the 2D Euler flux Jacobian along axis ax (0: x,
 * 1: y) at the conservative state W, as columns: waves un - c, un (entropy),
 * un (shear: the tangential velocity), un + c, with un, ut the normal and
 * tangential velocities.  Returns -1 for a nonphysical state. */
int orc_euler_eigvec_2d(double gamma, const double* W, int ax, double* Rout /* [4][4] */) {
  double rho = W[0];
  if (!(rho > 0.0)) return -1;
  double u = W[1] / rho, v = W[2] / rho, q = 0.5 * (u * u + v * v);
  double p = (gamma - 1.0) * (W[3] - rho * q);
  if (!(p > 0.0)) return -1;
  double c = sqrt(gamma * p / rho), H = (W[3] + p) / rho;
  double un = ax == 0 ? u : v;
  /* unit normal (nx, ny) and the tangential direction (-ny, nx) */
  double nx = ax == 0 ? 1.0 : 0.0, ny = ax == 0 ? 0.0 : 1.0, ut = -ny * u + nx * v;
  double col[4][4] = {{1.0, u - c * nx, v - c * ny, H - un * c},
                      {1.0, u, v, q},
                      {0.0, -ny, nx, ut},
                      {1.0, u + c * nx, v + c * ny, H + un * c}};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) Rout[i * 4 + j] = col[j][i];
  return 0;
}

/* inverse of a 4x4 matrix by Gaussian elimination, column by column */
static int invert4(const double* A /* [4][4] */, double* B /* [4][4] */) {
  for (int c = 0; c < 4; ++c) {
    double M[4][4], e[4] = {0, 0, 0, 0}, x[4];
    e[c] = 1.0;
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) M[i][j] = A[i * 4 + j];
    if (gauss_solve(4, M, e, x)) return -1;
    for (int i = 0; i < 4; ++i) B[i * 4 + c] = x[i];
  }
  return 0;
}

/* Sec. 3.2 on one 2D cell, all four components.  S[s][v]: the thirteen
 * stencil values in the order of orc_recon2d_scalar's arguments (Uc, Ue, Uw,
 * Un, Us, E+, E-, W+, W-, N+, N-, S+, S-) for conservative component v.
 * vars = 0: every component reconstructed on its own.  vars = 1 (reading of
 * the remark on characteristic variables in Sec. 4, carried to 2D): the
 * limiter of each direction acts in the characteristic variables of that
 * direction's flux Jacobian at the cell average -- the x-stencil data (Uc,
 * Ue, Uw, E+-, W+-) are multiplied by L_x = R_x^-1, the normal pair of each
 * field is formed and limited as for a scalar, and the limited (a2, a4) are
 * multiplied back by R_x; the y pair (a3, a5) likewise with R_y.  The cross
 * derivative, the central stencil and the weights stay in conservative
 * variables.  A nonphysical average gives the constant polynomial (p = 0).
 * Returns -1 in that case, else 0. */
int orc_recon2d_cell(int vars, double gamma, const double* S /* [13][4] */, double h, double k, double eps, double C,
                     double* pc /* [4][5] */) {
#define SV(s, v) S[(s) * 4 + (v)]
  double a[4][4]; /* a2, a3, a4, a5 of each conservative component */
  if (vars == 0) {
    for (int v = 0; v < 4; ++v) {
      limited_normal_pair(SV(0, v), SV(1, v), SV(2, v), SV(5, v), SV(6, v), SV(7, v), SV(8, v), h, &a[v][0], &a[v][2]);
      limited_normal_pair(SV(0, v), SV(3, v), SV(4, v), SV(9, v), SV(10, v), SV(11, v), SV(12, v), k, &a[v][1],
                          &a[v][3]);
    }
  } else {
    const double Wc[4] = {SV(0, 0), SV(0, 1), SV(0, 2), SV(0, 3)};
    /* x: stencil entries 0, 1, 2, 5..8; y: 0, 3, 4, 9..12 */
    const int ent[2][7] = {{0, 1, 2, 5, 6, 7, 8}, {0, 3, 4, 9, 10, 11, 12}};
    for (int ax = 0; ax < 2; ++ax) {
      double R[16], L[16];
      if (orc_euler_eigvec_2d(gamma, Wc, ax, R) || invert4(R, L)) {
        for (int v = 0; v < 4; ++v)
          for (int m = 0; m < 5; ++m) pc[v * 5 + m] = 0.0;
        return -1;
      }
      double ch[7][4];
      for (int e = 0; e < 7; ++e)
        for (int r = 0; r < 4; ++r) {
          ch[e][r] = 0.0;
          for (int v = 0; v < 4; ++v) ch[e][r] += L[r * 4 + v] * SV(ent[ax][e], v);
        }
      double d1[4], d2[4];
      for (int r = 0; r < 4; ++r)
        limited_normal_pair(ch[0][r], ch[1][r], ch[2][r], ch[3][r], ch[4][r], ch[5][r], ch[6][r], ax == 0 ? h : k,
                            &d1[r], &d2[r]);
      for (int v = 0; v < 4; ++v) {
        double s1 = 0.0, s2 = 0.0;
        for (int r = 0; r < 4; ++r) {
          s1 += R[v * 4 + r] * d1[r];
          s2 += R[v * 4 + r] * d2[r];
        }
        a[v][ax] = s1;
        a[v][2 + ax] = s2;
      }
    }
  }
  for (int v = 0; v < 4; ++v)
    recon2d_finish(SV(0, v), SV(1, v), SV(2, v), SV(3, v), SV(4, v), SV(5, v), SV(6, v), SV(7, v), SV(8, v), SV(9, v),
                   SV(10, v), SV(11, v), SV(12, v), h, k, eps, C, a[v][0], a[v][1], a[v][2], a[v][3], pc + v * 5);
#undef SV
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Whole-grid step                                                           */
/* ------------------------------------------------------------------------ */

static void prim_to_cons(int dim, double gamma, const double* q, double* W) {
  /* q = (rho, u, v, p) */
  double rho = q[0], u = q[1], v = dim == 2 ? q[2] : 0.0, p = q[3];
  W[0] = rho;
  W[1] = rho * u;
  if (dim == 2) {
    W[2] = rho * v;
    W[3] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v);
  } else {
    W[2] = p / (gamma - 1.0) + 0.5 * rho * u * u;
  }
}

/* point of boundary `side` of a curvilinear grid at logical coordinate s
 * along it (s = i or j of the vertices; linear along the straight edges,
 * extended linearly beyond the end vertices) */
static void wall_point(const orc_problem* P, int side, double s, double* x, double* y) {
  int along_j = side < 2, n = along_j ? P->ny : P->nx;
  int e = (int)floor(s);
  if (e < 0) e = 0;
  if (e > n - 1) e = n - 1;
  double f = s - e;
  int fix = side == 0 ? 0 : side == 1 ? P->nx : side == 2 ? 0 : P->ny;
  for (int c = 0; c < 2; ++c) {
    double a, b;
    if (along_j) {
      a = P->mesh[((size_t)e * (P->nx + 1) + fix) * 2 + c];
      b = P->mesh[((size_t)(e + 1) * (P->nx + 1) + fix) * 2 + c];
    } else {
      a = P->mesh[((size_t)fix * (P->nx + 1) + e) * 2 + c];
      b = P->mesh[((size_t)fix * (P->nx + 1) + e + 1) * 2 + c];
    }
    double v = a + f * (b - a);
    if (c == 0)
      *x = v;
    else
      *y = v;
  }
}

/* image of a mirrored state across a boundary whose normal is `axis`; s:
 * logical position along the boundary (curvilinear grids with a turning
 * wall: the wall velocity there) */
static void mirror_state(const orc_problem* P, int side, int kind, const double* Ws, double* Wg, double s) {
  int dim = P->dim, nv = dim + 2, axis = side / 2;
  double gamma = P->gamma;
  for (int i = 0; i < nv; ++i) Wg[i] = Ws[i];
  if (kind == ORC_BC_OUTFLOW) return;
  if (kind == ORC_BC_REFLECT || kind == ORC_BC_DMR_BOTTOM) {
    Wg[1 + axis] = -Ws[1 + axis];
    return;
  }
  if (kind == ORC_BC_NOSLIP_ISO || kind == ORC_BC_NOSLIP_ADIA) {
    double rho = Ws[0], u = Ws[1] / rho, v = dim == 2 ? Ws[2] / rho : 0.0;
    double p = pressure(dim, gamma, Ws), T = p / rho;
    double uw = P->bc_wall[side][0], vw = P->bc_wall[side][1], Tw = P->bc_wall[side][2];
    if (P->mesh && P->bc_omega[side] != 0.0) {
      double xw, yw;
      wall_point(P, side, s, &xw, &yw);
      uw -= P->bc_omega[side] * yw;
      vw += P->bc_omega[side] * xw;
    }
    double Tg = kind == ORC_BC_NOSLIP_ISO ? 2.0 * Tw - T : T;
    double q[4] = {rho, 2.0 * uw - u, 2.0 * vw - v, rho * Tg};
    prim_to_cons(dim, gamma, q, Wg);
  }
}

/* fixed state of a boundary at location (x, y), or 0 if the boundary
 * mirrors there */
static int fixed_state(const orc_problem* P, int side, int kind, double x, double y, double t, double* W) {
  double q[4];
  if (kind == ORC_BC_INFLOW) {
    memcpy(q, P->bc_state[side], sizeof(q));
  } else if (kind == ORC_BC_DMR_BOTTOM) {
    if (!(x < 1.0 / 6.0)) return 0;
    memcpy(q, P->bc_state[side], sizeof(q)); /* post-shock state */
  } else if (kind == ORC_BC_DMR_TOP) {
    /* the Mach-10 shock crosses height y at x = 1/6 + (y + 20 t)/sqrt(3):
     * post-shock state behind it, pre-shock state ahead */
    double xs = 1.0 / 6.0 + (y + 20.0 * t) / sqrt(3.0);
    if (x < xs)
      memcpy(q, P->bc_state[side], sizeof(q));
    else
      memcpy(q, P->bc_alt[side], sizeof(q));
  } else {
    return 0;
  }
  prim_to_cons(P->dim, P->gamma, q, W);
  return 1;
}

typedef struct {
  int nx, ny, nv;
  double *W, *FX, *FY, *PC; /* ghosted cells, x faces, y faces, reconstruction */
} grid2;

#define GW(G, v, j, i) (G)->W[((size_t)(v) * ((G)->ny + 4) + (size_t)((j) + 2)) * ((G)->nx + 4) + (size_t)((i) + 2)]
#define GFX(G, g, v, j, fi) \
  (G)->FX[(((size_t)(g) * (G)->nv + (v)) * ((G)->ny + 2) + (size_t)((j) + 1)) * ((G)->nx + 3) + (size_t)((fi) + 1)]
#define GFY(G, g, v, fj, i) \
  (G)->FY[(((size_t)(g) * (G)->nv + (v)) * ((G)->ny + 3) + (size_t)((fj) + 1)) * ((G)->nx + 2) + (size_t)((i) + 1)]
#define GPC(G, v, m, j, i) \
  (G)->PC[(((size_t)(v) * 5 + (m)) * ((G)->ny + 2) + (size_t)((j) + 1)) * ((G)->nx + 2) + (size_t)((i) + 1)]

static void get_cell(grid2* G, int j, int i, double* W) {
  for (int v = 0; v < G->nv; ++v) W[v] = GW(G, v, j, i);
}
static void set_cell(grid2* G, int j, int i, const double* W) {
  for (int v = 0; v < G->nv; ++v) GW(G, v, j, i) = W[v];
}

/* ghost cells (two layers, corners included) and ghost interface values */
static void fill_ghosts_2d(const orc_problem* P, grid2* G, double t) {
  int nx = G->nx, ny = G->ny, nv = G->nv;
  double h = (P->x1 - P->x0) / nx, k = (P->y1 - P->y0) / ny, dl = sqrt(3.0) / 6.0;
  double Ws[4], Wg[4];
  /* west / east, rows 0..ny-1 */
  for (int side = 0; side < 2; ++side) {
    int kind = P->bc_kind[side];
    for (int j = 0; j < ny; ++j) {
      double yc = P->y0 + (j + 0.5) * k;
      for (int m = 0; m < 2; ++m) {
        int ig = side == 0 ? -1 - m : nx + m;
        int is = kind == ORC_BC_PERIODIC ? (side == 0 ? ig + nx : ig - nx) : (side == 0 ? -1 - ig : 2 * nx - 1 - ig);
        double xc = P->x0 + (ig + 0.5) * h;
        if (fixed_state(P, side, kind, xc, yc, t, Wg)) {
        } else {
          get_cell(G, j, is, Ws);
          if (kind == ORC_BC_PERIODIC)
            memcpy(Wg, Ws, sizeof(Ws));
          else
            mirror_state(P, side, kind, Ws, Wg, j + 0.5);
        }
        set_cell(G, j, ig, Wg);
      }
      /* ghost x interface fi = -1 / nx+1 */
      int fg = side == 0 ? -1 : nx + 1;
      int fs = kind == ORC_BC_PERIODIC ? (side == 0 ? nx - 1 : 1) : (side == 0 ? 1 : nx - 1);
      for (int g = 0; g < 2; ++g) {
        double yg = yc + (g == 0 ? -dl : dl) * k, xg = P->x0 + fg * h;
        if (!fixed_state(P, side, kind, xg, yg, t, Wg)) {
          for (int v = 0; v < nv; ++v) Ws[v] = GFX(G, g, v, j, fs);
          if (kind == ORC_BC_PERIODIC)
            memcpy(Wg, Ws, sizeof(Ws));
          else
            mirror_state(P, side, kind, Ws, Wg, j + 0.5 + (g == 0 ? -dl : dl));
        }
        for (int v = 0; v < nv; ++v) GFX(G, g, v, j, fg) = Wg[v];
      }
    }
    /* y interfaces of the ghost column i = -1 / nx, fj = 0..ny */
    int ig = side == 0 ? -1 : nx;
    int is = kind == ORC_BC_PERIODIC ? (side == 0 ? nx - 1 : 0) : (side == 0 ? 0 : nx - 1);
    for (int fj = 0; fj <= ny; ++fj)
      for (int g = 0; g < 2; ++g) {
        double xg = P->x0 + (ig + 0.5 + (g == 0 ? -dl : dl)) * h, yg = P->y0 + fj * k;
        if (!fixed_state(P, side, kind, xg, yg, t, Wg)) {
          int gs = kind == ORC_BC_PERIODIC ? g : 1 - g; /* mirror flips the tangential Gauss points */
          for (int v = 0; v < nv; ++v) Ws[v] = GFY(G, gs, v, fj, is);
          if (kind == ORC_BC_PERIODIC)
            memcpy(Wg, Ws, sizeof(Ws));
          else
            mirror_state(P, side, kind, Ws, Wg, (double)fj);
        }
        for (int v = 0; v < nv; ++v) GFY(G, g, v, fj, ig) = Wg[v];
      }
  }
  /* south / north, columns -2..nx+1 (corners from the west/east ghosts) */
  for (int side = 2; side < 4; ++side) {
    int kind = P->bc_kind[side];
    for (int i = -2; i < nx + 2; ++i) {
      double xc = P->x0 + (i + 0.5) * h;
      for (int m = 0; m < 2; ++m) {
        int jg = side == 2 ? -1 - m : ny + m;
        int js = kind == ORC_BC_PERIODIC ? (side == 2 ? jg + ny : jg - ny) : (side == 2 ? -1 - jg : 2 * ny - 1 - jg);
        double yc = P->y0 + (jg + 0.5) * k;
        if (!fixed_state(P, side, kind, xc, yc, t, Wg)) {
          get_cell(G, js, i, Ws);
          if (kind == ORC_BC_PERIODIC)
            memcpy(Wg, Ws, sizeof(Ws));
          else
            mirror_state(P, side, kind, Ws, Wg, i + 0.5);
        }
        set_cell(G, jg, i, Wg);
      }
    }
    /* ghost y interface fj = -1 / ny+1, columns 0..nx-1 */
    int fg = side == 2 ? -1 : ny + 1;
    int fs = kind == ORC_BC_PERIODIC ? (side == 2 ? ny - 1 : 1) : (side == 2 ? 1 : ny - 1);
    for (int i = 0; i < nx; ++i)
      for (int g = 0; g < 2; ++g) {
        double xg = P->x0 + (i + 0.5 + (g == 0 ? -dl : dl)) * h, yg = P->y0 + fg * k;
        if (!fixed_state(P, side, kind, xg, yg, t, Wg)) {
          for (int v = 0; v < nv; ++v) Ws[v] = GFY(G, g, v, fs, i);
          if (kind == ORC_BC_PERIODIC)
            memcpy(Wg, Ws, sizeof(Ws));
          else
            mirror_state(P, side, kind, Ws, Wg, i + 0.5 + (g == 0 ? -dl : dl));
        }
        for (int v = 0; v < nv; ++v) GFY(G, g, v, fg, i) = Wg[v];
      }
    /* x interfaces of the ghost row j = -1 / ny, fi = 0..nx */
    int jg = side == 2 ? -1 : ny;
    int js = kind == ORC_BC_PERIODIC ? (side == 2 ? ny - 1 : 0) : (side == 2 ? 0 : ny - 1);
    for (int fi = 0; fi <= nx; ++fi)
      for (int g = 0; g < 2; ++g) {
        double xg = P->x0 + fi * h, yg = P->y0 + (jg + 0.5 + (g == 0 ? -dl : dl)) * k;
        if (!fixed_state(P, side, kind, xg, yg, t, Wg)) {
          int gs = kind == ORC_BC_PERIODIC ? g : 1 - g;
          for (int v = 0; v < nv; ++v) Ws[v] = GFX(G, gs, v, js, fi);
          if (kind == ORC_BC_PERIODIC)
            memcpy(Wg, Ws, sizeof(Ws));
          else
            mirror_state(P, side, kind, Ws, Wg, (double)fi);
        }
        for (int v = 0; v < nv; ++v) GFX(G, g, v, jg, fi) = Wg[v];
      }
  }
}

/* Reading (robustness at strong shocks, not printed; the paper names robust
 * reconstruction an open question at the end of Sec. 3.3).  The literal
 * scheme needs a positive density and pressure at the centre of every
 * interface of a cell (the interface Maxwellians of Sec. 2.2 exist only
 * then); mode 0 asks only that.  Mode 1 also asks that they lie within a
 * factor two of the range of the averages of the cell and its face
 * neighbours:
 *   rho_min / 2 <= rho <= 2 rho_max,  p_min / 2 <= p <= 2 p_max.
 * A cell that fails is reconstructed as its constant average for this step.
 * lo/hi: the neighbourhood's range of rho (index 0) and p (index 1). */
static int admissible(int dim, double gamma, int mode, const double* W, const double* lo, const double* hi) {
  double p = pressure(dim, gamma, W);
  if (!(W[0] > 0.0) || !(p > 0.0)) return 0;
  if (mode == 0) return 1;
  if (W[0] < 0.5 * lo[0] || W[0] > 2.0 * hi[0]) return 0;
  if (p < 0.5 * lo[1] || p > 2.0 * hi[1]) return 0;
  return 1;
}

static void range_add(int dim, double gamma, const double* W, double* lo, double* hi) {
  double q[2] = {W[0], pressure(dim, gamma, W)};
  for (int a = 0; a < 2; ++a) {
    if (q[a] < lo[a]) lo[a] = q[a];
    if (q[a] > hi[a]) hi[a] = q[a];
  }
}

/* reconstruction of cell (i, j), all components, with the admissibility
 * reading above; returns 1 when the cell fell back to its average */
static int recon_cell_2d(const orc_problem* P, grid2* G, int j, int i, double h, double k, double Cw) {
  double S[13][4], pc[4][5];
  for (int v = 0; v < G->nv; ++v) {
    S[0][v] = GW(G, v, j, i);
    S[1][v] = GW(G, v, j, i + 1);
    S[2][v] = GW(G, v, j, i - 1);
    S[3][v] = GW(G, v, j + 1, i);
    S[4][v] = GW(G, v, j - 1, i);
    S[5][v] = GFX(G, 1, v, j, i + 1);
    S[6][v] = GFX(G, 0, v, j, i + 1);
    S[7][v] = GFX(G, 1, v, j, i);
    S[8][v] = GFX(G, 0, v, j, i);
    S[9][v] = GFY(G, 1, v, j + 1, i);
    S[10][v] = GFY(G, 0, v, j + 1, i);
    S[11][v] = GFY(G, 1, v, j, i);
    S[12][v] = GFY(G, 0, v, j, i);
  }
  /* a nonphysical average (characteristic variables) leaves p = 0; the
   * interfaces of the cell report it */
  (void)orc_recon2d_cell(P->recon_vars, P->gamma, &S[0][0], h, k, P->weno_eps, Cw, &pc[0][0]);
  /* range of the averages of the cell and its four face neighbours */
  double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
  const int nb[5][2] = {{0, 0}, {0, 1}, {0, -1}, {1, 0}, {-1, 0}};
  for (int q = 0; q < 5; ++q) {
    double Wq[4];
    get_cell(G, j + nb[q][0], i + nb[q][1], Wq);
    range_add(2, P->gamma, Wq, lo, hi);
  }
  int ok = 1;
  for (int f = 0; f < 4; ++f) {
    /* interface centres: x = +-h/2 (y = 0), y = +-k/2 (x = 0) */
    double x = f == 0 ? 0.5 * h : f == 1 ? -0.5 * h : 0.0;
    double y = f == 2 ? 0.5 * k : f == 3 ? -0.5 * k : 0.0;
    double W[4];
    for (int v = 0; v < 4; ++v)
      W[v] = GW(G, v, j, i) + pc[v][0] * x + pc[v][1] * y + pc[v][2] * 0.5 * (x * x - h * h / 12.0) +
             pc[v][3] * 0.5 * (y * y - k * k / 12.0) + pc[v][4] * x * y;
    if (!admissible(2, P->gamma, P->admissibility, W, lo, hi)) ok = 0;
  }
  for (int v = 0; v < G->nv; ++v)
    for (int m = 0; m < 5; ++m) GPC(G, v, m, j, i) = ok ? pc[v][m] : 0.0;
  return !ok;
}

/* interface values of a cell polynomial on the side facing the interface
 * (a3): normal axis ax (0 = x, 1 = y), sgn = +1 for the interface on the
 * positive side of the cell.  hn, hs: normal and tangential cell sizes. */
static void side_values(double Ub, const double* p, int ax, double sgn, double hn, double hs, double* W, double* Wn,
                        double* Ws, double* Wnn, double* Wns, double* Wss) {
  double pn = ax == 0 ? p[0] : p[1], ps = ax == 0 ? p[1] : p[0];
  double pnn = ax == 0 ? p[2] : p[3], pss = ax == 0 ? p[3] : p[2], pns = p[4];
  double xn = 0.5 * sgn * hn;
  /* U = Ubar + pn xn + pnn w_n(xn) + pss w_s(0) with w(x) = (x^2 - h^2/12)/2 */
  *W = Ub + pn * xn + pnn * 0.5 * (xn * xn - hn * hn / 12.0) + pss * 0.5 * (0.0 - hs * hs / 12.0);
  *Wn = pn + pnn * xn;
  *Ws = ps + pns * xn;
  *Wnn = pnn;
  *Wns = pns;
  *Wss = pss;
}

/* ---- 2D solid step (Sec. 4.6) ---------------------------------------- */

/* cell (i, j) lies inside the solid step {i >= i0, j < nj} (ghost indices
 * included) */
static int solid(const orc_problem* P, int i, int j) {
  return P->obst_nj > 0 && i >= P->obst_i0 && j < P->obst_nj;
}

/* Reading (Sec. 4.6: reflective walls of the step): at an interface
 * between a gas cell and a solid cell, the solid side is the mirror image
 * of the gas side across that interface.  In the interface frame (component
 * 1 the normal momentum, derivatives n along the normal) its interface
 * values are the gas side's with the normal momentum negated and with every
 * odd order in n negated, and its row of the equilibrium stencil is the
 * image of the gas row.  The mirror makes the interface pass no mass.  The
 * layers of solid images (fill_obstacle_2d) still serve the reconstruction
 * of the gas cells; they cannot do this at the corner, where one solid cell
 * would have to be the image across two faces: with the solid cells' own
 * polynomials there, mass passes through the step's walls next to the
 * corner and the cell above the corner empties (240 x 80 and 360 x 120 cells
 * of the Mach 3 flow, before t = 2). */
static void wall_mirror(orc_face_input* in, int s, int nv) {
  int g = 1 - s;
  for (int v = 0; v < nv; ++v) {
    double sg = v == 1 ? -1.0 : 1.0;
    in->W[s][v] = sg * in->W[g][v];
    in->Wn[s][v] = -sg * in->Wn[g][v];
    in->Ws[s][v] = sg * in->Ws[g][v];
    in->Wnn[s][v] = sg * in->Wnn[g][v];
    in->Wns[s][v] = -sg * in->Wns[g][v];
    in->Wss[s][v] = sg * in->Wss[g][v];
    for (int n = 0; n < 3; ++n) in->Ueq[s][n][v] = sg * in->Ueq[g][n][v];
  }
}

/* negate the momentum along x (ax = 0) and/or y (ax = 1) */
static void flip(const double* Ws, int fu, int fv, double* Wg) {
  for (int v = 0; v < 4; ++v) Wg[v] = Ws[v];
  if (fu) Wg[1] = -Ws[1];
  if (fv) Wg[2] = -Ws[2];
}

/* Reading (the paper defers the corner to an external reference): the two
 * layers of solid cells along the step's faces are slip-wall images of the
 * gas, for the reconstruction of the gas cells next to the step (the
 * interfaces on the step's faces take the face-wise image of wall_mirror
 * instead): below the top face the image across it (v negated), and beside
 * the vertical face, below those two rows, the image across that face (u
 * negated).  The 2 x 2 block at the corner thus takes the image across the
 * top face.  (Its image through the corner point lets the expansion round
 * the corner empty the cells above the step: the Mach 3 flow of Sec. 4.6
 * leaves the physical states by t = 0.25 on 60 x 20 cells.)  The
 * Gauss-point values on the interfaces between those solid cells are imaged
 * the same way (a mirror swaps the Gauss points along it), and so are the
 * few boundary images next to the step that the first solid layer reads:
 * the south images below the vertical face's solid columns and the east
 * images of the top face's solid rows, each the boundary's own image of the
 * solid cell's.  Filled after the boundary images of the domain edges. */
static void fill_obstacle_2d(const orc_problem* P, grid2* G) {
  if (P->obst_nj <= 0) return;
  int nx = G->nx, i0 = P->obst_i0, nj = P->obst_nj;
  double Ws[4], Wg[4], Wm[4];
  /* cells: the two rows below the top face, then the two columns beside
   * the vertical face below them */
  for (int dy = 0; dy < 2; ++dy)
    for (int i = i0; i < nx; ++i) {
      get_cell(G, nj + dy, i, Ws);
      flip(Ws, 0, 1, Wg);
      set_cell(G, nj - 1 - dy, i, Wg);
    }
  for (int dx = 0; dx < 2; ++dx)
    for (int j = 0; j < nj - 2; ++j) {
      get_cell(G, j, i0 - 1 - dx, Ws);
      flip(Ws, 1, 0, Wg);
      set_cell(G, j, i0 + dx, Wg);
    }
  /* the south boundary's images of the vertical face's solid columns, the
   * east boundary's images of the top face's solid rows */
  for (int dx = 0; dx < 2; ++dx)
    for (int m = 0; m < 2; ++m) {
      get_cell(G, m, i0 - 1 - dx, Ws);
      flip(Ws, 1, 0, Wm);
      mirror_state(P, 2, P->bc_kind[2], Wm, Wg, 0.0);
      set_cell(G, -1 - m, i0 + dx, Wg);
    }
  for (int m = 0; m < 2; ++m)
    for (int dy = 0; dy < 2; ++dy) {
      get_cell(G, nj + dy, nx - 1 - m, Ws);
      flip(Ws, 0, 1, Wm);
      mirror_state(P, 1, P->bc_kind[1], Wm, Wg, 0.0);
      set_cell(G, nj - 1 - dy, nx + m, Wg);
    }
  /* x interfaces: fi = i0+1..nx in the two rows below the top face, fi =
   * i0 + 1 beside the vertical face below them */
  for (int dy = 0; dy < 2; ++dy)
    for (int fi = i0 + 1; fi <= nx; ++fi)
      for (int g = 0; g < 2; ++g) {
        for (int v = 0; v < 4; ++v) Ws[v] = GFX(G, 1 - g, v, nj + dy, fi);
        flip(Ws, 0, 1, Wg);
        for (int v = 0; v < 4; ++v) GFX(G, g, v, nj - 1 - dy, fi) = Wg[v];
      }
  for (int j = 0; j < nj - 2; ++j)
    for (int g = 0; g < 2; ++g) {
      for (int v = 0; v < 4; ++v) Ws[v] = GFX(G, g, v, j, i0 - 1);
      flip(Ws, 1, 0, Wg);
      for (int v = 0; v < 4; ++v) GFX(G, g, v, j, i0 + 1) = Wg[v];
    }
  /* y interfaces: fj = nj - 1 (columns i0..nx-1), column i0 (fj = 0..nj-2) */
  for (int i = i0; i < nx; ++i)
    for (int g = 0; g < 2; ++g) {
      for (int v = 0; v < 4; ++v) Ws[v] = GFY(G, g, v, nj + 1, i);
      flip(Ws, 0, 1, Wg);
      for (int v = 0; v < 4; ++v) GFY(G, g, v, nj - 1, i) = Wg[v];
    }
  for (int fj = 0; fj <= nj - 2; ++fj)
    for (int g = 0; g < 2; ++g) {
      for (int v = 0; v < 4; ++v) Ws[v] = GFY(G, 1 - g, v, fj, i0 - 1);
      flip(Ws, 1, 0, Wg);
      for (int v = 0; v < 4; ++v) GFY(G, g, v, fj, i0) = Wg[v];
    }
}

/* interior cells whose reconstruction fell back to the average in the last step */
/* ---- 2D curvilinear grids ----------------------------------------------
 * Reading (the remark closing Sec. 3.3 calls the compact reconstruction easy
 * to extend to other meshes and gives no formulas; Sec. 4.8 runs a polar
 * cavity).  Cells are the straight-edged quadrilaterals of the vertex grid.
 *   - Reconstruction: Sec. 3.2 verbatim in the logical coordinates (xi, eta)
 *     of the grid (unit spacing), from the cell averages and the interface
 *     Gauss-point values; the weight constant I(U1) = C |K| takes the cell's
 *     area, so that both indicators keep their physical scale.
 *   - Interface: straight edge of length L, unit tangent t along the edge
 *     (towards increasing eta on xi-interfaces, increasing xi on
 *     eta-interfaces), unit normal n from side 0 to side 1; Gauss points at
 *     the centre +- (sqrt(3)/6) L t.  Logical derivatives become interface
 *     derivatives through the metric at the interface centre: the logical
 *     normal step is the vector e between the two cell centres (the mean of
 *     each cell's corners; across a wall, the mirror image of the inside
 *     centre; across a periodic seam, the partner translated by the period),
 *     the logical tangential step is the edge L t, so
 *       d/dxi = (e.n) d/dn + (e.t) d/dt,  d/deta = L d/dt,
 *     whose inverse G gives first and (second-order terms of the map
 *     dropped) second derivatives.  Momentum is rotated to (n, t).
 *   - Flux and point values: Sec. 2.2 in that frame with the interface
 *     extent L; update eq. finite with the cell areas.
 *   - Time step: Sec. 4's CFL condition with the widths |K| / (mean length
 *     of the two opposite edges) across each logical direction and the
 *     speed |u|.
 * The map's own curvature is not carried into the second derivatives, so
 * the scheme is third order on affine grids (constant metric) and of lower
 * order where the grid curves. */
typedef struct {
  double *cx, *cy, *area, *h1, *h2; /* [ny][nx] */
  double *fx, *fy;                  /* x faces [ny][nx+1][7], y faces [ny+1][nx][7]: n, t, L, G_nn, G_ns */
} cgeom;

#define MV(P, j, i, c) (P)->mesh[((size_t)(j) * ((P)->nx + 1) + (size_t)(i)) * 2 + (c)]

static void cgeom_free(cgeom* g) {
  free(g->cx);
  free(g->cy);
  free(g->area);
  free(g->h1);
  free(g->h2);
  free(g->fx);
  free(g->fy);
}

/* centre of the cell on side `side` of a boundary face beyond the grid:
 * the periodic partner translated by the period, or the mirror image of the
 * inside centre (ix, iy) across the face line through (px, py) with normal n */
static void ghost_centre(const orc_problem* P, const cgeom* g, int axis, int high, int part_i, int part_j, double ix,
                         double iy, double px, double py, const double* n, double* ox, double* oy) {
  int nx = P->nx, ny = P->ny;
  if (P->bc_kind[axis * 2 + high] == ORC_BC_PERIODIC) {
    double sx = axis == 0 ? MV(P, 0, nx, 0) - MV(P, 0, 0, 0) : MV(P, ny, 0, 0) - MV(P, 0, 0, 0);
    double sy = axis == 0 ? MV(P, 0, nx, 1) - MV(P, 0, 0, 1) : MV(P, ny, 0, 1) - MV(P, 0, 0, 1);
    double sg = high ? 1.0 : -1.0;
    *ox = g->cx[(size_t)part_j * nx + part_i] + sg * sx;
    *oy = g->cy[(size_t)part_j * nx + part_i] + sg * sy;
  } else {
    double d = (ix - px) * n[0] + (iy - py) * n[1];
    *ox = ix - 2.0 * d * n[0];
    *oy = iy - 2.0 * d * n[1];
  }
}

/* frame and metric of one face from its edge (a -> b) and the centres of
 * its side cells (c0 -> c1); xface: n is t turned clockwise, else
 * anticlockwise */
static void face_frame(double ax, double ay, double bx, double by, int xface, double* fr) {
  double ex = bx - ax, ey = by - ay, L = sqrt(ex * ex + ey * ey);
  double tx = ex / L, ty = ey / L;
  fr[0] = xface ? ty : -ty;
  fr[1] = xface ? -tx : tx;
  fr[2] = tx;
  fr[3] = ty;
  fr[4] = L;
}

static void face_metric(double* fr, double c0x, double c0y, double c1x, double c1y) {
  /* Jacobian of (xi, eta) -> (n, t) coordinates: rows d/dxi, d/deta */
  double ex = c1x - c0x, ey = c1y - c0y, L = fr[4];
  double J[2][2] = {{ex * fr[0] + ey * fr[1], ex * fr[2] + ey * fr[3]}, {0.0, L}};
  double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  /* (d/dn, d/dt) = J^-1 (d/dxi, d/deta) */
  fr[5] = J[1][1] / det;
  fr[6] = -J[0][1] / det;
}

static void cgeom_build(const orc_problem* P, cgeom* g) {
  int nx = P->nx, ny = P->ny;
  size_t nc = (size_t)nx * ny;
  g->cx = malloc(nc * sizeof(double));
  g->cy = malloc(nc * sizeof(double));
  g->area = malloc(nc * sizeof(double));
  g->h1 = malloc(nc * sizeof(double));
  g->h2 = malloc(nc * sizeof(double));
  g->fx = malloc((size_t)ny * (nx + 1) * 7 * sizeof(double));
  g->fy = malloc((size_t)(ny + 1) * nx * 7 * sizeof(double));
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double x[4] = {MV(P, j, i, 0), MV(P, j, i + 1, 0), MV(P, j + 1, i + 1, 0), MV(P, j + 1, i, 0)};
      double y[4] = {MV(P, j, i, 1), MV(P, j, i + 1, 1), MV(P, j + 1, i + 1, 1), MV(P, j + 1, i, 1)};
      size_t c = (size_t)j * nx + i;
      g->cx[c] = 0.25 * (x[0] + x[1] + x[2] + x[3]);
      g->cy[c] = 0.25 * (y[0] + y[1] + y[2] + y[3]);
      /* half the cross product of the diagonals */
      g->area[c] = 0.5 * ((x[2] - x[0]) * (y[3] - y[1]) - (y[2] - y[0]) * (x[3] - x[1]));
    }
  for (int j = 0; j < ny; ++j)
    for (int fi = 0; fi <= nx; ++fi) {
      double* fr = g->fx + ((size_t)j * (nx + 1) + fi) * 7;
      face_frame(MV(P, j, fi, 0), MV(P, j, fi, 1), MV(P, j + 1, fi, 0), MV(P, j + 1, fi, 1), 1, fr);
      double px = 0.5 * (MV(P, j, fi, 0) + MV(P, j + 1, fi, 0)), py = 0.5 * (MV(P, j, fi, 1) + MV(P, j + 1, fi, 1));
      double c0x, c0y, c1x, c1y;
      if (fi > 0) {
        c0x = g->cx[(size_t)j * nx + fi - 1];
        c0y = g->cy[(size_t)j * nx + fi - 1];
      } else {
        ghost_centre(P, g, 0, 0, nx - 1, j, g->cx[(size_t)j * nx], g->cy[(size_t)j * nx], px, py, fr, &c0x, &c0y);
      }
      if (fi < nx) {
        c1x = g->cx[(size_t)j * nx + fi];
        c1y = g->cy[(size_t)j * nx + fi];
      } else {
        ghost_centre(P, g, 0, 1, 0, j, g->cx[(size_t)j * nx + nx - 1], g->cy[(size_t)j * nx + nx - 1], px, py, fr,
                     &c1x, &c1y);
      }
      face_metric(fr, c0x, c0y, c1x, c1y);
    }
  for (int fj = 0; fj <= ny; ++fj)
    for (int i = 0; i < nx; ++i) {
      double* fr = g->fy + ((size_t)fj * nx + i) * 7;
      face_frame(MV(P, fj, i, 0), MV(P, fj, i, 1), MV(P, fj, i + 1, 0), MV(P, fj, i + 1, 1), 0, fr);
      double px = 0.5 * (MV(P, fj, i, 0) + MV(P, fj, i + 1, 0)), py = 0.5 * (MV(P, fj, i, 1) + MV(P, fj, i + 1, 1));
      double c0x, c0y, c1x, c1y;
      if (fj > 0) {
        c0x = g->cx[(size_t)(fj - 1) * nx + i];
        c0y = g->cy[(size_t)(fj - 1) * nx + i];
      } else {
        ghost_centre(P, g, 1, 0, i, ny - 1, g->cx[i], g->cy[i], px, py, fr, &c0x, &c0y);
      }
      if (fj < ny) {
        c1x = g->cx[(size_t)fj * nx + i];
        c1y = g->cy[(size_t)fj * nx + i];
      } else {
        ghost_centre(P, g, 1, 1, i, 0, g->cx[(size_t)(ny - 1) * nx + i], g->cy[(size_t)(ny - 1) * nx + i], px, py, fr,
                     &c1x, &c1y);
      }
      face_metric(fr, c0x, c0y, c1x, c1y);
    }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t c = (size_t)j * nx + i;
      double lw = g->fx[((size_t)j * (nx + 1) + i) * 7 + 4], le = g->fx[((size_t)j * (nx + 1) + i + 1) * 7 + 4];
      double ls = g->fy[((size_t)j * nx + i) * 7 + 4], ln = g->fy[((size_t)(j + 1) * nx + i) * 7 + 4];
      g->h1[c] = g->area[c] / (0.5 * (lw + le));
      g->h2[c] = g->area[c] / (0.5 * (ls + ln));
    }
}

/* area of the cell (i, j) of the reconstruction range (-1..nx, -1..ny, no
 * corners): a ghost cell takes its image's (periodic partner or mirrored
 * inside cell) */
static double cell_area(const orc_problem* P, const cgeom* g, int i, int j) {
  int nx = P->nx, ny = P->ny;
  if (i < 0) i = P->bc_kind[0] == ORC_BC_PERIODIC ? i + nx : -1 - i;
  if (i >= nx) i = P->bc_kind[1] == ORC_BC_PERIODIC ? i - nx : 2 * nx - 1 - i;
  if (j < 0) j = P->bc_kind[2] == ORC_BC_PERIODIC ? j + ny : -1 - j;
  if (j >= ny) j = P->bc_kind[3] == ORC_BC_PERIODIC ? j - ny : 2 * ny - 1 - j;
  return g->area[(size_t)j * nx + i];
}

/* interface-frame data of side s of a face with frame fr: the side cell's
 * average Ub and logical polynomial p (p2..p6 of the cell), normal logical
 * axis ax (0: xi, 1: eta), at the logical normal offset xn (+1/2 for side
 * 0, -1/2 for side 1) */
static void curv_side(orc_face_input* in, int s, const double* fr, int ax, double xn, const double* Ub,
                      const double (*p)[5]) {
  double val[4], d[5][4];
  for (int v = 0; v < 4; ++v) {
    double pn = ax == 0 ? p[v][0] : p[v][1], ps = ax == 0 ? p[v][1] : p[v][0];
    double pnn = ax == 0 ? p[v][2] : p[v][3], pss = ax == 0 ? p[v][3] : p[v][2], pns = p[v][4];
    /* the polynomial Ubar + pn x + ps y + pnn (x^2 - 1/12)/2 + pss (y^2 - 1/12)/2 + pns x y at (xn, 0) */
    val[v] = Ub[v] + pn * xn + 0.5 * pnn * (xn * xn - 1.0 / 12.0) - pss / 24.0;
    double grad[2] = {pn + pnn * xn, ps + pns * xn};
    double hess[2][2] = {{pnn, pns}, {pns, pss}};
    double G[2][2] = {{fr[5], fr[6]}, {0.0, 1.0 / fr[4]}};
    double gf[2], hf[2][2];
    for (int a = 0; a < 2; ++a) {
      gf[a] = G[a][0] * grad[0] + G[a][1] * grad[1];
      for (int b = 0; b < 2; ++b) {
        hf[a][b] = 0.0;
        for (int c = 0; c < 2; ++c)
          for (int e = 0; e < 2; ++e) hf[a][b] += G[a][c] * hess[c][e] * G[b][e];
      }
    }
    d[0][v] = gf[0];
    d[1][v] = gf[1];
    d[2][v] = hf[0][0];
    d[3][v] = hf[0][1];
    d[4][v] = hf[1][1];
  }
  /* momentum to (n, t) */
  double* outs[6] = {in->W[s], in->Wn[s], in->Ws[s], in->Wnn[s], in->Wns[s], in->Wss[s]};
  const double* srcs[6] = {val, d[0], d[1], d[2], d[3], d[4]};
  for (int q = 0; q < 6; ++q) {
    const double* a = srcs[q];
    outs[q][0] = a[0];
    outs[q][1] = fr[0] * a[1] + fr[1] * a[2];
    outs[q][2] = fr[2] * a[1] + fr[3] * a[2];
    outs[q][3] = a[3];
  }
}

static void to_face_frame(const double* fr, const double* W, double* o) {
  o[0] = W[0];
  o[1] = fr[0] * W[1] + fr[1] * W[2];
  o[2] = fr[2] * W[1] + fr[3] * W[2];
  o[3] = W[3];
}

static void from_face_frame(const double* fr, const double* F, double* o) {
  o[0] = F[0];
  o[1] = fr[0] * F[1] + fr[2] * F[2];
  o[2] = fr[1] * F[1] + fr[3] * F[2];
  o[3] = F[3];
}

static long g_last_fallbacks = 0;
/* Readings of the domain-edge walls (Sec. 4.5-4.8 give their walls as slip
 * walls, a symmetry line or no-slip walls, isothermal or adiabatic, and
 * print no wall treatment beyond the ghost images); both act on
 * the interface fluxes and point values of the step, in the grid's
 * components, before the update.
 *
 * A no-slip wall is impermeable.  Its interface passes no mass, and the
 * (spurious) mass flux F_rho of the ghost-image evaluation takes with it the
 * momentum and energy it would carry at the velocity and total enthalpy of
 * the cell beside the wall (its average at the start of the step):
 * F_rho (u_c, v_c, h_c) is removed from the momentum and energy fluxes;
 * pressure, viscous stress and heat flux stay.
 *
 * A slip wall is the symmetry line of its image pair: its interface passes
 * normal momentum only (the mass, tangential momentum and energy fluxes are
 * odd under the mirror) and its new point values carry no normal momentum.
 * The ghost cell is reconstructed from its own stencil, which holds the
 * wall's point values as they are; their odd part, left by rounding, is not
 * mirrored there and can grow from step to step (it doubled each step at
 * one wall interface of the viscous shock tube on 1000 x 500 cells), so it
 * is set to zero where the pair defines it to be.
 *
 * wall_edge: 1 slip, 2 no-slip, 0 neither, for the interface at normal index
 * `index` of axis 0 (x) / 1 (y); `along`: the column of a y interface (the
 * south edge of the double Mach reflection is a slip wall from the cell
 * whose centre lies at x = 1/6 on). */
static int wall_edge(const orc_problem* P, int axis, int index, int along) {
  int n = axis == 0 ? P->nx : P->ny, side = axis * 2 + (index == 0 ? 0 : 1);
  if (index != 0 && index != n) return 0;
  int k = P->bc_kind[side];
  if (k == ORC_BC_NOSLIP_ISO || k == ORC_BC_NOSLIP_ADIA) return 2;
  if (k == ORC_BC_REFLECT) return 1;
  if (k == ORC_BC_DMR_BOTTOM) {
    double h = (P->x1 - P->x0) / P->nx, xc = P->x0 + (along + 0.5) * h;
    return xc < 1.0 / 6.0 ? 0 : 1;
  }
  return 0;
}

/* one wall interface: F[v] = its flux components (stride fs), pv[g][v] its
 * point values (Gauss point stride gs, component stride vs), Wc the average
 * of the cell beside it, axis its normal */
static void wall_interface(const orc_problem* P, int kind, int axis, const double* Wc, double* F, size_t fs,
                           double* pv, size_t gs, size_t vs) {
  if (kind == 2) {
    double rho = Wc[0], u = Wc[1] / rho, v = Wc[2] / rho, p = pressure(2, P->gamma, Wc), h = (Wc[3] + p) / rho;
    double m = F[0];
    F[fs] -= m * u;
    F[2 * fs] -= m * v;
    F[3 * fs] -= m * h;
    F[0] = 0.0;
  } else if (kind == 1) {
    int cn = 1 + axis, ct = 2 - axis;
    F[0] = 0.0;
    F[ct * fs] = 0.0;
    F[3 * fs] = 0.0;
    pv[cn * vs] = 0.0;
    pv[gs + cn * vs] = 0.0;
  }
}

/* every domain-edge wall interface of a 2D step (gas cells beside it) */
static void walls_2d(const orc_problem* P, const double* cell, double* FLX, double* FLY, double* fx, double* fy) {
  int nx = P->nx, ny = P->ny, nv = 4;
  double Wc[4];
  for (int e = 0; e < 2; ++e) {
    int fi = e == 0 ? 0 : nx, ic = e == 0 ? 0 : nx - 1;
    for (int j = 0; j < ny; ++j) {
      int kind = wall_edge(P, 0, fi, 0);
      if (!kind || solid(P, ic, j)) continue;
      for (int v = 0; v < nv; ++v) Wc[v] = cell[((size_t)v * ny + j) * nx + ic];
      wall_interface(P, kind, 0, Wc, &FLX[(size_t)j * (nx + 1) + fi], (size_t)ny * (nx + 1),
                     &fx[(size_t)j * (nx + 1) + fi], (size_t)nv * ny * (nx + 1), (size_t)ny * (nx + 1));
    }
  }
  for (int e = 0; e < 2; ++e) {
    int fj = e == 0 ? 0 : ny, jc = e == 0 ? 0 : ny - 1;
    for (int i = 0; i < nx; ++i) {
      int kind = wall_edge(P, 1, fj, i);
      if (!kind || solid(P, i, jc)) continue;
      for (int v = 0; v < nv; ++v) Wc[v] = cell[((size_t)v * ny + jc) * nx + i];
      wall_interface(P, kind, 1, Wc, &FLY[(size_t)fj * nx + i], (size_t)(ny + 1) * nx,
                     &fy[(size_t)fj * nx + i], (size_t)nv * (ny + 1) * nx, (size_t)(ny + 1) * nx);
    }
  }
}

/* 1D: a slip wall at either end (the same symmetry line) */
static void wall_1d(double* F, double* pv) {
  F[0] = 0.0;
  F[2] = 0.0;
  pv[1] = 0.0;
}

/* every interface of a curvilinear grid (fluxes FLX / FLY and the new
 * Gauss-point values in the grid's (x, y) components) */
static int curv_faces(const orc_problem* P, grid2* G, const cgeom* cg, double dt, double* fx, double* fy, double* FLX,
                      double* FLY) {
  int nx = P->nx, ny = P->ny, nv = 4, status = 0;
#pragma omp parallel for schedule(static) reduction(| : status)
  for (int j = 0; j < ny; ++j)
    for (int fi = 0; fi <= nx; ++fi) {
      const double* fr = cg->fx + ((size_t)j * (nx + 1) + fi) * 7;
      orc_face_input in;
      memset(&in, 0, sizeof(in));
      in.dn = 1.0;
      in.ds = fr[4];
      in.curv = 1;
      in.G[0] = fr[5];
      in.G[1] = fr[6];
      in.G[2] = 1.0 / fr[4];
      for (int s = 0; s < 2; ++s) {
        int ic = fi - 1 + s;
        double Ub[4], p[4][5];
        for (int v = 0; v < nv; ++v) {
          Ub[v] = GW(G, v, j, ic);
          for (int m = 0; m < 5; ++m) p[v][m] = GPC(G, v, m, j, ic);
        }
        curv_side(&in, s, fr, 0, s == 0 ? 0.5 : -0.5, Ub, p);
      }
      for (int m = 0; m < 2; ++m)
        for (int n = 0; n < 3; ++n) {
          double W[4];
          get_cell(G, j - 1 + n, fi - 1 + m, W);
          to_face_frame(fr, W, in.Ueq[m][n]);
        }
      orc_face_output o;
      if (orc_face(P, &in, dt, &o)) status |= 1;
      double F[4], pg[2][4];
      from_face_frame(fr, o.flux, F);
      from_face_frame(fr, o.pv[0], pg[0]);
      from_face_frame(fr, o.pv[1], pg[1]);
      for (int v = 0; v < nv; ++v) {
        FLX[((size_t)v * ny + j) * (nx + 1) + fi] = F[v];
        for (int g = 0; g < 2; ++g) fx[(((size_t)g * nv + v) * ny + j) * (nx + 1) + fi] = pg[g][v];
      }
    }
#pragma omp parallel for schedule(static) reduction(| : status)
  for (int fj = 0; fj <= ny; ++fj)
    for (int i = 0; i < nx; ++i) {
      const double* fr = cg->fy + ((size_t)fj * nx + i) * 7;
      orc_face_input in;
      memset(&in, 0, sizeof(in));
      in.dn = 1.0;
      in.ds = fr[4];
      in.curv = 1;
      in.G[0] = fr[5];
      in.G[1] = fr[6];
      in.G[2] = 1.0 / fr[4];
      for (int s = 0; s < 2; ++s) {
        int jc = fj - 1 + s;
        double Ub[4], p[4][5];
        for (int v = 0; v < nv; ++v) {
          Ub[v] = GW(G, v, jc, i);
          for (int m = 0; m < 5; ++m) p[v][m] = GPC(G, v, m, jc, i);
        }
        curv_side(&in, s, fr, 1, s == 0 ? 0.5 : -0.5, Ub, p);
      }
      for (int m = 0; m < 2; ++m)
        for (int n = 0; n < 3; ++n) {
          double W[4];
          get_cell(G, fj - 1 + m, i - 1 + n, W);
          to_face_frame(fr, W, in.Ueq[m][n]);
        }
      orc_face_output o;
      if (orc_face(P, &in, dt, &o)) status |= 1;
      double F[4], pg[2][4];
      from_face_frame(fr, o.flux, F);
      from_face_frame(fr, o.pv[0], pg[0]);
      from_face_frame(fr, o.pv[1], pg[1]);
      for (int v = 0; v < nv; ++v) {
        FLY[((size_t)v * (ny + 1) + fj) * nx + i] = F[v];
        for (int g = 0; g < 2; ++g) fy[(((size_t)g * nv + v) * (ny + 1) + fj) * nx + i] = pg[g][v];
      }
    }
  return status;
}


static int step2d(const orc_problem* P, double* cell, double* fx, double* fy, double dt, double t, double* fluxx,
                  double* fluxy) {
  grid2 Gs, *G = &Gs;
  int nx = P->nx, ny = P->ny, nv = 4;
  G->nx = nx;
  G->ny = ny;
  G->nv = nv;
  double h = (P->x1 - P->x0) / nx, k = (P->y1 - P->y0) / ny;
  G->W = calloc((size_t)nv * (ny + 4) * (nx + 4), sizeof(double));
  G->FX = calloc((size_t)2 * nv * (ny + 2) * (nx + 3), sizeof(double));
  G->FY = calloc((size_t)2 * nv * (ny + 3) * (nx + 2), sizeof(double));
  G->PC = calloc((size_t)nv * 5 * (ny + 2) * (nx + 2), sizeof(double));
  double* FLX = calloc((size_t)nv * ny * (nx + 1), sizeof(double));
  double* FLY = calloc((size_t)nv * (ny + 1) * nx, sizeof(double));
  int status = 0;
  for (int v = 0; v < nv; ++v)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) GW(G, v, j, i) = cell[((size_t)v * ny + j) * nx + i];
  for (int g = 0; g < 2; ++g)
    for (int v = 0; v < nv; ++v) {
      for (int j = 0; j < ny; ++j)
        for (int fi = 0; fi <= nx; ++fi) GFX(G, g, v, j, fi) = fx[(((size_t)g * nv + v) * ny + j) * (nx + 1) + fi];
      for (int fj = 0; fj <= ny; ++fj)
        for (int i = 0; i < nx; ++i) GFY(G, g, v, fj, i) = fy[(((size_t)g * nv + v) * (ny + 1) + fj) * nx + i];
    }
  fill_ghosts_2d(P, G, t);
  fill_obstacle_2d(P, G);
  cgeom cg;
  memset(&cg, 0, sizeof(cg));
  if (P->mesh) {
    /* curvilinear grid: logical coordinates with unit spacing */
    cgeom_build(P, &cg);
    h = 1.0;
    k = 1.0;
  }

  /* reconstruction: interior cells and the edge ghost cells; the count of
   * interior gas cells that fell back to their average */
  long fallbacks = 0;
#pragma omp parallel for schedule(static) reduction(+ : fallbacks)
  for (int j = -1; j <= ny; ++j)
    for (int i = -1; i <= nx; ++i) {
      int gx = (i < 0 || i >= nx), gy = (j < 0 || j >= ny);
      if (gx && gy) continue;
      double Cw = P->mesh ? P->weno_c * cell_area(P, &cg, i, j) : P->weno_c;
      int fb = recon_cell_2d(P, G, j, i, h, k, Cw);
      if (fb && !gx && !gy && !solid(P, i, j)) fallbacks += 1;
    }
  g_last_fallbacks = fallbacks;

  if (P->mesh) {
    status |= curv_faces(P, G, &cg, dt, fx, fy, FLX, FLY);
    goto update;
  }

  /* x interfaces */
#pragma omp parallel for schedule(static) reduction(| : status)
  for (int j = 0; j < ny; ++j)
    for (int fi = 0; fi <= nx; ++fi) {
      if (solid(P, fi - 1, j) && solid(P, fi, j)) continue; /* inside the step */
      orc_face_input in;
      memset(&in, 0, sizeof(in));
      in.dn = h;
      in.ds = k;
      for (int s = 0; s < 2; ++s) {
        int ic = fi - 1 + s;
        for (int v = 0; v < nv; ++v) {
          double p[5];
          for (int m = 0; m < 5; ++m) p[m] = GPC(G, v, m, j, ic);
          side_values(GW(G, v, j, ic), p, 0, s == 0 ? 1.0 : -1.0, h, k, &in.W[s][v], &in.Wn[s][v], &in.Ws[s][v],
                      &in.Wnn[s][v], &in.Wns[s][v], &in.Wss[s][v]);
        }
      }
      for (int m = 0; m < 2; ++m)
        for (int n = 0; n < 3; ++n)
          for (int v = 0; v < nv; ++v) in.Ueq[m][n][v] = GW(G, v, j - 1 + n, fi - 1 + m);
      if (solid(P, fi - 1, j) != solid(P, fi, j)) wall_mirror(&in, solid(P, fi - 1, j) ? 0 : 1, nv);
      orc_face_output o;
      if (orc_face(P, &in, dt, &o)) status |= 1;
      for (int v = 0; v < nv; ++v) {
        FLX[((size_t)v * ny + j) * (nx + 1) + fi] = o.flux[v];
        for (int g = 0; g < 2; ++g) fx[(((size_t)g * nv + v) * ny + j) * (nx + 1) + fi] = o.pv[g][v];
      }
    }

  /* y interfaces, evaluated in the transposed frame (x <-> y, u <-> v) */
  static const int sw[4] = {0, 2, 1, 3};
#pragma omp parallel for schedule(static) reduction(| : status)
  for (int fj = 0; fj <= ny; ++fj)
    for (int i = 0; i < nx; ++i) {
      if (solid(P, i, fj - 1) && solid(P, i, fj)) continue; /* inside the step */
      orc_face_input in;
      memset(&in, 0, sizeof(in));
      in.dn = k;
      in.ds = h;
      for (int s = 0; s < 2; ++s) {
        int jc = fj - 1 + s;
        for (int v = 0; v < nv; ++v) {
          double p[5];
          for (int m = 0; m < 5; ++m) p[m] = GPC(G, v, m, jc, i);
          int vl = sw[v];
          side_values(GW(G, v, jc, i), p, 1, s == 0 ? 1.0 : -1.0, k, h, &in.W[s][vl], &in.Wn[s][vl], &in.Ws[s][vl],
                      &in.Wnn[s][vl], &in.Wns[s][vl], &in.Wss[s][vl]);
        }
      }
      for (int m = 0; m < 2; ++m)
        for (int n = 0; n < 3; ++n)
          for (int v = 0; v < nv; ++v) in.Ueq[m][n][sw[v]] = GW(G, v, fj - 1 + m, i - 1 + n);
      if (solid(P, i, fj - 1) != solid(P, i, fj)) wall_mirror(&in, solid(P, i, fj - 1) ? 0 : 1, nv);
      orc_face_output o;
      if (orc_face(P, &in, dt, &o)) status |= 1;
      for (int v = 0; v < nv; ++v) {
        FLY[((size_t)v * (ny + 1) + fj) * nx + i] = o.flux[sw[v]];
        for (int g = 0; g < 2; ++g) fy[(((size_t)g * nv + v) * (ny + 1) + fj) * nx + i] = o.pv[g][sw[v]];
      }
    }

update:
  walls_2d(P, cell, FLX, FLY, fx, fy);
  /* eq. finite: conservative update */
  for (int v = 0; v < nv; ++v)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        if (solid(P, i, j)) continue;
        double d = FLX[((size_t)v * ny + j) * (nx + 1) + i] - FLX[((size_t)v * ny + j) * (nx + 1) + i + 1] +
                   FLY[((size_t)v * (ny + 1) + j) * nx + i] - FLY[((size_t)v * (ny + 1) + j + 1) * nx + i];
        cell[((size_t)v * ny + j) * nx + i] += d / (P->mesh ? cg.area[(size_t)j * nx + i] : h * k);
      }
  cgeom_free(&cg);
  if (fluxx) memcpy(fluxx, FLX, sizeof(double) * nv * ny * (nx + 1));
  if (fluxy) memcpy(fluxy, FLY, sizeof(double) * nv * (ny + 1) * nx);
  free(G->W);
  free(G->FX);
  free(G->FY);
  free(G->PC);
  free(FLX);
  free(FLY);
  return status ? -1 : 0;
}

/* ---- 1D ---------------------------------------------------------------- */

/* Right eigenvectors of the 1D Euler flux Jacobian at W (columns u-c, u, u+c) */
static int euler_eigvec_1d(double gamma, const double* W, double R[3][3]) {
  double rho = W[0], u = W[1] / rho, p = (gamma - 1.0) * (W[2] - 0.5 * rho * u * u);
  if (!(rho > 0.0) || !(p > 0.0)) return -1;
  double c = sqrt(gamma * p / rho), H = (W[2] + p) / rho;
  double col[3][3] = {{1.0, u - c, H - u * c}, {1.0, u, 0.5 * u * u}, {1.0, u + c, H + u * c}};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R[i][j] = col[j][i];
  return 0;
}

static int invert3(double A[3][3], double B[3][3]) {
  for (int c = 0; c < 3; ++c) {
    double e[4] = {0, 0, 0, 0}, x[4];
    e[c] = 1.0;
    double M[4][4];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) M[i][j] = A[i][j];
    if (gauss_solve(3, M, e, x)) return -1;
    for (int i = 0; i < 3; ++i) B[i][c] = x[i];
  }
  return 0;
}

static int step1d(const orc_problem* P, double* cell, double* fx, double dt, double t, double* fluxx) {
  (void)t;
  int nx = P->nx, nv = 3;
  double h = (P->x1 - P->x0) / nx;
  double* W = calloc((size_t)nv * (nx + 4), sizeof(double));
  double* F = calloc((size_t)nv * (nx + 3), sizeof(double));
  double* PC = calloc((size_t)nv * 2 * (nx + 2), sizeof(double));
  double* FL = calloc((size_t)nv * (nx + 1), sizeof(double));
#define W1(v, i) W[(size_t)(v) * (nx + 4) + (i) + 2]
#define F1(v, fi) F[(size_t)(v) * (nx + 3) + (fi) + 1]
#define P1(v, m, i) PC[((size_t)(v) * 2 + (m)) * (nx + 2) + (i) + 1]
  int status = 0;
  for (int v = 0; v < nv; ++v) {
    for (int i = 0; i < nx; ++i) W1(v, i) = cell[(size_t)v * nx + i];
    for (int fi = 0; fi <= nx; ++fi) F1(v, fi) = fx[(size_t)v * (nx + 1) + fi];
  }
  /* ghosts */
  for (int side = 0; side < 2; ++side) {
    int kind = P->bc_kind[side];
    double Ws[4], Wg[4];
    for (int m = 0; m < 2; ++m) {
      int ig = side == 0 ? -1 - m : nx + m;
      int is = kind == ORC_BC_PERIODIC ? (side == 0 ? ig + nx : ig - nx) : (side == 0 ? -1 - ig : 2 * nx - 1 - ig);
      if (!fixed_state(P, side, kind, 0.0, 0.0, t, Wg)) {
        for (int v = 0; v < nv; ++v) Ws[v] = W1(v, is);
        if (kind == ORC_BC_PERIODIC)
          memcpy(Wg, Ws, sizeof(Ws));
        else
          mirror_state(P, side, kind, Ws, Wg, 0.0);
      }
      for (int v = 0; v < nv; ++v) W1(v, ig) = Wg[v];
    }
    int fg = side == 0 ? -1 : nx + 1;
    int fs = kind == ORC_BC_PERIODIC ? (side == 0 ? nx - 1 : 1) : (side == 0 ? 1 : nx - 1);
    if (!fixed_state(P, side, kind, 0.0, 0.0, t, Wg)) {
      for (int v = 0; v < nv; ++v) Ws[v] = F1(v, fs);
      if (kind == ORC_BC_PERIODIC)
        memcpy(Wg, Ws, sizeof(Ws));
      else
        mirror_state(P, side, kind, Ws, Wg, 0.0);
    }
    for (int v = 0; v < nv; ++v) F1(v, fg) = Wg[v];
  }
  /* reconstruction, cells -1..nx */
#pragma omp parallel for schedule(static) reduction(| : status)
  for (int i = -1; i <= nx; ++i) {
    if (P->recon_vars == 1) {
      /* characteristic variables of the cell's own state (Sec. 4 remark) */
      double R[3][3], L[3][3], Wc[3];
      for (int v = 0; v < 3; ++v) Wc[v] = W1(v, i);
      if (euler_eigvec_1d(P->gamma, Wc, R) || invert3(R, L)) {
        status |= 1;
        continue;
      }
      double ch[5][3]; /* Uc, Ue, Uw, Fp, Fm in characteristic variables */
      const double* src[5];
      double s0[3], s1[3], s2[3], s3[3], s4[3];
      for (int v = 0; v < 3; ++v) {
        s0[v] = W1(v, i);
        s1[v] = W1(v, i + 1);
        s2[v] = W1(v, i - 1);
        s3[v] = F1(v, i + 1);
        s4[v] = F1(v, i);
      }
      src[0] = s0;
      src[1] = s1;
      src[2] = s2;
      src[3] = s3;
      src[4] = s4;
      for (int s = 0; s < 5; ++s)
        for (int r = 0; r < 3; ++r) {
          ch[s][r] = 0.0;
          for (int v = 0; v < 3; ++v) ch[s][r] += L[r][v] * src[s][v];
        }
      double pc[3][2];
      for (int r = 0; r < 3; ++r)
        orc_recon1d_scalar(ch[0][r], ch[1][r], ch[2][r], ch[3][r], ch[4][r], h, P->weno_eps, P->weno_c, pc[r]);
      for (int v = 0; v < 3; ++v)
        for (int m = 0; m < 2; ++m) {
          double s = 0.0;
          for (int r = 0; r < 3; ++r) s += R[v][r] * pc[r][m];
          P1(v, m, i) = s;
        }
    } else {
      for (int v = 0; v < nv; ++v) {
        double p[2];
        orc_recon1d_scalar(W1(v, i), W1(v, i + 1), W1(v, i - 1), F1(v, i + 1), F1(v, i), h, P->weno_eps, P->weno_c,
                           p);
        P1(v, 0, i) = p[0];
        P1(v, 1, i) = p[1];
      }
    }
  }
  /* admissibility reading (see above): interface values at x = +-h/2 of each
   * cell polynomial against the range of the cell and its two neighbours */
  long fallbacks = 0;
  for (int i = -1; i <= nx; ++i) {
    double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
    for (int q = -1; q <= 1; ++q) {
      double Wq[3] = {W1(0, i + q), W1(1, i + q), W1(2, i + q)};
      range_add(1, P->gamma, Wq, lo, hi);
    }
    int ok = 1;
    for (int sd = -1; sd <= 1; sd += 2) {
      double xn = 0.5 * sd * h, Wf[3];
      for (int v = 0; v < 3; ++v) Wf[v] = W1(v, i) + P1(v, 0, i) * xn + P1(v, 1, i) * 0.5 * (xn * xn - h * h / 12.0);
      if (!admissible(1, P->gamma, P->admissibility, Wf, lo, hi)) ok = 0;
    }
    if (!ok) {
      for (int v = 0; v < 3; ++v) P1(v, 0, i) = P1(v, 1, i) = 0.0;
      if (i >= 0 && i < nx) fallbacks += 1;
    }
  }
  g_last_fallbacks = fallbacks;
  /* interfaces */
#pragma omp parallel for schedule(static) reduction(| : status)
  for (int fi = 0; fi <= nx; ++fi) {
    orc_face_input in;
    memset(&in, 0, sizeof(in));
    in.dn = h;
    in.ds = 1.0;
    for (int s = 0; s < 2; ++s) {
      int ic = fi - 1 + s;
      double sg = s == 0 ? 1.0 : -1.0, xn = 0.5 * sg * h;
      for (int v = 0; v < nv; ++v) {
        double p2 = P1(v, 0, ic), p4 = P1(v, 1, ic);
        in.W[s][v] = W1(v, ic) + p2 * xn + p4 * 0.5 * (xn * xn - h * h / 12.0);
        in.Wn[s][v] = p2 + p4 * xn;
        in.Wnn[s][v] = p4;
      }
    }
    for (int m = 0; m < 2; ++m)
      for (int v = 0; v < nv; ++v) in.Ueq[m][1][v] = W1(v, fi - 1 + m);
    orc_face_output o;
    if (orc_face(P, &in, dt, &o)) status |= 1;
    if ((fi == 0 || fi == nx) && P->bc_kind[fi == 0 ? 0 : 1] == ORC_BC_REFLECT) wall_1d(o.flux, o.pv[0]);
    for (int v = 0; v < nv; ++v) {
      FL[(size_t)v * (nx + 1) + fi] = o.flux[v];
      fx[(size_t)v * (nx + 1) + fi] = o.pv[0][v];
    }
  }
  for (int v = 0; v < nv; ++v)
    for (int i = 0; i < nx; ++i)
      cell[(size_t)v * nx + i] += (FL[(size_t)v * (nx + 1) + i] - FL[(size_t)v * (nx + 1) + i + 1]) / h;
  if (fluxx) memcpy(fluxx, FL, sizeof(double) * nv * (nx + 1));
#undef W1
#undef F1
#undef P1
  free(W);
  free(F);
  free(PC);
  free(FL);
  return status ? -1 : 0;
}

/* ---- driver -------------------------------------------------------------- */

/* reading of the CFL condition: dt = CFL min over cells of
 * min(dx / (|u| + c + 2 nu/dx), dy / (|v| + c + 2 nu/dy)), nu = mu/rho */
double orc_dt(const orc_problem* P, const double* cell) {
  int dim = P->dim, nx = P->nx, ny = dim == 2 ? P->ny : 1, nv = dim + 2;
  double h = (P->x1 - P->x0) / nx, k = dim == 2 ? (P->y1 - P->y0) / ny : 1.0;
  double best = INFINITY;
  size_t n = (size_t)nx * ny;
  if (dim == 2 && P->mesh) {
    /* curvilinear grid: the widths across the two logical directions and
     * the speed */
    cgeom cg;
    cgeom_build(P, &cg);
    for (size_t c = 0; c < n; ++c) {
      double W[4];
      for (int v = 0; v < 4; ++v) W[v] = cell[(size_t)v * n + c];
      double rho = W[0], u = W[1] / rho, vv = W[2] / rho, p = pressure(2, P->gamma, W);
      if (!(rho > 0.0) || !(p > 0.0)) {
        cgeom_free(&cg);
        return -1.0;
      }
      double cs = sqrt(P->gamma * p / rho), nu = P->viscous ? P->mu / rho : 0.0, sp = sqrt(u * u + vv * vv);
      double w[2] = {cg.h1[c], cg.h2[c]};
      for (int d = 0; d < 2; ++d) {
        double b = w[d] / (sp + cs + 2.0 * nu / w[d]);
        if (b < best) best = b;
      }
    }
    cgeom_free(&cg);
    return P->cfl * best;
  }
  for (size_t c = 0; c < n; ++c) {
    if (dim == 2 && solid(P, (int)(c % nx), (int)(c / nx))) continue;
    double W[4];
    for (int v = 0; v < nv; ++v) W[v] = cell[(size_t)v * n + c];
    double rho = W[0], u = W[1] / rho, vv = dim == 2 ? W[2] / rho : 0.0;
    double p = pressure(dim, P->gamma, W);
    if (!(rho > 0.0) || !(p > 0.0)) return -1.0;
    double cs = sqrt(P->gamma * p / rho), nu = P->viscous ? P->mu / rho : 0.0;
    double dtx = h / (fabs(u) + cs + 2.0 * nu / h);
    if (dtx < best) best = dtx;
    if (dim == 2) {
      double dty = k / (fabs(vv) + cs + 2.0 * nu / k);
      if (dty < best) best = dty;
    }
  }
  return P->cfl * best;
}

static double* g_last_fx = NULL;
static double* g_last_fy = NULL;

int orc_step(const orc_problem* P, double* cell, double* fx, double* fy, double dt, double t) {
  int nv = P->dim + 2, nx = P->nx, ny = P->ny;
  free(g_last_fx);
  free(g_last_fy);
  g_last_fx = calloc((size_t)nv * ny * (nx + 1), sizeof(double));
  g_last_fy = P->dim == 2 ? calloc((size_t)nv * (ny + 1) * nx, sizeof(double)) : NULL;
  if (P->dim == 1) return step1d(P, cell, fx, dt, t, g_last_fx);
  return step2d(P, cell, fx, fy, dt, t, g_last_fx, g_last_fy);
}

int orc_last_fluxes(const orc_problem* P, double* fxflux, double* fyflux) {
  int nv = P->dim + 2, nx = P->nx, ny = P->ny;
  if (!g_last_fx) return -1;
  memcpy(fxflux, g_last_fx, sizeof(double) * nv * ny * (nx + 1));
  if (P->dim == 2 && fyflux) memcpy(fyflux, g_last_fy, sizeof(double) * nv * (ny + 1) * nx);
  return 0;
}

int orc_run(const orc_problem* P, double* cell, double* fx, double* fy, int nsteps, double dt_fixed, double t_end,
            double* t) {
  int n = 0;
  for (;;) {
    if (nsteps > 0 && n >= nsteps) break;
    if (t_end > 0.0 && *t >= t_end * (1.0 - 1e-14)) break;
    double dt = dt_fixed > 0.0 ? dt_fixed : orc_dt(P, cell);
    if (!(dt > 0.0)) return -1;
    if (t_end > 0.0 && *t + dt > t_end) dt = t_end - *t;
    if (orc_step(P, cell, fx, fy, dt, *t)) return -1;
    *t += dt;
    ++n;
    if (nsteps <= 0 && t_end <= 0.0) break;
  }
  return n;
}

long orc_last_fallbacks(void) { return g_last_fallbacks; }

/* interface sides whose Chapman-Enskog correction was capped (the Knudsen
 * reading of eq. dis2) since the last call */
long orc_take_capped(void) {
  long n = g_capped;
  g_capped = 0;
  return n;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
