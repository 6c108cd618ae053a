/*
 * gks_oracle.h -- plain FP64 CPU oracle for the compact third-order
 * gas-kinetic scheme of Pan & Xu (arXiv:1412.4489).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path; it is
 * loaded by tests/, by __graft_entry__.smoke() and by the cpu_baseline leg of
 * bench.py, and by nothing else.  It shares no code, header, table or
 * constant with the GPU library.
 *
 * The oracle follows the paper's steps in the paper's order and notation:
 *   Sec. 2.1  BGK model, compatibility, psi, K                 (eq. bgk, compatibility)
 *   Sec. 2.1  finite-volume update                             (eq. finite)
 *   Sec. 2.2  integral solution, Taylor f0, g, dis1/dis2, C_i  (eqs. integral, f0, dis2, equli, dis1)
 *   Sec. 2.2  coefficient systems for a,b,d,A,B                (system after eq. dis3)
 *   Sec. 3    point values (eq. point), 1D/2D compact reconstruction
 *             (limiter, average, over-sys), equilibrium quadratic (Sec. 3.3)
 *   Sec. 4    collision time, CFL
 * Everything is a polynomial in (u, v, xi^2) times a Maxwellian, integrated
 * monomial by monomial with Gaussian moment tables.
 */
#ifndef GKS_ORACLE_H
#define GKS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* boundary kinds of the oracle (its own numbering) */
enum {
  ORC_BC_PERIODIC = 0,
  ORC_BC_OUTFLOW = 1,      /* zero normal gradient (mirror image, no sign change) */
  ORC_BC_REFLECT = 2,      /* slip wall: mirror image, normal momentum negated */
  ORC_BC_NOSLIP_ISO = 3,   /* no-slip isothermal wall (wall u, v, T) */
  ORC_BC_NOSLIP_ADIA = 4,  /* no-slip adiabatic wall (wall u, v) */
  ORC_BC_INFLOW = 5,       /* fixed primitive state */
  ORC_BC_DMR_BOTTOM = 6,   /* fixed post-shock state for x < 1/6, slip wall beyond */
  ORC_BC_DMR_TOP = 7       /* exact Mach-10 shock motion along the top edge */
};

typedef struct {
  int dim;                 /* 1 or 2 */
  int nx, ny;              /* cells; ny = 1 when dim == 1 */
  double x0, x1, y0, y1;   /* domain */
  double gamma;            /* specific heat ratio -> K internal degrees of freedom */
  int viscous;             /* 0: Euler (f_G = g), 1: Navier-Stokes (eq. ns) */
  double mu, prandtl;      /* constant dynamic viscosity, Prandtl number */
  double tau_eps, tau_c;   /* collision time constants of Sec. 4 */
  double cfl;              /* CFL number for the time step */
  double weno_eps, weno_c; /* small number and I(U1) = C h^2 constant of Sec. 3.1 */
  int recon_vars;          /* 0 conservative, 1 characteristic variables */
  int exact_c;             /* 0: C4..C6 as printed; 1: exact exponential integrals */
  int bc_kind[4];          /* W, E, S, N */
  double bc_state[4][4];   /* primitive (rho, u, v, p): INFLOW state; DMR post-shock state */
  double bc_alt[4][4];     /* primitive (rho, u, v, p): DMR pre-shock state (top edge) */
  double bc_wall[4][3];    /* wall u, v, T for no-slip walls */
  int obst_i0, obst_nj;    /* 2D solid step: cells i >= obst_i0, j < obst_nj (none: obst_nj = 0) */
  int admissibility;       /* a reconstructed cell polynomial is kept if, at its interface centres,
                              0: rho > 0 and p > 0; 1: also within a factor two of the range of
                              the neighbouring averages (else the constant average is used) */
  /* 2D curvilinear grid (the extension the remark closing Sec. 3.3 points
   * to; the polar cavity of Sec. 4.8): vertex coordinates [ny+1][nx+1][2] of
   * straight-edged quadrilateral cells, cell (i, j) having the corners
   * (i, j), (i+1, j), (i+1, j+1), (i, j+1) counter-clockwise.  NULL: the
   * uniform grid of [x0, x1] x [y0, y1]. */
  const double* mesh;
  double bc_omega[4];      /* curvilinear grids: the no-slip wall also turns about the origin at this
                              angular velocity (wall velocity (u_w - omega y, v_w + omega x)) */
} orc_problem;

/* --- kinetic building blocks ------------------------------------------- */

/* Normalised moment tables of the Maxwellian of the conservative state W.
 * half = 0: whole velocity space; +1: u > 0; -1: u < 0.
 * Mu[n] = <u^n>, n < 16; Mv[n] = <v^n>, n < 16; Mx[e] = <xi^(2e)>, e < 8.
 * prim = (rho, U, V, lambda).  Returns 0, or -1 for a nonphysical state. */
int orc_moment_tables(int dim, double gamma, const double* W, int half,
                      double* Mu, double* Mv, double* Mx, double* prim);

/* Solve <a psi> = b for the coefficient vector a (a_1 + a_2 u + a_3 v + a_4 (u^2+v^2+xi^2)/2)
 * of the Maxwellian of W.  b has dim+2 entries (already divided by rho). */
int orc_solve(int dim, double gamma, const double* W, const double* b, double* a);

/* All expansion coefficients of the Maxwellian of W from the derivatives of
 * the conservative variables (order: ax, ay, A, dxx, dxy, dyy, bx, by, B;
 * each dim+2 long, stored with stride 4).  which: 0 = g0 (all nine),
 * 1 = side, Euler (ax..dyy), 2 = side, NS (adds A, bx, by). */
int orc_coefficients(int dim, double gamma, const double* W, const double* Wx,
                     const double* Wy, const double* Wxx, const double* Wxy,
                     const double* Wyy, int which, double* coef /* [9][4] */);

/* C_1..C_8, C_7 t, C_7 t^2 at time t (out[10]); and their integrals over
 * [0, dt] (out[10]). */
void orc_time_coefficients(double tau, double t, int exact_c, double* out);
void orc_time_integrals(double tau, double dt, int exact_c, double* out);

/* --- one interface ------------------------------------------------------ */

/* Interface data in the interface-normal frame (n normal, s tangential).
 * Vectors are conservative (rho, rho u_n, rho u_s, rho E) in 2D and
 * (rho, rho u, rho E) in 1D.  Side 0 = left (x < 0), side 1 = right. */
typedef struct {
  double W[2][4], Wn[2][4], Ws[2][4], Wnn[2][4], Wns[2][4], Wss[2][4];
  double Ueq[2][3][4]; /* cell averages of the equilibrium stencil [normal m][tangential n] */
  double dn, ds;       /* cell size normal / tangential to the interface */
  /* curv = 1 (an interface of a curvilinear grid): the equilibrium quadratic
   * of Sec. 3.3 is formed from Ueq with unit spacing (logical coordinates)
   * and mapped to the interface frame with G = (G_nn, G_ns, G_ss): d/dn =
   * G_nn d/dxi + G_ns d/deta, d/ds = G_ss d/deta (dn is then unused) */
  int curv;
  double G[3];
} orc_face_input;

typedef struct {
  double flux[4];     /* time- and face-integrated flux */
  double pv[2][4];    /* point values at t+dt, tangential -delta / +delta (1D: pv[0]) */
  double W0[4];       /* interface equilibrium state */
  double q[5][4];     /* b2..b6 of the equilibrium quadratic */
  double tau;
  double heat;        /* time- and face-integrated heat flux (NS) */
} orc_face_output;

int orc_face(const orc_problem* P, const orc_face_input* in, double dt, orc_face_output* out);

/* Values of the assembled gas distribution function (eq. dis1 + eq. dis2) at
 * the interface, position y and time t, for n particle velocities
 * (u[q], v[q], xi2[q]) (test pin).  prim[3][4] = (rho, U, V, lambda) of g_l,
 * g_r, g0; coef[3][9][4] their coefficient sets. */
void orc_f_assembled(int dim, double gamma, int viscous, int exact_c, double tau,
                     const double* prim, const double* coef, double y, double t,
                     int n, const double* u, const double* v, const double* xi2, double* out);

/* --- reconstruction ----------------------------------------------------- */

/* 2D reconstruction of one scalar on cell (i,j): returns p = (p2..p6) of
 * U(x,y) = Ubar + p2 x + p3 y + p4 w_x + p5 w_y + p6 x y. */
void orc_recon2d_scalar(double Uc, double Ue, double Uw, double Un, double Us,
                        double Ep, double Em, double Wp, double Wm,
                        double Np, double Nm, double Sp, double Sm,
                        double h, double k, double eps, double C, double* p);

/* Right eigenvectors (columns; row-major [4][4]) of the 2D Euler flux
 * Jacobian along axis ax (0: x, 1: y) at the conservative state W: waves
 * un - c, un (entropy), un (shear), un + c.  Returns -1 for a nonphysical W. */
int orc_euler_eigvec_2d(double gamma, const double* W, int ax, double* R);

/* 2D reconstruction of one cell, all four conservative components.
 * S[13][4]: Uc, Ue, Uw, Un, Us, E+, E-, W+, W-, N+, N-, S+, S- of each
 * component; vars 0 = conservative, 1 = the limiter of each direction in the
 * characteristic variables of that direction at the cell average.  pc[4][5]:
 * p2..p6 of each component.  Returns -1 (and pc = 0) when vars = 1 and the
 * cell average is nonphysical. */
int orc_recon2d_cell(int vars, double gamma, const double* S, double h, double k,
                     double eps, double C, double* pc);

/* 1D reconstruction of one scalar: p = (p2, p4) of Ubar + p2 x + p4 w_x.
 * Fm, Fp = point values at x_{i-1/2}, x_{i+1/2}. */
void orc_recon1d_scalar(double Uc, double Ue, double Uw, double Fp, double Fm,
                        double h, double eps, double C, double* p);

/* Equilibrium quadratic b2..b6 (2D) from six cell averages U[m][n][var] and U0. */
void orc_equilibrium_poly(int dim, const double* Ueq, const double* U0,
                          double dn, double ds, double* q /* [5][4] */);

/* --- whole scheme ------------------------------------------------------- */

/* Host layouts without ghosts: cell[nvar][ny][nx];
 * fx[ng][nvar][ny][nx+1]; fy[2][nvar][ny+1][nx] (unused in 1D);
 * ng = 2 in 2D (Gauss points -, +), 1 in 1D. */
double orc_dt(const orc_problem* P, const double* cell);
int orc_step(const orc_problem* P, double* cell, double* fx, double* fy, double dt, double t);
/* Runs nsteps (or until t_end if t_end > t).  dt_fixed > 0 fixes the step.
 * Returns the number of steps taken, or < 0 on failure; *t updated. */
int orc_run(const orc_problem* P, double* cell, double* fx, double* fy, int nsteps,
            double dt_fixed, double t_end, double* t);

/* Interior (gas) cells whose reconstruction fell back to the constant
 * average in the last orc_step */
long orc_last_fallbacks(void);
/* interface sides whose Chapman-Enskog correction was capped since the last
 * call (and resets the count) */
long orc_take_capped(void);

/* Flux diagnostics of the last orc_step (x faces then y faces, [nvar][..]) */
int orc_last_fluxes(const orc_problem* P, double* fxflux, double* fyflux);

int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
