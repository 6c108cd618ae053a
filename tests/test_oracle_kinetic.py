"""Pins of the oracle's kinetic building blocks against mathematics that does
not go through the oracle's own formulas.

* Maxwellian moment tables (whole and half space) vs direct quadrature and the
  chi-square moments of the internal degrees of freedom (Sec. 2.1).
* <psi g> = W and <u psi g> = Euler flux (Sec. 2.1, compatibility).
* The coefficient systems (Sec. 2.2, system after eq. dis3): for the Maxwellian
  of a smooth field W(x, y, t) obeying the Euler equations, the nine
  coefficient sets are exactly the derivatives of ln g, computed here by
  forward-mode differentiation (truncated Taylor jets) of the physics.
* C_1..C_8 (Sec. 2.2): their time integrals vs quadrature; the exact-integral
  variant vs the defining integral of the hydrodynamic part.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special


def _state(rng, dim=2):
    rho = rng.uniform(0.5, 2.0)
    u, v = rng.uniform(-1.5, 1.5, 2)
    p = rng.uniform(0.4, 3.0)
    g = 1.4
    if dim == 2:
        return np.array([rho, rho * u, rho * v, p / (g - 1) + 0.5 * rho * (u * u + v * v)])
    return np.array([rho, rho * u, p / (g - 1) + 0.5 * rho * u * u])


@pytest.mark.parametrize("half", [0, 1, -1])
@pytest.mark.parametrize("seed", range(3))
def test_moment_tables_vs_quadrature(oracle, half, seed):
    rng = np.random.default_rng(seed)
    W = _state(rng)
    Mu, Mv, Mx, prim = oracle.moment_tables(2, 1.4, W, half)
    rho, U, V, lam = prim
    K = (4 - 2 * 1.4) / (1.4 - 1)
    dens = lambda x, c: math.sqrt(lam / math.pi) * math.exp(-lam * (x - c) ** 2)
    lo, hi = -np.inf, np.inf
    if half > 0:
        lo = 0.0
    if half < 0:
        hi = 0.0
    for n in range(10):
        ref, _ = integrate.quad(lambda x: x ** n * dens(x, U), lo, hi, epsabs=0, epsrel=1e-13, limit=200)
        assert Mu[n] == pytest.approx(ref, rel=1e-11, abs=1e-13 * max(1, abs(U)) ** n)
        refv, _ = integrate.quad(lambda x: x ** n * dens(x, V), -np.inf, np.inf, epsabs=0, epsrel=1e-13, limit=200)
        assert Mv[n] == pytest.approx(refv, rel=1e-11, abs=1e-13)
    # xi^2 = chi^2_K / (2 lambda): <(xi^2)^e> = Gamma(K/2 + e) / Gamma(K/2) / lambda^e
    for e in range(5):
        ref = special.gamma(K / 2 + e) / special.gamma(K / 2) / lam ** e
        assert Mx[e] == pytest.approx(ref, rel=1e-13)


def test_moments_reproduce_state_and_euler_flux(oracle):
    g = 1.4
    rng = np.random.default_rng(7)
    for dim in (1, 2):
        for _ in range(4):
            W = _state(rng, dim)
            Mu, Mv, Mx, (rho, U, V, lam) = oracle.moment_tables(dim, g, W)
            if dim == 2:
                psi = np.array([1.0, Mu[1], Mv[1], 0.5 * (Mu[2] + Mv[2] + Mx[1])])
                upsi = np.array([Mu[1], Mu[2], Mu[1] * Mv[1], 0.5 * (Mu[3] + Mu[1] * Mv[2] + Mu[1] * Mx[1])])
                p = (g - 1) * (W[3] - 0.5 * rho * (U * U + V * V))
                F = np.array([rho * U, rho * U * U + p, rho * U * V, U * (W[3] + p)])
            else:
                psi = np.array([1.0, Mu[1], 0.5 * (Mu[2] + Mx[1])])
                upsi = np.array([Mu[1], Mu[2], 0.5 * (Mu[3] + Mu[1] * Mx[1])])
                p = (g - 1) * (W[2] - 0.5 * rho * U * U)
                F = np.array([rho * U, rho * U * U + p, U * (W[2] + p)])
            np.testing.assert_allclose(rho * psi, W, rtol=1e-14, atol=1e-14)
            np.testing.assert_allclose(rho * upsi, F, rtol=1e-13, atol=1e-13)
            # half spaces add up to the whole space
            Mp = oracle.moment_tables(dim, g, W, +1)[0]
            Mm = oracle.moment_tables(dim, g, W, -1)[0]
            np.testing.assert_allclose(Mp + Mm, Mu, rtol=1e-12, atol=1e-12)


def test_solve_residual(oracle):
    rng = np.random.default_rng(3)
    for dim in (1, 2):
        for _ in range(5):
            W = _state(rng, dim)
            b = rng.normal(size=dim + 2)
            a = oracle.solve(dim, 1.4, W, b)
            Mu, Mv, Mx, _ = oracle.moment_tables(dim, 1.4, W)
            # <psi_i psi_j> a_j, written out with the tables
            if dim == 2:
                def m(i, j, k=0):
                    return Mu[i] * Mv[j] * Mx[k]
                z = lambda i, j: 0.5 * (m(i + 2, j) + m(i, j + 2) + m(i, j, 1))
                zz = 0.25 * (m(4, 0) + m(0, 4) + m(0, 0, 2) + 2 * m(2, 2) + 2 * m(2, 0, 1) + 2 * m(0, 2, 1))
                G = np.array([[1, m(1, 0), m(0, 1), z(0, 0)],
                              [m(1, 0), m(2, 0), m(1, 1), z(1, 0)],
                              [m(0, 1), m(1, 1), m(0, 2), z(0, 1)],
                              [z(0, 0), z(1, 0), z(0, 1), zz]])
            else:
                m = lambda i, k=0: Mu[i] * Mx[k]
                z = lambda i: 0.5 * (m(i + 2) + m(i, 1))
                zz = 0.25 * (m(4) + m(0, 2) + 2 * m(2, 1))
                G = np.array([[1, m(1), z(0)], [m(1), m(2), z(1)], [z(0), z(1), zz]])
            np.testing.assert_allclose(G @ a, b, rtol=1e-10, atol=1e-10)


# --- coefficient systems vs the Euler physics of a Maxwellian field ----------

class Jet:
    """Truncated Taylor polynomial (total degree <= 2) in the variables
    (x, y, t, e) about the origin: forward-mode automatic differentiation
    independent of the oracle."""
    NV = 4
    IDX = [m for m in np.ndindex(3, 3, 3, 3) if sum(m) <= 2]

    def __init__(self, c=None):
        self.c = {} if c is None else c

    @classmethod
    def const(cls, a):
        return cls({(0, 0, 0, 0): float(a)})

    @classmethod
    def poly(cls, terms):
        return cls({k: float(v) for k, v in terms.items() if sum(k) <= 2})

    def _lift(self, o):
        return o if isinstance(o, Jet) else Jet.const(o)

    def __add__(self, o):
        o = self._lift(o)
        c = dict(self.c)
        for k, v in o.c.items():
            c[k] = c.get(k, 0.0) + v
        return Jet(c)

    __radd__ = __add__

    def __neg__(self):
        return Jet({k: -v for k, v in self.c.items()})

    def __sub__(self, o):
        return self + (-self._lift(o))

    def __rsub__(self, o):
        return self._lift(o) - self

    def __mul__(self, o):
        o = self._lift(o)
        c = {}
        for k1, v1 in self.c.items():
            for k2, v2 in o.c.items():
                k = tuple(a + b for a, b in zip(k1, k2))
                if sum(k) <= 2:
                    c[k] = c.get(k, 0.0) + v1 * v2
        return Jet(c)

    __rmul__ = __mul__

    def c0(self):
        return self.c.get((0, 0, 0, 0), 0.0)

    def _series(self, f0, f1, f2):
        """f(c0 + r) = f0 + f1 r + f2 r^2 / 2 with r the non-constant part."""
        r = self - self.c0()
        return Jet.const(f0) + f1 * r + (0.5 * f2) * (r * r)

    def inv(self):
        a = self.c0()
        return self._series(1 / a, -1 / a ** 2, 2 / a ** 3)

    def __truediv__(self, o):
        return self * self._lift(o).inv()

    def __rtruediv__(self, o):
        return self._lift(o) * self.inv()

    def log(self):
        a = self.c0()
        return self._series(math.log(a), 1 / a, -1 / a ** 2)

    def d(self, var):
        """partial derivative (a Jet of one degree less accuracy)"""
        c = {}
        for k, v in self.c.items():
            if k[var] > 0:
                kk = list(k)
                kk[var] -= 1
                c[tuple(kk)] = c.get(tuple(kk), 0.0) + v * k[var]
        return Jet(c)

    def deriv0(self, *vars_):
        k = [0, 0, 0, 0]
        for v in vars_:
            k[v] += 1
        fac = 1
        for n in k:
            fac *= math.factorial(n)
        return self.c.get(tuple(k), 0.0) * fac


X, Y, T, EPS = 0, 1, 2, 3


def _euler_maxwellian_derivatives(seed, dim=2):
    """Coefficient sets of ln g for the Maxwellian of a random quadratic
    primitive field W(x, y) that evolves by the Euler equations:
    ax = d_x ln g, A = d_t ln g, dxx = d_xx ln g, ..., B = d_tt ln g, written in
    the basis (1, u, v, (u^2 + v^2 + xi^2)/2).  Returns the derivatives of W at
    the origin and the nine exact sets."""
    rng = np.random.default_rng(seed)
    g = 1.4
    K = (4 - 2 * g) / (g - 1) if dim == 2 else (3 - g) / (g - 1)
    N = K + 2 if dim == 2 else K + 1

    def field(base):
        terms = {(0, 0, 0, 0): base, (1, 0, 0, 0): rng.uniform(-0.3, 0.3), (2, 0, 0, 0): rng.uniform(-0.3, 0.3)}
        if dim == 2:
            terms.update({(0, 1, 0, 0): rng.uniform(-0.3, 0.3), (0, 2, 0, 0): rng.uniform(-0.3, 0.3),
                          (1, 1, 0, 0): rng.uniform(-0.3, 0.3)})
        return Jet.poly(terms)

    rho = field(rng.uniform(0.8, 1.5))
    U = field(rng.uniform(-0.5, 0.5))
    V = field(rng.uniform(-0.5, 0.5)) if dim == 2 else Jet.const(0.0)
    p = field(rng.uniform(0.8, 1.5))

    def cons(rho, U, V, p):
        E = p / (g - 1) + rho * (U * U + V * V) * 0.5
        return [rho, rho * U, rho * V, E] if dim == 2 else [rho, rho * U, E]

    def fluxes(W):
        r = W[0]
        u = W[1] / r
        v = W[2] / r if dim == 2 else Jet.const(0.0)
        pp = (g - 1) * (W[-1] - r * (u * u + v * v) * 0.5)
        if dim == 2:
            return [W[1], W[1] * u + pp, W[1] * v, u * (W[3] + pp)], [W[2], W[2] * u, W[2] * v + pp, v * (W[3] + pp)]
        return [W[1], W[1] * u + pp, u * (W[2] + pp)], None

    def div(W):
        F, G = fluxes(W)
        out = [f.d(X) for f in F]
        if dim == 2:
            out = [a + gg.d(Y) for a, gg in zip(out, G)]
        return out

    W = cons(rho, U, V, p)
    Wt = [-a for a in div(W)]                                   # Euler: W_t = -div F(W)
    eps = Jet.poly({(0, 0, 0, 1): 1.0})
    dirn = div([a + eps * b for a, b in zip(W, Wt)])            # div F(W + e W_t)
    Wtt0 = [-a.d(EPS).c0() for a in dirn]                        # W_tt = -div(F'(W) W_t) at the origin
    tj = Jet.poly({(0, 0, 1, 0): 1.0})
    Wfull = [a + tj * b + (0.5 * c) * (tj * tj) for a, b, c in zip(W, Wt, Wtt0)]
    r = Wfull[0]
    uu = Wfull[1] / r
    vv = Wfull[2] / r if dim == 2 else Jet.const(0.0)
    pp = (g - 1) * (Wfull[-1] - r * (uu * uu + vv * vv) * 0.5)
    lam = r / (2 * pp)
    # ln g = ln rho + (N/2) ln lambda - lambda ((u-U)^2 + (v-V)^2 + xi^2) + const
    c0 = r.log() + (N / 2) * lam.log() - lam * (uu * uu + vv * vv)
    lng = [c0, 2 * lam * uu] + ([2 * lam * vv] if dim == 2 else []) + [-2 * lam]

    def coefset(*vars_):
        return np.array([c.deriv0(*vars_) for c in lng])

    sets = {"ax": coefset(X), "A": coefset(T), "dxx": coefset(X, X), "bx": coefset(X, T), "B": coefset(T, T)}
    if dim == 2:
        sets.update(ay=coefset(Y), dxy=coefset(X, Y), dyy=coefset(Y, Y), by=coefset(Y, T))
    Wd = {"W": np.array([a.c0() for a in W])}
    for name, vars_ in {"Wx": (X,), "Wy": (Y,), "Wxx": (X, X), "Wxy": (X, Y), "Wyy": (Y, Y)}.items():
        Wd[name] = np.array([a.deriv0(*vars_) for a in W])
    return Wd, sets


@pytest.mark.parametrize("dim", [1, 2])
@pytest.mark.parametrize("seed", range(3))
def test_coefficients_are_derivatives_of_ln_g(oracle, dim, seed):
    Wd, exact = _euler_maxwellian_derivatives(seed, dim)
    coef = oracle.coefficients(dim, 1.4, Wd["W"], Wd["Wx"], Wd["Wy"], Wd["Wxx"], Wd["Wxy"], Wd["Wyy"], which=0)
    names = ["ax", "ay", "A", "dxx", "dxy", "dyy", "bx", "by", "B"]
    nv = dim + 2
    for i, name in enumerate(names):
        if name not in exact:
            continue
        np.testing.assert_allclose(coef[i, :nv], exact[name], rtol=1e-9, atol=1e-9 * np.abs(exact[name]).max(),
                                   err_msg=name)


@pytest.mark.parametrize("tau_over_dt", [0.0, 0.01, 0.05, 0.3, 1.0, 5.0])
def test_time_integrals_vs_quadrature(oracle, tau_over_dt):
    dt = 0.013
    tau = tau_over_dt * dt
    for exact_c in (False, True):
        I = oracle.time_integrals(tau, dt, exact_c)
        for k in range(10):
            ref, _ = integrate.quad(lambda s: oracle.time_coefficients(tau, s, exact_c)[k], 0, dt, epsabs=0,
                                    epsrel=1e-13, limit=100)
            assert I[k] == pytest.approx(ref, rel=1e-9, abs=1e-15 * dt ** 3)


def test_time_coefficients_tau_zero_limits(oracle):
    dt = 0.02
    C = oracle.time_coefficients(0.0, dt)
    np.testing.assert_allclose(C, [1, 0, dt, 0, dt * dt, 0, 0, 0, 0, 0], atol=1e-18)
    I = oracle.time_integrals(0.0, dt)
    np.testing.assert_allclose(I, [dt, 0, dt * dt / 2, 0, dt ** 3 / 3, 0, 0, 0, 0, 0], atol=1e-18)


@pytest.mark.parametrize("tau", [0.003, 0.02, 0.1])
def test_exact_c_are_the_exponential_integrals(oracle, tau):
    """With exact_c the hydrodynamic weights are (1/tau) int_0^t s(t') exp(-(t-t')/tau) dt'
    of the Taylor terms 1, -u s, t', (u s)^2 ..., i.e. C1 <- 1, C2 <- -s, C3 <- t - s,
    C4 <- s^2, C5 <- (t-s)^2, C6 <- -s (t-s) with s = t - t'."""
    t = 0.017
    C = oracle.time_coefficients(tau, t, exact_c=True)
    w = lambda fn: integrate.quad(lambda s: fn(s) * math.exp(-s / tau) / tau, 0, t, epsabs=0, epsrel=1e-13)[0]
    ref = [w(lambda s: 1.0), w(lambda s: -s), w(lambda s: t - s), w(lambda s: s * s), w(lambda s: (t - s) ** 2),
           w(lambda s: -s * (t - s))]
    np.testing.assert_allclose(C[:6], ref, rtol=1e-10, atol=1e-16)
    # the printed C4..C6 drop 2 tau^2 (1 - e^(-t/tau)) from each (reading kept in the scheme)
    Cp = oracle.time_coefficients(tau, t, exact_c=False)
    np.testing.assert_allclose(C[3:6] - Cp[3:6], 2 * tau * tau * (1 - math.exp(-t / tau)), rtol=1e-10)
