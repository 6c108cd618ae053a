"""Pins of the oracle's compact reconstruction (Sec. 3.1, 3.2) and the
equilibrium quadratic (Sec. 3.3): exactness on global quadratics (every
one-sided stencil, the central stencil and the equilibrium least squares
reproduce a quadratic), and the limiter's behaviour at a jump."""
import math

import numpy as np
import pytest

S3 = math.sqrt(3.0)


def _quad2d(rng):
    c = rng.normal(size=6)

    def U(x, y):
        return c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * y * y + c[5] * x * y

    def avg(xc, yc, h, k):  # exact average of a quadratic over a cell
        return U(xc, yc) + c[3] * h * h / 12 + c[4] * k * k / 12

    return c, U, avg


@pytest.mark.parametrize("seed", range(5))
def test_recon2d_exact_on_quadratics(oracle, seed):
    rng = np.random.default_rng(seed)
    c, U, avg = _quad2d(rng)
    h, k = 0.07, 0.05
    d = S3 / 6
    p = oracle.recon2d_scalar(avg(0, 0, h, k), avg(h, 0, h, k), avg(-h, 0, h, k), avg(0, k, h, k),
                              avg(0, -k, h, k), U(h / 2, d * k), U(h / 2, -d * k), U(-h / 2, d * k),
                              U(-h / 2, -d * k), U(d * h, k / 2), U(-d * h, k / 2), U(d * h, -k / 2),
                              U(-d * h, -k / 2), h, k)
    # U = Ubar + p2 x + p3 y + p4 (x^2 - h^2/12)/2 + p5 (y^2 - k^2/12)/2 + p6 x y
    np.testing.assert_allclose(p, [c[1], c[2], 2 * c[3], 2 * c[4], c[5]], rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("weights", [(1e-6, 1.0), (1e-6, 1e8), (1e-14, 1e-12)])
def test_recon2d_each_stencil_family_exact(oracle, weights):
    """Exactness holds whichever stencil family the weights pick."""
    rng = np.random.default_rng(11)
    c, U, avg = _quad2d(rng)
    h = k = 0.04
    d = S3 / 6
    p = oracle.recon2d_scalar(avg(0, 0, h, k), avg(h, 0, h, k), avg(-h, 0, h, k), avg(0, k, h, k),
                              avg(0, -k, h, k), U(h / 2, d * k), U(h / 2, -d * k), U(-h / 2, d * k),
                              U(-h / 2, -d * k), U(d * h, k / 2), U(-d * h, k / 2), U(d * h, -k / 2),
                              U(-d * h, -k / 2), h, k, *weights)
    np.testing.assert_allclose(p, [c[1], c[2], 2 * c[3], 2 * c[4], c[5]], rtol=1e-8, atol=1e-8)


def test_recon1d_exact_on_quadratics(oracle):
    rng = np.random.default_rng(2)
    a, b, cc = rng.normal(size=3)
    h = 0.1
    U = lambda x: a + b * x + cc * x * x
    avg = lambda xc: U(xc) + cc * h * h / 12
    p = oracle.recon1d_scalar(avg(0), avg(h), avg(-h), U(h / 2), U(-h / 2), h)
    np.testing.assert_allclose(p, [b, 2 * cc], rtol=1e-10)


def test_recon1d_limits_at_a_jump(oracle):
    """A step between the cell and its right neighbour: the one-sided curvatures
    disagree in sign, minmod zeroes the curvature and the weights select the
    one-sided polynomial, so the reconstruction stays within the data."""
    h = 0.01
    p = oracle.recon1d_scalar(1.0, 0.0, 1.0, 0.5, 1.0, h)
    Ur = 1.0 + p[0] * h / 2 + p[1] * h * h / 12
    Ul = 1.0 - p[0] * h / 2 + p[1] * h * h / 12
    # the central polynomial keeps a weight of O((h^2 / I2)^2) only
    assert -1e-6 <= Ur <= 1.0 + 1e-6 and -1e-6 <= Ul <= 1.0 + 1e-6
    assert abs(Ul - 1.0) < 1e-6  # the smooth (left) side is reproduced
    # a smooth cell keeps the central polynomial's accuracy (weights near the average)
    x = np.array([-h, 0, h])
    f = lambda x: np.sin(3 * x)
    avg = lambda xc: (np.cos(3 * (xc - h / 2)) - np.cos(3 * (xc + h / 2))) / (3 * h)
    p = oracle.recon1d_scalar(avg(0), avg(h), avg(-h), f(h / 2), f(-h / 2), h)
    assert abs(p[0] - 3.0) < 1e-3


@pytest.mark.parametrize("seed", range(3))
def test_equilibrium_poly_exact_on_quadratics(oracle, seed):
    rng = np.random.default_rng(20 + seed)
    c, U, avg = _quad2d(rng)
    h, k = 0.06, 0.045
    Ueq = np.zeros((2, 3, 1))
    for m in range(2):
        for n in range(3):
            Ueq[m, n, 0] = avg((m - 0.5) * h, (n - 1) * k, h, k)
    q = oracle.equilibrium_poly(2, np.repeat(Ueq, 4, axis=2), np.full(4, U(0, 0)), h, k)
    # U0 + b2 x + b3 y + b4 x^2/2 + b5 y^2/2 + b6 x y
    np.testing.assert_allclose(q[:, 0], [c[1], c[2], 2 * c[3], 2 * c[4], c[5]], rtol=1e-9, atol=1e-9)


def test_equilibrium_poly_1d_exact(oracle):
    a, b, cc = 0.3, -1.2, 2.5
    h = 0.05
    U = lambda x: a + b * x + cc * x * x
    avg = lambda xc: U(xc) + cc * h * h / 12
    Ueq = np.zeros((2, 3, 3))
    Ueq[0, 1, :] = avg(-h / 2)
    Ueq[1, 1, :] = avg(h / 2)
    q = oracle.equilibrium_poly(1, Ueq, np.full(3, U(0)), h, 1.0)
    np.testing.assert_allclose(q[0], b, rtol=1e-12)
    np.testing.assert_allclose(q[2], 2 * cc, rtol=1e-10)


# --------------------------------------------------------------------------
# The choice of the cross derivative (Sec. 3.2) under mirror images
# --------------------------------------------------------------------------

def _stencil_args(rng, jumpy=True):
    """Thirteen stencil values (Uc, Ue, Uw, Un, Us, E+, E-, W+, W-, N+, N-,
    S+, S-) of rough data: random with jumps of order one."""
    return list(rng.normal(size=13) * (1.0 if jumpy else 1e-3) + 1.0)


def _mirror_y(a):
    Uc, Ue, Uw, Un, Us, Ep, Em, Wp, Wm, Np, Nm, Sp, Sm = a
    # y -> -y: north and south swap, the two Gauss points of the x interfaces swap
    return [Uc, Ue, Uw, Us, Un, Em, Ep, Wm, Wp, Sp, Sm, Np, Nm]


def _mirror_x(a):
    Uc, Ue, Uw, Un, Us, Ep, Em, Wp, Wm, Np, Nm, Sp, Sm = a
    return [Uc, Uw, Ue, Un, Us, Wp, Wm, Ep, Em, Nm, Np, Sm, Sp]


@pytest.mark.parametrize("seed", range(20))
def test_recon2d_commutes_with_mirror_images(oracle, seed):
    """The Euler equations and the stencils of Sec. 3.2 are symmetric under
    x -> -x and y -> -y, so the reconstruction of mirrored data is the mirrored
    reconstruction: p3, p6 change sign under y -> -y; p2, p6 under x -> -x;
    the rest are unchanged, bit for bit (every step is an exact negation).
    Half of the cases are built with ties between the cross-derivative
    candidates (data symmetric in y), where the choice must give zero."""
    rng = np.random.default_rng(100 + seed)
    h, k = 0.03, 0.02
    a = _stencil_args(rng)
    if seed % 2:
        a = _mirror_y(a)
        b = _stencil_args(rng)
        # symmetric in y: Un = Us, E+ = E-, W+ = W-, N+- = S+-
        a[4], a[6], a[8], a[11], a[12] = a[3], a[5], a[7], a[9], a[10]
    p = oracle.recon2d_scalar(*a, h, k)
    py = oracle.recon2d_scalar(*_mirror_y(a), h, k)
    px = oracle.recon2d_scalar(*_mirror_x(a), h, k)
    np.testing.assert_array_equal(py, p * np.array([1, -1, 1, 1, -1]))
    np.testing.assert_array_equal(px, p * np.array([-1, 1, 1, 1, -1]))
    if seed % 2:
        assert p[4] == 0.0 and p[1] == 0.0


def test_recon2d_y_uniform_jump_has_no_cross_term(oracle):
    """A jump across x in data that do not vary with y: every cross-derivative
    candidate has the same magnitude, two of each sign; the polynomial must
    not vary with y (p3 = p6 = 0), whereas taking the first candidate would
    give p6 = +-|a6|."""
    h = k = 0.01
    d = S3 / 6
    # the jump sits between the cell and its east neighbour, off the Gauss points
    U = lambda x: np.where(x < 0.3 * h, 1.0, 0.125)
    Uc = (0.8 * 1.0 + 0.2 * 0.125)
    p = oracle.recon2d_scalar(Uc, 0.125, 1.0, Uc, Uc, 0.125, 0.125, 1.0, 1.0,
                              float(U(d * h)), float(U(-d * h)), float(U(d * h)), float(U(-d * h)), h, k,
                              1e-14, 1e-12)
    assert p[1] == 0.0 and p[4] == 0.0
    assert p[0] != 0.0


# --------------------------------------------------------------------------
# Characteristic variables in 2D
# --------------------------------------------------------------------------

def _euler_flux(U, ax, g=1.4):
    rho, m, n, E = U
    p = (g - 1.0) * (E - 0.5 * (m * m + n * n) / rho)
    un = (m if ax == 0 else n) / rho
    return np.array([rho * un, m * un + (p if ax == 0 else 0.0), n * un + (p if ax == 1 else 0.0),
                     (E + p) * un])


def _jacobian(U, ax, g=1.4):
    """dF/dU by the complex step (exact to rounding: no subtraction)."""
    J = np.zeros((4, 4))
    for j in range(4):
        Uz = np.array(U, dtype=complex)
        Uz[j] += 1e-30j
        J[:, j] = _euler_flux(Uz, ax, g).imag / 1e-30
    return J


def _random_state(rng, g=1.4):
    from paper_1412_4489_amd import workloads as W
    rho, p = rng.uniform(0.1, 5.0, size=2)
    u, v = rng.normal(size=2) * 2.0
    return W.cons(g, rho, u, v, p)


@pytest.mark.parametrize("ax", [0, 1])
@pytest.mark.parametrize("seed", range(4))
def test_euler_eigvec_2d_diagonalises_the_flux_jacobian(oracle, ax, seed):
    rng = np.random.default_rng(300 + seed)
    g = 1.4
    Wc = _random_state(rng, g)
    R = oracle.euler_eigvec_2d(g, Wc, ax)
    J = _jacobian(Wc, ax, g)
    rho, u, v = Wc[0], Wc[1] / Wc[0], Wc[2] / Wc[0]
    p = (g - 1.0) * (Wc[3] - 0.5 * rho * (u * u + v * v))
    c, un = np.sqrt(g * p / rho), (u if ax == 0 else v)
    lam = np.array([un - c, un, un, un + c])
    np.testing.assert_allclose(J @ R, R * lam[None, :], rtol=1e-12, atol=1e-12 * np.abs(J).max())
    assert abs(np.linalg.det(R)) > 1e-6


def _quad_fields(rng, g=1.4):
    """Quadratic conservative fields around a physical state."""
    base = _random_state(rng, g)
    cs = [rng.normal(size=6) * np.array([1.0, 0.5, 0.5, 0.3, 0.3, 0.3]) * 0.2 * abs(b) for b in base]
    for v in range(4):
        cs[v][0] = base[v]
    return cs


def _stencil_from(fun_avg, fun, h, k):
    d = S3 / 6
    return [fun_avg(0, 0), fun_avg(h, 0), fun_avg(-h, 0), fun_avg(0, k), fun_avg(0, -k),
            fun(h / 2, d * k), fun(h / 2, -d * k), fun(-h / 2, d * k), fun(-h / 2, -d * k),
            fun(d * h, k / 2), fun(-d * h, k / 2), fun(d * h, -k / 2), fun(-d * h, -k / 2)]


@pytest.mark.parametrize("weights", [(1e-6, 10.0), (1e-14, 1e-12)], ids=["default", "one_sided"])
@pytest.mark.parametrize("seed", range(3))
def test_recon2d_characteristic_exact_on_quadratics(oracle, weights, seed):
    """The transforms are linear, so quadratic data stay quadratic in every
    characteristic field and the limiter keeps them; mapping back must give
    the quadratic's coefficients (a wrong inverse or a transposed product
    fails this)."""
    rng = np.random.default_rng(400 + seed)
    h, k = 0.05, 0.04
    cs = _quad_fields(rng)
    S = np.zeros((13, 4))
    for v, c in enumerate(cs):
        U = lambda x, y, c=c: c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * y * y + c[5] * x * y
        avg = lambda x, y, c=c, U=U: U(x, y) + c[3] * h * h / 12 + c[4] * k * k / 12
        S[:, v] = _stencil_from(avg, U, h, k)
    pc, rc = oracle.recon2d_cell(S, h, k, vars=1, eps=weights[0], Cw=weights[1])
    assert rc == 0
    for v, c in enumerate(cs):
        np.testing.assert_allclose(pc[v], [c[1], c[2], 2 * c[3], 2 * c[4], c[5]], rtol=1e-8,
                                   atol=1e-8 * np.abs(c).max())


def test_recon2d_conservative_cell_is_per_component(oracle):
    rng = np.random.default_rng(7)
    S = rng.normal(size=(13, 4)) + 2.0
    pc, rc = oracle.recon2d_cell(S, 0.02, 0.03, vars=0, Cw=10.0)
    for v in range(4):
        np.testing.assert_array_equal(pc[v], oracle.recon2d_scalar(*S[:, v], 0.02, 0.03, 1e-6, 10.0))


@pytest.mark.parametrize("ax", [0, 1])
@pytest.mark.parametrize("seed", range(4))
def test_recon2d_characteristic_limits_each_wave_as_a_scalar(oracle, ax, seed):
    """Data made of simple waves of the flux Jacobian at the cell average
    along one axis -- U = Wc + sum_r alpha_r(s) r_r, s the coordinate along
    that axis, the alpha_r rough profiles with jumps and zero average on the
    cell itself (so that Wc is the cell average), the r_r eigenvectors of the
    complex-step Jacobian at Wc (an independent basis; one vector of the
    double eigenvalue) -- are limited wave by wave: the limited pair of that
    axis (p2, p4 for x; p3, p5 for y, with the weights giving the one-sided
    polynomial) is sum_r lim(alpha_r) r_r, lim being the scalar
    reconstruction of the profile.  Limiting in conservative variables
    gives another answer on the same data."""
    rng = np.random.default_rng(500 + seed)
    g = 1.4
    h, k = 0.02, 0.02
    Wc = _random_state(rng, g)
    lam, vec = np.linalg.eig(_jacobian(Wc, ax, g))
    vec = vec[:, np.argsort(lam.real)].real
    waves = [vec[:, 0], vec[:, 1], vec[:, 3]]  # un - c, one of the un pair, un + c
    d = S3 / 6
    profiles = []
    for r in range(3):
        a, b = rng.normal(size=2) * 0.05
        jump = rng.normal() * 0.05
        xj = rng.choice([-0.8, -0.3, 0.3, 0.8, 1.4, -1.3]) * h
        f = lambda s, a=a, b=b, jump=jump, xj=xj: a * s + b * s * s + jump * (s > xj)
        # cell average of the profile over [s0 - h/2, s0 + h/2]
        favg = lambda s0, a=a, b=b, jump=jump, xj=xj: (a * s0 + b * (s0 * s0 + h * h / 12)
                                                       + jump * np.clip((s0 + h / 2 - xj) / h, 0.0, 1.0))
        if ax == 0:
            vals = [favg(0), favg(h), favg(-h), favg(0), favg(0), f(h / 2), f(h / 2), f(-h / 2), f(-h / 2),
                    f(d * h), f(-d * h), f(d * h), f(-d * h)]
        else:
            vals = [favg(0), favg(0), favg(0), favg(k), favg(-k), f(d * k), f(-d * k), f(d * k), f(-d * k),
                    f(k / 2), f(k / 2), f(-k / 2), f(-k / 2)]
        vals = np.array(vals, dtype=float)
        profiles.append(vals - vals[0])
    S = Wc[None, :] + sum(np.outer(pr, r) for pr, r in zip(profiles, waves))
    assert np.array_equal(S[0], Wc)
    weights = dict(eps=1e-14, Cw=1e-12)
    pc, rc = oracle.recon2d_cell(S, h, k, gamma=g, vars=1, **weights)
    assert rc == 0
    expect = np.zeros((4, 2))
    for pr, r in zip(profiles, waves):
        ps = oracle.recon2d_scalar(*[float(x) for x in pr], h, k, weights["eps"], weights["Cw"])
        expect += np.outer(r, (ps[0], ps[2]) if ax == 0 else (ps[1], ps[3]))
    got = pc[:, [0, 2]] if ax == 0 else pc[:, [1, 3]]
    # rounding: the transforms carry Wc (of order ten) next to data of order
    # 0.05, and the second derivative divides by h^2
    np.testing.assert_allclose(got, expect, rtol=0, atol=1e-9 * np.abs(expect).max())
    cons, _ = oracle.recon2d_cell(S, h, k, gamma=g, vars=0, **weights)
    got_c = cons[:, [0, 2]] if ax == 0 else cons[:, [1, 3]]
    assert np.abs(got_c - expect).max() > 1e-3 * np.abs(expect).max()


def test_recon2d_cross_derivative_near_ties(oracle):
    """Ties of the cross-derivative candidates (Sec. 3.2, smallest |a6|) are
    taken up to the rounding noise of FP64 inputs: a relative perturbation d of
    the Gauss values and slopes moves a candidate by at most d M,
    M = sqrt(3) sum|G| / (h k) + |a2| / k + |a3| / h, and candidates within
    2^-46 M of the smallest magnitude count as tied (zero when both signs
    are among them).  A y-uniform jump has candidates +-3500: perturbing one
    north Gauss value so that one candidate moves by half the band keeps the
    tie (a6 = 0, only the central polynomial's share, weighted ~1e-24, is
    left); by twice the band the smallest candidate wins.  A rounding-level
    perturbation (1e-15) is a tie, one of 1e-12 is not."""
    h = k = 0.01
    d = S3 / 6
    U = lambda x: 1.0 if x < 0.3 * h else 0.125
    Uc = 0.8 * 1.0 + 0.2 * 0.125
    base = [Uc, 0.125, 1.0, Uc, Uc, 0.125, 0.125, 1.0, 1.0, U(d * h), U(-d * h), U(d * h), U(-d * h)]
    # the limited slopes of the base data: a2 from the x pair, a3 = 0
    p0 = oracle.recon2d_scalar(*base, h, k, 1e-14, 1e-12)
    a2 = p0[0]
    M = S3 * sum(abs(x) for x in base[5:]) / (h * k) + abs(a2) / k
    band = 2.0 ** -46 * M
    # a north Gauss value enters the NE / NW candidates with weight sqrt(3)/(h k)
    step = S3 / (h * k)
    for eps, zero in ((0.0, True), (1e-15, True), (0.5 * band / step, True), (2.0 * band / step, False),
                      (1e-12, False), (1e-6, False)):
        a = list(base)
        a[9] += eps
        p = oracle.recon2d_scalar(*a, h, k, 1e-14, 1e-12)
        if zero:
            assert abs(p[4]) < 1e-20, (eps, p[4])
        else:
            assert abs(p[4]) > 1e3, (eps, p[4])
