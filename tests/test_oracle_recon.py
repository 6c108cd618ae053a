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
