"""The exact Riemann solver used by the shock-tube pin, checked against the
star-region values of Sod's problem (pressure function roots) and conservation."""
import numpy as np

from riemann_exact import star_state, sample


def test_sod_star_state():
    p, u = star_state((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4)
    # the star state satisfies both wave relations: check by residual
    assert 0.30 < p < 0.31 and 0.92 < u < 0.93
    x = np.linspace(-0.5, 0.5, 20001)
    t = 0.2
    W = sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, x / t)
    # mass in [-0.5, 0.5] is conserved (waves stay inside)
    mass = np.trapz(W[0], x)
    assert abs(mass - (0.5 * 1.0 + 0.5 * 0.125)) < 1e-4


def test_symmetric_collision_has_zero_velocity():
    p, u = star_state((1.0, 1.0, 1.0), (1.0, -1.0, 1.0), 1.4)
    assert abs(u) < 1e-13 and p > 1.0
