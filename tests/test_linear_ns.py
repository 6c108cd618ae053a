"""Pins of the linearised Navier-Stokes reference (tests/linear_ns.py)."""
import numpy as np

from linear_ns import density_wave_amplitude, entropy_wave_temperature, shear_rate


def test_no_dissipation_keeps_the_entropy_wave():
    # uniform pressure, no conduction: a steady entropy wave, no acoustics
    for t in (0.1, 0.5, 2.0):
        assert abs(entropy_wave_temperature(0.0, 1.0, t) - 1.0) < 1e-12


def test_long_waves_decay_at_the_conduction_rate():
    # k -> 0 (here: small mu relative to c / k): rate -> kappa k^2 / (rho c_p) = mu k^2 / Pr
    mu, k = 1e-5, 2 * np.pi
    for pr in (1.0, 0.72):
        t = 2.0 / (mu * k * k / pr)  # two e-foldings
        rate = -np.log(entropy_wave_temperature(mu, pr, t)) / t
        assert abs(rate / (mu * k * k / pr) - 1.0) < 1e-4


def test_shear_rate():
    assert abs(shear_rate(0.01) - 0.01 * 4 * np.pi ** 2) < 1e-15


def test_density_wave_amplitude_limits():
    # no dissipation: the entropy wave stands (advected) at its amplitude
    for t in (0.1, 2.0):
        assert abs(density_wave_amplitude(0.0, t) - 1.0) < 1e-12
    # long waves: the conduction rate mu k^2 / Pr (rho = p = 1)
    mu, k = 1e-6, np.pi
    for pr in (1.0, 0.72):
        t = 2.0 / (mu * k * k / pr)
        rate = -np.log(density_wave_amplitude(mu, t, k=k, prandtl=pr)) / t
        assert abs(rate / (mu * k * k / pr) - 1.0) < 1e-4
