"""Linearised Navier-Stokes solutions for the decay tests (independent of the
scheme): a shear wave and an entropy wave of wavenumber k on a uniform gas
at rest (rho = p = T = 1, gas constant 1).  The longitudinal system (density,
velocity along k, temperature) is integrated exactly through its
eigen-decomposition, with the heat conductivity kappa = c_p mu / Pr and the
longitudinal viscosity (2 - 2/N) mu of the BGK model with N = K + 2
translational and internal degrees of freedom in 2D (N = 5 for gamma = 1.4):
its Chapman-Enskog stress is mu (du_i/dx_j + du_j/dx_i - (2/N) delta_ij div u),
which carries a bulk viscosity beside the two-dimensional shear viscosity."""
import numpy as np


def shear_rate(mu, k=2 * np.pi, rho=1.0):
    """decay rate of the transverse velocity of a shear wave"""
    return mu / rho * k * k


def entropy_wave_temperature(mu, prandtl, t, gamma=1.4, k=2 * np.pi):
    """Amplitude of T' (relative to its initial amplitude) at time t for the
    initial data T' = a sin(kx), rho' = -a sin(kx), u' = 0 (uniform pressure)."""
    cv = 1.0 / (gamma - 1.0)
    cp = gamma / (gamma - 1.0)
    kappa = cp * mu / prandtl
    n_dof = 2.0 / (gamma - 1.0)  # N = K + 2 with gamma = (N + 2) / N
    nu_l = (2.0 - 2.0 / n_dof) * mu
    # perturbations ~ exp(i k x): d/dt (rho, u, T) = A (rho, u, T), p' = rho' + T'
    A = np.array([[0.0, -1j * k, 0.0],
                  [-1j * k, -nu_l * k * k, -1j * k],
                  [0.0, -1j * k / cv, -kappa * k * k / cv]], dtype=complex)
    w, V = np.linalg.eig(A)
    c = np.linalg.solve(V, np.array([-1.0, 0.0, 1.0], dtype=complex))
    return float((V @ (c * np.exp(w * t)))[2].real)


def density_wave_amplitude(mu, t, gamma=1.4, k=np.pi, prandtl=1.0):
    """|rho'(t)| / |rho'(0)| of the Fourier mode k for the initial data
    rho' = a sin(kx), T' = -a sin(kx), u' = 0 (an entropy wave at uniform
    pressure; in the frame moving with the mean flow), with the same
    longitudinal system: heat conduction turns part of it into two weak sound
    waves, and the modulus of the complex density amplitude counts both."""
    cv = 1.0 / (gamma - 1.0)
    cp = gamma / (gamma - 1.0)
    kappa = cp * mu / prandtl
    n_dof = 2.0 / (gamma - 1.0)
    nu_l = (2.0 - 2.0 / n_dof) * mu
    A = np.array([[0.0, -1j * k, 0.0],
                  [-1j * k, -nu_l * k * k, -1j * k],
                  [0.0, -1j * k / cv, -kappa * k * k / cv]], dtype=complex)
    w, V = np.linalg.eig(A)
    c = np.linalg.solve(V, np.array([1.0, 0.0, -1.0], dtype=complex))
    return float(abs((V @ (c * np.exp(w * t)))[0]))
