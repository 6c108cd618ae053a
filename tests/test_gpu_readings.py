"""GPU checks of two readings of the paper against the oracle and the
mathematics, through the C ABI:

* the inviscid collision time tau = tau_eps dt (Sec. 4) acts as a
  Navier-Stokes viscosity mu = tau_eff p with
  tau_eff = tau - tau^2 (1 - e^(-dt/tau)) / dt: the density wave of Table 1
  decays, relative to the run with tau_eps = 0, like the linearised
  Navier-Stokes solution with that viscosity (tests/linear_ns.py);
* the admissibility fallback of the reconstruction (robust reconstruction is
  left open at the end of Sec. 3.3) fires on the same cells as in the oracle:
  the per-problem count of (cell, step) fallbacks equals the oracle's on the
  double Mach reflection (Sec. 4.5) in the double-precision form."""
import numpy as np
import pytest

from paper_1412_4489_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1412_4489_amd import gks
    gks.lib()
    return gks


def _advected_amplitude(prob, cell, t):
    x = prob.x0 + (np.arange(prob.nx) + 0.5) * prob.dx
    r = cell[0].reshape(-1) - 1.0
    return np.hypot(2 * np.mean(r * np.sin(np.pi * (x - t))), 2 * np.mean(r * np.cos(np.pi * (x - t))))


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("tau_eps", [0.05, 0.5])
def test_tau_eps_heat_conduction_on_the_gpu(G, oracle, prec, tau_eps):
    from linear_ns import density_wave_amplitude
    p = G.GKS_FP64 if prec == "fp64" else G.GKS_FP32_MIXED
    amps = {}
    for te in (0.0, tau_eps):
        prob, st = W.advection_1d(100, cfl=0.5, tau_eps=te, amp=1e-3)
        dt = oracle.dt(prob, st)
        n = int(round(2.0 / dt))
        dt = 2.0 / n
        a0 = _advected_amplitude(prob, st.cell, 0.0)
        with G.Solver(prob, st, p) as S:
            S.step(n, dt=dt)
            got, t, steps = S.fetch()
        assert steps == n
        amps[te] = _advected_amplitude(prob, got.cell, 2.0) / a0
    rate = -np.log(amps[tau_eps] / amps[0.0]) / 2.0
    tau = tau_eps * dt
    tau_eff = tau - tau * tau * (1.0 - np.exp(-dt / tau)) / dt
    exact = -np.log(density_wave_amplitude(tau_eff, 2.0, gamma=prob.gamma)) / 2.0
    assert abs(rate / exact - 1.0) < 5e-3, (rate, exact)


def test_fallback_count_matches_the_oracle(G, oracle):
    """Double Mach reflection 96 x 24, admissibility 1, 60 fixed steps from
    the initial state: the GPU's count of reconstruction fallbacks (summed
    over cells and steps) is the oracle's; with admissibility 0 the smooth
    vortex never falls back."""
    prob, st = W.dmr(96, 24)
    ref = st.copy()
    dt = oracle.dt(prob, st)
    fb = 0
    for k in range(60):
        oracle.step(prob, ref, dt, k * dt)
        fb += oracle.last_fallbacks()
    assert fb > 0
    with G.Solver(prob, st, G.GKS_FP64) as S:
        S.step(60, dt=dt)
        got, t, n = S.fetch()
        assert S.fallbacks() == fb
    assert np.abs(got.cell - ref.cell).max() < 1e-9 * np.abs(ref.cell).max()
    prob, st = W.vortex_2d(32)
    with G.Solver(prob, st, G.GKS_FP32_MIXED) as S:
        S.step(20)
        S.fetch()
        assert S.fallbacks() == 0
