"""Parity of the 1D HIP path (Sec. 3.1 reconstruction, fused interface,
update) with the FP64 oracle, through the C ABI.

Tolerances as in test_gpu_parity: GKS_FP64 1e-11 relative to the field's
magnitude (same formulas, different evaluation order), GKS_FP32_MIXED 5e-6
after tens of steps on smooth data (single-precision correction terms over
double-precision leading terms).  The 1D characteristic variables use the
closed-form left eigenvectors on the GPU and a numerical inverse in the
oracle, so their branch decisions agree up to rounding-level near-ties; the
discontinuous cases are compared step by step from the oracle's state."""
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


def _rel(a, b):
    scale = np.abs(b).max(axis=tuple(range(1, b.ndim)), keepdims=True)
    assert np.isfinite(a).all()
    return float((np.abs(a - b) / scale).max())


CASES = {
    "advection": lambda: W.advection_1d(100),
    "advection_tau": lambda: W.advection_1d(64, tau_eps=0.05),
    "sod_char": lambda: W.sod_1d(100),
    "sod_cons": lambda: W.sod_1d(100, recon_vars=0),
    "blast_char": lambda: W.blast_1d(400),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
def test_parity_1d_one_step(G, oracle, case, prec):
    prob, st = CASES[case]()
    dt = 0.8 * oracle.dt(prob, st)
    ref = st.copy()
    oracle.step(prob, ref, dt, 0.0)
    p = G.GKS_FP64 if prec == "fp64" else G.GKS_FP32_MIXED
    with G.Solver(prob, st, p) as S:
        S.step(1, dt=dt)
        got, t, n = S.fetch()
    assert n == 1 and t == pytest.approx(dt, rel=1e-15)
    tol = 1e-11 if prec == "fp64" else 2e-6
    assert _rel(got.cell, ref.cell) < tol
    assert _rel(got.fx, ref.fx) < 10 * tol


@pytest.mark.parametrize("prec, tol", [("fp64", 1e-11), ("fp32_mixed", 5e-6)])
def test_parity_1d_advection_free_running(G, oracle, prec, tol):
    prob, st = W.advection_1d(100)
    dt = oracle.dt(prob, st)
    ref = st.copy()
    for n in range(40):
        oracle.step(prob, ref, dt, n * dt)
    p = G.GKS_FP64 if prec == "fp64" else G.GKS_FP32_MIXED
    with G.Solver(prob, st, p) as S:
        S.step(40, dt=dt)
        got, t, n = S.fetch()
    assert n == 40
    assert _rel(got.cell, ref.cell) < tol
    assert _rel(got.fx, ref.fx) < 10 * tol


@pytest.mark.parametrize("case, nsteps", [("sod_char", 6), ("sod_cons", 6), ("blast_char", 6)])
def test_parity_1d_per_step(G, oracle, case, nsteps):
    """Shocked 1D data, compared step by step from the oracle's state."""
    prob, st = CASES[case]()
    t = 0.0
    for n in range(nsteps):
        dt = 0.8 * oracle.dt(prob, st)  # from the present state: the flow speeds up
        ref = st.copy()
        oracle.step(prob, ref, dt, t)
        with G.Solver(prob, st, G.GKS_FP64, t0=t) as S:
            S.step(1, dt=dt)
            got, _, _ = S.fetch()
        assert _rel(got.cell, ref.cell) < 1e-11, f"step {n}"
        assert _rel(got.fx, ref.fx) < 1e-10, f"step {n}"
        st, t = ref, t + dt


def test_advection_full_run_cfl05(G, oracle):
    """Config of Table 1 at N = 100: CFL 0.5 from the device's own CFL
    condition every step, to t = 2 (one period); GPU FP64 against the oracle
    run the same way, and both against the exact cell averages."""
    prob, st = W.advection_1d(100, cfl=0.5)
    ref, t, nref = st.copy(), 0.0, 0
    while t < 2.0 - 1e-14:
        dt = min(oracle.dt(prob, ref), 2.0 - t)
        oracle.step(prob, ref, dt, t)
        t += dt
        nref += 1
    with G.Solver(prob, st, G.GKS_FP64) as S:
        S.step(nref + 5, t_end=2.0)
        got, tg, n = S.fetch()
    assert n == nref and tg == pytest.approx(2.0, rel=1e-14)
    rel_l1 = np.abs(got.cell[0] - ref.cell[0]).mean() / np.abs(ref.cell[0]).mean()
    assert rel_l1 < 1e-12
    exact = W.advection_1d_exact_average(100, 2.0)
    e_gpu = np.abs(got.cell[0, 0] - exact).mean()
    e_orc = np.abs(ref.cell[0, 0] - exact).mean()
    assert e_gpu == pytest.approx(e_orc, rel=1e-6)
    assert e_gpu < 1e-4


def test_blast_wave_full_run(G, oracle):
    """Sec. 4.2 blast wave, 400 cells, characteristic variables, CFL 0.2 from
    each side's own CFL condition, to t = 3.8: GPU FP64 against the oracle
    (relative L1 of the density; limiter branches may flip on rounding-level
    differences over thousands of steps of shocked data)."""
    prob, st = W.blast_1d(400)
    ref = st.copy()
    n, t = oracle.run(prob, ref, t_end=3.8)
    with G.Solver(prob, st, G.GKS_FP64) as S:
        S.step(n + 200, t_end=3.8)
        got, tg, ng = S.fetch()
    assert tg == pytest.approx(3.8, rel=1e-14) and abs(ng - n) <= 2
    l1 = np.abs(got.cell[0] - ref.cell[0]).mean() / np.abs(ref.cell[0]).mean()
    assert l1 < 1e-3
