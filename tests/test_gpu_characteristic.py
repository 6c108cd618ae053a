"""The 2D reconstruction in characteristic variables (recon_vars = 1) on the
GPU, and the discontinuous problems of Sec. 4.2 - 4.4 at the paper's
resolutions.

* Parity with the oracle step by step (each step from the oracle's state, as
  for the other discontinuous cases: a limiter decision near a tie may go
  either way on rounding-level differences) on the 2D Riemann problems, the
  double Mach reflection, the shock-vortex interaction and Sod's problem in a
  channel along x and along y; FP64 to 1e-11 of each field, FP32-mixed to
  1e-6 (one step).
* Invariants the mathematics fixes: Sod's problem in a channel stays uniform
  across it with no transverse momentum, and is Sod's profile; the
  stationary shock of Sec. 4.4 stays at x = 0.5 with the mass in the domain
  conserved.
* Riemann cases 1 and 2 at 200^2 and 400^2 and the shock-vortex interaction
  at 201 x 101, 401 x 201 and 801 x 401 cells to the paper's end times: every
  state physical, and one further step from the final state matches the
  oracle's step of the same full-size grid.
"""
import numpy as np
import pytest

from paper_1412_4489_amd import workloads as W
from parity_bounds import one_step

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
    """max |a - b| relative to each component's magnitude; the two momentum
    components share the magnitude of the momentum vector (a channel flow has
    no transverse momentum in the oracle, and the GPU's contracted
    multiply-adds leave it at the rounding level of the momentum)"""
    assert np.isfinite(a).all() and np.isfinite(b).all()
    vax = b.ndim - 3
    scale = np.abs(b).max(axis=tuple(k for k in range(b.ndim) if k != vax), keepdims=True)
    idx = [slice(None)] * b.ndim
    idx[vax] = slice(1, 3)
    scale[tuple(idx)] = scale[tuple(idx)].max()
    return float((np.abs(a - b) / np.maximum(scale, 1e-300)).max())


def _across(c, axis=1):
    """largest variation across a channel and largest transverse momentum,
    relative to the magnitudes of the fields"""
    scale = np.abs(c).max(axis=(1, 2))
    scale[1:3] = scale[1:3].max()
    var = (np.ptp(c, axis=axis) / scale[:, None]).max()
    return float(var), float(np.abs(c[2]).max() / scale[2])


def _steps_for(prob, st, t_end):
    """A step count that reaches t_end (twice the count at the initial CFL
    step: the waves of these problems do not speed up by more); the steps
    after t_end are empty."""
    import oracle
    return int(2.0 * t_end / oracle.dt(prob, st)) + 50


def _physical(prob, c):
    pr = (prob.gamma - 1.0) * (c[3] - 0.5 * (c[1] ** 2 + c[2] ** 2) / c[0])
    return bool((c[0] > 0).all() and (pr > 0).all())


CASES = {
    "riemann1": lambda: W.riemann_2d(1, n=30, recon_vars=1),
    "riemann2": lambda: W.riemann_2d(2, n=28, nx=31, recon_vars=1),
    "dmr": lambda: W.dmr(48, 12, recon_vars=1),
    "shock_vortex": lambda: W.shock_vortex(60, 30),
    "sod_x": lambda: W.sod_2d(60, 4, axis=0),
    "sod_y": lambda: W.sod_2d(60, 5, axis=1),
}


@pytest.mark.parametrize("case", list(CASES))
def test_characteristic_parity_fp64_per_step(G, oracle, case):
    prob, st = CASES[case]()
    assert prob.recon_vars == 1
    dt = 0.8 * oracle.dt(prob, st)
    t = 0.0
    print(f"characteristic {case} fp64", flush=True)
    for n in range(4):
        ref = st.copy()
        oracle.step(prob, ref, dt, t)
        with G.Solver(prob, st, G.GKS_FP64, t0=t) as S:
            S.step(1, dt=dt)
            got, tg, steps = S.fetch()
        assert _rel(got.cell, ref.cell) < 1e-11, n
        assert _rel(got.fx, ref.fx) < 1e-10, n
        assert _rel(got.fy, ref.fy) < 1e-10, n
        st, t = ref, t + dt


@pytest.mark.parametrize("case", list(CASES))
def test_characteristic_parity_fp32_mixed(G, oracle, case):
    """One step: the derivative terms in single precision (unit roundoff
    6e-8) on discontinuous data."""
    prob, st = CASES[case]()
    dt = 0.8 * oracle.dt(prob, st)
    ref = st.copy()
    oracle.step(prob, ref, dt, 0.0)
    print(f"characteristic {case} fp32_mixed", flush=True)
    with G.Solver(prob, st, G.GKS_FP32_MIXED) as S:
        S.step(1, dt=dt)
        got, tg, steps = S.fetch()
    assert _rel(got.cell, ref.cell) < 1e-6
    # point values on the interfaces the Mach 10 shock crosses: the
    # correction terms of the point-value update are as large as the value,
    # and single precision leaves up to 3e-4 of the field there (as in the
    # conservative form)
    ptol = 1e-3 if case == "dmr" else 1e-5
    assert _rel(got.fx, ref.fx) < ptol
    assert _rel(got.fy, ref.fy) < ptol


def test_mixed_reconstruction_kinds_in_one_handle(G, oracle):
    """Conservative and characteristic 2D problems of both precisions in one
    handle (two reconstruction launches per precision) match each problem's
    oracle step."""
    items = [W.riemann_2d(1, n=12, recon_vars=0), W.riemann_2d(1, n=12, recon_vars=1),
             W.shock_vortex(40, 20), W.vortex_2d(16), W.sod_1d(30)]
    probs, states = [p for p, _ in items], [s for _, s in items]
    precs = [G.GKS_FP64, G.GKS_FP64, G.GKS_FP32_MIXED, G.GKS_FP32_MIXED, G.GKS_FP64]
    dts = [0.7 * oracle.dt(p, s) for p, s in items]
    refs = []
    for p, s, dt in zip(probs, states, dts):
        r = s.copy()
        oracle.step(p, r, dt, 0.0)
        refs.append(r)
    with G.Solver(probs, states, precs) as S:
        S.step(1, dt=dts)
        for k, (p, r) in enumerate(zip(probs, refs)):
            got, t, n = S.fetch(k)
            tol = 1e-11 if precs[k] == G.GKS_FP64 else 1e-6
            assert _rel(got.cell, r.cell) < tol, p.name
    # the two Riemann problems differ only in the reconstruction variables
    assert not np.array_equal(refs[0].cell, refs[1].cell)


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("vars_", [0, 1], ids=["conservative", "characteristic"])
def test_sod_channel_invariants(G, prec, vars_):
    """Sod's problem (Sec. 4.2) along a periodic channel to t = 0.2: nothing
    varies across the channel and the transverse momentum stays zero up to
    rounding -- the choice of the cross derivative gives zero on the
    symmetric ties; the first choice would give 1e-4 -- and the density is
    Sod's profile (L1 error against the exact solution and overshoot as in
    1D)."""
    import sys
    import os
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from riemann_exact import cell_average_density
    p = G.GKS_FP64 if prec == "fp64" else G.GKS_FP32_MIXED
    prob, st = W.sod_2d(100, 4, 0, recon_vars=vars_)
    with G.Solver(prob, st, p) as S:
        S.step(_steps_for(prob, st, 0.2), t_end=0.2)
        got, t, n = S.fetch()
    assert t == pytest.approx(0.2, rel=0, abs=1e-14)
    c = got.cell
    # (the oracle keeps these exactly zero; the GPU's contracted multiply-adds
    # are not mirror-symmetric bit for bit: rounding of the double, or in the
    # mixed form of the single-precision terms)
    var, trans = _across(c)
    print(f"across the channel: variation {var:.1e}, transverse momentum {trans:.1e}", flush=True)
    bound = 1e-13 if prec == "fp64" else 1e-6
    assert var < bound and trans < bound, (var, trans)
    assert np.abs(got.fy[:, 2]).max() < bound * np.abs(got.fy[:, 1:3]).max()
    rho = c[0, 0]
    ex = cell_average_density((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, 0.5, t, np.linspace(0, 1, 101))
    assert np.abs(rho - ex).mean() < 6e-3
    assert rho.min() > 0.98 * 0.125 and rho.max() < 1.02


def test_stationary_shock_on_the_gpu(G):
    """The shock of Sec. 4.4 without the vortex on 201 x 101 cells to t = 0.3:
    mass conserved (the two boundary mass fluxes are equal up to the small
    disturbance the kinetic flux carries upstream), the shock stays at
    x = 0.5 within a quarter cell, and nothing varies across the channel
    beyond rounding (FP64 3e-15; FP32-mixed 3e-8: the interfaces along the
    channel carry the single-precision rounding of the correction terms in
    their odd components, which the slip walls, symmetry lines, set to
    zero, so the rows beside the walls differ from the others at that
    level; the rows were bit-equal before the walls were made exact
    symmetry lines).  With bit-equal ties
    only in the cross-derivative choice, the rounding of the GPU's contracted
    multiply-adds picked one sign of a spurious cross derivative near the
    shock and the variation grew to 6e-5, as in the oracle seeded with
    relative noise of 1e-15; with the tie band the seeded oracle stays at
    4e-15."""
    M = W.SHOCK_VORTEX_MACH
    r1 = M * M
    r2 = r1 * 2.4 * M * M / (0.4 * M * M + 2.0)
    for p in (G.GKS_FP64, G.GKS_FP32_MIXED):
        prob, st = W.shock_vortex(201, 101, kappa=0.0, t_end=0.3)
        m0 = st.cell[0].sum()
        with G.Solver(prob, st, p) as S:
            S.step(_steps_for(prob, st, 0.3), t_end=0.3)
            got, t, n = S.fetch()
        assert t == pytest.approx(0.3, rel=0, abs=1e-12)
        c = got.cell
        # (FP32-mixed: the disturbance carries single-precision rounding)
        assert abs(c[0].sum() - m0) < (1e-11 if p == G.GKS_FP64 else 1e-9) * m0, p
        var, trans = _across(c)
        print(f"precision {p}: across the channel: variation {var:.1e}, transverse momentum {trans:.1e}",
              flush=True)
        bound = 1e-12 if p == G.GKS_FP64 else 1e-6
        assert var < bound and trans < bound, (p, var, trans)
        row, h = c[0, 0], prob.dx
        xc = (np.arange(prob.nx) + 0.5) * h
        mid = 0.5 * (r1 + r2)
        k = int(np.argmax(row > mid))
        xs = xc[k - 1] + (mid - row[k - 1]) / (row[k] - row[k - 1]) * h
        assert abs(xs - 0.5) < 0.25 * h, (p, xs)


def _end_state_parity(G, oracle, prob, st, prec, t_end, label):
    """Run to t_end on the GPU; then one more step from the final state, on
    the GPU and in the oracle, compared element by element: FP64 to 1e-11
    (cells) and 1e-10 (point values) of each component's magnitude;
    FP32-mixed with the per-step bound of parity_bounds.one_step (relative
    L1 per component 5e-6 for the cells and 1e-5 for the point values, 1e-3
    for any single value): the mixed form takes its limiter decisions in
    single precision (cross-derivative candidates within one unit of
    single-precision rounding count as tied, the oracle's within its
    double-precision rounding), so a near-tie between the two bands may go
    the other way in a few cells (2.2e-6 measured on Riemann case 2 at
    400^2, 5.7e-6 in one cell of the 800 x 200 double Mach reflection)."""
    p = G.GKS_FP64 if prec == "fp64" else G.GKS_FP32_MIXED
    print(f"{label} {prec}: to t = {t_end}", flush=True)
    nmax = _steps_for(prob, st, t_end)
    with G.Solver(prob, st, p) as S:
        S.step(nmax, t_end=t_end)
        got, t, n = S.fetch()
    assert t == pytest.approx(t_end, rel=0, abs=1e-12) and n < nmax
    assert _physical(prob, got.cell), label
    dt = 0.8 * oracle.dt(prob, got)
    ref = got.copy()
    oracle.step(prob, ref, dt, t)
    with G.Solver(prob, got, p, t0=t) as S:
        S.step(1, dt=dt)
        nxt, _, _ = S.fetch()
    if prec == "fp64":
        assert _rel(nxt.cell, ref.cell) < 1e-11, label
        assert _rel(nxt.fx, ref.fx) < 1e-10, label
        assert _rel(nxt.fy, ref.fy) < 1e-10, label
    else:
        print(f"{label} fp32_mixed, one step from the end state:", one_step("fp32_mixed", nxt, ref, label), flush=True)
    return got, n


@pytest.mark.parametrize("n", [200, 400])
@pytest.mark.parametrize("case", [1, 2])
def test_riemann_at_the_paper_resolutions(G, oracle, case, n):
    """Sec. 4.3 cases 1 and 2 at 200^2 and 400^2 to t = 0.2.  Case 1 is its
    own mirror image across the diagonal: on 200^2 the density stays
    symmetric within 1e-6 (3.5e-9 measured; the oracle's own run: 1.9e-9).
    On 400^2 it is only reported (1.8e-2 measured): the x and y paths round
    differently, and over 899 steps the flow on the diagonal amplifies that
    difference."""
    prob, st = W.riemann_2d(case, n=n, recon_vars=1)
    got, steps = _end_state_parity(G, oracle, prob, st, "fp64", 0.2, prob.name)
    c = got.cell
    asym = np.abs(c[0] - c[0].T).max() if case == 1 else float("nan")
    print(f"{prob.name}: {steps} steps, rho in [{c[0].min():.4f}, {c[0].max():.4f}], "
          f"diagonal asymmetry {asym:.1e}", flush=True)
    if case == 1 and n == 200:
        assert asym < 1e-6


def test_riemann_fp32_mixed_at_400(G, oracle):
    prob, st = W.riemann_2d(2, n=400, recon_vars=1)
    _end_state_parity(G, oracle, prob, st, "fp32_mixed", 0.2, prob.name)


@pytest.mark.parametrize("shape", [(201, 101), (401, 201), (801, 401)])
def test_shock_vortex_at_the_paper_resolutions(G, oracle, shape):
    """Sec. 4.4 to t = 0.8 (the vortex has passed the shock and one branch of
    the bifurcated shock has reached the top wall); the oracle's step of the
    final full-size grid is the check (801 x 401: the FP64 GPU run only)."""
    prob, st = W.shock_vortex(*shape, t_end=0.8)
    precs = ["fp64", "fp32_mixed"] if shape[0] < 801 else ["fp64"]
    for prec in precs:
        got, steps = _end_state_parity(G, oracle, prob, st, prec, 0.8, prob.name)
        row = got.cell[0, prob.ny // 2]
        print(f"{prob.name} {prec}: {steps} steps, centre-line density in [{row.min():.4f}, {row.max():.4f}]",
              flush=True)


def _shock_x(row, xc, hi=8.0, lo=1.4):
    """first crossing of the mid density between the post- and pre-shock
    states along a row (linear interpolation)"""
    mid = 0.5 * (hi + lo)
    k = int(np.argmax(row < mid))
    return xc[k - 1] + (row[k - 1] - mid) / (row[k - 1] - row[k]) * (xc[k] - xc[k - 1])


@pytest.mark.parametrize("shape", [(400, 100), (800, 200)])
@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
def test_dmr_at_the_paper_resolutions(G, oracle, shape, prec):
    """Sec. 4.5 on the paper's 400 x 100 and 800 x 200 cells, characteristic
    variables, to t = 0.2: every state physical, the oracle's step of the
    final grid matched, and on three upper rows the incident shock's
    mid-density crossing within two cells of its exact line
    x = 1/6 + (y + 20 t) / sqrt(3)."""
    prob, st = W.dmr(*shape, recon_vars=1)
    got, steps = _end_state_parity(G, oracle, prob, st, prec, 0.2, prob.name)
    xc = prob.x0 + (np.arange(prob.nx) + 0.5) * prob.dx
    worst = 0.0
    for j in (prob.ny // 2, 3 * prob.ny // 4, prob.ny - 1):
        y = prob.y0 + (j + 0.5) * prob.dy
        exact = 1.0 / 6.0 + (y + 4.0) / np.sqrt(3.0)
        worst = max(worst, abs(_shock_x(got.cell[0, j], xc) - exact) / prob.dx)
    print(f"{prob.name} {prec}: {steps} steps, incident shock within {worst:.2f} cells of the exact line",
          flush=True)
    assert worst < 2.0
