"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Both sides start from the same seeded initial data (paper_1412_4489_amd.workloads)
and take the same fixed time steps; cell averages and interface point values
are compared element by element.

Tolerances:
  * GKS_FP64: the two sides evaluate the same formulas in different orders
    (closed-form peculiar-frame moments on the GPU, term-by-term polynomial
    moments in the oracle); after n steps the relative difference stays at a
    few ulps times the condition of the step: 1e-11 relative to the field's
    magnitude.
  * GKS_FP32_MIXED: the derivative terms of the interface distribution are
    single precision (unit roundoff 6e-8) while cell averages, U0 and the
    leading flux terms are double; the per-step relative error is ~1e-7 of the
    flux correction, so 5e-6 after tens of steps on smooth data.
Where floating point decides a branch (minmod zero, smallest cross
derivative), both sides take it in double precision (the reconstruction is
double precision in both forms).
"""
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


def _compare(a, b, rtol, what):
    scale = np.abs(b).max(axis=tuple(range(1, b.ndim)), keepdims=True) if b.ndim > 1 else np.abs(b).max()
    err = np.abs(a - b) / np.maximum(scale, 1e-300)
    assert np.isfinite(a).all(), f"{what}: non-finite values"
    assert err.max() <= rtol, f"{what}: max relative diff {err.max():.3e} > {rtol:.1e} at {np.unravel_index(err.argmax(), err.shape)}"


def _run_both(G, oracle, prob, st, nsteps, dt, precision):
    ref = st.copy()
    t = 0.0
    for n in range(nsteps):
        oracle.step(prob, ref, dt, t)
        t += dt
    with G.Solver(prob, st, precision) as S:
        S.step(nsteps, dt=dt)
        got, tg, steps = S.fetch()
    assert steps == nsteps
    assert tg == pytest.approx(t, rel=1e-14)
    return got, ref


CASES = {
    "smooth": lambda: W.smooth_periodic_2d(nx=24, ny=19, seed=1),
    "rough": lambda: W.random_perturbed_2d(nx=21, ny=17, seed=2, amp=0.15),
    "vortex": lambda: W.vortex_2d(32),
    "riemann": lambda: W.riemann_2d(1, n=30),
    "ns_smooth": lambda: W.smooth_periodic_2d(nx=20, ny=18, seed=3, viscous=True, mu=2e-3, prandtl=0.72,
                                              tau_eps=0.0),
    "dmr": lambda: W.dmr(48, 12),
    "cavity": lambda: W.cavity(24, re=100.0),
}
SMOOTH = ["smooth", "vortex", "ns_smooth"]


@pytest.mark.parametrize("case", list(CASES))
def test_parity_fp64_one_step(G, oracle, case):
    prob, st = CASES[case]()
    dt = 0.8 * oracle.dt(prob, st)
    got, ref = _run_both(G, oracle, prob, st, 1, dt, G.GKS_FP64)
    _compare(got.cell, ref.cell, 1e-11, "cell")
    _compare(got.fx, ref.fx, 1e-10, "x point values")
    _compare(got.fy, ref.fy, 1e-10, "y point values")


@pytest.mark.parametrize("case", SMOOTH)
def test_parity_fp64_free_running(G, oracle, case):
    """Smooth data: no limiter decision sits near a tie, both sides run on their own."""
    prob, st = CASES[case]()
    dt = 0.8 * oracle.dt(prob, st)
    got, ref = _run_both(G, oracle, prob, st, 8, dt, G.GKS_FP64)
    _compare(got.cell, ref.cell, 1e-11, "cell")
    _compare(got.fx, ref.fx, 1e-10, "x point values")
    _compare(got.fy, ref.fy, 1e-10, "y point values")


@pytest.mark.parametrize("case", ["rough", "riemann", "dmr", "cavity"])
def test_parity_fp64_per_step(G, oracle, case):
    """Discontinuous data: the smallest-|cross derivative| choice and minmod
    are discontinuous in their arguments, so rounding-level differences left
    by an earlier step can legitimately select another branch.  Each step is
    therefore compared from the oracle's own state (the GPU restarts from it,
    with its time), for several consecutive steps."""
    prob, st = CASES[case]()
    dt = 0.8 * oracle.dt(prob, st)
    t = 0.0
    for n in range(4):
        ref = st.copy()
        oracle.step(prob, ref, dt, t)
        with G.Solver(prob, st, G.GKS_FP64, t0=t) as S:
            S.step(1, dt=dt)
            got, tg, steps = S.fetch()
        _compare(got.cell, ref.cell, 1e-11, f"cell, step {n}")
        _compare(got.fx, ref.fx, 1e-10, f"x point values, step {n}")
        _compare(got.fy, ref.fy, 1e-10, f"y point values, step {n}")
        st, t = ref, t + dt


@pytest.mark.parametrize("case", ["smooth", "vortex", "ns_smooth"])
def test_parity_fp32_mixed(G, oracle, case):
    prob, st = CASES[case]()
    dt = 0.8 * oracle.dt(prob, st)
    got, ref = _run_both(G, oracle, prob, st, 10, dt, G.GKS_FP32_MIXED)
    _compare(got.cell, ref.cell, 5e-6, "cell")
    _compare(got.fx, ref.fx, 2e-5, "x point values")
    _compare(got.fy, ref.fy, 2e-5, "y point values")


def test_cfl_step_matches_oracle(G, oracle):
    prob, st = W.vortex_2d(24)
    ref = st.copy()
    dt = oracle.dt(prob, ref)
    oracle.step(prob, ref, dt, 0.0)
    with G.Solver(prob, st) as S:
        S.step(1)
        got, t, steps = S.fetch()
    assert t == pytest.approx(dt, rel=1e-14)
    _compare(got.cell, ref.cell, 1e-11, "cell")


@pytest.mark.parametrize("hot", [(190, 100), (100, 0), (0, 5)])
def test_cfl_minimum_over_many_waves(G, oracle, hot):
    """A 256 x 200 grid has 800 waves of cells (cell (j, i) is in wave
    (256 j + i) / 64) and 512 CFL slots (wave w reduces into slot w % 512), so
    waves 0..287 share their slot with waves 512..799.  One hot cell (three
    times the energy) holds the CFL minimum: cell (190, 100) is in wave 761,
    which shares slot 249 with wave 249; cell (100, 0) is in wave 400, alone
    on slot 400; cell (0, 5) is in wave 0, on slot 0 with wave 512.  The first
    step (initial scan) and the second (the update's reduction) equal the
    oracle's CFL steps."""
    prob, st = W.vortex_2d(256, ny=200)
    st.cell[3, hot[0], hot[1]] *= 3.0
    ref = st.copy()
    dt1 = oracle.dt(prob, ref)
    oracle.step(prob, ref, dt1, 0.0)
    dt2 = oracle.dt(prob, ref)
    with G.Solver(prob, st) as S:
        S.step(1)
        _, t1, _ = S.fetch()
        S.step(1)
        _, t2, steps = S.fetch()
    print(f"hot cell {hot}: dt1 {t1:.17g} vs {dt1:.17g}, dt2 {t2 - t1:.17g} vs {dt2:.17g}", flush=True)
    assert steps == 2
    assert t1 == pytest.approx(dt1, rel=1e-14)
    assert t2 - t1 == pytest.approx(dt2, rel=1e-10)


def test_t_end_clips_last_step(G, oracle):
    prob, st = W.vortex_2d(16)
    with G.Solver(prob, st) as S:
        dt = 0.05
        S.step(5, dt=dt, t_end=0.12)
        got, t, steps = S.fetch()
    assert t == pytest.approx(0.12, rel=1e-14) and steps == 3


def test_batch_of_uneven_grids(G, oracle):
    probs, states = [], []
    for k, (n, seed) in enumerate([(12, 0), (17, 1), (9, 2)]):
        p, s = W.smooth_periodic_2d(nx=n, ny=n + k, seed=seed)
        probs.append(p)
        states.append(s)
    dts = [0.7 * oracle.dt(p, s) for p, s in zip(probs, states)]
    refs = [s.copy() for s in states]
    for p, r, dt in zip(probs, refs, dts):
        for n in range(3):
            oracle.step(p, r, dt, n * dt)
    with G.Solver(probs, states) as S:
        S.step(3, dt=np.array(dts))
        for k in range(3):
            got, t, steps = S.fetch(k)
            _compare(got.cell, refs[k].cell, 1e-11, f"cell {k}")


def test_nonphysical_state_is_reported(G):
    prob, st = W.riemann_2d(2, n=16)
    with G.Solver(prob, st) as S:
        S.step(3, dt=5.0)  # far beyond any CFL limit: the state blows up (no memory access depends on values)
        # the steps after the failing one are empty: time and step count stop
        got, t, n, rc = S.fetch(check=False)
        assert rc == G.GKS_ENONPHYS and 1 <= n < 3 and t == 5.0 * n
        with pytest.raises(G.GKSError) as e:
            S.fetch()
        assert e.value.code == G.GKS_ENONPHYS
        assert "nonphysical" in G.gks_last_error(S.h)
        with pytest.raises(G.GKSError) as e2:
            S.step(1, dt=0.01)
        assert e2.value.code == G.GKS_ESTATE


def test_periodic_seam_is_one_interface(G, oracle):
    """On a periodic axis the last interface is the first one: gks_init takes
    the seam's point values from the first interface, the seam is computed
    once, and the fetched state keeps the two equal; the result equals the
    oracle's from the same (consistent) data."""
    prob, st = W.smooth_periodic_2d(nx=14, ny=11, seed=4)
    bad = st.copy()
    bad.fx[..., prob.nx] += 0.01   # inconsistent seam values are overridden
    bad.fy[..., prob.ny, :] -= 0.01
    dt = 0.8 * oracle.dt(prob, st)
    ref = st.copy()
    oracle.step(prob, ref, dt, 0.0)
    with G.Solver(prob, bad) as S:
        S.step(1, dt=dt)
        got, _, _ = S.fetch()
    assert np.array_equal(got.fx[..., prob.nx], got.fx[..., 0])
    assert np.array_equal(got.fy[..., prob.ny, :], got.fy[..., 0, :])
    _compare(got.cell, ref.cell, 1e-11, "cell")
    _compare(got.fx, ref.fx, 1e-10, "x point values")


@pytest.mark.parametrize("axis", [0, 1], ids=["x", "y"])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32_mixed"])
def test_reflecting_wall_is_the_mirror_extension(G, axis, prec):
    """The GPU's slip wall against its own mirror extension (the oracle's
    pin of the boundary images, here on the kernels): rough data between
    two reflecting walls and the same data doubled across one wall, stepped
    in one handle; after four steps both halves of the doubled problem equal
    the original to rounding (9e-16 in FP64, 4e-16 in FP32-mixed measured)."""
    nx, ny = (12, 20) if axis == 0 else (24, 12)
    h = 1.0 / 24
    walls = [W.BC(), W.BC(), W.BC(), W.BC()]
    walls[2 * axis] = W.BC("reflect")
    walls[2 * axis + 1] = W.BC("reflect")
    P = W.Problem(dim=2, nx=nx, ny=ny, x0=0.0, x1=nx * h, y0=0.0, y1=ny * h, gamma=1.4, tau_eps=0.05,
                  cfl=0.2, recon_vars=1, bc=walls)
    sP = W.random_perturbed_2d(nx=nx, ny=ny, seed=3 + axis, amp=0.2)[1]
    if axis == 1:
        sP.fy[:, 2, 0, :] = 0.0
        sP.fy[:, 2, ny, :] = 0.0
        sP.fx[..., nx] = sP.fx[..., 0]
    else:
        sP.fx[:, 1, :, 0] = 0.0
        sP.fx[:, 1, :, nx] = 0.0
        sP.fy[:, :, ny, :] = sP.fy[:, :, 0, :]
    D, sD = W.mirror_extension(P, sP, axis)
    dt = 0.004
    with G.Solver([P, D], [sP, sD], prec) as S:
        S.step(4, dt=[dt, dt])
        gP, _, _ = S.fetch(0)
        gD, _, _ = S.fetch(1)
    sign = np.array([1.0, 1.0, 1.0, 1.0])
    sign[1 + axis] = -1.0
    if axis == 1:
        upper, lower = gD.cell[:, ny:], gD.cell[:, :ny][:, ::-1] * sign[:, None, None]
    else:
        upper, lower = gD.cell[:, :, nx:], gD.cell[:, :, :nx][:, :, ::-1] * sign[:, None, None]
    tol = 1e-13
    d = max(np.abs(upper - gP.cell).max(), np.abs(lower - gP.cell).max())
    print(f"mirror extension axis {axis} precision {prec}: {d:.1e}", flush=True)
    assert d < tol


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32_mixed"])
@pytest.mark.parametrize("case", ["vortex", "dmr"])
def test_restart_is_bitwise(G, prec, case):
    """Checkpoint and resume: N CFL steps, fetch, a new handle from the
    fetched state at the fetched time, N more steps, equal bitwise to 2N
    steps in one handle (cells and point values; the mixed form's point
    values travel through the host as doubles and back without loss, and the
    restart's initial CFL scan reduces the same cell bounds as the update's)."""
    prob, st = W.vortex_2d(48) if case == "vortex" else W.dmr(96, 24)
    p = [G.GKS_FP64, G.GKS_FP32_MIXED][prec]
    n = 15
    with G.Solver(prob, st, p) as S:
        S.step(2 * n)
        full, t_full, n_full = S.fetch()
    with G.Solver(prob, st, p) as S:
        S.step(n)
        half, t_half, _ = S.fetch()
    with G.Solver(prob, half, p, t0=t_half) as S:
        S.step(n)
        got, t_got, n_got = S.fetch()
    assert n_full == 2 * n and n_got == n and t_got == t_full
    for a, b in ((got.cell, full.cell), (got.fx, full.fx), (got.fy, full.fy)):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("bs,rows", [(64, 1), (128, 2), (256, 4), (256, 1)])
def test_tiled_reconstruction_is_the_row_order_form(G, bs, rows):
    """The reconstruction with its averages staged in LDS tiles gives the
    row-order form's results bitwise (uniform, characteristic-variable,
    stepped and curvilinear grids of uneven sizes, both forms)."""
    items = [W.smooth_periodic_2d(nx=37, ny=29, seed=5), W.riemann_2d(2, n=41, recon_vars=1),
             W.forward_facing_step(60, 20), W.polar_cavity(33, re=100.0)]
    precs = [G.GKS_FP64, G.GKS_FP32_MIXED, G.GKS_FP64, G.GKS_FP32_MIXED]
    dts = [1e-3, 1e-4, 1e-3, 1e-3]
    out = {}
    for shape in ((bs, 0), (bs, rows)):
        with G.Solver([p for p, _ in items], [s for _, s in items], precision=precs) as S:
            S.set_launch("recon", *shape)
            assert S.launch_shape("recon") == shape
            S.step(3, dt=dts)
            out[shape] = [S.fetch(k)[0] for k in range(len(items))]
    for a, b in zip(out[(bs, 0)], out[(bs, rows)]):
        assert np.array_equal(a.cell, b.cell) and np.array_equal(a.fx, b.fx) and np.array_equal(a.fy, b.fy)
