"""Parity at the full sizes of the paper-shaped workloads, in the launch
configuration the benchmark uses: the isentropic vortex on 256^2 cells, the
lid-driven cavity on 512^2 and the double Mach reflection on 1920 x 480.  The
oracle computes whole steps of the same grids (seconds per step on the host
cores); smooth flows run free for three steps, the double Mach reflection
(discontinuous) is compared after one step."""
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


def _rel(a, b, floor=None):
    """max |a - b| relative to each component's magnitude; `floor` bounds the
    magnitude of the momentum components from below (the cavity starts at
    rest: its momentum scale is the lid's, rho U_lid)."""
    assert np.isfinite(a).all() and np.isfinite(b).all()
    vax = b.ndim - 3  # component axis
    scale = np.abs(b).max(axis=tuple(k for k in range(b.ndim) if k != vax), keepdims=True)
    if floor is not None:
        idx = [slice(None)] * b.ndim
        idx[vax] = slice(1, 3)
        scale[tuple(idx)] = np.maximum(scale[tuple(idx)], floor)
    return float((np.abs(a - b) / scale).max())


FULL = {
    "vortex_256": (lambda: W.vortex_2d(256), 3),
    "cavity_512": (lambda: W.cavity(512), 3),
    "dmr_1920x480": (lambda: W.dmr(1920, 480), 1),
}
_refs = {}


def _reference(oracle, case):
    if case not in _refs:
        mk, nsteps = FULL[case]
        prob, st = mk()
        dt = 0.8 * oracle.dt(prob, st)
        ref = st.copy()
        for n in range(nsteps):
            oracle.step(prob, ref, dt, n * dt)
        _refs[case] = (prob, st, ref, dt, nsteps)
    return _refs[case]


@pytest.mark.parametrize("case", list(FULL))
@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
def test_full_size_parity(G, oracle, case, prec):
    prob, st, ref, dt, nsteps = _reference(oracle, case)
    p = G.GKS_FP64 if prec == "fp64" else G.GKS_FP32_MIXED
    with G.Solver(prob, st, p) as S:
        S.step(nsteps, dt=dt)
        got, t, n, rc = S.fetch(check=False)
    assert n == nsteps
    # the GPU flags a nonphysical state exactly when the oracle's has one
    # (the double Mach reflection at this resolution has a few such cells
    # after the first step in both implementations)
    c = ref.cell
    pr = (prob.gamma - 1.0) * (c[3] - 0.5 * (c[1] ** 2 + c[2] ** 2) / c[0])
    bad = (c[0] <= 0) | (pr <= 0)
    assert (rc == G.GKS_ENONPHYS) == bool(bad.any())
    # FP32-mixed: 5e-6 on the smooth and shocked flows.  In the first steps of
    # the cavity the impulsively started lid meets the side walls in the two
    # top corner cells, where the velocity jumps by U_lid across one cell and
    # the correction terms are as large as the leading ones: their single-
    # precision evaluation leaves 3e-5 of the lid momentum there (the same
    # kernels emulated on the host give the same figure; the density's
    # relative L1 difference is 2e-10)
    tol = 1e-11 if prec == "fp64" else (1e-4 if case == "cavity_512" else 5e-6)
    floor = 0.15 * np.sqrt(prob.gamma) if case == "cavity_512" else None
    if bad.any() and prec != "fp64":
        # next to the cells that left the physical states the correction terms
        # dominate the flux (the anomaly of the reconstruction at the shock):
        # single precision leaves 1e-5 of the field there (host emulation of
        # the same kernels: 1.2e-5), 6e-7 elsewhere
        from scipy.ndimage import binary_dilation
        near = binary_dilation(bad, iterations=2)
        scale = np.abs(ref.cell).max(axis=(1, 2), keepdims=True)
        d = np.abs(got.cell - ref.cell) / scale
        assert d[:, ~near].max() < tol
        assert d[:, near].max() < 1e-4
        return
    assert _rel(got.cell, ref.cell, floor) < tol
    assert _rel(got.fx, ref.fx, floor) < 10 * tol
    assert _rel(got.fy, ref.fy, floor) < 10 * tol
    # conservation on the periodic grid: every total to round-off (the walls
    # of the cavity are not mass-tight in the ghost-cell wall treatment; the
    # drift is the oracle's, to parity)
    if case == "vortex_256":
        for v in range(4):
            tot, tot0 = got.cell[v].sum(dtype=np.float64), st.cell[v].sum(dtype=np.float64)
            assert abs(tot - tot0) <= 1e-12 * np.abs(st.cell[v]).sum()
