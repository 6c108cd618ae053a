"""Batched form: many independent grids of uneven size, both dimensions and
both precisions in one handle, advanced by one launch per phase (block-owner
tables) replayed from one captured hipGraph per step.  Every problem is
compared with the FP64 oracle run alone; the graph replay with the eager
(profiled) launches, and autotuned launch shapes with the defaults, bitwise.
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


def _rel(a, b):
    assert np.isfinite(a).all()
    return float(np.abs(a - b).max() / np.abs(b).max())


def _smooth(prob):
    return "vortex" in prob.name or "smooth" in prob.name or "advection" in prob.name


def _mini_batch():
    items = W.batch(12, seed=7, sizes=(8, 12, 17, 24))
    items += [W.smooth_periodic_2d(nx=11, ny=9, seed=2), W.advection_1d(30), W.sod_1d(40)]
    return items


def test_mixed_batch_matches_oracle_alone(G, oracle):
    items = _mini_batch()
    probs, states = [p for p, _ in items], [s for _, s in items]
    prec = [G.GKS_FP64 if k % 2 == 0 else G.GKS_FP32_MIXED for k in range(len(items))]
    dts = [0.7 * oracle.dt(p, s) for p, s in items]
    refs = []
    for p, s, dt in zip(probs, states, dts):
        r1 = s.copy()
        oracle.step(p, r1, dt, 0.0)
        r2 = r1.copy()
        oracle.step(p, r2, dt, dt)
        refs.append((r1, r2))
    with G.Solver(probs, states, precision=prec) as S:
        for nstep in (1, 2):
            S.step(1, dt=dts)
            for k, p in enumerate(probs):
                if nstep == 2 and not _smooth(p):
                    continue  # a limiter branch may flip on rounding-level differences
                got, t, n = S.fetch(k)
                assert n == nstep and t == pytest.approx(nstep * dts[k], rel=1e-14)
                tol = 1e-11 if prec[k] == G.GKS_FP64 else 5e-6
                assert _rel(got.cell, refs[k][nstep - 1].cell) < tol, (nstep, p.name)


def test_graph_replay_equals_eager_launches(G):
    items = _mini_batch()
    probs, states = [p for p, _ in items], [s for _, s in items]
    out = []
    for eager in (False, True):
        with G.Solver(probs, states, precision=G.GKS_FP32_MIXED) as S:
            if eager:
                G.gks_profile(S.h, 1)  # events around every launch: no graph
            S.step(3)
            out.append([S.fetch(k)[0].cell for k in range(len(probs))])
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_tuned_launch_shapes_are_bitwise_neutral(G):
    items = _mini_batch()
    probs, states = [p for p, _ in items], [s for _, s in items]
    out = []
    for tune in (False, True):
        with G.Solver(probs, states, precision=G.GKS_FP64) as S:
            if tune:
                sizes = S.tune(2)
                assert all(v in (64, 128, 256) for v in sizes.values())
                assert all(S.fetch(k)[2] == 0 for k in range(len(probs)))
            S.step(3)
            out.append([S.fetch(k)[0].cell for k in range(len(probs))])
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_full_batch_96_grids_sampled(G, oracle):
    """The 96-grid batch (vortex and Riemann problems, 64^2 .. 384^2, Euler and
    Navier-Stokes) in one FP32-mixed handle: two steps; the smallest problem
    of each kind is compared with the oracle run alone (vortex after two
    steps, Riemann after one)."""
    items = W.batch()
    probs, states = [p for p, _ in items], [s for _, s in items]
    dts = [0.7 * oracle.dt(p, s) for p, s in items]
    kinds = {}
    for k, p in enumerate(probs):
        key = (p.name.split("_")[1], p.viscous)
        if key not in kinds or p.ncells < probs[kinds[key]].ncells:
            kinds[key] = k
    sample = sorted(kinds.values())
    with G.Solver(probs, states, precision=G.GKS_FP32_MIXED) as S:
        S.step(1, dt=dts)
        first = {k: S.fetch(k)[0] for k in sample}
        S.step(1, dt=dts)
        second = {k: S.fetch(k)[0] for k in sample}
        for k in range(len(probs)):
            assert S.fetch(k)[2] == 2
    for k in sample:
        p, s = items[k]
        r = s.copy()
        oracle.step(p, r, dts[k], 0.0)
        assert _rel(first[k].cell, r.cell) < 5e-6, p.name
        if _smooth(p):
            oracle.step(p, r, dts[k], dts[k])
            assert _rel(second[k].cell, r.cell) < 5e-6, p.name


@pytest.mark.parametrize("grid", [8, 256, 2048])
def test_persistent_interface_launch_is_bitwise_neutral(G, grid):
    """The persistent form of the interface launch (grid blocks taking the
    tiles in turn) gives the one-block-per-tile results bitwise, in both
    forms; bad shapes are refused."""
    items = _mini_batch()
    probs, states = [p for p, _ in items], [s for _, s in items]
    for prec in (G.GKS_FP64, G.GKS_FP32_MIXED):
        out = []
        for pers in (False, True):
            with G.Solver(probs, states, precision=prec) as S:
                if pers:
                    S.set_launch("interface", 128, grid)
                    assert S.launch_shape("interface") == (128, grid)
                S.step(3)
                out.append([S.fetch(k)[0] for k in range(len(probs))])
        for a, b in zip(*out):
            assert np.array_equal(a.cell, b.cell) and np.array_equal(a.fx, b.fx) and np.array_equal(a.fy, b.fy)
    with G.Solver(probs, states) as S:
        for kernel, threads, g in (("interface", 128, 12), ("recon", 128, 8), ("interface", 96, 0)):
            with pytest.raises(G.GKSError):
                S.set_launch(kernel, threads, g)
