"""Accuracy of the HIP path on the paper's smooth tests (Sec. 4.1).  Table 1:
the 1D density wave after one period at CFL 0.2, third order and the L1
magnitude within the band of the oracle's own test.  Table 2:
the isentropic vortex after one period (t = 10, steps from the CFL
condition, CFL 0.2), L1 error of the cell-average density against the exact
cell averages.  The printed rows (21 .. 121 cells per side) are reproduced
in both forms (errors within the printed decade, orders as printed beyond the
coarsest pair), and the order of accuracy over 64 .. 512 cells per side is
about three (above 2.5 for every doubling)."""
import os

import numpy as np
import pytest

from paper_1412_4489_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1412_4489_amd import gks
    gks.lib()
    return gks


def _table(name):
    rows = {}
    for line in open(os.path.join(GOLDEN, name)):
        if line.strip() and not line.startswith("#"):
            f = line.split()
            rows[int(f[0])] = float(f[1])
    return rows


def _vortex_error(G, oracle, n, precision, t_end=10.0):
    """L1 density error of the vortex on n x n cells at t_end (one period)."""
    prob, st = W.vortex_2d(n, nq=6)
    # enough steps to reach t_end (the ones after it are empty)
    nsteps = int(1.5 * t_end / oracle.dt(prob, st)) + 20
    print(f"vortex {n}x{n} precision {precision}: up to {nsteps} steps", flush=True)
    with G.Solver(prob, st, precision) as S:
        S.step(nsteps, t_end=t_end)
        got, t, steps = S.fetch()
    assert t == pytest.approx(t_end, rel=0, abs=1e-12) and steps < nsteps
    return float(np.abs(got.cell[0] - W.vortex_2d_exact_density(prob, t)).mean())


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32_mixed"])
def test_table2_rows_on_the_gpu(G, oracle, prec):
    rows = _table("table2_vortex.txt")
    errs = {n: _vortex_error(G, oracle, n, prec) for n in sorted(rows)}
    print({n: f"{e:.4e} (paper {rows[n]:.4e})" for n, e in errs.items()}, flush=True)
    ns = sorted(rows)
    # within the printed decade (the band of the oracle's own Table 2 test;
    # with the weights' constant C = 10 the errors here are about a third of
    # the printed ones)
    for n in ns:
        assert rows[n] / 10 < errs[n] < rows[n] * 2, (n, errs[n], rows[n])
    # orders between the printed rows (paper: 2.66, 2.71, 2.95); the first pair
    # is pre-asymptotic (21 cells across the side of 10 give the vortex core of
    # unit radius about two cells), bounded as in the oracle's own test
    for a, b in zip(ns, ns[1:]):
        order = np.log(errs[a] / errs[b]) / np.log(b / a)
        assert order > (2.0 if a == ns[0] else 2.6), (a, b, order)


def test_third_order_64_to_512(G, oracle):
    ns = (64, 128, 256, 512)
    e64 = {n: _vortex_error(G, oracle, n, G.GKS_FP64) for n in ns}
    e32 = {n: _vortex_error(G, oracle, n, G.GKS_FP32_MIXED) for n in ns}
    orders = [np.log2(e64[a] / e64[b]) for a, b in zip(ns, ns[1:])]
    print("L1 errors", {n: f"{e64[n]:.3e} / {e32[n]:.3e}" for n in ns}, "orders", np.round(orders, 3), flush=True)
    orders32 = [np.log2(e32[a] / e32[b]) for a, b in zip(ns, ns[1:])]
    assert all(o > 2.5 for o in orders), orders
    assert all(o > 2.4 for o in orders32), orders32
    # the mixed-precision form: its rounding (FP32 corrections) stays a small
    # part of the truncation error even at 512^2 after ~6700 steps
    for n in ns:
        assert abs(e32[n] - e64[n]) < 0.05 * e64[n], (n, e32[n], e64[n])


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32_mixed"])
def test_table1_rows_on_the_gpu(G, oracle, prec):
    """Third order, and the magnitude between the semi-discrete predictions
    of the oracle's own Table 1 test (the dissipation of the central
    polynomial's interface values); the printed magnitudes are about 14x
    smaller and not reproduced."""
    rows = _table("table1_advection.txt")
    errs = {}
    for n in sorted(rows):
        prob, st = W.advection_1d(n, cfl=0.2)
        nsteps = int(1.5 * 2.0 / oracle.dt(prob, st)) + 20
        with G.Solver(prob, st, prec) as S:
            S.step(nsteps, t_end=2.0)
            got, t, steps = S.fetch()
        assert t == pytest.approx(2.0, rel=0, abs=1e-12)
        errs[n] = float(np.abs(got.cell[0, 0] - W.advection_1d_exact_average(n, t)).mean())
    print({n: f"{e:.3e} (paper {rows[n]:.3e})" for n, e in errs.items()}, flush=True)
    ns = sorted(rows)
    for a, b in zip(ns, ns[1:]):
        order = np.log2(errs[a] / errs[b])
        assert 2.7 < order < 3.3, (a, b, order)
    from math import erfc, exp, pi, sqrt
    from test_oracle_scheme import table1_symbol_l1
    m = lambda r: r * (0.5 * erfc(-sqrt(r / 2)) + exp(-r / 2) / (2 * sqrt(pi * r / 2)))
    a_rho, a_mass = 0.5 * erfc(-sqrt(0.5)), (m(1 + 1e-6) - m(1 - 1e-6)) / 2e-6
    for n in ns:
        assert table1_symbol_l1(n, a_rho) < errs[n] < table1_symbol_l1(n, a_mass), (n, errs[n], rows[n])
