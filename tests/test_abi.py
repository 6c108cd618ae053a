"""The C ABI library loads, exports every entry point include/gks.h declares,
and rejects invalid arguments on the host before any device work (no GPU is
needed for these checks)."""
import os
import re

import numpy as np
import pytest

from paper_1412_4489_amd import gks
from paper_1412_4489_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "gks.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gks_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("gks_init", "gks_step", "gks_fetch", "gks_destroy", "gks_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = gks.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert set(_declared()) == set(gks.EXPORTED)


@pytest.mark.parametrize("mutate, why", [
    (lambda p: setattr(p, "gamma", 0.9), "gamma"),
    (lambda p: setattr(p, "nx", 1), "nx"),
    (lambda p: setattr(p, "cfl", -1.0), "cfl"),
    (lambda p: setattr(p.bc[0], "kind", "outflow"), "periodic"),
    (lambda p: setattr(p, "recon_vars", 2), "recon_vars"),
    (lambda p: setattr(p, "dim", 3), "dim"),
])
def test_init_rejects_invalid_problems(mutate, why):
    p, s = W.vortex_2d(8)
    mutate(p)
    if p.nx != 8:  # keep the arrays consistent with the claimed size check
        s = W.State(np.zeros((4, p.ny, p.nx)), np.zeros((2, 4, p.ny, p.nx + 1)), np.zeros((2, 4, p.ny + 1, p.nx)))
    with pytest.raises(gks.GKSError) as e:
        gks.gks_init([p], [s])
    assert e.value.code == gks.GKS_EINVAL
    assert why in str(e.value)


def test_init_rejects_nonphysical_initial_state():
    p, s = W.vortex_2d(8)
    s.cell[3, 2, 3] = -1.0  # negative energy
    with pytest.raises(gks.GKSError) as e:
        gks.gks_init([p], [s])
    assert e.value.code == gks.GKS_EINVAL and "nonphysical" in str(e.value)


def test_state_extent_counts_the_ghosted_layouts():
    # host-only: the element counts of the device buffers of gks_init_device
    p, _ = W.vortex_2d(12)
    p.ny = 7
    assert gks.gks_state_extent(p, gks.GKS_FP64) == (4 * 11 * 16, 2 * 4 * 9 * 15, 2 * 4 * 10 * 14, 8)
    assert gks.gks_state_extent(p, gks.GKS_FP32_MIXED)[3] == 4
    q, _ = W.sod_1d(10)
    assert gks.gks_state_extent(q) == (3 * 14, 3 * 13, 0, 8)
    p.gamma = 0.5
    with pytest.raises(gks.GKSError) as e:
        gks.gks_state_extent(p)
    assert e.value.code == gks.GKS_EINVAL and "gamma" in str(e.value)


def test_ghosted_layouts_round_trip():
    for prob, st in (W.vortex_2d(6), W.sod_1d(9)):
        for prec in (gks.GKS_FP64, gks.GKS_FP32_MIXED):
            arrs = gks.ghosted(prob, st, prec)
            ext = gks.gks_state_extent(prob, prec)
            assert [0 if a is None else a.size for a in arrs] == list(ext[:3])
            assert arrs[1].itemsize == ext[3]
            back = gks.unghosted(prob, *arrs)
            tol = 0 if prec == gks.GKS_FP64 else 1e-6
            assert np.allclose(back.cell, st.cell, rtol=0, atol=0)
            assert np.allclose(back.fx, st.fx, rtol=tol, atol=0)
            if prob.dim == 2:
                assert np.allclose(back.fy, st.fy, rtol=tol, atol=0)
            assert np.isnan(arrs[0]).sum() == arrs[0].size - st.cell.size
