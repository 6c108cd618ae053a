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
    (lambda p: setattr(p, "recon_vars", 1), "conservative"),
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
