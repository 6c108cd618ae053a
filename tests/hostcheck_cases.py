"""Runs the kernels of the HIP library through the serial host emulation
(paper_1412_4489_amd/csrc/hostcheck) under AddressSanitizer, for the cases of
the GPU parity tests, and compares one FP64 step with the oracle.  Executed in
a subprocess by test_hostcheck.py with libasan preloaded; prints one line per
case and exits non-zero on a mismatch (ASan aborts on a bad access)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1412_4489_amd import gks  # noqa: E402
from paper_1412_4489_amd import workloads as W  # noqa: E402

gks.LIB_PATH = sys.argv[1]
CASES = {
    "smooth": lambda: W.smooth_periodic_2d(nx=17, ny=13, seed=1),
    "rough": lambda: W.random_perturbed_2d(nx=15, ny=11, seed=2, amp=0.15),
    "vortex": lambda: W.vortex_2d(16),
    "riemann": lambda: W.riemann_2d(1, n=14),
    "ns_smooth": lambda: W.smooth_periodic_2d(nx=12, ny=14, seed=3, viscous=True, mu=2e-3, prandtl=0.72,
                                              tau_eps=0.0),
    "dmr": lambda: W.dmr(32, 8),
    "cavity": lambda: W.cavity(12, re=100.0),
}
bad = 0
for name, mk in CASES.items():
    for prec in (gks.GKS_FP64, gks.GKS_FP32_MIXED):
        prob, st = mk()
        dt = 0.8 * O.dt(prob, st)
        ref = st.copy()
        O.step(prob, ref, dt, 0.0)
        with gks.Solver(prob, st, prec) as S:
            S.step(1, dt=dt)
            got, t, n = S.fetch()
            S.step(2)  # CFL steps (block reductions are not emulated exactly)
            S.fetch()
        err = np.abs(got.cell - ref.cell).max() / np.abs(ref.cell).max()
        tol = 1e-12 if prec == gks.GKS_FP64 else 1e-6
        ok = err < tol
        bad += not ok
        print(f"{name} {'fp64' if prec == gks.GKS_FP64 else 'fp32_mixed'} rel_diff {err:.2e} {'ok' if ok else 'FAIL'}",
              flush=True)
# a batch of uneven grids in one handle
probs, states = zip(*[W.smooth_periodic_2d(nx=n, ny=n + 2, seed=n) for n in (5, 9, 7)])
with gks.Solver(list(probs), list(states)) as S:
    S.step(2, dt=[1e-3, 1e-3, 1e-3])
    for k in range(3):
        S.fetch(k)
print("batch ok", flush=True)
sys.exit(1 if bad else 0)
