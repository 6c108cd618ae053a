"""Writes tests/golden/cavity512_re1000_200steps.npz: the lid-driven cavity
of Sec. 4.8 (512 x 512 cells, Re 1000, Mach 0.15, Pr 0.72, gamma 5/3,
isothermal no-slip walls) after 200 steps of the FP64 oracle from rest,
each step 0.8 times the initial CFL step.  Stored: that step, and the change
of the cell averages from the initial state (mostly zero: the lid's
disturbance has crossed a few dozen cells), compressed.

    python tests/golden/make_cavity512.py     (about 20 minutes on 8 cores)

Calls the oracle only."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1412_4489_amd import workloads as W  # noqa: E402

STEPS = 200


def main():
    prob, st = W.cavity(512)
    init = st.cell.copy()
    dt = 0.8 * oracle.dt(prob, st)
    n, t = oracle.run(prob, st, nsteps=STEPS, dt_fixed=dt)
    assert n == STEPS
    np.savez_compressed(os.path.join(HERE, "cavity512_re1000_200steps.npz"), dt=np.array(dt), steps=np.array(STEPS),
                        dcell=st.cell - init)


if __name__ == "__main__":
    main()
