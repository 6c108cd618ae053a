"""Comparison measures of the GPU parity tests (shared by several files)."""
import numpy as np


def rel_max(a, b):
    """max |a - b| relative to each component's magnitude (the momenta share
    the momentum vector's); a and b are cell[nv][ny][nx] or
    faces[ng][nv][..][..]"""
    assert np.isfinite(a).all() and np.isfinite(b).all()
    vax = b.ndim - 3
    scale = np.abs(b).max(axis=tuple(k for k in range(b.ndim) if k != vax), keepdims=True)
    idx = [slice(None)] * b.ndim
    idx[vax] = slice(1, 3)
    scale[tuple(idx)] = scale[tuple(idx)].max()
    return float((np.abs(a - b) / np.maximum(scale, 1e-300)).max())


def rel_l1_each(a, b):
    """largest over the components of the relative L1 difference (axis -3 is
    the component axis)"""
    assert np.isfinite(a).all() and np.isfinite(b).all()
    vax = b.ndim - 3
    ax = tuple(k for k in range(b.ndim) if k != vax)
    return float((np.abs(a - b).sum(axis=ax) / np.maximum(np.abs(b).sum(axis=ax), 1e-300)).max())


def one_step(form, nxt, ref, what):
    """One step from the same state.  FP64: every cell average and point
    value to 1e-11 / 1e-10 of its component's magnitude.  FP32-mixed: the
    limiter's decisions (minmod signs, the smallest cross-derivative
    candidate, the admissibility fallback) are taken in single precision, and
    a decision within its rounding may go the other way than the oracle's
    double-precision one, a legitimate alternative result; so the bound is
    5e-6 relative L1 per component for the cell averages and 1e-5 for the
    point values, and 1e-3 of the component's magnitude for any one value.
    Returns a summary line."""
    if form == "fp64":
        ec, ef, eg = rel_max(nxt.cell, ref.cell), rel_max(nxt.fx, ref.fx), rel_max(nxt.fy, ref.fy)
        assert ec < 1e-11 and ef < 1e-10 and eg < 1e-10, (what, ec, ef, eg)
        return f"max {ec:.1e} cells, {max(ef, eg):.1e} point values"
    lc = rel_l1_each(nxt.cell, ref.cell)
    lp = max(rel_l1_each(nxt.fx, ref.fx), rel_l1_each(nxt.fy, ref.fy))
    mc = rel_max(nxt.cell, ref.cell)
    mp = max(rel_max(nxt.fx, ref.fx), rel_max(nxt.fy, ref.fy))
    assert lc < 5e-6 and lp < 1e-5 and mc < 1e-3 and mp < 1e-3, (what, lc, lp, mc, mp)
    scale = np.abs(ref.cell).max(axis=(1, 2), keepdims=True)
    scale[1:3] = scale[1:3].max()
    over = int((np.abs(nxt.cell - ref.cell) / scale > 5e-6).any(axis=0).sum())
    return (f"L1 {lc:.1e} cells, {lp:.1e} point values; max {mc:.1e}, {mp:.1e}; "
            f"{over} of {ref.cell[0].size} cells beyond 5e-6")
