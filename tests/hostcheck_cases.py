"""Runs the kernels of the HIP library through the host emulation
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

# the device code's division by a divisor with a known reciprocal
# (div_by(a, divisor(b))) must give the correctly rounded quotient, i.e. the
# bits of a / b: random operands over 80 binades, and the divisors the
# reconstruction uses (cell sizes and their products, 6)
import ctypes as _C  # noqa: E402
_L = _C.CDLL(sys.argv[1])
_L.gks_emu_div_by.restype = _C.c_double
_L.gks_emu_div_by.argtypes = [_C.c_double, _C.c_double]
_rng = np.random.default_rng(20141215)
_a = _rng.uniform(1.0, 2.0, 200000) * np.exp2(_rng.integers(-40, 40, 200000)) * _rng.choice([-1.0, 1.0], 200000)
_b = _rng.uniform(1.0, 2.0, 200000) * np.exp2(_rng.integers(-30, 30, 200000))
_h = 10.0 / np.array([64, 96, 128, 192, 256, 384, 512], dtype=np.float64)
_b[:7000] = np.tile(np.concatenate([_h, _h * _h, 2.0 * _h, [6.0, 12.0, 3.0, 1.0 / 3.0]]), 1000)[:7000]
_bad = sum(1 for x, y in zip(_a.tolist(), _b.tolist()) if _L.gks_emu_div_by(x, y) != x / y)
print(f"division: {_bad} of {len(_a)} quotients differ from a / b", flush=True)
if _bad == 0:
    print("division ok", flush=True)
CASES = {
    "smooth": lambda: W.smooth_periodic_2d(nx=17, ny=13, seed=1),
    "rough": lambda: W.random_perturbed_2d(nx=15, ny=11, seed=2, amp=0.15),
    "vortex": lambda: W.vortex_2d(16),
    "riemann": lambda: W.riemann_2d(1, n=14),
    "riemann_char": lambda: W.riemann_2d(2, n=13, recon_vars=1),
    "sod_2d_char_y": lambda: W.sod_2d(20, 3, axis=1),
    "shock_vortex_char": lambda: W.shock_vortex(40, 20),
    "viscous_shock_tube": lambda: W.viscous_shock_tube(16, 8, re=200.0),
    "forward_facing_step": lambda: W.forward_facing_step(30, 20),
    "ns_smooth": lambda: W.smooth_periodic_2d(nx=12, ny=14, seed=3, viscous=True, mu=2e-3, prandtl=0.72,
                                              tau_eps=0.0),
    "dmr": lambda: W.dmr(32, 8),
    "cavity": lambda: W.cavity(12, re=100.0),
    "advection_1d": lambda: W.advection_1d(20),
    "sod_1d_char": lambda: W.sod_1d(24),
    "sod_1d_cons": lambda: W.sod_1d(24, recon_vars=0),
    "blast_1d": lambda: W.blast_1d(30),
    # curvilinear grids
    "curv_vortex_wavy": lambda: W.vortex_mapped(14, amp=0.04),
    "curv_vortex_sheared": lambda: W.vortex_mapped(12, shear=0.3, angle=0.5),
    "curv_polar_cavity": lambda: W.polar_cavity(12, re=50.0),
    "curv_solid_rotation_ns": lambda: W.solid_rotation(6, viscous=True, mu=0.01),
}


def _gas(prob, c):
    """the cells outside a solid step (whose cells hold images, not gas)"""
    i0, nj = prob.obstacle
    if not nj:
        return c
    c = c.copy()
    c[:, :nj, i0:] = 0.0
    return c


bad = 0
for name, mk in CASES.items():
    for prec in (gks.GKS_FP64, gks.GKS_FP32_MIXED):
        prob, st = mk()
        dt = 0.8 * O.dt(prob, st)
        ref = st.copy()
        O.step(prob, ref, dt, 0.0)
        # two more steps from the CFL condition; the oracle decides whether
        # they stay physical (a coarse blast wave does not)
        ref2, t2, ok2 = ref.copy(), dt, True
        for n in range(2):
            d = O.dt(prob, ref2)
            try:
                O.step(prob, ref2, d, t2)
            except FloatingPointError:
                ok2 = False
                break
            t2 += d
        with gks.Solver(prob, st, prec) as S:
            S.step(1, dt=dt)
            got, t, n = S.fetch()
            S.step(2)
            try:
                got2, _, _ = S.fetch()
                gok2 = True
            except gks.GKSError as e:
                assert e.code == gks.GKS_ENONPHYS, e
                gok2 = False
        same = gok2 == ok2
        if ok2 and gok2 and not any(k in name for k in ("rough", "riemann", "dmr", "sod", "blast", "shock", "step")):
            # free-running on smooth data (discontinuous data may flip a
            # limiter branch on rounding-level differences)
            e2 = np.abs(_gas(prob, got2.cell) - _gas(prob, ref2.cell)).max() / np.abs(ref2.cell).max()
            same = e2 < (1e-11 if prec == gks.GKS_FP64 else 1e-5)
        bad += not same
        if not same:
            print(f"{name} CFL steps differ from the oracle (physical: gpu {gok2}, oracle {ok2})", flush=True)
        err = np.abs(_gas(prob, got.cell) - _gas(prob, ref.cell)).max() / np.abs(ref.cell).max()
        tol = 1e-12 if prec == gks.GKS_FP64 else 1e-6
        ok = err < tol
        bad += not ok
        print(f"{name} {'fp64' if prec == gks.GKS_FP64 else 'fp32_mixed'} rel_diff {err:.2e} {'ok' if ok else 'FAIL'}",
              flush=True)
# a batch of uneven grids of both dimensions and precisions in one handle,
# each problem compared with the oracle run alone
mixed = [W.smooth_periodic_2d(nx=n, ny=n + 2, seed=n) for n in (5, 9, 7)] + [W.sod_1d(12), W.advection_1d(9)]
mixed += W.batch(4, seed=3, sizes=(6, 8)) + [W.riemann_2d(1, n=9, recon_vars=1)]
precs = [gks.GKS_FP64, gks.GKS_FP32_MIXED] * 5
probs, states = [m[0] for m in mixed], [m[1] for m in mixed]
dts = [0.7 * O.dt(p, s) for p, s in mixed]
# one step each (a second one for the smooth problems: on discontinuous data
# a rounding-level difference may legitimately flip a limiter branch)
smooth = [not any(k in p.name for k in ("riemann", "sod")) for p in probs]
refs1, refs2 = [], []
for p, s, dt in zip(probs, states, dts):
    r = s.copy()
    O.step(p, r, dt, 0.0)
    refs1.append(r.copy())
    O.step(p, r, dt, dt)
    refs2.append(r)
with gks.Solver(probs, states, precision=precs[:len(probs)]) as S:
    for nstep, refs in ((1, refs1), (2, refs2)):
        S.step(1, dt=dts)
        for k in range(len(probs)):
            if nstep == 2 and not smooth[k]:
                continue
            got, t, n = S.fetch(k)
            err = np.abs(got.cell - refs[k].cell).max() / np.abs(refs[k].cell).max()
            tol = 1e-12 if precs[k] == gks.GKS_FP64 else 1e-6
            bad += not err < tol
            print(f"batch step {nstep} {k} {probs[k].name} rel_diff {err:.2e} {'ok' if err < tol else 'FAIL'}",
                  flush=True)
# a curvilinear grid beside uniform ones in one handle (its own launches)
mixed = [W.vortex_mapped(10, amp=0.05), W.smooth_periodic_2d(nx=9, ny=7, seed=4), W.polar_cavity(8, re=50.0)]
probs, states = [m[0] for m in mixed], [m[1] for m in mixed]
dts = [0.7 * O.dt(p, s) for p, s in mixed]
refs = []
for p, s, dt in zip(probs, states, dts):
    r = s.copy()
    O.step(p, r, dt, 0.0)
    O.step(p, r, dt, dt)
    refs.append(r)
with gks.Solver(probs, states, precision=[gks.GKS_FP64, gks.GKS_FP32_MIXED, gks.GKS_FP64]) as S:
    S.step(2, dt=dts)
    for k in range(3):
        got, t, n = S.fetch(k)
        err = np.abs(got.cell - refs[k].cell).max() / np.abs(refs[k].cell).max()
        tol = 1e-12 if k != 1 else 1e-6
        bad += not err < tol
        print(f"curvilinear batch {k} {probs[k].name} rel_diff {err:.2e} {'ok' if err < tol else 'FAIL'}", flush=True)
print("batch ok", flush=True)
# autotuned launch shapes: bitwise the same results, the state not advanced
# (with a solid step: its image launch takes the boundary kernel's size)
pair = [W.smooth_periodic_2d(nx=13, ny=11, seed=5), W.sod_1d(20), W.forward_facing_step(30, 20)]
outs = []
for tune in (False, True):
    with gks.Solver([q[0] for q in pair], [q[1] for q in pair],
                    precision=[gks.GKS_FP64, gks.GKS_FP32_MIXED, gks.GKS_FP64]) as S:
        if tune:
            sizes = S.tune(2)
            assert all(S.fetch(k)[2] == 0 for k in range(3)), "tuning advanced the state"
        S.step(2, dt=[1e-3, 1e-3, 1e-3])
        outs.append([S.fetch(k)[0].cell for k in range(3)])
same = all(np.array_equal(a, b) for a, b in zip(*outs))
bad += not same
print(f"tuned block sizes {sizes}: results {'identical' if same else 'DIFFER'}", flush=True)
# the persistent interface launch (8 blocks taking the tiles in turn)
with gks.Solver([q[0] for q in pair], [q[1] for q in pair],
                precision=[gks.GKS_FP64, gks.GKS_FP32_MIXED, gks.GKS_FP64]) as S:
    S.set_launch("interface", 64, 8)
    shape = S.launch_shape("interface")
    S.step(2, dt=[1e-3, 1e-3, 1e-3])
    pers = [S.fetch(k)[0].cell for k in range(3)]
same = shape == (64, 8) and all(np.array_equal(a, b) for a, b in zip(outs[0], pers))
bad += not same
print(f"persistent interface launch {shape}: results {'identical' if same else 'DIFFER'}", flush=True)
# the tiled reconstruction (averages staged in LDS): bitwise the row-order
# form's results for 1, 2 and 4 rows at 64 and 256 threads, on uniform,
# characteristic-variable, stepped and curvilinear grids of uneven sizes
quad = [W.smooth_periodic_2d(nx=13, ny=11, seed=5), W.riemann_2d(2, n=9, recon_vars=1), W.forward_facing_step(30, 20),
        W.polar_cavity(11, re=50.0)]
precs4 = [gks.GKS_FP64, gks.GKS_FP32_MIXED, gks.GKS_FP64, gks.GKS_FP32_MIXED]
base = None
for bs, rows in ((64, 0), (64, 1), (64, 2), (64, 4), (256, 1), (256, 4)):
    with gks.Solver([q[0] for q in quad], [q[1] for q in quad], precision=precs4) as S:
        S.set_launch("recon", bs, rows)
        shape = S.launch_shape("recon")
        S.step(2, dt=[1e-3, 1e-4, 1e-3, 1e-3])
        got = [S.fetch(k)[0] for k in range(4)]
    if base is None:
        base = got
        continue
    same = shape == (bs, rows) and all(np.array_equal(a.cell, b.cell) and np.array_equal(a.fx, b.fx)
                                       and np.array_equal(a.fy, b.fy) for a, b in zip(got, base))
    bad += not same
    print(f"tiled reconstruction {shape}: results {'identical' if same else 'DIFFER'}", flush=True)
# device-borrow form: the caller's buffers (emulated device memory) with NaN in
# every ghost entry, stepped in place; bitwise the host-copy form's results
import ctypes as C  # noqa: E402
L = gks.lib()
L.gks_emu_alloc.restype = C.c_void_p
L.gks_emu_alloc.argtypes = [C.c_size_t]
L.gks_emu_free.argtypes = [C.c_void_p]


def emu_buffers(arrs):
    out = []
    for a in arrs:
        if a is None:
            out.append(None)
            continue
        ptr = L.gks_emu_alloc(a.nbytes)
        C.memmove(ptr, a.ctypes.data, a.nbytes)
        out.append(ptr)
    return out


def emu_read(ptr, like):
    a = np.empty_like(like)
    C.memmove(a.ctypes.data, ptr, a.nbytes)
    return a


for name in ("vortex", "dmr", "cavity", "ns_smooth", "advection_1d", "sod_1d_char"):
    for prec in (gks.GKS_FP64, gks.GKS_FP32_MIXED):
        prob, st = CASES[name]()
        if prob.bc[0].kind == "periodic":  # both forms take the seam from the first interface
            st.fx[..., -1] += 0.25
        if prob.dim == 2 and prob.bc[2].kind == "periodic":
            st.fy[..., -1, :] += 0.25
        host = gks.ghosted(prob, st, prec)
        ptrs = emu_buffers(host)
        h = gks.gks_init_device([prob], [ptrs[0]], [ptrs[1]], [ptrs[2]], prec)
        gks.gks_step(h, 3, dt_fixed=[0.5 * O.dt(prob, st)])
        got, t, n = gks.gks_fetch(h, 0, prob)
        gks.gks_destroy(h)
        direct = gks.unghosted(prob, *[None if q is None else emu_read(q, a) for q, a in zip(ptrs, host)])
        with gks.Solver(prob, st, prec) as S:
            S.step(3, dt=0.5 * O.dt(prob, st))
            ref, tr, nr = S.fetch()
        same = (n == nr == 3 and t == tr and np.array_equal(got.cell, ref.cell) and np.array_equal(got.fx, ref.fx)
                and np.array_equal(got.fy, ref.fy) and np.array_equal(direct.cell, ref.cell)
                and np.array_equal(direct.fx, ref.fx) and np.array_equal(direct.fy, ref.fy))
        bad += not same
        print(f"device-borrow {name} {prec}: {'identical' if same else 'DIFFER'}", flush=True)
        for q in ptrs:
            if q is not None:
                L.gks_emu_free(q)
# the allocation-free entry point on emulated device buffers: bitwise the
# device-borrow handle form, two calls in a row (the second smaller), then a
# 1D problem; the scratch array's bounds are checked by ASan
for mk, nsteps in ((CASES["dmr"], 3), (CASES["vortex"], 2), (CASES["sod_1d_char"], 3)):
    for prec in (gks.GKS_FP64, gks.GKS_FP32_MIXED):
        prob, st = mk()
        host = gks.ghosted(prob, st, prec)
        pa, pb = emu_buffers(host), emu_buffers(host)
        status = L.gks_emu_alloc(32)
        dt = 0.5 * O.dt(prob, st)
        h = gks.gks_init_device([prob], [pa[0]], [pa[1]], [pa[2]], prec)
        gks.gks_step(h, nsteps, dt_fixed=[dt])
        ref, tr, nr = gks.gks_fetch(h, 0, prob)
        fb = gks.gks_fallbacks(h, 0)
        gks.gks_destroy(h)
        gks.gks_step_noalloc(prob, pb[0], pb[1], pb[2], nsteps, dt, 0.0, status, prec)
        got = gks.unghosted(prob, *[None if q is None else emu_read(q, a) for q, a in zip(pb, host)])
        raw = np.zeros(4, dtype=np.int64)
        C.memmove(raw.ctypes.data, status, 32)
        t = raw[0:1].view(np.float64)[0]
        same = (np.array_equal(got.cell, ref.cell) and np.array_equal(got.fx, ref.fx) and np.array_equal(got.fy, ref.fy)
                and t == tr and raw[1] == nr == nsteps and raw[2] == 0 and raw[3] == fb)
        bad += not same
        print(f"noalloc {prob.name} {prec}: {'identical' if same else 'DIFFER'}", flush=True)
        for q in pa + pb + [status]:
            if q is not None:
                L.gks_emu_free(q)
# device-borrow rejections: a nonphysical initial cell (found by the scan), a
# buffer too small for the extent, host memory
prob, st = CASES["vortex"]()
st.cell[0, 3, 5] = -1.0
ptrs = emu_buffers(gks.ghosted(prob, st))
try:
    gks.gks_init_device([prob], [ptrs[0]], [ptrs[1]], [ptrs[2]])
    bad += 1
    print("nonphysical initial cell not rejected", flush=True)
except gks.GKSError as e:
    ok = e.code == gks.GKS_EINVAL and "(i, j) = (5, 3)" in str(e)
    bad += not ok
    print(f"nonphysical initial cell: {e} {'ok' if ok else 'FAIL'}", flush=True)
prob, st = CASES["vortex"]()
host = gks.ghosted(prob, st)
small = L.gks_emu_alloc(host[1].nbytes - 8)
for args, what in (((ptrs[0], small, ptrs[2]), "is smaller"), ((ptrs[0], host[1].ctypes.data, ptrs[2]), "not device")):
    try:
        gks.gks_init_device([prob], [args[0]], [args[1]], [args[2]])
        bad += 1
        print(f"bad buffer ({what}) not rejected", flush=True)
    except gks.GKSError as e:
        ok = e.code == gks.GKS_EINVAL and what in str(e)
        bad += not ok
        print(f"bad buffer: {e} {'ok' if ok else 'FAIL'}", flush=True)
L.gks_emu_free(small)
for q in ptrs:
    L.gks_emu_free(q)
sys.exit(1 if bad or _bad else 0)
