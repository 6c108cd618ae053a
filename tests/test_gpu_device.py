"""Device-borrow form (gks_init_device): the state lives in caller-owned torch
tensors in the ghosted device layouts, every ghost entry NaN on entry, and is
stepped in place on torch's stream.  The results must be bitwise those of the
host-copy form (gks_init), read both through gks_fetch and from the tensors
directly; bad buffers and a nonphysical initial state are refused before any
step."""
import numpy as np
import pytest

from paper_1412_4489_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1412_4489_amd import gks
    gks.lib()
    return gks, torch


CASES = {
    "vortex": lambda: W.vortex_2d(24),
    "dmr": lambda: W.dmr(48, 12),
    "cavity": lambda: W.cavity(16, re=100.0),
    "ns_smooth": lambda: W.smooth_periodic_2d(nx=14, ny=18, seed=3, viscous=True, mu=2e-3, prandtl=0.72,
                                              tau_eps=0.0),
    "advection_1d": lambda: W.advection_1d(40),
    "sod_1d_char": lambda: W.sod_1d(48),
    "forward_facing_step": lambda: W.forward_facing_step(30, 20),
}


def _perturb_seams(prob, st):
    # both forms take a periodic seam's values from the first interface
    if prob.bc[0].kind == "periodic":
        st.fx[..., -1] += 0.25
    if prob.dim == 2 and prob.bc[2].kind == "periodic":
        st.fy[..., -1, :] += 0.25


def _tensors(gks, torch, prob, st, prec):
    return [None if a is None else torch.from_numpy(a).cuda() for a in gks.ghosted(prob, st, prec)]


def _same(a, b):
    return (np.array_equal(a.cell, b.cell) and np.array_equal(a.fx, b.fx) and np.array_equal(a.fy, b.fy))


def _host_copy(gks, probs, states, precs, steps):
    with gks.Solver(probs, states, precs) as S:
        S.step(steps)
        return [S.fetch(k) for k in range(len(probs))]


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32_mixed"])
def test_device_borrow_is_the_host_copy_form(env, name, prec):
    gks, torch = env
    prob, st = CASES[name]()
    _perturb_seams(prob, st)
    T = _tensors(gks, torch, prob, st, prec)
    torch.cuda.synchronize()  # the initial contents are complete before the call
    # a torch stream of its own (torch's legacy default stream has handle 0,
    # which the library reads as "use a stream of your own")
    stream = torch.cuda.Stream()
    assert stream.cuda_stream != 0
    print(f"device-borrow {name} precision {prec}", flush=True)
    h = gks.gks_init_device([prob], [T[0]], [T[1]], [T[2]], prec, stream=stream.cuda_stream)
    try:
        gks.gks_step(h, 6)
        stream.synchronize()
        direct = gks.unghosted(prob, *[None if x is None else x.cpu().numpy() for x in T])
        got, t, n = gks.gks_fetch(h, 0, prob)
    finally:
        gks.gks_destroy(h)
    (ref, tr, nr), = _host_copy(gks, [prob], [st], [prec], 6)
    assert n == nr == 6 and t == tr
    assert _same(got, ref) and _same(direct, ref)
    # the tensors stay the caller's: usable after the handle is gone
    assert torch.isfinite(T[0][:, 2:-2, 2:-2] if prob.dim == 2 else T[0][:, 2:-2]).all()


def test_device_borrow_batch(env):
    gks, torch = env
    items = W.batch(10, seed=11, sizes=(8, 12, 20)) + [W.advection_1d(30), W.sod_1d(36)]
    probs, states = [p for p, _ in items], [s for _, s in items]
    precs = [k % 2 for k in range(len(items))]
    T = [_tensors(gks, torch, p, s, q) for p, s, q in zip(probs, states, precs)]
    torch.cuda.synchronize()
    # no stream: the library's own; the device-wide synchronisation waits for it
    h = gks.gks_init_device(probs, [t[0] for t in T], [t[1] for t in T], [t[2] for t in T], precs)
    try:
        gks.gks_tune(h, 1)
        gks.gks_step(h, 4)
        torch.cuda.synchronize()
        got = [gks.gks_fetch(h, k, p) for k, p in enumerate(probs)]
    finally:
        gks.gks_destroy(h)
    ref = _host_copy(gks, probs, states, precs, 4)
    for k, p in enumerate(probs):
        direct = gks.unghosted(p, *[None if x is None else x.cpu().numpy() for x in T[k]])
        assert got[k][1:] == ref[k][1:], p.name
        assert _same(got[k][0], ref[k][0]) and _same(direct, ref[k][0]), p.name


def test_device_borrow_full_size_vortex(env):
    gks, torch = env
    prob, st = W.vortex_2d(256)
    T = _tensors(gks, torch, prob, st, gks.GKS_FP32_MIXED)
    torch.cuda.synchronize()
    h = gks.gks_init_device([prob], [T[0]], [T[1]], [T[2]], gks.GKS_FP32_MIXED)
    try:
        gks.gks_step(h, 20)
        got, t, n = gks.gks_fetch(h, 0, prob)
    finally:
        gks.gks_destroy(h)
    (ref, tr, nr), = _host_copy(gks, [prob], [st], [gks.GKS_FP32_MIXED], 20)
    assert n == nr == 20 and t == tr and _same(got, ref)


def test_device_borrow_rejects_bad_buffers(env):
    gks, torch = env
    prob, st = W.vortex_2d(16)
    T = _tensors(gks, torch, prob, st, gks.GKS_FP64)
    # tensors: checked by the binding (device, dtype, contiguity, size)
    host = torch.from_numpy(gks.ghosted(prob, st)[1])
    for fx in (T[1][:-1], host, T[1].float(), T[1].view(2, 4, 18, 19)[:, :, :, 1:]):
        with pytest.raises(gks.GKSError) as e:
            gks.gks_init_device([prob], [T[0]], [fx], [T[2]])
        assert e.value.code == gks.GKS_EINVAL and "d_face_x" in str(e.value), str(e.value)
    # raw addresses: checked by the library against the allocation that holds them
    import ctypes as C
    hip = gks.lib()  # hipMalloc / hipFree of the runtime the library uses
    hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    hip.hipFree.argtypes = [C.c_void_p]
    big, _ = W.vortex_2d(256)
    need = gks.gks_state_extent(big)[1] * 8  # 4.3 MB
    raw = C.c_void_p()
    assert hip.hipMalloc(C.byref(raw), need // 4) == 0
    try:
        Tb = _tensors(gks, torch, big, W.vortex_2d(256)[1], gks.GKS_FP64)
        with pytest.raises(gks.GKSError) as e:
            gks.gks_init_device([big], [Tb[0]], [raw.value], [Tb[2]])
        assert e.value.code == gks.GKS_EINVAL and "smaller" in str(e.value), str(e.value)
        with pytest.raises(gks.GKSError) as e:
            gks.gks_init_device([prob], [T[0]], [host.data_ptr()], [T[2]])
        assert e.value.code == gks.GKS_EINVAL and "not device memory" in str(e.value), str(e.value)
    finally:
        hip.hipFree(raw)
    # a nonphysical initial cell, found by the initial scan on the device
    bad = st.copy()
    bad.cell[0, 5, 7] = -0.5
    B = _tensors(gks, torch, prob, bad, gks.GKS_FP64)
    with pytest.raises(gks.GKSError) as e:
        gks.gks_init_device([prob], [B[0]], [B[1]], [B[2]])
    assert e.value.code == gks.GKS_EINVAL and "(i, j) = (7, 5)" in str(e.value)
