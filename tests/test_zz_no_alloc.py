"""The allocation-free entry point gks_step_noalloc (for callers that cannot
allocate device memory) against the device-borrow handle form
(gks_init_device + gks_step + gks_fetch) on the same initial buffers,
through the C ABI: two calls in a row on one GPU, the second with a smaller
problem (then a third, 1D one), each in both precision forms.  The same
kernels run in the same order on the same data, so the states must be
bitwise equal (the bar for the double form is 1e-11; equality is checked),
and so must the time, the step count, the error word and the fallback
count.  A problem larger than the static scratch array is refused before
any device work."""
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


def _tensors(gks, torch, prob, st, prec):
    return [None if a is None else torch.from_numpy(a).cuda() for a in gks.ghosted(prob, st, prec)]


def _handle_run(gks, torch, prob, st, prec, nsteps, dt, t_end):
    T = _tensors(gks, torch, prob, st, prec)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    h = gks.gks_init_device([prob], [T[0]], [T[1]], [T[2]], prec, stream=stream.cuda_stream)
    try:
        gks.gks_step(h, nsteps, None if dt == 0.0 else [dt], None if t_end == 0.0 else [t_end])
        got, t, n = gks.gks_fetch(h, 0, prob)
        fb = gks.gks_fallbacks(h, 0)
    finally:
        gks.gks_destroy(h)
    return got, t, n, fb


# (workload, steps, fixed step as a fraction of the CFL step (0: CFL), end time)
CALLS = [
    (lambda: W.vortex_2d(64), 6, 0.0, 0.0),              # periodic, CFL steps
    (lambda: W.dmr(48, 12), 5, 0.7, 0.0),                # smaller; inflow/outflow/DMR walls, fixed steps
    (lambda: W.sod_1d(40), 8, 0.0, 0.02),                # 1D, CFL steps clipped to an end time
]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32_mixed"])
def test_noalloc_matches_the_device_borrow_form(env, oracle, prec):
    gks, torch = env
    for mk, nsteps, frac, t_end in CALLS:
        prob, st = mk()
        dt = frac * oracle.dt(prob, st) if frac else 0.0
        ref, t_ref, n_ref, fb_ref = _handle_run(gks, torch, prob, st, prec, nsteps, dt, t_end)
        T = _tensors(gks, torch, prob, st, prec)
        status = torch.full((4,), -1, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        stream = torch.cuda.Stream()
        gks.gks_step_noalloc(prob, T[0], T[1], T[2], nsteps, dt, t_end, status, prec, stream.cuda_stream)
        stream.synchronize()
        got = gks.unghosted(prob, *[None if x is None else x.cpu().numpy() for x in T])
        raw = status.cpu().numpy()
        t = raw[0:1].view(np.float64)[0]
        assert raw[1] == n_ref and n_ref > 0, (raw, n_ref)
        assert t == t_ref and raw[2] == 0 and raw[3] == fb_ref, (raw, t_ref, fb_ref)
        assert np.array_equal(got.cell, ref.cell), prob.name
        assert np.array_equal(got.fx, ref.fx) and np.array_equal(got.fy, ref.fy), prob.name


def test_noalloc_refuses_a_problem_beyond_the_scratch(env):
    gks, torch = env
    prob, st = W.vortex_2d(16)
    T = _tensors(gks, torch, prob, st, 0)
    from dataclasses import replace
    big = replace(prob, nx=1024, ny=1024)  # about 1.2 GB of scratch in double precision
    n = gks.gks_state_extent(big, 0)
    bufs = [torch.zeros(n[0], dtype=torch.float64, device="cuda"), torch.zeros(n[1], dtype=torch.float64, device="cuda"),
            torch.zeros(n[2], dtype=torch.float64, device="cuda")]
    with pytest.raises(gks.GKSError) as e:
        gks.gks_step_noalloc(big, *bufs, 1)
    assert e.value.code == gks.GKS_EINVAL and "scratch" in str(e.value)
