#!/usr/bin/env python3
"""Throughput of the compact third-order gas-kinetic scheme on one MI355X.

Workload: the 2D isentropic vortex of Sec. 4.1 (Table 2) on the periodic
square [0, 10]^2 with 256 x 256 cells, gamma = 1.4, CFL 0.2 (time step from
the CFL condition on the device every step), synthetic initial data.

A step is one pass of the whole scheme: boundary images, CFL time step,
compact reconstruction, every x and y interface (flux and point values),
conservative update.  The state stays resident in HBM; W untimed warm-up
steps, then K timed steps bracketed by device synchronisation.

Printed: one JSON line.  value = Mcell-updates/s of the GKS_FP32_MIXED form
(the headline form), replayed as one hipGraph per step after the launch
shapes are tuned (gks_tune); the GKS_FP64 form and the batched form (96
grids of mixed sizes and flows, one launch per phase for all of them) are
reported beside it.  The interface phases (the dominant kernels) are timed
live with HIP events on the stream they run on, in an eager run of the same
steps; `roofline` prices their algorithmic floating-point operations (the
straight-line operation count of the generated interface arithmetic plus the
double-precision prologue) against the vector ALU peak (and against the rate
without packed FP32, which this build does not use); `traffic` (HBM bytes) and
`valu_busy` (rocprofv3's VALUBusy of the interface kernels) come from the
committed counter record while the kernel sources still match it.  `configs`
gives the throughput of the other full-size 2D workloads (lid-driven cavity
512^2, Navier-Stokes; double Mach reflection 1920x480 with the reconstruction
in conservative and in characteristic variables; in characteristic variables
the shock-vortex interaction of Sec. 4.4 on 801x401, Riemann case 2 on 400^2
and the forward-facing step of Sec. 4.6 on 240x80; the viscous shock tube of
Sec. 4.7 on 600x300 at Re 1000) in both forms.
`cpu_baseline` times the FP64 oracle on this host for a bounded number of
steps of the same workload; the same steps on the GPU give the L1 difference
to the oracle and the conservation drift (largest relative change of the
totals of mass, momentum and energy).

`--pmc-probe` runs the counter-collection workload (a 256 MiB calibration
copy, then a few eager steps of the tuned FP32-mixed vortex).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

N = 256
PEAK_FP32 = 157.3e12  # MI355X vector FP32, FLOP/s
# the same without packed FP32 (not used by this build): 256 CU x 4 SIMD x 16
# lanes x 2 (FMA) x 2.4 GHz
PEAK_FP32_NONPACKED = 78.6e12
PEAK_FP64 = 78.6e12   # MI355X vector FP64, FLOP/s
# double-precision work per interface outside the generated functions
# (interface values, primitives, half-space moments, U0, equilibrium
# quadratic, collision time, time integrals, frame transforms, leading terms)
PROLOGUE_FLOPS = 1000


HYDRO_TERMS = ("conv", "A", "quad", "ttt", "tlin", "dyy", "ay", "inner", "ty")
KIN_TERMS_EULER = ("conv", "quad", "dyy", "ay", "inner")
KIN_TERMS_NS = KIN_TERMS_EULER + ("A", "tlin", "ty")


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_iface_vortex256_fp32mixed.json")


def counter_record():
    """The committed counter record of the interface kernels (HBM bytes per
    launch set from FETCH_SIZE + WRITE_SIZE scaled by the copy-kernel factors,
    VALUBusy), or {} if there is none for the present kernel sources."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return {}
    from paper_1412_4489_amd.profiling import source_hash
    if rec.get("source_hash") != source_hash():
        return {}
    return rec



def pmc_probe():
    """Workload for counter collection: a plain 256 MiB device copy (the
    calibration of FETCH_SIZE / WRITE_SIZE), then the tuned FP32-mixed 256^2
    vortex for a few steps with eager launches."""
    import torch
    from paper_1412_4489_amd import gks
    from paper_1412_4489_amd import workloads as W
    x = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    prob, st = W.vortex_2d(N)
    side = torch.cuda.Stream()  # a torch stream the library borrows (handle 0 would mean its own)
    with gks.Solver(prob, st, gks.GKS_FP32_MIXED, stream=side.cuda_stream) as S:
        S.tune(3)
        gks.gks_profile(S.h, 1)
        S.step(5)
        S.fetch()
    torch.cuda.synchronize()
    print("pmc probe done", flush=True)


def interface_flops(viscous=False):
    """Floating-point operations of one 2D interface: the generated coefficient
    systems and term moments of g0 and of the two sides, plus the prologue."""
    ops = json.load(open(os.path.join(ROOT, "paper_1412_4489_amd", "csrc", "interface_ops.json")))
    side = "ns" if viscous else "euler"
    kin_terms = KIN_TERMS_NS if viscous else KIN_TERMS_EULER
    hydro = ops["coef_g0_2d"] + sum(ops[f"mom_full_{t}_2d"] for t in HYDRO_TERMS)
    kin = ops[f"coef_side_{side}_2d"] + sum(ops[f"mom_half_{t}_2d"] for t in kin_terms)
    return hydro + 2 * kin + PROLOGUE_FLOPS


def run_gpu(precision, steps, warmup, items=None):
    """Times `steps` steps of the given problems (default: the 256^2 vortex)
    after autotuning the launch shapes: once with HIP events around every
    kernel class (kernel times), once as plain graph replays (wall time)."""
    import torch
    from paper_1412_4489_amd import gks
    from paper_1412_4489_amd import workloads as W

    if items is None:
        items = [W.vortex_2d(N)]
    probs, states = [p for p, _ in items], [s for _, s in items]
    side = torch.cuda.Stream()  # a torch stream the library borrows (handle 0 would mean its own)
    S = gks.Solver(probs, states, precision, stream=side.cuda_stream)
    sizes = S.tune(3)
    S.step(warmup)
    torch.cuda.synchronize()
    gks.gks_profile(S.h, 1)
    gks.gks_profile(S.h, 2)
    torch.cuda.synchronize()
    S.step(steps)
    torch.cuda.synchronize()
    gks.gks_profile(S.h, 0)
    kt = {k: gks.gks_kernel_time(S.h, k) for k in gks.KERNELS}
    S.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for k in range(len(probs)):
        S.fetch(k)  # raises if the run produced a nonphysical state
    S.close()
    return wall, kt, probs, sizes


def config_rates(steps=20, warmup=3):
    """Throughput of the other full-size 2D workloads of the paper (FP32-mixed
    and FP64): tuned launch shapes, graph replays, steps from the CFL
    condition.  Returns {name: {precision: Mcell-updates/s}}."""
    import torch
    from paper_1412_4489_amd import gks
    from paper_1412_4489_amd import workloads as W
    out = {}
    for name, mk in (("cavity_512x512_ns_re1000", lambda: W.cavity(512)),
                     ("double_mach_reflection_1920x480", lambda: W.dmr(1920, 480)),
                     ("double_mach_reflection_1920x480_characteristic", lambda: W.dmr(1920, 480, recon_vars=1)),
                     ("shock_vortex_801x401_characteristic", lambda: W.shock_vortex(801, 401)),
                     ("riemann2_400x400_characteristic", lambda: W.riemann_2d(2, n=400, recon_vars=1)),
                     ("forward_facing_step_240x80_characteristic", lambda: W.forward_facing_step(240, 80)),
                     ("viscous_shock_tube_600x300_re1000", lambda: W.viscous_shock_tube(600, 300, re=1000.0))):
        prob, st = mk()
        out[name] = {}
        for pname, prec in (("fp32_mixed", gks.GKS_FP32_MIXED), ("fp64", gks.GKS_FP64)):
            side = torch.cuda.Stream()
            with gks.Solver(prob, st, prec, stream=side.cuda_stream) as S:
                S.tune(2)
                S.step(warmup)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                S.step(steps)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                S.fetch()
            i0, nj = prob.obstacle
            gas = prob.ncells - (prob.nx - i0) * nj if nj else prob.ncells  # cells of a solid step are not updated
            out[name][pname] = round(gas * steps / wall / 1e6, 3)
        print(f"# {name}: {out[name]}", file=sys.stderr, flush=True)
    return out


def gpu_fixed_steps(precision, nsteps, dt):
    """The vortex after nsteps fixed steps on the GPU, and its initial state."""
    from paper_1412_4489_amd import gks
    from paper_1412_4489_amd import workloads as W
    prob, st = W.vortex_2d(N)
    with gks.Solver(prob, st, precision) as S:
        S.step(nsteps, dt=dt)
        got, t, n = S.fetch()
    return got, st


def conservation_drift(init, got):
    """Largest relative change of the totals of mass, both momenta and energy
    (the periodic vortex conserves all four exactly)."""
    t0 = init.cell.sum(axis=(1, 2))
    t1 = got.cell.sum(axis=(1, 2))
    return float(np.max(np.abs(t1 - t0) / np.abs(t0)))


def cpu_baseline(budget_s=15.0):
    import oracle
    from paper_1412_4489_amd import workloads as W
    prob, st = W.vortex_2d(N)
    oracle.lib()
    dt = oracle.dt(prob, st)
    t0 = time.perf_counter()
    n = 0
    while n < 2 or (time.perf_counter() - t0 < budget_s and n < 40):
        oracle.step(prob, st, dt, n * dt)
        n += 1
    sec = time.perf_counter() - t0
    return {"value": round(prob.ncells * n / sec / 1e6, 4), "unit": "Mcell-updates/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{n} steps of the same 256x256 vortex (fixed dt {dt:.6g}), FP64, OpenMP over rows"}, st, n, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the 96-grid batched form")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the cavity 512^2 and double Mach reflection 1920x480 throughputs")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only run the copy calibration and a few vortex steps (for rocprofv3 --pmc)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (the method's single-GPU path); "
              "--gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if a.pmc_probe:
        pmc_probe()
        return
    from paper_1412_4489_amd import gks

    res = {}
    for name, prec in (("fp32_mixed", gks.GKS_FP32_MIXED), ("fp64", gks.GKS_FP64)):
        res[name] = run_gpu(prec, a.steps, a.warmup)
        wall, kt, _, sizes = res[name]
        print(f"# {name}: {a.steps} steps in {wall * 1e3:.2f} ms; block sizes {sizes}; kernel ms: "
              + ", ".join(f"{k} {v[0]:.2f} ({v[1]})" for k, v in kt.items()), file=sys.stderr, flush=True)

    wall, kt, probs, _ = res["fp32_mixed"]
    prob = probs[0]
    cells = prob.ncells
    value = cells * a.steps / wall / 1e6
    wall64, kt64, _, _ = res["fp64"]
    value64 = cells * a.steps / wall64 / 1e6
    # distinct interfaces (on a periodic axis the last interface is the first)
    n_if = ((prob.nx if prob.bc[0].kind == "periodic" else prob.nx + 1) * prob.ny
            + prob.nx * (prob.ny if prob.bc[2].kind == "periodic" else prob.ny + 1))
    fl = interface_flops(False) * n_if
    ms_if, nl = kt["interface"]
    t_if = ms_if / 1e3 / max(nl, 1)
    achieved = fl / t_if
    ms64, nl64 = kt64["interface"]
    achieved64 = fl / (ms64 / 1e3 / max(nl64, 1))

    batched = None
    if not a.no_batch:
        from paper_1412_4489_amd import workloads as W
        items = W.batch()
        bsteps = max(2, a.steps // 10)
        bwall, bkt, bprobs, bsizes = run_gpu(gks.GKS_FP32_MIXED, bsteps, 2, items)
        bcells = sum(p.ncells for p in bprobs)
        batched = {"value": round(bcells * bsteps / bwall / 1e6, 3), "unit": "Mcell-updates/s",
                   "problems": len(bprobs), "cells": bcells, "steps": bsteps,
                   "ms_per_step": round(bwall / bsteps * 1e3, 4),
                   "viscous": sum(bool(p.viscous) for p in bprobs),
                   "interface_ms": round(bkt["interface"][0] / max(bkt["interface"][1], 1), 4),
                   "block_sizes": bsizes,
                   "workload": "96 grids (isentropic vortex 1/2, 2D Riemann cases 1 and 2 1/4 each), n^2 cells with "
                               "n in {64,96,128,192,256,384}, Euler or Navier-Stokes (Re 100-5000), seed 14124489, "
                               "GKS_FP32_MIXED, one launch per phase for all grids, one hipGraph per step"}
        print(f"# batched: {bsteps} steps of {len(bprobs)} grids ({bcells} cells) in {bwall * 1e3:.2f} ms",
              file=sys.stderr, flush=True)

    rec = counter_record()
    out = {
        "metric": "Mcell-updates/s (FP32 & batched vs FP64) at stated L1 err vs oracle",
        "value": round(value, 3),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "isentropic vortex (Sec. 4.1), 256x256 cells, periodic [0,10]^2, gamma 1.4, "
                               "CFL 0.2, Euler, GKS_FP32_MIXED", "cells": cells, "interfaces": n_if},
        "fp64": {"value": round(value64, 3), "ms_per_step": round(wall64 / a.steps * 1e3, 5),
                 "interface_ms": round(ms64 / max(nl64, 1), 5),
                 "interface_tflops": round(achieved64 / 1e12, 3)},
        "batched": batched,
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 4), "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32, 5), "traffic": rec.get("bytes_per_launch_set"),
                     "peak_nonpacked": PEAK_FP32_NONPACKED / 1e12,
                     "frac_nonpacked": round(achieved / PEAK_FP32_NONPACKED, 5),
                     "valu_busy": rec.get("valu_busy_launch_set"),
                     "kernel": "k_iface_{pro,corr,kin1}_2d<float> (one launch set per step)",
                     "flops_per_interface": interface_flops(False),
                     "interface_ms": round(t_if * 1e3, 5)},
    }
    if not a.no_configs:
        out["configs"] = config_rates()
    if not a.no_cpu:
        cb, ref, nref, dt = cpu_baseline()
        out["cpu_baseline"] = cb
        errs, drift = {}, {}
        for name, prec in (("fp32_mixed", gks.GKS_FP32_MIXED), ("fp64", gks.GKS_FP64)):
            got, init = gpu_fixed_steps(prec, nref, dt)
            errs[name] = float(np.abs(got.cell[0] - ref.cell[0]).mean() / np.abs(ref.cell[0]).mean())
            drift[name] = conservation_drift(init, got)
        out["l1_rel_err_vs_oracle"] = {k: float(f"{v:.3e}") for k, v in errs.items()}
        out["conservation_drift"] = {k: float(f"{v:.3e}") for k, v in drift.items()}
        out["l1_sample_steps"] = nref
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
