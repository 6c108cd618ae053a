#!/usr/bin/env python3
"""Throughput of the compact third-order gas-kinetic scheme on one MI355X.

Headline workload (`value`): the batched form -- 96 independent 2D grids of
uneven size advanced together, one launch per phase for all grids and one
hipGraph replay per step: the isentropic vortex of Sec. 4.1 (half of the
grids, periodic [0, 10]^2, Euler or Navier-Stokes) and the quadrant Riemann
problems 1 and 2 of Sec. 4.3 (a quarter each), n^2 cells with n drawn from
{64, 96, 128, 192, 256, 384} by a seeded generator (4.13 M cells per step),
in the FP32-mixed form (single-precision correction terms over
double-precision leading terms and accumulation).  Each grid takes its own
time step from the CFL condition on the device every step.  Synthetic
initial data built from the paper's formulas; the state stays resident in
HBM.

A step is one pass of the whole scheme over every grid: boundary images and
time step, compact reconstruction, every x and y interface (flux and point
values), conservative update.  W untimed warm-up steps, then exactly K timed
steps bracketed by device synchronisation; value = cell-updates / second.

Beside it: the same batch in the FP64 form and over a 200-step window; the
256^2 vortex (Table 2) in both forms; the other full-size workloads of the
paper (`configs`), among them curvilinear grids (the vortex on a waved
512^2 grid, the polar cavity of Sec. 4.8).

`roofline`: the dominant kernel is the interface kernel k_iface_2d; its
algorithmic floating-point operations per launch (the operation count of
the device source per interface, paper_1412_4489_amd/csrc/opcount, Euler or
Navier-Stokes per grid, times the interfaces of each grid) over its average
launch duration, timed live with HIP events on the library's stream in an
eager run of the same K steps; `peak` = 78.6 TFLOP/s, the vector rate this
instruction mix can reach (256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x
2.4 GHz: FP64 and unpacked FP32; packed FP32 is not used); `traffic` from
the committed counter record of the batch while the kernel sources still
match it.

`cpu_baseline`: the FP64 oracle on this host (all its cores) for one step of
every grid of the batch (a fixed step per grid, the grid's first CFL step);
the same step on the GPU gives the L1 difference to the oracle per grid.

`--pmc-probe` runs the counter-collection workload (a 256 MiB calibration
copy, then a few eager steps of the tuned FP32-mixed batch).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_ALU = 78.6e12          # 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz (FP64, unpacked FP32)
PEAK_FP32_PACKED = 157.3e12  # the published vector FP32 figure (packed FP32, not used here)
OPCOUNTS = os.path.join(ROOT, "paper_1412_4489_amd", "csrc", "opcount", "opcounts.json")
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_iface_batch96_fp32mixed.json")
BATCH_WORKLOAD = ("96 grids (isentropic vortex 1/2, 2D Riemann cases 1 and 2 1/4 each), n^2 cells with n in "
                  "{64,96,128,192,256,384}, Euler or Navier-Stokes (Re 100-5000), seed 14124489, CFL steps per grid, "
                  "one launch per phase for all grids, one hipGraph per step")


def n_interfaces(prob):
    """distinct interfaces of a 2D grid (on a periodic axis the last one is the first)"""
    px = prob.bc[0].kind == "periodic"
    py = prob.bc[2].kind == "periodic"
    return (prob.nx if px else prob.nx + 1) * prob.ny + prob.nx * (prob.ny if py else prob.ny + 1)


def interface_flops(probs, form="fp32_mixed"):
    """algorithmic operations of one interface launch covering `probs`"""
    ops = json.load(open(OPCOUNTS))
    return sum(n_interfaces(p) * ops[f"interface_{'ns' if p.viscous else 'euler'}_{form}"]["total"] for p in probs)


def counter_record():
    """The committed counter record of the interface kernel on the batch, or
    {} if there is none for the present kernel sources."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return {}
    from paper_1412_4489_amd.profiling import source_hash
    return rec if rec.get("source_hash") == source_hash() else {}


def pmc_probe():
    """Counter-collection workload: a plain 256 MiB device copy (the
    calibration of FETCH_SIZE / WRITE_SIZE), then the tuned FP32-mixed batch
    for a few eager steps."""
    import torch
    from paper_1412_4489_amd import gks
    from paper_1412_4489_amd import workloads as W
    x = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    items = W.batch()
    side = torch.cuda.Stream()
    with gks.Solver([p for p, _ in items], [s for _, s in items], gks.GKS_FP32_MIXED, stream=side.cuda_stream) as S:
        S.tune(2)
        gks.gks_profile(S.h, 1)
        S.step(3)
        S.fetch()
    torch.cuda.synchronize()
    print("pmc probe done", flush=True)


def launch_forms(S, steps):
    """Interface kernel time per launch (HIP events) at the tuned block size
    in the one-block-per-tile form and in the persistent form (the tuner's
    grid, else four waves per compute unit), and the reconstruction's time in
    row order and in LDS tiles; the tuned shapes are restored."""
    import torch
    from paper_1412_4489_amd import gks
    bs, grid = S.launch_shape("interface")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = {}
    for name, g in (("per_tile", 0), ("persistent", grid or cus * 256 // bs)):
        S.set_launch("interface", bs, g)
        S.step(2)
        torch.cuda.synchronize()
        gks.gks_profile(S.h, 1)
        gks.gks_profile(S.h, 2)
        S.step(steps)
        torch.cuda.synchronize()
        gks.gks_profile(S.h, 0)
        ms, n = gks.gks_kernel_time(S.h, "interface")
        out[name] = {"threads": bs, "grid": g, "interface_ms": round(ms / max(n, 1), 5)}
    S.set_launch("interface", bs, grid)
    out["tuned"] = "persistent" if grid else "per_tile"
    # the reconstruction in row order and in LDS tiles of 1, 2 and 4 rows
    rbs, rrows = S.launch_shape("recon")
    rec = {}
    for rows in (0, 1, 2, 4):
        S.set_launch("recon", rbs, rows)
        S.step(2)
        torch.cuda.synchronize()
        gks.gks_profile(S.h, 1)
        gks.gks_profile(S.h, 2)
        S.step(steps)
        torch.cuda.synchronize()
        gks.gks_profile(S.h, 0)
        ms, n = gks.gks_kernel_time(S.h, "recon")
        rec[f"rows_{rows}" if rows else "row_order"] = round(ms / max(n, 1), 5)
    S.set_launch("recon", rbs, rrows)
    out["recon_ms"] = {"threads": rbs, **rec, "tuned": f"rows_{rrows}" if rrows else "row_order"}
    return out


def run_gpu(items, precision, steps, warmup, long_steps=0, forms=False):
    """Times `steps` graph-replayed steps after `warmup` (tuned launch shapes)
    and, in an eager run of the same number of steps, every kernel class with
    HIP events on the library's stream.  Returns (wall, kernel times, probs,
    launch shapes, long-window wall, interface launch forms or None)."""
    import torch
    from paper_1412_4489_amd import gks
    probs, states = [p for p, _ in items], [s for _, s in items]
    side = torch.cuda.Stream()  # a torch stream the library borrows
    S = gks.Solver(probs, states, precision, stream=side.cuda_stream)
    S.tune(3)
    sizes = {k: S.launch_shape(k) for k in ("ghost", "recon", "interface", "update")}
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
    wall_long = None
    if long_steps:
        t0 = time.perf_counter()
        S.step(long_steps)
        torch.cuda.synchronize()
        wall_long = time.perf_counter() - t0
    lf = launch_forms(S, steps) if forms else None
    for k in range(len(probs)):
        S.fetch(k)  # raises if a grid produced a nonphysical state
    S.close()
    return wall, kt, probs, sizes, wall_long, lf


def config_rates(steps=20, warmup=3):
    """Throughput of the other full-size 2D workloads of the paper (FP32-mixed
    and FP64): tuned launch shapes, graph replays, steps from the CFL
    condition.  Returns {name: {form: Mcell-updates/s}}."""
    import torch
    from paper_1412_4489_amd import gks
    from paper_1412_4489_amd import workloads as W
    out = {}
    for name, mk in (("isentropic_vortex_256x256", lambda: W.vortex_2d(256)),
                     ("cavity_512x512_ns_re1000", lambda: W.cavity(512)),
                     ("double_mach_reflection_1920x480", lambda: W.dmr(1920, 480)),
                     ("double_mach_reflection_1920x480_characteristic", lambda: W.dmr(1920, 480, recon_vars=1)),
                     ("shock_vortex_801x401_characteristic", lambda: W.shock_vortex(801, 401)),
                     ("riemann2_400x400_characteristic", lambda: W.riemann_2d(2, n=400, recon_vars=1)),
                     ("forward_facing_step_240x80_characteristic", lambda: W.forward_facing_step(240, 80)),
                     ("viscous_shock_tube_600x300_re1000", lambda: W.viscous_shock_tube(600, 300, re=1000.0)),
                     ("curvilinear_waved_vortex_512x512", lambda: W.vortex_mapped(512, amp=0.05)),
                     ("curvilinear_polar_cavity_65x65_re350", lambda: W.polar_cavity(65, re=350.0))):
        prob, st = mk()
        out[name] = {}
        for fname, prec in (("fp32_mixed", gks.GKS_FP32_MIXED), ("fp64", gks.GKS_FP64)):
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
            out[name][fname] = round(gas * steps / wall / 1e6, 3)
        print(f"# {name}: {out[name]}", file=sys.stderr, flush=True)
    return out


def cpu_baseline(items):
    """The oracle (FP64, all host cores) for one step of every grid, each with
    its first CFL step; returns the baseline record, the oracle's states and
    the steps."""
    import oracle
    oracle.lib()
    dts = [oracle.dt(p, s) for p, s in items]
    refs = [s.copy() for _, s in items]
    t0 = time.perf_counter()
    for (p, _), r, dt in zip(items, refs, dts):
        oracle.step(p, r, dt, 0.0)
    sec = time.perf_counter() - t0
    cells = sum(p.ncells for p, _ in items)
    rec = {"value": round(cells / sec / 1e6, 4), "unit": "Mcell-updates/s", "cores": oracle.num_threads(),
           "kind": "oracle",
           "sample": f"one step of each of the 96 grids of the batch ({cells} cell-updates, each grid with its "
                     f"first CFL step), FP64, OpenMP over rows; {sec:.1f} s"}
    return rec, refs, dts


def gpu_one_step(items, precision, dts):
    from paper_1412_4489_amd import gks
    probs, states = [p for p, _ in items], [s for _, s in items]
    with gks.Solver(probs, states, precision) as S:
        S.step(1, dt=dts)
        return [S.fetch(k)[0] for k in range(len(probs))]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--long-steps", type=int, default=200, help="steps of the long window of the headline form")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-configs", action="store_true", help="skip the other full-size workloads")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only run the copy calibration and a few batch steps (for rocprofv3 --pmc)")
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
    from paper_1412_4489_amd import workloads as W

    items = W.batch()
    wall, kt, probs, sizes, wall_long, forms = run_gpu(items, gks.GKS_FP32_MIXED, a.steps, a.warmup, a.long_steps,
                                                       forms=True)
    cells = sum(p.ncells for p in probs)
    value = cells * a.steps / wall / 1e6
    print(f"# batch fp32_mixed: {a.steps} steps in {wall * 1e3:.2f} ms; launch shapes {sizes}; kernel ms: "
          + ", ".join(f"{k} {v[0]:.2f} ({v[1]})" for k, v in kt.items()), file=sys.stderr, flush=True)
    ms_if, nl = kt["interface"]
    t_if = ms_if / 1e3 / max(nl, 1)
    fl = interface_flops(probs, "fp32_mixed")
    achieved = fl / t_if

    wall64, kt64, _, sizes64, _, _ = run_gpu(items, gks.GKS_FP64, a.steps, a.warmup)
    ms64, nl64 = kt64["interface"]
    t_if64 = ms64 / 1e3 / max(nl64, 1)
    achieved64 = interface_flops(probs, "fp64") / t_if64
    print(f"# batch fp64: {a.steps} steps in {wall64 * 1e3:.2f} ms; launch shapes {sizes64}", file=sys.stderr, flush=True)

    rec = counter_record()
    ops = json.load(open(OPCOUNTS))
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
        "config": {"workload": BATCH_WORKLOAD, "form": "GKS_FP32_MIXED", "problems": len(probs), "cells": cells,
                   "interfaces": sum(n_interfaces(p) for p in probs),
                   "viscous_grids": sum(bool(p.viscous) for p in probs)},
        "launch": {"fp32_mixed": sizes, "fp64": sizes64, "interface_forms_fp32_mixed": forms},
        "long_window": None if wall_long is None else {
            "steps": a.long_steps, "value": round(cells * a.long_steps / wall_long / 1e6, 3),
            "ms_per_step": round(wall_long / a.long_steps * 1e3, 5)},
        "fp64": {"value": round(cells * a.steps / wall64 / 1e6, 3), "ms_per_step": round(wall64 / a.steps * 1e3, 5),
                 "interface_ms": round(t_if64 * 1e3, 5), "interface_tflops": round(achieved64 / 1e12, 3),
                 "interface_frac": round(achieved64 / PEAK_ALU, 4)},
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 4), "peak": PEAK_ALU / 1e12,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_ALU, 5),
                     "traffic": rec.get("bytes_per_launch"),
                     "kernel": (f"k_iface_2d_loop<float> (persistent, {sizes['interface'][1]} blocks of "
                                f"{sizes['interface'][0]}; one launch per step for all 96 grids)"
                                if sizes["interface"][1] else
                                f"k_iface_2d<float> (blocks of {sizes['interface'][0]}; one launch per step for all "
                                "96 grids)"),
                     "interface_ms": round(t_if * 1e3, 5), "flops_per_launch": fl,
                     "flops_per_interface": {"euler": ops["interface_euler_fp32_mixed"]["total"],
                                             "navier_stokes": ops["interface_ns_fp32_mixed"]["total"]},
                     "peak_fp32_packed": PEAK_FP32_PACKED / 1e12,
                     "frac_of_fp32_packed": round(achieved / PEAK_FP32_PACKED, 5),
                     "valu_busy": rec.get("valu_busy"),
                     "traffic_per_algorithmic_bytes": rec.get("traffic_per_algorithmic_bytes")},
    }
    if not a.no_configs:
        out["configs"] = config_rates()
    if not a.no_cpu:
        cb, refs, dts = cpu_baseline(items)
        out["cpu_baseline"] = cb
        errs, drift = {}, {}
        for name, prec in (("fp32_mixed", gks.GKS_FP32_MIXED), ("fp64", gks.GKS_FP64)):
            got = gpu_one_step(items, prec, dts)
            e_v, e_r, d_v = [], [], []
            for (p, st0), g_, r in zip(items, got, refs):
                e = float(np.abs(g_.cell[0] - r.cell[0]).mean() / np.abs(r.cell[0]).mean())
                (e_v if "vortex" in p.name else e_r).append(e)
                if "vortex" in p.name:  # periodic: mass, momentum and energy are conserved exactly
                    t0_ = st0.cell.sum(axis=(1, 2))
                    d_v.append(float(np.max(np.abs(g_.cell.sum(axis=(1, 2)) - t0_) / np.abs(t0_))))
            errs[name] = {"vortex_max": float(f"{max(e_v):.3e}"), "riemann_max": float(f"{max(e_r):.3e}")}
            drift[name] = float(f"{max(d_v):.3e}")
        out["l1_rel_err_vs_oracle"] = errs
        out["conservation_drift"] = drift
        out["l1_sample"] = "rho after one step of every grid from the same initial state and step, per grid"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
