"""Summaries of rocprofv3 output for the kernels of libgks.so.

Reads the CSV files of `rocprofv3 --kernel-trace --stats --output-format csv`
and of `rocprofv3 --pmc <counters> --output-format csv` runs and writes short
Markdown / JSON summaries:

  * kernel_table: per kernel and launch size, calls and average / min / max
    duration (selected by grid size: one workload of a run);
  * traffic: HBM bytes per dispatch of the interface kernels from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by the factor a plain device copy
    of known size needs (the 256 MiB copies at the start of `bench.py
    --pmc-probe`: bytes read and written = 256 MiB each);
  * sq: VALU instructions and wave counts per dispatch.

    python -m paper_1412_4489_amd.profiling --trace T.csv --fetch F.csv \\
        --write W.csv --sq S.csv --out profiles/

writes kernels_vortex256_fp32mixed_fp64.md, kernels_batch96_fp32mixed.md,
counters_iface_vortex256_fp32mixed.md and traffic_iface_vortex256_fp32mixed.json
(the record bench.py reads while the kernel sources still hash to the same
value).

Nothing here runs on the GPU.
"""
from __future__ import annotations

import argparse
import collections
import csv
import json
import os
import re

COPY_BYTES = 256 << 20  # the calibration copies of bench.py --pmc-probe
IFACE = ("k_iface_pro_2d", "k_iface_corr_2d", "k_iface_kin1_2d")
FACES_256 = 131072  # interface threads of the periodic 256 x 256 grid
CUS, CLOCK_MHZ = 256, 2400  # MI355X compute units and clock (VALUBusy below)
BATCH_MIN_GRID = 400000  # launches of the 96-grid batch are larger than this
KERNEL_SOURCES = ("gks.hip", "gks_device.h", "interface_gen.h")
HERE = os.path.dirname(os.path.abspath(__file__))


def source_hash():
    """Hash of the kernel sources: a stored counter record is valid only for them."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _short(name):
    m = re.search(r"(k_[a-z_0-9]+)<([a-z]+)", name)
    return (m.group(1), m.group(2)) if m else (name.split("(")[0][:40], "")


def kernel_table(trace_csv, grid_sizes=None):
    """{(kernel, type, grid): [durations in us]} from a kernel-trace CSV."""
    agg = collections.defaultdict(list)
    with open(trace_csv) as fh:
        for r in csv.DictReader(fh):
            k, t = _short(r["Kernel_Name"])
            if not k.startswith("k_"):
                continue
            g = int(r["Grid_Size_X"])
            if grid_sizes is not None and g not in grid_sizes:
                continue
            agg[(k, t, g)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0)
    return agg


def kernel_markdown(agg, title, command):
    lines = [f"# {title}", "", "Command (on the machine with the GPU, repository root R, output directory O):", "", "    " + command, "",
             "| kernel | type | grid (threads) | calls | average (us) | min (us) | max (us) |",
             "|---|---|---:|---:|---:|---:|---:|"]
    for (k, t, g), v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| {k} | {t} | {g} | {len(v)} | {sum(v) / len(v):.2f} | {min(v):.2f} | {max(v):.2f} |")
    return "\n".join(lines) + "\n"


def threads(kernel, faces):
    """Launch size of an interface kernel: the combined hydrodynamic / kinetic
    side 0 launch has two blocks per tile."""
    return 2 * faces if kernel == "k_iface_corr_2d" else faces


def _counter_rows(path):
    with open(path) as fh:
        return list(csv.DictReader(fh))


def traffic(fetch_csv, write_csv, faces, ttype="float"):
    """Scaled HBM bytes per dispatch of the interface kernels."""
    out = {}
    for name, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = _counter_rows(path)
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]][:3]
        if len(copies) < 3:
            raise ValueError(f"{path}: the three calibration copies are missing")
        factor = (COPY_BYTES / 1024.0) / (sum(copies) / 3)
        per = collections.defaultdict(list)
        for r in rows:
            k, t = _short(r["Kernel_Name"])
            if k in IFACE and t == ttype and int(r["Grid_Size"]) == threads(k, faces):
                per[k].append(float(r["Counter_Value"]))
        out[name] = {"factor": factor, "copy_kib": sum(copies) / 3,
                     "kib_per_dispatch": {k: sum(v) / len(v) for k, v in per.items()}}
    per_set = 0.0
    for name in ("fetch", "write"):
        d = out[name]
        for k, kib in d["kib_per_dispatch"].items():
            per_set += kib * 1024.0 * d["factor"]
    out["bytes_per_launch_set"] = per_set
    return out


def sq_summary(sq_csv, faces, ttype="float"):
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in _counter_rows(sq_csv):
        k, t = _short(r["Kernel_Name"])
        if k.startswith("k_") and t == ttype:
            per[(k, int(r["Grid_Size"]))][r["Counter_Name"]].append(float(r["Counter_Value"]))
    res = {}
    for key, d in per.items():
        m = {c: sum(v) / len(v) for c, v in d.items()}
        if m.get("SQ_WAVES"):
            res[key] = {"waves": m["SQ_WAVES"], "valu_per_wave": m["SQ_INSTS_VALU"] / m["SQ_WAVES"],
                        "valu_quad_cycles": m.get("SQ_ACTIVE_INST_VALU", 0.0)}
    return res


def valu_busy(quad_cycles, duration_us):
    """rocprofv3's VALUBusy (sum of SQ_ACTIVE_INST_VALU / CUs / GPU cycles),
    with the kernel's own duration from the kernel trace as the cycle count:
    the fraction of time the vector ALUs of a CU (4 SIMDs, one quad-cycle per
    wave instruction) are issuing."""
    return quad_cycles / CUS / (duration_us * CLOCK_MHZ)


TRACE_CMD = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats -d $O/prof_bench "
             "-o bench --output-format csv -- python -u $R/bench.py --steps 50 --warmup 5 --no-cpu --no-configs")
PMC_PASSES = (("FETCH_SIZE", "pmc_fetch", "f"), ("WRITE_SIZE", "pmc_write", "w"),
              ("SQ_WAVES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_WAVE_CYCLES SQ_BUSY_CYCLES GRBM_GUI_ACTIVE",
               "pmc_sq", "s"))
SUMMARY_CMD = ("python -m paper_1412_4489_amd.profiling --trace $O/prof_bench/bench_kernel_trace.csv "
               "--fetch $O/pmc_fetch/f_counter_collection.csv "
               "--write $O/pmc_write/w_counter_collection.csv "
               "--sq $O/pmc_sq/s_counter_collection.csv --out $R/profiles")


def _averages(agg):
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    for (k, t, _g), v in agg.items():
        per[t][k].extend(v)
    return {t: {k: sum(v) / len(v) for k, v in d.items()} for t, d in per.items()}


def _step_line(d):
    iface = d["k_iface_pro_2d"] + d["k_iface_corr_2d"] + d["k_iface_kin1_2d"]
    tot = iface + d["k_recon_2d"] + d["k_update_2d"] + d["k_ghost_2d"]
    return (f"interface phases {d['k_iface_pro_2d']:.1f} + {d['k_iface_corr_2d']:.1f} + "
            f"{d['k_iface_kin1_2d']:.1f} = {iface:.1f} us; reconstruction {d['k_recon_2d']:.1f}, update "
            f"{d['k_update_2d']:.1f}, boundary (+ time step) {d['k_ghost_2d']:.1f}; sum {tot:.1f} us")


def write_kernel_summaries(trace_csv, out):
    agg = kernel_table(trace_csv)
    small = {k: v for k, v in agg.items() if k[2] < BATCH_MIN_GRID}
    big = {k: v for k, v in agg.items() if k[2] >= BATCH_MIN_GRID}
    avg = _averages(small)
    md = kernel_markdown(small, "Kernel trace: isentropic vortex 256 x 256, GKS_FP32_MIXED and GKS_FP64", TRACE_CMD)
    md += ("\nPer step (averages over the launch sizes of a kernel):\n\n"
           f"* FP32-mixed: {_step_line(avg['float'])}\n* FP64: {_step_line(avg['double'])}\n\n"
           f"{FACES_256} interface threads: on the periodic grid the last interface of each row and column is "
           "the first.\nThe same run also holds the 96-grid batch (kernels_batch96_fp32mixed.md).\n")
    with open(os.path.join(out, "kernels_vortex256_fp32mixed_fp64.md"), "w") as fh:
        fh.write(md)
    if big:
        d = _averages(big)["float"]
        md = kernel_markdown(big, "Kernel trace: 96-grid batch (4 130 816 cells), GKS_FP32_MIXED", TRACE_CMD)
        md += (f"\nPer step: {_step_line(d)}; each launch covers all 96 grids (the launch sizes of a "
               "kind differ with the tuned block size).\n")
        with open(os.path.join(out, "kernels_batch96_fp32mixed.md"), "w") as fh:
            fh.write(md)


def write_counter_summaries(fetch_csv, write_csv, sq_csv, out, trace_csv=None):
    tr = traffic(fetch_csv, write_csv, FACES_256)
    sq = sq_summary(sq_csv, FACES_256) if sq_csv else {}
    # kernel durations of the same workload (FP32-mixed, 256 x 256) from the trace
    dur = {}
    if trace_csv:
        for (k, t, g), v in kernel_table(trace_csv).items():
            if t == "float" and k in IFACE and g == threads(k, FACES_256):
                dur[k] = sum(v) / len(v)
    busy = {k: valu_busy(sq[(k, threads(k, FACES_256))]["valu_quad_cycles"], dur[k])
            for k in IFACE if k in dur and (k, threads(k, FACES_256)) in sq}
    busy_set = None
    if len(busy) == len(IFACE):
        busy_set = (sum(sq[(k, threads(k, FACES_256))]["valu_quad_cycles"] for k in IFACE) / CUS
                    / (sum(dur[k] for k in IFACE) * CLOCK_MHZ))
    rec = {"source_hash": source_hash(),
           "workload": "isentropic vortex 256x256, GKS_FP32_MIXED, tuned launch shapes",
           "bytes_per_launch_set": round(tr["bytes_per_launch_set"]),
           "fetch_factor": tr["fetch"]["factor"], "write_factor": tr["write"]["factor"],
           "fetch_kib_per_dispatch": tr["fetch"]["kib_per_dispatch"],
           "write_kib_per_dispatch": tr["write"]["kib_per_dispatch"],
           "valu_busy": {k: round(v, 4) for k, v in busy.items()},
           "valu_busy_launch_set": None if busy_set is None else round(busy_set, 4)}
    with open(os.path.join(out, "traffic_iface_vortex256_fp32mixed.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    t = ["# Counters: interface kernels, isentropic vortex 256 x 256, GKS_FP32_MIXED", "",
         "Commands (on the machine with the GPU, from /tmp with TMPDIR=/tmp, repository root R, output directory O), one counter pass per run:", ""]
    t += [f"    timeout -s KILL 120 rocprofv3 --pmc {c} -d $O/{d} -o {o} --output-format csv "
          "-- python -u $R/bench.py --pmc-probe" for c, d, o in PMC_PASSES]
    t += ["", "Summary:", "", "    " + SUMMARY_CMD, "",
          "Calibration: `bench.py --pmc-probe` first copies 256 MiB three times (`__amd_rocclr_copyBuffer`).",
          f"FETCH_SIZE reads {tr['fetch']['copy_kib']:.0f} KiB per copy (factor {tr['fetch']['factor']:.4f}), "
          f"WRITE_SIZE {tr['write']['copy_kib']:.0f} KiB (factor {tr['write']['factor']:.4f}).", "",
          "VALUBusy = SQ_ACTIVE_INST_VALU (quad-cycles, all CUs) / 256 CUs / kernel cycles (the kernel's mean "
          "duration in the kernel trace x 2.4 GHz).", "",
          "| kernel | FETCH_SIZE (KiB/dispatch) | WRITE_SIZE (KiB/dispatch) | HBM bytes/dispatch (scaled) | waves "
          "| VALU instr./wave | duration (us) | VALUBusy |", "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for k in IFACE:
        f_, w_ = tr["fetch"]["kib_per_dispatch"][k], tr["write"]["kib_per_dispatch"][k]
        b = (f_ * tr["fetch"]["factor"] + w_ * tr["write"]["factor"]) * 1024
        s_ = sq.get((k, threads(k, FACES_256)), {})
        t.append(f"| {k} | {f_:.0f} | {w_:.0f} | {b / 1e6:.1f} MB | {s_.get('waves', 0):.0f} "
                 f"| {s_.get('valu_per_wave', 0):.0f} | {dur.get(k, 0):.2f} | {100 * busy.get(k, 0):.0f} % |")
    t += ["", f"Interface launch set (prologue, hydrodynamic + kinetic side 0, kinetic side 1): "
          f"{tr['bytes_per_launch_set'] / 1e6:.1f} MB "
          "of HBM traffic per step; the algorithmic bytes of the whole step are 12.6 MB (65536 cells x 192 B).",
          "Most of the difference is the frame record: the prologue writes 9 doubles + 36 coefficients per "
          "interface, kinetic side 0 leaves 4 doubles + 8 point values for side 1, and the phases "
          "read-modify-write the fluxes and point values.",
          "" if busy_set is None else f"VALUBusy of the launch set: {100 * busy_set:.0f} %.", "",
          "traffic_iface_vortex256_fp32mixed.json holds these figures with the hash of the kernel sources they "
          "were taken from (bench.py reports `traffic` only while the sources match)."]
    with open(os.path.join(out, "counters_iface_vortex256_fp32mixed.md"), "w") as fh:
        fh.write("\n".join(t) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--sq")
    ap.add_argument("--out", default="profiles")
    a = ap.parse_args()
    if a.trace:
        write_kernel_summaries(a.trace, a.out)
    if a.fetch and a.write:
        write_counter_summaries(a.fetch, a.write, a.sq, a.out, a.trace)


if __name__ == "__main__":
    main()
