"""Summaries of rocprofv3 output for the kernels of libgks.so.

Reads the CSV files of `rocprofv3 --kernel-trace --stats --output-format csv`
and of `rocprofv3 --pmc <counters> --output-format csv` runs and writes short
Markdown / JSON summaries:

  * kernel_table: per kernel and launch size, calls and average / min / max
    duration;
  * traffic: HBM bytes per dispatch of the interface kernel from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by the factor a plain device copy
    of known size needs (the 256 MiB copies at the start of `bench.py
    --pmc-probe`: bytes read and written = 256 MiB each);
  * sq: VALU instructions and wave counts per dispatch.

    python -m paper_1412_4489_amd.profiling --trace T.csv --fetch F.csv \\
        --write W.csv --sq S.csv --out profiles/

writes kernels_batch96.md (both forms of the 96-grid batch),
counters_iface_batch96_fp32mixed.md and traffic_iface_batch96_fp32mixed.json
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
IFACE = "k_iface_2d"
IFACE_NAMES = ("k_iface_2d", "k_iface_2d_loop")  # one block per tile; persistent form
CUS, CLOCK_MHZ = 256, 2400  # MI355X compute units and clock (VALUBusy below)
PROBE_STEPS = 3  # the tuned-shape steps that end bench.py --pmc-probe
BATCH_CELLS = 4130816
BATCH_ALG_BYTES = BATCH_CELLS * 192  # state read once and written once per step, FP32-mixed
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


def _counter_rows(path):
    with open(path) as fh:
        return list(csv.DictReader(fh))


def _batch_iface_rows(rows, ttype="float"):
    """counter rows of the interface launches of the probe's last steps (the
    tuned launch shape; the tuner's trial launches come before them)"""
    rows = [(n, r) for n, r in enumerate(rows) if _short(r["Kernel_Name"]) in [(k, ttype) for k in IFACE_NAMES]]
    ids = sorted({int(r.get("Dispatch_Id", n)) for n, r in rows})[-PROBE_STEPS:]
    return [r for n, r in rows if int(r.get("Dispatch_Id", n)) in ids]


def traffic(fetch_csv, write_csv):
    """Scaled HBM bytes per dispatch of the interface kernel on the batch."""
    out = {}
    for name, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = _counter_rows(path)
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]][:3]
        if len(copies) < 3:
            raise ValueError(f"{path}: the three calibration copies are missing")
        factor = (COPY_BYTES / 1024.0) / (sum(copies) / 3)
        per = collections.defaultdict(float)
        for n, r in enumerate(_batch_iface_rows(rows)):
            per[r.get("Dispatch_Id", n)] += float(r["Counter_Value"])
        vals = list(per.values())
        out[name] = {"factor": factor, "copy_kib": sum(copies) / 3, "kib_per_dispatch": sum(vals) / len(vals),
                     "dispatches": len(vals)}
    out["bytes_per_launch"] = sum(out[n]["kib_per_dispatch"] * 1024.0 * out[n]["factor"] for n in ("fetch", "write"))
    return out


def sq_summary(sq_csv):
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    for n, r in enumerate(_batch_iface_rows(_counter_rows(sq_csv))):
        per[r.get("Dispatch_Id", n)][r["Counter_Name"]] += float(r["Counter_Value"])
    d = list(per.values())
    m = {c: sum(x.get(c, 0.0) for x in d) / len(d) for c in d[0]}
    return {"waves": m["SQ_WAVES"], "valu_per_wave": m["SQ_INSTS_VALU"] / m["SQ_WAVES"],
            "valu_quad_cycles": m.get("SQ_ACTIVE_INST_VALU", 0.0)}


def valu_busy(quad_cycles, duration_us):
    """rocprofv3's VALUBusy (sum of SQ_ACTIVE_INST_VALU / CUs / GPU cycles),
    with the kernel's own duration from the kernel trace as the cycle count:
    the fraction of time the vector ALUs of a CU (4 SIMDs, one quad-cycle per
    wave instruction) are issuing."""
    return quad_cycles / CUS / (duration_us * CLOCK_MHZ)


TRACE_CMD = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats -d $O/prof_bench "
             "-o bench --output-format csv -- python -u $R/bench.py --steps 20 --warmup 5 --long-steps 0 "
             "--no-cpu --no-configs")
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


def _step_line(d, iface):
    tot = iface + d["k_recon_2d"] + d["k_update_2d"] + d["k_ghost_2d"]
    return (f"interface {iface:.1f} us; reconstruction {d['k_recon_2d']:.1f}, update "
            f"{d['k_update_2d']:.1f}, boundary (+ time step) {d['k_ghost_2d']:.1f}; sum {tot:.1f} us")


def headline_iface(agg, ttype="float"):
    """(kernel, type, grid) and durations of the interface launches of the
    tuned shape: the group with the most calls (the timed steps; the tuner's
    trial shapes have a few each)"""
    groups = [(key, v) for key, v in agg.items() if key[0] in IFACE_NAMES and key[1] == ttype]
    return max(groups, key=lambda kv: len(kv[1])) if groups else (None, [])


def batch_iface_duration(trace_csv, ttype="float"):
    """average duration (us) of the interface kernel's launches in the tuned shape"""
    _, v = headline_iface(kernel_table(trace_csv), ttype)
    return sum(v) / len(v) if v else None


def write_kernel_summaries(trace_csv, out):
    agg = kernel_table(trace_csv)
    avg = _averages({k: v for k, v in agg.items() if k[0] not in IFACE_NAMES})
    md = kernel_markdown(agg, f"Kernel trace: 96-grid batch ({BATCH_CELLS} cells), GKS_FP32_MIXED and GKS_FP64",
                         TRACE_CMD)
    md += "\nPer step (averages over the launch sizes of a kernel; each launch covers all 96 grids):\n\n"
    for t, name in (("float", "FP32-mixed"), ("double", "FP64")):
        key, v = headline_iface(agg, t)
        if t in avg and v:
            md += (f"* {name} (interface launch {key[0]}, {key[2]} threads): "
                   f"{_step_line(avg[t], sum(v) / len(v))}\n")
    md += ("\nThe tuned shape of the interface launch is the row with the most calls; the tuner's timing steps "
           "(64, 128, 256 threads per block, and the persistent form) add launches of other sizes, also to the "
           "smaller kernels' rows.\n")
    with open(os.path.join(out, "kernels_batch96.md"), "w") as fh:
        fh.write(md)


def counted_shape(counter_csv):
    """(kernel, type, grid threads) of the interface dispatches a counter
    pass counted (each pass is its own process, which tunes its own launch
    shapes)"""
    rows = _batch_iface_rows(_counter_rows(counter_csv))
    shapes = {(*_short(r["Kernel_Name"]), int(r["Grid_Size"])) for r in rows}
    if len(shapes) != 1:
        raise ValueError(f"{counter_csv}: the counted interface dispatches have several shapes {shapes}")
    return shapes.pop()


def write_counter_summaries(fetch_csv, write_csv, sq_csv, out, trace_csv=None):
    shapes = {path: counted_shape(path) for path in (fetch_csv, write_csv, sq_csv) if path}
    if len(set(shapes.values())) != 1:
        raise ValueError(f"the counter passes counted different launch shapes: {shapes}")
    shape = next(iter(shapes.values()))
    tr = traffic(fetch_csv, write_csv)
    sq = sq_summary(sq_csv) if sq_csv else {}
    # the kernel's duration: the trace's launches of the counted shape
    dur = None
    if trace_csv:
        v = kernel_table(trace_csv).get(shape)
        dur = sum(v) / len(v) if v else None
    busy = valu_busy(sq["valu_quad_cycles"], dur) if sq and dur else None
    rec = {"source_hash": source_hash(),
           "workload": "96-grid batch, GKS_FP32_MIXED, tuned launch shapes",
           "bytes_per_launch": round(tr["bytes_per_launch"]),
           "algorithmic_bytes_per_step": BATCH_ALG_BYTES,
           "traffic_per_algorithmic_bytes": round(tr["bytes_per_launch"] / BATCH_ALG_BYTES, 3),
           "fetch_factor": tr["fetch"]["factor"], "write_factor": tr["write"]["factor"],
           "fetch_kib_per_dispatch": tr["fetch"]["kib_per_dispatch"],
           "write_kib_per_dispatch": tr["write"]["kib_per_dispatch"],
           "waves": sq.get("waves"), "valu_instructions_per_wave": sq.get("valu_per_wave"),
           "launch": {"kernel": shape[0], "type": shape[1], "grid_threads": shape[2]},
           "duration_us": dur, "valu_busy": None if busy is None else round(busy, 4)}
    with open(os.path.join(out, "traffic_iface_batch96_fp32mixed.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    t = ["# Counters: interface kernel (tuned launch shape), 96-grid batch, GKS_FP32_MIXED", "",
         "Commands (on the machine with the GPU, from /tmp with TMPDIR=/tmp, repository root R, output directory O), "
         "one counter pass per run:", ""]
    t += [f"    timeout -s KILL 120 rocprofv3 --pmc {c} -d $O/{d} -o {o} --output-format csv "
          "-- python -u $R/bench.py --pmc-probe" for c, d, o in PMC_PASSES]
    t += ["", "Summary:", "", "    " + SUMMARY_CMD, "",
          "Calibration: `bench.py --pmc-probe` first copies 256 MiB three times (`__amd_rocclr_copyBuffer`).",
          f"FETCH_SIZE reads {tr['fetch']['copy_kib']:.0f} KiB per copy (factor {tr['fetch']['factor']:.4f}), "
          f"WRITE_SIZE {tr['write']['copy_kib']:.0f} KiB (factor {tr['write']['factor']:.4f}).", "",
          f"Counted launch (the same in every pass): {shape[0]}<{shape[1]}> over {shape[2]} threads.", "",
          "VALUBusy = SQ_ACTIVE_INST_VALU (quad-cycles, all CUs) / 256 CUs / kernel cycles (the mean duration "
          "of the same launch shape in the kernel trace x 2.4 GHz).", "",
          "| FETCH_SIZE (KiB/dispatch) | WRITE_SIZE (KiB/dispatch) | HBM bytes/dispatch (scaled) | waves "
          "| VALU instr./wave | duration (us) | VALUBusy |", "|---:|---:|---:|---:|---:|---:|---:|",
          f"| {tr['fetch']['kib_per_dispatch']:.0f} | {tr['write']['kib_per_dispatch']:.0f} "
          f"| {tr['bytes_per_launch'] / 1e6:.1f} MB | {sq.get('waves', 0):.0f} | {sq.get('valu_per_wave', 0):.0f} "
          f"| {dur or 0:.1f} | {100 * (busy or 0):.0f} % |", "",
          f"Algorithmic bytes of the whole step: {BATCH_ALG_BYTES / 1e6:.0f} MB ({BATCH_CELLS} cells x 192 B: four "
          "double averages and sixteen single-precision point values read once and written once); the interface "
          f"launch moves {tr['bytes_per_launch'] / BATCH_ALG_BYTES:.2f} times that.", "",
          "traffic_iface_batch96_fp32mixed.json holds these figures with the hash of the kernel sources they "
          "were taken from (bench.py reports `traffic` only while the sources match)."]
    with open(os.path.join(out, "counters_iface_batch96_fp32mixed.md"), "w") as fh:
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
