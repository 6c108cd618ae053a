"""The counter summary pairs each counter figure with the launch shape it
counted: every pass must have counted the same interface launch shape, and
the kernel's duration comes from the trace's launches of exactly that shape
(host-only, synthetic rocprofv3 CSV files)."""
import csv
import json

import pytest

from paper_1412_4489_amd import profiling as P

NAME = "void (anonymous namespace)::k_iface_2d<float, float, float, false, 64u>(KA)"
LOOP = "void (anonymous namespace)::k_iface_2d_loop<float, float, float, false, 64u>(KA)"


def _trace(path):
    rows = []
    for name, grid, us, n in ((NAME, 8277632, 2200.0, 30), (LOOP, 65536, 2300.0, 40)):
        for k in range(n):
            rows.append({"Kernel_Name": name, "Grid_Size_X": grid, "Start_Timestamp": 10 ** 9 * k,
                         "End_Timestamp": 10 ** 9 * k + int(us * 1000)})
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def _counters(path, counters, name=NAME, grid=8277632):
    rows, d = [], 0
    for _ in range(3):
        d += 1
        for c in counters:
            rows.append({"Dispatch_Id": d, "Kernel_Name": "__amd_rocclr_copyBuffer", "Grid_Size": 1,
                         "Counter_Name": c, "Counter_Value": P.COPY_BYTES / 1024.0})
    for _ in range(P.PROBE_STEPS):
        d += 1
        for c in counters:
            rows.append({"Dispatch_Id": d, "Kernel_Name": name, "Grid_Size": grid, "Counter_Name": c,
                         "Counter_Value": 1000.0 if c != "SQ_WAVES" else 129338.0})
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_duration_of_the_counted_shape(tmp_path):
    tr = tmp_path / "trace.csv"
    _trace(tr)
    f, w, s = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "s.csv"
    _counters(f, ["FETCH_SIZE"])
    _counters(w, ["WRITE_SIZE"])
    _counters(s, ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU"])
    P.write_counter_summaries(str(f), str(w), str(s), str(tmp_path), str(tr))
    rec = json.load(open(tmp_path / "traffic_iface_batch96_fp32mixed.json"))
    # the per-tile launch was counted: its 2200 us, not the persistent
    # form's 2300 us, though the trace holds more persistent launches
    assert rec["duration_us"] == pytest.approx(2200.0)
    assert rec["launch"] == {"kernel": "k_iface_2d", "type": "float", "grid_threads": 8277632}


def test_passes_of_different_shapes_are_refused(tmp_path):
    tr = tmp_path / "trace.csv"
    _trace(tr)
    f, w, s = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "s.csv"
    _counters(f, ["FETCH_SIZE"])
    _counters(w, ["WRITE_SIZE"], name=LOOP, grid=65536)
    _counters(s, ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU"])
    with pytest.raises(ValueError, match="different launch shapes"):
        P.write_counter_summaries(str(f), str(w), str(s), str(tmp_path), str(tr))
