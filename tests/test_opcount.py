"""The algorithmic operation counts that bench.py prices its roofline with
(paper_1412_4489_amd/csrc/opcount/opcounts.json) are those of the present
device source: the counting harness is built and run again here and must
give the committed figures."""
import json
import os
import shutil

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
OPC = os.path.join(os.path.dirname(HERE), "paper_1412_4489_amd", "csrc", "opcount")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_opcounts_match_the_source():
    import sys
    sys.path.insert(0, OPC)
    import opcount
    now = opcount.measure()
    with open(os.path.join(OPC, "opcounts.json")) as fh:
        committed = json.load(fh)
    assert now == committed
    # the Navier-Stokes interface adds the brackets of eq. dis2; both forms
    # run the same source, split between double and the compute type
    e, n = now["interface_euler_fp32_mixed"], now["interface_ns_fp32_mixed"]
    assert 1e4 < e["total"] < n["total"] < 3e4
    assert abs(now["interface_euler_fp64"]["total"] - e["total"]) < 0.01 * e["total"]
    assert now["interface_euler_fp64"]["compute"] == 0
