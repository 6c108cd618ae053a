"""Bounds check of every kernel launch of the HIP library on the CPU: the
kernel code is compiled for the host in a serial emulation of the launch
grid (paper_1412_4489_amd/csrc/hostcheck) with AddressSanitizer, and the
cases of the GPU parity tests are run through the C ABI; the FP64 step also
matches the oracle.  The same build checks that the device code's division
with a precomputed reciprocal gives the bits of the IEEE quotient.  No GPU
is needed."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(_asan() is None, reason="libasan not available")
def test_kernels_in_bounds_under_asan(tmp_path):
    sys.path.insert(0, os.path.join(ROOT, "paper_1412_4489_amd", "csrc", "hostcheck"))
    import make_hostcheck
    lib = make_hostcheck.main(str(tmp_path))
    env = dict(os.environ, LD_PRELOAD=_asan(), ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "hostcheck_cases.py"), lib],
                       capture_output=True, text=True, env=env, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    assert "ERROR: AddressSanitizer" not in r.stderr
    assert "batch ok" in r.stdout
    assert "division ok" in r.stdout
    assert "persistent interface launch (64, 8): results identical" in r.stdout
    assert r.stdout.count("tiled reconstruction") == 5 and "DIFFER" not in r.stdout
