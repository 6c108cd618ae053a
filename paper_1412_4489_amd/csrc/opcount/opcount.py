"""Algorithmic operation counts of the GPU path's arithmetic, per 2D
interface and per cell, written to opcounts.json beside this file.

    python -m paper_1412_4489_amd.csrc.opcount.opcount     (or python opcount.py)

opcount.cpp runs the device functions of gks_device.h / interface_gen.h on
the host with counting scalar types (count_scalar.h): every +, -, *, / of a
double or of the compute type counts one operation, fma two, sqrt / exp /
erfc one transcendental (reported apart).  The operations that the kernels
in gks.hip add around those functions are counted here from that source:

* accumulation of the sections of k_iface_2d: the hydrodynamic part and the
  kinetic part of each side add their 4 fluxes and 8 point values to the
  running sums (3 x 12 double additions): 36 per interface;
* the Prandtl-number fix (Navier-Stokes): the three sections' <psi f> added
  to the prologue's (12 additions), k2 = (U0^2 + V0^2)/2 (4), the heat flux
  q (14), F_E += (1/Pr - 1) q (2): 32;
* the update per cell: the flux differences (12), 1/(h k) (2), W += d/(h k)
  (8), the pressure check (8), the CFL bound (22 and one square root): 52.
"""
import json
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.dirname(HERE)
OUT = os.path.join(HERE, "opcounts.json")

ACCUMULATE = 36
PRANDTL_FIX = 32
UPDATE_CELL = 52


def measure():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "opcount")
        subprocess.check_call(["g++", "-std=c++17", "-O1", "-w", "-I", HERE, "-I", CSRC, "-o", exe,
                               os.path.join(HERE, "opcount.cpp")])
        raw = json.loads(subprocess.check_output([exe]).decode())
    out = {"counted": "floating-point operations of the device source per item: +, -, *, / one each, "
                      "fma two; transcendentals (sqrt, exp, erfc) apart",
           "raw": raw}
    for form in ("fp32_mixed", "fp64"):
        for kind in ("euler", "ns"):
            d, f, t = raw[f"interface_{kind}_{form}"]
            extra = ACCUMULATE + (PRANDTL_FIX if kind == "ns" else 0)
            out[f"interface_{kind}_{form}"] = {"double": d + extra, "compute": f, "total": d + extra + f,
                                               "transcendental": t}
    d, f, t = raw["recon_cell"]
    out["recon_cell"] = {"double": d, "total": d + f}
    out["update_cell"] = {"double": UPDATE_CELL, "total": UPDATE_CELL}
    return out


if __name__ == "__main__":
    res = measure()
    with open(OUT, "w") as fh:
        json.dump(res, fh, indent=1)
        fh.write("\n")
    print(json.dumps(res, indent=1))
    sys.exit(0)
