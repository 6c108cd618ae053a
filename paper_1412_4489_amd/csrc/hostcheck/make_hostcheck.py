#!/usr/bin/env python3
"""Bounds-checked host build of the kernel code in gks.hip.

Copies gks.hip and its headers to a build directory, rewrites each
triple-chevron launch `K<<<grid, block, shmem, stream>>>(args);` into a serial
host emulation (emulation.h), and compiles the result with g++ and
AddressSanitizer into libgks_hostcheck.so.  The library has the C ABI of
include/gks.h; loading it with libasan preloaded checks every memory access
of every kernel launch against the exact size of its allocation.

    python make_hostcheck.py [outdir]
"""
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.dirname(HERE)
ROOT = os.path.dirname(os.path.dirname(CSRC))


def rewrite_launches(src):
    out, pos = [], 0
    while True:
        k = src.find("<<<", pos)
        if k < 0:
            out.append(src[pos:])
            return "".join(out)
        # the kernel expression starts after the previous statement boundary
        start = max(src.rfind(c, 0, k) for c in (";", "{", "}", "\n")) + 1
        while src[start] in " \t":
            start += 1
        kernel = src[start:k]
        e = src.index(">>>", k)
        cfg = [c.strip() for c in split_top(src[k + 3:e])]
        assert src[e + 3] == "(", src[start:e + 10]
        depth, q = 0, e + 3
        while True:
            if src[q] == "(":
                depth += 1
            elif src[q] == ")":
                depth -= 1
                if depth == 0:
                    break
            q += 1
        args = src[e + 4:q]
        out.append(src[pos:start])
        shm = cfg[2] if len(cfg) > 2 else "0"
        out.append(f"gks_emulated_launch(dim3({cfg[0]}), dim3({cfg[1]}), [=]() {{ {kernel}({args}); }}, (size_t)({shm}))")
        pos = q + 1


def split_top(s):
    parts, depth, cur = [], 0, ""
    for ch in s:
        if ch in "(<[":
            depth += 1
        elif ch in ")>]":
            depth -= 1
        if ch == "," and depth == 0:
            parts.append(cur)
            cur = ""
        else:
            cur += ch
    parts.append(cur)
    return parts


def main(outdir=None):
    outdir = outdir or os.path.join(ROOT, "_build", "hostcheck")
    os.makedirs(outdir, exist_ok=True)
    for name in ("gks_device.h", "interface_gen.h"):
        s = open(os.path.join(CSRC, name)).read()
        s = s.replace("#include <hip/hip_runtime.h>", '#include "emulation.h"')
        open(os.path.join(outdir, name), "w").write(s)
    s = open(os.path.join(CSRC, "gks.hip")).read()
    s = s.replace("#include <hip/hip_runtime.h>", '#include "emulation.h"')
    s = re.sub(r"__attribute__\(\(amdgpu_waves_per_eu\([^)]*\)\)\)", "", s)
    # the serial emulation has no cross-lane shuffles: every lane takes part
    # in the wave minimum's atomic directly, which gives the same minimum
    s, n = re.subn(r"if \(\(threadIdx\.x & 63\) == 0\) (atomicMin\()", r"\1", s)
    assert n == 1, "wave-minimum pattern not found"
    # dynamic LDS: the emulation's per-launch buffer
    s, n = re.subn(r"extern __shared__ (?:__align__\(\d+\) )?unsigned char (\w+)\[\];",
                   r"unsigned char* \1 = emu_dynamic_lds();", s)
    assert n >= 1, "dynamic LDS declaration not found"
    s = rewrite_launches(s)
    # the correctly rounded division helper of the device code, for a host test
    s += ('\nextern "C" double gks_emu_div_by(double a, double b) { return gks::div_by(a, gks::divisor(b)); }\n')
    # emulated device memory for callers of gks_init_device
    s += ('\nextern "C" void* gks_emu_alloc(size_t n) {\n  void* p = nullptr;\n'
          '  return hipMalloc(&p, n) == hipSuccess ? p : nullptr;\n}\n'
          'extern "C" void gks_emu_free(void* p) { (void)hipFree(p); }\n')
    open(os.path.join(outdir, "gks_hostcheck.cpp"), "w").write(s)
    open(os.path.join(outdir, "emulation.h"), "w").write(open(os.path.join(HERE, "emulation.h")).read())
    lib = os.path.join(outdir, "libgks_hostcheck.so")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-shared", "-fsanitize=address", "-fno-omit-frame-pointer",
           "-Wno-unknown-pragmas", "-Wno-attributes", "-I", outdir, "-I", os.path.join(ROOT, "include"),
           "-o", lib, os.path.join(outdir, "gks_hostcheck.cpp")]
    subprocess.check_call(cmd)
    return lib


if __name__ == "__main__":
    print(main(sys.argv[1] if len(sys.argv) > 1 else None))
