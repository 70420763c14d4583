"""Build the gfx950 shared library libsgh.so in-tree with hipcc.

    python -m paper_1309_0392_amd.build

Sources: csrc/sgh_kernels_<f64|f32>_<h|d|a>.hip (device code from the templates
in csrc/sgh_kernels.inc, one unit per element type and operation, compiled in
parallel), csrc/sgh_api.cpp (host side, C ABI from include/sgh.h), csrc/sgh_combi.cpp
(combination-technique sparse grid: layout, gather / scatter, reduce).  Packed FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsgh.so")
ARCH = os.environ.get("SGH_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC, "-Wall"]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

UNITS = [("sgh_kernels_%s_%s.hip" % (t, o), ["-x", "hip"] + DEVICE) for t in ("f64", "f32") for o in "hda"]
UNITS.append(("sgh_api.cpp", ["-x", "hip"] + DEVICE))
UNITS.append(("sgh_combi.cpp", ["-x", "hip"] + DEVICE))


def build(verbose: bool = True, out: str = LIB, defines=(), build_dir: str = BUILD) -> str:
    """Compile every unit and link the library (always rebuilds).  `defines` are
    extra -D flags for tuning variants built elsewhere than the default path."""
    os.makedirs(build_dir, exist_ok=True)
    extra = ["-D" + d for d in defines]

    def one(u):
        src, flags = u
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        subprocess.run([HIPCC] + COMMON + extra + flags + ["-c", os.path.join(CSRC, src), "-o", obj], check=True)
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(len(UNITS), max(1, os.cpu_count() or 1))) as ex:
        objs = list(ex.map(one, UNITS))
    LIB_OUT = out
    tmp = LIB_OUT + ".tmp%d" % os.getpid()
    subprocess.run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs, check=True)
    os.replace(tmp, LIB_OUT)
    if verbose:
        print("built", LIB_OUT)
    return LIB_OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
