"""Build the HIP library (gfx950) in-tree: ``paper_2504_20169_amd/liblbm_mi355x.so``, and with
``bounds=True`` its bounds-checked debug build ``liblbm_mi355x_bounds.so`` (same sources and ABI,
compiled with LBM_BOUNDS: every element index of the step kernels is checked against its buffer).

Flags: -O3, FP contraction only within an expression (-ffp-contract=on, so the same source
expression rounds the same way in every kernel that inlines it), no fast-math, packed-FP32
instructions disabled.  The translation units compile in parallel to objects, then link.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblbm_mi355x.so")
LIB_BOUNDS = os.path.join(HERE, "liblbm_mi355x_bounds.so")
# lbm_kernels_d2q17.hip and lbm_kernels_d2q9.hip compile lbm_kernels.hip again for the D2Q17 and
# D2Q9 stencils
SOURCES = [os.path.join(HERE, "csrc", n)
           for n in ("lbm_kernels.hip", "lbm_kernels_d2q17.hip", "lbm_kernels_d2q9.hip", "lbm_capi.hip")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-ffp-contract=on",
         "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
# roctx (the ranges of LBM_DEBUG_RANGES), from the ROCm installation
ROCM_LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(HIPCC))), "lib")
LINK = ["-L" + ROCM_LIB, "-lrocprofiler-sdk-roctx", "-Wl,-rpath," + ROCM_LIB]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
    return res.returncode


def build(verbose: bool = False, bounds: bool = False) -> str:
    lib = LIB_BOUNDS if bounds else LIB
    flags = FLAGS + (["-DLBM_BOUNDS"] if bounds else [])
    with tempfile.TemporaryDirectory(prefix="lbm_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in SOURCES]
        cmds = [[HIPCC] + flags + ["-c", s, "-o", o] for s, o in zip(SOURCES, objs)]
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            rcs = list(ex.map(lambda c: _run(c, verbose), cmds))
        if any(rcs):
            raise RuntimeError("hipcc failed compiling for %s" % lib)
        tmp = lib + ".tmp"
        if _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + LINK + ["-o", tmp], verbose):
            raise RuntimeError("hipcc failed linking %s" % lib)
        os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True, bounds="--bounds" in sys.argv))
