"""Build libodf.so (HIP, gfx950) in-tree with hipcc.

Usage: ``python -m paper_1009_0958_amd.build`` or ``build()`` from Python.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libodf.so")
ARCH = os.environ.get("ODF_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=" + ARCH,
    # packed FP32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False, extra=None) -> str:
    """Compile every HIP source into ``libodf.so`` (always recompiles): one
    object per source, compiled in parallel, then one link."""
    import shutil
    import tempfile
    from concurrent.futures import ThreadPoolExecutor

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    objdir = tempfile.mkdtemp(prefix="odf_build_")
    cflags = [f for f in HIPCC_FLAGS if f != "-shared"]

    def compile_one(src):
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [hipcc, *cflags, *(extra or []), "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        return obj

    try:
        srcs = sources()
        # the large forward units first, so that they start early
        srcs.sort(key=lambda f: 0 if os.path.basename(f).startswith("fwd") else 1)
        workers = max(1, min(len(srcs), os.cpu_count() or 4, 8))
        with ThreadPoolExecutor(max_workers=workers) as ex:
            objs = list(ex.map(compile_one, srcs))
        cmd = [hipcc, *HIPCC_FLAGS, *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
    finally:
        shutil.rmtree(objdir, ignore_errors=True)
    os.replace(tmp, LIB)
    return LIB


def build_microbench(verbose: bool = False) -> str:
    """Compile the VALU-rate / copy-bandwidth microbenchmark executable."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    src = os.path.join(HERE, "microbench", "valu_rates.hip")
    exe = os.path.join(HERE, "microbench", "valu_rates")
    flags = [f for f in HIPCC_FLAGS if f not in ("-fPIC", "-shared")]
    cmd = [hipcc, *flags, src, "-o", exe]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return exe


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
