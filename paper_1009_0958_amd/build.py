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


SANITIZED_LIB = os.path.join(HERE, "libodf_hostsan.so")


def build_host_sanitized(verbose: bool = False) -> str:
    """Compile the library with AddressSanitizer and UndefinedBehaviorSanitizer
    on its host code only (argument validation, plans, tuning table; the device
    code is built as usual) into ``libodf_hostsan.so``.  Load it with the clang
    ASan runtime preloaded (see ``asan_runtime()``) and ``ODF_LIB`` naming it."""
    import shutil
    import tempfile
    from concurrent.futures import ThreadPoolExecutor

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host",
           "-fno-omit-frame-pointer"]
    cflags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *san]
    objdir = tempfile.mkdtemp(prefix="odf_hostsan_")
    tmp = SANITIZED_LIB + ".tmp%d" % os.getpid()

    def compile_one(src):
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [hipcc, *cflags, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", src,
               "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
        return obj

    try:
        srcs = sorted(sources(), key=lambda f: 0 if os.path.basename(f).startswith("fwd") else 1)
        with ThreadPoolExecutor(max_workers=max(1, min(len(srcs), os.cpu_count() or 4, 8))) as ex:
            objs = list(ex.map(compile_one, srcs))
        subprocess.check_call([hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH, *san,
                               "-shared-libsan", *objs, "-o", tmp])
    finally:
        shutil.rmtree(objdir, ignore_errors=True)
    os.replace(tmp, SANITIZED_LIB)
    return SANITIZED_LIB


def asan_runtime() -> str:
    """Path of the clang AddressSanitizer runtime the sanitized build links."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out = subprocess.check_output([hipcc, "-print-file-name=libclang_rt.asan-x86_64.so"],
                                  text=True).strip()
    if os.path.isabs(out) and os.path.exists(out):
        return out
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc)), "..", "lib", "llvm", "lib",
                         "clang")
    for ver in sorted(os.listdir(clang)):
        cand = os.path.join(clang, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(cand):
            return os.path.realpath(cand)
    raise FileNotFoundError("libclang_rt.asan-x86_64.so")


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
    if sys.argv[1:] == ["--sanitize-host"]:
        print(build_host_sanitized(verbose=True))
    else:
        build(verbose=True, extra=sys.argv[1:])
