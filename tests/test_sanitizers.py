"""The C code under AddressSanitizer and UndefinedBehaviorSanitizer, on the
CPU: the oracle (gcc) through its own pin tests, and the host side of the HIP
library (argument validation, plans, tuning table; clang, device code built
as usual) through the C-ABI host tests.  Each runs in a child process with the
sanitizer runtime preloaded; any report fails the test (undefined behaviour
aborts: -fno-sanitize-recover)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-O1", "-g"]


def _run(env_extra, test_files, timeout):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1", **env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", *test_files, "-q", "-x",
                        "-p", "no:cacheprovider", "-m", "not gpu"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", *SAN_FLAGS, "-std=c99", "-fopenmp", "-fPIC", "-shared",
                           "-o", lib, os.path.join(ROOT, "oracle", "odf_oracle.c"), "-lm"])
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    out = _run({"LD_PRELOAD": asan, "ODF_ORACLE_LIB": lib},
               ["tests/test_oracle_pins.py", "tests/test_oracle_cw.py",
                "tests/test_oracle_acwddf.py"], 900)
    assert " passed" in out


@pytest.mark.skipif(os.environ.get("ODF_SANITIZE_HOST") != "1",
                    reason="builds the host-sanitized library first (about 2 minutes): "
                           "set ODF_SANITIZE_HOST=1")
def test_host_library_under_asan_ubsan():
    sys.path.insert(0, ROOT)
    from paper_1009_0958_amd import build

    lib = build.build_host_sanitized()
    out = _run({"LD_PRELOAD": build.asan_runtime(), "ODF_LIB": lib},
               ["tests/test_capi_host.py"], 600)
    assert " passed" in out
