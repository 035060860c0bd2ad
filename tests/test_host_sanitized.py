"""Host-side library logic under AddressSanitizer and UBSan: the table cache
(LRU by bytes, pins held by plans, eviction rounds) and the argument
validation of the C ABI, compiled from the library's own headers with g++
and run without a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2310_08408_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_cache_and_validation_sanitized(tmp_path):
    exe = str(tmp_path / "cache_validate_test")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-Wall", "-Wextra", "-Werror=return-type",
           "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host", "cache_validate_test.cpp"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=240)
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "passed" in r.stdout


def test_abi_validation_under_sanitizers(tmp_path):
    """tests/test_abi.py against a libprop build whose ABI layer (argument
    validation, caches, plans) is compiled with ASan + UBSan, with the
    sanitizer runtime preloaded into the Python process."""
    import sys
    from paper_2310_08408_amd import build as b
    try:
        rt = b.sanitizer_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    lib = b.build_host_sanitized()
    env = dict(os.environ, LD_PRELOAD=rt, LIBPROP_PATH=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       capture_output=True, text=True, timeout=600, env=env, cwd=ROOT)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in out
