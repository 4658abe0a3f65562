"""Host code of libdfmm under AddressSanitizer and UndefinedBehaviorSanitizer
(and the serving scheduler also under ThreadSanitizer).

The workspace layout and the stage-timer book are plain C++ (no HIP types);
tests/host/bookkeeping_test.cpp drives them through their edge cases (every
buffer of every layout written through its offset, pool exhaustion, intervals
of the second stream, out-of-range stage ids) in a g++ build with
-fsanitize=address,undefined.  The same headers are compiled into libdfmm.so.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bookkeeping_under_asan_and_ubsan(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "bookkeeping_test"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "paper_1311_4257_amd", "csrc"),
           os.path.join(ROOT, "tests", "host", "bookkeeping_test.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True,
                       env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0"})
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host bookkeeping: ok" in r.stdout


@pytest.mark.parametrize("sanitizer", ["address,undefined", "thread"])
def test_serving_scheduler_under_sanitizers(tmp_path, sanitizer):
    """The request scheduler of the serving loop (csrc/batcher.hpp) against a
    stand-in device: pass formation (submission order, rhs and request caps, a
    long request alone), HBM admission with grow-only workspaces, DFMM_ENOMEM at
    submission and at the front of a queue, the single-request form, launch
    failures, argument errors, and many submitting threads against a device
    thread (each request in exactly one pass, no plan with two passes in
    flight, destruction waiting for queued requests)."""
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "batcher_test"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", f"-fsanitize={sanitizer}",
           "-fno-sanitize-recover=all", "-pthread", "-I", os.path.join(ROOT, "paper_1311_4257_amd", "csrc"),
           os.path.join(ROOT, "tests", "host", "batcher_test.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120,
                       env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0"})
    assert r.returncode == 0, r.stdout + r.stderr
    assert "batcher: ok" in r.stdout
