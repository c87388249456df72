"""Host-side code of the serving runtime, checked without a GPU.

The arena allocator (csrc/server_arena.h) is compiled into a small checker
program (tests/host/arena_check.cpp) with AddressSanitizer and
UndefinedBehaviorSanitizer and run: resident uploads between running queries
leave the query space whole, and random interleavings of query scratch and
resident uploads keep the free list disjoint, coalesced and complete.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_arena_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "arena_check"
    src = os.path.join(ROOT, "tests", "host", "arena_check.cpp")
    r = subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", src, "-o", str(exe)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "arena checks passed" in r.stdout
