"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Every source is compiled with the host pass instrumented (the device code is
built as usual; GPU sanitizers are not used), linked into a separate
libdmimo.so in a temporary folder, and the C-ABI checks of test_abi_cpu.py
(exports, status strings, workspace sizes and every argument-validation path
of every entry point) run against it in a child Python with the sanitizer
runtime preloaded.  Any invalid access or undefined behaviour in the host
code those paths reach fails the test.
"""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2304_12745_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer"]

RUNNER = """
import functools, sys
sys.path.insert(0, {root!r})
from paper_2304_12745_amd import dmimo as D
D.load_library = functools.partial(D.load_library, {lib!r})
import pytest
sys.exit(pytest.main(["-q", "-p", "no:cacheprovider", {tests!r}]))
"""


def _runtime():
    c = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return c[-1] if c else None


@pytest.mark.slow
def test_abi_validation_under_host_sanitizers(tmp_path):
    rt = _runtime()
    if not os.path.exists(HIPCC) or rt is None:
        pytest.skip("hipcc or the clang sanitizer runtime is not installed")
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang",
              "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include")]
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src)[:-4] + ".o"))
        r = subprocess.run([HIPCC, *common, *SAN, "-c", src, "-o", obj], capture_output=True,
                           text=True, timeout=600)
        assert r.returncode == 0, r.stderr
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = str(tmp_path / "libdmimo.so")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *SAN, *objs, "-o", lib],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr
    nm = shutil.which("nm")
    if nm:
        syms = subprocess.run([nm, "-D", lib], capture_output=True, text=True).stdout
        assert "__asan_report" in syms and "__ubsan_handle" in syms   # really instrumented
    runner = tmp_path / "run_abi.py"
    runner.write_text(RUNNER.format(root=ROOT, lib=lib,
                                    tests=os.path.join(ROOT, "tests", "test_abi_cpu.py")))
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, str(runner)], capture_output=True, text=True, timeout=600,
                       env=env, cwd=str(tmp_path))
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
