"""AddressSanitizer and UndefinedBehaviorSanitizer builds, on the CPU:

* the FP64 oracle (oracle/fastfca_oracle.c) compiled with gcc's sanitizers
  and driven through every entry point by tests/sanitize/oracle_driver.c;
* the library's host runtime (csrc/runtime.hip, host code only: the
  sanitizers are applied to the host compilation alone) linked with the
  other objects of the build, and its argument validation driven by
  tests/sanitize/abi_driver.c, whose calls are all rejected before any GPU
  work, so no GPU is needed.
A sanitizer report makes the driver exit non-zero (halt_on_error).
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
ENV = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:detect_leaks=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    return p.returncode, p.stdout


def test_oracle_under_asan_and_ubsan():
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "oracle_driver")
        rc, out = _run(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fno-omit-frame-pointer",
                        "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "fastfca_oracle.c"),
                        "-o", exe, "-lm"])
        assert rc == 0, out
        rc, out = _run([exe], env=ENV, timeout=300)
        assert rc == 0 and "oracle driver: ok" in out, out


def test_runtime_host_validation_under_asan_and_ubsan():
    build = os.path.join(ROOT, "paper_2101_08563_amd", "_build")
    objs = [os.path.join(build, f) for f in sorted(os.listdir(build))
            if f.endswith(".o") and f != "runtime.o"] if os.path.isdir(build) else []
    if not objs or not os.path.exists(HIPCC) or not os.path.exists(CLANG):
        pytest.skip("library objects or the ROCm compilers are not available (run the build first)")
    with tempfile.TemporaryDirectory() as td:
        rt = os.path.join(td, "runtime_san.o")
        # the sanitizers instrument the host compilation only; the device code is untouched
        rc, out = _run([HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                        "-Xarch_host", "-fno-omit-frame-pointer",
                        "-c", os.path.join(ROOT, "paper_2101_08563_amd", "csrc", "runtime.hip"), "-o", rt])
        assert rc == 0, out
        lib = os.path.join(td, "libfastfca_san.so")
        rc, out = _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", lib, rt] + objs)
        assert rc == 0, out
        exe = os.path.join(td, "abi_driver")
        rc, out = _run([CLANG, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                        os.path.join(SAN, "abi_driver.c"), "-o", exe, lib, "-Wl,-rpath," + td])
        assert rc == 0, out
        rc, out = _run([exe], env=ENV, timeout=300)
        assert rc == 0 and "abi driver: ok" in out, out
