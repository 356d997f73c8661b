"""Build the HIP library (libfastfca.so) for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfastfca.so")
# (source, extra defines, object name); the wide family is compiled once per M
SOURCES = [("em_kernel.hip", [], "em_kernel.o"), ("em_cov_kernel.hip", [], "em_cov_kernel.o"),
           ("mnmf_kernels.hip", [], "mnmf_kernels.o"), ("aux_kernels.hip", [], "aux_kernels.o"),
           ("runtime.hip", [], "runtime.o"), ("synth_kernels.hip", [], "synth_kernels.o"),
           ("net_kernels.hip", [], "net_kernels.o"), ("net_api.hip", [], "net_api.o")] + [
    ("em_wide_kernel.hip", ["-DFFCA_WIDE_M=%d" % m], "em_wide_m%d.o" % m) for m in range(2, 9)]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-value",
]


def build(verbose: bool = True, jobs: int = 0) -> str:
    """Compile every source to an object, in parallel, then link the shared library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    t0 = time.time()
    procs = []
    objs = []
    for src, defs, oname in SOURCES:
        obj = os.path.join(objdir, oname)
        objs.append(obj)
        cmd = [hipcc, *HIPCC_FLAGS, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((oname, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write(text)
        elif verbose and text.strip():
            sys.stderr.write(text)
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print("built %s in %.1f s" % (LIB, time.time() - t0))
    return LIB


if __name__ == "__main__":
    build()
