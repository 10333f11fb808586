"""Build libpa.so (the HIP kernels and the C ABI) in place for gfx950.

hipcc cross-compiles without a GPU.  Host code is compiled with
-ffp-contract=off so that the double-precision reweighting tables are the
plain IEEE operations written in the source; device code is compiled with
packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
SO = os.path.join(HERE, "libpa.so")
SOURCES = ["pa_kernels.hip", "pa_tables.hip", "pa_api.hip", "pa_batch.hip",
           "pa_mlp.hip", "pa_potts.hip"]
ARCH = os.environ.get("PA_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found: cannot build libpa.so")
    return p


def build(verbose: bool = False) -> str:
    """Compile libpa.so (always recompiles) and return its path."""
    tmp = SO + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
           "-shared", "-ffp-contract=off", "-Wall", "-Wno-unused-function",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", INCLUDE, "-I", CSRC, "-o", tmp]
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=ROOT)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libpa.so")
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
